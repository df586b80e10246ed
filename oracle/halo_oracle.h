/*
 * halo_oracle.h -- plain, serial, FP64 CPU oracle of the ROCKSTAR hot path.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path links or calls this
 * library; only the tests, the smoke check and the benchmark's CPU-baseline
 * leg do.  It shares no source with the GPU library.
 *
 * Stages (Behroozi, Wechsler & Wu 2013, Section 3 and Appendix B):
 *   orc_fof3d     3D friends-of-friends, standard definition (Section 3.1)
 *   orc_refine6d  recursive phase-space FOF hierarchy (Section 3.2, Eq. 1)
 *   orc_assign    seeds, Poisson seed merging (Eq. 2), hierarchical particle
 *                 assignment (Eqs. 3-4), host/subhalo relation (Section 3.4)
 *   orc_unbind    single-pass unbinding with an exact direct-sum potential
 *                 (Section 3.5.3, Appendix B)
 *   orc_props     centre, virial SO mass and radius, vmax, core and bulk
 *                 velocity, core-bulk offset (Sections 3.5.1-3.5.4)
 *   orc_props_extra  the sums behind the additional properties of Sections
 *                 3.5.2 and 3.5.4 (further SO thresholds, centre-of-mass
 *                 offset, angular momentum, energies, shape tensor); the
 *                 properties themselves are derived from them in oracle.py
 *
 * All pointers are host pointers owned by the caller.  Return 0 on success,
 * a negative code on error (ORC_E*).
 */
#ifndef HALO_ORACLE_H
#define HALO_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define ORC_OK 0
#define ORC_EINVAL (-1)
#define ORC_ENOMEM (-2)
#define ORC_ECAPACITY (-4)
#define ORC_EGEOMETRY (-5)

typedef struct {
  double box;               /* periodic box side L */
  double b;                 /* FOF linking parameter (0.28) */
  double f;                 /* linked fraction for the 6D linking length (0.7) */
  int32_t min_members;      /* smallest (sub)group that is refined / kept (10) */
  int32_t max_levels;       /* hierarchy depth limit */
  double merge_q2;          /* seed merge threshold on q^2, (10 sqrt 2)^2 = 200 */
  double particle_mass;     /* m */
  double G;                 /* gravitational constant in (Mpc/h)(km/s)^2/(Msun/h) */
  double rho_vir;           /* virial density (360 rho_m at z = 0) */
  double softening;         /* Plummer softening eps */
  double core_frac;         /* core radius as a fraction of R_vir (0.1) */
  double unbound_threshold; /* minimum bound fraction of a valid halo (0.5) */
  int32_t ell_subset;       /* 0: l from every particle's nearest neighbour; else nodes
                               of more particles take it from a hashed subset of about
                               this many (the paper's 10^4) */
  double major_merger;      /* MP: a subhalo with |S(h)| >= MP |S(host)| is unbound in
                               the merging system's potential; 0 = off */
  int32_t fof_dense;        /* 0: standard FOF; t > 0: a particle with more than t
                               friends within ll also links everything within 2 ll
                               (the paper's dense-particle shortcut, t = 16) */
} orc_params;

typedef struct {            /* node table, structure of arrays, capacity cap */
  int32_t *parent, *level, *first_child, *n_children;
  uint32_t *count, *canon, *fof, *flags;
  double *cx, *cy, *cz, *vx, *vy, *vz, *sx2, *sv2;
  float *ell2;
} orc_nodes;

typedef struct {            /* seed / halo table, one row per leaf node */
  int32_t *seed_node, *merged_into, *host;
  uint32_t *fof, *n_assigned;
  double *xs, *ys, *zs, *vxs, *vys, *vzs, *sv2, *vmax2;
} orc_halos;

typedef struct {            /* unbinding results per halo */
  uint32_t *n_bound_own, *n_s, *n_bound_s;
  uint8_t *valid;
  double *vbx, *vby, *vbz;
} orc_unbound;

typedef struct {            /* halo properties */
  double *px, *py, *pz, *vcx, *vcy, *vcz, *vbx, *vby, *vbz;
  double *mvir, *rvir, *vmax, *voff;
  uint32_t *n_bound;
} orc_props_out;

typedef struct {            /* sums behind the additional properties, per halo */
  double *sx, *sy, *sz;     /* sum of x - centre over the set V(h) */
  double *jx, *jy, *jz;     /* sum of (x - centre) x (v - v_bulk) over V(h) */
  double *t2;               /* sum of |v - v_bulk|^2 over V(h) */
  double *uinv;             /* sum over pairs of V(h) of 1/sqrt(r^2 + eps^2) */
  double *mxx, *myy, *mzz, *mxy, *mxz, *myz; /* sum of (x - centre)_a (x - centre)_b,
                                                own particles of V(h) */
  uint32_t *k, *n_own;      /* |V(h)|, own particles in V(h) */
  uint32_t *k_so;           /* SO count per extra threshold, [n_so * n_halos] */
} orc_extra_sums;

#define ORC_EXTRA_NSUM 15

#define ORC_NODE_LEAF 1u
#define ORC_NODE_DEGENERATE 2u  /* zero position or velocity dispersion */
#define ORC_NODE_WHOLE 4u       /* the only child would equal the node */

int orc_fof3d(const orc_params* p, int64_t n, int pos_f64, const void* x,
              const void* y, const void* z, uint32_t* label);

int orc_refine6d(const orc_params* p, int64_t n, int pos_f64, const void* x,
                 const void* y, const void* z, const float* vx, const float* vy,
                 const float* vz, const uint32_t* label, int64_t node_cap,
                 orc_nodes* nodes, int32_t* deepest, int64_t* n_nodes);

int orc_assign(const orc_params* p, int64_t n, int pos_f64, const void* x,
               const void* y, const void* z, const float* vx, const float* vy,
               const float* vz, const orc_nodes* nodes, int64_t n_nodes,
               const int32_t* deepest, int64_t halo_cap, orc_halos* halos,
               int32_t* halo_of, int64_t* n_halos);

int orc_unbind(const orc_params* p, int64_t n, int pos_f64, const void* x,
               const void* y, const void* z, const float* vx, const float* vy,
               const float* vz, const orc_halos* halos, int64_t n_halos,
               const int32_t* halo_of, uint8_t* bound, double* phi,
               double* phi_abs, orc_unbound* out);

int orc_props(const orc_params* p, int64_t n, int pos_f64, const void* x,
              const void* y, const void* z, const float* vx, const float* vy,
              const float* vz, const orc_nodes* nodes, int64_t n_nodes,
              const orc_halos* halos, int64_t n_halos, const int32_t* halo_of,
              const uint8_t* bound, orc_props_out* out);

int orc_props_extra(const orc_params* p, int64_t n, int pos_f64, const void* x,
                    const void* y, const void* z, const float* vx, const float* vy,
                    const float* vz, const orc_halos* halos, int64_t n_halos,
                    const int32_t* halo_of, const uint8_t* bound, const orc_props_out* props,
                    int32_t n_so, const double* so_rho, orc_extra_sums* out);

/* Exposed single steps, for the pins. */
void orc_halo_sums(int64_t k, const double* dx, const double* dy, const double* dz,
                   const double* vx, const double* vy, const double* vz, const uint8_t* own,
                   const double* vbulk, double eps2, double* sums15);
int64_t orc_so_count(int64_t nb, const double* r2_sorted, double C);
int orc_node_normalise(const orc_params* p, int64_t n_members, int pos_f64,
                       const void* x, const void* y, const void* z,
                       const float* vx, const float* vy, const float* vz,
                       const int64_t* members, float* xi6, double* moments8);
void orc_nn6d(int64_t n, const float* xi6, float* dmin);
float orc_ell2(int64_t n, const float* dmin, double f);
void orc_fof6d(int64_t n, const float* xi6, float ell2, int64_t* comp);
void orc_nn6d_range(int64_t n, const float* xi6, int64_t i0, int64_t i1, float* dmin);
int64_t orc_friends6d_range(int64_t n, const float* xi6, float ell2, int64_t i0, int64_t i1,
                            int64_t cap, int64_t* pairs);
void orc_phi_points(const orc_params* p, int pos_f64, const void* x, const void* y,
                    const void* z, const int64_t* src, int64_t nsrc, const int64_t* tgt,
                    int64_t ntgt, double* phi);
int32_t orc_position_shift(double box);
int orc_in_subset(uint64_t index, int64_t n, int64_t m);

#ifdef __cplusplus
}
#endif
#endif
