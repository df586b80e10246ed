/*
 * libhalo.h -- C ABI of the MI355X (gfx950) phase-space halo-finding path.
 *
 * The five stages follow the method of Behroozi, Wechsler & Wu (2013), "The
 * ROCKSTAR phase-space temporal halo finder", Section 3 and Appendix B:
 *
 *   libhalo_fof3d     3D friends-of-friends groups             (Section 3.1)
 *   libhalo_refine6d  recursive 6D phase-space FOF hierarchy   (Section 3.2, Eq. 1)
 *   libhalo_assign    seeds, seed merging, particle assignment (Section 3.3, Eqs. 2-4)
 *                     and host/subhalo relation                (Section 3.4)
 *   libhalo_unbind    single-pass unbinding                    (Section 3.5.3, App. B)
 *   libhalo_props     halo centre, SO mass/radius, vmax, core  (Sections 3.5.1-3.5.4)
 *                     and bulk velocity, core-bulk offset
 *   libhalo_props_extra  libhalo_props plus further SO masses,  (Sections 3.5.2, 3.5.4,
 *                     X_off, spins, T/|U|, Klypin concentration   Eqs. 5-11)
 *                     and shape
 *
 * Conventions shared by every entry point
 *   - Particles are given in structure-of-arrays form in input order:
 *     positions x, y, z as float32 or float64 (pos_dtype), in [0, box);
 *     velocities vx, vy, vz as float32 (km/s).  Particle i is the i-th element.
 *   - Every array argument is a DEVICE pointer owned by the caller, unless
 *     documented as a host pointer (the n_* counts and the parameter block).
 *     The library never frees caller memory.  Its workspace (device memory
 *     beyond the inputs and outputs) comes only from the allocator callback
 *     given to libhalo_ctx_create, and goes back through the matching free
 *     callback; the library itself allocates no device memory.
 *   - Work is enqueued on `stream` (a hipStream_t, NULL = default stream).  A
 *     call returns after its host-visible counts are known, which needs a
 *     few small synchronous read-backs on that stream; device outputs are
 *     complete when the stream is.
 *   - Errors: every call returns LIBHALO_OK (0) or a negative status; the
 *     message is in libhalo_last_error(ctx).  On error the device outputs are
 *     unspecified.  LIBHALO_ECAPACITY writes the required count into the
 *     n_* host output so the caller can grow the buffer and call again.
 *   - One context per stream at a time; a context is not thread safe.
 *
 * Floating point: 3D friendship uses FP64 minimum-image distances; group
 * moments use positions (relative to the group's smallest-index particle) and
 * velocities quantised to fixed point (2^-S Mpc/h with S = 40 -
 * ceil(log2(box/2)), and 2^-24 km/s) and summed exactly in 128-bit integers,
 * so results do not depend on summation order; 6D distances are FP32 on
 * coordinates normalised in FP64 and rounded once.
 */
#ifndef LIBHALO_H
#define LIBHALO_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  LIBHALO_OK = 0,
  LIBHALO_EINVAL = -1,     /* bad argument, parameter or input value */
  LIBHALO_ENOMEM = -2,     /* the allocator callback returned no workspace */
  LIBHALO_EHIP = -3,       /* a HIP runtime call failed */
  LIBHALO_ECAPACITY = -4,  /* an output table is too small; n_* holds the need */
  LIBHALO_EGEOMETRY = -5   /* a FOF group spans half the box or more */
} libhalo_status;

typedef enum { LIBHALO_F32 = 0, LIBHALO_F64 = 1 } libhalo_dtype;

/* How the hierarchy and potential kernels are scheduled. */
typedef enum {
  LIBHALO_PLAIN = 0,   /* one launch sequence per node / halo */
  LIBHALO_BATCHED = 1  /* all nodes of a level / all halos per launch */
} libhalo_mode;

/* Arithmetic of the unbinding potential. */
typedef enum {
  LIBHALO_PREC_FP64 = 0,  /* FP64 direct sum */
  LIBHALO_PREC_MIXED = 1  /* FP32 halo-local tiles, compensated FP32 sums,
                             FP64 recheck of energies near zero */
} libhalo_prec;

/* Method parameters (Table 2 and Section 3 of the paper for the defaults). */
typedef struct {
  double box;               /* periodic box side L (Mpc/h) */
  double b;                 /* FOF linking parameter; ll = b L / N^(1/3) (0.28) */
  double f;                 /* linked fraction for the 6D linking length (0.7) */
  int32_t min_members;      /* smallest group / subgroup refined or kept (10) */
  int32_t max_levels;       /* hierarchy depth limit (EINVAL beyond it) */
  double merge_q2;          /* seed merge threshold on q^2 = (10 sqrt 2)^2 = 200 */
  double particle_mass;     /* m (Msun/h) */
  double G;                 /* gravitational constant, (Mpc/h)(km/s)^2/(Msun/h) */
  double rho_vir;           /* virial density, 360 rho_m at z = 0 ((Msun/h)/(Mpc/h)^3) */
  double softening;         /* Plummer softening eps of the potential (Mpc/h) */
  double core_frac;         /* core radius as a fraction of R_vir (0.1) */
  double unbound_threshold; /* minimum bound fraction of a valid halo (0.5) */
  double e_recheck;         /* mixed precision: FP64 recheck when |E| <
                               e_recheck (|K| + |phi|) (1e-4) */
  int32_t mode;             /* libhalo_mode */
  int32_t prec;             /* libhalo_prec */
  int32_t grid_min;         /* nodes with more particles use the exact tree
                               search instead of all pairs; 0 = 16384 on levels of
                               >= 2^23 particles and 131072 on smaller ones, else
                               >= 64 (results are identical either way) */
  int32_t ell_subset;       /* 0: ell from every particle's nearest neighbour (exact);
                               m > 0: nodes of more than m particles take it from a
                               subset drawn with probability m / n per particle
                               (SplitMix64 of the input index; Section 3.2, paper: 10^4) */
  double major_merger;      /* MP (Section 3.5.3, Table 2): the particles of a subhalo
                               with |S(h)| >= MP |S(host)| take their potential from the
                               merging system (the outermost halo reached through such
                               host links); 0 = off, the single-halo pass (paper: 0.3) */
  int32_t fof_dense;        /* 0: standard FOF; t > 0: the dense-particle variant of
                               Section 3.1 -- a particle with more than t friends within
                               ll also links every particle within 2 ll (paper: 16);
                               EINVAL when the box holds fewer than 2Q+1 cells of the
                               2 ll stencil */
  int32_t bh_min;           /* with bh_theta > 0: halos with |S(h)| >= bh_min (0 = 32768)
                               take their particles' potential from a tree */
  double bh_theta;          /* 0: exact direct sum; > 0: the tree potential of
                               Appendix B, a cell's monopole accepted at distances
                               d >= r_max/2 + sqrt((r_max/2)^2 + sigma^2/theta) */
  /* Work-unit sizes of the batched kernels, a speed choice (0 picks the
   * default).  nn_chunk and fof_chunk change no result bit; pot_chunk groups
   * the potential's partial sums differently, so phi changes at the rounding
   * level (and a bound flag only inside that band). */
  int32_t nn_chunk;         /* all-pairs nearest neighbours: smallest j-chunk of a
                               unit on levels of >= 262144 particles; a multiple of
                               256 in [256, 4096] (0 = 1024) */
  int32_t fof_chunk;        /* all-pairs 6D FOF: j particles per unit on those
                               levels; a multiple of 256 in [256, 16384] (0 = 2048) */
  int32_t pot_chunk;        /* direct-sum potential: j particles per unit; 1024,
                               2048 or 4096 (0 = 2048) */
  int32_t kd_leaf;          /* most particles of a leaf of the 6D search trees,
                               in [4, 64] (0 = 16); no result bit depends on it */
  int32_t bh_leaf;          /* most particles of a leaf of the tree potential's
                               trees, in [4, 64] (0 = 16); changes which cells are
                               accepted, so phi changes within the theta bound */
  double nn_bracket;        /* exact ell (ell_subset = 0), tree-searched nodes of more
                               than 4096 particles: the nearest-neighbour walks stop
                               once a point's distance is certainly below or above a
                               bracket of ell^2 taken from every 64th point's exact
                               distance, nn_bracket binomial standard deviations of
                               the sample rank either side (0 = 4); a node whose
                               ell^2 falls outside its bracket walks again without
                               one.  < 0: no bracket.  No result bit depends on it */
} libhalo_params;

/* Node table (refine6d output), structure of arrays, capacity `cap` rows.
 * Row order is breadth first: level by level; within a level, children of a
 * node follow their parents' order and, among siblings, their smallest
 * particle index.  Level-0 rows are the FOF groups of >= min_members. */
typedef struct {
  int32_t* parent;      /* parent row, -1 for a FOF group */
  int32_t* level;       /* depth, 0 for a FOF group */
  int32_t* first_child; /* first child row (children are contiguous), -1 if leaf */
  int32_t* n_children;  /* number of subgroups with >= min_members */
  uint32_t* count;      /* number of particles */
  uint32_t* canon;      /* smallest particle index (node identity) */
  uint32_t* fof;        /* FOF label of the group the node belongs to */
  uint32_t* flags;      /* LIBHALO_NODE_* */
  double *cx, *cy, *cz; /* centre (mean position), wrapped into [0, L) */
  double *vx, *vy, *vz; /* mean velocity */
  double* sx2;          /* position dispersion sigma_x^2 (3D, 1/n) */
  double* sv2;          /* velocity dispersion sigma_v^2 (3D, 1/n) */
  float* ell2;          /* squared 6D linking length, -1 if not computed */
  int64_t cap;
} libhalo_nodes;

#define LIBHALO_NODE_LEAF 1u
#define LIBHALO_NODE_DEGENERATE 2u /* sigma_x or sigma_v is zero */
#define LIBHALO_NODE_WHOLE 4u      /* the only subgroup would be the node */

/* Seed / halo table (assign output), one row per leaf node, in node order. */
typedef struct {
  int32_t* seed_node;   /* leaf node row of the seed */
  int32_t* merged_into; /* itself if kept, else the kept seed it merged into */
  int32_t* host;        /* host halo row (Section 3.4), -1 for a FOF's main halo */
  uint32_t* fof;        /* FOF label */
  uint32_t* n_assigned; /* particles assigned to the halo */
  double *xs, *ys, *zs;    /* seed position (leaf mean) */
  double *vxs, *vys, *vzs; /* seed velocity (leaf mean) */
  double* sv2;          /* final velocity dispersion of the assigned particles */
  double* vmax2;        /* final vmax^2 of the assigned particles about the seed */
  int64_t cap;
} libhalo_halos;

/* Unbinding results per halo row. */
typedef struct {
  uint32_t* n_bound_own; /* bound particles among those assigned to the halo */
  uint32_t* n_s;         /* |S(h)|: the halo's particles plus its subhalos' */
  uint32_t* n_bound_s;   /* bound particles in S(h) */
  uint8_t* valid;        /* n_bound_s >= unbound_threshold * n_s */
  double *vbx, *vby, *vbz; /* bulk velocity of S(h) */
} libhalo_unbound;

/* Halo properties per halo row (zeros for merged seeds). */
typedef struct {
  double *px, *py, *pz;    /* centre */
  double *vcx, *vcy, *vcz; /* core velocity (within core_frac R_vir) */
  double *vbx, *vby, *vbz; /* bulk velocity (within R_vir) */
  double *mvir, *rvir, *vmax, *voff;
  uint32_t* n_bound;       /* bound particles of S(h) */
} libhalo_props_out;

/* Additional halo properties per halo row (zeros for merged seeds), over
 * V(h) = the bound particles of S(h) inside R_vir (the k* innermost, the set
 * that defines M_vir), about the libhalo_props centre and bulk velocity. */
#define LIBHALO_MAX_SO 8
typedef struct {
  double* xoff;            /* |centre of mass of V(h) - centre| */
  double *jx, *jy, *jz;    /* angular momentum m sum (x - c) x (v - v_bulk) */
  double *kin, *pot;       /* T = m/2 sum |v - v_bulk|^2; U = -G m^2 sum over
                              pairs of 1/sqrt(r^2 + softening^2) */
  double* t_u;             /* T / |U| (0 when U = 0) */
  double *spin, *spin_bullock; /* Eq. 9 and Eq. 10 */
  double *c_klypin, *rs_klypin; /* Eq. 7-8 concentration and R_vir / c */
  double *b_to_a, *c_to_a; /* Eq. 11 axis ratios, own particles of V(h) */
  double *ax, *ay, *az;    /* major axis a e_1, largest component positive */
  uint32_t* n_shape;       /* own particles of V(h) */
  double *m_so, *r_so;     /* [n_so * cap], threshold-major */
  int64_t cap;             /* rows of each array above (m_so, r_so: n_so * cap) */
} libhalo_props_extra_out;

typedef struct libhalo_ctx libhalo_ctx;

/* Device memory provider of the workspace (for example a caching allocator).
 *   alloc_fn(bytes, user, stream): return `bytes` (> 0) of device memory on
 *     the context's device (current when called), aligned to 256 bytes, for
 *     use by work enqueued on `stream` (a hipStream_t, NULL = default
 *     stream); return NULL when it cannot, and the calling entry point fails
 *     with LIBHALO_ENOMEM.  Each entry point takes its main workspace before
 *     it writes any output, so a refusal there leaves the outputs untouched
 *     (the tree potential's own workspace, when it needs one, is taken later
 *     inside libhalo_unbind).
 *   free_fn(ptr, user, stream): take back a block from alloc_fn.  The library
 *     calls it only once the work it enqueued on `stream` is complete (after
 *     a stream synchronisation; at libhalo_ctx_destroy after a device
 *     synchronisation), when a workspace grows and when the context ends.
 * `user` is passed through unchanged.  The callbacks are called on the
 * thread that calls the library, from inside its entry points. */
typedef void* (*libhalo_alloc_fn)(size_t bytes, void* user, void* stream);
typedef void (*libhalo_free_fn)(void* ptr, void* user, void* stream);

/* Create a context on HIP device `device` with parameters *p (host) and the
 * workspace allocator (alloc_fn, free_fn, user; both functions required).
 * Takes a 256-byte error word from alloc_fn; every later workspace is sized
 * by the entry point that needs it, grown only when a larger one is needed,
 * and kept for reuse until libhalo_ctx_destroy.
 * Errors: EINVAL (bad parameters or device, a null callback), ENOMEM
 * (alloc_fn returned NULL), EHIP. */
int libhalo_ctx_create(const libhalo_params* p, int device, libhalo_alloc_fn alloc_fn,
                       libhalo_free_fn free_fn, void* user, libhalo_ctx** out);
/* Return the workspace to free_fn and release the context. */
int libhalo_ctx_destroy(libhalo_ctx* ctx);
/* Message of the last error on this context (static storage of the ctx). */
const char* libhalo_last_error(const libhalo_ctx* ctx);
/* Replace the parameters (EINVAL if invalid). */
int libhalo_set_params(libhalo_ctx* ctx, const libhalo_params* p);
/* Version string of the library. */
const char* libhalo_version(void);

/* Kernel timing (tracing aid).  enable bit 0: the library brackets its hot
 * kernel launches with HIP events on the launch stream; bit 1: the tree walks
 * run in a form that counts their work (libhalo_profile_work), which costs
 * them time, so timing and counting belong in separate runs.
 * libhalo_profile_read waits for those events and returns the summed device
 * time (ms) and the number of launches of `kernel` (a kernel name such as
 * "k_potential_f64") recorded since the last reset.  Errors: EINVAL, EHIP. */
int libhalo_profile(libhalo_ctx* ctx, int enable);
int libhalo_profile_reset(libhalo_ctx* ctx);
int libhalo_profile_read(libhalo_ctx* ctx, const char* kernel, double* total_ms,
                         int64_t* launches);
/* Work counted by the tree walks while counting is enabled, since the last
 * reset: for "k_kd_walk_nn" (nearest neighbours) and "k_kd_walk_fof" (6D FOF)
 * of large hierarchy nodes, the node boxes tested and the particle distances
 * evaluated; for "k_bh_walk" (tree potential), summed over target particles,
 * the cells tested and the terms added (monopoles and leaf particles).
 * Errors: EINVAL (another kernel name), EHIP. */
int libhalo_profile_work(libhalo_ctx* ctx, const char* kernel, double* tests, double* evals);

/*
 * 3D friends-of-friends (Section 3.1), standard definition: particles i and
 * j are friends when their minimum-image separation is <= ll = b L / n^(1/3)
 * (FP64); groups are connected components.  Exact: independent of order.
 *   fof_label[n]  out: smallest particle index of i's group
 *   perm[n]       out: first *n_members entries are the particles of groups
 *                 with >= min_members, ordered by (label, index)
 *   grp_first[grp_cap], grp_count[grp_cap]
 *                 out: range of each such group in perm, groups by label
 *   n_groups, n_members  host out
 * Errors: EINVAL (n < 1, n >= 2^32 - 1, a position outside [0, L) or NaN),
 * ECAPACITY (n_groups > grp_cap).
 */
int libhalo_fof3d(libhalo_ctx* ctx, int64_t n, int pos_dtype, const void* x,
                  const void* y, const void* z, uint32_t* fof_label, uint32_t* perm,
                  uint32_t* grp_first, uint32_t* grp_count, int64_t grp_cap,
                  int64_t* n_groups, int64_t* n_members, void* stream);

/*
 * libhalo_fof3d for callers that cannot allocate device memory during the
 * call (code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc).  Same arguments, results and errors as libhalo_fof3d,
 * but the workspace is a fixed device array of LIBHALO_NOALLOC_SCRATCH_BYTES
 * inside the library (each device that loads the library holds one copy until
 * the process ends; its address is looked up when a context is created on
 * that device), never the context's allocator: the call allocates nothing.
 * The caller still passes every input and output buffer.
 * Limit: ENOMEM, before any work, when the particles need more scratch than
 * the array holds (about 80 bytes per particle plus 4 per cell row of the
 * linking grid: up to about 3 million particles).
 * Concurrency: every call on a device shares that device's array, so calls
 * that overlap on one device (other threads, other contexts, other streams)
 * race and must be serialised by the caller; the call returns after its work
 * on `stream` has finished.
 */
#define LIBHALO_NOALLOC_SCRATCH_BYTES (256u << 20)
int libhalo_fof3d_noalloc(libhalo_ctx* ctx, int64_t n, int pos_dtype, const void* x,
                          const void* y, const void* z, uint32_t* fof_label, uint32_t* perm,
                          uint32_t* grp_first, uint32_t* grp_count, int64_t grp_cap,
                          int64_t* n_groups, int64_t* n_members, void* stream);

/*
 * Recursive phase-space FOF hierarchy (Section 3.2) of every FOF group given
 * by (perm, grp_first, grp_count) as produced by libhalo_fof3d.  For each
 * (sub)group: Eq. 1 metric (positions and velocities divided by the group's
 * 3D dispersions), squared linking length ell^2 = the ceil(f n)-th smallest
 * nearest-neighbour squared distance (so that a fraction >= f of the
 * particles have a friend), 6D FOF at ell^2; components of >= min_members
 * become subgroups, recursively.  A node with a zero dispersion, or whose
 * only subgroup would hold all its particles, is a leaf.
 *   nodes         out: node table (cap rows)
 *   deepest[n]    out: deepest node row holding particle i, -1 if none
 *   n_nodes       host out
 * Errors: ECAPACITY (n_nodes > nodes->cap), EGEOMETRY (group extent >= L/2
 * on an axis), EINVAL (depth beyond max_levels, |v| >= 2^16 km/s).
 */
int libhalo_refine6d(libhalo_ctx* ctx, int64_t n, int pos_dtype, const void* x,
                     const void* y, const void* z, const float* vx, const float* vy,
                     const float* vz, const uint32_t* perm, const uint32_t* grp_first,
                     const uint32_t* grp_count, int64_t n_groups, libhalo_nodes* nodes,
                     int32_t* deepest, int64_t* n_nodes, void* stream);

/*
 * Seeds, merging, assignment and host/subhalo relation (Sections 3.3-3.4).
 * One seed per leaf node.  Within a FOF group, seeds are visited by
 * decreasing size (ties: lower row); a seed merges into the closest kept
 * seed when |dx|^2/mu_x^2 + |dv|^2/mu_v^2 < merge_q2 (Eq. 2, mu = sigma /
 * sqrt(n) of the visited, smaller seed).  Bottom-up over levels, the
 * particles of a node outside all its subgroups go to its only seed, or to
 * the seed minimising |dx|^2/r_dyn^2 + |dv|^2/sigma_v^2 (Eqs. 3-4; r_dyn =
 * vmax / sqrt(4/3 pi G rho_vir); sigma_v and vmax from the particles already
 * assigned to that seed; ties: lower row).  Within a FOF group each halo but
 * the one with most particles becomes a sub of the closest halo (same metric)
 * earlier in the order (n_assigned desc, row asc).
 *   halos         out: seed / halo table (cap rows)
 *   halo_of[n]    out: halo row of particle i, -1 outside refined groups
 *   n_halos       host out (number of seeds = leaf nodes)
 * Errors: ECAPACITY (n_halos > halos->cap), EINVAL.
 */
int libhalo_assign(libhalo_ctx* ctx, int64_t n, int pos_dtype, const void* x,
                   const void* y, const void* z, const float* vx, const float* vy,
                   const float* vz, const libhalo_nodes* nodes, int64_t n_nodes,
                   const int32_t* deepest, libhalo_halos* halos, int32_t* halo_of,
                   int64_t* n_halos, void* stream);

/*
 * Single-pass unbinding (Section 3.5.3; exact direct sum in place of the
 * paper's tree code of Appendix B).  For particle i assigned to halo h:
 * phi_i = -G m sum_{j in S(h), j != i} (r_ij^2 + eps^2)^-1/2, S(h) = the
 * particles of h and of all its subhalos; bound iff
 * 1/2 |v_i - v_bulk(h)|^2 + phi_i < 0 with v_bulk(h) the mean velocity of
 * S(h).  A halo is valid when n_bound_s >= unbound_threshold * n_s.
 *   bound[n]      out: 1 if bound, 0 otherwise (0 outside halos)
 *   phi[n]        out (may be NULL): potential, 0 outside halos
 *   out           out: per-halo results
 * Errors: EINVAL.
 */
int libhalo_unbind(libhalo_ctx* ctx, int64_t n, int pos_dtype, const void* x,
                   const void* y, const void* z, const float* vx, const float* vy,
                   const float* vz, const libhalo_halos* halos, int64_t n_halos,
                   const int32_t* halo_of, uint8_t* bound, double* phi,
                   libhalo_unbound* out, void* stream);

/*
 * Halo properties from bound particles (Sections 3.5.1-3.5.4):
 * centre = mean position of the node, on the chain from the halo's seed leaf
 * up while the node holds no other halo's seed, minimising sigma_x / sqrt(n)
 * (ties: deeper); B(h) = bound particles of S(h) by distance from the
 * centre; virial SO mass M = k* m with k* the largest k such that every
 * j <= k has 3 j m / (4 pi r_j^3) >= rho_vir, R_vir = (3 M / (4 pi
 * rho_vir))^(1/3); vmax = max_{j <= k*} sqrt(G j m / max(r_j, eps)); bulk
 * velocity = mean of the k* innermost; core velocity = mean within core_frac
 * R_vir (the innermost particle if none); voff = |core - bulk|.
 * Errors: EINVAL.
 */
int libhalo_props(libhalo_ctx* ctx, int64_t n, int pos_dtype, const void* x,
                  const void* y, const void* z, const float* vx, const float* vy,
                  const float* vz, const libhalo_nodes* nodes, int64_t n_nodes,
                  const libhalo_halos* halos, int64_t n_halos, const int32_t* halo_of,
                  const uint8_t* bound, libhalo_props_out* out, void* stream);

/*
 * libhalo_props plus the additional properties of Sections 3.5.2 and 3.5.4
 * (writes *out exactly as libhalo_props does, and *ext):
 *  - m_so / r_so: SO mass and radius at each of n_so further thresholds
 *    so_rho[t] (host array, same units as rho_vir, each > 0), by the same
 *    first-downcrossing rule as M_vir over the bound particles of S(h);
 *  - xoff: distance from the centre to the centre of mass of V(h);
 *  - angular momentum, T, U and T/|U| of V(h) with the Plummer softening of
 *    unbinding; spin (Eq. 9, E = T + U, M = M_vir) and spin_bullock (Eq. 10);
 *  - c_klypin: root c >= 2.1626 of Eq. 7, clamped to [2.1626, 1e4] (2.1626
 *    when v_max^2 R_vir / (G M_vir) lies below the branch), rs_klypin =
 *    R_vir / c;
 *  - the Eq. 11 tensor (1/N) sum x_a x_b over the halo's own particles in
 *    V(h) (substructure excluded), positions about the centre: b/a, c/a from
 *    its sorted eigenvalues a^2 >= b^2 >= c^2 and the major axis vector.
 * The potential energy costs sum_h |V(h)|^2 / 2 pair terms (FP64, fixed-point
 * sums independent of scheduling).  Errors: EINVAL (n_so outside
 * [0, LIBHALO_MAX_SO], a threshold <= 0, null pointers, ext->cap < n_halos).
 */
int libhalo_props_extra(libhalo_ctx* ctx, int64_t n, int pos_dtype, const void* x,
                        const void* y, const void* z, const float* vx, const float* vy,
                        const float* vz, const libhalo_nodes* nodes, int64_t n_nodes,
                        const libhalo_halos* halos, int64_t n_halos, const int32_t* halo_of,
                        const uint8_t* bound, libhalo_props_out* out, int n_so,
                        const double* so_rho, libhalo_props_extra_out* ext, void* stream);

#ifdef __cplusplus
}
#endif
#endif
