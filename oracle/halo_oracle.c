/*
 * halo_oracle.c -- plain, serial, FP64 CPU oracle of the ROCKSTAR hot path
 * (Behroozi, Wechsler & Wu 2013, "The ROCKSTAR phase-space temporal halo
 * finder", Section 3 and Appendix B).
 *
 * TEST INFRASTRUCTURE: only the tests, the smoke check and the benchmark's
 * CPU-baseline leg load this library.  It shares no code with the GPU path.
 * Build: gcc -O2 -ffp-contract=off -fPIC -shared halo_oracle.c -lm
 *
 * Where the paper leaves a step open, the reading taken here is stated at
 * the step.  Readings that make the result independent of summation order
 * (so that a parallel implementation can reproduce it exactly):
 *   - Moments (mean and dispersion of positions and velocities) are computed
 *     from values quantised to fixed point and summed exactly in 128-bit
 *     integers: positions relative to the group's anchor particle at a
 *     resolution of 2^-S Mpc/h (S = 40 - ceil(log2(L/2))), velocities at
 *     2^-24 km/s.
 *   - 6D phase-space distances (Eq. 1) are evaluated in FP32 on coordinates
 *     normalised in FP64 and rounded once to FP32, with one fixed expression.
 * Parity status of each stage is recorded in the header of each function.
 */
#include "halo_oracle.h"

#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef __int128 i128;

#define VEL_SHIFT 24

/* ------------------------------------------------------------------ helpers */

static double pos_at(const void* a, int f64, int64_t i) {
  return f64 ? ((const double*)a)[i] : (double)((const float*)a)[i];
}

/* Minimum-image separation along one axis of the periodic box. */
static double min_image(double d, double box) {
  double h = 0.5 * box;
  if (d > h) return d - box;
  if (d < -h) return d + box;
  return d;
}

static double sq3(double a, double b, double c) { return fma(c, c, fma(b, b, a * a)); }

/* Double of a 128-bit integer (an exact fixed-point sum), by one fixed
 * sequence of roundings, within an ulp: the magnitude's two 64-bit words are
 * each rounded once and combined by one fma, then the sign is applied. */
static double i128_to_f64(i128 v) {
  const int neg = v < 0;
  const unsigned __int128 m = neg ? (unsigned __int128)(-v) : (unsigned __int128)v;
  const uint64_t hi = (uint64_t)(m >> 64), lo = (uint64_t)m;
  const double d = fma((double)hi, 18446744073709551616.0, (double)lo);
  return neg ? -d : d;
}

int32_t orc_position_shift(double box) {
  int e = 0;
  frexp(0.5 * box, &e);
  return 40 - e;
}

static int64_t quantise(double v, int shift) { return (int64_t)llrint(ldexp(v, shift)); }

typedef struct {
  i128 s1[3];
  i128 s2;
  int64_t n;
} qsum;

static void qsum_add(qsum* s, int64_t a, int64_t b, int64_t c) {
  s->s1[0] += a;
  s->s1[1] += b;
  s->s1[2] += c;
  s->s2 += (i128)a * a + (i128)b * b + (i128)c * c;
  s->n += 1;
}

/* Mean (per axis) and 3D variance (1/n) sum |q - mean|^2 from exact sums. */
static void qsum_finish(const qsum* s, int shift, double mean[3], double* var) {
  double n = (double)s->n;
  double mq[3];
  for (int a = 0; a < 3; ++a) mq[a] = i128_to_f64(s->s1[a]) / n;
  double s2q = i128_to_f64(s->s2) / n;
  double t = mq[0] * mq[0];
  t = fma(mq[1], mq[1], t);
  t = fma(mq[2], mq[2], t);
  double vq = s2q - t;
  if (!(vq > 0.0)) vq = 0.0;
  for (int a = 0; a < 3; ++a) mean[a] = ldexp(mq[a], -shift);
  *var = ldexp(vq, -2 * shift);
}

/* Canonical FP32 squared phase-space distance between normalised points. */
static float d2_6d(const float* a, const float* b) {
  float d0 = b[0] - a[0], d1 = b[1] - a[1], d2 = b[2] - a[2];
  float e0 = b[3] - a[3], e1 = b[4] - a[4], e2 = b[5] - a[5];
  float s = d0 * d0;
  s = fmaf(d1, d1, s);
  s = fmaf(d2, d2, s);
  s = fmaf(e0, e0, s);
  s = fmaf(e1, e1, s);
  s = fmaf(e2, e2, s);
  return s;
}

static int64_t uf_find(int64_t* par, int64_t i) {
  while (par[i] != i) {
    par[i] = par[par[i]];
    i = par[i];
  }
  return i;
}

/* Union keeping the smaller index as root, so a root is its set's minimum. */
static void uf_union(int64_t* par, int64_t a, int64_t b) {
  int64_t ra = uf_find(par, a), rb = uf_find(par, b);
  if (ra == rb) return;
  if (ra < rb)
    par[rb] = ra;
  else
    par[ra] = rb;
}

static int cmp_u64(const void* a, const void* b) {
  uint64_t x = *(const uint64_t*)a, y = *(const uint64_t*)b;
  return x < y ? -1 : x > y;
}

static int cmp_f32(const void* a, const void* b) {
  float x = *(const float*)a, y = *(const float*)b;
  return x < y ? -1 : x > y;
}

typedef struct {
  double r2;
  int64_t idx;
} rad_t;

typedef struct {
  uint64_t cell;
  int64_t idx;
} cellkey;

static int cmp_cellkey(const void* a, const void* b) {
  const cellkey* x = (const cellkey*)a;
  const cellkey* y = (const cellkey*)b;
  if (x->cell != y->cell) return x->cell < y->cell ? -1 : 1;
  return x->idx < y->idx ? -1 : x->idx > y->idx;
}

/* Sort record for seeds and halos: (fof asc, size desc, id asc). */
typedef struct {
  uint32_t fof, size;
  int64_t id;
} grpkey;

static int cmp_grpkey(const void* a, const void* b) {
  const grpkey* x = (const grpkey*)a;
  const grpkey* y = (const grpkey*)b;
  if (x->fof != y->fof) return x->fof < y->fof ? -1 : 1;
  if (x->size != y->size) return x->size > y->size ? -1 : 1;
  return x->id < y->id ? -1 : x->id > y->id;
}

static int cmp_rad(const void* a, const void* b) {
  const rad_t* x = (const rad_t*)a;
  const rad_t* y = (const rad_t*)b;
  if (x->r2 < y->r2) return -1;
  if (x->r2 > y->r2) return 1;
  return x->idx < y->idx ? -1 : x->idx > y->idx;
}

/* ------------------------------------------------------------- 3D FOF ---- */
/*
 * Friends of particle i within radius r (r2 = r^2): among the particles of
 * the 27 cells around i's cell in a grid of nc2 >= 3 cells of side >= r
 * (key sorted by cell, then index), or among all particles when key is NULL.
 * mode 0 returns the count (j != i), stopping once it exceeds limit; mode 1
 * unions i with each of them.
 */
static int64_t near_pass(const orc_params* p, int64_t n, int pos_f64, const void* x,
                         const void* y, const void* z, const cellkey* key, int64_t nc2,
                         int64_t i, double r2, int mode, int64_t limit, int64_t* par) {
  const double L = p->box;
  const double pc[3] = {pos_at(x, pos_f64, i), pos_at(y, pos_f64, i), pos_at(z, pos_f64, i)};
  int64_t cnt = 0;
  int64_t c[3] = {0, 0, 0};
  if (key) {
    const double inv = (double)nc2 / L;
    for (int a = 0; a < 3; ++a) {
      int64_t ci = (int64_t)floor(pc[a] * inv);
      if (ci < 0) ci = 0;
      if (ci >= nc2) ci = nc2 - 1;
      c[a] = ci;
    }
  }
  const int span = key ? 1 : 0;
  for (int dz = -span; dz <= span; ++dz)
    for (int dy = -span; dy <= span; ++dy)
      for (int dx = -span; dx <= span; ++dx) {
        int64_t lo = 0, hi = n;
        uint64_t cell = 0;
        if (key) {
          int64_t nx = (c[0] + dx + nc2) % nc2, ny = (c[1] + dy + nc2) % nc2,
                  nz = (c[2] + dz + nc2) % nc2;
          cell = (uint64_t)((nz * nc2 + ny) * nc2 + nx);
          while (lo < hi) {
            int64_t mid = (lo + hi) / 2;
            if (key[mid].cell < cell)
              lo = mid + 1;
            else
              hi = mid;
          }
        }
        for (int64_t b = lo; b < n && (!key || key[b].cell == cell); ++b) {
          int64_t j = key ? key[b].idx : b;
          if (j == i) continue;
          double ex = min_image(pos_at(x, pos_f64, j) - pc[0], L);
          double ey = min_image(pos_at(y, pos_f64, j) - pc[1], L);
          double ez = min_image(pos_at(z, pos_f64, j) - pc[2], L);
          if (sq3(ex, ey, ez) <= r2) {
            if (mode == 1)
              uf_union(par, i, j);
            else if (++cnt > limit)
              return cnt;
          }
        }
      }
  return cnt;
}

/* The dense-particle links of the FOF variant (orc_fof3d). */
static void dense_links(const orc_params* p, int64_t n, int pos_f64, const void* x,
                        const void* y, const void* z, double ll, int64_t* par) {
  const double L = p->box;
  const int64_t nc2 = (int64_t)floor(L / (2.0 * ll * (1.0 + 1e-9)));
  cellkey* key = NULL;
  if (nc2 >= 3) {
    key = (cellkey*)malloc(sizeof(cellkey) * n);
    const double inv = (double)nc2 / L;
    for (int64_t i = 0; i < n; ++i) {
      int64_t c[3];
      const void* ax[3] = {x, y, z};
      for (int a = 0; a < 3; ++a) {
        int64_t ci = (int64_t)floor(pos_at(ax[a], pos_f64, i) * inv);
        if (ci < 0) ci = 0;
        if (ci >= nc2) ci = nc2 - 1;
        c[a] = ci;
      }
      key[i].cell = (uint64_t)((c[2] * nc2 + c[1]) * nc2 + c[0]);
      key[i].idx = i;
    }
    qsort(key, (size_t)n, sizeof(cellkey), cmp_cellkey);
  }
  const int64_t t = p->fof_dense;
  for (int64_t i = 0; i < n; ++i)
    if (near_pass(p, n, pos_f64, x, y, z, key, nc2, i, ll * ll, 0, t, par) > t)
      near_pass(p, n, pos_f64, x, y, z, key, nc2, i, 4.0 * ll * ll, 1, 0, par);
  free(key);
}

/*
 * Standard friends-of-friends (Section 3.1): two particles are friends when
 * their minimum-image separation is at most ll = b * (L^3/N)^(1/3); groups
 * are the connected components.  The paper's faster variant (skip the
 * neighbour search around particles with more than 16 friends, link groups
 * within 2 ll instead) links a superset that depends on visiting order; the
 * default reading is the standard definition, the subset the paper
 * guarantees.  With fof_dense = t > 0 the variant is taken in an order-free
 * form: every particle with more than t friends within ll (itself excluded)
 * also links every particle within 2 ll.  Whatever the visiting order, the
 * paper's groups lie between the standard ones and these (a skipped
 * particle lies within ll of the dense particle that skipped it, so its
 * standard links are implied by that particle's 2 ll links, and only
 * visited dense particles add 2 ll links).  Pinned by brute force with and
 * without the variant.
 * Label = smallest 0-based input index in the group.
 * Neighbour search: particles sorted by a uniform grid of cells no smaller
 * than ll, so that friends lie in the same or adjacent cells.
 * Parity pinned: brute-force components, permutation and periodic-shift
 * invariance, lattice cases, isolated-particle fraction.
 */
int orc_fof3d(const orc_params* p, int64_t n, int pos_f64, const void* x, const void* y,
              const void* z, uint32_t* label) {
  if (n <= 0) return ORC_OK;
  if (n >= 0xFFFFFFFFll) return ORC_EINVAL;
  const double L = p->box;
  const double ll = p->b * L / cbrt((double)n);
  const double ll2 = ll * ll;
  int64_t* par = (int64_t*)malloc(sizeof(int64_t) * n);
  if (!par) return ORC_ENOMEM;
  for (int64_t i = 0; i < n; ++i) par[i] = i;

  int64_t nc = (int64_t)floor(L / (ll * (1.0 + 1e-9)));
  if (nc < 3) {
    for (int64_t i = 0; i < n; ++i)
      for (int64_t j = i + 1; j < n; ++j) {
        double dx = min_image(pos_at(x, pos_f64, j) - pos_at(x, pos_f64, i), L);
        double dy = min_image(pos_at(y, pos_f64, j) - pos_at(y, pos_f64, i), L);
        double dz = min_image(pos_at(z, pos_f64, j) - pos_at(z, pos_f64, i), L);
        if (sq3(dx, dy, dz) <= ll2) uf_union(par, i, j);
      }
  } else {
    /* (cell id, particle index) pairs sorted by cell, then index. */
    cellkey* key = (cellkey*)malloc(sizeof(cellkey) * n);
    if (!key) {
      free(par);
      return ORC_ENOMEM;
    }
    const double inv = (double)nc / L;
    for (int64_t i = 0; i < n; ++i) {
      int64_t c[3];
      const void* ax[3] = {x, y, z};
      for (int a = 0; a < 3; ++a) {
        int64_t ci = (int64_t)floor(pos_at(ax[a], pos_f64, i) * inv);
        if (ci < 0) ci = 0;
        if (ci >= nc) ci = nc - 1;
        c[a] = ci;
      }
      key[i].cell = (uint64_t)((c[2] * nc + c[1]) * nc + c[0]);
      key[i].idx = i;
    }
    qsort(key, (size_t)n, sizeof(cellkey), cmp_cellkey);
    int64_t s = 0;
    while (s < n) {
      uint64_t cell = key[s].cell;
      int64_t e = s;
      while (e < n && key[e].cell == cell) ++e;
      int64_t cx = (int64_t)(cell % (uint64_t)nc);
      int64_t cy = (int64_t)((cell / (uint64_t)nc) % (uint64_t)nc);
      int64_t cz = (int64_t)(cell / ((uint64_t)nc * (uint64_t)nc));
      for (int dz = -1; dz <= 1; ++dz)
        for (int dy = -1; dy <= 1; ++dy)
          for (int dx = -1; dx <= 1; ++dx) {
            int64_t nx = (cx + dx + nc) % nc, ny = (cy + dy + nc) % nc,
                    nz = (cz + dz + nc) % nc;
            uint64_t ncell = (uint64_t)((nz * nc + ny) * nc + nx);
            int64_t lo = 0, hi = n;
            while (lo < hi) {
              int64_t mid = (lo + hi) / 2;
              if (key[mid].cell < ncell)
                lo = mid + 1;
              else
                hi = mid;
            }
            for (int64_t a = s; a < e; ++a) {
              int64_t i = key[a].idx;
              double xi = pos_at(x, pos_f64, i), yi = pos_at(y, pos_f64, i),
                     zi = pos_at(z, pos_f64, i);
              for (int64_t b = lo; b < n && key[b].cell == ncell; ++b) {
                int64_t j = key[b].idx;
                if (j <= i) continue;
                double ddx = min_image(pos_at(x, pos_f64, j) - xi, L);
                double ddy = min_image(pos_at(y, pos_f64, j) - yi, L);
                double ddz = min_image(pos_at(z, pos_f64, j) - zi, L);
                if (sq3(ddx, ddy, ddz) <= ll2) uf_union(par, i, j);
              }
            }
          }
      s = e;
    }
    free(key);
  }
  if (p->fof_dense > 0) dense_links(p, n, pos_f64, x, y, z, ll, par);
  for (int64_t i = 0; i < n; ++i) label[i] = (uint32_t)uf_find(par, i);
  free(par);
  return ORC_OK;
}

/* ------------------------------------------------- phase-space metric ---- */
/*
 * Eq. 1 metric of one (sub)group: positions and velocities divided by the
 * group's position and velocity dispersions.  Readings: dispersions are the
 * 3D RMS about the mean, normalised by 1/n; positions are unwrapped about the
 * anchor (the member with the smallest input index) by the minimum image.
 * moments8 = centre (wrapped into [0,L)), mean velocity, sigma_x^2, sigma_v^2.
 * Normalised coordinates: fl32((u - mean u) * (1/sigma_x)) in FP64.
 * Returns ORC_EGEOMETRY when the unwrapped extent reaches L/2 on an axis.
 * Parity pinned: constructed sets with known moments, dyadic translation.
 */
int orc_node_normalise(const orc_params* p, int64_t nm, int pos_f64, const void* x,
                       const void* y, const void* z, const float* vx, const float* vy,
                       const float* vz, const int64_t* mem, float* xi6, double* mom) {
  const double L = p->box;
  const int sx = orc_position_shift(L);
  const void* ax[3] = {x, y, z};
  const float* av[3] = {vx, vy, vz};
  const int64_t a = mem[0];
  double xa[3];
  for (int c = 0; c < 3; ++c) xa[c] = pos_at(ax[c], pos_f64, a);
  double* u = (double*)malloc(sizeof(double) * 3 * (size_t)nm);
  if (!u) return ORC_ENOMEM;
  qsum qp, qv;
  memset(&qp, 0, sizeof qp);
  memset(&qv, 0, sizeof qv);
  double umin[3] = {0, 0, 0}, umax[3] = {0, 0, 0};
  for (int64_t k = 0; k < nm; ++k) {
    int64_t i = mem[k];
    int64_t q[3], w[3];
    for (int c = 0; c < 3; ++c) {
      double d = min_image(pos_at(ax[c], pos_f64, i) - xa[c], L);
      u[3 * k + c] = d;
      if (d < umin[c]) umin[c] = d;
      if (d > umax[c]) umax[c] = d;
      q[c] = quantise(d, sx);
      w[c] = quantise((double)av[c][i], VEL_SHIFT);
    }
    qsum_add(&qp, q[0], q[1], q[2]);
    qsum_add(&qv, w[0], w[1], w[2]);
  }
  for (int c = 0; c < 3; ++c)
    if (umax[c] - umin[c] >= 0.5 * L) {
      free(u);
      return ORC_EGEOMETRY;
    }
  double ubar[3], vbar[3], sx2, sv2;
  qsum_finish(&qp, sx, ubar, &sx2);
  qsum_finish(&qv, VEL_SHIFT, vbar, &sv2);
  for (int c = 0; c < 3; ++c) {
    double cc = xa[c] + ubar[c];
    if (cc < 0.0)
      cc += L;
    else if (cc >= L)
      cc -= L;
    mom[c] = cc;
    mom[3 + c] = vbar[c];
  }
  mom[6] = sx2;
  mom[7] = sv2;
  if (xi6 && sx2 > 0.0 && sv2 > 0.0) {
    double isx = 1.0 / sqrt(sx2), isv = 1.0 / sqrt(sv2);
    for (int64_t k = 0; k < nm; ++k) {
      int64_t i = mem[k];
      for (int c = 0; c < 3; ++c) {
        xi6[6 * k + c] = (float)((u[3 * k + c] - ubar[c]) * isx);
        xi6[6 * k + 3 + c] = (float)(((double)av[c][i] - vbar[c]) * isv);
      }
    }
  }
  free(u);
  return ORC_OK;
}

/*
 * Nearest-neighbour squared phase-space distance of every point (Section
 * 3.2): dmin_i = min over j != i.  Parity pinned against brute force in
 * FP64 on the same FP32 coordinates.
 */
void orc_nn6d(int64_t n, const float* xi6, float* dmin) {
  for (int64_t i = 0; i < n; ++i) {
    float best = INFINITY;
    for (int64_t j = 0; j < n; ++j) {
      if (j == i) continue;
      float d = d2_6d(xi6 + 6 * i, xi6 + 6 * j);
      if (d < best) best = d;
    }
    dmin[i] = best;
  }
}

/*
 * Adaptive linking length (Section 3.2): chosen so that a fraction f of the
 * particles have a friend within it.  Reading: ell^2 is the k-th smallest
 * nearest-neighbour distance with k = ceil(f n) (FP64) and friendship is
 * inclusive (d^2 <= ell^2), so at least k particles are linked.
 * Pinned by the linked-fraction invariant.
 */
float orc_ell2(int64_t n, const float* dmin, double f) {
  float* s = (float*)malloc(sizeof(float) * (size_t)n);
  memcpy(s, dmin, sizeof(float) * (size_t)n);
  qsort(s, (size_t)n, sizeof(float), cmp_f32);
  int64_t k = (int64_t)ceil(f * (double)n);
  if (k < 1) k = 1;
  if (k > n) k = n;
  float r = s[k - 1];
  free(s);
  return r;
}

/*
 * SplitMix64 (Steele, Lea & Flood 2014): the output for counter x.  It draws
 * the random subset of Section 3.2 from the particle's input index.
 */
static uint64_t splitmix64(uint64_t x) {
  uint64_t z = x + 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

/*
 * Subset membership for the linking length of a node of n > m particles
 * (Section 3.2: in large groups the nearest neighbours are found for a random
 * subset of 10^4 only).  Reading: each particle is drawn independently with
 * probability m / n, decided exactly as splitmix64(index) * n < m * 2^64
 * (128-bit integers), so the subset's expected size is m.
 */
int orc_in_subset(uint64_t index, int64_t n, int64_t m) {
  if (m <= 0 || n <= m) return 1;
  unsigned __int128 lhs = (unsigned __int128)splitmix64(index) * (unsigned __int128)n;
  unsigned __int128 rhs = (unsigned __int128)m << 64;
  return lhs < rhs;
}

/*
 * Linking length from a subset: the nearest-neighbour distance (against every
 * particle of the node) of each subset member, and ell^2 = the k-th smallest
 * of those, k = ceil(f n_sub) (orc_ell2).  An empty subset (possible only
 * by chance) falls back to every particle.
 */
static float ell2_subset(int64_t n, const float* xi6, const int64_t* mem, int32_t m, double f) {
  int64_t ns = 0;
  for (int64_t i = 0; i < n; ++i) ns += orc_in_subset((uint64_t)mem[i], n, m);
  if (ns == 0) ns = n, m = 0;
  float* d = (float*)malloc(sizeof(float) * (size_t)ns);
  int64_t q = 0;
  for (int64_t i = 0; i < n; ++i) {
    if (!orc_in_subset((uint64_t)mem[i], n, m)) continue;
    float best = INFINITY;
    for (int64_t j = 0; j < n; ++j) {
      if (j == i) continue;
      float dd = d2_6d(xi6 + 6 * i, xi6 + 6 * j);
      if (dd < best) best = dd;
    }
    d[q++] = best;
  }
  float r = orc_ell2(ns, d, f);
  free(d);
  return r;
}

/* 6D FOF at ell^2: comp[i] = smallest local index of i's component. */
/*
 * The same two definitions for a range of particles, so that a caller can
 * split one node's O(n^2) work over several threads: the nearest-neighbour
 * d^2 of particles [i0, i1) among all n, and the friend pairs (i, j > i) with
 * d^2 <= ell2 for i in [i0, i1), at most `cap` of them (returns the number
 * found, which may exceed cap; only the first cap are written).
 */
void orc_nn6d_range(int64_t n, const float* xi6, int64_t i0, int64_t i1, float* dmin) {
  for (int64_t i = i0; i < i1; ++i) {
    float best = INFINITY;
    for (int64_t j = 0; j < n; ++j) {
      if (j == i) continue;
      float d = d2_6d(xi6 + 6 * i, xi6 + 6 * j);
      if (d < best) best = d;
    }
    dmin[i - i0] = best;
  }
}

int64_t orc_friends6d_range(int64_t n, const float* xi6, float ell2, int64_t i0, int64_t i1,
                            int64_t cap, int64_t* pairs) {
  int64_t k = 0;
  for (int64_t i = i0; i < i1; ++i)
    for (int64_t j = i + 1; j < n; ++j)
      if (d2_6d(xi6 + 6 * i, xi6 + 6 * j) <= ell2) {
        if (k < cap) {
          pairs[2 * k] = i;
          pairs[2 * k + 1] = j;
        }
        ++k;
      }
  return k;
}

void orc_fof6d(int64_t n, const float* xi6, float ell2, int64_t* comp) {
  for (int64_t i = 0; i < n; ++i) comp[i] = i;
  for (int64_t i = 0; i < n; ++i)
    for (int64_t j = i + 1; j < n; ++j)
      if (d2_6d(xi6 + 6 * i, xi6 + 6 * j) <= ell2) uf_union(comp, i, j);
  for (int64_t i = 0; i < n; ++i) comp[i] = uf_find(comp, i);
}

/* ------------------------------------------------- 6D hierarchy ---------- */

typedef struct {
  int64_t n, cap;
  int32_t *parent, *level, *first_child, *n_children;
  uint32_t *count, *canon, *fof, *flags;
  double* mom; /* 8 per node */
  float* ell2;
} nodevec;

static int nodevec_push(nodevec* v) {
  if (v->n == v->cap) {
    int64_t c = v->cap ? 2 * v->cap : 1024;
#define GROW(f, t)                                       \
  do {                                                   \
    void* q = realloc(v->f, sizeof(t) * (size_t)c);      \
    if (!q) return -1;                                   \
    v->f = (t*)q;                                        \
  } while (0)
    GROW(parent, int32_t);
    GROW(level, int32_t);
    GROW(first_child, int32_t);
    GROW(n_children, int32_t);
    GROW(count, uint32_t);
    GROW(canon, uint32_t);
    GROW(fof, uint32_t);
    GROW(flags, uint32_t);
    GROW(ell2, float);
    {
      void* q = realloc(v->mom, sizeof(double) * 8 * (size_t)c);
      if (!q) return -1;
      v->mom = (double*)q;
    }
#undef GROW
    v->cap = c;
  }
  v->n++;
  return 0;
}

static void nodevec_free(nodevec* v) {
  free(v->parent); free(v->level); free(v->first_child); free(v->n_children);
  free(v->count); free(v->canon); free(v->fof); free(v->flags); free(v->mom);
  free(v->ell2);
}

/*
 * Recursive phase-space FOF hierarchy (Section 3.2) for every 3D FOF group
 * with at least min_members particles.  For each (sub)group: Eq. 1 metric,
 * adaptive ell, 6D FOF; components with at least min_members particles become
 * subgroups, recursively, until none remains.  Readings: a node whose
 * dispersions vanish is a leaf; a node whose only subgroup would contain all
 * of its particles is a leaf (the recursion would not change).
 * Node order: breadth first -- level by level, children of a node in the
 * order of their smallest input index, nodes of a level in their parents'
 * order.  deepest[i] = deepest node holding particle i, or -1.
 * Parity pinned: linked fraction at every node, brute-force NN, 2^k scaling
 * invariance, two velocity-separated blobs.
 */
int orc_refine6d(const orc_params* p, int64_t n, int pos_f64, const void* x,
                 const void* y, const void* z, const float* vx, const float* vy,
                 const float* vz, const uint32_t* label, int64_t node_cap,
                 orc_nodes* out, int32_t* deepest, int64_t* n_nodes) {
  const int64_t mm = p->min_members;
  for (int64_t i = 0; i < n; ++i) deepest[i] = -1;
  /* group members, ascending index, groups in label order */
  int64_t* cnt = (int64_t*)calloc((size_t)n + 1, sizeof(int64_t));
  for (int64_t i = 0; i < n; ++i) cnt[label[i]]++;
  int64_t* cur = (int64_t*)malloc(sizeof(int64_t) * (size_t)(n ? n : 1));
  int64_t* curoff = (int64_t*)malloc(sizeof(int64_t) * (size_t)(n + 1));
  int64_t* curnode = (int64_t*)malloc(sizeof(int64_t) * (size_t)(n + 1));
  int64_t* start = (int64_t*)malloc(sizeof(int64_t) * (size_t)(n + 1));
  nodevec nv;
  memset(&nv, 0, sizeof nv);
  int64_t ncur = 0, m = 0;
  {
    int64_t acc = 0;
    for (int64_t g = 0; g < n; ++g) {
      start[g] = acc;
      if (cnt[g] >= mm) acc += cnt[g];
    }
    for (int64_t i = 0; i < n; ++i) {
      int64_t g = label[i];
      if (cnt[g] >= mm) cur[start[g]++] = i;
    }
    for (int64_t g = 0; g < n; ++g)
      if (cnt[g] >= mm) {
        nodevec_push(&nv);
        int64_t k = nv.n - 1;
        nv.parent[k] = -1;
        nv.level[k] = 0;
        nv.count[k] = (uint32_t)cnt[g];
        nv.canon[k] = (uint32_t)g;
        nv.fof[k] = (uint32_t)g;
        curoff[ncur] = m;
        curnode[ncur] = k;
        m += cnt[g];
        ncur++;
      }
    curoff[ncur] = m;
  }
  free(cnt);
  free(start);
  int rc = ORC_OK;
  int64_t* nxt = (int64_t*)malloc(sizeof(int64_t) * (size_t)(n ? n : 1));
  int64_t* nxtoff = (int64_t*)malloc(sizeof(int64_t) * (size_t)(n + 1));
  int64_t* nxtnode = (int64_t*)malloc(sizeof(int64_t) * (size_t)(n + 1));
  for (int lev = 0; ncur > 0; ++lev) {
    if (lev >= p->max_levels) {
      rc = ORC_EINVAL;
      break;
    }
    int64_t nn = 0, mnext = 0;
    for (int64_t t = 0; t < ncur; ++t) {
      int64_t k = curnode[t];
      const int64_t* mem = cur + curoff[t];
      int64_t nm = curoff[t + 1] - curoff[t];
      for (int64_t q = 0; q < nm; ++q) deepest[mem[q]] = (int32_t)k;
      float* xi = (float*)malloc(sizeof(float) * 6 * (size_t)nm);
      double mom[8];
      int r = orc_node_normalise(p, nm, pos_f64, x, y, z, vx, vy, vz, mem, xi, mom);
      if (r != ORC_OK) {
        free(xi);
        rc = r;
        goto done;
      }
      memcpy(nv.mom + 8 * k, mom, sizeof mom);
      nv.first_child[k] = -1;
      nv.n_children[k] = 0;
      nv.flags[k] = 0;
      nv.ell2[k] = -1.0f;
      if (!(mom[6] > 0.0) || !(mom[7] > 0.0)) {
        nv.flags[k] = ORC_NODE_LEAF | ORC_NODE_DEGENERATE;
        free(xi);
        continue;
      }
      float l2;
      if (p->ell_subset > 0 && nm > p->ell_subset) {
        l2 = ell2_subset(nm, xi, mem, p->ell_subset, p->f);
      } else {
        float* dmin = (float*)malloc(sizeof(float) * (size_t)nm);
        orc_nn6d(nm, xi, dmin);
        l2 = orc_ell2(nm, dmin, p->f);
        free(dmin);
      }
      nv.ell2[k] = l2;
      int64_t* comp = (int64_t*)malloc(sizeof(int64_t) * (size_t)nm);
      int64_t* csz = (int64_t*)calloc((size_t)nm, sizeof(int64_t));
      orc_fof6d(nm, xi, l2, comp);
      free(xi);
      for (int64_t q = 0; q < nm; ++q) csz[comp[q]]++;
      /* children in order of their smallest member (= smallest input index) */
      int64_t nch = 0, whole = 0;
      for (int64_t q = 0; q < nm; ++q)
        if (comp[q] == q && csz[q] >= mm) {
          nch++;
          if (csz[q] == nm) whole = 1;
        }
      if (nch == 0 || whole) {
        nv.flags[k] = ORC_NODE_LEAF | (whole ? ORC_NODE_WHOLE : 0u);
        free(comp);
        free(csz);
        continue;
      }
      nv.first_child[k] = (int32_t)nv.n;
      nv.n_children[k] = (int32_t)nch;
      /* child slot of each root, members appended in ascending order */
      int64_t* slot = (int64_t*)malloc(sizeof(int64_t) * (size_t)nm);
      int64_t base = mnext;
      for (int64_t q = 0; q < nm; ++q) {
        if (comp[q] == q && csz[q] >= mm) {
          if (nodevec_push(&nv)) {
            rc = ORC_ENOMEM;
            goto done;
          }
          int64_t c = nv.n - 1;
          nv.parent[c] = (int32_t)k;
          nv.level[c] = lev + 1;
          nv.count[c] = (uint32_t)csz[q];
          nv.canon[c] = (uint32_t)mem[q];
          nv.fof[c] = nv.fof[k];
          nxtoff[nn] = base;
          nxtnode[nn] = c;
          slot[q] = base;
          base += csz[q];
          nn++;
        }
      }
      for (int64_t q = 0; q < nm; ++q) {
        int64_t r0 = comp[q];
        if (csz[r0] >= mm) nxt[slot[r0]++] = mem[q];
      }
      mnext = base;
      free(slot);
      free(comp);
      free(csz);
    }
    nxtoff[nn] = mnext;
    {
      int64_t* t;
      t = cur; cur = nxt; nxt = t;
      t = curoff; curoff = nxtoff; nxtoff = t;
      t = curnode; curnode = nxtnode; nxtnode = t;
    }
    ncur = nn;
  }
done:
  *n_nodes = nv.n;
  if (rc == ORC_OK && nv.n > node_cap) rc = ORC_ECAPACITY;
  if (rc == ORC_OK) {
    for (int64_t k = 0; k < nv.n; ++k) {
      out->parent[k] = nv.parent[k];
      out->level[k] = nv.level[k];
      out->first_child[k] = nv.first_child[k];
      out->n_children[k] = nv.n_children[k];
      out->count[k] = nv.count[k];
      out->canon[k] = nv.canon[k];
      out->fof[k] = nv.fof[k];
      out->flags[k] = nv.flags[k];
      out->cx[k] = nv.mom[8 * k + 0];
      out->cy[k] = nv.mom[8 * k + 1];
      out->cz[k] = nv.mom[8 * k + 2];
      out->vx[k] = nv.mom[8 * k + 3];
      out->vy[k] = nv.mom[8 * k + 4];
      out->vz[k] = nv.mom[8 * k + 5];
      out->sx2[k] = nv.mom[8 * k + 6];
      out->sv2[k] = nv.mom[8 * k + 7];
      out->ell2[k] = nv.ell2[k];
    }
  }
  nodevec_free(&nv);
  free(cur); free(curoff); free(curnode); free(nxt); free(nxtoff); free(nxtnode);
  return rc;
}

/* ------------------------------------------------- seeds and assignment -- */

/* Seed set of every node: the distinct merged-halo ids of the leaves below. */
typedef struct {
  int64_t* off; /* n_nodes + 1 */
  int32_t* ids; /* sorted ascending within a node */
} seedsets;

static int cmp_i32(const void* a, const void* b) {
  int32_t x = *(const int32_t*)a, y = *(const int32_t*)b;
  return x < y ? -1 : x > y;
}

static int build_seedsets(const orc_nodes* nd, int64_t nn, const int32_t* node_seed,
                          const int32_t* merged, seedsets* ss) {
  /* sizes bottom-up (children have larger indices than parents) */
  int64_t* sz = (int64_t*)calloc((size_t)nn, sizeof(int64_t));
  int32_t** lists = (int32_t**)calloc((size_t)nn, sizeof(int32_t*));
  for (int64_t k = nn - 1; k >= 0; --k) {
    if (nd->n_children[k] == 0) {
      lists[k] = (int32_t*)malloc(sizeof(int32_t));
      lists[k][0] = merged[node_seed[k]];
      sz[k] = 1;
    } else {
      int64_t tot = 0;
      for (int32_t c = 0; c < nd->n_children[k]; ++c) tot += sz[nd->first_child[k] + c];
      int32_t* l = (int32_t*)malloc(sizeof(int32_t) * (size_t)tot);
      int64_t w = 0;
      for (int32_t c = 0; c < nd->n_children[k]; ++c) {
        int64_t ch = nd->first_child[k] + c;
        memcpy(l + w, lists[ch], sizeof(int32_t) * (size_t)sz[ch]);
        w += sz[ch];
      }
      qsort(l, (size_t)tot, sizeof(int32_t), cmp_i32);
      int64_t u = 0;
      for (int64_t q = 0; q < tot; ++q)
        if (u == 0 || l[u - 1] != l[q]) l[u++] = l[q];
      lists[k] = l;
      sz[k] = u;
    }
  }
  ss->off = (int64_t*)malloc(sizeof(int64_t) * (size_t)(nn + 1));
  int64_t tot = 0;
  for (int64_t k = 0; k < nn; ++k) {
    ss->off[k] = tot;
    tot += sz[k];
  }
  ss->off[nn] = tot;
  ss->ids = (int32_t*)malloc(sizeof(int32_t) * (size_t)(tot ? tot : 1));
  for (int64_t k = 0; k < nn; ++k) {
    memcpy(ss->ids + ss->off[k], lists[k], sizeof(int32_t) * (size_t)sz[k]);
    free(lists[k]);
  }
  free(lists);
  free(sz);
  return 0;
}

typedef struct {
  int64_t n, cap;
  int64_t* v;
} ivec;

static void ivec_push(ivec* a, int64_t x) {
  if (a->n == a->cap) {
    a->cap = a->cap ? 2 * a->cap : 16;
    a->v = (int64_t*)realloc(a->v, sizeof(int64_t) * (size_t)a->cap);
  }
  a->v[a->n++] = x;
}

/*
 * "Current" properties of a halo from the particles assigned to it so far
 * (Section 3.3): velocity dispersion sigma_v^2 (3D, exact fixed-point sums)
 * and vmax^2 = G m max_k k / max(r_k, eps), r_k the k-th smallest distance
 * from the seed position.  Evaluated as G m sqrt(max_k k^2 / max(r_k^2, eps^2)).
 */
static void halo_current(const orc_params* p, int pos_f64, const void* x, const void* y,
                         const void* z, const float* vx, const float* vy, const float* vz,
                         const ivec* mem, const double xs[3], double* sv2, double* vmax2) {
  qsum qv;
  memset(&qv, 0, sizeof qv);
  rad_t* r = (rad_t*)malloc(sizeof(rad_t) * (size_t)(mem->n ? mem->n : 1));
  for (int64_t k = 0; k < mem->n; ++k) {
    int64_t i = mem->v[k];
    qsum_add(&qv, quantise((double)vx[i], VEL_SHIFT), quantise((double)vy[i], VEL_SHIFT),
             quantise((double)vz[i], VEL_SHIFT));
    double dx = min_image(pos_at(x, pos_f64, i) - xs[0], p->box);
    double dy = min_image(pos_at(y, pos_f64, i) - xs[1], p->box);
    double dz = min_image(pos_at(z, pos_f64, i) - xs[2], p->box);
    r[k].r2 = sq3(dx, dy, dz);
    r[k].idx = i;
  }
  double vm[3];
  if (mem->n > 0)
    qsum_finish(&qv, VEL_SHIFT, vm, sv2);
  else
    *sv2 = 0.0;
  qsort(r, (size_t)mem->n, sizeof(rad_t), cmp_rad);
  double e2 = p->softening * p->softening, best = 0.0;
  for (int64_t k = 0; k < mem->n; ++k) {
    double kk = (double)(k + 1);
    double t = (kk * kk) / fmax(r[k].r2, e2);
    if (t > best) best = t;
  }
  *vmax2 = p->G * p->particle_mass * sqrt(best);
  free(r);
}

/* Eq. 3 squared distance from halo h (metric inv_rdyn2, inv_sv2) to a point. */
static double eq3_d2(double box, const double xh[3], const double vh[3], double inv_rd2,
                     double inv_sv2, double px, double py, double pz, double qx, double qy,
                     double qz) {
  double dx = min_image(px - xh[0], box), dy = min_image(py - xh[1], box),
         dz = min_image(pz - xh[2], box);
  double ux = qx - vh[0], uy = qy - vh[1], uz = qz - vh[2];
  return fma(sq3(dx, dy, dz), inv_rd2, sq3(ux, uy, uz) * inv_sv2);
}

static double dyn_const(const orc_params* p) { return (4.0 * M_PI / 3.0) * p->G * p->rho_vir; }

/*
 * Seeds, seed merging, hierarchical assignment and host/subhalo relation
 * (Sections 3.3-3.4).
 *  - One seed per leaf node; seed ids follow node order.
 *  - Merging (Eq. 2): within a 3D FOF group, seeds are visited by decreasing
 *    size (ties: lower id); a seed b merges into the closest already-kept
 *    seed a when |dx|^2/mu_x^2 + |dv|^2/mu_v^2 < merge_q2, mu = sigma/sqrt(n)
 *    of b (the smaller seed).  The kept seed keeps its position/velocity.
 *    merged_into[s] = s for kept seeds.
 *  - Assignment, bottom-up level by level: the particles of a node that lie
 *    in none of its subgroups go to its only seed, or, when it holds several,
 *    to the closest by Eq. 3 (ties: lower id), using each seed's current
 *    sigma_v and vmax computed from the particles assigned before the level;
 *    r_dyn = vmax / sqrt(4/3 pi G rho_vir).  Seed positions and velocities
 *    stay at the leaf means (reading of "current").
 *  - Host/sub: within a FOF group, kept halos by decreasing assigned count
 *    (ties: lower id); each halo after the first becomes a sub of the closest
 *    earlier halo by Eq. 3 with that halo's final metric (ties: lower id).
 * Parity: single-seed and two-seed pins; merge threshold pin; the merge
 * visit and the host choice are checked against brute-force numpy forms of
 * the same readings (tests/test_oracle_readings.py).  The readings of merge
 * order, "current" and host choice themselves are not fixed by the paper.
 */
int orc_assign(const orc_params* p, int64_t n, int pos_f64, const void* x, const void* y,
               const void* z, const float* vx, const float* vy, const float* vz,
               const orc_nodes* nd, int64_t nn, const int32_t* deepest, int64_t halo_cap,
               orc_halos* h, int32_t* halo_of, int64_t* n_halos) {
  int64_t ns = 0;
  for (int64_t k = 0; k < nn; ++k)
    if (nd->n_children[k] == 0) ns++;
  *n_halos = ns;
  if (ns > halo_cap) return ORC_ECAPACITY;
  int32_t* node_seed = (int32_t*)malloc(sizeof(int32_t) * (size_t)(nn ? nn : 1));
  ns = 0;
  for (int64_t k = 0; k < nn; ++k) {
    node_seed[k] = -1;
    if (nd->n_children[k] == 0) {
      h->seed_node[ns] = (int32_t)k;
      h->fof[ns] = nd->fof[k];
      h->xs[ns] = nd->cx[k];
      h->ys[ns] = nd->cy[k];
      h->zs[ns] = nd->cz[k];
      h->vxs[ns] = nd->vx[k];
      h->vys[ns] = nd->vy[k];
      h->vzs[ns] = nd->vz[k];
      node_seed[k] = (int32_t)ns;
      ns++;
    }
  }
  /* ---- merging, per FOF group ---- */
  int64_t* ord = (int64_t*)malloc(sizeof(int64_t) * (size_t)(ns ? ns : 1));
  for (int64_t s = 0; s < ns; ++s) ord[s] = s;
  {
    grpkey* gk = (grpkey*)malloc(sizeof(grpkey) * (size_t)(ns ? ns : 1));
    for (int64_t s = 0; s < ns; ++s) {
      gk[s].fof = h->fof[s];
      gk[s].size = nd->count[h->seed_node[s]];
      gk[s].id = s;
    }
    qsort(gk, (size_t)ns, sizeof(grpkey), cmp_grpkey);
    for (int64_t s = 0; s < ns; ++s) ord[s] = gk[s].id;
    free(gk);
  }
  int64_t* kept = (int64_t*)malloc(sizeof(int64_t) * (size_t)(ns ? ns : 1));
  for (int64_t s0 = 0; s0 < ns;) {
    int64_t s1 = s0;
    while (s1 < ns && h->fof[ord[s1]] == h->fof[ord[s0]]) ++s1;
    int64_t nk = 0;
    for (int64_t t = s0; t < s1; ++t) {
      int64_t b = ord[t];
      int64_t kb = h->seed_node[b];
      double cb = (double)nd->count[kb];
      double sx2 = nd->sx2[kb], sv2 = nd->sv2[kb];
      int64_t best = -1;
      double bq = INFINITY;
      if (sx2 > 0.0 && sv2 > 0.0) {
        double imx = cb / sx2, imv = cb / sv2;
        for (int64_t q = 0; q < nk; ++q) {
          int64_t a = kept[q];
          double dx = min_image(h->xs[b] - h->xs[a], p->box);
          double dy = min_image(h->ys[b] - h->ys[a], p->box);
          double dz = min_image(h->zs[b] - h->zs[a], p->box);
          double ux = h->vxs[b] - h->vxs[a], uy = h->vys[b] - h->vys[a],
                 uz = h->vzs[b] - h->vzs[a];
          double qq = fma(sq3(dx, dy, dz), imx, sq3(ux, uy, uz) * imv);
          if (qq < bq || (qq == bq && a < best)) {
            bq = qq;
            best = a;
          }
        }
      }
      if (best >= 0 && bq < p->merge_q2) {
        h->merged_into[b] = (int32_t)best;
      } else {
        h->merged_into[b] = (int32_t)b;
        kept[nk++] = b;
      }
    }
    s0 = s1;
  }
  free(kept);

  seedsets ss;
  build_seedsets(nd, nn, node_seed, h->merged_into, &ss);

  /* own particles of each node, ascending index */
  int64_t* ooff = (int64_t*)calloc((size_t)nn + 1, sizeof(int64_t));
  for (int64_t i = 0; i < n; ++i)
    if (deepest[i] >= 0) ooff[deepest[i] + 1]++;
  for (int64_t k = 0; k < nn; ++k) ooff[k + 1] += ooff[k];
  int64_t* own = (int64_t*)malloc(sizeof(int64_t) * (size_t)(ooff[nn] ? ooff[nn] : 1));
  {
    int64_t* fill = (int64_t*)malloc(sizeof(int64_t) * (size_t)(nn ? nn : 1));
    for (int64_t k = 0; k < nn; ++k) fill[k] = ooff[k];
    for (int64_t i = 0; i < n; ++i)
      if (deepest[i] >= 0) own[fill[deepest[i]]++] = i;
    free(fill);
  }
  for (int64_t i = 0; i < n; ++i) halo_of[i] = -1;
  ivec* mem = (ivec*)calloc((size_t)(ns ? ns : 1), sizeof(ivec));
  double* cur_sv2 = (double*)malloc(sizeof(double) * (size_t)(ns ? ns : 1));
  double* cur_vm2 = (double*)malloc(sizeof(double) * (size_t)(ns ? ns : 1));
  uint8_t* cand = (uint8_t*)malloc((size_t)(ns ? ns : 1));
  int32_t maxlev = -1;
  for (int64_t k = 0; k < nn; ++k)
    if (nd->level[k] > maxlev) maxlev = nd->level[k];
  const double cdyn = dyn_const(p);
  for (int32_t lev = maxlev; lev >= 0; --lev) {
    memset(cand, 0, (size_t)(ns ? ns : 1));
    for (int64_t k = 0; k < nn; ++k)
      if (nd->level[k] == lev && ss.off[k + 1] - ss.off[k] >= 2)
        for (int64_t q = ss.off[k]; q < ss.off[k + 1]; ++q) cand[ss.ids[q]] = 1;
    for (int64_t s = 0; s < ns; ++s)
      if (cand[s]) {
        double xs[3] = {h->xs[s], h->ys[s], h->zs[s]};
        halo_current(p, pos_f64, x, y, z, vx, vy, vz, &mem[s], xs, &cur_sv2[s], &cur_vm2[s]);
      }
    for (int64_t k = 0; k < nn; ++k) {
      if (nd->level[k] != lev) continue;
      int64_t nsk = ss.off[k + 1] - ss.off[k];
      const int32_t* ids = ss.ids + ss.off[k];
      for (int64_t q = ooff[k]; q < ooff[k + 1]; ++q) {
        int64_t i = own[q];
        int32_t best = ids[0];
        if (nsk > 1) {
          double bd = INFINITY;
          best = -1;
          for (int64_t t = 0; t < nsk; ++t) {
            int32_t s = ids[t];
            double xh[3] = {h->xs[s], h->ys[s], h->zs[s]};
            double vh[3] = {h->vxs[s], h->vys[s], h->vzs[s]};
            double d = eq3_d2(p->box, xh, vh, cdyn / cur_vm2[s], 1.0 / fmax(cur_sv2[s], 1e-300),
                              pos_at(x, pos_f64, i), pos_at(y, pos_f64, i),
                              pos_at(z, pos_f64, i), (double)vx[i], (double)vy[i],
                              (double)vz[i]);
            if (d < bd || (d == bd && s < best)) {
              bd = d;
              best = s;
            }
          }
        }
        halo_of[i] = best;
        ivec_push(&mem[best], i);
      }
    }
  }
  /* final metric of kept halos, host/sub relation */
  for (int64_t s = 0; s < ns; ++s) {
    h->n_assigned[s] = (uint32_t)mem[s].n;
    h->host[s] = -1;
    if (h->merged_into[s] == s) {
      double xs[3] = {h->xs[s], h->ys[s], h->zs[s]};
      /* member lists were filled in level order; sort for a canonical order */
      qsort(mem[s].v, (size_t)mem[s].n, sizeof(int64_t), cmp_u64);
      halo_current(p, pos_f64, x, y, z, vx, vy, vz, &mem[s], xs, &h->sv2[s], &h->vmax2[s]);
    } else {
      h->sv2[s] = 0.0;
      h->vmax2[s] = 0.0;
    }
  }
  /* kept halos of each FOF, by (n_assigned desc, id asc) */
  {
    int64_t nk = 0;
    grpkey* gk = (grpkey*)malloc(sizeof(grpkey) * (size_t)(ns ? ns : 1));
    for (int64_t s = 0; s < ns; ++s)
      if (h->merged_into[s] == s) {
        gk[nk].fof = h->fof[s];
        gk[nk].size = h->n_assigned[s];
        gk[nk].id = s;
        nk++;
      }
    qsort(gk, (size_t)nk, sizeof(grpkey), cmp_grpkey);
    for (int64_t a = 0; a < nk; ++a) ord[a] = gk[a].id;
    free(gk);
    for (int64_t a0 = 0; a0 < nk;) {
      int64_t a1 = a0;
      while (a1 < nk && h->fof[ord[a1]] == h->fof[ord[a0]]) ++a1;
      for (int64_t t = a0 + 1; t < a1; ++t) {
        int64_t s = ord[t];
        double bd = INFINITY;
        int64_t best = -1;
        /* candidates: halos of the group with strictly more assigned
           particles (Section 3.4); none -> the halo is a host itself */
        for (int64_t u = a0; u < t; ++u) {
          int64_t H = ord[u];
          if (h->n_assigned[H] <= h->n_assigned[s]) break;
          double xh[3] = {h->xs[H], h->ys[H], h->zs[H]};
          double vh[3] = {h->vxs[H], h->vys[H], h->vzs[H]};
          double d = eq3_d2(p->box, xh, vh, cdyn / h->vmax2[H], 1.0 / fmax(h->sv2[H], 1e-300),
                            h->xs[s], h->ys[s], h->zs[s], h->vxs[s], h->vys[s], h->vzs[s]);
          if (d < bd || (d == bd && H < best)) {
            bd = d;
            best = H;
          }
        }
        h->host[s] = (int32_t)best;
      }
      a0 = a1;
    }
  }
  for (int64_t s = 0; s < ns; ++s) free(mem[s].v);
  free(mem); free(cur_sv2); free(cur_vm2); free(cand); free(own); free(ooff);
  free(ss.off); free(ss.ids); free(ord); free(node_seed);
  return ORC_OK;
}

/* ------------------------------------------------- unbinding ------------- */

/* Children of every halo in the host/sub forest (CSR, ascending ids). */
typedef struct {
  int64_t* off;
  int64_t* ids;
} halo_tree;

static void build_halo_tree(int64_t ns, const int32_t* host, halo_tree* t) {
  t->off = (int64_t*)calloc((size_t)ns + 1, sizeof(int64_t));
  for (int64_t s = 0; s < ns; ++s)
    if (host[s] >= 0) t->off[host[s] + 1]++;
  for (int64_t s = 0; s < ns; ++s) t->off[s + 1] += t->off[s];
  t->ids = (int64_t*)malloc(sizeof(int64_t) * (size_t)(t->off[ns] ? t->off[ns] : 1));
  int64_t* fill = (int64_t*)malloc(sizeof(int64_t) * (size_t)(ns ? ns : 1));
  for (int64_t s = 0; s < ns; ++s) fill[s] = t->off[s];
  for (int64_t s = 0; s < ns; ++s)
    if (host[s] >= 0) t->ids[fill[host[s]]++] = s;
  free(fill);
}

/* Members of S(h): the particles of h and of every halo below it, ascending. */
static void subtree_members(const halo_tree* t, const int64_t* hoff, const int64_t* hmem,
                            int64_t root, ivec* out, ivec* stack) {
  out->n = 0;
  stack->n = 0;
  ivec_push(stack, root);
  while (stack->n > 0) {
    int64_t s = stack->v[--stack->n];
    for (int64_t q = hoff[s]; q < hoff[s + 1]; ++q) ivec_push(out, hmem[q]);
    for (int64_t q = t->off[s]; q < t->off[s + 1]; ++q) ivec_push(stack, t->ids[q]);
  }
  qsort(out->v, (size_t)out->n, sizeof(int64_t), cmp_u64);
}

/*
 * Potential of each target from a source list, excluding the target itself:
 * phi = -G m sum 1/sqrt(r^2 + eps^2) (Plummer softening; the paper does not
 * state a softening -- reading).  Exact direct sum in FP64 with Neumaier
 * compensation, sources in the given order.  phi_abs = |phi|.
 * Pinned: two-particle closed form, analytic NFW potential.
 */
void orc_phi_points(const orc_params* p, int pos_f64, const void* x, const void* y,
                    const void* z, const int64_t* src, int64_t nsrc, const int64_t* tgt,
                    int64_t ntgt, double* phi) {
  const double e2 = p->softening * p->softening;
  for (int64_t t = 0; t < ntgt; ++t) {
    int64_t i = tgt[t];
    double xi = pos_at(x, pos_f64, i), yi = pos_at(y, pos_f64, i), zi = pos_at(z, pos_f64, i);
    double s = 0.0, c = 0.0;
    for (int64_t q = 0; q < nsrc; ++q) {
      int64_t j = src[q];
      if (j == i) continue;
      double dx = min_image(pos_at(x, pos_f64, j) - xi, p->box);
      double dy = min_image(pos_at(y, pos_f64, j) - yi, p->box);
      double dz = min_image(pos_at(z, pos_f64, j) - zi, p->box);
      double term = 1.0 / sqrt(sq3(dx, dy, dz) + e2);
      double u = s + term;
      if (fabs(s) >= fabs(term))
        c += (s - u) + term;
      else
        c += (term - u) + s;
      s = u;
    }
    phi[t] = -p->G * p->particle_mass * (s + c);
  }
}

/*
 * Single-pass unbinding (Section 3.5.3): a particle assigned to h is bound
 * when 1/2 |v - v_bulk|^2 + phi < 0, phi from all particles of S(h) (h with
 * its subhalos, the mass convention of Section 3.4) and v_bulk the mean
 * velocity of S(h) (exact fixed-point sums).  A halo is valid when the bound
 * fraction of S(h) is at least unbound_threshold.  The potential is the exact
 * direct sum in place of the paper's Barnes-Hut tree (Appendix B).
 * phi_abs[i] = |phi_i| is returned for the error band of a comparison.
 *
 * Major mergers (Section 3.5.3, parameter MP of Table 2; off when
 * major_merger = 0): the particles of a subhalo h whose merger ratio with its
 * host, |S(h)| / |S(host)| (masses with substructure, as in Section 3.4), is
 * at least MP take their potential from the merging system S(t), where t is
 * reached from h by following host links while each link is such a major
 * merger (reading: the system is the outermost halo joined by major
 * mergers).  The paper changes only the potential, so the kinetic term keeps
 * h's own v_bulk (reading), and a particle can only gain boundness.  Pinned:
 * MP = 0 and MP > 1 leave every output unchanged; with MP no flag turns
 * unbound and no potential gets shallower; a two-clump case against a
 * brute-force numpy evaluation.
 */
int orc_unbind(const orc_params* p, int64_t n, int pos_f64, const void* x, const void* y,
               const void* z, const float* vx, const float* vy, const float* vz,
               const orc_halos* h, int64_t ns, const int32_t* halo_of, uint8_t* bound,
               double* phi, double* phi_abs, orc_unbound* out) {
  int64_t* hoff = (int64_t*)calloc((size_t)ns + 1, sizeof(int64_t));
  for (int64_t i = 0; i < n; ++i)
    if (halo_of[i] >= 0) hoff[halo_of[i] + 1]++;
  for (int64_t s = 0; s < ns; ++s) hoff[s + 1] += hoff[s];
  int64_t* hmem = (int64_t*)malloc(sizeof(int64_t) * (size_t)(hoff[ns] ? hoff[ns] : 1));
  {
    int64_t* fill = (int64_t*)malloc(sizeof(int64_t) * (size_t)(ns ? ns : 1));
    for (int64_t s = 0; s < ns; ++s) fill[s] = hoff[s];
    for (int64_t i = 0; i < n; ++i)
      if (halo_of[i] >= 0) hmem[fill[halo_of[i]]++] = i;
    free(fill);
  }
  for (int64_t i = 0; i < n; ++i) {
    bound[i] = 0;
    if (phi) phi[i] = 0.0;
    if (phi_abs) phi_abs[i] = 0.0;
  }
  ivec S = {0, 0, NULL}, stk = {0, 0, NULL};
  halo_tree tree;
  build_halo_tree(ns, h->host, &tree);
  for (int64_t s = 0; s < ns; ++s) {
    out->n_bound_own[s] = 0;
    out->n_s[s] = 0;
    out->n_bound_s[s] = 0;
    out->valid[s] = 0;
    out->vbx[s] = out->vby[s] = out->vbz[s] = 0.0;
  }
  /* |S(h)| and the bulk velocity of S(h) of every kept halo */
  for (int64_t s = 0; s < ns; ++s) {
    if (h->merged_into[s] != s) continue;
    subtree_members(&tree, hoff, hmem, s, &S, &stk);
    qsum qv;
    memset(&qv, 0, sizeof qv);
    for (int64_t q = 0; q < S.n; ++q) {
      int64_t j = S.v[q];
      qsum_add(&qv, quantise((double)vx[j], VEL_SHIFT), quantise((double)vy[j], VEL_SHIFT),
               quantise((double)vz[j], VEL_SHIFT));
    }
    double vb[3], dummy;
    qsum_finish(&qv, VEL_SHIFT, vb, &dummy);
    out->vbx[s] = vb[0];
    out->vby[s] = vb[1];
    out->vbz[s] = vb[2];
    out->n_s[s] = (uint32_t)S.n;
  }
  for (int64_t s = 0; s < ns; ++s) {
    if (h->merged_into[s] != s) continue;
    /* the system whose potential decides h's particles */
    int64_t t = s;
    if (p->major_merger > 0.0)
      while (h->host[t] >= 0 &&
             (double)out->n_s[t] >= p->major_merger * (double)out->n_s[h->host[t]])
        t = h->host[t];
    subtree_members(&tree, hoff, hmem, t, &S, &stk);
    const double vb[3] = {out->vbx[s], out->vby[s], out->vbz[s]};
    int64_t nown = hoff[s + 1] - hoff[s];
    double* ph = (double*)malloc(sizeof(double) * (size_t)(nown ? nown : 1));
    orc_phi_points(p, pos_f64, x, y, z, S.v, S.n, hmem + hoff[s], nown, ph);
    for (int64_t q = 0; q < nown; ++q) {
      int64_t i = hmem[hoff[s] + q];
      double ux = (double)vx[i] - vb[0], uy = (double)vy[i] - vb[1], uz = (double)vz[i] - vb[2];
      double e = 0.5 * sq3(ux, uy, uz) + ph[q];
      bound[i] = e < 0.0;
      if (phi) phi[i] = ph[q];
      if (phi_abs) phi_abs[i] = fabs(ph[q]);
      out->n_bound_own[s] += bound[i];
    }
    free(ph);
  }
  for (int64_t s = 0; s < ns; ++s) {
    if (h->merged_into[s] != s) continue;
    int64_t nb = 0;
    subtree_members(&tree, hoff, hmem, s, &S, &stk);
    for (int64_t q = 0; q < S.n; ++q) nb += bound[S.v[q]];
    out->n_bound_s[s] = (uint32_t)nb;
    out->valid[s] = (double)nb >= p->unbound_threshold * (double)out->n_s[s];
  }
  free(S.v);
  free(stk.v);
  free(tree.off);
  free(tree.ids);
  free(hoff);
  free(hmem);
  return ORC_OK;
}

/* ------------------------------------------------- properties ------------ */

/*
 * Halo properties (Sections 3.5.1-3.5.4), bound particles only (BP = 1):
 *  - centre: mean position of the node, on the chain from the halo's seed
 *    leaf towards the root while the node holds no other halo's seed, that
 *    minimises sigma_x/sqrt(n) (ties: the deeper node);
 *  - B(h): bound particles of S(h), sorted by distance from the centre;
 *  - virial SO (reading: first downcrossing): k* = largest k with
 *    3 j m / (4 pi r_j^3) >= rho_vir for all j <= k; M = k* m,
 *    R = (3 M / (4 pi rho_vir))^(1/3);
 *  - vmax = max over j <= k* of sqrt(G j m / max(r_j, eps));
 *  - v_bulk = mean velocity of the k* innermost; v_core = mean velocity of
 *    B(h) within core_frac R (the innermost particle if none);
 *  - V_off = |v_core - v_bulk|.
 * Merged seeds get zeros.  Pinned: NFW vmax, M_vir ~ n m, kicked-core V_off
 * (statistical); the centre chain against a brute-force numpy form
 * (tests/test_oracle_readings.py).  The readings of the centre chain and the
 * SO crossing themselves are not fixed by the paper.
 */
int orc_props(const orc_params* p, int64_t n, int pos_f64, const void* x, const void* y,
              const void* z, const float* vx, const float* vy, const float* vz,
              const orc_nodes* nd, int64_t nn, const orc_halos* h, int64_t ns,
              const int32_t* halo_of, const uint8_t* bound, orc_props_out* o) {
  int32_t* node_seed = (int32_t*)malloc(sizeof(int32_t) * (size_t)(nn ? nn : 1));
  for (int64_t k = 0; k < nn; ++k) node_seed[k] = -1;
  for (int64_t s = 0; s < ns; ++s) node_seed[h->seed_node[s]] = (int32_t)s;
  seedsets ss;
  build_seedsets(nd, nn, node_seed, h->merged_into, &ss);
  int64_t* hoff = (int64_t*)calloc((size_t)ns + 1, sizeof(int64_t));
  for (int64_t i = 0; i < n; ++i)
    if (halo_of[i] >= 0) hoff[halo_of[i] + 1]++;
  for (int64_t s = 0; s < ns; ++s) hoff[s + 1] += hoff[s];
  int64_t* hmem = (int64_t*)malloc(sizeof(int64_t) * (size_t)(hoff[ns] ? hoff[ns] : 1));
  {
    int64_t* fill = (int64_t*)malloc(sizeof(int64_t) * (size_t)(ns ? ns : 1));
    for (int64_t s = 0; s < ns; ++s) fill[s] = hoff[s];
    for (int64_t i = 0; i < n; ++i)
      if (halo_of[i] >= 0) hmem[fill[halo_of[i]]++] = i;
    free(fill);
  }
  const double C = (3.0 * p->particle_mass) / (4.0 * M_PI * p->rho_vir);
  const double e2 = p->softening * p->softening;
  ivec S = {0, 0, NULL}, stk = {0, 0, NULL};
  halo_tree tree;
  build_halo_tree(ns, h->host, &tree);
  for (int64_t s = 0; s < ns; ++s) {
    o->px[s] = o->py[s] = o->pz[s] = 0.0;
    o->vcx[s] = o->vcy[s] = o->vcz[s] = 0.0;
    o->vbx[s] = o->vby[s] = o->vbz[s] = 0.0;
    o->mvir[s] = o->rvir[s] = o->vmax[s] = o->voff[s] = 0.0;
    o->n_bound[s] = 0;
    if (h->merged_into[s] != s) continue;
    /* centre */
    int64_t k = h->seed_node[s], best = k;
    double bv = nd->sx2[k] / (double)nd->count[k];
    for (int64_t q = nd->parent[k]; q >= 0; q = nd->parent[q]) {
      if (ss.off[q + 1] - ss.off[q] != 1 || ss.ids[ss.off[q]] != s) break;
      double v = nd->sx2[q] / (double)nd->count[q];
      if (v < bv) {
        bv = v;
        best = q;
      }
    }
    double c[3] = {nd->cx[best], nd->cy[best], nd->cz[best]};
    o->px[s] = c[0];
    o->py[s] = c[1];
    o->pz[s] = c[2];
    /* bound members of S(h), by radius */
    subtree_members(&tree, hoff, hmem, s, &S, &stk);
    rad_t* r = (rad_t*)malloc(sizeof(rad_t) * (size_t)(S.n ? S.n : 1));
    int64_t nb = 0;
    for (int64_t q = 0; q < S.n; ++q) {
      int64_t i = S.v[q];
      if (!bound[i]) continue;
      double dx = min_image(pos_at(x, pos_f64, i) - c[0], p->box);
      double dy = min_image(pos_at(y, pos_f64, i) - c[1], p->box);
      double dz = min_image(pos_at(z, pos_f64, i) - c[2], p->box);
      r[nb].r2 = sq3(dx, dy, dz);
      r[nb].idx = i;
      nb++;
    }
    o->n_bound[s] = (uint32_t)nb;
    if (nb == 0) {
      free(r);
      continue;
    }
    qsort(r, (size_t)nb, sizeof(rad_t), cmp_rad);
    int64_t kstar = 0;
    for (int64_t j = 0; j < nb; ++j) {
      double r2 = r[j].r2;
      double r6 = r2 * r2 * r2;
      double jc = (double)(j + 1) * C;
      if (r6 <= jc * jc)
        kstar = j + 1;
      else
        break;
    }
    double mvir = (double)kstar * p->particle_mass;
    double rvir = cbrt((double)kstar * C);
    double vmx = 0.0, sb[3] = {0, 0, 0};
    for (int64_t j = 0; j < kstar; ++j) {
      double jj = (double)(j + 1);
      double t = (jj * jj) / fmax(r[j].r2, e2);
      if (t > vmx) vmx = t;
      int64_t i = r[j].idx;
      sb[0] += (double)vx[i];
      sb[1] += (double)vy[i];
      sb[2] += (double)vz[i];
    }
    double vb[3], vc[3];
    if (kstar > 0) {
      for (int a = 0; a < 3; ++a) vb[a] = sb[a] / (double)kstar;
    } else {
      int64_t i = r[0].idx;
      vb[0] = vx[i];
      vb[1] = vy[i];
      vb[2] = vz[i];
    }
    double rc = p->core_frac * rvir, rc2 = rc * rc, sc[3] = {0, 0, 0};
    int64_t nc = 0;
    for (int64_t j = 0; j < nb && r[j].r2 < rc2; ++j) {
      int64_t i = r[j].idx;
      sc[0] += (double)vx[i];
      sc[1] += (double)vy[i];
      sc[2] += (double)vz[i];
      nc++;
    }
    if (nc > 0) {
      for (int a = 0; a < 3; ++a) vc[a] = sc[a] / (double)nc;
    } else {
      int64_t i = r[0].idx;
      vc[0] = vx[i];
      vc[1] = vy[i];
      vc[2] = vz[i];
    }
    o->mvir[s] = mvir;
    o->rvir[s] = rvir;
    o->vmax[s] = kstar > 0 ? sqrt(p->G * p->particle_mass * sqrt(vmx)) : 0.0;
    o->vbx[s] = vb[0];
    o->vby[s] = vb[1];
    o->vbz[s] = vb[2];
    o->vcx[s] = vc[0];
    o->vcy[s] = vc[1];
    o->vcz[s] = vc[2];
    o->voff[s] = sqrt(sq3(vc[0] - vb[0], vc[1] - vb[1], vc[2] - vb[2]));
    free(r);
  }
  free(S.v);
  free(stk.v);
  free(tree.off);
  free(tree.ids);
  free(hoff);
  free(hmem);
  free(ss.off);
  free(ss.ids);
  free(node_seed);
  return ORC_OK;
}

/* ------------------------------------------------ additional properties -- */

/*
 * Spherical-overdensity count (Section 3.5.2): the largest k such that every
 * j <= k of the radially sorted particles encloses a mean density
 * 3 j m / (4 pi r_j^3) of at least the threshold, tested as r_j^6 <= (j C)^2
 * with C = 3 m / (4 pi rho_threshold).  Pinned: constructed radii with a
 * known crossing; the virial threshold reproduces orc_props' M_vir.
 */
int64_t orc_so_count(int64_t nb, const double* r2, double C) {
  int64_t k = 0;
  for (int64_t j = 0; j < nb; ++j) {
    double r6 = r2[j] * r2[j] * r2[j];
    double jc = (double)(j + 1) * C;
    if (r6 <= jc * jc)
      k = j + 1;
    else
      break;
  }
  return k;
}

static void neumaier(double* s, double* c, double term) {
  double u = *s + term;
  if (fabs(*s) >= fabs(term))
    *c += (*s - u) + term;
  else
    *c += (term - u) + *s;
  *s = u;
}

/*
 * Sums over one halo's set V (Section 3.5.4), positions dx relative to the
 * halo centre and velocities v (km/s), in plain FP64 with Neumaier
 * compensation:
 *   0-2   sum of dx                      (centre of mass: X_off)
 *   3-5   sum of dx x (v - v_bulk)       (angular momentum J / m)
 *   6     sum of |v - v_bulk|^2          (kinetic energy 2T / m)
 *   7     sum over pairs i < j of 1/sqrt(|dx_i - dx_j|^2 + eps^2)
 *                                        (potential energy -U / (G m^2),
 *                                         Plummer softening as in unbinding)
 *   8-13  sums of dx_a dx_b over the own particles (own[i] != 0), in the
 *         order xx, yy, zz, xy, xz, yz   (the mass distribution tensor of
 *                                         Eq. 11 times the count)
 *   14    number of own particles
 * Pinned: rigid rotation (J and T in closed form), a regular tetrahedron
 * and a brute-force pair sum by another route (U), a rotated axis-aligned
 * point set (tensor), a shifted set (centre of mass).
 */
void orc_halo_sums(int64_t k, const double* dx, const double* dy, const double* dz,
                   const double* vx, const double* vy, const double* vz, const uint8_t* own,
                   const double* vb, double eps2, double* o) {
  double s[ORC_EXTRA_NSUM], c[ORC_EXTRA_NSUM];
  for (int q = 0; q < ORC_EXTRA_NSUM; ++q) s[q] = c[q] = 0.0;
  for (int64_t i = 0; i < k; ++i) {
    double rx = dx[i], ry = dy[i], rz = dz[i];
    double ux = vx[i] - vb[0], uy = vy[i] - vb[1], uz = vz[i] - vb[2];
    neumaier(&s[0], &c[0], rx);
    neumaier(&s[1], &c[1], ry);
    neumaier(&s[2], &c[2], rz);
    neumaier(&s[3], &c[3], ry * uz - rz * uy);
    neumaier(&s[4], &c[4], rz * ux - rx * uz);
    neumaier(&s[5], &c[5], rx * uy - ry * ux);
    neumaier(&s[6], &c[6], ux * ux + uy * uy + uz * uz);
    for (int64_t j = i + 1; j < k; ++j) {
      double ex = dx[j] - rx, ey = dy[j] - ry, ez = dz[j] - rz;
      neumaier(&s[7], &c[7], 1.0 / sqrt(ex * ex + ey * ey + ez * ez + eps2));
    }
    if (own[i]) {
      neumaier(&s[8], &c[8], rx * rx);
      neumaier(&s[9], &c[9], ry * ry);
      neumaier(&s[10], &c[10], rz * rz);
      neumaier(&s[11], &c[11], rx * ry);
      neumaier(&s[12], &c[12], rx * rz);
      neumaier(&s[13], &c[13], ry * rz);
      s[14] += 1.0;
    }
  }
  for (int q = 0; q < ORC_EXTRA_NSUM; ++q) o[q] = s[q] + c[q];
}

/*
 * The sums of orc_halo_sums for every kept halo, over the set V(h) = the
 * bound particles of S(h) inside the virial radius, that is the k* innermost
 * by distance from the halo centre (the particles that define M_vir; the
 * paper computes J, the energies and T/|U| from the bound particles within
 * the halo radius -- reading: S(h), as for the mass), with the centre and
 * the bulk velocity of orc_props.  Own particles (halo_of == h) give the
 * shape tensor: the paper excludes substructure there.  k_so: the SO count
 * of each extra threshold so_rho[t] (Section 3.5.2), over the same radial
 * order of the bound particles of S(h).  Merged seeds get zeros.
 */
int orc_props_extra(const orc_params* p, int64_t n, int pos_f64, const void* x, const void* y,
                    const void* z, const float* vx, const float* vy, const float* vz,
                    const orc_halos* h, int64_t ns, const int32_t* halo_of,
                    const uint8_t* bound, const orc_props_out* pr, int32_t n_so,
                    const double* so_rho, orc_extra_sums* o) {
  if (n_so < 0 || (n_so > 0 && !so_rho)) return ORC_EINVAL;
  for (int32_t t = 0; t < n_so; ++t)
    if (!(so_rho[t] > 0.0)) return ORC_EINVAL;
  int64_t* hoff = (int64_t*)calloc((size_t)ns + 1, sizeof(int64_t));
  for (int64_t i = 0; i < n; ++i)
    if (halo_of[i] >= 0) hoff[halo_of[i] + 1]++;
  for (int64_t s = 0; s < ns; ++s) hoff[s + 1] += hoff[s];
  int64_t* hmem = (int64_t*)malloc(sizeof(int64_t) * (size_t)(hoff[ns] ? hoff[ns] : 1));
  {
    int64_t* fill = (int64_t*)malloc(sizeof(int64_t) * (size_t)(ns ? ns : 1));
    for (int64_t s = 0; s < ns; ++s) fill[s] = hoff[s];
    for (int64_t i = 0; i < n; ++i)
      if (halo_of[i] >= 0) hmem[fill[halo_of[i]]++] = i;
    free(fill);
  }
  const double m = p->particle_mass;
  const double Cvir = (3.0 * m) / (4.0 * M_PI * p->rho_vir);
  const double e2 = p->softening * p->softening;
  ivec S = {0, 0, NULL}, stk = {0, 0, NULL};
  halo_tree tree;
  build_halo_tree(ns, h->host, &tree);
  int rc = ORC_OK;
  for (int64_t s = 0; s < ns; ++s) {
    double sums[ORC_EXTRA_NSUM];
    for (int q = 0; q < ORC_EXTRA_NSUM; ++q) sums[q] = 0.0;
    int64_t kstar = 0;
    for (int32_t t = 0; t < n_so; ++t) o->k_so[(size_t)t * (size_t)ns + (size_t)s] = 0;
    if (h->merged_into[s] == s) {
      const double c[3] = {pr->px[s], pr->py[s], pr->pz[s]};
      const double vb[3] = {pr->vbx[s], pr->vby[s], pr->vbz[s]};
      subtree_members(&tree, hoff, hmem, s, &S, &stk);
      rad_t* r = (rad_t*)malloc(sizeof(rad_t) * (size_t)(S.n ? S.n : 1));
      int64_t nb = 0;
      for (int64_t q = 0; q < S.n; ++q) {
        int64_t i = S.v[q];
        if (!bound[i]) continue;
        double dx = min_image(pos_at(x, pos_f64, i) - c[0], p->box);
        double dy = min_image(pos_at(y, pos_f64, i) - c[1], p->box);
        double dz = min_image(pos_at(z, pos_f64, i) - c[2], p->box);
        r[nb].r2 = sq3(dx, dy, dz);
        r[nb].idx = i;
        nb++;
      }
      qsort(r, (size_t)nb, sizeof(rad_t), cmp_rad);
      double* r2 = (double*)malloc(sizeof(double) * (size_t)(nb ? nb : 1));
      for (int64_t j = 0; j < nb; ++j) r2[j] = r[j].r2;
      kstar = orc_so_count(nb, r2, Cvir);
      if ((double)kstar * m != pr->mvir[s]) rc = ORC_EINVAL; /* not orc_props' M_vir */
      for (int32_t t = 0; t < n_so; ++t) {
        double Ct = (3.0 * m) / (4.0 * M_PI * so_rho[t]);
        o->k_so[(size_t)t * (size_t)ns + (size_t)s] = (uint32_t)orc_so_count(nb, r2, Ct);
      }
      int64_t kk = kstar ? kstar : 1;
      double* d = (double*)malloc(sizeof(double) * 6 * (size_t)kk);
      uint8_t* own = (uint8_t*)malloc((size_t)kk);
      for (int64_t j = 0; j < kstar; ++j) {
        int64_t i = r[j].idx;
        d[j] = min_image(pos_at(x, pos_f64, i) - c[0], p->box);
        d[kk + j] = min_image(pos_at(y, pos_f64, i) - c[1], p->box);
        d[2 * kk + j] = min_image(pos_at(z, pos_f64, i) - c[2], p->box);
        d[3 * kk + j] = (double)vx[i];
        d[4 * kk + j] = (double)vy[i];
        d[5 * kk + j] = (double)vz[i];
        own[j] = halo_of[i] == s;
      }
      orc_halo_sums(kstar, d, d + kk, d + 2 * kk, d + 3 * kk, d + 4 * kk, d + 5 * kk, own, vb,
                    e2, sums);
      free(d);
      free(own);
      free(r2);
      free(r);
    }
    o->sx[s] = sums[0];
    o->sy[s] = sums[1];
    o->sz[s] = sums[2];
    o->jx[s] = sums[3];
    o->jy[s] = sums[4];
    o->jz[s] = sums[5];
    o->t2[s] = sums[6];
    o->uinv[s] = sums[7];
    o->mxx[s] = sums[8];
    o->myy[s] = sums[9];
    o->mzz[s] = sums[10];
    o->mxy[s] = sums[11];
    o->mxz[s] = sums[12];
    o->myz[s] = sums[13];
    o->n_own[s] = (uint32_t)sums[14];
    o->k[s] = (uint32_t)kstar;
  }
  free(S.v);
  free(stk.v);
  free(tree.off);
  free(tree.ids);
  free(hoff);
  free(hmem);
  return rc;
}
