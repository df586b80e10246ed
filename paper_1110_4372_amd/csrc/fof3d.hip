// 3D friends-of-friends on a radix-sorted cell list (Section 3.1 of the paper,
// standard FOF definition), for gfx950.
//
// Cells have side s <= ll / sqrt(3) (1 - 1e-6), so any two particles in one
// cell are friends: every occupied cell is a clique and union-find runs over
// cells, not particles.  Each occupied cell visits the half stencil of cells
// within reach R = ceil(ll / s) and stops testing a cell pair at its first
// friendly pair (or skips it when both cells already share a root).  The
// result is the exact standard FOF partition, the dense cores costing about
// one test per cell pair -- the role the paper's dense-particle shortcut
// plays on the CPU, without its order-dependent superset.
#include "fof3d.hpp"
#include "primitives.hpp"

namespace halo {

namespace {

struct Grid {
  double box, hbox, ll2, inv_side;
  int64_t nc;   // cells per axis
  int reach;    // stencil reach in cells
};

template <class T>
__global__ void k_cell_keys(const T* x, const T* y, const T* z, int64_t n, Grid g,
                            unsigned long long* key, uint32_t* err) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double p[3] = {(double)x[i], (double)y[i], (double)z[i]};
  int64_t c[3];
  bool bad = false;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    if (!(p[a] >= 0.0 && p[a] < g.box)) bad = true;
    int64_t ci = (int64_t)floor(p[a] * g.inv_side);
    ci = ci < 0 ? 0 : (ci >= g.nc ? g.nc - 1 : ci);
    c[a] = ci;
  }
  if (bad) atomicOr(err, kErrPosRange);
  key[i] = (unsigned long long)((c[2] * g.nc + c[1]) * g.nc + c[0]);
}

template <class T>
__global__ void k_gather3(const T* x, const T* y, const T* z, const uint32_t* perm, int64_t n,
                          T* xs, T* ys, T* zs) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  uint32_t j = perm[i];
  xs[i] = x[j];
  ys[i] = y[j];
  zs[i] = z[j];
}

// head[i] = 1 where the sorted key changes.
__global__ void k_heads(const unsigned long long* key, int64_t n, uint32_t* head) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  head[i] = (i == 0 || key[i] != key[i - 1]) ? 1u : 0u;
}

// cell_of[i] = cell index of sorted particle i; cell table start / key.
__global__ void k_cells(const unsigned long long* key, const uint32_t* hscan, int64_t n,
                        uint32_t* cell_of, uint32_t* cell_start,
                        unsigned long long* cell_key) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  bool h = (i == 0 || key[i] != key[i - 1]);
  uint32_t c = hscan[i] + (h ? 0u : 0xFFFFFFFFu);  // inclusive scan - 1
  cell_of[i] = c;
  if (h) {
    cell_start[c] = (uint32_t)i;
    cell_key[c] = key[i];
  }
}

// row_start[r] = first cell whose key is >= r * nc (rows are (cz, cy)).
__global__ void k_rows(const unsigned long long* cell_key, int64_t ncell, int64_t nc,
                       int64_t nrow, uint32_t* row_start) {
  int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r > nrow) return;
  unsigned long long target = (unsigned long long)(r * nc);
  int64_t lo = 0, hi = ncell;
  while (lo < hi) {
    int64_t mid = (lo + hi) >> 1;
    if (cell_key[mid] < target)
      lo = mid + 1;
    else
      hi = mid;
  }
  row_start[r] = (uint32_t)lo;
}

// First cell of [lo, hi) whose key is >= want (keys ascend within a row).
__device__ __forceinline__ uint32_t lower_cell(const unsigned long long* cell_key, uint32_t lo,
                                               uint32_t hi, unsigned long long want) {
  while (lo < hi) {
    const uint32_t mid = (lo + hi) >> 1;
    if (cell_key[mid] < want)
      lo = mid + 1;
    else
      hi = mid;
  }
  return lo;
}

// Links cell c with occupied cell d (key kd) at offset (dx, dy, dz) when they
// do not share a root yet and hold a friendly pair: the cells' particles are
// tested until the first pair within ll.
template <class T>
__device__ __forceinline__ void link_pair(const T* xs, const T* ys, const T* zs,
                                          const uint32_t* cell_start, int64_t ncell, int64_t n,
                                          const Grid& g, uint32_t c, uint32_t a0, uint32_t a1,
                                          uint32_t d, uint32_t* par) {
  if (uf_find(par, c) == uf_find(par, d)) return;
  const uint32_t b0 = cell_start[d];
  const uint32_t b1 = (d + 1 < ncell) ? cell_start[d + 1] : (uint32_t)n;
  for (uint32_t i = a0; i < a1; ++i) {
    const double xi = (double)xs[i], yi = (double)ys[i], zi = (double)zs[i];
    for (uint32_t j = b0; j < b1; ++j) {
      const double ex = min_image((double)xs[j] - xi, g.box);
      const double ey = min_image((double)ys[j] - yi, g.box);
      const double ez = min_image((double)zs[j] - zi, g.box);
      if (sq3(ex, ey, ez) <= g.ll2) {
        uf_union(par, c, d);
        return;
      }
    }
  }
}

// Link pass over the half stencil.  phase 0: offsets within one cell on every
// axis; phase 1: the others.  One thread per occupied cell.  The stencil is
// visited row by row (rows are (cz, cy)): an empty row costs its two bounds,
// and the occupied cells of the x range [cx - R, cx + R] (periodic, so up to
// two intervals) are found by one search.
template <class T>
__global__ void k_link(const T* xs, const T* ys, const T* zs, const uint32_t* cell_start,
                       const unsigned long long* cell_key, const uint32_t* row_start,
                       int64_t ncell, int64_t n, Grid g, int phase, uint32_t* par) {
  // neighbouring cells, whose stencils read the same rows, on one XCD
  int64_t c = (int64_t)xcd_block() * blockDim.x + threadIdx.x;
  if (c >= ncell) return;
  const int64_t nc = g.nc;
  const unsigned long long kc = cell_key[c];
  const int64_t cx = (int64_t)(kc % (unsigned long long)nc);
  const int64_t cy = (int64_t)((kc / (unsigned long long)nc) % (unsigned long long)nc);
  const int64_t cz = (int64_t)(kc / ((unsigned long long)nc * (unsigned long long)nc));
  const uint32_t a0 = cell_start[c];
  const uint32_t a1 = (c + 1 < ncell) ? cell_start[c + 1] : (uint32_t)n;
  const int R = g.reach;
  const double side = g.box / (double)nc;
  for (int dz = 0; dz <= R; ++dz) {
    for (int dy = (dz == 0 ? 0 : -R); dy <= R; ++dy) {
      const int xlo = (dz == 0 && dy == 0) ? 1 : -R;
      // phase 0 holds only |dx|, |dy|, dz <= 1
      if (phase == 0 && (dz > 1 || dy > 1 || dy < -1)) continue;
      int64_t ny = cy + dy, nz = cz + dz;
      ny = ny < 0 ? ny + nc : (ny >= nc ? ny - nc : ny);
      nz = nz < 0 ? nz + nc : (nz >= nc ? nz - nc : nz);
      const int64_t row = nz * nc + ny;
      const uint32_t r0 = row_start[row], r1 = row_start[row + 1];
      if (r0 == r1) continue;
      const unsigned long long rbase = (unsigned long long)row * (unsigned long long)nc;
      // x range [cx + xlo, cx + R] as up to two intervals of [0, nc)
      int64_t u0 = cx + xlo, u1 = cx + R;
      int64_t iv[2][2];
      int nv = 0;
      if (u0 < 0) {
        iv[nv][0] = u0 + nc; iv[nv][1] = nc - 1; ++nv;
        u0 = 0;
      }
      if (u1 >= nc) {
        iv[nv][0] = 0; iv[nv][1] = u1 - nc; ++nv;
        u1 = nc - 1;
      }
      iv[nv][0] = u0; iv[nv][1] = u1; ++nv;
      for (int q = 0; q < nv; ++q) {
        uint32_t p = lower_cell(cell_key, r0, r1, rbase + (unsigned long long)iv[q][0]);
        for (; p < r1; ++p) {
          const unsigned long long kd = cell_key[p];
          const int64_t x = (int64_t)(kd - rbase);
          if (x > iv[q][1]) break;
          int64_t dx = x - cx;
          dx = dx > R ? dx - nc : (dx < -R ? dx + nc : dx);
          const int far = (dx > 1 || dx < -1 || dy > 1 || dy < -1 || dz > 1);
          if (far != phase) continue;
          // smallest possible separation of the two cells
          const double gx = (double)(dx < 0 ? -dx - 1 : (dx > 0 ? dx - 1 : 0));
          const double gy = (double)(dy < 0 ? -dy - 1 : (dy > 0 ? dy - 1 : 0));
          const double gz = (double)(dz > 0 ? dz - 1 : 0);
          if ((gx * gx + gy * gy + gz * gz) * side * side > g.ll2 * (1.0 + 1e-9)) continue;
          link_pair(xs, ys, zs, cell_start, ncell, n, g, (uint32_t)c, a0, a1, p, par);
        }
      }
    }
  }
}

// ---------------------------------------------- dense-particle variant ----
// Section 3.1's faster FOF, in an order-free form: a particle with more than
// t friends within ll also links every particle within 2 ll.  (The paper
// skips the searches of a dense particle's neighbours, which makes its result
// depend on the visiting order; these links give a superset of any order's
// groups, and like the paper's at least the standard ones.)

// Visits the occupied cells within `reach` cells of cell (cx, cy, cz), all
// offsets but the cell itself, whose closest point can lie within r2 of
// it; f(cell) returns true to stop.
template <class F>
__device__ __forceinline__ void for_stencil(const unsigned long long* cell_key,
                                            const uint32_t* row_start, const Grid& g,
                                            int64_t cx, int64_t cy, int64_t cz, int reach,
                                            double r2, F&& f) {
  const int64_t nc = g.nc;
  const double side = g.box / (double)nc;
  for (int dz = -reach; dz <= reach; ++dz) {
    for (int dy = -reach; dy <= reach; ++dy) {
      int64_t ny = cy + dy, nz = cz + dz;
      ny = ny < 0 ? ny + nc : (ny >= nc ? ny - nc : ny);
      nz = nz < 0 ? nz + nc : (nz >= nc ? nz - nc : nz);
      const int64_t row = nz * nc + ny;
      const uint32_t r0 = row_start[row], r1 = row_start[row + 1];
      if (r0 == r1) continue;
      const unsigned long long rbase = (unsigned long long)row * (unsigned long long)nc;
      int64_t u0 = cx - reach, u1 = cx + reach;
      int64_t iv[2][2];
      int nv = 0;
      if (u0 < 0) {
        iv[nv][0] = u0 + nc; iv[nv][1] = nc - 1; ++nv;
        u0 = 0;
      }
      if (u1 >= nc) {
        iv[nv][0] = 0; iv[nv][1] = u1 - nc; ++nv;
        u1 = nc - 1;
      }
      iv[nv][0] = u0; iv[nv][1] = u1; ++nv;
      for (int q = 0; q < nv; ++q) {
        uint32_t p = lower_cell(cell_key, r0, r1, rbase + (unsigned long long)iv[q][0]);
        for (; p < r1; ++p) {
          const int64_t x = (int64_t)(cell_key[p] - rbase);
          if (x > iv[q][1]) break;
          int64_t dx = x - cx;
          dx = dx > reach ? dx - nc : (dx < -reach ? dx + nc : dx);
          if (dx == 0 && dy == 0 && dz == 0) continue;
          const double gx = (double)(dx < 0 ? -dx - 1 : (dx > 0 ? dx - 1 : 0));
          const double gy = (double)(dy < 0 ? -dy - 1 : (dy > 0 ? dy - 1 : 0));
          const double gz = (double)(dz < 0 ? -dz - 1 : (dz > 0 ? dz - 1 : 0));
          if ((gx * gx + gy * gy + gz * gz) * side * side > r2 * (1.0 + 1e-9)) continue;
          if (f(p)) return;
        }
      }
    }
  }
}

// dense[i] = 1 when sorted particle i has more than t friends within ll
// (its own cell's others all are: the cell is a clique).
template <class T>
__global__ void k_dense_flags(const T* xs, const T* ys, const T* zs, const uint32_t* cell_of,
                              const uint32_t* cell_start, const unsigned long long* cell_key,
                              const uint32_t* row_start, int64_t ncell, int64_t n, Grid g,
                              uint32_t t, uint32_t* dense) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const uint32_t c = cell_of[i];
  const uint32_t a0 = cell_start[c];
  const uint32_t a1 = (c + 1 < ncell) ? cell_start[c + 1] : (uint32_t)n;
  uint32_t cnt = a1 - a0 - 1;
  if (cnt <= t) {
    const unsigned long long kc = cell_key[c];
    const int64_t nc = g.nc;
    const int64_t cx = (int64_t)(kc % (unsigned long long)nc);
    const int64_t cy = (int64_t)((kc / (unsigned long long)nc) % (unsigned long long)nc);
    const int64_t cz = (int64_t)(kc / ((unsigned long long)nc * (unsigned long long)nc));
    const double xi = (double)xs[i], yi = (double)ys[i], zi = (double)zs[i];
    for_stencil(cell_key, row_start, g, cx, cy, cz, g.reach, g.ll2, [&](uint32_t d) {
      const uint32_t b0 = cell_start[d];
      const uint32_t b1 = (d + 1 < ncell) ? cell_start[d + 1] : (uint32_t)n;
      for (uint32_t j = b0; j < b1; ++j) {
        const double ex = min_image((double)xs[j] - xi, g.box);
        const double ey = min_image((double)ys[j] - yi, g.box);
        const double ez = min_image((double)zs[j] - zi, g.box);
        if (sq3(ex, ey, ez) <= g.ll2 && ++cnt > t) return true;
      }
      return false;
    });
  }
  dense[i] = cnt > t ? 1u : 0u;
}

// A dense particle joins its cell with every cell holding a particle within
// 2 ll (cells are cliques, so one such particle per cell suffices).
template <class T>
__global__ void k_dense_links(const T* xs, const T* ys, const T* zs, const uint32_t* cell_of,
                              const uint32_t* cell_start, const unsigned long long* cell_key,
                              const uint32_t* row_start, int64_t ncell, int64_t n, Grid g,
                              int reach2, const uint32_t* dense, uint32_t* par) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n || !dense[i]) return;
  const uint32_t c = cell_of[i];
  const unsigned long long kc = cell_key[c];
  const int64_t nc = g.nc;
  const int64_t cx = (int64_t)(kc % (unsigned long long)nc);
  const int64_t cy = (int64_t)((kc / (unsigned long long)nc) % (unsigned long long)nc);
  const int64_t cz = (int64_t)(kc / ((unsigned long long)nc * (unsigned long long)nc));
  const double xi = (double)xs[i], yi = (double)ys[i], zi = (double)zs[i];
  const double r2 = 4.0 * g.ll2;
  for_stencil(cell_key, row_start, g, cx, cy, cz, reach2, r2, [&](uint32_t d) {
    if (uf_find(par, c) == uf_find(par, d)) return false;
    const uint32_t b0 = cell_start[d];
    const uint32_t b1 = (d + 1 < ncell) ? cell_start[d + 1] : (uint32_t)n;
    for (uint32_t j = b0; j < b1; ++j) {
      const double ex = min_image((double)xs[j] - xi, g.box);
      const double ey = min_image((double)ys[j] - yi, g.box);
      const double ez = min_image((double)zs[j] - zi, g.box);
      if (sq3(ex, ey, ez) <= r2) {
        uf_union(par, c, d);
        break;
      }
    }
    return false;
  });
}

// Every parent becomes its root.  Roots do not change during this pass (no
// unions), so each thread may store the root it reads.
__global__ void k_compress(uint32_t* par, int64_t n) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  uf_store(par + i, uf_root(par, (uint32_t)i));
}

// minidx[root] = smallest input index in the component: per-cell minimum,
// then one wave-aggregated atomic per cell (neighbouring cells share roots).
__global__ void k_cell_min(const uint32_t* cell_start, int64_t ncell, int64_t n,
                           const uint32_t* perm, const uint32_t* par, uint32_t* minidx) {
  const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const bool ok = c < ncell;
  uint32_t mn = 0xFFFFFFFFu, root = 0;
  if (ok) {
    const uint32_t a0 = cell_start[c];
    const uint32_t a1 = (c + 1 < ncell) ? cell_start[c + 1] : (uint32_t)n;
    for (uint32_t i = a0; i < a1; ++i) mn = min(mn, perm[i]);
    root = par[c];
  }
  agg_min_u32(minidx, root, mn, ok);
}

// Group sizes by label, one wave-aggregated atomic per cell.
__global__ void k_cell_sizes(const uint32_t* cell_start, int64_t ncell, int64_t n,
                             const uint32_t* par, const uint32_t* minidx, uint32_t* gsize) {
  const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const bool ok = c < ncell;
  uint32_t cnt = 0, lab = 0;
  if (ok) {
    const uint32_t a0 = cell_start[c];
    const uint32_t a1 = (c + 1 < ncell) ? cell_start[c + 1] : (uint32_t)n;
    cnt = a1 - a0;
    lab = minidx[par[c]];
  }
  agg_add_u32(gsize, lab, cnt, ok);
}

__global__ void k_labels(const uint32_t* cell_of, const uint32_t* perm, const uint32_t* par,
                         const uint32_t* minidx, int64_t n, uint32_t* label) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  label[perm[i]] = minidx[par[cell_of[i]]];
}

__global__ void k_member_flags(const uint32_t* label, const uint32_t* gsize, int64_t n,
                               uint32_t mm, uint32_t* flag) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  flag[i] = gsize[label[i]] >= mm ? 1u : 0u;
}

__global__ void k_member_compact(const uint32_t* label, const uint32_t* gsize,
                                 const uint32_t* pos, int64_t n, uint32_t mm, uint32_t* key,
                                 uint32_t* val) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  uint32_t l = label[i];
  if (gsize[l] >= mm) {
    key[pos[i]] = l;
    val[pos[i]] = (uint32_t)i;
  }
}

__global__ void k_group_heads(const uint32_t* key, int64_t m, uint32_t* head) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= m) return;
  head[i] = (i == 0 || key[i] != key[i - 1]) ? 1u : 0u;
}

__global__ void k_group_table(const uint32_t* key, const uint32_t* hscan, int64_t m,
                              const uint32_t* gsize, uint32_t* grp_first,
                              uint32_t* grp_count, int64_t cap) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= m) return;
  if (i == 0 || key[i] != key[i - 1]) {
    uint32_t g = hscan[i];
    if ((int64_t)g < cap) {
      grp_first[g] = (uint32_t)i;
      grp_count[g] = gsize[key[i]];
    }
  }
}

__global__ void k_copy_u32(const uint32_t* a, uint32_t* b, int64_t n) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) b[i] = a[i];
}

template <class T>
void fof3d_impl(Ctx& ctx, int64_t n, const T* x, const T* y, const T* z, uint32_t* label,
                uint32_t* perm_out, uint32_t* grp_first, uint32_t* grp_count, int64_t grp_cap,
                int64_t* n_groups, int64_t* n_members, hipStream_t s) {
  const libhalo_params& P = ctx.p;
  const double ll = P.b * P.box / cbrt((double)n);
  const double smax = ll / sqrt(3.0) * (1.0 - 1e-6);
  Grid g;
  g.box = P.box;
  g.hbox = 0.5 * P.box;
  g.ll2 = ll * ll;
  g.nc = (int64_t)ceil(P.box / smax);
  const double side = P.box / (double)g.nc;
  g.inv_side = (double)g.nc / P.box;
  g.reach = (int)ceil(ll / side);
  HALO_CHECK(g.nc >= 2 * g.reach + 1, LIBHALO_EINVAL,
             "box too small for the linking length (fewer than 2R+1 cells per side)");
  HALO_CHECK((double)g.nc * (double)g.nc * (double)g.nc < 1.8e19, LIBHALO_EINVAL,
             "cell grid exceeds 64-bit keys");
  const int64_t nrow = g.nc * g.nc;
  HALO_CHECK(nrow < 0xFFFFFFFFll, LIBHALO_EINVAL, "cell rows exceed 32-bit table");
  const int reach2 = (int)ceil(2.0 * ll / side);  // stencil of the 2 ll links
  HALO_CHECK(P.fof_dense == 0 || g.nc >= 2 * reach2 + 1, LIBHALO_EINVAL,
             "box too small for the dense-particle variant (fewer than 2Q+1 cells per side)");

  Arena& A = ctx.ws;
  A.reset();
  auto* key0 = A.take<unsigned long long>(n);
  auto* key1 = A.take<unsigned long long>(n);
  auto* v0 = A.take<uint32_t>(n);
  auto* v1 = A.take<uint32_t>(n);
  T* xs = A.take<T>(n);
  T* ys = A.take<T>(n);
  T* zs = A.take<T>(n);
  auto* cell_of = A.take<uint32_t>(n);
  auto* hscan = A.take<uint32_t>(n + 1);
  auto* cell_start = A.take<uint32_t>(n);
  auto* cell_key = A.take<unsigned long long>(n);
  auto* row_start = A.take<uint32_t>(nrow + 1);
  auto* par = A.take<uint32_t>(n);
  auto* minidx = A.take<uint32_t>(n);
  auto* gsize = A.take<uint32_t>(n);
  auto* cnt = A.take<uint32_t>(8);
  uint32_t* dense = P.fof_dense > 0 ? A.take<uint32_t>(n) : nullptr;
  void* rtmp = A.take<char>(radix_tmp_bytes(n));
  uint32_t* stmp = A.take<uint32_t>(scan_tmp_elems<uint32_t>(n + 1));

  const int TB = 256;
  const unsigned nb = blocks_for(n, TB);
  HALO_HIP(hipMemsetAsync(ctx.d_err, 0, sizeof(uint32_t), s));
  k_cell_keys<T><<<nb, TB, 0, s>>>(x, y, z, n, g, key0, ctx.d_err);
  k_iota<<<nb, TB, 0, s>>>(v0, n);
  int kb = bits_for((unsigned long long)(g.nc * g.nc * g.nc - 1));
  bool flip = radix_sort_pairs<unsigned long long>(key0, v0, key1, v1, n, kb, rtmp, s);
  unsigned long long* skey = flip ? key1 : key0;
  uint32_t* sperm = flip ? v1 : v0;
  k_gather3<T><<<nb, TB, 0, s>>>(x, y, z, sperm, n, xs, ys, zs);
  k_heads<<<nb, TB, 0, s>>>(skey, n, hscan);
  exclusive_scan<uint32_t>(hscan, hscan, n, cnt, stmp, s);
  k_cells<<<nb, TB, 0, s>>>(skey, hscan, n, cell_of, cell_start, cell_key);
  // number of occupied cells = cnt[0] (exclusive scan of heads, total)
  uint32_t* h = ctx.host_slot<uint32_t>(0);
  HALO_HIP(hipMemcpyAsync(h, cnt, sizeof(uint32_t), hipMemcpyDeviceToHost, s));
  HALO_HIP(hipMemcpyAsync(h + 1, ctx.d_err, sizeof(uint32_t), hipMemcpyDeviceToHost, s));
  HALO_HIP(hipStreamSynchronize(s));
  HALO_CHECK((h[1] & kErrPosRange) == 0, LIBHALO_EINVAL, "a position lies outside [0, box)");
  const int64_t ncell = h[0];
  k_rows<<<blocks_for(nrow + 1, TB), TB, 0, s>>>(cell_key, ncell, g.nc, nrow, row_start);
  k_iota<<<blocks_for(ncell, TB), TB, 0, s>>>(par, ncell);
  for (int phase = 0; phase < 2; ++phase) {
    HALO_PROF(ctx, "k_link", s, k_link<T><<<blocks_for(ncell, 128), 128, 0, s>>>(xs, ys, zs, cell_start, cell_key,
                                                       row_start, ncell, n, g, phase, par));
    k_compress<<<blocks_for(ncell, TB), TB, 0, s>>>(par, ncell);
  }
  if (P.fof_dense > 0) {
    k_dense_flags<T><<<nb, TB, 0, s>>>(xs, ys, zs, cell_of, cell_start, cell_key, row_start,
                                       ncell, n, g, (uint32_t)P.fof_dense, dense);
    HALO_PROF(ctx, "k_dense_links", s,
              k_dense_links<T><<<nb, TB, 0, s>>>(xs, ys, zs, cell_of, cell_start, cell_key,
                                                 row_start, ncell, n, g, reach2, dense, par));
    k_compress<<<blocks_for(ncell, TB), TB, 0, s>>>(par, ncell);
  }
  k_fill_u32<<<nb, TB, 0, s>>>(minidx, ncell, 0xFFFFFFFFu);
  k_fill_u32<<<nb, TB, 0, s>>>(gsize, n, 0u);
  k_cell_min<<<blocks_for(ncell, TB), TB, 0, s>>>(cell_start, ncell, n, sperm, par, minidx);
  k_cell_sizes<<<blocks_for(ncell, TB), TB, 0, s>>>(cell_start, ncell, n, par, minidx, gsize);
  k_labels<<<nb, TB, 0, s>>>(cell_of, sperm, par, minidx, n, label);
  // members of groups with >= min_members, in input order, keyed by label
  const uint32_t mm = (uint32_t)P.min_members;
  k_member_flags<<<nb, TB, 0, s>>>(label, gsize, n, mm, v0);
  exclusive_scan<uint32_t>(v0, hscan, n, cnt + 1, stmp, s);
  uint32_t* mkey0 = reinterpret_cast<uint32_t*>(key0);
  uint32_t* mkey1 = reinterpret_cast<uint32_t*>(key1);
  k_member_compact<<<nb, TB, 0, s>>>(label, gsize, hscan, n, mm, mkey0, v0);
  HALO_HIP(hipMemcpyAsync(h + 2, cnt + 1, sizeof(uint32_t), hipMemcpyDeviceToHost, s));
  HALO_HIP(hipStreamSynchronize(s));
  const int64_t m = h[2];
  bool f2 = radix_sort_pairs<uint32_t>(mkey0, v0, mkey1, v1, m, bits_for((uint64_t)n), rtmp, s);
  uint32_t* gkey = f2 ? mkey1 : mkey0;
  uint32_t* gval = f2 ? v1 : v0;
  if (m > 0) {
    k_copy_u32<<<blocks_for(m, TB), TB, 0, s>>>(gval, perm_out, m);
    k_group_heads<<<blocks_for(m, TB), TB, 0, s>>>(gkey, m, hscan);
    exclusive_scan<uint32_t>(hscan, hscan, m, cnt + 2, stmp, s);
    k_group_table<<<blocks_for(m, TB), TB, 0, s>>>(gkey, hscan, m, gsize, grp_first,
                                                  grp_count, grp_cap);
    HALO_HIP(hipMemcpyAsync(h + 3, cnt + 2, sizeof(uint32_t), hipMemcpyDeviceToHost, s));
  } else {
    h[3] = 0;
  }
  HALO_HIP(hipStreamSynchronize(s));
  *n_members = m;
  *n_groups = h[3];
  HALO_CHECK(*n_groups <= grp_cap, LIBHALO_ECAPACITY, "group table too small");
}

}  // namespace

size_t fof3d_workspace(const libhalo_params& P, int64_t n, int pos_dtype) {
  const double ll = P.b * P.box / cbrt((double)n);
  const double smax = ll / sqrt(3.0) * (1.0 - 1e-6);
  int64_t nc = (int64_t)ceil(P.box / smax);
  size_t tsz = pos_dtype == LIBHALO_F64 ? 8 : 4;
  size_t b = 0;
  auto add = [&](size_t bytes) { b += (bytes + 255) & ~size_t(255); };
  add(8 * n); add(8 * n); add(4 * n); add(4 * n);
  add(tsz * n); add(tsz * n); add(tsz * n);
  add(4 * n); add(4 * (n + 1)); add(4 * n); add(8 * n);
  add(4 * ((size_t)nc * nc + 1));
  add(4 * n); add(4 * n); add(4 * n); add(32);
  if (P.fof_dense > 0) add(4 * n);
  add(radix_tmp_bytes(n));
  add(4 * scan_tmp_elems<uint32_t>(n + 1));
  return b + 4096;
}

void fof3d(Ctx& ctx, int64_t n, int pos_dtype, const void* x, const void* y, const void* z,
           uint32_t* label, uint32_t* perm, uint32_t* grp_first, uint32_t* grp_count,
           int64_t grp_cap, int64_t* n_groups, int64_t* n_members, hipStream_t s) {
  if (pos_dtype == LIBHALO_F64)
    fof3d_impl<double>(ctx, n, (const double*)x, (const double*)y, (const double*)z, label,
                       perm, grp_first, grp_count, grp_cap, n_groups, n_members, s);
  else
    fof3d_impl<float>(ctx, n, (const float*)x, (const float*)y, (const float*)z, label, perm,
                      grp_first, grp_count, grp_cap, n_groups, n_members, s);
}

}  // namespace halo
