// Recursive phase-space FOF hierarchy (Section 3.2 of the paper) on gfx950,
// level-synchronous: every kernel of a level covers all nodes of that level.
//
// Per level, for each node (a subgroup of particles, contiguous in the level
// array, ordered by input index):
//   1. moments: exact fixed-point sums (positions about the node's anchor --
//      its smallest-index particle -- and velocities), 128-bit accumulators;
//   2. normalised FP32 coordinates (Eq. 1 metric);
//   3. nearest-neighbour squared distance of every particle (LDS-tiled
//      all-pairs within the node);
//   4. ell^2 = k-th smallest of them, k = ceil(f n): radix selection on the
//      FP32 bit patterns (in LDS for nodes <= 4096, multi-block above);
//   5. 6D FOF at ell^2: union-find over level positions with CAS hooking;
//   6. children = components of >= min_members: a stable radix sort by child
//      id builds the next level's array in (parent, smallest index) order.
#include <algorithm>

#include "lanes.hpp"
#include "primitives.hpp"
#include "refine_common.hpp"
#include "stages.hpp"

namespace halo {

namespace {
using namespace refine;

// ------------------------------------------------------------ level 0 ------
template <class T>
struct Members {  // the FOF members' positions and velocities in member order
  T *x, *y, *z;
  float *vx, *vy, *vz;
};

// The level arrays index the members in their FOF order (lidx holds member
// positions; perm maps them to input indices), and the members' positions and
// velocities are gathered once into that order: every level's particles are a
// subsequence of it, so the later levels read them in increasing order.
template <class T>
__global__ void k_level0(const uint32_t* perm, const uint32_t* grp_first,
                         const uint32_t* grp_count, uint32_t G, uint32_t M, uint32_t* lidx,
                         uint32_t* lnode, const T* x, const T* y, const T* z, const float* vx,
                         const float* vy, const float* vz, Members<T> g) {
  uint32_t m = blockIdx.x * blockDim.x + threadIdx.x;
  if (m >= M) return;
  lidx[m] = m;
  const uint32_t i = perm[m];
  g.x[m] = x[i];
  g.y[m] = y[i];
  g.z[m] = z[i];
  g.vx[m] = vx[i];
  g.vy[m] = vy[i];
  g.vz[m] = vz[i];
  // groups are contiguous and in order: last g with first[g] <= m
  uint32_t lo = 0, hi = G;
  while (hi - lo > 1) {
    uint32_t mid = (lo + hi) >> 1;
    if (grp_first[mid] <= m)
      lo = mid;
    else
      hi = mid;
  }
  lnode[m] = lo;
}

__global__ void k_level0_nodes(const uint32_t* perm, const uint32_t* grp_first,
                               const uint32_t* grp_count, uint32_t G, LevelNodes nd) {
  uint32_t g = blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= G) return;
  nd.first[g] = grp_first[g];
  nd.count[g] = grp_count[g];
  nd.parent[g] = -1;
  uint32_t lab = perm[grp_first[g]];
  nd.fof[g] = lab;
  nd.canon[g] = lab;
}

// ------------------------------------------------------------ moments ------
__global__ void k_mom_items(const uint32_t* count, uint32_t K, uint32_t* items) {
  uint32_t k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k < K) items[k] = (count[k] + kMomTile - 1) / kMomTile;
}

template <class T>
__global__ void __launch_bounds__(TB)
    k_mom_accum(const T* x, const T* y, const T* z, const float* vx, const float* vy,
                const float* vz, const uint32_t* lidx, LevelNodes nd, uint32_t K,
                const uint32_t* woff, uint32_t w_begin_node, uint32_t w_end_node, double box,
                int sx, int level0, NodeScratch sc, uint32_t* err) {
  __shared__ I128 red[TB / kWave][8];
  const uint32_t w0 = woff[w_begin_node], w1 = woff[w_end_node];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  for (uint32_t w = w0 + blockIdx.x; w < w1; w += gridDim.x) {
    const uint32_t k = seg_of(woff, K, w);
    const uint32_t t = w - woff[k];
    const uint32_t first = nd.first[k], cnt = nd.count[k];
    const uint32_t a = lidx[first];
    const double xa[3] = {(double)x[a], (double)y[a], (double)z[a]};
    I128 s[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) s[q] = i128_from(0);
    double umin[3] = {0, 0, 0}, umax[3] = {0, 0, 0};
    uint32_t bad = 0;
    for (uint32_t e = t * kMomTile + threadIdx.x; e < cnt && e < (t + 1) * kMomTile;
         e += TB) {
      const uint32_t i = lidx[first + e];
      const double p[3] = {(double)x[i], (double)y[i], (double)z[i]};
      const float v[3] = {vx[i], vy[i], vz[i]};
      long long q[3], wq[3];
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        double u = min_image(p[c] - xa[c], box);
        umin[c] = fmin(umin[c], u);
        umax[c] = fmax(umax[c], u);
        q[c] = quantise(u, sx);
        if (!(fabsf(v[c]) < 65536.0f)) bad = 1;
        wq[c] = quantise((double)v[c], kVelShift);
      }
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        s[c] = i128_add(s[c], i128_from(q[c]));
        s[4 + c] = i128_add(s[4 + c], i128_from(wq[c]));
      }
      s[3] = i128_add(s[3], i128_add(i128_sqr(q[0]), i128_add(i128_sqr(q[1]), i128_sqr(q[2]))));
      s[7] = i128_add(s[7],
                      i128_add(i128_sqr(wq[0]), i128_add(i128_sqr(wq[1]), i128_sqr(wq[2]))));
    }
    if (bad) atomicOr(err, kErrVelRange);
#pragma unroll
    for (int q = 0; q < 8; ++q) s[q] = wave_sum_i128(s[q]);
    if (level0) {
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        double mn = umin[c], mx = umax[c];
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) {
          mn = fmin(mn, __shfl_xor(mn, o));
          mx = fmax(mx, __shfl_xor(mx, o));
        }
        if (lane == 0) {
          atomicMin(sc.ext + 6 * k + c, f64_ord(mn));
          atomicMax(sc.ext + 6 * k + 3 + c, f64_ord(mx));
        }
      }
    }
    if (lane == 0) {
#pragma unroll
      for (int q = 0; q < 8; ++q) red[wid][q] = s[q];
    }
    __syncthreads();
    if (threadIdx.x < 8) {
      I128 tot = red[0][threadIdx.x];
      for (int ww = 1; ww < TB / kWave; ++ww) tot = i128_add(tot, red[ww][threadIdx.x]);
      atomic_add_i128(sc.acc + 8 * k + threadIdx.x, tot);
    }
    __syncthreads();
  }
}

// Mean and 3D variance from exact sums (same evaluation order as the
// definition in the header comment of libhalo.h).
__device__ void finish_moments(const I128* s, double n, int shift, double mean[3],
                               double* var) {
  double mq[3];
#pragma unroll
  for (int c = 0; c < 3; ++c) mq[c] = i128_to_f64(s[c]) / n;
  double s2q = i128_to_f64(s[3]) / n;
  double t = mq[0] * mq[0];
  t = __fma_rn(mq[1], mq[1], t);
  t = __fma_rn(mq[2], mq[2], t);
  double vq = s2q - t;
  if (!(vq > 0.0)) vq = 0.0;
#pragma unroll
  for (int c = 0; c < 3; ++c) mean[c] = ldexp(mq[c], -shift);
  *var = ldexp(vq, -2 * shift);
}

template <class T>
__global__ void k_mom_final(const T* x, const T* y, const T* z, const uint32_t* lidx,
                            LevelNodes nd, uint32_t k0, uint32_t k1, double box, int sx,
                            int level0, double f, NodeScratch sc, double* mom_out,
                            uint32_t* err) {
  uint32_t k = k0 + blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= k1) return;
  const double n = (double)nd.count[k];
  const uint32_t a = lidx[nd.first[k]];
  const double xa[3] = {(double)x[a], (double)y[a], (double)z[a]};
  double ubar[3], vbar[3], sx2, sv2;
  finish_moments(sc.acc + 8 * k, n, sx, ubar, &sx2);
  finish_moments(sc.acc + 8 * k + 4, n, kVelShift, vbar, &sv2);
  if (level0) {
    for (int c = 0; c < 3; ++c)
      if (ord_f64(sc.ext[6 * k + 3 + c]) - ord_f64(sc.ext[6 * k + c]) >= 0.5 * box)
        atomicOr(err, kErrGeometry);
  }
  double* mo = mom_out + 8 * (size_t)k;
  for (int c = 0; c < 3; ++c) {
    double cc = xa[c] + ubar[c];
    if (cc < 0.0)
      cc += box;
    else if (cc >= box)
      cc -= box;
    mo[c] = cc;
    mo[3 + c] = vbar[c];
  }
  mo[6] = sx2;
  mo[7] = sv2;
  double* pr = sc.prm + 12 * (size_t)k;
  bool active = (sx2 > 0.0) && (sv2 > 0.0);
  for (int c = 0; c < 3; ++c) {
    pr[c] = xa[c];
    pr[3 + c] = ubar[c];
    pr[6 + c] = vbar[c];
  }
  pr[9] = active ? 1.0 / sqrt(sx2) : 0.0;
  pr[10] = active ? 1.0 / sqrt(sv2) : 0.0;
  pr[11] = active ? 1.0 : 0.0;
  uint32_t kk = (uint32_t)ceil(f * n);
  if (kk < 1) kk = 1;
  if (kk > nd.count[k]) kk = nd.count[k];
  sc.kth[k] = kk;
  sc.ell2[k] = -1.0f;
  sc.whole[k] = 0;
  sc.nch[k] = 0;
  sc.fch[k] = 0xFFFFFFFFu;
}

// Normalised coordinates, written as six FP32 planes of stride S.
template <class T>
__global__ void k_norm6(const T* x, const T* y, const T* z, const float* vx, const float* vy,
                        const float* vz, const uint32_t* lidx, const uint32_t* lnode,
                        uint32_t m0, uint32_t m1, double box, NodeScratch sc, float* xi,
                        size_t S) {
  uint32_t m = m0 + blockIdx.x * blockDim.x + threadIdx.x;
  if (m >= m1) return;
  const uint32_t k = lnode[m];
  const double* pr = sc.prm + 12 * (size_t)k;
  if (pr[11] == 0.0) return;
  const uint32_t i = lidx[m];
  const double p[3] = {(double)x[i], (double)y[i], (double)z[i]};
  const float v[3] = {vx[i], vy[i], vz[i]};
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    double u = min_image(p[c] - pr[c], box);
    xi[(size_t)c * S + m] = (float)((u - pr[3 + c]) * pr[9]);
    xi[(size_t)(3 + c) * S + m] = (float)(((double)v[c] - pr[6 + c]) * pr[10]);
  }
}

// ------------------------------------------------------------ pair kernels --
// Nearest-neighbour work unit: 256 particles of a node (a block, four waves
// of 64) against one j-chunk.  The chunk is a multiple of 256 particles, at
// least jmin (kNNJ, or kNNJSmall on a small level, where more and shorter
// units spread its few nodes over more of the chip) and at most kSymJMax, so a
// chunk's j-minima fit in LDS.
__host__ __device__ __forceinline__ uint32_t nn_chunk(uint32_t n, uint32_t jmin) {
  uint32_t c = (n + 63u) / 64u;
  c = (c + 255u) & ~255u;
  return c < jmin ? jmin : (c > kSymJMax ? kSymJMax : c);
}

__host__ __device__ __forceinline__ uint32_t nn_units(uint32_t n, uint32_t jmin) {
  const uint32_t J = nn_chunk(n, jmin);
  return ((n + 255u) / 256u) * ((n + J - 1) / J);
}

// Units of the all-pairs nodes (those not searched by a tree).
__global__ void k_pair_items(const uint32_t* count, const double* prm, const uint32_t* gstate,
                             uint32_t K, uint32_t jmin, uint32_t* items) {
  uint32_t k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= K) return;
  const uint32_t n = count[k];
  const bool active = prm[12 * (size_t)k + 11] != 0.0;
  items[k] = (active && gstate[k] == 0u) ? nn_units(n, jmin) : 0u;
}


// The cross-lane minima work on FP32 bit patterns as unsigned integers: every
// value is a non-negative float or +inf, whose bits order like the values.
// Minimum over the wave's 64 lanes of each of d[0..7] (FP32 bits), transposed:
// lane l returns the minimum of d[u] with u = 4 b0 + 2 b1 + b2 (b0..b2 the low
// bits of l).  Each halving step keeps the half of the values selected by one
// lane bit and takes the partner's copy of the same half.
__device__ __forceinline__ uint32_t wave_min8(const uint32_t* d) {
  const uint32_t l = threadIdx.x & 63u;
  const bool b0 = l & 1u, b1 = l & 2u, b2 = l & 4u;
  uint32_t r1[4], r2[2];
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const uint32_t keep = b0 ? d[4 + k] : d[k];
    const uint32_t send = b0 ? d[k] : d[4 + k];
    r1[k] = min(keep, lane_xor1(send));
  }
#pragma unroll
  for (int k = 0; k < 2; ++k) {
    const uint32_t keep = b1 ? r1[2 + k] : r1[k];
    const uint32_t send = b1 ? r1[k] : r1[2 + k];
    r2[k] = min(keep, lane_xor2(send));
  }
  const uint32_t keep = b2 ? r2[1] : r2[0];
  const uint32_t send = b2 ? r2[0] : r2[1];
  uint32_t r = min(keep, lane_xor4(send));
  r = min(r, lane_xor8(r));
  r = min(r, lane_xor16(r));
  r = min(r, lane_xor32(r));
  return r;
}

__device__ __forceinline__ uint32_t wave_min1(uint32_t r) {
  r = min(r, lane_xor1(r));
  r = min(r, lane_xor2(r));
  r = min(r, lane_xor4(r));
  r = min(r, lane_xor8(r));
  r = min(r, lane_xor16(r));
  r = min(r, lane_xor32(r));
  return r;
}

// Pairs of the wave's particles with j in [j0, j1) (all j above every i of
// the wave), each pair evaluated once: the lane keeps its own minimum, and the
// minimum over the wave for each j goes to jmin[j - jc] (LDS, as FP32 bits).
// Lanes without a particle carry coordinates of 1e30, so their d2 is +inf.
__device__ __forceinline__ float nn_sym_span(const float* __restrict__ xi, size_t S,
                                             uint32_t first, uint32_t j0, uint32_t j1,
                                             uint32_t jc, const float* a, float best,
                                             uint32_t* jmin) {
  const uint32_t l = threadIdx.x & 63u;
  const uint32_t ul = ((l & 1u) << 2) | (l & 2u) | ((l >> 2) & 1u);
  uint32_t j = j0;
  for (; j + 8 <= j1; j += 8) {
    float b[6][8];
#pragma unroll
    for (int c = 0; c < 6; ++c) {
      const float* __restrict__ p = xi + (size_t)c * S + first + j;
#pragma unroll
      for (int u = 0; u < 8; ++u) b[c][u] = p[u];
    }
    uint32_t d[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const float e = d2_6(a[0], a[1], a[2], a[3], a[4], a[5], b[0][u], b[1][u], b[2][u],
                           b[3][u], b[4][u], b[5][u]);
      best = fminf(best, e);
      d[u] = __float_as_uint(e);
    }
    const uint32_t r = wave_min8(d);
    if (l < 8u) atomicMin(jmin + (j - jc + ul), r);
  }
  for (; j < j1; ++j) {
    const uint32_t g = first + j;
    const float d = d2_6(a[0], a[1], a[2], a[3], a[4], a[5], xi[g], xi[S + g], xi[2 * S + g],
                         xi[3 * S + g], xi[4 * S + g], xi[5 * S + g]);
    best = fminf(best, d);
    const uint32_t r = wave_min1(__float_as_uint(d));
    if (l == 0u) atomicMin(jmin + (j - jc), r);
  }
  return best;
}

// Nearest-neighbour squared distance: D[i] = min_{j != i in node} d2(i, j),
// over the units [woff[kb], woff[ke]).  Each unordered pair of 64-particle
// tiles is evaluated once, by the wave owning the lower tile; the tile itself
// is evaluated in full.  Minima are folded into D with atomic min on the FP32
// bits (non-negative floats order as integers), skipped when D is already
// lower.
__global__ void __launch_bounds__(TB)
    k_nn(const float* __restrict__ xi, size_t S, LevelNodes nd, uint32_t K,
         const uint32_t* __restrict__ woff, uint32_t kb, uint32_t ke, uint32_t* ctr,
         uint32_t chmin, uint32_t* D) {
  __shared__ uint32_t jmin[kSymJMax];
  __shared__ uint32_t su;
  const uint32_t inf = 0x7F800000u;
  const uint32_t u0 = woff[kb], u1 = woff[ke];
  for (uint32_t t = 0;; ++t) {
    uint32_t v;
    if (ctr) {
      __syncthreads();
      if (threadIdx.x == 0) su = atomicAdd(ctr, 1u);
      __syncthreads();
      v = su;
    } else {
      v = blockIdx.x + t * gridDim.x;
    }
    const uint32_t u = u0 + __builtin_amdgcn_readfirstlane(v);
    if (u >= u1) break;
    const uint32_t k = seg_of(woff, K, u);
    const uint32_t local = u - woff[k];
    const uint32_t first = nd.first[k], n = nd.count[k];
    const uint32_t J = nn_chunk(n, chmin);
    const uint32_t nb = (n + 255u) / 256u;
    const uint32_t c = local / nb, b = local - c * nb;
    const uint32_t j0 = c * J, j1 = min(j0 + J, n);
    if (j1 <= b * 256u) continue;  // chunk below the block's particles (block-uniform)
    // the wave's tile (readfirstlane: uniform to the compiler, so spans stay scalar)
    const uint32_t t0 = __builtin_amdgcn_readfirstlane(b * 256u + (threadIdx.x & ~63u));
    const uint32_t li = t0 + (threadIdx.x & 63u);
    const bool ok = li < n;
    const uint32_t gi = first + (ok ? li : 0u);
    float a[6];
#pragma unroll
    for (int q = 0; q < 6; ++q) a[q] = ok ? xi[(size_t)q * S + gi] : 1e30f;
    for (uint32_t q = threadIdx.x; q < j1 - j0; q += TB) jmin[q] = inf;
    __syncthreads();
    float best = __int_as_float(inf);
    if (t0 < n) {
      if (t0 >= j0 && t0 < j1)
        best = nn_span<true>(xi, S, first + t0, first + min(t0 + 64u, n), first + li, a, best);
      const uint32_t js = max(j0, t0 + 64u);
      if (js < j1) best = nn_sym_span(xi, S, first, js, j1, j0, a, best, jmin);
    }
    __syncthreads();
    for (uint32_t q = threadIdx.x; q < j1 - j0; q += TB) {
      const uint32_t m = jmin[q];
      if (m < D[first + j0 + q]) atomicMin(D + first + j0 + q, m);
    }
    if (ok && __float_as_uint(best) < D[gi]) atomicMin(D + gi, __float_as_uint(best));
  }
}

// Particles that can link (D <= ell^2) of the all-pairs nodes, compacted in
// level order so that each node's linkable particles stay contiguous.
__global__ void k_link_flags(const uint32_t* lnode, const uint32_t* D, uint32_t M,
                             NodeScratch sc, uint32_t* flag) {
  uint32_t m = blockIdx.x * blockDim.x + threadIdx.x;
  if (m >= M) return;
  const uint32_t k = lnode[m];
  flag[m] = (sc.prm[12 * (size_t)k + 11] != 0.0 && sc.gstate[k] != 1u &&
             __uint_as_float(D[m]) <= sc.ell2[k])
                ? 1u
                : 0u;
}

__global__ void k_link_gather(const float* xi, size_t S, const uint32_t* flag,
                              const uint32_t* pos, uint32_t M, float* cxi, uint32_t* lpos) {
  uint32_t m = blockIdx.x * blockDim.x + threadIdx.x;
  if (m >= M || !flag[m]) return;
  const uint32_t c = pos[m];
  lpos[c] = m;
#pragma unroll
  for (int p = 0; p < 6; ++p) cxi[(size_t)p * S + c] = xi[(size_t)p * S + m];
}

__global__ void k_link_nodes(LevelNodes nd, const uint32_t* pos, uint32_t K, LevelNodes cn) {
  uint32_t k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= K) return;
  const uint32_t a = pos[nd.first[k]], b = pos[nd.first[k] + nd.count[k]];
  cn.first[k] = a;
  cn.count[k] = b - a;
}

__global__ void k_link_items(const uint32_t* ccount, uint32_t K, uint32_t pj, uint32_t* items) {
  uint32_t k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= K) return;
  const uint32_t n = ccount[k];
  items[k] = ((n + kPairI - 1) / kPairI) * ((n + pj - 1) / pj);
}

// One block of at most 64 j (node-local [jb, je)) against the wave's particles:
// bit q of the lane's mask marks j = jb + q as a friend of particle li.  rootv
// holds roots of the block's particles found when its tile was staged; a lane
// joins its set with a friend only when that root differs from its own (a
// skipped pair had equal roots at some point, and sets only merge).
// kDiag: the block holding the wave's own particles, where only j > i counts.
template <bool kDiag>
__device__ __forceinline__ void fof_block(const float* __restrict__ cxi, size_t S,
                                          uint32_t first, uint32_t jb, uint32_t je,
                                          uint32_t li, bool ok, const float* a, float l2,
                                          const uint32_t* __restrict__ lpos, uint32_t mi,
                                          uint32_t& ri, uint32_t* par, const uint32_t* rootv) {
  unsigned long long fm = 0ull;
  uint32_t j = jb;
  for (; j + 8 <= je; j += 8) {
    float b[6][8];
#pragma unroll
    for (int c = 0; c < 6; ++c) {
      const float* __restrict__ p = cxi + (size_t)c * S + first + j;
#pragma unroll
      for (int u = 0; u < 8; ++u) b[c][u] = p[u];
    }
    uint32_t m8 = 0;  // bit u: j + u is a friend (built from u = 7 down to 0)
#pragma unroll
    for (int u = 7; u >= 0; --u) {
      const float d = d2_6(a[0], a[1], a[2], a[3], a[4], a[5], b[0][u], b[1][u], b[2][u],
                           b[3][u], b[4][u], b[5][u]);
      const bool f = ok && d <= l2 && (!kDiag || j + u > li);
      m8 = 2u * m8 + (f ? 1u : 0u);
    }
    fm |= (unsigned long long)m8 << (j - jb);
  }
  for (; j < je; ++j) {
    const uint32_t g = first + j;
    const float d = d2_6(a[0], a[1], a[2], a[3], a[4], a[5], cxi[g], cxi[S + g],
                         cxi[2 * S + g], cxi[3 * S + g], cxi[4 * S + g], cxi[5 * S + g]);
    const bool f = ok && d <= l2 && (!kDiag || j > li);
    fm |= f ? (1ull << (j - jb)) : 0ull;
  }
  while (fm) {
    const uint32_t q = (uint32_t)__builtin_ctzll(fm);
    fm &= fm - 1ull;
    if (rootv[q] != ri) ri = uf_union(par, mi, lpos[first + jb + q]);
  }
}

// 6D FOF at ell^2 over the compacted linkable particles of all-pairs nodes,
// pairs j > i.  Work item: kPairI particles of a node (a block, one per
// thread) against a kPairJ chunk, taken in tiles of TB: the block finds the
// roots of a tile's particles (one per thread, into LDS), then each wave
// streams the tile's coordinates as scalar loads in blocks of 64.
__global__ void __launch_bounds__(TB)
    k_fof6(const float* __restrict__ cxi, size_t S, LevelNodes cn,
           const uint32_t* __restrict__ lpos, uint32_t K, const uint32_t* __restrict__ woff,
           uint32_t kb, uint32_t ke, uint32_t* ctr, const float* __restrict__ ell2,
           uint32_t pj, uint32_t* par) {
  __shared__ uint32_t troot[TB];
  __shared__ uint32_t su;
  const uint32_t u0 = woff[kb], u1 = woff[ke];
  for (uint32_t t = 0;; ++t) {
    uint32_t v;
    if (ctr) {
      __syncthreads();
      if (threadIdx.x == 0) su = atomicAdd(ctr, 1u);
      __syncthreads();
      v = su;
    } else {
      v = blockIdx.x + t * gridDim.x;
    }
    const uint32_t u = u0 + __builtin_amdgcn_readfirstlane(v);
    if (u >= u1) break;
    const uint32_t k = seg_of(woff, K, u);
    const uint32_t r = u - woff[k];
    const uint32_t first = cn.first[k], n = cn.count[k];
    const uint32_t tj = (n + pj - 1) / pj;
    const uint32_t it = r / tj, jc = r - it * tj;
    const uint32_t i0 = it * kPairI;
    const uint32_t j0 = jc * pj, j1 = min(n, j0 + pj);
    if (j1 <= i0 + 1) continue;  // block-uniform: no pair with j > i
    const uint32_t li = i0 + threadIdx.x;
    const bool ok = li < n;
    const uint32_t gi = first + (ok ? li : 0u);
    const uint32_t mi = lpos[gi];
    uint32_t ri = mi;
    const float l2 = ell2[k];
    float a[6];
#pragma unroll
    for (int q = 0; q < 6; ++q) a[q] = cxi[(size_t)q * S + gi];
    const uint32_t w0 = i0 + (threadIdx.x & ~63u);  // the wave's first particle
    for (uint32_t jt = max(j0, i0); jt < j1; jt += TB) {
      __syncthreads();
      const uint32_t lj = jt + threadIdx.x;
      troot[threadIdx.x] = lj < j1 ? uf_find(par, lpos[first + lj]) : 0xFFFFFFFFu;
      if (ok) ri = uf_find(par, mi);  // a current root: more blocks can be skipped
      __syncthreads();
      const uint32_t te = min(jt + TB, j1);
      for (uint32_t jb = jt; jb < te; jb += 64u) {
        if (jb < w0) continue;  // every j of the block is below the wave's i
        const uint32_t je = min(jb + 64u, te);
        // a block whose particles all share the root of all the wave's
        // particles holds no pair that can join two sets
        const uint32_t r0 = __builtin_amdgcn_readfirstlane(ri);
        const uint32_t q = jb + (threadIdx.x & 63u);
        if (__all((!ok || ri == r0) && (q >= je || troot[q - jt] == r0))) continue;
        if (jb == w0)
          fof_block<true>(cxi, S, first, jb, je, li, ok, a, l2, lpos, mi, ri, par,
                          troot + (jb - jt));
        else
          fof_block<false>(cxi, S, first, jb, je, li, ok, a, l2, lpos, mi, ri, par,
                           troot + (jb - jt));
      }
    }
  }
}

// ------------------------------------------------------------ selection ----
// Radix-select step over a 256-bin histogram, one wave: lane l holds bins
// 4l..4l+3 in c[].  Finds the bin d where the running count first reaches kk
// (kk >= 1) and returns it with kk minus the count before d, in every lane;
// d = 256 when the histogram holds fewer than kk values.
__device__ __forceinline__ void wave_select_bin(const uint32_t* c, uint32_t kk, uint32_t& d,
                                                uint32_t& rest) {
  const uint32_t lane = threadIdx.x & 63u;
  const uint32_t s = c[0] + c[1] + c[2] + c[3];
  uint32_t inc = s;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const uint32_t t = __shfl_up(inc, o);
    if ((int)lane >= o) inc += t;
  }
  const uint32_t exc = inc - s;
  const unsigned long long hit = __ballot(kk > exc && kk <= inc);
  uint32_t dd = 256u, rr = kk;
  if (hit) {
    const int L = __ffsll((long long)hit) - 1;
    if ((int)lane == L) {
      uint32_t run = exc;
      for (int q = 0; q < 4; ++q) {
        if (run + c[q] >= kk) {
          dd = 4u * lane + q;
          rr = kk - run;
          break;
        }
        run += c[q];
      }
    }
    dd = __shfl(dd, L);
    rr = __shfl(rr, L);
  }
  d = dd;
  rest = rr;
}

// ell^2 of nodes with at most kSelSmall particles: radix select in LDS.
__global__ void __launch_bounds__(TB)
    k_select_small(const uint32_t* D, LevelNodes nd, uint32_t k0, uint32_t k1,
                   NodeScratch sc) {
  __shared__ uint32_t v[kSelSmall];
  __shared__ uint32_t hist[256];
  __shared__ uint32_t s_pre, s_k;
  const uint32_t k = k0 + blockIdx.x;
  if (k >= k1) return;
  const uint32_t n = nd.count[k];
  if (n > kSelSmall || sc.prm[12 * (size_t)k + 11] == 0.0) return;
  const uint32_t first = nd.first[k];
  for (uint32_t e = threadIdx.x; e < n; e += TB) v[e] = D[first + e];
  if (threadIdx.x == 0) {
    s_pre = 0;
    s_k = sc.kth[k];
  }
  __syncthreads();
  for (int pass = 0; pass < 4; ++pass) {
    const int shift = 24 - 8 * pass;
    hist[threadIdx.x] = 0;
    __syncthreads();
    const uint32_t pre = s_pre;
    for (uint32_t e = threadIdx.x; e < n; e += TB) {
      uint32_t b = v[e];
      if (pass == 0 || (b >> (shift + 8)) == (pre >> (shift + 8)))
        atomicAdd(&hist[(b >> shift) & 255u], 1u);
    }
    __syncthreads();
    if (threadIdx.x < 64) {
      uint32_t c[4];
      for (int q = 0; q < 4; ++q) c[q] = hist[4 * threadIdx.x + q];
      uint32_t d, rest;
      wave_select_bin(c, s_k, d, rest);
      if (threadIdx.x == 0 && d < 256u) {
        s_pre = pre | (d << shift);
        s_k = rest;
      }
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) sc.ell2[k] = __uint_as_float(s_pre);
}

// ------------------------------------------------------- subset ell ----
// Section 3.2: in large groups the nearest neighbours are found for a random
// subset only.  A particle of a node of n > m particles belongs to the subset
// when SplitMix64 (Steele, Lea & Flood 2014) of its input index times n is
// below m 2^64 (exact 128-bit comparison): probability m / n, expected size m.
// Its nearest-neighbour distance is the exact one against the whole node, so
// D stays exact for every particle (the 6D FOF pass prunes with it); only the
// selection of ell^2 reads the subset.
__device__ __forceinline__ unsigned long long splitmix64(unsigned long long x) {
  unsigned long long z = x + 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

__device__ __forceinline__ bool in_subset(uint32_t index, uint32_t n, uint32_t m) {
  if (n <= m) return true;
  const unsigned __int128 l = (unsigned __int128)splitmix64(index) * n;
  return l < ((unsigned __int128)m << 64);
}

// nsub[k] = subset size of each node above m (zero-initialised).
__global__ void k_subset_count(const uint32_t* perm, const uint32_t* lidx, const uint32_t* lnode,
                               LevelNodes nd, uint32_t Mi, uint32_t m, uint32_t* nsub) {
  const uint32_t q = blockIdx.x * blockDim.x + threadIdx.x;
  const bool ok = q < Mi;
  const uint32_t k = ok ? lnode[q] : 0u;
  const uint32_t n = ok ? nd.count[k] : 0u;
  agg_add_u32(nsub, k, 1u, ok && n > m && in_subset(perm[lidx[q]], n, m));
}

// Dsel = D on the subset, +inf elsewhere; a node whose draw came out empty
// keeps every particle.
__global__ void k_subset_sel(const uint32_t* perm, const uint32_t* lidx, const uint32_t* lnode,
                             LevelNodes nd, uint32_t Mi, uint32_t m, const uint32_t* nsub,
                             const uint32_t* D, uint32_t* Dsel) {
  const uint32_t q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= Mi) return;
  const uint32_t k = lnode[q], n = nd.count[k];
  const bool keep = n <= m || nsub[k] == 0u || in_subset(perm[lidx[q]], n, m);
  Dsel[q] = keep ? D[q] : 0x7F800000u;
}

// Rank of ell^2 within the subset: ceil(f n_sub), clamped to [1, n_sub].
__global__ void k_subset_kth(LevelNodes nd, uint32_t K, uint32_t m, double f,
                             const uint32_t* nsub, NodeScratch sc) {
  const uint32_t k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= K || nd.count[k] <= m || nsub[k] == 0u) return;
  const uint32_t ns = nsub[k];
  uint32_t kk = (uint32_t)ceil(f * ns);
  if (kk < 1) kk = 1;
  if (kk > ns) kk = ns;
  sc.kth[k] = kk;
}

__global__ void k_big_flags(LevelNodes nd, uint32_t K, NodeScratch sc, uint32_t* flag) {
  uint32_t k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= K) return;
  flag[k] = (nd.count[k] > kSelSmall && sc.prm[12 * (size_t)k + 11] != 0.0) ? 1u : 0u;
}

__global__ void k_big_list(const uint32_t* flag, const uint32_t* pos, uint32_t K,
                           LevelNodes nd, NodeScratch sc) {
  uint32_t k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= K) return;
  if (flag[k]) {
    uint32_t b = pos[k];
    sc.big[b] = k;
    sc.wbig[b] = (nd.count[k] + kSelTile - 1) / kSelTile;
    sc.selp[2 * b] = 0;
    sc.selp[2 * b + 1] = sc.kth[k];
  }
}

__global__ void k_zero_hist(NodeScratch sc, const uint32_t* nbig) {
  uint32_t e = blockIdx.x * blockDim.x + threadIdx.x;
  for (; e < 256u * nbig[0]; e += gridDim.x * blockDim.x) sc.ghist[e] = 0;
}

__global__ void __launch_bounds__(TB)
    k_select_big_hist(const uint32_t* D, LevelNodes nd, NodeScratch sc, const uint32_t* nbig,
                      int pass) {
  __shared__ uint32_t hist[256];
  const uint32_t B = nbig[0];
  const uint32_t W = sc.wbig[B];  // total items (exclusive scan total)
  const int shift = 24 - 8 * pass;
  for (uint32_t w = blockIdx.x; w < W; w += gridDim.x) {
    const uint32_t b = seg_of(sc.wbig, B, w);
    const uint32_t t = w - sc.wbig[b];
    const uint32_t k = sc.big[b];
    const uint32_t first = nd.first[k], n = nd.count[k];
    const uint32_t pre = sc.selp[2 * b];
    hist[threadIdx.x] = 0;
    __syncthreads();
    for (uint32_t e = t * kSelTile + threadIdx.x; e < n && e < (t + 1) * kSelTile; e += TB) {
      uint32_t bits = D[first + e];
      if (pass == 0 || (bits >> (shift + 8)) == (pre >> (shift + 8)))
        atomicAdd(&hist[(bits >> shift) & 255u], 1u);
    }
    __syncthreads();
    if (hist[threadIdx.x]) atomicAdd(sc.ghist + 256 * (size_t)b + threadIdx.x, hist[threadIdx.x]);
    __syncthreads();
  }
}

// One wave per big node: reads and clears its histogram, then narrows the
// prefix and the rank to the selected bin.  The value goes to the node's
// ell^2, or, with out, to out[omap[b]].
__global__ void k_select_big_resolve(NodeScratch sc, const uint32_t* nbig, int pass, float* out,
                                     const uint32_t* omap) {
  const uint32_t B = nbig[0];
  const int shift = 24 - 8 * pass;
  const uint32_t lane = threadIdx.x & 63u;
  const uint32_t nw = (gridDim.x * blockDim.x) >> 6;
  for (uint32_t b = (blockIdx.x * blockDim.x + threadIdx.x) >> 6; b < B; b += nw) {
    uint32_t* h = sc.ghist + 256 * (size_t)b;
    uint32_t c[4];
    for (int q = 0; q < 4; ++q) {
      c[q] = h[4 * lane + q];
      h[4 * lane + q] = 0;
    }
    const uint32_t kk = sc.selp[2 * b + 1];
    uint32_t pre = sc.selp[2 * b];
    uint32_t d = 256u, rest = kk;
    if (kk != 0) wave_select_bin(c, kk, d, rest);
    if (d < 256u) pre |= d << shift;
    if (lane == 0) {
      if (d < 256u) {
        sc.selp[2 * b] = pre;
        sc.selp[2 * b + 1] = rest;
      }
      if (pass == 3) (out ? out[omap[b]] : sc.ell2[sc.big[b]]) = __uint_as_float(pre);
    }
  }
}

// ------------------------------------------- nearest-neighbour bracket ----
// ell^2 is the kth smallest D of a node, and only the points whose D lies
// near it need their exact distance: a point with D < ell^2 is linkable
// whatever its D, one with D > ell^2 is not.  For a tree node of more than
// kSelSmall points, the exact D of every kNNSample-th sorted point brackets
// the kth value by two sample order statistics [tl, th), kBracketSigma
// binomial standard deviations of the sample rank either side; the walks of
// all points then start with th as their best distance and end once it is
// below tl.  The stored D is exact inside [tl, th), below tl where the true
// one is, and th where the true one is th or more, so the kth smallest stored
// value is the exact ell^2 whenever it lies inside [tl, th); otherwise the
// node's walks are run again without a bracket.
constexpr uint32_t kNNSample = 64;
constexpr double kBracketSigma = 4.0;

// Sample count and 1-based sample ranks [rlo, rhi] bracketing the node's kth
// value; rlo < 1: no lower bound, rhi > ms: no upper bound.
__device__ __forceinline__ void bracket_ranks(uint32_t n, uint32_t kth, uint32_t p0, double z,
                                              uint32_t& ms, int64_t& rlo, int64_t& rhi) {
  ms = (p0 + n + kNNSample - 1) / kNNSample - (p0 + kNNSample - 1) / kNNSample;
  const double rho = ((double)kth - 0.5) / (double)n;
  const double c = rho * (double)ms;
  const double sig = sqrt((double)ms * rho * (1.0 - rho)) + 1.0;
  rlo = (int64_t)floor(c - z * sig);
  rhi = (int64_t)ceil(c + z * sig) + 1;
}

__global__ void k_bracket_flags(GridBufs g, LevelNodes nd, uint32_t NB, uint32_t* flag) {
  const uint32_t b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= NB) return;
  flag[b] = nd.count[g.gnode[b]] > (uint32_t)kSelSmall ? 1u : 0u;
  g.tl[b] = 0.0f;
  g.th[b] = __int_as_float(0x7F800000);
}

// The selection list of the bracketed trees for sample rank rlo (hi = 0) or
// rhi (hi = 1); a rank outside the sample selects nothing (kth 0).
__global__ void k_bracket_list(GridBufs g, LevelNodes nd, NodeScratch sc, uint32_t NB,
                               const uint32_t* flag, const uint32_t* pos, double z, int hi) {
  const uint32_t b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= NB || !flag[b]) return;
  const uint32_t k = g.gnode[b], n = nd.count[k], i = pos[b];
  uint32_t ms;
  int64_t rlo, rhi;
  bracket_ranks(n, sc.kth[k], g.pstart[b], z, ms, rlo, rhi);
  const int64_t r = hi ? rhi : rlo;
  sc.big[i] = k;
  sc.wbig[i] = (n + kSelTile - 1) / kSelTile;
  sc.selp[2 * i] = 0;
  sc.selp[2 * i + 1] = (r >= 1 && r <= (int64_t)ms) ? (uint32_t)r : 0u;
  g.tmap[i] = b;
}

// Ranks outside the sample: no bound on that side.  An empty bracket (equal
// sample values) would always fail, so such a tree walks without one.
__global__ void k_bracket_final(GridBufs g, LevelNodes nd, NodeScratch sc, uint32_t NB,
                                const uint32_t* flag, double z) {
  const uint32_t b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= NB || !flag[b]) return;
  const uint32_t k = g.gnode[b];
  uint32_t ms;
  int64_t rlo, rhi;
  bracket_ranks(nd.count[k], sc.kth[k], g.pstart[b], z, ms, rlo, rhi);
  float lo = g.tl[b], hi = g.th[b];
  if (rlo < 1) lo = 0.0f;
  if (rhi > (int64_t)ms) hi = __int_as_float(0x7F800000);
  if (!(lo < hi)) {
    lo = 0.0f;
    hi = __int_as_float(0x7F800000);
  }
  g.tl[b] = lo;
  g.th[b] = hi;
}

// A tree whose ell^2 fell outside its bracket walks again without one.
__global__ void k_bracket_check(GridBufs g, NodeScratch sc, uint32_t NB, uint32_t* nredo) {
  const uint32_t b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= NB) return;
  const float lo = g.tl[b], hi = g.th[b];
  const bool bracketed = lo > 0.0f || hi < __int_as_float(0x7F800000);
  const float l2 = sc.ell2[g.gnode[b]];
  const bool redo = bracketed && !(l2 >= lo && l2 < hi);
  g.redo[b] = redo ? 1u : 0u;
  if (redo) atomicAdd(nredo, 1u);
}

// ------------------------------------------------------------ children -----
__global__ void k_comp_size(const uint32_t* par, const uint32_t* lnode, uint32_t M,
                            NodeScratch sc, uint32_t* csize) {
  const uint32_t m = blockIdx.x * blockDim.x + threadIdx.x;
  const bool ok = m < M && sc.prm[12 * (size_t)lnode[m < M ? m : 0] + 11] != 0.0;
  agg_add_u32(csize, ok ? par[m] : 0u, 1u, ok);
}

__global__ void k_whole(const uint32_t* par, const uint32_t* lnode, const uint32_t* csize,
                        uint32_t M, LevelNodes nd, NodeScratch sc) {
  uint32_t m = blockIdx.x * blockDim.x + threadIdx.x;
  if (m >= M) return;
  const uint32_t k = lnode[m];
  if (sc.prm[12 * (size_t)k + 11] == 0.0) return;
  if (par[m] == m && csize[m] == nd.count[k]) sc.whole[k] = 1u;
}

__global__ void k_child_flags(const uint32_t* par, const uint32_t* lnode,
                              const uint32_t* csize, uint32_t M, uint32_t mm, NodeScratch sc,
                              uint32_t* cflag, uint32_t* head) {
  uint32_t m = blockIdx.x * blockDim.x + threadIdx.x;
  if (m >= M) return;
  const uint32_t k = lnode[m];
  bool child = sc.prm[12 * (size_t)k + 11] != 0.0 && sc.whole[k] == 0 && csize[par[m]] >= mm;
  cflag[m] = child ? 1u : 0u;
  head[m] = (child && par[m] == m) ? 1u : 0u;
}

__global__ void k_child_nodes(const uint32_t* par, const uint32_t* lnode,
                              const uint32_t* csize, const uint32_t* perm, const uint32_t* lidx,
                              const uint32_t* hrank, const uint32_t* head, uint32_t M,
                              LevelNodes nd, int32_t base, NodeScratch sc, LevelNodes nx,
                              uint32_t* cid) {
  uint32_t m = blockIdx.x * blockDim.x + threadIdx.x;
  if (m >= M || !head[m]) return;
  const uint32_t k = lnode[m];
  const uint32_t c = hrank[m];
  nx.count[c] = csize[m];
  nx.canon[c] = perm[lidx[m]];
  nx.parent[c] = base + (int32_t)k;
  nx.fof[c] = nd.fof[k];
  cid[m] = c;
  atomicAdd(sc.nch + k, 1u);
  atomicMin(sc.fch + k, c);
}

__global__ void k_child_keys(const uint32_t* par, const uint32_t* cflag, const uint32_t* crank,
                             const uint32_t* cid, uint32_t M, uint32_t* key, uint32_t* val) {
  uint32_t m = blockIdx.x * blockDim.x + threadIdx.x;
  if (m >= M || !cflag[m]) return;
  const uint32_t p = crank[m];
  key[p] = cid[par[m]];
  val[p] = m;
}

__global__ void k_next_level(const uint32_t* skey, const uint32_t* sval, const uint32_t* lidx,
                             uint32_t M2, uint32_t* lidx2, uint32_t* lnode2) {
  uint32_t q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= M2) return;
  lidx2[q] = lidx[sval[q]];
  lnode2[q] = skey[q];
}

__global__ void k_next_first(const uint32_t* skey, uint32_t M2, uint32_t* first2) {
  uint32_t q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= M2) return;
  if (q == 0 || skey[q] != skey[q - 1]) first2[skey[q]] = q;
}

__global__ void k_deepest(const uint32_t* perm, const uint32_t* lidx, const uint32_t* lnode,
                          uint32_t M, int32_t base, int32_t* deepest) {
  uint32_t m = blockIdx.x * blockDim.x + threadIdx.x;
  if (m >= M) return;
  deepest[perm[lidx[m]]] = base + (int32_t)lnode[m];
}

__global__ void k_node_out(LevelNodes nd, uint32_t K, int32_t base, int32_t level,
                           int32_t next_base, const double* mom, NodeScratch sc,
                           libhalo_nodes out) {
  uint32_t k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= K) return;
  const int64_t row = (int64_t)base + k;
  if (row >= out.cap) return;
  const bool active = sc.prm[12 * (size_t)k + 11] != 0.0;
  const uint32_t nch = sc.nch[k];
  uint32_t flags = 0;
  if (nch == 0) flags |= LIBHALO_NODE_LEAF;
  if (!active) flags |= LIBHALO_NODE_DEGENERATE;
  if (sc.whole[k]) flags |= LIBHALO_NODE_WHOLE;
  out.parent[row] = nd.parent[k];
  out.level[row] = level;
  out.first_child[row] = nch ? next_base + (int32_t)sc.fch[k] : -1;
  out.n_children[row] = (int32_t)nch;
  out.count[row] = nd.count[k];
  out.canon[row] = nd.canon[k];
  out.fof[row] = nd.fof[k];
  out.flags[row] = flags;
  const double* mo = mom + 8 * (size_t)k;
  out.cx[row] = mo[0];
  out.cy[row] = mo[1];
  out.cz[row] = mo[2];
  out.vx[row] = mo[3];
  out.vy[row] = mo[4];
  out.vz[row] = mo[5];
  out.sx2[row] = mo[6];
  out.sv2[row] = mo[7];
  out.ell2[row] = active ? sc.ell2[k] : -1.0f;
}

// Every parent becomes its root (read-only walks; see uf_root).
__global__ void k_compress(uint32_t* par, uint32_t M) {
  uint32_t m = blockIdx.x * blockDim.x + threadIdx.x;
  if (m < M) uf_store(par + m, uf_root(par, m));
}

__global__ void k_fill_i32(int32_t* a, int64_t n, int32_t v) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) a[i] = v;
}

__global__ void k_zero_node_scratch(NodeScratch sc, uint32_t K) {
  uint32_t k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= K) return;
  for (int q = 0; q < 8; ++q) sc.acc[8 * (size_t)k + q] = I128{0ull, 0ll};
  for (int c = 0; c < 3; ++c) {
    sc.ext[6 * (size_t)k + c] = ~0ull;
    sc.ext[6 * (size_t)k + 3 + c] = 0ull;
  }
}

// ------------------------------------------------------------ host side ----
struct Rd {  // small read-back helper on the pinned host block
  Ctx& c;
  hipStream_t s;
  uint32_t* h;
  uint32_t get(const uint32_t* d, int slot = 0) {
    HALO_HIP(hipMemcpyAsync(h + slot, d, sizeof(uint32_t), hipMemcpyDeviceToHost, s));
    HALO_HIP(hipStreamSynchronize(s));
    return h[slot];
  }
};

template <class T>
void refine_impl(Ctx& ctx, int64_t n, const T* x, const T* y, const T* z, const float* vx,
                 const float* vy, const float* vz, const uint32_t* perm,
                 const uint32_t* grp_first, const uint32_t* grp_count, int64_t G,
                 libhalo_nodes* out, int32_t* deepest, int64_t* n_nodes, hipStream_t s) {
  const libhalo_params& P = ctx.p;
  const double box = P.box;
  int e2 = 0;
  frexp(0.5 * box, &e2);
  const int sx = 40 - e2;
  const bool plain = P.mode == LIBHALO_PLAIN;
  Rd rd{ctx, s, ctx.host_slot<uint32_t>(0)};

  *n_nodes = 0;
  if (G == 0) {
    k_fill_i32<<<blocks_for(n, TB), TB, 0, s>>>(deepest, n, -1);
    HALO_HIP(hipStreamSynchronize(s));
    return;
  }
  // number of members = first + count of the last group
  HALO_HIP(hipMemcpyAsync(rd.h, grp_first + G - 1, 4, hipMemcpyDeviceToHost, s));
  HALO_HIP(hipMemcpyAsync(rd.h + 1, grp_count + G - 1, 4, hipMemcpyDeviceToHost, s));
  HALO_HIP(hipStreamSynchronize(s));
  const uint32_t M = rd.h[0] + rd.h[1];
  const uint32_t Kmax = std::max<uint32_t>((uint32_t)G, M / (uint32_t)P.min_members + 1);

  // workspace (sized by a dry run of the same carving)
  uint32_t *lidx, *lnode, *lidx2, *lnode2, *D, *par, *csize, *cflag, *head, *crank, *hrank,
      *cid, *k0, *v0, *k1, *v1, *stmp, *dcnt, *lpos, *Dsel = nullptr, *nsub = nullptr;
  const uint32_t msub = (uint32_t)P.ell_subset;  // 0: exact ell
  float *xi, *cxi;
  Members<T> mem;
  LevelNodes cnodes;
  void* rtmp;
  double* mom;
  LevelNodes L[2];
  NodeScratch sc;
  GridBufs gb;
  MTree gtree;  // topology of the large nodes' trees
  gb.mt = &gtree;
  carve_workspace(ctx, [&](Arena& A) {
    lidx = A.take<uint32_t>(M);
    lnode = A.take<uint32_t>(M);
    lidx2 = A.take<uint32_t>(M);
    lnode2 = A.take<uint32_t>(M);
    xi = A.take<float>(6ull * M);
    mem.x = A.take<T>(M);
    mem.y = A.take<T>(M);
    mem.z = A.take<T>(M);
    mem.vx = A.take<float>(M);
    mem.vy = A.take<float>(M);
    mem.vz = A.take<float>(M);
    cxi = A.take<float>(6ull * M);
    lpos = A.take<uint32_t>(M + 1);
    cnodes.first = A.take<uint32_t>(Kmax + 1);
    cnodes.count = A.take<uint32_t>(Kmax + 1);
    D = A.take<uint32_t>(M + 1);
    if (msub > 0) {
      Dsel = A.take<uint32_t>(M + 1);
      nsub = A.take<uint32_t>(Kmax + 1);
    }
    par = A.take<uint32_t>(M + 1);
    csize = A.take<uint32_t>(M + 1);
    cflag = A.take<uint32_t>(M + 1);
    head = A.take<uint32_t>(M + 1);
    crank = A.take<uint32_t>(M + 1);
    hrank = A.take<uint32_t>(M + 1);
    cid = A.take<uint32_t>(M + 1);
    k0 = A.take<uint32_t>(M + 1);
    v0 = A.take<uint32_t>(M + 1);
    k1 = A.take<uint32_t>(M + 1);
    v1 = A.take<uint32_t>(M + 1);
    rtmp = A.take<char>(radix_tmp_bytes(M));
    stmp = A.take<uint32_t>(scan_tmp_elems<uint32_t>(M + 1));
    for (int q = 0; q < 2; ++q) {
      L[q].first = A.take<uint32_t>(Kmax + 1);
      L[q].count = A.take<uint32_t>(Kmax + 1);
      L[q].parent = A.take<int32_t>(Kmax + 1);
      L[q].fof = A.take<uint32_t>(Kmax + 1);
      L[q].canon = A.take<uint32_t>(Kmax + 1);
    }
    sc.gstate = A.take<uint32_t>(Kmax + 2);
    sc.acc = A.take<I128>(8ull * Kmax);
    sc.ext = A.take<unsigned long long>(6ull * Kmax);
    sc.prm = A.take<double>(12ull * Kmax);
    mom = A.take<double>(8ull * Kmax);
    sc.kth = A.take<uint32_t>(Kmax + 2);
    sc.ell2 = A.take<float>(Kmax + 2);
    sc.whole = A.take<uint32_t>(Kmax + 2);
    sc.nch = A.take<uint32_t>(Kmax + 2);
    sc.fch = A.take<uint32_t>(Kmax + 2);
    sc.wmom = A.take<uint32_t>(Kmax + 2);
    sc.wpair = A.take<uint32_t>(Kmax + 2);
    sc.big = A.take<uint32_t>(Kmax + 2);
    sc.wbig = A.take<uint32_t>(Kmax + 2);
    sc.selp = A.take<uint32_t>(2ull * (M / kSelSmall + 2));
    sc.ghist = A.take<uint32_t>(256ull * (M / kSelSmall + 2));
    dcnt = A.take<uint32_t>(16);
    grid_take(A, gb, M, Kmax, P.kd_leaf > 0 ? (uint32_t)P.kd_leaf : kKdLeaf);
  });
  // outputs are written only once the workspace is in place
  k_fill_i32<<<blocks_for(n, TB), TB, 0, s>>>(deepest, n, -1);

  HALO_HIP(hipMemsetAsync(ctx.d_err, 0, sizeof(uint32_t), s));
  k_level0<T><<<blocks_for(M, TB), TB, 0, s>>>(perm, grp_first, grp_count, (uint32_t)G, M,
                                               lidx, lnode, x, y, z, vx, vy, vz, mem);
  k_level0_nodes<<<blocks_for(G, TB), TB, 0, s>>>(perm, grp_first, grp_count, (uint32_t)G,
                                                  L[0]);
  uint32_t K = (uint32_t)G, Mi = M;
  int cur = 0;
  int32_t base = 0;
  std::vector<uint32_t> hcount;
  for (int level = 0; K > 0; ++level) {
    HALO_CHECK(level < P.max_levels, LIBHALO_EINVAL, "hierarchy deeper than max_levels");
    LevelNodes nd = L[cur], nx = L[cur ^ 1];
    const size_t S = Mi;  // plane stride of xi for this level
    // persistent grids sized to the level: units are fetched from a counter, so
    // any grid is correct, and a deep level's few units need no 4096 blocks
    const unsigned pgrid = (unsigned)std::min<uint64_t>(
        kPersist, std::max<uint64_t>(256, 4 * (((uint64_t)Mi + 255) / 256)));
    // pair-unit chunks: shorter on small levels
    const bool small_level = Mi < kSmallLevel;
    const uint32_t nnj = small_level ? kNNJSmall
                                     : (P.nn_chunk > 0 ? (uint32_t)P.nn_chunk : (uint32_t)kNNJ);
    const uint32_t pj = small_level ? kPairJSmall
                                    : (P.fof_chunk > 0 ? (uint32_t)P.fof_chunk : (uint32_t)kPairJ);
    const int level0 = level == 0;
    k_zero_node_scratch<<<blocks_for(K, TB), TB, 0, s>>>(sc, K);
    k_mom_items<<<blocks_for(K, TB), TB, 0, s>>>(nd.count, K, sc.wmom);
    exclusive_scan<uint32_t>(sc.wmom, sc.wmom, K, sc.wmom + K, stmp, s);
    if (plain) {
      hcount.resize(K);
      HALO_HIP(hipMemcpyAsync(hcount.data(), nd.count, 4ull * K, hipMemcpyDeviceToHost, s));
      HALO_HIP(hipStreamSynchronize(s));
    }
    // 1. moments
    if (plain) {
      for (uint32_t k = 0; k < K; ++k) {
        unsigned g = (hcount[k] + kMomTile - 1) / kMomTile;
        HALO_PROF(ctx, "k_mom_accum", s, k_mom_accum<T><<<g, TB, 0, s>>>(mem.x, mem.y, mem.z, mem.vx, mem.vy, mem.vz, lidx, nd, K, sc.wmom, k, k + 1,
                                        box, sx, level0, sc, ctx.d_err));
        k_mom_final<T><<<1, 64, 0, s>>>(mem.x, mem.y, mem.z, lidx, nd, k, k + 1, box, sx, level0, P.f, sc,
                                        mom, ctx.d_err);
      }
    } else {
      HALO_PROF(ctx, "k_mom_accum", s, k_mom_accum<T><<<pgrid, TB, 0, s>>>(mem.x, mem.y, mem.z, mem.vx, mem.vy, mem.vz, lidx, nd, K, sc.wmom, 0, K,
                                             box, sx, level0, sc, ctx.d_err));
      k_mom_final<T><<<blocks_for(K, 128), 128, 0, s>>>(mem.x, mem.y, mem.z, lidx, nd, 0, K, box, sx,
                                                        level0, P.f, sc, mom, ctx.d_err);
    }
    if (level0) {
      uint32_t e = rd.get(ctx.d_err, 2);
      HALO_CHECK((e & kErrGeometry) == 0, LIBHALO_EGEOMETRY,
                 "a FOF group spans half the box or more");
      HALO_CHECK((e & kErrVelRange) == 0, LIBHALO_EINVAL, "a velocity is >= 2^16 km/s or NaN");
    }
    // 2. normalised coordinates
    k_norm6<T><<<blocks_for(Mi, TB), TB, 0, s>>>(mem.x, mem.y, mem.z, mem.vx, mem.vy, mem.vz, lidx, lnode, 0, Mi, box,
                                                 sc, xi, S);
    // 3. nearest neighbours: tree search for large nodes, all-pairs for the rest
    k_fill_u32<<<blocks_for(Mi, TB), TB, 0, s>>>(D, Mi, 0x7F800000u);
    k_iota<<<blocks_for(Mi, TB), TB, 0, s>>>(par, Mi);
    HALO_PROF(ctx, "grid_build", s,
              grid_build(gb, xi, S, nd, K, lnode, Mi, M, sc, rd.h + 8, s,
                         P.grid_min > 0 ? (uint32_t)P.grid_min : default_grid_min(Mi)));
    // a bracket of ell^2 from sampled walks, then every point's walk within it
    const bool bracket = msub == 0 && gb.NB > 0 && P.nn_bracket >= 0.0;
    const double zb = P.nn_bracket > 0.0 ? P.nn_bracket : kBracketSigma;
    if (bracket) {
      const uint32_t NB = gb.NB;
      HALO_PROF(ctx, "k_kd_walk_nn", s,
                grid_nn(gb, sc, D, kNNSample, nullptr, nullptr, nullptr, ctx.work_counters(),
                        s));
      k_bracket_flags<<<blocks_for(NB, TB), TB, 0, s>>>(gb, nd, NB, cflag);
      exclusive_scan<uint32_t>(cflag, head, NB, dcnt + 10, stmp, s);
      for (int hi = 0; hi < 2; ++hi) {
        k_fill_u32<<<blocks_for(NB + 1, TB), TB, 0, s>>>(sc.wbig, NB + 1, 0u);
        k_bracket_list<<<blocks_for(NB, TB), TB, 0, s>>>(gb, nd, sc, NB, cflag, head, zb, hi);
        exclusive_scan<uint32_t>(sc.wbig, sc.wbig, NB, sc.wbig + NB, stmp, s);
        k_zero_hist<<<64, TB, 0, s>>>(sc, dcnt + 10);
        for (int pass = 0; pass < 4; ++pass) {
          k_select_big_hist<<<pgrid, TB, 0, s>>>(D, nd, sc, dcnt + 10, pass);
          k_select_big_resolve<<<blocks_for(NB, TB / 64), TB, 0, s>>>(
              sc, dcnt + 10, pass, hi ? gb.th : gb.tl, gb.tmap);
        }
      }
      k_bracket_final<<<blocks_for(NB, TB), TB, 0, s>>>(gb, nd, sc, NB, cflag, zb);
      HALO_PROF(ctx, "k_kd_walk_nn", s,
                grid_nn(gb, sc, D, 1, gb.tl, gb.th, nullptr, ctx.work_counters(), s));
    } else {
      HALO_PROF(ctx, "k_kd_walk_nn", s,
                grid_nn(gb, sc, D, 1, nullptr, nullptr, nullptr, ctx.work_counters(), s));
    }
    k_pair_items<<<blocks_for(K, TB), TB, 0, s>>>(nd.count, sc.prm, sc.gstate, K, nnj,
                                                   sc.wpair);
    exclusive_scan<uint32_t>(sc.wpair, sc.wpair, K, sc.wpair + K, stmp, s);
    if (plain) {
      for (uint32_t k = 0; k < K; ++k) {
        uint32_t nn = hcount[k];
        const unsigned g = nn_units(nn, nnj);
        HALO_PROF(ctx, "k_nn", s,
                  k_nn<<<g, TB, 0, s>>>(xi, S, nd, K, sc.wpair, k, k + 1, nullptr, nnj, D));
        if (msub == 0 && nn <= (uint32_t)kSelSmall)
          HALO_PROF(ctx, "k_select_small", s,
                    k_select_small<<<1, TB, 0, s>>>(D, nd, k, k + 1, sc));
      }
    } else {
      k_fill_u32<<<1, 64, 0, s>>>(dcnt + 8, 1, 0u);
      HALO_PROF(ctx, "k_nn", s,
                k_nn<<<pgrid, TB, 0, s>>>(xi, S, nd, K, sc.wpair, 0, K, dcnt + 8, nnj, D));
      if (msub == 0)
        HALO_PROF(ctx, "k_select_small", s, k_select_small<<<K, TB, 0, s>>>(D, nd, 0, K, sc));
    }
    // subset form of ell (Section 3.2): select over the subset's distances
    const uint32_t* Dsl = msub > 0 ? Dsel : D;
    if (msub > 0) {
      k_fill_u32<<<blocks_for(K, TB), TB, 0, s>>>(nsub, K, 0u);
      k_subset_count<<<blocks_for(Mi, TB), TB, 0, s>>>(perm, lidx, lnode, nd, Mi, msub, nsub);
      k_subset_sel<<<blocks_for(Mi, TB), TB, 0, s>>>(perm, lidx, lnode, nd, Mi, msub, nsub, D,
                                                      Dsel);
      k_subset_kth<<<blocks_for(K, TB), TB, 0, s>>>(nd, K, msub, P.f, nsub, sc);
      HALO_PROF(ctx, "k_select_small", s, k_select_small<<<K, TB, 0, s>>>(Dsel, nd, 0, K, sc));
    }
    // 4. selection for big nodes (both forms: a handful of nodes)
    auto select_big = [&]() {
      k_big_flags<<<blocks_for(K, TB), TB, 0, s>>>(nd, K, sc, cflag);
      exclusive_scan<uint32_t>(cflag, head, K, dcnt, stmp, s);
      k_big_list<<<blocks_for(K, TB), TB, 0, s>>>(cflag, head, K, nd, sc);
      uint32_t nbig = rd.get(dcnt, 3);
      if (nbig > 0) {
        exclusive_scan<uint32_t>(sc.wbig, sc.wbig, nbig, sc.wbig + nbig, stmp, s);
        k_zero_hist<<<64, TB, 0, s>>>(sc, dcnt);
        for (int pass = 0; pass < 4; ++pass) {
          k_select_big_hist<<<pgrid, TB, 0, s>>>(Dsl, nd, sc, dcnt, pass);
          k_select_big_resolve<<<blocks_for(nbig, TB / 64), TB, 0, s>>>(sc, dcnt, pass,
                                                                        nullptr, nullptr);
        }
      }
    };
    if (Mi > (uint32_t)kSelSmall) select_big();  // else no node is above kSelSmall
    if (bracket) {  // ell^2 outside a tree's bracket: its exact walks, then select again
      k_fill_u32<<<1, 64, 0, s>>>(dcnt + 11, 1, 0u);
      k_bracket_check<<<blocks_for(gb.NB, TB), TB, 0, s>>>(gb, sc, gb.NB, dcnt + 11);
      if (rd.get(dcnt + 11, 16) > 0) {
        HALO_PROF(ctx, "k_kd_walk_nn", s,
                  grid_nn(gb, sc, D, 1, nullptr, nullptr, gb.redo, ctx.work_counters(), s));
        select_big();
      }
    }
    // 5. 6D FOF: all-pairs nodes over their compacted linkable particles
    k_link_flags<<<blocks_for(Mi, TB), TB, 0, s>>>(lnode, D, Mi, sc, cflag);
    exclusive_scan<uint32_t>(cflag, crank, Mi, crank + Mi, stmp, s);
    k_link_gather<<<blocks_for(Mi, TB), TB, 0, s>>>(xi, S, cflag, crank, Mi, cxi, lpos);
    k_link_nodes<<<blocks_for(K, TB), TB, 0, s>>>(nd, crank, K, cnodes);
    k_link_items<<<blocks_for(K, TB), TB, 0, s>>>(cnodes.count, K, pj, sc.wpair);
    exclusive_scan<uint32_t>(sc.wpair, sc.wpair, K, sc.wpair + K, stmp, s);
    if (plain) {
      for (uint32_t k = 0; k < K; ++k) {
        const uint32_t nn = hcount[k];
        const unsigned g = ((nn + kPairI - 1) / kPairI) * ((nn + pj - 1) / pj);
        HALO_PROF(ctx, "k_fof6", s,
                  k_fof6<<<g, TB, 0, s>>>(cxi, S, cnodes, lpos, K, sc.wpair, k, k + 1, nullptr,
                                          sc.ell2, pj, par));
      }
    } else {
      k_fill_u32<<<1, 64, 0, s>>>(dcnt + 8, 1, 0u);
      HALO_PROF(ctx, "k_fof6", s,
                k_fof6<<<pgrid, TB, 0, s>>>(cxi, S, cnodes, lpos, K, sc.wpair, 0, K,
                                               dcnt + 8, sc.ell2, pj, par));
    }
    HALO_PROF(ctx, "k_kd_group_fof", s, grid_fof_groups(gb, sc, D, par, s));
    HALO_PROF(ctx, "k_kd_walk_fof", s, grid_fof(gb, sc, D, par, ctx.work_counters(), s));
    k_compress<<<blocks_for(Mi, TB), TB, 0, s>>>(par, Mi);
    // 6. children
    k_fill_u32<<<blocks_for(Mi, TB), TB, 0, s>>>(csize, Mi, 0u);
    k_comp_size<<<blocks_for(Mi, TB), TB, 0, s>>>(par, lnode, Mi, sc, csize);
    k_whole<<<blocks_for(Mi, TB), TB, 0, s>>>(par, lnode, csize, Mi, nd, sc);
    k_child_flags<<<blocks_for(Mi, TB), TB, 0, s>>>(par, lnode, csize, Mi,
                                                    (uint32_t)P.min_members, sc, cflag, head);
    exclusive_scan<uint32_t>(head, hrank, Mi, dcnt, stmp, s);
    exclusive_scan<uint32_t>(cflag, crank, Mi, dcnt + 1, stmp, s);
    HALO_HIP(hipMemcpyAsync(rd.h + 4, dcnt, 8, hipMemcpyDeviceToHost, s));
    HALO_HIP(hipStreamSynchronize(s));
    const uint32_t K2 = rd.h[4], M2 = rd.h[5];
    const int32_t next_base = base + (int32_t)K;
    if (K2 > 0) {
      k_child_nodes<<<blocks_for(Mi, TB), TB, 0, s>>>(par, lnode, csize, perm, lidx, hrank, head, Mi,
                                                      nd, base, sc, nx, cid);
      k_child_keys<<<blocks_for(Mi, TB), TB, 0, s>>>(par, cflag, crank, cid, Mi, k0, v0);
      bool f = radix_sort_pairs<uint32_t>(k0, v0, k1, v1, M2, bits_for(K2), rtmp, s);
      uint32_t* sk = f ? k1 : k0;
      uint32_t* sv = f ? v1 : v0;
      k_next_level<<<blocks_for(M2, TB), TB, 0, s>>>(sk, sv, lidx, M2, lidx2, lnode2);
      k_next_first<<<blocks_for(M2, TB), TB, 0, s>>>(sk, M2, nx.first);
    }
    k_deepest<<<blocks_for(Mi, TB), TB, 0, s>>>(perm, lidx, lnode, Mi, base, deepest);
    k_node_out<<<blocks_for(K, TB), TB, 0, s>>>(nd, K, base, level, next_base, mom, sc, *out);
    base = next_base;
    K = K2;
    Mi = M2;
    std::swap(lidx, lidx2);
    std::swap(lnode, lnode2);
    cur ^= 1;
  }
  HALO_HIP(hipStreamSynchronize(s));
  *n_nodes = base;
  HALO_CHECK(base <= out->cap, LIBHALO_ECAPACITY, "node table too small");
}

}  // namespace

void refine6d(Ctx& ctx, int64_t n, int pos_dtype, const void* x, const void* y, const void* z,
              const float* vx, const float* vy, const float* vz, const uint32_t* perm,
              const uint32_t* grp_first, const uint32_t* grp_count, int64_t n_groups,
              libhalo_nodes* nodes, int32_t* deepest, int64_t* n_nodes, hipStream_t s) {
  if (pos_dtype == LIBHALO_F64)
    refine_impl<double>(ctx, n, (const double*)x, (const double*)y, (const double*)z, vx, vy,
                        vz, perm, grp_first, grp_count, n_groups, nodes, deepest, n_nodes, s);
  else
    refine_impl<float>(ctx, n, (const float*)x, (const float*)y, (const float*)z, vx, vy, vz,
                       perm, grp_first, grp_count, n_groups, nodes, deepest, n_nodes, s);
}

}  // namespace halo
