// Exact fixed-radius 6D neighbour search for large hierarchy nodes (the
// nearest-neighbour distances and 6D FOF of Section 3.2 without the
// all-pairs cost), as block-sparse all-pairs over bounding boxes.
//
// For each node above the grid threshold:
//   1. exact nearest-neighbour distances of a deterministic sample of kSamples
//      particles give an estimate of the linking length; the search radius
//      is R^2 = 2 x (the sample's f-quantile);
//   2. the node's particles are ordered along a 6D Morton curve (8 bits per
//      coordinate over [-A, A], clamped) and cut into tiles of 64; each tile
//      gets its 6D bounding box;
//   3. one wavefront per target tile tests the boxes of super-tiles (64
//      consecutive tiles, 64 super-tiles at a time, one per lane), then the
//      tiles of each super-tile within R, and evaluates every tile whose box
//      lies within R of its own box: the canonical FP32 d^2 of its pairs,
//      unless no lane's particle is close enough to the tile's box to gain
//      from it.  Every pair closer than R lies in such a tile pair, so D_i is
//      exact whenever D_i <= R^2 and exceeds R^2 otherwise;
//   4. after the selection of ell^2 (the k-th smallest D) the node's result is
//      exact iff ell^2 <= R^2; a node failing the check is redone all-pairs;
//   5. 6D FOF at ell^2 uses the same tiles, pruned at ell.
#include "primitives.hpp"
#include "refine_common.hpp"

namespace halo {
namespace refine {

namespace {

constexpr float kHalfRange = 4.0f;  // Morton quantisation range [-A, A] (unit 3D variance)
constexpr int kTile = 64;           // particles per tile = one wavefront

__global__ void k_grid_classify(LevelNodes nd, uint32_t K, NodeScratch sc, uint32_t gmin,
                                uint32_t* flag) {
  uint32_t k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= K) return;
  bool g = sc.prm[12 * (size_t)k + 11] != 0.0 && nd.count[k] > gmin;
  sc.gstate[k] = g ? 1u : 0u;
  flag[k] = g ? 1u : 0u;
}

__global__ void k_grid_list(const uint32_t* flag, const uint32_t* pos, uint32_t K,
                            LevelNodes nd, GridBufs g) {
  uint32_t k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= K) return;
  if (flag[k]) {
    const uint32_t b = pos[k];
    g.gnode[b] = k;
    g.nb_rank[k] = b;
    g.ncell[b] = (nd.count[k] + kTile - 1) / kTile;  // tiles of the node
  } else {
    g.nb_rank[k] = 0xFFFFFFFFu;
  }
}

// Exact nearest-neighbour d^2 of sample particle s of grid node b.
__global__ void __launch_bounds__(TB)
    k_sample_nn(const float* xi, size_t S, LevelNodes nd, GridBufs g, uint32_t NB) {
  __shared__ float red[TB];
  for (uint32_t blk = blockIdx.x; blk < NB * kSamples; blk += gridDim.x) {
    const uint32_t b = blk / kSamples, sm = blk % kSamples;
    const uint32_t k = g.gnode[b];
    const uint32_t first = nd.first[k], n = nd.count[k];
    const uint32_t li = (uint32_t)(((uint64_t)sm * n) / kSamples);
    const uint32_t gi = first + li;
    float a[6];
    for (int c = 0; c < 6; ++c) a[c] = xi[(size_t)c * S + gi];
    float best = __int_as_float(0x7F800000);
    for (uint32_t j = threadIdx.x; j < n; j += TB) {
      if (j == li) continue;
      const uint32_t gj = first + j;
      float d = d2_6(a[0], a[1], a[2], a[3], a[4], a[5], xi[gj], xi[S + gj], xi[2 * S + gj],
                     xi[3 * S + gj], xi[4 * S + gj], xi[5 * S + gj]);
      best = fminf(best, d);
    }
    red[threadIdx.x] = best;
    __syncthreads();
    for (int o = TB / 2; o > 0; o >>= 1) {
      if (threadIdx.x < o) red[threadIdx.x] = fminf(red[threadIdx.x], red[threadIdx.x + o]);
      __syncthreads();
    }
    if (threadIdx.x == 0) g.samp[(size_t)b * kSamples + sm] = red[0];
    __syncthreads();
  }
}

// Search radius of each grid node from its sample (one block per node).
__global__ void __launch_bounds__(TB) k_grid_params(GridBufs g, uint32_t NB, double f) {
  __shared__ float v[kSamples];
  __shared__ float pick;
  const uint32_t b = blockIdx.x;
  if (b >= NB) return;
  for (int e = threadIdx.x; e < kSamples; e += TB) v[e] = g.samp[(size_t)b * kSamples + e];
  __syncthreads();
  // rank margin of ~2 standard deviations of the sample quantile's rank
  int kq = (int)ceil((f + kSampleMargin) * (double)kSamples);
  kq = kq < 1 ? 1 : (kq > kSamples ? kSamples : kq);
  for (int e = threadIdx.x; e < kSamples; e += TB) {
    int rank = 0;
    const float x = v[e];
    for (int q = 0; q < kSamples; ++q) rank += (v[q] < x || (v[q] == x && q < e)) ? 1 : 0;
    if (rank == kq - 1) pick = x;
  }
  __syncthreads();
  if (threadIdx.x == 0) g.r2[b] = fmaxf(kRadiusFactor * pick, 1e-30f);
}

__global__ void k_grid_flags(const uint32_t* lnode, uint32_t M, GridBufs g, uint32_t* flag) {
  uint32_t m = blockIdx.x * blockDim.x + threadIdx.x;
  if (m < M) flag[m] = g.nb_rank[lnode[m]] != 0xFFFFFFFFu ? 1u : 0u;
}

__device__ __forceinline__ uint32_t quant8(float v) {
  float t = (v + kHalfRange) * (256.0f / (2.0f * kHalfRange));
  t = fminf(fmaxf(t, 0.0f), 255.0f);
  return (uint32_t)t;
}

// key = node rank (16 bits) | 6D Morton code (48 bits)
__global__ void k_grid_keys(const float* xi, size_t S, const uint32_t* lnode, uint32_t M,
                            const uint32_t* flag, const uint32_t* pos, GridBufs g) {
  uint32_t m = blockIdx.x * blockDim.x + threadIdx.x;
  if (m >= M || !flag[m]) return;
  const uint32_t b = g.nb_rank[lnode[m]];
  uint32_t qd[6];
  for (int c = 0; c < 6; ++c) qd[c] = quant8(xi[(size_t)c * S + m]);
  unsigned long long code = 0;
  for (int bit = 7; bit >= 0; --bit)
    for (int c = 0; c < 6; ++c) code = (code << 1) | ((qd[c] >> bit) & 1u);
  const uint32_t p = pos[m];
  g.k0[p] = ((unsigned long long)b << 48) | code;
  g.v0[p] = m;
}

__global__ void k_grid_gather(const uint32_t* val, const float* xi, size_t S, uint32_t MB,
                              GridBufs g) {
  uint32_t q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= MB) return;
  const uint32_t m = val[q];
  g.gm[q] = m;
  for (int c = 0; c < 6; ++c) g.gx[(size_t)c * MB + q] = xi[(size_t)c * S + m];
}

// Tiles: tile t of node b covers sorted positions [pstart_b + 64 t', ...).
// pstart_b = sum of the sizes of the grid nodes before b (sort order).
__global__ void k_tile_setup(LevelNodes nd, GridBufs g, uint32_t NB) {
  uint32_t b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= NB) return;
  const uint32_t nt = g.ncell[b], t0 = g.cellbase[b];
  const uint32_t n = nd.count[g.gnode[b]];
  for (uint32_t t = 0; t < nt; ++t) g.gtile_node[t0 + t] = b;
  g.gcount[b] = n;
}

// Bounding box of each tile, one wavefront per tile.
__global__ void k_tile_boxes(GridBufs g, uint32_t MB, uint32_t NT) {
  const uint32_t wave = (blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const int lane = threadIdx.x & 63;
  if (wave >= NT) return;
  const uint32_t b = g.gtile_node[wave];
  const uint32_t t = wave - g.cellbase[b];
  const uint32_t p0 = g.pstart[b] + t * kTile;
  const uint32_t p1 = min(g.pstart[b] + g.gcount[b], p0 + kTile);
  const bool ok = p0 + lane < p1;
  const uint32_t q = ok ? p0 + lane : p0;
  for (int c = 0; c < 6; ++c) {
    float v = g.gx[(size_t)c * MB + q];
    float mn = v, mx = v;
    for (int o = 32; o > 0; o >>= 1) {
      mn = fminf(mn, __shfl_xor(mn, o));
      mx = fmaxf(mx, __shfl_xor(mx, o));
    }
    if (lane == 0) {
      g.tbox[12 * (size_t)wave + c] = mn;
      g.tbox[12 * (size_t)wave + 6 + c] = mx;
    }
  }
}

// Box of each super-tile: the union of the boxes of tiles [64 g, 64 g + 64),
// one wavefront per super-tile.  A super-tile may hold tiles of two nodes; its
// box then bounds both, which only weakens the pruning.
__global__ void k_super_boxes(GridBufs g, uint32_t NT, uint32_t NS) {
  const uint32_t wave = (blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const uint32_t lane = threadIdx.x & 63u;
  if (wave >= NS) return;
  const uint32_t t = wave * 64u + lane;
  const bool ok = t < NT;
  const uint32_t tt = ok ? t : wave * 64u;
  for (int c = 0; c < 6; ++c) {
    float mn = g.tbox[12 * (size_t)tt + c], mx = g.tbox[12 * (size_t)tt + 6 + c];
    for (int o = 32; o > 0; o >>= 1) {
      mn = fminf(mn, __shfl_xor(mn, o));
      mx = fmaxf(mx, __shfl_xor(mx, o));
    }
    if (lane == 0) {
      g.sbox[12 * (size_t)wave + c] = mn;
      g.sbox[12 * (size_t)wave + 6 + c] = mx;
    }
  }
}

__device__ __forceinline__ float box_gap2(const float* a, const float* b) {
  float s = 0.0f;
#pragma unroll
  for (int c = 0; c < 6; ++c) {
    float gap = fmaxf(0.0f, fmaxf(b[c] - a[6 + c], a[c] - b[6 + c]));
    s = __fmaf_rn(gap, gap, s);
  }
  return s;
}

// Squared gap between a point and a tile's box, in the component order and
// FP32 operations of d2_6: each step is monotone and the per-axis gap is at
// most |b_c - a_c| for every b in the box, so the result never exceeds d2_6
// of the point and any particle of the tile.  The box is wave-uniform.
__device__ __forceinline__ float point_gap2(const float* a, const float* __restrict__ box) {
  float s = 0.0f;
#pragma unroll
  for (int c = 0; c < 6; ++c) {
    const float gap = fmaxf(0.0f, fmaxf(box[c] - a[c], a[c] - box[6 + c]));
    s = c == 0 ? gap * gap : __fmaf_rn(gap, gap, s);
  }
  return s;
}

// Block-sparse pass of one target tile per wavefront.  mode 0: nearest
// neighbour within the node; mode 1: 6D FOF unions at ell^2.
template <int MODE>
__global__ void __launch_bounds__(kTile)
    k_tile_pass(GridBufs g, uint32_t MB, uint32_t NT, NodeScratch sc, uint32_t* D,
                uint32_t* par) {
  __shared__ float t[6][kTile];
  __shared__ uint32_t troot[kTile];
  __shared__ float ibox[12];
  const int lane = threadIdx.x;
  for (uint32_t it = blockIdx.x; it < NT; it += gridDim.x) {
    const uint32_t b = g.gtile_node[it];
    const uint32_t k = g.gnode[b];
    const uint32_t tb0 = g.cellbase[b], tb1 = g.cellbase[b + 1];
    const uint32_t ps = g.pstart[b], pe = g.pstart[b] + g.gcount[b];
    const uint32_t p0 = ps + (it - tb0) * kTile;
    const uint32_t p1 = min(pe, p0 + kTile);
    const bool ok = p0 + lane < p1;
    const uint32_t qi = ok ? p0 + lane : p0;
    const float* X = g.gx;
    const float a0 = X[qi], a1 = X[MB + qi], a2 = X[2 * (size_t)MB + qi],
                a3 = X[3 * (size_t)MB + qi], a4 = X[4 * (size_t)MB + qi],
                a5 = X[5 * (size_t)MB + qi];
    const uint32_t mi = g.gm[qi];
    float radius2;
    bool active = ok;
    uint32_t ri = 0;
    if (MODE == 0) {
      radius2 = g.r2[b] * 1.00001f;
    } else {
      radius2 = sc.ell2[k] * 1.00001f;
      if (sc.gstate[k] != 1u) continue;  // uniform over the wave
      active = ok && __uint_as_float(D[mi]) <= sc.ell2[k];
      ri = active ? uf_find(par, mi) : 0xFFFFFFFFu;
    }
    const float l2 = MODE == 1 ? sc.ell2[k] : 0.0f;
    if (lane < 12) ibox[lane] = g.tbox[12 * (size_t)it + lane];
    __builtin_amdgcn_wave_barrier();
    __syncthreads();
    float best = __int_as_float(0x7F800000);
    const float av[6] = {a0, a1, a2, a3, a4, a5};
    if (MODE == 0) {
      // the own tile first: a close first minimum for the per-lane pruning
      const uint32_t q0 = p0, q1 = p1;
      best = nn_span<true>(X, MB, q0, q1, qi, av, best);
    }
    // j tiles through super-tiles of 64, 64 super-tiles at a time; the NN pass
    // starts at the super-tile holding the target (near it on the Morton
    // curve); FOF considers each unordered pair once, so its j tiles start at
    // the target
    const uint32_t jt0 = MODE == 1 ? it : tb0;
    const uint32_t s0 = jt0 >> 6, ns = ((tb1 - 1) >> 6) - s0 + 1;
    const uint32_t rot = MODE == 1 ? 0u : (it >> 6) - s0;
    for (uint32_t sb = 0; sb < ns; sb += kTile) {
      const uint32_t sl = sb + lane;
      bool scand = false;
      if (sl < ns) {
        const uint32_t sg = s0 + (sl + rot < ns ? sl + rot : sl + rot - ns);
        scand = box_gap2(ibox, g.sbox + 12 * (size_t)sg) <= radius2;
      }
      unsigned long long smask = __ballot(scand);
      while (smask) {
        const int sbit = __ffsll((long long)smask) - 1;
        smask &= smask - 1;
        const uint32_t sl2 = sb + sbit;
        const uint32_t sg = __builtin_amdgcn_readfirstlane(
            s0 + (sl2 + rot < ns ? sl2 + rot : sl2 + rot - ns));
        const uint32_t ta = max(sg * 64u, jt0), tz = min(sg * 64u + 64u, tb1);
        const uint32_t jt = ta + lane;
        bool cand = false;
        if (jt < tz && (MODE == 1 || jt != it))
          cand = box_gap2(ibox, g.tbox + 12 * (size_t)jt) <= radius2;
        unsigned long long mask = __ballot(cand);
        while (mask) {
          const int bit = __ffsll((long long)mask) - 1;
          mask &= mask - 1;
          const uint32_t jtile = __builtin_amdgcn_readfirstlane(ta + bit);
          // skip the tile unless some lane could gain from it
          const float gp = point_gap2(av, g.tbox + 12 * (size_t)jtile);
          if (MODE == 0 ? !__any(ok && gp < best) : !__any(active && gp <= l2)) continue;
          const uint32_t q0 = ps + (jtile - tb0) * kTile;
          const uint32_t q1 = min(pe, q0 + kTile);
          if (MODE == 1) {  // the FOF pass stages the tile and its roots
            __syncthreads();
            if (q0 + lane < q1) {
              const uint32_t qj = q0 + lane;
              for (int c = 0; c < 6; ++c) t[c][lane] = X[(size_t)c * MB + qj];
              const uint32_t mj = g.gm[qj];
              troot[lane] = __uint_as_float(D[mj]) <= l2 ? uf_find(par, mj) : 0xFFFFFFFEu;
            }
            __syncthreads();
            if (active) {
              // a j already in the lane's set (equal roots at some point; sets
              // only merge) needs no distance
              const uint32_t nj = q1 - q0;
              const uint32_t qstart = (jtile == it) ? (uint32_t)lane + 1 : 0u;
              for (uint32_t q = qstart; q < nj; ++q) {
                if (troot[q] == 0xFFFFFFFEu || troot[q] == ri) continue;
                const float d = d2_6(a0, a1, a2, a3, a4, a5, t[0][q], t[1][q], t[2][q],
                                     t[3][q], t[4][q], t[5][q]);
                if (d <= l2) {
                  uf_union(par, mi, g.gm[q0 + q]);
                  ri = uf_find(par, mi);
                }
              }
            }
          } else {
            best = nn_span<false>(X, MB, q0, q1, 0u, av, best);
          }
        }
      }
    }
    if (MODE == 0 && ok) D[mi] = __float_as_uint(best);
    __syncthreads();
  }
}

__global__ void k_grid_check(GridBufs g, uint32_t NB, NodeScratch sc, uint32_t* nfail) {
  uint32_t b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= NB) return;
  const uint32_t k = g.gnode[b];
  if (!(sc.ell2[k] <= g.r2[b])) {
    sc.gstate[k] = 2u;
    atomicAdd(nfail, 1u);
  }
}

__global__ void k_grid_reset_failed(const uint32_t* lnode, uint32_t M, NodeScratch sc,
                                    uint32_t* D) {
  uint32_t m = blockIdx.x * blockDim.x + threadIdx.x;
  if (m < M && sc.gstate[lnode[m]] == 2u) D[m] = 0x7F800000u;
}

__global__ void k_pstart(GridBufs g, uint32_t NB) {
  // exclusive prefix of the grid nodes' sizes, in rank order (sort order)
  if (blockIdx.x != 0 || threadIdx.x != 0) return;
  uint32_t acc = 0;
  for (uint32_t b = 0; b < NB; ++b) {
    g.pstart[b] = acc;
    acc += g.gcount[b];
  }
  g.pstart[NB] = acc;
}

__global__ void k_gcount(LevelNodes nd, GridBufs g, uint32_t NB) {
  uint32_t b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b < NB) g.gcount[b] = nd.count[g.gnode[b]];
}

}  // namespace

void grid_take(Arena& A, GridBufs& g, uint32_t M, uint32_t Kmax) {
  const uint32_t NBmax = M / kGridFloor + 2;
  const uint32_t NTmax = M / kTile + NBmax + 2;
  g.nb_rank = A.take<uint32_t>(Kmax + 2);
  g.gnode = A.take<uint32_t>(NBmax);
  g.samp = A.take<float>((size_t)NBmax * kSamples);
  g.r2 = A.take<float>(NBmax);
  g.ncell = A.take<uint32_t>(NBmax + 1);
  g.cellbase = A.take<uint32_t>(NBmax + 1);
  g.pstart = A.take<uint32_t>(NBmax + 1);
  g.gcount = A.take<uint32_t>(NBmax + 1);
  g.gtile_node = A.take<uint32_t>(NTmax);
  g.tbox = A.take<float>(12ull * NTmax);
  g.sbox = A.take<float>(12ull * (NTmax / 64 + 2));
  g.flag = A.take<uint32_t>((size_t)M + 2);
  g.pos = A.take<uint32_t>((size_t)M + 2);
  g.k0 = A.take<unsigned long long>((size_t)M + 2);
  g.k1 = A.take<unsigned long long>((size_t)M + 2);
  g.v0 = A.take<uint32_t>((size_t)M + 2);
  g.v1 = A.take<uint32_t>((size_t)M + 2);
  g.gm = A.take<uint32_t>((size_t)M + 2);
  g.gx = A.take<float>(6ull * (M + 2));
  g.cnt = A.take<uint32_t>(16);
  g.rtmp = A.take<char>(radix_tmp_bytes((int64_t)M + 2));
  g.stmp = A.take<uint32_t>(scan_tmp_elems<uint32_t>((int64_t)M + Kmax + 4));
}

uint32_t grid_build(GridBufs& g, const float* xi, size_t S, LevelNodes nd, uint32_t K,
                    const uint32_t* lnode, uint32_t Mi, uint32_t M, NodeScratch sc, double f,
                    uint32_t* hb, hipStream_t s, uint32_t* D, uint32_t gmin) {
  g.NB = 0;
  g.MB = 0;
  g.NT = 0;
  if (Mi <= gmin) {  // no node of the level can exceed the threshold: no read-back needed
    k_fill_u32<<<blocks_for(K, TB), TB, 0, s>>>(sc.gstate, K, 0u);
    return 0;
  }
  k_grid_classify<<<blocks_for(K, TB), TB, 0, s>>>(nd, K, sc, gmin, g.flag);
  exclusive_scan<uint32_t>(g.flag, g.pos, K, g.cnt, g.stmp, s);
  k_grid_list<<<blocks_for(K, TB), TB, 0, s>>>(g.flag, g.pos, K, nd, g);
  HALO_HIP(hipMemcpyAsync(hb, g.cnt, 4, hipMemcpyDeviceToHost, s));
  HALO_HIP(hipStreamSynchronize(s));
  const uint32_t NB = hb[0];
  if (NB == 0) return 0;
  HALO_CHECK(NB < 65536, LIBHALO_EINVAL, "too many grid nodes in one level");
  k_sample_nn<<<(unsigned)std::min<uint64_t>((uint64_t)NB * kSamples, 65535), TB, 0, s>>>(
      xi, S, nd, g, NB);
  k_grid_params<<<NB, TB, 0, s>>>(g, NB, f);
  exclusive_scan<uint32_t>(g.ncell, g.cellbase, NB, g.cellbase + NB, g.stmp, s);
  k_gcount<<<blocks_for(NB, TB), TB, 0, s>>>(nd, g, NB);
  k_pstart<<<1, 1, 0, s>>>(g, NB);
  k_grid_flags<<<blocks_for(Mi, TB), TB, 0, s>>>(lnode, Mi, g, g.flag);
  exclusive_scan<uint32_t>(g.flag, g.pos, Mi, g.cnt + 1, g.stmp, s);
  k_grid_keys<<<blocks_for(Mi, TB), TB, 0, s>>>(xi, S, lnode, Mi, g.flag, g.pos, g);
  HALO_HIP(hipMemcpyAsync(hb + 1, g.cnt + 1, 4, hipMemcpyDeviceToHost, s));
  HALO_HIP(hipMemcpyAsync(hb + 2, g.cellbase + NB, 4, hipMemcpyDeviceToHost, s));
  HALO_HIP(hipStreamSynchronize(s));
  const uint32_t MB = hb[1], NT = hb[2];
  g.MB = MB;
  g.NB = NB;
  g.NT = NT;
  bool fl = radix_sort_pairs<unsigned long long>(g.k0, g.v0, g.k1, g.v1, MB,
                                                 48 + bits_for(NB > 1 ? NB - 1 : 1), g.rtmp, s);
  uint32_t* sv = fl ? g.v1 : g.v0;
  k_grid_gather<<<blocks_for(MB, TB), TB, 0, s>>>(sv, xi, S, MB, g);
  k_tile_setup<<<blocks_for(NB, TB), TB, 0, s>>>(nd, g, NB);
  k_tile_boxes<<<blocks_for((int64_t)NT * 64, TB), TB, 0, s>>>(g, MB, NT);
  const uint32_t NS = (NT + 63) / 64;
  k_super_boxes<<<blocks_for((int64_t)NS * 64, TB), TB, 0, s>>>(g, NT, NS);
  k_tile_pass<0><<<std::min<uint32_t>(NT, 16384), kTile, 0, s>>>(g, MB, NT, sc, D, nullptr);
  return NB;
}

uint32_t grid_check(GridBufs& g, NodeScratch sc, const uint32_t* lnode, uint32_t Mi,
                    uint32_t* D, uint32_t* hb, hipStream_t s) {
  if (g.NB == 0) return 0;
  k_fill_u32<<<1, 64, 0, s>>>(g.cnt + 2, 1, 0u);
  k_grid_check<<<blocks_for(g.NB, TB), TB, 0, s>>>(g, g.NB, sc, g.cnt + 2);
  HALO_HIP(hipMemcpyAsync(hb + 3, g.cnt + 2, 4, hipMemcpyDeviceToHost, s));
  HALO_HIP(hipStreamSynchronize(s));
  if (hb[3] > 0) k_grid_reset_failed<<<blocks_for(Mi, TB), TB, 0, s>>>(lnode, Mi, sc, D);
  return hb[3];
}

void grid_fof(GridBufs& g, NodeScratch sc, const uint32_t* D, uint32_t* par, hipStream_t s) {
  if (g.NB == 0 || g.MB == 0) return;
  k_tile_pass<1><<<std::min<uint32_t>(g.NT, 16384), kTile, 0, s>>>(g, g.MB, g.NT, sc,
                                                                   const_cast<uint32_t*>(D), par);
}

}  // namespace refine
}  // namespace halo
