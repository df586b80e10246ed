// Exact nearest-neighbour distances and 6D FOF for large hierarchy nodes
// (Section 3.2) by per-particle searches of a binary space partition.
//
// For every node above the tree threshold of a level:
//   1. its particles are sorted along a 6D Morton curve (8 bits per
//      normalised coordinate over [-A, A], clamped), keyed by node first;
//   2. a binary tree is built top down over the sorted order: a node whose
//      range holds more than kKdLeaf particles splits where the highest Morton
//      bit that differs across its range changes (at the middle of the range
//      when every key is equal), so each child covers one cell of the curve;
//      its box is the exact bounding box of its particles.  The split is the
//      one of a radix tree over Morton codes (Karras 2012, "Maximizing
//      parallelism in the construction of BVHs, octrees, and k-d trees"),
//      built here level by level;
//   3. one thread per particle walks its node's tree depth first, nearer child
//      first, and skips a subtree whose box lies no closer than the best
//      distance found so far (nearest-neighbour pass), or farther than ell
//      (FOF pass, which also skips subtrees holding no particle after the
//      walker in the sorted order, so each pair is met once).
// The box test computes the point-to-box gap in the component order and FP32
// operations of the distance, so it never exceeds the distance to any particle
// in the box: no particle that could change the result is skipped.  D is
// exact for every particle and the FOF links every pair within ell^2, so the
// results equal those of the all-pairs passes bit for bit.
#include "primitives.hpp"
#include "refine_common.hpp"

namespace halo {
namespace refine {

namespace {

constexpr float kHalfRange = 4.0f;      // Morton quantisation range [-A, A]
constexpr int kStack = kKdMaxDepth + 1; // one pushed subtree per depth at most
constexpr int kWalkTB = 64;             // one wavefront per block: LDS stack per lane

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
    g.gcount[b] = nd.count[k];
  } else {
    g.nb_rank[k] = 0xFFFFFFFFu;
  }
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

// key = tree-node rank (16 bits) | 6D Morton code (48 bits)
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

__global__ void k_pstart(GridBufs g, uint32_t NB) {
  // exclusive prefix of the tree nodes' sizes, in rank order (sort order)
  if (blockIdx.x != 0 || threadIdx.x != 0) return;
  uint32_t acc = 0;
  for (uint32_t b = 0; b < NB; ++b) {
    g.pstart[b] = acc;
    acc += g.gcount[b];
  }
  g.pstart[NB] = acc;
}

// Sorted points (AoS, 32 bytes) from the level's coordinate planes.
__global__ void k_kd_gather(const uint32_t* val, const float* xi, size_t S, uint32_t MB,
                            const uint32_t* lnode, GridBufs g) {
  uint32_t q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= MB) return;
  const uint32_t m = val[q];
  KdPoint p;
  for (int c = 0; c < 6; ++c) p.x[c] = xi[(size_t)c * S + m];
  p.m = m;
  p.b = g.nb_rank[lnode[m]];
  g.pt[q] = p;
}

__global__ void k_kd_roots(GridBufs g, uint32_t NB) {
  uint32_t b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= NB) return;
  KdNode r;
  r.lo = g.pstart[b];
  r.hi = g.pstart[b] + g.gcount[b];
  r.left = kKdNone;
  r.depth = 0;
  g.node[b] = r;
}

// Split point of each frontier node that holds more than a leaf: where the
// highest differing Morton bit of its sorted keys changes.
__global__ void k_kd_split(GridBufs g, const unsigned long long* __restrict__ key, uint32_t f0,
                           uint32_t nf, uint32_t* flag, uint32_t* split) {
  uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nf) return;
  const KdNode& u = g.node[f0 + i];
  const uint32_t lo = u.lo, hi = u.hi;
  if (hi - lo <= kKdLeaf || u.depth >= (uint32_t)kKdMaxDepth) {
    flag[i] = 0u;
    return;
  }
  const unsigned long long kx = key[lo] ^ key[hi - 1];
  uint32_t sp;
  if (kx == 0ull) {
    sp = lo + (hi - lo) / 2;
  } else {
    const int bit = 63 - __clzll((long long)kx);
    uint32_t a = lo + 1, z = hi - 1;  // first index whose key has the bit set
    while (a < z) {
      const uint32_t mid = a + (z - a) / 2;
      if ((key[mid] >> bit) & 1ull)
        z = mid;
      else
        a = mid + 1;
    }
    sp = a;
  }
  flag[i] = 1u;
  split[i] = sp;
}

// Children of the split frontier nodes, appended in frontier order after f1;
// a split whose children would pass the node capacity is not made (the node
// stays a leaf and is searched in full).
__global__ void k_kd_children(GridBufs g, uint32_t f0, uint32_t nf, uint32_t f1,
                              const uint32_t* flag, const uint32_t* pos, const uint32_t* split) {
  uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nf || !flag[i]) return;
  const uint32_t c = f1 + 2u * pos[i];
  if (c + 2u > g.node_cap) return;
  KdNode& u = g.node[f0 + i];
  KdNode a, b;
  a.lo = u.lo;
  a.hi = split[i];
  b.lo = split[i];
  b.hi = u.hi;
  a.left = b.left = kKdNone;
  a.depth = b.depth = u.depth + 1;
  g.node[c] = a;
  g.node[c + 1] = b;
  u.left = c;
}

// Boxes of the nodes [u0, u0 + nu) of one depth: leaves from their particles,
// internal nodes from their children (one depth deeper, already done).
__global__ void k_kd_boxes(GridBufs g, uint32_t u0, uint32_t nu) {
  uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nu) return;
  KdNode& u = g.node[u0 + i];
  float mn[6], mx[6];
  for (int c = 0; c < 6; ++c) {
    mn[c] = __int_as_float(0x7F800000);
    mx[c] = -__int_as_float(0x7F800000);
  }
  if (u.left == kKdNone) {
    for (uint32_t q = u.lo; q < u.hi; ++q) {
      const KdPoint p = g.pt[q];
      for (int c = 0; c < 6; ++c) {
        mn[c] = fminf(mn[c], p.x[c]);
        mx[c] = fmaxf(mx[c], p.x[c]);
      }
    }
  } else {
    const KdNode& a = g.node[u.left];
    const KdNode& b = g.node[u.left + 1];
    for (int c = 0; c < 6; ++c) {
      mn[c] = fminf(a.mn[c], b.mn[c]);
      mx[c] = fmaxf(a.mx[c], b.mx[c]);
    }
  }
  for (int c = 0; c < 6; ++c) {
    u.mn[c] = mn[c];
    u.mx[c] = mx[c];
  }
}

// Squared gap between a point and a box, in the component order and FP32
// operations of d2_6: each step is monotone and the per-axis gap is at most
// |b_c - a_c| for every b in the box, so the result never exceeds d2_6 of the
// point and any particle inside.
__device__ __forceinline__ float point_gap2(const float* a, const float4* r) {
  // r[0..2]: mn[0..5], mx[0..5]
  const float mn[6] = {r[0].x, r[0].y, r[0].z, r[0].w, r[1].x, r[1].y};
  const float mx[6] = {r[1].z, r[1].w, r[2].x, r[2].y, r[2].z, r[2].w};
  float s = 0.0f;
#pragma unroll
  for (int c = 0; c < 6; ++c) {
    const float gap = fmaxf(0.0f, fmaxf(mn[c] - a[c], a[c] - mx[c]));
    s = c == 0 ? gap * gap : __fmaf_rn(gap, gap, s);
  }
  return s;
}

// A stacked subtree keeps a lower bound of its gap: the top 16 bits of the
// FP32 pattern (truncation rounds a non-negative float down).
__device__ __forceinline__ uint16_t gap_lb16(float g) { return (uint16_t)(__float_as_uint(g) >> 16); }
__device__ __forceinline__ float gap_from16(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

// Block -> share of the points: the blocks that run on one XCD (blockIdx mod
// 8) take one contiguous run of waves, so walks of neighbouring particles
// share that XCD's L2.
__device__ __forceinline__ uint32_t xcd_wave(uint32_t bid, uint32_t G) {
  const uint32_t x = bid & 7u;
  uint32_t start = 0;
  for (uint32_t y = 0; y < x; ++y) start += (G - y + 7u) >> 3;
  return start + (bid >> 3);
}

// One thread per sorted point.  MODE 0: nearest-neighbour distance within its
// tree node (D[m] = min over j != i of d2_6).  MODE 1: 6D FOF at the node's
// ell^2 for points with D <= ell^2, over the points after it in the order.
template <int MODE>
__global__ void __launch_bounds__(kWalkTB)
    k_kd_walk(const KdNode* __restrict__ T, const KdPoint* __restrict__ pt, uint32_t MB,
              const uint32_t* __restrict__ gnode, NodeScratch sc, uint32_t* D, uint32_t* par) {
  __shared__ uint32_t stn[kStack][kWalkTB];
  __shared__ uint16_t stg[kStack][kWalkTB];
  const int lane = threadIdx.x;
  const uint32_t q = xcd_wave(blockIdx.x, gridDim.x) * kWalkTB + lane;
  const bool valid = q < MB;
  const KdPoint P = pt[valid ? q : MB - 1];
  const float a[6] = {P.x[0], P.x[1], P.x[2], P.x[3], P.x[4], P.x[5]};
  bool done = !valid;
  float best = __int_as_float(0x7F800000);  // MODE 0: nearest so far
  float l2 = 0.0f;                          // MODE 1: ell^2 of the node
  uint32_t ri = 0;
  if (MODE == 1 && !done) {
    l2 = sc.ell2[gnode[P.b]];
    if (!(__uint_as_float(D[P.m]) <= l2))
      done = true;
    else
      ri = uf_find(par, P.m);
  }
  // current node: the root of the point's tree
  uint32_t lo = 0, hi = 0, left = kKdNone;
  {
    const uint4 h = reinterpret_cast<const uint4*>(T + P.b)[3];
    lo = h.x;
    hi = h.y;
    left = h.z;
  }
  int sp = 0;
  bool leaf = false;
  // pop the next stacked subtree still worth a visit; false when none is left
  auto pop = [&]() -> bool {
    while (sp > 0) {
      --sp;
      const uint32_t u = stn[sp][lane];
      if (MODE == 1 || gap_from16(stg[sp][lane]) < best) {
        const uint4 h = reinterpret_cast<const uint4*>(T + u)[3];
        lo = h.x;
        hi = h.y;
        left = h.z;
        return true;
      }
    }
    return false;
  };
  while (__any(!done)) {
    // descend until every walking lane stands at a leaf
    while (__any(!done && !leaf)) {
      if (!done && !leaf) {
        if (left == kKdNone) {
          leaf = true;
        } else {
          const float4* r0 = reinterpret_cast<const float4*>(T + left);
          const float4 c0[4] = {r0[0], r0[1], r0[2], r0[3]};
          const float4 c1[4] = {r0[4], r0[5], r0[6], r0[7]};
          const float g0 = point_gap2(a, c0), g1 = point_gap2(a, c1);
          bool ok0, ok1;
          if (MODE == 0) {
            ok0 = g0 < best;
            ok1 = g1 < best;
          } else {
            ok0 = g0 <= l2 && __float_as_uint(c0[3].y) > q + 1u;  // hi of child 0
            ok1 = g1 <= l2 && __float_as_uint(c1[3].y) > q + 1u;
          }
          const bool near0 = g0 <= g1;
          if (ok0 || ok1) {
            const bool go0 = ok0 && (near0 || !ok1);
            if (ok0 && ok1) {  // stack the farther child
              stn[sp][lane] = near0 ? left + 1u : left;
              stg[sp][lane] = gap_lb16(near0 ? g1 : g0);
              ++sp;
            }
            const float4 h = go0 ? c0[3] : c1[3];
            lo = __float_as_uint(h.x);
            hi = __float_as_uint(h.y);
            left = __float_as_uint(h.z);
          } else if (!pop()) {
            done = true;
          }
        }
      }
    }
    if (!done && leaf) {
      if (MODE == 0) {
        for (uint32_t j = lo; j < hi; ++j) {
          const float4* pj = reinterpret_cast<const float4*>(pt + j);
          const float4 u = pj[0], v = pj[1];
          const float d = d2_6(a[0], a[1], a[2], a[3], a[4], a[5], u.x, u.y, u.z, u.w, v.x, v.y);
          best = j != q ? fminf(best, d) : best;
        }
      } else {
        for (uint32_t j = max(lo, q + 1u); j < hi; ++j) {
          const float4* pj = reinterpret_cast<const float4*>(pt + j);
          const float4 u = pj[0], v = pj[1];
          const float d = d2_6(a[0], a[1], a[2], a[3], a[4], a[5], u.x, u.y, u.z, u.w, v.x, v.y);
          if (d <= l2) {
            const uint32_t rj = uf_find(par, __float_as_uint(v.z));
            if (rj != ri) ri = uf_union(par, ri, rj);
          }
        }
      }
      leaf = false;
      if (!pop()) done = true;
    }
  }
  if (MODE == 0 && valid) D[P.m] = __float_as_uint(best);
}

unsigned walk_grid(uint32_t MB) { return (MB + kWalkTB - 1) / kWalkTB; }

}  // namespace

void grid_take(Arena& A, GridBufs& g, uint32_t M, uint32_t Kmax) {
  const uint32_t NBmax = M / kGridFloor + 2;
  g.nb_rank = A.take<uint32_t>(Kmax + 2);
  g.gnode = A.take<uint32_t>(NBmax);
  g.pstart = A.take<uint32_t>(NBmax + 1);
  g.gcount = A.take<uint32_t>(NBmax + 1);
  // tree nodes: the capacity bounds memory, not results (a node that finds no
  // room for its children stays a leaf); trees of 16-particle leaves use about
  // 0.2 nodes per particle
  g.node_cap = M / 2 + NBmax + 64;
  g.node = A.take<KdNode>(g.node_cap);
  g.split = A.take<uint32_t>(g.node_cap);
  g.flag = A.take<uint32_t>(std::max<size_t>((size_t)M + 2, g.node_cap));
  g.pos = A.take<uint32_t>(std::max<size_t>((size_t)M + 2, g.node_cap));
  g.k0 = A.take<unsigned long long>((size_t)M + 2);
  g.k1 = A.take<unsigned long long>((size_t)M + 2);
  g.v0 = A.take<uint32_t>((size_t)M + 2);
  g.v1 = A.take<uint32_t>((size_t)M + 2);
  g.pt = A.take<KdPoint>((size_t)M + 2);
  g.cnt = A.take<uint32_t>(16);
  g.rtmp = A.take<char>(radix_tmp_bytes((int64_t)M + 2));
  g.stmp = A.take<uint32_t>(
      scan_tmp_elems<uint32_t>(std::max<int64_t>((int64_t)M + Kmax + 4, g.node_cap)));
}

uint32_t grid_build(GridBufs& g, const float* xi, size_t S, LevelNodes nd, uint32_t K,
                    const uint32_t* lnode, uint32_t Mi, uint32_t M, NodeScratch sc,
                    uint32_t* hb, hipStream_t s, uint32_t* D, uint32_t gmin) {
  g.NB = 0;
  g.MB = 0;
  g.NN = 0;
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
  HALO_CHECK(NB < 65536, LIBHALO_EINVAL, "too many tree nodes in one level");
  k_pstart<<<1, 1, 0, s>>>(g, NB);
  k_grid_flags<<<blocks_for(Mi, TB), TB, 0, s>>>(lnode, Mi, g, g.flag);
  exclusive_scan<uint32_t>(g.flag, g.pos, Mi, g.cnt + 1, g.stmp, s);
  k_grid_keys<<<blocks_for(Mi, TB), TB, 0, s>>>(xi, S, lnode, Mi, g.flag, g.pos, g);
  HALO_HIP(hipMemcpyAsync(hb + 1, g.cnt + 1, 4, hipMemcpyDeviceToHost, s));
  HALO_HIP(hipStreamSynchronize(s));
  const uint32_t MB = hb[1];
  g.MB = MB;
  g.NB = NB;
  const bool fl = radix_sort_pairs<unsigned long long>(
      g.k0, g.v0, g.k1, g.v1, MB, 48 + bits_for(NB > 1 ? NB - 1 : 1), g.rtmp, s);
  const unsigned long long* key = fl ? g.k1 : g.k0;
  k_kd_gather<<<blocks_for(MB, TB), TB, 0, s>>>(fl ? g.v1 : g.v0, xi, S, MB, lnode, g);
  // top-down build, one depth per step; lev[d] = first node of depth d
  std::vector<uint32_t> lev{0u, NB};
  k_kd_roots<<<blocks_for(NB, TB), TB, 0, s>>>(g, NB);
  for (int d = 0; d < kKdMaxDepth; ++d) {
    const uint32_t f0 = lev[d], f1 = lev[d + 1], nf = f1 - f0;
    if (nf == 0) break;
    k_kd_split<<<blocks_for(nf, TB), TB, 0, s>>>(g, key, f0, nf, g.flag, g.split);
    exclusive_scan<uint32_t>(g.flag, g.pos, nf, g.cnt + 2, g.stmp, s);
    k_kd_children<<<blocks_for(nf, TB), TB, 0, s>>>(g, f0, nf, f1, g.flag, g.pos, g.split);
    HALO_HIP(hipMemcpyAsync(hb + 2, g.cnt + 2, 4, hipMemcpyDeviceToHost, s));
    HALO_HIP(hipStreamSynchronize(s));
    const uint32_t room = (g.node_cap - f1) / 2u;
    lev.push_back(f1 + 2u * std::min(hb[2], room));
  }
  g.NN = lev.back();
  for (int d = (int)lev.size() - 2; d >= 0; --d) {
    const uint32_t nu = lev[d + 1] - lev[d];
    if (nu) k_kd_boxes<<<blocks_for(nu, TB), TB, 0, s>>>(g, lev[d], nu);
  }
  k_kd_walk<0><<<walk_grid(MB), kWalkTB, 0, s>>>(g.node, g.pt, MB, g.gnode, sc, D, nullptr);
  return NB;
}

void grid_fof(GridBufs& g, NodeScratch sc, const uint32_t* D, uint32_t* par, hipStream_t s) {
  if (g.NB == 0 || g.MB == 0) return;
  k_kd_walk<1><<<walk_grid(g.MB), kWalkTB, 0, s>>>(g.node, g.pt, g.MB, g.gnode, sc,
                                                   const_cast<uint32_t*>(D), par);
}

}  // namespace refine
}  // namespace halo
