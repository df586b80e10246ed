// Exact nearest-neighbour distances and 6D FOF for large hierarchy nodes
// (Section 3.2) by per-particle searches of a binary space partition.
//
// For every node above the tree threshold of a level:
//   1. its particles are sorted along a 6D Morton curve (8 bits per
//      normalised coordinate over [-A, A], clamped), keyed by node first;
//   2. a binary tree is built top down over the sorted order: a node whose
//      range holds more than kd_leaf particles (16 by default) splits where the highest Morton
//      bit that differs across its range changes (at the middle of the range
//      when every key is equal), so each child covers one cell of the curve;
//      its box is the exact bounding box of its particles.  The split is the
//      one of a radix tree over Morton codes (Karras 2012, "Maximizing
//      parallelism in the construction of BVHs, octrees, and k-d trees"),
//      built here level by level;
//   3. the nodes are stored in depth-first preorder, left child first, each
//      with the record that follows its subtree, so a walk needs no stack:
//      one thread per particle tests records in order and enters a node whose
//      box is close enough (next record) or skips it.  The nearest-neighbour
//      pass searches the particle's own leaf first and then skips every box no
//      closer than the best distance so far; the FOF pass first links the
//      pairs inside each group (the largest subtree of at most 64 points
//      around a leaf), then each particle walks from the record after its
//      group (the preorder meets index ranges in increasing order, so each
//      pair is met once, from its first particle), entering boxes within ell
//      except a node of at most 64 points whose points all share the
//      particle's union-find root already (sets only merge, so such a node
//      holds no new link).
// The box test computes the point-to-box gap in the component order and FP32
// operations of the distance, so it never exceeds the distance to any particle
// in the box: no particle that could change the result is skipped.  D is
// exact for every particle (or, when the walks are given a bracket of ell^2,
// exact inside it and on the right side of it elsewhere, which fixes ell^2 and
// every linkable flag; refine6d.hip) and the FOF links every pair within
// ell^2, so the results equal those of the all-pairs passes bit for bit.
#include <hip/hip_fp16.h>

#include "primitives.hpp"
#include "refine_common.hpp"

namespace halo {
namespace refine {

namespace {

constexpr float kHalfRange = 4.0f;      // Morton quantisation range [-A, A]
constexpr int kWalkTB = 256;            // threads per block of the walks
constexpr uint32_t kWalkChunk = 64;     // points a wave takes from the queue at a time
// leaf points a walk evaluates per step: nearest neighbours 4, FOF 2 (at
// 1024^3 with 1, 2, 4 and 8 points per step: NN - / 0.82 / 0.81 / 0.92 s,
// FOF 1.46 / 1.43 / 1.49 / 1.73 s per step)
template <int MODE>
constexpr uint32_t kLeafStep = MODE == 0 ? 4u : 2u;
constexpr uint32_t kNoRoot = 0xFFFFFFFFu;  // a node whose points are in several sets

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

// Sorted points (six coordinates, 24 bytes) from the level's coordinate planes.
__global__ void k_kd_gather(const uint32_t* val, const float* xi, size_t S, uint32_t MB,
                            const uint32_t* lnode, GridBufs g) {
  uint32_t q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= MB) return;
  const uint32_t m = val[q];
  for (int c = 0; c < 6; ++c) g.pt[6ull * q + c] = xi[(size_t)c * S + m];
  g.pm[q] = m;
  g.pb[q] = g.nb_rank[lnode[m]];
}

__device__ __forceinline__ uint16_t h_down(float v) {
  return __half_as_ushort(__float2half_rd(v));
}
__device__ __forceinline__ uint16_t h_up(float v) { return __half_as_ushort(__float2half_ru(v)); }
__device__ __forceinline__ float h_f(uint16_t b) { return __half2float(__ushort_as_half(b)); }

// Preorder records of the nodes [u0, u0 + nu) of one depth: a leaf's box from
// its particles (which also learn their leaf), an internal node's from its
// children's records (one depth deeper, already written; the union of
// half-precision bounds is exact).
__global__ void k_kd_records(GridBufs g, const MtNode* bnode, const uint32_t* pre, uint32_t u0,
                             uint32_t nu) {
  uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nu) return;
  const MtNode u = bnode[u0 + i];
  const uint32_t p = pre[u0 + i];
  KdNode r;
  if (u.left == kMtNone) {
    float mn[6], mx[6];
    for (int c = 0; c < 6; ++c) {
      mn[c] = __int_as_float(0x7F800000);
      mx[c] = -__int_as_float(0x7F800000);
    }
    for (uint32_t q = u.lo; q < u.hi; ++q) {
      for (int c = 0; c < 6; ++c) {
        const float v = g.pt[6ull * q + c];
        mn[c] = fminf(mn[c], v);
        mx[c] = fmaxf(mx[c], v);
      }
      g.leafof[q] = p;
    }
    for (int c = 0; c < 6; ++c) {
      r.mn[c] = h_down(mn[c]);
      r.mx[c] = h_up(mx[c]);
    }
  } else {
    const uint32_t pl = pre[u.left], pr = pre[u.left + 1];
    const KdNode& a = g.node[pl];
    const KdNode& b = g.node[pr];
    for (int c = 0; c < 6; ++c) {
      r.mn[c] = h_down(fminf(h_f(a.mn[c]), h_f(b.mn[c])));
      r.mx[c] = h_up(fmaxf(h_f(a.mx[c]), h_f(b.mx[c])));
    }
    // each child's parent, its sibling and the record after the sibling's subtree
    g.up[pl] = make_uint4(p, pr, p + u.aux, 0u);
    g.up[pr] = make_uint4(p, pl, pr, 0u);
  }
  r.lo = u.lo;
  r.skip = p + u.aux;
  g.node[p] = r;
}

// The record after the last tree: its `lo` ends the last leaf's range.
__global__ void k_kd_sentinel(KdNode* node, uint32_t NN, uint32_t MB) {
  KdNode r;
  for (int c = 0; c < 6; ++c) r.mn[c] = r.mx[c] = 0;
  r.lo = MB;
  r.skip = NN + 1u;
  node[NN] = r;
}

// Squared gap between a point and a box, in the component order and FP32
// operations of d2_6: each step is monotone and the per-axis gap is at most
// |b_c - a_c| for every b in the box, so the result never exceeds d2_6 of the
// point and any particle inside.
__device__ __forceinline__ float point_gap2(const float* a, const KdNode& r) {
  float s = 0.0f;
#pragma unroll
  for (int c = 0; c < 6; ++c) {
    const float gap = fmaxf(0.0f, fmaxf(h_f(r.mn[c]) - a[c], a[c] - h_f(r.mx[c])));
    s = c == 0 ? gap * gap : __fmaf_rn(gap, gap, s);
  }
  return s;
}

// One lane per query point q, walking its tree's preorder records: a node
// whose box is close enough is entered (next record), else skipped (its
// `skip`).  MODE 0: nearest-neighbour distance within the point's tree node
// (D[m] = min over j != q of d2_6), starting from its own leaf's particles,
// then, from the own leaf upwards, the sibling subtree of each ancestor in
// turn, every leaf no farther than the best so far: the nearest subtrees come
// first, so the best distance shrinks early and prunes the far ones (a CPU
// count on a 3e5-point NFW halo: 12% fewer box tests, 15% fewer distances
// than one walk from the root).  MODE 1: 6D FOF at
// the node's ell^2 for points with D <= ell^2, over the points after q's
// first-pass group in the order: the records after that group's subtree (the
// preorder visits index ranges in increasing order), skipping a node whose
// points all share q's root (a CPU count on the same halo: 40% fewer
// distances and 12% fewer box tests, with a 64k-point window of walks in
// flight whose links the others do not see yet).  Each lane advances its
// own walk by one step per iteration, a record test or up to kLeafStep leaf
// points: the walks diverge at every record, and lanes that waited for the
// others to reach a leaf left four in five lanes of the issued instructions
// idle.
//
// The walks differ in length by several times within a wave, so the grid is
// persistent and a lane whose walk ends takes the next query at once: each
// wave takes chunks of kWalkChunk consecutive points (neighbours on the Morton
// curve) from a queue counter and hands them out in order to its idle lanes.
// The points are split into eight contiguous ranges with a queue each, one
// per XCD (blocks are dispatched to the XCDs round robin, so block b runs on
// XCD b mod 8): an XCD's waves walk neighbouring points, whose tree records
// and leaves its L2 then holds.  A wave whose range is drained takes chunks
// from the next ranges in turn.  The kernel ends when all eight are drained
// and every lane is idle; every walk ends because u only grows and is
// bounded by its tree's end.
template <int MODE, bool COUNT>
__global__ void __launch_bounds__(kWalkTB)
    k_kd_walk(const KdNode* __restrict__ T, const float* __restrict__ pt,
              const uint32_t* __restrict__ pm, const uint32_t* __restrict__ pb,
              const uint32_t* __restrict__ leafof, const uint32_t* __restrict__ troot,
              uint32_t MB, const uint32_t* __restrict__ gnode, NodeScratch sc, uint32_t* D,
              uint32_t* par, uint32_t* queue, const uint4* __restrict__ UP,
              const uint32_t* __restrict__ GS, const uint32_t* __restrict__ UR,
              uint32_t MQ, uint32_t stride, const float* __restrict__ TL,
              const float* __restrict__ TH, const uint32_t* __restrict__ ONLY,
              unsigned long long* work) {
  const uint32_t lane = threadIdx.x & 63u;
  const unsigned long long below = (1ull << lane) - 1ull;
  uint32_t cbase = 0, cend = 0, cnext = kWalkChunk;  // the wave's chunk [cbase, cend)
  uint32_t qx = blockIdx.x & 7u, tried = 0;           // current range, ranges drained
  bool drained = false;
  // this lane's query
  bool active = false, have = false;
  uint32_t q = 0, m = 0, own = 0, end = 0, lo = 0, hi = 0, u = 0, ri = 0;
  uint32_t anc = 0, root = 0;  // MODE 0: the node whose sibling subtree is walked
  float a[6] = {0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f};
  float best = __int_as_float(0x7F800000);  // MODE 0: nearest so far
  float tlo = 0.0f;                         // MODE 0: the walk ends once best < tlo
  float l2 = 0.0f;                          // MODE 1: ell^2 of the node
  uint32_t ntest = 0, neval = 0;            // work counts (profiling)
  while (true) {
    // idle lanes take the next points of the wave's chunk
    while (!drained) {
      const unsigned long long idle = __ballot(!active);
      if (idle == 0) break;
      if (cnext >= kWalkChunk) {
        // range qx holds the queries [MQ qx / 8, MQ (qx + 1) / 8)
        const uint32_t r0 = (uint32_t)(((unsigned long long)MQ * qx) >> 3);
        const uint32_t r1 = (uint32_t)(((unsigned long long)MQ * (qx + 1u)) >> 3);
        uint32_t c = 0;
        if (lane == 0) c = atomicAdd(queue + 16u * qx, kWalkChunk);
        c = __shfl(c, 0);
        if (c >= r1 - r0) {  // this range is drained: the next one
          qx = (qx + 1u) & 7u;
          if (++tried == 8u) drained = true;
          continue;
        }
        cbase = r0 + c;
        cend = min(cbase + kWalkChunk, r1);
        cnext = 0;
      }
      const uint32_t left = cend - cbase > cnext ? cend - cbase - cnext : 0u;
      const uint32_t avail = min(kWalkChunk - cnext, left);
      const uint32_t rank = (uint32_t)__popcll(idle & below);
      if (!active && rank < avail) {
        q = (cbase + cnext + rank) * stride;  // query -> sorted point
        for (int c = 0; c < 6; ++c) a[c] = pt[6ull * q + c];
        const uint32_t b = pb[q];
        m = pm[q];
        own = leafof[q];
        hi = T[own + 1].lo;
        if (MODE == 0) {
          lo = T[own].lo;
          root = troot[b];
          anc = own;
          u = end = 0u;  // no subtree yet: the first step goes up from the own leaf
          best = TH ? TH[b] : __int_as_float(0x7F800000);
          tlo = TL ? TL[b] : 0.0f;
          active = ONLY == nullptr || ONLY[b] != 0u;
        } else {
          end = troot[b + 1];  // the record after the point's tree
          l2 = sc.ell2[gnode[b]];
          u = GS[q];  // the own group was linked by the first pass
          active = __uint_as_float(D[m]) <= l2;
          if (active) ri = uf_find(par, m);
        }
        have = MODE == 0;  // MODE 0: the own leaf first
      }
      const uint32_t took = min((uint32_t)__popcll(idle), avail);
      cnext = avail == 0 ? kWalkChunk : cnext + took;
    }
    if (!__any(active)) break;
    // one step of this lane's walk: up to kLeafStep points of the leaf it is
    // searching, else one record.  Lanes in either kind of step run together,
    // so no lane waits for the others to reach a leaf.
    if (active) {
      if (have) {
        const uint32_t jn = lo < hi ? min(hi, lo + kLeafStep<MODE>) : lo;
        if (COUNT) neval += jn - lo;
#pragma unroll
        for (uint32_t k = 0; k < kLeafStep<MODE>; ++k) {
          const uint32_t j = lo + k;
          if (j < jn) {
            const float* pj = pt + 6ull * j;
            const float d = d2_6(a[0], a[1], a[2], a[3], a[4], a[5], pj[0], pj[1], pj[2],
                                 pj[3], pj[4], pj[5]);
            if (MODE == 0) {
              best = j != q ? fminf(best, d) : best;
            } else if (d <= l2) {
              const uint32_t rj = uf_find(par, pm[j]);
              if (rj != ri) ri = uf_union(par, ri, rj);
            }
          }
        }
        lo = jn;
        have = jn < hi;
        if (MODE == 0 && best < tlo) {  // certainly below the bracket: done
          D[m] = __float_as_uint(best);
          active = false;
        }
      } else if (u >= end) {
        if (MODE == 1 || anc == root) {
          if (MODE == 0) D[m] = __float_as_uint(best);
          active = false;
        } else {  // the next subtree: the sibling of anc, whose parent is next
          const uint4 up = UP[anc];
          anc = up.x;
          u = up.y;
          end = up.z;
        }
      } else {
        const KdNode r = T[u];
        const float g = point_gap2(a, r);
        if (COUNT) ++ntest;
        bool in = MODE == 0 ? g < best : g <= l2;
        if (MODE == 1 && in) {
          // a node whose points all share one root holds no new link for a
          // lane in that set (sets only merge)
          const uint32_t ur = UR[u];
          if (ur != kNoRoot) {
            const uint32_t rr = uf_find(par, ur);
            if (rr != ri) ri = uf_find(par, ri);
            in = rr != ri;
          }
        }
        if (!in) {
          u = r.skip;
        } else {
          if (r.skip == u + 1u) {  // a leaf
            lo = r.lo;
            hi = T[u + 1].lo;
            have = true;
          }
          u = u + 1u;
        }
      }
    }
  }
  if (COUNT) {
    unsigned long long t = ntest, e = neval;
    for (int o = 32; o > 0; o >>= 1) {
      t += __shfl_xor(t, o);
      e += __shfl_xor(e, o);
    }
    if (lane == 0) {
      atomicAdd(work + 2 * MODE, t);
      atomicAdd(work + 2 * MODE + 1, e);
    }
  }
}

// First pass of the FOF search, one lane per sorted point q: its group is
// the largest subtree of at most kFofGroup points that holds its leaf (the
// leaf itself when that is larger), found by climbing from the leaf; a point
// with D <= ell^2 links the points after it in its group.  The record after
// the group's subtree is where q's walk starts.
__global__ void k_kd_group_fof(const KdNode* __restrict__ T, const float* __restrict__ pt,
                               const uint32_t* __restrict__ pm, const uint32_t* __restrict__ pb,
                               const uint32_t* __restrict__ leafof,
                               const uint32_t* __restrict__ troot, const uint4* __restrict__ UP,
                               uint32_t MB, const uint32_t* __restrict__ gnode, NodeScratch sc,
                               const uint32_t* D, uint32_t* par, uint32_t* gskip) {
  const uint32_t q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= MB) return;
  const uint32_t b = pb[q], root = troot[b];
  uint32_t u = leafof[q];
  KdNode r = T[u];
  while (u != root) {  // every node but a root has its parent in UP
    const uint32_t p = UP[u].x;
    const KdNode rp = T[p];
    if (T[rp.skip].lo - rp.lo > kFofGroup) break;
    u = p;
    r = rp;
  }
  gskip[q] = r.skip;
  const uint32_t m = pm[q];
  const float l2 = sc.ell2[gnode[b]];
  if (!(__uint_as_float(D[m]) <= l2)) return;
  float a[6];
  for (int c = 0; c < 6; ++c) a[c] = pt[6ull * q + c];
  const uint32_t hi = T[r.skip].lo;
  uint32_t ri = uf_find(par, m);
  for (uint32_t j = q + 1u; j < hi; ++j) {
    const float* pj = pt + 6ull * j;
    const float d =
        d2_6(a[0], a[1], a[2], a[3], a[4], a[5], pj[0], pj[1], pj[2], pj[3], pj[4], pj[5]);
    if (d <= l2) {
      const uint32_t rj = uf_find(par, pm[j]);
      if (rj != ri) ri = uf_union(par, ri, rj);
    }
  }
}

// The root shared by all points of each node of at most kFofGroup points, or
// kNoRoot (read-only finds: nothing else runs on the forest meanwhile).
__global__ void k_kd_uroot(const KdNode* __restrict__ T, const uint32_t* __restrict__ pm,
                           uint32_t NN, const uint32_t* par, uint32_t* uroot) {
  const uint32_t u = blockIdx.x * blockDim.x + threadIdx.x;
  if (u >= NN) return;
  const KdNode r = T[u];
  const uint32_t lo = r.lo, hi = T[r.skip].lo;
  uint32_t ur = kNoRoot;
  if (hi > lo && hi - lo <= kFofGroup) {
    ur = uf_root(par, pm[lo]);
    for (uint32_t j = lo + 1u; j < hi && ur != kNoRoot; ++j)
      if (uf_root(par, pm[j]) != ur) ur = kNoRoot;
  }
  uroot[u] = ur;
}

// Persistent grid of the walks: as many waves as the chip holds at the
// kernel's occupancy (8 per SIMD), fewer when there are fewer chunks.
unsigned walk_grid(uint32_t MB) {
  const uint32_t chunks = (MB + kWalkChunk - 1) / kWalkChunk;
  const uint32_t waves = min(chunks, 256u * 4u * 8u);
  return (waves + kWalkTB / 64 - 1) / (kWalkTB / 64);
}

}  // namespace

void grid_take(Arena& A, GridBufs& g, uint32_t M, uint32_t Kmax, uint32_t leaf) {
  const uint32_t NBmax = M / kGridFloor + 2;
  g.nb_rank = A.take<uint32_t>(Kmax + 2);
  g.gnode = A.take<uint32_t>(NBmax);
  g.pstart = A.take<uint32_t>(NBmax + 1);
  g.gcount = A.take<uint32_t>(NBmax + 1);
  g.tl = A.take<float>(NBmax + 1);
  g.th = A.take<float>(NBmax + 1);
  g.tmap = A.take<uint32_t>(NBmax + 1);
  g.redo = A.take<uint32_t>(NBmax + 1);
  // tree nodes: the capacity bounds memory, not results (a node that finds no
  // room for its children stays a leaf and is searched in full); trees of
  // leaves of at most L particles use about 3.2 / L nodes per particle
  g.leaf = leaf;
  const uint32_t cap = (uint32_t)((4ull * M) / leaf) + NBmax + 64;
  mtree_take(A, *g.mt, cap, NBmax);
  g.node = A.take<KdNode>(cap + 1);
  g.up = A.take<uint4>(cap + 1);
  g.uroot = A.take<uint32_t>(cap + 1);
  g.gskip = A.take<uint32_t>((size_t)M + 2);
  g.flag = A.take<uint32_t>((size_t)M + 2);
  g.pos = A.take<uint32_t>((size_t)M + 2);
  g.k0 = A.take<unsigned long long>((size_t)M + 2);
  g.k1 = A.take<unsigned long long>((size_t)M + 2);
  g.v0 = A.take<uint32_t>((size_t)M + 2);
  g.v1 = A.take<uint32_t>((size_t)M + 2);
  g.pt = A.take<float>(6ull * ((size_t)M + 2));
  g.pm = A.take<uint32_t>((size_t)M + 2);
  g.pb = A.take<uint32_t>((size_t)M + 2);
  g.leafof = A.take<uint32_t>((size_t)M + 2);
  g.cnt = A.take<uint32_t>(16);
  g.queue = A.take<uint32_t>(128);
  g.rtmp = A.take<char>(radix_tmp_bytes((int64_t)M + 2));
  g.stmp = A.take<uint32_t>(scan_tmp_elems<uint32_t>((int64_t)M + Kmax + 4));
}

uint32_t grid_build(GridBufs& g, const float* xi, size_t S, LevelNodes nd, uint32_t K,
                    const uint32_t* lnode, uint32_t Mi, uint32_t M, NodeScratch sc,
                    uint32_t* hb, hipStream_t s, uint32_t gmin) {
  g.NB = 0;
  g.MB = 0;
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
  MTree& t = *g.mt;
  mtree_build(t, key, g.pstart, g.gcount, NB, g.leaf, kKdMaxDepth, hb + 2, s);
  g.troot = t.troot;
  for (int d = (int)t.lev.size() - 2; d >= 0; --d) {
    const uint32_t nu = t.lev[d + 1] - t.lev[d];
    k_kd_records<<<blocks_for(nu, TB), TB, 0, s>>>(g, t.bnode, t.pre, t.lev[d], nu);
  }
  k_kd_sentinel<<<1, 1, 0, s>>>(g.node, t.NN, MB);
  return NB;
}

void grid_nn(GridBufs& g, NodeScratch sc, uint32_t* D, uint32_t stride, const float* tl,
             const float* th, const uint32_t* only, unsigned long long* work, hipStream_t s) {
  if (g.NB == 0 || g.MB == 0) return;
  const uint32_t MQ = (g.MB + stride - 1) / stride;
  k_fill_u32<<<1, 128, 0, s>>>(g.queue, 128, 0u);
  if (work)
    k_kd_walk<0, true><<<walk_grid(MQ), kWalkTB, 0, s>>>(
        g.node, g.pt, g.pm, g.pb, g.leafof, g.troot, g.MB, g.gnode, sc, D, nullptr, g.queue,
        g.up, nullptr, nullptr, MQ, stride, tl, th, only, work);
  else
    k_kd_walk<0, false><<<walk_grid(MQ), kWalkTB, 0, s>>>(
        g.node, g.pt, g.pm, g.pb, g.leafof, g.troot, g.MB, g.gnode, sc, D, nullptr, g.queue,
        g.up, nullptr, nullptr, MQ, stride, tl, th, only, nullptr);
}

void grid_fof_groups(GridBufs& g, NodeScratch sc, const uint32_t* D, uint32_t* par,
                     hipStream_t s) {
  if (g.NB == 0 || g.MB == 0) return;
  k_kd_group_fof<<<blocks_for(g.MB, TB), TB, 0, s>>>(g.node, g.pt, g.pm, g.pb, g.leafof, g.troot,
                                                    g.up, g.MB, g.gnode, sc, D, par, g.gskip);
  const uint32_t NN = g.mt->NN;
  k_kd_uroot<<<blocks_for(NN, TB), TB, 0, s>>>(g.node, g.pm, NN, par, g.uroot);
}

void grid_fof(GridBufs& g, NodeScratch sc, const uint32_t* D, uint32_t* par,
              unsigned long long* work, hipStream_t s) {
  if (g.NB == 0 || g.MB == 0) return;
  k_fill_u32<<<1, 128, 0, s>>>(g.queue, 128, 0u);
  uint32_t* Dm = const_cast<uint32_t*>(D);
  if (work)
    k_kd_walk<1, true><<<walk_grid(g.MB), kWalkTB, 0, s>>>(
        g.node, g.pt, g.pm, g.pb, g.leafof, g.troot, g.MB, g.gnode, sc, Dm, par, g.queue, g.up,
        g.gskip, g.uroot, g.MB, 1u, nullptr, nullptr, nullptr, work);
  else
    k_kd_walk<1, false><<<walk_grid(g.MB), kWalkTB, 0, s>>>(
        g.node, g.pt, g.pm, g.pb, g.leafof, g.troot, g.MB, g.gnode, sc, Dm, par, g.queue, g.up,
        g.gskip, g.uroot, g.MB, 1u, nullptr, nullptr, nullptr, nullptr);
}

}  // namespace refine
}  // namespace halo
