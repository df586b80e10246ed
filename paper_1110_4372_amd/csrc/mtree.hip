// Binary trees over Morton-sorted ranges (see mtree.hpp): top-down splits one
// depth per step, then subtree counts and the depth-first preorder.
#include <algorithm>

#include "mtree.hpp"
#include "primitives.hpp"

namespace halo {

namespace {

constexpr int TB = 256;

__global__ void k_mt_roots(MtNode* bnode, const uint32_t* first, const uint32_t* count,
                           uint32_t NB) {
  const uint32_t b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b < NB) bnode[b] = MtNode{first[b], first[b] + count[b], kMtNone, 0u};
}

// Split point of each frontier node that holds more than a leaf.
__global__ void k_mt_split(const MtNode* bnode, const unsigned long long* __restrict__ key,
                           uint32_t f0, uint32_t nf, uint32_t leaf, uint32_t max_depth,
                           uint32_t* flag, uint32_t* split) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nf) return;
  const MtNode u = bnode[f0 + i];
  const uint32_t lo = u.lo, hi = u.hi;
  if (hi - lo <= leaf || u.aux >= max_depth) {
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
// a split whose children would pass the capacity is not made.
__global__ void k_mt_children(MtNode* bnode, uint32_t cap, uint32_t f0, uint32_t nf, uint32_t f1,
                              const uint32_t* flag, const uint32_t* pos, const uint32_t* split) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nf || !flag[i]) return;
  const uint32_t c = f1 + 2u * pos[i];
  if (c + 2u > cap) return;
  MtNode& u = bnode[f0 + i];
  bnode[c] = MtNode{u.lo, split[i], kMtNone, u.aux + 1u};
  bnode[c + 1] = MtNode{split[i], u.hi, kMtNone, u.aux + 1u};
  u.left = c;
}

// Subtree node counts of one depth from the deeper depth's; roots' counts are
// copied out for the prefix of the trees' preorder bases.
__global__ void k_mt_sizes(MtNode* bnode, uint32_t u0, uint32_t nu, uint32_t NB,
                           uint32_t* rsize) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nu) return;
  MtNode& u = bnode[u0 + i];
  const uint32_t c =
      u.left == kMtNone ? 1u : 1u + bnode[u.left].aux + bnode[u.left + 1].aux;
  u.aux = c;
  if (u0 + i < NB) rsize[u0 + i] = c;
}

__global__ void k_mt_pre_roots(const uint32_t* troot, uint32_t NB, uint32_t* pre,
                               uint32_t* ppar) {
  const uint32_t b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= NB) return;
  pre[b] = troot[b];
  ppar[troot[b]] = kMtNone;
}

// Preorder indices of the children of one depth's nodes: the first child right
// after its parent, the second after the first child's subtree.
__global__ void k_mt_pre(const MtNode* bnode, uint32_t u0, uint32_t nu, uint32_t* pre,
                         uint32_t* ppar) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nu) return;
  const MtNode u = bnode[u0 + i];
  if (u.left == kMtNone) return;
  const uint32_t p = pre[u0 + i];
  const uint32_t a = p + 1u, b = p + 1u + bnode[u.left].aux;
  pre[u.left] = a;
  pre[u.left + 1] = b;
  ppar[a] = p;
  ppar[b] = p;
}

}  // namespace

void mtree_take(Arena& A, MTree& t, uint32_t cap, uint32_t nb_max) {
  t.cap = cap;
  t.bnode = A.take<MtNode>(cap);
  t.pre = A.take<uint32_t>(cap);
  t.ppar = A.take<uint32_t>(cap);
  t.split = A.take<uint32_t>(cap);
  t.flag = A.take<uint32_t>(cap);
  t.pos = A.take<uint32_t>(cap);
  t.troot = A.take<uint32_t>(nb_max + 1);
  t.cnt = A.take<uint32_t>(16);
  t.stmp = A.take<uint32_t>(scan_tmp_elems<uint32_t>(cap));
}

void mtree_build(MTree& t, const unsigned long long* key, const uint32_t* first,
                 const uint32_t* count, uint32_t NB, uint32_t leaf, uint32_t max_depth,
                 uint32_t* hb, hipStream_t s) {
  HALO_CHECK(NB > 0 && NB <= t.cap, LIBHALO_EINVAL, "tree roots exceed the node capacity");
  t.lev.assign({0u, NB});
  k_mt_roots<<<blocks_for(NB, TB), TB, 0, s>>>(t.bnode, first, count, NB);
  for (uint32_t d = 0; d < max_depth; ++d) {
    const uint32_t f0 = t.lev[d], f1 = t.lev[d + 1], nf = f1 - f0;
    if (nf == 0) break;
    k_mt_split<<<blocks_for(nf, TB), TB, 0, s>>>(t.bnode, key, f0, nf, leaf, max_depth, t.flag,
                                                 t.split);
    exclusive_scan<uint32_t>(t.flag, t.pos, nf, t.cnt, t.stmp, s);
    k_mt_children<<<blocks_for(nf, TB), TB, 0, s>>>(t.bnode, t.cap, f0, nf, f1, t.flag, t.pos,
                                                    t.split);
    HALO_HIP(hipMemcpyAsync(hb, t.cnt, 4, hipMemcpyDeviceToHost, s));
    HALO_HIP(hipStreamSynchronize(s));
    const uint32_t room = (t.cap - f1) / 2u;
    t.lev.push_back(f1 + 2u * std::min(hb[0], room));
  }
  while (t.lev.size() > 2 && t.lev[t.lev.size() - 2] == t.lev.back()) t.lev.pop_back();
  t.NN = t.lev.back();
  const int depths = (int)t.lev.size() - 1;
  for (int d = depths - 1; d >= 0; --d) {
    const uint32_t nu = t.lev[d + 1] - t.lev[d];
    k_mt_sizes<<<blocks_for(nu, TB), TB, 0, s>>>(t.bnode, t.lev[d], nu, NB, t.flag);
  }
  exclusive_scan<uint32_t>(t.flag, t.troot, NB, t.troot + NB, t.stmp, s);
  k_mt_pre_roots<<<blocks_for(NB, TB), TB, 0, s>>>(t.troot, NB, t.pre, t.ppar);
  for (int d = 0; d < depths; ++d) {
    const uint32_t nu = t.lev[d + 1] - t.lev[d];
    k_mt_pre<<<blocks_for(nu, TB), TB, 0, s>>>(t.bnode, t.lev[d], nu, t.pre, t.ppar);
  }
}

}  // namespace halo
