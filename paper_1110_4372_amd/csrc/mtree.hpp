// Binary trees over Morton-sorted ranges, shared by the 6D neighbour search of
// large hierarchy nodes and the tree potential of large haloes.
#pragma once
#include <vector>

#include "common.hpp"

namespace halo {

constexpr uint32_t kMtNone = 0xFFFFFFFFu;

// A node while its tree is built, level by level: its range [lo, hi) of the
// sorted order, its first child (the second is next to it) or kMtNone, and its
// depth (replaced by its subtree's node count once the tree is built).
struct __align__(16) MtNode {
  uint32_t lo, hi, left, aux;
};

// Trees over NB sorted ranges [first[b], first[b] + count[b]) of 64-bit keys.
// A node holding more than `leaf` elements splits where the highest key bit
// that differs across its range changes, at the middle of the range when all
// its keys are equal: the split of a radix tree over Morton codes (Karras 2012,
// "Maximizing parallelism in the construction of BVHs, octrees, and k-d
// trees"), so each child covers one cell of the curve.  Nodes at depth
// `max_depth`, and nodes whose children would pass the capacity, stay leaves.
// After mtree_build:
//   - bnode[lev[d] .. lev[d+1]) are the nodes of depth d (roots: 0 .. NB-1),
//     bnode[u].aux the node count of u's subtree;
//   - pre[u] is u's index in the depth-first preorder (first child first) of
//     all trees, tree b occupying [troot[b], troot[b+1]); in that order a
//     node's first child is the next index and pre[u] + aux the index after
//     its subtree;
//   - ppar[pre[u]] is the preorder index of u's parent (kMtNone for roots).
struct MTree {
  MtNode* bnode = nullptr;
  uint32_t *pre = nullptr, *ppar = nullptr, *troot = nullptr;
  uint32_t *split = nullptr, *flag = nullptr, *pos = nullptr, *cnt = nullptr, *stmp = nullptr;
  uint32_t cap = 0, NN = 0;
  std::vector<uint32_t> lev;
};

void mtree_take(Arena& A, MTree& t, uint32_t cap, uint32_t nb_max);
void mtree_build(MTree& t, const unsigned long long* key, const uint32_t* first,
                 const uint32_t* count, uint32_t NB, uint32_t leaf, uint32_t max_depth,
                 uint32_t* hb, hipStream_t s);

}  // namespace halo
