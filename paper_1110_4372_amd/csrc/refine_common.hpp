// Level-synchronous hierarchy state shared by the refinement kernels.
#pragma once
#include <algorithm>

#include "common.hpp"
#include "mtree.hpp"

namespace halo {
namespace refine {

constexpr int TB = 256;
constexpr int kMomTile = 1024;       // particles per moment work item
constexpr int kPairI = 256;          // i particles per pair work item
constexpr int kPairJ = 2048;         // j particles per pair work item
constexpr int kNNJ = 1024;           // minimum j-chunk of a nearest-neighbour unit
constexpr uint32_t kSmallLevel = 262144;  // levels below this many particles use
constexpr uint32_t kNNJSmall = 256;       //   these shorter chunks
constexpr uint32_t kPairJSmall = 512;
constexpr uint32_t kSymJMax = 4096;  // maximum j-chunk (its minima sit in LDS)
constexpr int kSelSmall = 4096;      // nodes up to this size select in LDS
constexpr int kSelTile = 4096;       // elements per big-node select item
constexpr unsigned kPersist = 4096;  // persistent grid of pair / moment kernels

struct LevelNodes {
  uint32_t* first;
  uint32_t* count;
  int32_t* parent;  // global row of the parent, -1 at level 0
  uint32_t* fof;
  uint32_t* canon;
};

struct NodeScratch {
  uint32_t* gstate;          // 0 all-pairs, 1 tree search
  I128* acc;                 // 8 per node: sum qx, qy, qz, q^2, sum wx, wy, wz, w^2
  unsigned long long* ext;   // 6 per node: ordered min/max of u per axis (level 0)
  double* prm;               // 12 per node: anchor xyz, ubar xyz, vbar xyz, isx, isv, active
  uint32_t* kth;             // target rank (1-based)
  float* ell2;
  uint32_t* whole;
  uint32_t* nch;
  uint32_t* fch;
  uint32_t* wmom;            // worklist offsets (K+1)
  uint32_t* wpair;
  uint32_t* big;             // big-node list for selection
  uint32_t* wbig;
  uint32_t* selp;            // prefix / remaining per big node
  uint32_t* ghist;           // 256 per big node
};

__device__ __forceinline__ uint32_t seg_of(const uint32_t* off, uint32_t K, uint32_t w) {
  // last k with off[k] <= w (off non-decreasing, off[0] = 0)
  uint32_t lo = 0, hi = K;
  while (hi - lo > 1) {
    uint32_t mid = (lo + hi) >> 1;
    if (off[mid] <= w)
      lo = mid;
    else
      hi = mid;
  }
  return lo;
}


// ---- exact tree search for large nodes (grid6d.hip) ----
// Default tree threshold: nodes above it use the tree search.  The walks need
// many points to fill the chip (a launch's slowest walks set its tail), so the
// low threshold applies only on levels of at least kGridLevel particles.
constexpr uint32_t kGridMin = 16384;
constexpr uint32_t kGridMinSmall = 131072;
constexpr uint32_t kGridLevel = 1u << 23;
__host__ __device__ inline uint32_t default_grid_min(uint32_t level_particles) {
  return level_particles >= kGridLevel ? kGridMin : kGridMinSmall;
}
constexpr uint32_t kGridFloor = 64;   // smallest accepted threshold
constexpr uint32_t kKdLeaf = 16;      // default: a tree node of at most this many particles is a leaf
constexpr int kKdMaxDepth = 64;       // nodes at this depth are leaves whatever their size
constexpr uint32_t kFofGroup = 64;    // most points of a group of the FOF search's first pass

// A tree node as the walks read it, in depth-first preorder (first child
// first) so that a node's first child is the next record and `skip` is the
// record after its subtree: the bounding box of its particles in half
// precision, each bound rounded outward (so the box holds every particle and
// a gap computed from it never exceeds the FP32 one), and the first particle
// of its range in the sorted order.  A node is a leaf when skip is the next
// record; its range ends where the next record's begins (the preorder tiles
// the sorted order from left to right; a sentinel record closes the last
// tree).  32 bytes.
struct __align__(16) KdNode {
  uint16_t mn[6], mx[6];  // binary16 bit patterns
  uint32_t lo, skip;
};

struct GridBufs {
  uint32_t *nb_rank, *gnode, *pstart, *gcount;
  uint32_t *flag, *pos, *v0, *v1, *cnt, *stmp, *leafof;
  uint32_t* queue;   // the walks' eight work-queue counters, 64 B apart (zeroed before each)
  unsigned long long *k0, *k1;
  float* pt;         // MB points in sorted order, six normalised coordinates each
  uint32_t *pm, *pb; // their positions in the level arrays and their grid nodes
  KdNode* node;      // tree nodes in preorder; tree b is [troot[b], troot[b+1])
  uint4* up;         // per node: parent, sibling, the record after the sibling's subtree
  uint32_t* gskip;   // per sorted point: the record after its first-pass group's subtree
  uint32_t* uroot;   // per node of at most kFofGroup points: the root all its points share
  const uint32_t* troot;
  void* rtmp;
  // nearest-neighbour bracket of each tree node b: walks start at best = th[b]
  // and end once best < tl[b]; tmap lists the bracketed trees, redo flags a
  // tree whose ell^2 fell outside its bracket
  float *tl, *th;
  uint32_t *tmap, *redo;
  MTree* mt;         // host object: the trees' topology (mtree.hpp)
  uint32_t MB = 0, NB = 0;  // sorted points, grid nodes
  uint32_t leaf = kKdLeaf;  // most points of a leaf
};

void grid_take(Arena& A, GridBufs& g, uint32_t M, uint32_t Kmax, uint32_t leaf);
// Classifies the level's nodes (sc.gstate 1 for tree nodes) and builds the
// trees of those above gmin.  Returns their number.
uint32_t grid_build(GridBufs& g, const float* xi, size_t S, LevelNodes nd, uint32_t K,
                    const uint32_t* lnode, uint32_t Mi, uint32_t M, NodeScratch sc,
                    uint32_t* hb, hipStream_t s, uint32_t gmin);
// Nearest-neighbour walks of the tree nodes' particles, one per stride-th
// sorted point (1: every point).  tl, th (may be null: 0 and +inf): the walk
// of a point of tree b starts with th[b] as its best distance and ends as
// soon as its best is below tl[b], so D[m] is exact when it lies in
// [tl[b], th[b]), below tl[b] (an upper bound) when the true distance is, and
// th[b] when the true distance is at least th[b].  only (may be null): walk
// just the trees b with only[b] != 0.  work (may be null): adds the walk's
// box tests and distances to work[0], [1].
void grid_nn(GridBufs& g, NodeScratch sc, uint32_t* D, uint32_t stride, const float* tl,
             const float* th, const uint32_t* only, unsigned long long* work, hipStream_t s);
// 6D FOF at each tree node's ell^2 over its particles with D <= ell^2; work
// (may be null): box tests and distances added to work[2], [3].
void grid_fof(GridBufs& g, NodeScratch sc, const uint32_t* D, uint32_t* par,
              unsigned long long* work, hipStream_t s);
// First pass of that FOF: links the pairs within each group (the largest
// subtree of at most kFofGroup points holding a point's leaf), then records
// the nodes of at most kFofGroup points whose points share one root.  Runs
// before grid_fof, which then skips each point's own group.
void grid_fof_groups(GridBufs& g, NodeScratch sc, const uint32_t* D, uint32_t* par,
                     hipStream_t s);

// min over j in [j0, j1) of d2(i, j) over six FP32 coordinate planes of stride
// S; j is wave-uniform, so the j coordinates are scalar loads feeding the
// vector ops.  kSelf: skip j == self.
template <bool kSelf>
__device__ __forceinline__ float nn_span(const float* __restrict__ xi, size_t S, uint32_t j0,
                                         uint32_t j1, uint32_t self, const float* a,
                                         float best) {
  uint32_t j = j0;
  for (; j + 8 <= j1; j += 8) {
    float b[6][8];
#pragma unroll
    for (int c = 0; c < 6; ++c) {
      const float* __restrict__ p = xi + (size_t)c * S + j;
#pragma unroll
      for (int u = 0; u < 8; ++u) b[c][u] = p[u];
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const float d = d2_6(a[0], a[1], a[2], a[3], a[4], a[5], b[0][u], b[1][u], b[2][u],
                           b[3][u], b[4][u], b[5][u]);
      if (kSelf)
        best = (j + u != self) ? fminf(best, d) : best;
      else
        best = fminf(best, d);
    }
  }
  for (; j < j1; ++j) {
    const float d = d2_6(a[0], a[1], a[2], a[3], a[4], a[5], xi[j], xi[S + j], xi[2 * S + j],
                         xi[3 * S + j], xi[4 * S + j], xi[5 * S + j]);
    if (!kSelf || j != self) best = fminf(best, d);
  }
  return best;
}

}  // namespace refine
}  // namespace halo
