// Seeds, Poisson seed merging (Eq. 2), hierarchical particle assignment
// (Eqs. 3-4) and the single-timestep host/subhalo relation (Sections 3.3-3.4)
// on gfx950.
//
//  - seeds: one per leaf node, in node order;
//  - merging: one wavefront per FOF group walks its seeds by decreasing size
//    and compares each with the kept ones lane-parallel;
//  - seed sets: every (ancestor, merged seed) pair of every leaf, sorted and
//    made unique, gives the distinct halos below each node;
//  - assignment, deepest level first: the particles a node holds outside its
//    subgroups go to its only halo or to the Eq. 3 argmin (a wave of
//    spatially close particles first drops the seeds that cannot be nearest
//    to any of them), with sigma_v and
//    vmax of each candidate halo recomputed from its current particles by a
//    segmented radial sort (exact, order-independent reductions);
//  - host/sub: one wavefront per FOF group over halos by decreasing size.
#include <algorithm>
#include <cmath>

#include "primitives.hpp"
#include "radial.hpp"
#include "stages.hpp"

namespace halo {

namespace {

constexpr int TB = 256;

struct SeedT {  // internal seed table
  uint32_t* cnt;
  double* sx2;
  double* sv2;
};

__global__ void k_leaf_flags(const int32_t* n_children, uint32_t NN, uint32_t* flag) {
  uint32_t k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k < NN) flag[k] = n_children[k] == 0 ? 1u : 0u;
}

__global__ void k_seeds(libhalo_nodes nd, uint32_t NN, const uint32_t* flag,
                        const uint32_t* pos, libhalo_halos h, SeedT st, int32_t* node_seed) {
  uint32_t k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= NN) return;
  if (!flag[k]) {
    node_seed[k] = -1;
    return;
  }
  uint32_t s = pos[k];
  node_seed[k] = (int32_t)s;
  h.seed_node[s] = (int32_t)k;
  h.fof[s] = nd.fof[k];
  h.xs[s] = nd.cx[k];
  h.ys[s] = nd.cy[k];
  h.zs[s] = nd.cz[k];
  h.vxs[s] = nd.vx[k];
  h.vys[s] = nd.vy[k];
  h.vzs[s] = nd.vz[k];
  h.host[s] = -1;
  st.cnt[s] = nd.count[k];
  st.sx2[s] = nd.sx2[k];
  st.sv2[s] = nd.sv2[k];
}

// key = fof * 2^32 + (2^32 - 1 - size): ascending key = (fof asc, size desc)
__global__ void k_group_size_keys(const uint32_t* fof, const uint32_t* size, uint32_t S,
                                  unsigned long long* key, uint32_t* val) {
  uint32_t s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= S) return;
  key[s] = ((unsigned long long)fof[s] << 32) | (unsigned long long)(0xFFFFFFFFu - size[s]);
  val[s] = s;
}

__global__ void k_fof_heads(const unsigned long long* key, uint32_t S, uint32_t* head) {
  uint32_t q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= S) return;
  head[q] = (q == 0 || (key[q] >> 32) != (key[q - 1] >> 32)) ? 1u : 0u;
}

__global__ void k_fof_segments(const uint32_t* head, const uint32_t* hpos, uint32_t S,
                               uint32_t* seg_start) {
  uint32_t q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= S) return;
  if (head[q]) seg_start[hpos[q]] = q;
}

// Eq. 2 merging, one wavefront per FOF group of at most kMergeWave seeds.
// kept[] holds, per group, the kept seeds in visiting order (at the group's
// slice of ord).
constexpr uint32_t kMergeWave = 512;
constexpr int kMergeTB = 1024;
constexpr uint32_t kMergeLds = 1024;  // kept seeds held in LDS by k_merge_big
__global__ void k_merge(const uint32_t* ord, const uint32_t* seg_start, const uint32_t* nseg,
                        uint32_t S, double box, double q2, libhalo_halos h, SeedT st,
                        uint32_t* kept) {
  const uint32_t F = nseg[0];
  const uint32_t wave = (blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const int lane = threadIdx.x & 63;
  if (wave >= F) return;
  const uint32_t a0 = seg_start[wave];
  const uint32_t a1 = (wave + 1 < F) ? seg_start[wave + 1] : S;
  if (a1 - a0 > kMergeWave) return;  // k_merge_big
  uint32_t nk = 0;
  for (uint32_t t = a0; t < a1; ++t) {
    const uint32_t b = ord[t];
    const double cb = (double)st.cnt[b], sx2 = st.sx2[b], sv2 = st.sv2[b];
    double bq = INFINITY;
    uint32_t best = 0xFFFFFFFFu;
    if (sx2 > 0.0 && sv2 > 0.0) {
      const double imx = cb / sx2, imv = cb / sv2;
      for (uint32_t q = lane; q < nk; q += 64) {
        const uint32_t a = kept[a0 + q];
        double dx = min_image(h.xs[b] - h.xs[a], box);
        double dy = min_image(h.ys[b] - h.ys[a], box);
        double dz = min_image(h.zs[b] - h.zs[a], box);
        double ux = h.vxs[b] - h.vxs[a], uy = h.vys[b] - h.vys[a], uz = h.vzs[b] - h.vzs[a];
        double qq = __fma_rn(sq3(dx, dy, dz), imx, sq3(ux, uy, uz) * imv);
        if (qq < bq || (qq == bq && a < best)) {
          bq = qq;
          best = a;
        }
      }
      for (int o = 32; o > 0; o >>= 1) {
        double oq = __shfl_xor(bq, o);
        uint32_t ob = __shfl_xor(best, o);
        if (oq < bq || (oq == bq && ob < best)) {
          bq = oq;
          best = ob;
        }
      }
    }
    if (best != 0xFFFFFFFFu && bq < q2) {
      if (lane == 0) h.merged_into[b] = (int32_t)best;
    } else {
      if (lane == 0) {
        h.merged_into[b] = (int32_t)b;
        kept[a0 + nk] = b;
      }
      ++nk;
    }
    __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "workgroup");
    __builtin_amdgcn_wave_barrier();
  }
}

// Eq. 2 merging of the groups with more than kMergeWave seeds, one block
// per group: the same sequential visit as k_merge, with the kept seeds'
// positions and velocities in LDS (beyond kMergeLds read from the halo table)
// and a block-wide argmin per visited seed (ties to the lower id).
__global__ void __launch_bounds__(kMergeTB)
    k_merge_big(const uint32_t* ord, const uint32_t* seg_start, const uint32_t* nseg,
                uint32_t S, double box, double q2, libhalo_halos h, SeedT st,
                uint32_t* kept) {
  constexpr int NW = kMergeTB / 64;
  __shared__ double kx[kMergeLds], ky[kMergeLds], kz[kMergeLds];
  __shared__ double kvx[kMergeLds], kvy[kMergeLds], kvz[kMergeLds];
  __shared__ uint32_t kid[kMergeLds];
  __shared__ double wq[NW];
  __shared__ uint32_t wb[NW];
  __shared__ uint32_t s_big[kMergeTB];
  __shared__ uint32_t s_nbig;
  const uint32_t F = nseg[0];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  for (uint32_t g0 = blockIdx.x * kMergeTB; g0 < F; g0 += gridDim.x * kMergeTB) {
    // the big groups among groups g0 .. g0 + kMergeTB - 1
    if (threadIdx.x == 0) s_nbig = 0;
    __syncthreads();
    {
      const uint32_t g = g0 + threadIdx.x;
      if (g < F) {
        const uint32_t a1 = (g + 1 < F) ? seg_start[g + 1] : S;
        if (a1 - seg_start[g] > kMergeWave) s_big[atomicAdd(&s_nbig, 1u)] = g;
      }
    }
    __syncthreads();
    const uint32_t nbig = s_nbig;
    for (uint32_t gi = 0; gi < nbig; ++gi) {
      const uint32_t g = s_big[gi];
      const uint32_t a0 = seg_start[g];
      const uint32_t a1 = (g + 1 < F) ? seg_start[g + 1] : S;
      uint32_t nk = 0;
      for (uint32_t t = a0; t < a1; ++t) {
        const uint32_t b = ord[t];
        const double cb = (double)st.cnt[b], sx2 = st.sx2[b], sv2 = st.sv2[b];
        const double xb = h.xs[b], yb = h.ys[b], zb = h.zs[b];
        const double vxb = h.vxs[b], vyb = h.vys[b], vzb = h.vzs[b];
        double bq = INFINITY;
        uint32_t best = 0xFFFFFFFFu;
        const bool can = sx2 > 0.0 && sv2 > 0.0;
        if (can) {
          const double imx = cb / sx2, imv = cb / sv2;
          for (uint32_t q = threadIdx.x; q < nk; q += kMergeTB) {
            uint32_t a;
            double ax, ay, az, avx, avy, avz;
            if (q < kMergeLds) {
              a = kid[q];
              ax = kx[q]; ay = ky[q]; az = kz[q];
              avx = kvx[q]; avy = kvy[q]; avz = kvz[q];
            } else {
              a = kept[a0 + q];
              ax = h.xs[a]; ay = h.ys[a]; az = h.zs[a];
              avx = h.vxs[a]; avy = h.vys[a]; avz = h.vzs[a];
            }
            double dx = min_image(xb - ax, box);
            double dy = min_image(yb - ay, box);
            double dz = min_image(zb - az, box);
            double ux = vxb - avx, uy = vyb - avy, uz = vzb - avz;
            double qq = __fma_rn(sq3(dx, dy, dz), imx, sq3(ux, uy, uz) * imv);
            if (qq < bq || (qq == bq && a < best)) {
              bq = qq;
              best = a;
            }
          }
          for (int o = 32; o > 0; o >>= 1) {
            double oq = __shfl_xor(bq, o);
            uint32_t ob = __shfl_xor(best, o);
            if (oq < bq || (oq == bq && ob < best)) {
              bq = oq;
              best = ob;
            }
          }
          if (lane == 0) {
            wq[wid] = bq;
            wb[wid] = best;
          }
        }
        __syncthreads();
        if (can) {
          bq = wq[0];
          best = wb[0];
          for (int w = 1; w < NW; ++w)
            if (wq[w] < bq || (wq[w] == bq && wb[w] < best)) {
              bq = wq[w];
              best = wb[w];
            }
        }
        const bool merge = best != 0xFFFFFFFFu && bq < q2;
        if (threadIdx.x == 0) {
          if (merge) {
            h.merged_into[b] = (int32_t)best;
          } else {
            h.merged_into[b] = (int32_t)b;
            kept[a0 + nk] = b;
            if (nk < kMergeLds) {
              kid[nk] = b;
              kx[nk] = xb; ky[nk] = yb; kz[nk] = zb;
              kvx[nk] = vxb; kvy[nk] = vyb; kvz[nk] = vzb;
            }
          }
        }
        if (!merge) ++nk;
        __syncthreads();
      }
    }
    __syncthreads();
  }
}

// Eq. 2 merging of the groups with more than kMergeWave seeds, in parallel
// over all their seeds: the visit in k_merge_big decides seed b (position t of
// its group's slice of ord) from the kept seeds before it, and merges b into
// the argmin a of q(a, b) when that is below q2.  Only earlier seeds with
// q(a, b) < q2 can matter, so they are listed for every b first (the same FP64
// expression as the visit), and one thread per group then resolves its seeds
// in order, visiting only those with a candidate: b stays kept unless some
// candidate is still kept, and merges into the kept candidate of least q
// (ties to the lower id).
template <bool kWrite>
__global__ void k_merge_cand(const uint32_t* ord, const uint32_t* head, const uint32_t* hpos,
                             const uint32_t* seg_start, const uint32_t* nseg, uint32_t S,
                             double box, double q2, libhalo_halos h, SeedT st, uint32_t* ccnt,
                             const uint32_t* cstart, uint32_t* cpos, double* cq) {
  const uint32_t t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= S) return;
  const uint32_t F = nseg[0];
  const uint32_t g = hpos[t] + head[t] - 1u;
  const uint32_t a0 = seg_start[g], a1 = (g + 1 < F) ? seg_start[g + 1] : S;
  uint32_t c = 0, w = kWrite ? cstart[t] : 0u;
  if (a1 - a0 > kMergeWave) {
    const uint32_t b = ord[t];
    const double cb = (double)st.cnt[b], sx2 = st.sx2[b], sv2 = st.sv2[b];
    if (sx2 > 0.0 && sv2 > 0.0) {
      const double imx = cb / sx2, imv = cb / sv2;
      const double xb = h.xs[b], yb = h.ys[b], zb = h.zs[b];
      const double vxb = h.vxs[b], vyb = h.vys[b], vzb = h.vzs[b];
      for (uint32_t pa = a0; pa < t; ++pa) {
        const uint32_t a = ord[pa];
        const double dx = min_image(xb - h.xs[a], box);
        const double dy = min_image(yb - h.ys[a], box);
        const double dz = min_image(zb - h.zs[a], box);
        const double ux = vxb - h.vxs[a], uy = vyb - h.vys[a], uz = vzb - h.vzs[a];
        const double qq = __fma_rn(sq3(dx, dy, dz), imx, sq3(ux, uy, uz) * imv);
        if (qq < q2) {
          if (kWrite) {
            cpos[w] = pa;
            cq[w] = qq;
            ++w;
          } else {
            ++c;
          }
        }
      }
    }
  }
  if (!kWrite) ccnt[t] = c;
}

// Seeds of big groups start kept; those with candidates are listed in order.
__global__ void k_merge_big_init(const uint32_t* ord, const uint32_t* head, const uint32_t* hpos,
                                 const uint32_t* seg_start, const uint32_t* nseg, uint32_t S,
                                 const uint32_t* ccnt, libhalo_halos h, uint8_t* status,
                                 uint32_t* hflag) {
  const uint32_t t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= S) return;
  const uint32_t F = nseg[0];
  const uint32_t g = hpos[t] + head[t] - 1u;
  const uint32_t a0 = seg_start[g], a1 = (g + 1 < F) ? seg_start[g + 1] : S;
  const bool big = a1 - a0 > kMergeWave;
  if (big) {
    const uint32_t b = ord[t];
    h.merged_into[b] = (int32_t)b;
    status[t] = 1;
  }
  hflag[t] = (big && ccnt[t] > 0) ? 1u : 0u;
}

__global__ void k_merge_list(const uint32_t* hflag, const uint32_t* lpos, uint32_t S,
                             uint32_t* list) {
  const uint32_t t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t < S && hflag[t]) list[lpos[t]] = t;
}

// One thread per group: its seeds with candidates, in visiting order.  A
// thread reads only statuses it wrote itself or that were set before the
// kernel.
__global__ void k_merge_resolve(const uint32_t* ord, const uint32_t* seg_start,
                                const uint32_t* nseg, uint32_t S, const uint32_t* lpos,
                                const uint32_t* list, const uint32_t* cstart,
                                const uint32_t* cpos, const double* cq, libhalo_halos h,
                                uint8_t* status) {
  const uint32_t g = blockIdx.x * blockDim.x + threadIdx.x;
  const uint32_t F = nseg[0];
  if (g >= F) return;
  const uint32_t a0 = seg_start[g], a1 = (g + 1 < F) ? seg_start[g + 1] : S;
  if (a1 - a0 <= kMergeWave) return;
  for (uint32_t e = lpos[a0]; e < lpos[a1]; ++e) {
    const uint32_t t = list[e];
    double bq = INFINITY;
    uint32_t best = 0xFFFFFFFFu;
    for (uint32_t k = cstart[t]; k < cstart[t + 1]; ++k) {
      const uint32_t pa = cpos[k];
      if (!status[pa]) continue;
      const uint32_t a = ord[pa];
      const double q = cq[k];
      if (q < bq || (q == bq && a < best)) {
        bq = q;
        best = a;
      }
    }
    if (best != 0xFFFFFFFFu) {
      h.merged_into[ord[t]] = (int32_t)best;
      status[t] = 0;
    }
  }
}

// Pairs (ancestor node, merged halo) of every leaf.
__global__ void k_pair_count(const libhalo_halos h, const libhalo_nodes nd, uint32_t S,
                             uint32_t* cnt) {
  uint32_t s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s < S) cnt[s] = (uint32_t)nd.level[h.seed_node[s]] + 1u;
}

__global__ void k_pair_emit(const libhalo_halos h, const libhalo_nodes nd, uint32_t S,
                            const uint32_t* off, unsigned long long* key, uint32_t* val) {
  uint32_t s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= S) return;
  const unsigned long long mh = (unsigned long long)(uint32_t)h.merged_into[s];
  uint32_t o = off[s];
  for (int32_t k = h.seed_node[s]; k >= 0; k = nd.parent[k]) {
    key[o] = ((unsigned long long)(uint32_t)k << 32) | mh;
    val[o] = 0;
    ++o;
  }
}

__global__ void k_uniq_flags(const unsigned long long* key, uint32_t P, uint32_t* flag) {
  uint32_t q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q < P) flag[q] = (q == 0 || key[q] != key[q - 1]) ? 1u : 0u;
}

__global__ void k_uniq_write(const unsigned long long* key, const uint32_t* flag,
                             const uint32_t* pos, uint32_t P, uint32_t* ids, uint32_t* soff) {
  uint32_t q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= P || !flag[q]) return;
  const uint32_t u = pos[q];
  const uint32_t node = (uint32_t)(key[q] >> 32);
  ids[u] = (uint32_t)key[q];
  if (q == 0 || (key[q] >> 32) != (key[q - 1] >> 32)) soff[node] = u;
}

// Own particles: deepest >= 0, keyed by node.
__global__ void k_own_flags(const int32_t* deepest, uint32_t n, uint32_t* flag) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) flag[i] = deepest[i] >= 0 ? 1u : 0u;
}

// off[k] = first position of node k in the node-sorted own list (lower bound).
__global__ void k_own_offsets(const uint32_t* okey, uint32_t M, uint32_t NN, uint32_t* off) {
  const uint32_t k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k > NN) return;
  uint32_t lo = 0, hi = M;
  while (lo < hi) {
    const uint32_t mid = (lo + hi) >> 1;
    if (okey[mid] < k)
      lo = mid + 1;
    else
      hi = mid;
  }
  off[k] = lo;
}

__device__ __forceinline__ uint32_t spread10(uint32_t v) {  // bit b -> bit 3b
  v &= 0x3FFu;
  v = (v | (v << 16)) & 0x030000FFu;
  v = (v | (v << 8)) & 0x0300F00Fu;
  v = (v | (v << 4)) & 0x030C30C3u;
  v = (v | (v << 2)) & 0x09249249u;
  return v;
}

// Own particles in compacted order with a 30-bit Morton key of the position
// relative to the node's centre, 64 cells per sigma_x over +-8 sigma_x
// (clamped): sorted by node, then by this key, the particles of a wave lie
// close together.  The order changes no result.
template <class T>
__global__ void k_own_compact(const int32_t* deepest, const uint32_t* flag, const uint32_t* pos,
                              uint32_t n, const T* x, const T* y, const T* z, double box,
                              libhalo_nodes nd, uint32_t* key, uint32_t* val) {
  uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n || !flag[i]) return;
  const uint32_t k = (uint32_t)deepest[i];
  const double sx = sqrt(nd.sx2[k]);
  const double sc = sx > 0.0 ? 64.0 / sx : 0.0;
  const double p[3] = {(double)x[i], (double)y[i], (double)z[i]};
  const double c[3] = {nd.cx[k], nd.cy[k], nd.cz[k]};
  uint32_t m = 0;
  for (int a = 0; a < 3; ++a) {
    double t = min_image(p[a] - c[a], box) * sc + 512.0;
    t = fmin(fmax(t, 0.0), 1023.0);
    m |= spread10((uint32_t)t) << a;
  }
  key[pos[i]] = m;
  val[pos[i]] = i;
}

__global__ void k_own_node_keys(const int32_t* deepest, const uint32_t* val, uint32_t m,
                                uint32_t* key) {
  const uint32_t q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q < m) key[q] = (uint32_t)deepest[val[q]];
}

__global__ void k_level_start(const int32_t* level, uint32_t NN, uint32_t* lstart) {
  uint32_t k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= NN) return;
  if (k == 0 || level[k] != level[k - 1]) lstart[level[k]] = k;
}

__global__ void k_multi_per_level(const int32_t* level, const uint32_t* soff, uint32_t NN,
                                  uint32_t* lmulti) {
  uint32_t k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= NN) return;
  if (soff[k + 1] - soff[k] >= 2) atomicAdd(lmulti + level[k], 1u);
}

__global__ void k_mark_cand(const uint32_t* soff, const uint32_t* ids, uint32_t k0, uint32_t k1,
                            uint32_t* cand) {
  uint32_t k = k0 + blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= k1) return;
  if (soff[k + 1] - soff[k] < 2) return;
  for (uint32_t q = soff[k]; q < soff[k + 1]; ++q) cand[ids[q]] = 1u;
}

// Assigned particles so far whose halo is a candidate: flag for compaction.
__global__ void k_cand_flags(const uint32_t* own, uint32_t q0, uint32_t q1,
                             const int32_t* halo_of, const uint32_t* cand, uint32_t* flag) {
  uint32_t q = q0 + blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= q1) return;
  int32_t hh = halo_of[own[q]];
  flag[q - q0] = (hh >= 0 && cand[hh]) ? 1u : 0u;
}

__global__ void k_cand_compact(const uint32_t* own, uint32_t q0, uint32_t q1,
                               const int32_t* halo_of, const uint32_t* flag,
                               const uint32_t* pos, uint32_t* seg, uint32_t* pidx) {
  uint32_t q = q0 + blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= q1 || !flag[q - q0]) return;
  uint32_t i = own[q];
  seg[pos[q - q0]] = (uint32_t)halo_of[i];
  pidx[pos[q - q0]] = i;
}

// Eq. 3 parameters of a seed, one 64-byte record: its position and velocity
// (the leaf means) and the weights of its current particles, 1/r_dyn^2 =
// cdyn / v_max^2 and 1/sigma_v^2 (floored at 1e-300).
struct __align__(16) SeedM {
  double xs, ys, zs, vxs, vys, vzs, ird, isv;
};

__global__ void k_seed_metric_init(const libhalo_halos h, uint32_t S, SeedM* sm) {
  uint32_t s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= S) return;
  sm[s].xs = h.xs[s];
  sm[s].ys = h.ys[s];
  sm[s].zs = h.zs[s];
  sm[s].vxs = h.vxs[s];
  sm[s].vys = h.vys[s];
  sm[s].vzs = h.vzs[s];
}

__global__ void k_metric_weights(const double* sv2, const double* vm2, uint32_t S, double cdyn,
                                 SeedM* sm) {
  uint32_t h = blockIdx.x * blockDim.x + threadIdx.x;
  if (h >= S) return;
  sm[h].ird = cdyn / vm2[h];
  sm[h].isv = 1.0 / fmax(sv2[h], 1e-300);
}

// Eq. 3 argmin over the seeds of the particle's node: FP64, ties to the lower
// row (the node's seed list is ascending).
__device__ __forceinline__ void eq3_min(double px, double py, double pz, double ux0, double uy0,
                                        double uz0, double box, const SeedM& m, uint32_t hid,
                                        double& bd, uint32_t& best) {
  double dx = min_image(px - m.xs, box), dy = min_image(py - m.ys, box),
         dz = min_image(pz - m.zs, box);
  double ux = ux0 - m.vxs, uy = uy0 - m.vys, uz = uz0 - m.vzs;
  double d = __fma_rn(sq3(dx, dy, dz), m.ird, sq3(ux, uy, uz) * m.isv);
  if (d < bd) {
    bd = d;
    best = hid;
  }
}

__device__ __forceinline__ double wave_min_f64(double v) {
  for (int o = 32; o > 0; o >>= 1) v = fmin(v, __shfl_xor(v, o));
  return v;
}
__device__ __forceinline__ double wave_max_f64(double v) {
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o));
  return v;
}

// Box bounds of one coordinate (the wave's interval [lo, hi], widened by w)
// against a seed's value c: the smallest and the largest distance, squared,
// added to g2 and f2.
__device__ __forceinline__ void box_axis(double c, double lo, double hi, double w, double& g2,
                                         double& f2) {
  const double l = lo - w, h = hi + w;
  const double g = fmax(0.0, fmax(l - c, c - h));
  const double f = fmax(fabs(c - l), fabs(h - c));
  g2 = __fma_rn(g, g, g2);
  f2 = __fma_rn(f, f, f2);
}

// Seeds of a node above which a wave first bounds them against its box.
constexpr uint32_t kPruneSeeds = 32;

// One thread per own particle of the level's nodes (sorted by node, then
// spatially).  When the whole wave belongs to one node its seed list and
// records are wave-uniform (scalar loads); otherwise each lane reads its own.
//
// A wave in one node with more than kPruneSeeds seeds first bounds every
// seed s against the box of its particles' positions (relative to the node's
// centre, where the node's extent, below half the box, makes the difference
// of two such offsets the minimum image) and velocities: the Eq. 3 distance
// of any of its particles to s lies between lo(s) and hi(s).  With T the
// least hi(s), a seed with lo(s) > T is farther than that seed from every
// particle of the wave and cannot be its argmin or tie with it; the others
// are evaluated exactly, in the node's order.  The box is widened by 1e-9 of
// the box side (positions) and 1e-4 km/s (velocities), far above the
// rounding of the offsets, and T by a factor 1 + 1e-9 above that of the sums,
// so the argmin is the one of the full scan bit for bit.
template <class T>
__global__ void k_assign_level(const T* x, const T* y, const T* z, const float* vx,
                               const float* vy, const float* vz, double box,
                               const uint32_t* own, const uint32_t* okey, uint32_t q0,
                               uint32_t q1, const uint32_t* __restrict__ soff,
                               const uint32_t* __restrict__ ids, const SeedM* __restrict__ sm,
                               const double* __restrict__ ncx, const double* __restrict__ ncy,
                               const double* __restrict__ ncz, int32_t* halo_of) {
  const uint32_t q = q0 + blockIdx.x * blockDim.x + threadIdx.x;
  const bool ok = q < q1;
  if (!__any(ok)) return;  // wave-uniform
  const uint32_t i = ok ? own[q] : 0u, k = ok ? okey[q] : okey[q0];
  const uint32_t kw = __builtin_amdgcn_readfirstlane(k);
  double px = 0.0, py = 0.0, pz = 0.0, ux0 = 0.0, uy0 = 0.0, uz0 = 0.0;
  if (ok) {
    px = (double)x[i];
    py = (double)y[i];
    pz = (double)z[i];
    ux0 = (double)vx[i];
    uy0 = (double)vy[i];
    uz0 = (double)vz[i];
  }
  uint32_t best;
  if (__all(k == kw)) {
    const uint32_t s0 = soff[kw], s1 = soff[kw + 1];
    best = ids[s0];
    if (s1 - s0 > kPruneSeeds) {
      // the wave's box: positions relative to the node's centre, velocities
      const double cx = ncx[kw], cy = ncy[kw], cz = ncz[kw];
      const double inf = INFINITY;
      const double rx = min_image(px - cx, box), ry = min_image(py - cy, box),
                   rz = min_image(pz - cz, box);
      const double lx = wave_min_f64(ok ? rx : inf), hx = wave_max_f64(ok ? rx : -inf);
      const double ly = wave_min_f64(ok ? ry : inf), hy = wave_max_f64(ok ? ry : -inf);
      const double lz = wave_min_f64(ok ? rz : inf), hz = wave_max_f64(ok ? rz : -inf);
      const double lu = wave_min_f64(ok ? ux0 : inf), hu = wave_max_f64(ok ? ux0 : -inf);
      const double lv = wave_min_f64(ok ? uy0 : inf), hv = wave_max_f64(ok ? uy0 : -inf);
      const double lw = wave_min_f64(ok ? uz0 : inf), hw = wave_max_f64(ok ? uz0 : -inf);
      const double wx = 1e-9 * box, wv = 1e-4;
      const uint32_t lane = threadIdx.x & 63u;
      // lane j bounds seed t = c0 + j of each run of 64
      auto bounds = [&](uint32_t t, double& lo, double& hi) {
        const SeedM m = sm[ids[t]];
        double gx = 0.0, fx = 0.0, gv = 0.0, fv = 0.0;
        box_axis(min_image(m.xs - cx, box), lx, hx, wx, gx, fx);
        box_axis(min_image(m.ys - cy, box), ly, hy, wx, gx, fx);
        box_axis(min_image(m.zs - cz, box), lz, hz, wx, gx, fx);
        box_axis(m.vxs, lu, hu, wv, gv, fv);
        box_axis(m.vys, lv, hv, wv, gv, fv);
        box_axis(m.vzs, lw, hw, wv, gv, fv);
        lo = __fma_rn(gx, m.ird, gv * m.isv);
        hi = __fma_rn(fx, m.ird, fv * m.isv);
      };
      double tl = inf;
      for (uint32_t c0 = s0; c0 < s1; c0 += 64u) {
        const uint32_t t = c0 + lane;
        if (t < s1) {
          double lo, hi;
          bounds(t, lo, hi);
          tl = fmin(tl, hi);
        }
      }
      const double lim = wave_min_f64(tl) * (1.0 + 1e-9);
      double bd = INFINITY;
      for (uint32_t c0 = s0; c0 < s1; c0 += 64u) {
        const uint32_t t = c0 + lane;
        bool keep = false;
        if (t < s1) {
          double lo, hi;
          bounds(t, lo, hi);
          keep = lo <= lim;
        }
        unsigned long long left = __ballot(keep);
        while (left) {  // wave-uniform: the surviving seeds in order
          const uint32_t j = (uint32_t)__builtin_ctzll(left);
          left &= left - 1ull;
          const uint32_t hid = ids[c0 + j];
          eq3_min(px, py, pz, ux0, uy0, uz0, box, sm[hid], hid, bd, best);
        }
      }
    } else if (s1 - s0 > 1) {
      double bd = INFINITY;
      for (uint32_t t = s0; t < s1; ++t) {
        const uint32_t hid = ids[t];
        eq3_min(px, py, pz, ux0, uy0, uz0, box, sm[hid], hid, bd, best);
      }
    }
  } else {
    const uint32_t s0 = soff[k], s1 = soff[k + 1];
    best = ids[s0];
    if (s1 - s0 > 1) {
      double bd = INFINITY;
      for (uint32_t t = s0; t < s1; ++t) {
        const uint32_t hid = ids[t];
        eq3_min(px, py, pz, ux0, uy0, uz0, box, sm[hid], hid, bd, best);
      }
    }
  }
  if (ok) halo_of[i] = (int32_t)best;
}

__global__ void k_all_assigned(const int32_t* halo_of, uint32_t n, uint32_t* flag) {
  uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) flag[i] = halo_of[i] >= 0 ? 1u : 0u;
}

__global__ void k_all_compact(const int32_t* halo_of, const uint32_t* flag, const uint32_t* pos,
                              uint32_t n, uint32_t* seg, uint32_t* pidx) {
  uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n || !flag[i]) return;
  seg[pos[i]] = (uint32_t)halo_of[i];
  pidx[pos[i]] = i;
}

__global__ void k_finish_halos(libhalo_halos h, uint32_t S, const uint32_t* start,
                               const double* sv2, const double* vm2) {
  uint32_t s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= S) return;
  h.n_assigned[s] = start[s + 1] - start[s];
  bool kept = h.merged_into[s] == (int32_t)s;
  h.sv2[s] = kept ? sv2[s] : 0.0;
  h.vmax2[s] = kept ? vm2[s] : 0.0;
}

__global__ void k_kept_flags(const libhalo_halos h, uint32_t S, uint32_t* flag) {
  uint32_t s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s < S) flag[s] = h.merged_into[s] == (int32_t)s ? 1u : 0u;
}

__global__ void k_kept_keys(const libhalo_halos h, uint32_t S, const uint32_t* flag,
                            const uint32_t* pos, unsigned long long* key, uint32_t* val) {
  uint32_t s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= S || !flag[s]) return;
  uint32_t p = pos[s];
  key[p] = ((unsigned long long)h.fof[s] << 32) |
           (unsigned long long)(0xFFFFFFFFu - h.n_assigned[s]);
  val[p] = s;
}

// Host of each halo (Section 3.4): argmin of the Eq. 3 distance over the
// halos of its FOF group with strictly more assigned particles (a prefix of
// the group in ord), in the candidate host's metric; -1 when there is none.
// One wavefront per halo, its group located by binary search.
__global__ void k_hostsub(const uint32_t* ord, const uint32_t* seg_start, const uint32_t* nseg,
                          uint32_t KH, double box, double cdyn, libhalo_halos h) {
  const uint32_t F = nseg[0];
  const int lane = threadIdx.x & 63;
  const uint32_t nw = (gridDim.x * blockDim.x) >> 6;
  for (uint32_t t = (blockIdx.x * blockDim.x + threadIdx.x) >> 6; t < KH; t += nw) {
    uint32_t lo = 0, hi = F;  // last group start <= t
    while (hi - lo > 1) {
      const uint32_t mid = (lo + hi) >> 1;
      if (seg_start[mid] <= t)
        lo = mid;
      else
        hi = mid;
    }
    const uint32_t a0 = seg_start[lo];
    if (t == a0) continue;  // the group's first halo has no host
    const uint32_t s = ord[t];
    const uint32_t ns = h.n_assigned[s];
    double bd = INFINITY;
    uint32_t best = 0xFFFFFFFFu;
    for (uint32_t u = a0 + lane; u < t; u += 64) {
      const uint32_t H = ord[u];
      if (h.n_assigned[H] <= ns) continue;
      const double ird = cdyn / h.vmax2[H];
      const double isv = 1.0 / fmax(h.sv2[H], 1e-300);
      double dx = min_image(h.xs[s] - h.xs[H], box), dy = min_image(h.ys[s] - h.ys[H], box),
             dz = min_image(h.zs[s] - h.zs[H], box);
      double ux = h.vxs[s] - h.vxs[H], uy = h.vys[s] - h.vys[H], uz = h.vzs[s] - h.vzs[H];
      double d = __fma_rn(sq3(dx, dy, dz), ird, sq3(ux, uy, uz) * isv);
      if (d < bd || (d == bd && H < best)) {
        bd = d;
        best = H;
      }
    }
    for (int o = 32; o > 0; o >>= 1) {
      double od = __shfl_xor(bd, o);
      uint32_t ob = __shfl_xor(best, o);
      if (od < bd || (od == bd && ob < best)) {
        bd = od;
        best = ob;
      }
    }
    if (lane == 0) h.host[s] = (int32_t)best;
  }
}

__global__ void k_copy_one(const uint32_t* a, uint32_t* b) { *b = *a; }

__global__ void k_fill_i32(int32_t* a, int64_t n, int32_t v) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) a[i] = v;
}

template <class T>
void assign_impl(Ctx& ctx, int64_t n, int pos_dtype, const T* x, const T* y, const T* z,
                 const float* vx, const float* vy, const float* vz, const libhalo_nodes& nd,
                 int64_t NN, const int32_t* deepest, libhalo_halos& h, int32_t* halo_of,
                 int64_t* n_halos, hipStream_t s) {
  const libhalo_params& P = ctx.p;
  const double box = P.box;
  const double cdyn = (4.0 * M_PI / 3.0) * P.G * P.rho_vir;
  const double Gm = P.G * P.particle_mass;
  const double eps2 = P.softening * P.softening;
  uint32_t* hb = ctx.host_slot<uint32_t>(0);
  auto readu = [&](const uint32_t* d, int slot) {
    HALO_HIP(hipMemcpyAsync(hb + slot, d, 4, hipMemcpyDeviceToHost, s));
    HALO_HIP(hipStreamSynchronize(s));
    return hb[slot];
  };
  *n_halos = 0;
  if (NN == 0) {
    k_fill_i32<<<blocks_for(n, TB), TB, 0, s>>>(halo_of, n, -1);
    HALO_HIP(hipStreamSynchronize(s));
    return;
  }
  // sizes known before any work: node count, deepest level, particle count
  int32_t maxlev = 0;
  HALO_HIP(hipMemcpyAsync(&maxlev, nd.level + NN - 1, 4, hipMemcpyDeviceToHost, s));
  HALO_HIP(hipStreamSynchronize(s));
  const int nlev = maxlev + 1;
  const int64_t NPmax = NN * (int64_t)nlev;  // (ancestor, leaf) pairs
  struct W {
    uint32_t *flag, *pos, *dcnt, *stmp, *cnt, *seg_start, *kept, *pcnt, *poff;
    int32_t* node_seed;
    double *sx2, *sv2, *cur_sv2, *cur_vm2;
    SeedM* sm;
    unsigned long long *k64a, *k64b, *pk0, *pk1, *vm;
    uint32_t *va, *vb, *pv0, *pv1, *pflag, *ppos, *soff, *ids, *ocnt, *iflag, *ipos;
    uint32_t *ok0, *ov0, *ok1, *ov1, *ooff, *lstart, *lmulti, *cand, *na;
    uint32_t *mc_cnt, *mc_start, *mc_flag, *mc_lpos, *mc_list, *mc_pos;
    double* mc_q;
    uint8_t* mc_status;
    int64_t mc_cap;
    void *rtmp, *rtmp2;
    I128* acc;
    RadialBufs rb;
  } w;
  carve_workspace(ctx, [&](Arena& A) {
    const int64_t K2 = NN + 2;
    w.flag = A.take<uint32_t>(K2);
    w.pos = A.take<uint32_t>(K2);
    w.node_seed = A.take<int32_t>(K2);
    w.dcnt = A.take<uint32_t>(16);
    w.stmp = A.take<uint32_t>(scan_tmp_elems<uint32_t>(std::max<int64_t>(n, NPmax) + 2));
    w.cnt = A.take<uint32_t>(K2);
    w.sx2 = A.take<double>(K2);
    w.sv2 = A.take<double>(K2);
    w.k64a = A.take<unsigned long long>(K2);
    w.k64b = A.take<unsigned long long>(K2);
    w.va = A.take<uint32_t>(K2);
    w.vb = A.take<uint32_t>(K2);
    w.seg_start = A.take<uint32_t>(K2);
    w.kept = A.take<uint32_t>(K2);
    w.mc_cnt = A.take<uint32_t>(K2);
    w.mc_start = A.take<uint32_t>(K2 + 1);
    w.mc_flag = A.take<uint32_t>(K2);
    w.mc_lpos = A.take<uint32_t>(K2 + 1);
    w.mc_list = A.take<uint32_t>(K2);
    w.mc_status = A.take<uint8_t>(K2);
    w.mc_cap = 8 * K2 + 4096;  // candidate pairs; more falls back to the visit
    w.mc_pos = A.take<uint32_t>(w.mc_cap);
    w.mc_q = A.take<double>(w.mc_cap);
    w.rtmp = A.take<char>(radix_tmp_bytes(std::max<int64_t>(NPmax, 1)));
    w.pcnt = A.take<uint32_t>(K2);
    w.poff = A.take<uint32_t>(K2);
    w.pk0 = A.take<unsigned long long>(NPmax + 2);
    w.pk1 = A.take<unsigned long long>(NPmax + 2);
    w.pv0 = A.take<uint32_t>(NPmax + 2);
    w.pv1 = A.take<uint32_t>(NPmax + 2);
    w.pflag = A.take<uint32_t>(NPmax + 2);
    w.ppos = A.take<uint32_t>(NPmax + 2);
    w.soff = A.take<uint32_t>(K2);
    w.ids = A.take<uint32_t>(NPmax + 2);
    w.ocnt = A.take<uint32_t>(K2);
    w.iflag = A.take<uint32_t>(n + 2);
    w.ipos = A.take<uint32_t>(n + 2);
    w.ok0 = A.take<uint32_t>(n + 2);
    w.ov0 = A.take<uint32_t>(n + 2);
    w.ok1 = A.take<uint32_t>(n + 2);
    w.ov1 = A.take<uint32_t>(n + 2);
    w.rtmp2 = A.take<char>(radix_tmp_bytes(n));
    w.ooff = A.take<uint32_t>(K2);
    w.lstart = A.take<uint32_t>(nlev + 2);
    w.lmulti = A.take<uint32_t>(nlev + 2);
    w.cand = A.take<uint32_t>(K2);
    w.cur_sv2 = A.take<double>(K2);
    w.cur_vm2 = A.take<double>(K2);
    w.sm = A.take<SeedM>(K2);
    w.acc = A.take<I128>(4 * K2);
    w.vm = A.take<unsigned long long>(K2);
    w.na = A.take<uint32_t>(K2);
    w.rb = radial_take(A, n, K2);
  });
  // outputs are written only once the workspace is in place
  k_fill_i32<<<blocks_for(n, TB), TB, 0, s>>>(halo_of, n, -1);
  uint32_t *flag = w.flag, *pos = w.pos, *dcnt = w.dcnt, *stmp = w.stmp;
  int32_t* node_seed = w.node_seed;
  k_leaf_flags<<<blocks_for(NN, TB), TB, 0, s>>>(nd.n_children, (uint32_t)NN, flag);
  exclusive_scan<uint32_t>(flag, pos, NN, dcnt, stmp, s);
  const uint32_t S = readu(dcnt, 0);
  *n_halos = S;
  HALO_CHECK((int64_t)S <= h.cap, LIBHALO_ECAPACITY, "halo table too small");
  SeedT st{w.cnt, w.sx2, w.sv2};
  k_seeds<<<blocks_for(NN, TB), TB, 0, s>>>(nd, (uint32_t)NN, flag, pos, h, st, node_seed);

  // ---- merging
  unsigned long long *k64a = w.k64a, *k64b = w.k64b;
  uint32_t *va = w.va, *vb = w.vb, *seg_start = w.seg_start, *kept = w.kept;
  void* rtmp = w.rtmp;
  k_group_size_keys<<<blocks_for(S, TB), TB, 0, s>>>(h.fof, st.cnt, S, k64a, va);
  bool f = radix_sort_pairs<unsigned long long>(k64a, va, k64b, vb, S, 64, rtmp, s);
  unsigned long long* skey = f ? k64b : k64a;
  uint32_t* ord = f ? vb : va;
  k_fof_heads<<<blocks_for(S, TB), TB, 0, s>>>(skey, S, flag);
  exclusive_scan<uint32_t>(flag, pos, S, dcnt + 1, stmp, s);
  k_fof_segments<<<blocks_for(S, TB), TB, 0, s>>>(flag, pos, S, seg_start);
  const uint32_t F = readu(dcnt + 1, 1);
  k_merge<<<blocks_for((int64_t)F * 64, TB), TB, 0, s>>>(ord, seg_start, dcnt + 1, S, box,
                                                         P.merge_q2, h, st, kept);
  {
    // big groups: candidate lists in parallel, then an in-order resolution
    k_merge_cand<false><<<blocks_for(S, TB), TB, 0, s>>>(ord, flag, pos, seg_start, dcnt + 1, S,
                                                         box, P.merge_q2, h, st, w.mc_cnt,
                                                         nullptr, nullptr, nullptr);
    exclusive_scan<uint32_t>(w.mc_cnt, w.mc_start, S, w.mc_start + S, stmp, s);
    const uint32_t NC = readu(w.mc_start + S, 8);
    if ((int64_t)NC <= w.mc_cap) {
      k_merge_cand<true><<<blocks_for(S, TB), TB, 0, s>>>(ord, flag, pos, seg_start, dcnt + 1,
                                                          S, box, P.merge_q2, h, st, nullptr,
                                                          w.mc_start, w.mc_pos, w.mc_q);
      k_merge_big_init<<<blocks_for(S, TB), TB, 0, s>>>(ord, flag, pos, seg_start, dcnt + 1, S,
                                                        w.mc_cnt, h, w.mc_status, w.mc_flag);
      exclusive_scan<uint32_t>(w.mc_flag, w.mc_lpos, S, w.mc_lpos + S, stmp, s);
      k_merge_list<<<blocks_for(S, TB), TB, 0, s>>>(w.mc_flag, w.mc_lpos, S, w.mc_list);
      k_merge_resolve<<<blocks_for(F, TB), TB, 0, s>>>(ord, seg_start, dcnt + 1, S, w.mc_lpos,
                                                       w.mc_list, w.mc_start, w.mc_pos,
                                                       w.mc_q, h, w.mc_status);
    } else {
      k_merge_big<<<std::min<int64_t>(blocks_for(F, kMergeTB), 256), kMergeTB, 0, s>>>(
          ord, seg_start, dcnt + 1, S, box, P.merge_q2, h, st, kept);
    }
  }

  // ---- seed sets per node
  uint32_t *pcnt = w.pcnt, *poff = w.poff;
  k_pair_count<<<blocks_for(S, TB), TB, 0, s>>>(h, nd, S, pcnt);
  exclusive_scan<uint32_t>(pcnt, poff, S, poff + S, stmp, s);
  const uint32_t NP = readu(poff + S, 2);
  HALO_CHECK((int64_t)NP <= NPmax, LIBHALO_EINVAL, "seed-set pairs exceed their bound");
  unsigned long long *pk0 = w.pk0, *pk1 = w.pk1;
  uint32_t *pv0 = w.pv0, *pv1 = w.pv1, *pflag = w.pflag, *ppos = w.ppos;
  k_pair_emit<<<blocks_for(S, TB), TB, 0, s>>>(h, nd, S, poff, pk0, pv0);
  bool fp = radix_sort_pairs<unsigned long long>(pk0, pv0, pk1, pv1, NP,
                                                 32 + bits_for((uint64_t)NN), rtmp, s);
  unsigned long long* psk = fp ? pk1 : pk0;
  k_uniq_flags<<<blocks_for(NP, TB), TB, 0, s>>>(psk, NP, pflag);
  exclusive_scan<uint32_t>(pflag, ppos, NP, dcnt + 2, stmp, s);
  uint32_t *soff = w.soff, *ids = w.ids;
  k_uniq_write<<<blocks_for(NP, TB), TB, 0, s>>>(psk, pflag, ppos, NP, ids, soff);
  k_copy_one<<<1, 1, 0, s>>>(dcnt + 2, soff + NN);

  // ---- own particles per node, sorted by node then index
  uint32_t *ocnt = w.ocnt, *iflag = w.iflag, *ipos = w.ipos;
  uint32_t *ok0 = w.ok0, *ov0 = w.ov0, *ok1 = w.ok1, *ov1 = w.ov1;
  void* rtmp2 = w.rtmp2;
  k_own_flags<<<blocks_for(n, TB), TB, 0, s>>>(deepest, (uint32_t)n, iflag);
  exclusive_scan<uint32_t>(iflag, ipos, n, dcnt + 3, stmp, s);
  k_own_compact<T><<<blocks_for(n, TB), TB, 0, s>>>(deepest, iflag, ipos, (uint32_t)n, x, y, z,
                                                    box, nd, ok0, ov0);
  const uint32_t M = readu(dcnt + 3, 4);
  // by the spatial key, then stably by node
  const bool f1 = radix_sort_pairs<uint32_t>(ok0, ov0, ok1, ov1, M, 30, rtmp2, s);
  uint32_t* vsp = f1 ? ov1 : ov0;  // values in key order
  uint32_t* kfree = f1 ? ok0 : ok1;
  uint32_t* kold = f1 ? ok1 : ok0;
  uint32_t* vfree = f1 ? ov0 : ov1;
  k_own_node_keys<<<blocks_for(M, TB), TB, 0, s>>>(deepest, vsp, M, kfree);
  const bool fo =
      radix_sort_pairs<uint32_t>(kfree, vsp, kold, vfree, M, bits_for((uint64_t)NN), rtmp2, s);
  uint32_t* okey = fo ? kold : kfree;
  uint32_t* own = fo ? vfree : vsp;
  uint32_t* ooff = w.ooff;
  k_own_offsets<<<blocks_for(NN + 1, TB), TB, 0, s>>>(okey, M, (uint32_t)NN, ooff);

  // ---- levels
  uint32_t *lstart = w.lstart, *lmulti = w.lmulti;
  k_level_start<<<blocks_for(NN, TB), TB, 0, s>>>(nd.level, (uint32_t)NN, lstart);
  k_fill_u32<<<1, 64, 0, s>>>(lmulti, nlev + 1, 0u);
  k_multi_per_level<<<blocks_for(NN, TB), TB, 0, s>>>(nd.level, soff, (uint32_t)NN, lmulti);
  std::vector<uint32_t> hls(nlev + 1), hlm(nlev + 1), hoo(NN + 1);
  HALO_HIP(hipMemcpyAsync(hls.data(), lstart, 4ull * nlev, hipMemcpyDeviceToHost, s));
  HALO_HIP(hipMemcpyAsync(hlm.data(), lmulti, 4ull * nlev, hipMemcpyDeviceToHost, s));
  HALO_HIP(hipMemcpyAsync(hoo.data(), ooff, 4ull * (NN + 1), hipMemcpyDeviceToHost, s));
  HALO_HIP(hipStreamSynchronize(s));
  hls[nlev] = (uint32_t)NN;

  uint32_t *cand = w.cand, *na = w.na;
  double *cur_sv2 = w.cur_sv2, *cur_vm2 = w.cur_vm2;
  I128* acc = w.acc;
  unsigned long long* vm = w.vm;
  RadialBufs& rb = w.rb;
  k_seed_metric_init<<<blocks_for(S, TB), TB, 0, s>>>(h, S, w.sm);
  for (int lev = maxlev; lev >= 0; --lev) {
    const uint32_t k0 = hls[lev], k1 = hls[lev + 1];
    const uint32_t q0 = hoo[k0], q1 = hoo[k1];  // own particles of this level
    if (hlm[lev] > 0) {
      k_fill_u32<<<blocks_for(S, TB), TB, 0, s>>>(cand, S, 0u);
      k_mark_cand<<<blocks_for(k1 - k0, TB), TB, 0, s>>>(soff, ids, k0, k1, cand);
      // particles assigned so far: own particles of deeper levels
      const uint32_t a0 = q1, a1 = hoo[NN];
      uint32_t m = 0;
      if (a1 > a0) {
        k_cand_flags<<<blocks_for(a1 - a0, TB), TB, 0, s>>>(own, a0, a1, halo_of, cand, iflag);
        exclusive_scan<uint32_t>(iflag, ipos, a1 - a0, dcnt + 4, stmp, s);
        k_cand_compact<<<blocks_for(a1 - a0, TB), TB, 0, s>>>(own, a0, a1, halo_of, iflag,
                                                              ipos, rb.seg, rb.pidx);
        m = readu(dcnt + 4, 5);
      }
      radial_sort(pos_dtype, x, y, z, box, h.xs, h.ys, h.zs, m, S, rb, s);
      radial_sigma_vmax(vx, vy, vz, m, S, rb, Gm, eps2, acc, vm, cur_sv2, cur_vm2, s);
      k_metric_weights<<<blocks_for(S, TB), TB, 0, s>>>(cur_sv2, cur_vm2, S, cdyn, w.sm);
    }
    if (q1 > q0)
      HALO_PROF(ctx, "k_assign_level", s,
                (k_assign_level<T><<<blocks_for(q1 - q0, TB), TB, 0, s>>>(
                    x, y, z, vx, vy, vz, box, own, okey, q0, q1, soff, ids, w.sm, nd.cx, nd.cy,
                    nd.cz, halo_of)));
  }

  // ---- final metric of every halo from all its particles
  k_all_assigned<<<blocks_for(n, TB), TB, 0, s>>>(halo_of, (uint32_t)n, iflag);
  exclusive_scan<uint32_t>(iflag, ipos, n, dcnt + 5, stmp, s);
  k_all_compact<<<blocks_for(n, TB), TB, 0, s>>>(halo_of, iflag, ipos, (uint32_t)n, rb.seg,
                                                 rb.pidx);
  const uint32_t MA = readu(dcnt + 5, 6);
  radial_sort(pos_dtype, x, y, z, box, h.xs, h.ys, h.zs, MA, S, rb, s);
  radial_sigma_vmax(vx, vy, vz, MA, S, rb, Gm, eps2, acc, vm, cur_sv2, cur_vm2, s);
  k_finish_halos<<<blocks_for(S, TB), TB, 0, s>>>(h, S, rb.start, cur_sv2, cur_vm2);

  // ---- host/sub relation
  k_kept_flags<<<blocks_for(S, TB), TB, 0, s>>>(h, S, flag);
  exclusive_scan<uint32_t>(flag, pos, S, dcnt + 6, stmp, s);
  k_kept_keys<<<blocks_for(S, TB), TB, 0, s>>>(h, S, flag, pos, k64a, va);
  const uint32_t KH = readu(dcnt + 6, 7);
  bool fk = radix_sort_pairs<unsigned long long>(k64a, va, k64b, vb, KH, 64, rtmp, s);
  unsigned long long* kk = fk ? k64b : k64a;
  uint32_t* kord = fk ? vb : va;
  k_fof_heads<<<blocks_for(KH, TB), TB, 0, s>>>(kk, KH, flag);
  exclusive_scan<uint32_t>(flag, pos, KH, dcnt + 7, stmp, s);
  k_fof_segments<<<blocks_for(KH, TB), TB, 0, s>>>(flag, pos, KH, seg_start);
  const uint32_t FH = readu(dcnt + 7, 8);
  k_hostsub<<<blocks_for((int64_t)KH * 64, TB), TB, 0, s>>>(kord, seg_start, dcnt + 7, KH, box,
                                                             cdyn, h);
  HALO_HIP(hipStreamSynchronize(s));
}

}  // namespace

void assign(Ctx& ctx, int64_t n, int pos_dtype, const void* x, const void* y, const void* z,
            const float* vx, const float* vy, const float* vz, const libhalo_nodes* nodes,
            int64_t n_nodes, const int32_t* deepest, libhalo_halos* halos, int32_t* halo_of,
            int64_t* n_halos, hipStream_t s) {
  if (pos_dtype == LIBHALO_F64)
    assign_impl<double>(ctx, n, pos_dtype, (const double*)x, (const double*)y,
                        (const double*)z, vx, vy, vz, *nodes, n_nodes, deepest, *halos,
                        halo_of, n_halos, s);
  else
    assign_impl<float>(ctx, n, pos_dtype, (const float*)x, (const float*)y, (const float*)z,
                       vx, vy, vz, *nodes, n_nodes, deepest, *halos, halo_of, n_halos, s);
}

}  // namespace halo
