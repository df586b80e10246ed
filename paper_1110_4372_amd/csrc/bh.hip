// Tree potential for the largest haloes on gfx950 (Appendix B of the paper:
// a binary space-partitioning tree whose cells are accepted as monopoles
// beyond the Salmon-Warren distance).
//
// Per halo the particles of S(h) are sorted along a 48-bit Morton curve over
// their bounding box, and a binary tree is built over that order (mtree.hpp):
// a cell holding more than kLeaf particles splits where the highest differing
// Morton bit of its particles changes, so each child is one cell of the curve
// (an octree cell, shrunk to its particles).  A cell's mass centre x0, its
// dispersion sigma^2 about x0 and r_max (the largest distance of its
// particles from x0, found by a pass over the particles) give the acceptance
// distance d >= r_max / 2 + sqrt((r_max / 2)^2 + sigma^2 / theta), beyond
// which the monopole's relative error is at most theta.  The cells are stored
// in depth-first preorder with the index after each subtree, and one
// wavefront per 64 Morton-consecutive particles walks them in order: a cell
// acceptable for every target lane adds m / sqrt(d^2 + eps^2) to each and is
// skipped, a leaf that is not adds its particles one by one, any other cell
// is entered.  The walk needs no stack.  Each lane sums in the wave's fixed
// order, so the result does not depend on scheduling.
#include <algorithm>
#include <cmath>
#include <type_traits>
#include <vector>

#include "bh.hpp"
#include "mtree.hpp"
#include "primitives.hpp"

namespace halo {

namespace {

constexpr int TB = 256;
constexpr uint32_t kLeaf = 16;     // default: a cell of at most this many particles is a leaf
constexpr uint32_t kMaxDepth = 64; // cells at this depth are leaves whatever their size
constexpr int kFrac = 32;  // fractional bits of the potential accumulators

__device__ __forceinline__ uint32_t seg_find(const uint32_t* off, uint32_t K, uint32_t w) {
  uint32_t lo = 0, hi = K;
  while (hi - lo > 1) {
    const uint32_t mid = (lo + hi) >> 1;
    if (off[mid] <= w)
      lo = mid;
    else
      hi = mid;
  }
  return lo;
}

// round(v 2^frac), 0 <= v 2^frac < 2^94, as a 128-bit integer.
__device__ __forceinline__ I128 fixed128(double v, int frac) {
  const double s = rint(ldexp(v, frac));
  const double hi = floor(s * 0x1p-64);
  const double lo = __fma_rn(-hi, 0x1p64, s);
  const double l1 = floor(lo * 0x1p-32);
  const double l0 = __fma_rn(-l1, 0x1p32, lo);
  I128 r;
  r.lo = ((unsigned long long)(uint32_t)l1 << 32) | (uint32_t)l0;
  r.hi = (long long)hi;
  return r;
}

// A coordinate of up to 21 bits spread to every third bit (bit i -> bit 3i).
__host__ __device__ __forceinline__ unsigned long long spread3(uint32_t v) {
  unsigned long long x = v & 0x1FFFFFull;
  x = (x | (x << 32)) & 0x001F00000000FFFFull;
  x = (x | (x << 16)) & 0x001F0000FF0000FFull;
  x = (x | (x << 8)) & 0x100F00F00F00F00Full;
  x = (x | (x << 4)) & 0x10C30C30C30C30C3ull;
  x = (x | (x << 2)) & 0x1249249249249249ull;
  return x;
}

__global__ void k_bh_flags(const libhalo_halos h, uint32_t S, const uint32_t* nS, double theta,
                           uint32_t bh_min, uint32_t* flag) {
  const uint32_t s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= S) return;
  flag[s] = bh_takes(h.merged_into[s] == (int32_t)s, h.n_assigned[s], nS[s], theta, bh_min)
                ? 1u : 0u;
}

struct BhList {
  uint32_t *big, *nel, *nown, *eoff;
};

__global__ void k_bh_list(const uint32_t* flag, const uint32_t* pos, uint32_t S,
                          const libhalo_halos h, const uint32_t* nS, BhList L) {
  const uint32_t s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= S || !flag[s]) return;
  const uint32_t b = pos[s];
  L.big[b] = s;
  L.nel[b] = nS[s];
  L.nown[b] = h.n_assigned[s];
}

__global__ void k_bh_bbox_init(unsigned long long* bb, uint32_t B) {
  const uint32_t b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= B) return;
  for (int c = 0; c < 3; ++c) {
    bb[6 * (size_t)b + c] = 0xFFFFFFFFFFFFFFFFull;  // min
    bb[6 * (size_t)b + 3 + c] = 0ull;                // max
  }
}

// Bounding box per halo as ordered-integer min / max.  A wave takes a tile of
// kBoxTile consecutive elements (coalesced, 64 apart per lane); a tile inside
// one halo sends one set of atomics, a tile across a halo boundary (at most
// two per halo) sends each element's own.
constexpr uint32_t kBoxTile = 1024;

__global__ void k_bh_bbox(const double* ux, const double* uy, const double* uz, BhList L,
                          const uint32_t* slot, uint32_t B, uint32_t E,
                          unsigned long long* bb) {
  const uint32_t lane = threadIdx.x & 63u;
  const uint32_t t0 = (blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6)) * kBoxTile;
  if (t0 >= E) return;  // wave-uniform
  const uint32_t t1 = min(t0 + kBoxTile, E);
  const uint32_t b0 = seg_find(L.eoff, B, t0), b1 = seg_find(L.eoff, B, t1 - 1u);
  if (b0 == b1) {
    const uint32_t q0 = slot[L.big[b0]] + (t0 - L.eoff[b0]);
    unsigned long long mn[3] = {~0ull, ~0ull, ~0ull}, mx[3] = {0ull, 0ull, 0ull};
    for (uint32_t e = t0 + lane; e < t1; e += 64u) {
      const uint32_t q = q0 + (e - t0);
      const unsigned long long v[3] = {f64_ord(ux[q]), f64_ord(uy[q]), f64_ord(uz[q])};
      for (int c = 0; c < 3; ++c) {
        mn[c] = v[c] < mn[c] ? v[c] : mn[c];
        mx[c] = v[c] > mx[c] ? v[c] : mx[c];
      }
    }
    for (int o = 32; o > 0; o >>= 1)
      for (int c = 0; c < 3; ++c) {
        const unsigned long long a = __shfl_xor(mn[c], o), z = __shfl_xor(mx[c], o);
        mn[c] = a < mn[c] ? a : mn[c];
        mx[c] = z > mx[c] ? z : mx[c];
      }
    if (lane == 0)
      for (int c = 0; c < 3; ++c) {
        atomicMin(bb + 6 * (size_t)b0 + c, mn[c]);
        atomicMax(bb + 6 * (size_t)b0 + 3 + c, mx[c]);
      }
  } else {
    for (uint32_t e = t0 + lane; e < t1; e += 64u) {
      const uint32_t b = seg_find(L.eoff, B, e);
      const uint32_t q = slot[L.big[b]] + (e - L.eoff[b]);
      const double p[3] = {ux[q], uy[q], uz[q]};
      for (int c = 0; c < 3; ++c) {
        atomicMin(bb + 6 * (size_t)b + c, f64_ord(p[c]));
        atomicMax(bb + 6 * (size_t)b + 3 + c, f64_ord(p[c]));
      }
    }
  }
}

__global__ void k_bh_keys(const double* ux, const double* uy, const double* uz, BhList L,
                          const uint32_t* slot, uint32_t B, uint32_t E,
                          const unsigned long long* bb, unsigned long long* key,
                          uint32_t* val) {
  const uint32_t e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= E) return;
  const uint32_t b = seg_find(L.eoff, B, e);
  const uint32_t q = slot[L.big[b]] + (e - L.eoff[b]);
  const double p[3] = {ux[q], uy[q], uz[q]};
  double ext = 0.0, lo[3];
  for (int c = 0; c < 3; ++c) {
    lo[c] = ord_f64(bb[6 * (size_t)b + c]);
    ext = fmax(ext, ord_f64(bb[6 * (size_t)b + 3 + c]) - lo[c]);
  }
  const double scale = ext > 0.0 ? 65535.0 / ext : 0.0;
  unsigned long long m = 0ull;
  for (int c = 0; c < 3; ++c) {
    double u = floor((p[c] - lo[c]) * scale);
    u = u < 0.0 ? 0.0 : (u > 65535.0 ? 65535.0 : u);
    m |= spread3((uint32_t)u) << c;
  }
  key[e] = ((unsigned long long)b << 48) | m;
  val[e] = q;
}

// Sorted positions (FP64); with f non-null also their FP32 roundings, which
// the mixed form's walk reads, 16 bytes per particle (x, y, z, 0) so that a
// leaf's particles are whole scalar loads.
__global__ void k_bh_gather(const double* ux, const double* uy, const double* uz,
                            const uint32_t* sval, uint32_t E, double* px, double* py,
                            double* pz, float* f) {
  const uint32_t e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= E) return;
  const uint32_t q = sval[e];
  const double x = ux[q], y = uy[q], z = uz[q];
  px[e] = x;
  py[e] = y;
  pz[e] = z;
  if (f) {
    f[4ull * e] = (float)x;
    f[4ull * e + 1] = (float)y;
    f[4ull * e + 2] = (float)z;
    f[4ull * e + 3] = 0.0f;
  }
}

// A cell as the walk reads it (one 64-byte scalar fetch), in preorder: mass
// centre, mass (particles), dispersion, squared acceptance distance, its range
// of the sorted order, the index after its subtree, and whether it is a leaf.
// Once the acceptance distance is set, the mixed form's walk takes the centre
// rounded to FP32 and the squared acceptance distance rounded down to FP32
// from the 16 bytes of the dispersion and that distance: for an FP32 squared
// distance d, d <= crit2 exactly when d <= crit2 rounded down.
struct __align__(16) BhRec {
  double cx, cy, cz, cm;
  union {
    struct {
      double sig2, crit2;
    } d;
    struct {
      float cx, cy, cz, crit2;
    } f;
  } a;
  uint32_t lo, hi, skip, leaf;
};

// The lanes l of a wave whose element e0 + l lies in [lo, hi) (32-bit
// arithmetic on wave-uniform values, so it stays on the scalar unit).
__device__ __forceinline__ unsigned long long lane_span(uint32_t lo, uint32_t hi, uint32_t e0) {
  // element indices stay below 2^31, so the differences fit a signed int
  const int32_t a = max((int32_t)(lo - e0), 0);
  const int32_t b = min(max((int32_t)(hi - e0), 0), 64);
  if (a >= b) return 0ull;
  const unsigned long long upto = b == 64 ? ~0ull : ((1ull << b) - 1ull);
  return upto & ~((1ull << a) - 1ull);
}

// Cell statistics of the nodes [u0, u0 + nu) of one depth: leaves from their
// particles, others from their children's records (one depth deeper, already
// written); r_max follows from a pass over the particles.
__global__ void k_bh_records(const MtNode* bnode, const uint32_t* pre, uint32_t u0, uint32_t nu,
                             const double* px, const double* py, const double* pz, BhRec* R) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nu) return;
  const MtNode u = bnode[u0 + i];
  const uint32_t p = pre[u0 + i];
  double x0[3], m, s2;
  if (u.left == kMtNone) {
    double sx = 0.0, sy = 0.0, sz = 0.0;
    for (uint32_t e = u.lo; e < u.hi; ++e) {
      sx += px[e];
      sy += py[e];
      sz += pz[e];
    }
    m = (double)(u.hi - u.lo);
    x0[0] = sx / m;
    x0[1] = sy / m;
    x0[2] = sz / m;
    s2 = 0.0;
    for (uint32_t e = u.lo; e < u.hi; ++e)
      s2 += sq3(px[e] - x0[0], py[e] - x0[1], pz[e] - x0[2]);
    s2 /= m;
  } else {
    const BhRec& a = R[pre[u.left]];
    const BhRec& b = R[pre[u.left + 1]];
    const double m1 = a.cm, m2 = b.cm;
    m = m1 + m2;
    x0[0] = (m1 * a.cx + m2 * b.cx) / m;
    x0[1] = (m1 * a.cy + m2 * b.cy) / m;
    x0[2] = (m1 * a.cz + m2 * b.cz) / m;
    const double d1 = sq3(a.cx - x0[0], a.cy - x0[1], a.cz - x0[2]);
    const double d2 = sq3(b.cx - x0[0], b.cy - x0[1], b.cz - x0[2]);
    s2 = (m1 * (a.a.d.sig2 + d1) + m2 * (b.a.d.sig2 + d2)) / m;
  }
  BhRec r;
  r.cx = x0[0];
  r.cy = x0[1];
  r.cz = x0[2];
  r.cm = m;
  r.a.d.sig2 = s2;
  r.a.d.crit2 = 0.0;
  r.lo = u.lo;
  r.hi = u.hi;
  r.skip = p + u.aux;
  r.leaf = u.left == kMtNone ? 1u : 0u;
  R[p] = r;
}

// Exact r_max of every cell in one launch: each particle starts at the root of
// its halo's tree (roots are 0 .. B-1, level order) and follows its cell down
// to its leaf, one depth per iteration; at each depth the particles of a wave,
// whose cells form runs along the sorted order, reduce each run to one atomic
// maximum (ordered integers) of the squared distance to the cell's centre.
// sqrt is monotone, so the root of the largest square is the largest
// distance, taken once per cell in k_bh_crit.
__global__ void k_bh_rmax(BhList L, uint32_t B, uint32_t E, const double* px, const double* py,
                          const double* pz, const MtNode* bnode, const uint32_t* pre,
                          const BhRec* R, unsigned long long* rmx) {
  const uint32_t e = blockIdx.x * blockDim.x + threadIdx.x;
  const uint32_t lane = threadIdx.x & 63u;
  uint32_t u = e < E ? seg_find(L.eoff, B, e) : kMtNone;
  const double x = e < E ? px[e] : 0.0, y = e < E ? py[e] : 0.0, z = e < E ? pz[e] : 0.0;
  while (__any(u != kMtNone)) {
    unsigned long long v = 0ull;
    uint32_t p = kMtNone;
    if (u != kMtNone) {
      p = pre[u];
      v = f64_ord(sq3(x - R[p].cx, y - R[p].cy, z - R[p].cz));
    }
    // maximum over the rest of this lane's run (runs of equal cells are
    // contiguous): lane i ends with the maximum over [i, end of its run]
    for (uint32_t o = 1; o < 64u; o <<= 1) {
      const unsigned long long vo = __shfl_down(v, o);
      const uint32_t po = __shfl_down(p, o);
      if (lane + o < 64u && po == p && vo > v) v = vo;
    }
    const uint32_t pp = __shfl_up(p, 1);
    // the maximum only grows: a run below the value already there sends no atomic
    if (p != kMtNone && (lane == 0u || pp != p) && v > __atomic_load_n(rmx + p, __ATOMIC_RELAXED))
      atomicMax(rmx + p, v);
    if (u != kMtNone) {
      const MtNode n = bnode[u];
      u = n.left == kMtNone ? kMtNone : (e < bnode[n.left].hi ? n.left : n.left + 1u);
    }
  }
}

// Acceptance distances from the exact r_max.
__global__ void k_bh_crit(uint32_t T, double theta, const unsigned long long* rmx, int f32,
                          BhRec* R) {
  const uint32_t t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= T) return;
  const double r = sqrt(ord_f64(rmx[t]));  // r_max from the largest squared distance
  const double dc = 0.5 * r + sqrt(0.25 * r * r + R[t].a.d.sig2 / theta);
  if (f32) {
    BhRec& c = R[t];
    c.a.f.cx = (float)c.cx;
    c.a.f.cy = (float)c.cy;
    c.a.f.cz = (float)c.cz;
    c.a.f.crit2 = __double2float_rd(dc * dc);
  } else {
    R[t].a.d.crit2 = dc * dc;
  }
}

// Wave units of each tree halo: its sorted elements in runs of 64.
__global__ void k_bh_wave_counts(BhList L, uint32_t B, uint32_t* wcnt) {
  const uint32_t b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= B) return;
  wcnt[b] = (L.nel[b] + 63u) / 64u;
}

// The walk, one wavefront per 64 consecutive sorted elements of one halo
// (spatially close along the curve); lanes holding an own particle are the
// targets, the others only ride along.  The wave reads the halo's cells in
// preorder: a cell acceptable for every target lane (it lies beyond the
// acceptance distance and does not hold the target) is taken as a monopole and
// skipped, a leaf that is not is searched particle by particle, any other cell
// is entered (its first child is the next record).  Cell records and
// leaf particles are read at wave-uniform addresses (scalar loads), and each
// lane sums its terms in the wave's fixed order.
//
// F32 (the mixed form): distances and reciprocal square roots in FP32 from the
// halo-local positions rounded to FP32 (their rounding, about 1e-7 of a halo's
// extent, is far below the monopole error the acceptance distance allows); a
// leaf's terms are summed in FP32, the target's own term subtracted once
// afterwards instead of masked per term, and each leaf's and monopole's sum is
// added to the lane's FP64 total.
template <bool F32, bool COUNT>
__global__ void __launch_bounds__(TB)
    k_bh_walk(BhList L, uint32_t B, const uint32_t* woff, uint32_t nwave, const uint32_t* slot,
              const double* __restrict__ px, const double* __restrict__ py,
              const double* __restrict__ pz, const float* __restrict__ pf,
              const uint32_t* __restrict__ pidx, const BhRec* __restrict__ R,
              const uint32_t* __restrict__ troot, double eps2, I128* __restrict__ pacc,
              unsigned long long* work) {
  // blocks go to the eight XCDs in turn (block b to XCD b mod 8): the blocks
  // of one XCD take a contiguous eighth of the waves, so the waves sharing an
  // L2 walk neighbouring targets and read the same cells (a bijection; the
  // last gridDim mod 8 blocks keep their own index)
  const uint32_t g8 = gridDim.x >> 3;
  const uint32_t blk = blockIdx.x < 8u * g8 ? (blockIdx.x & 7u) * g8 + (blockIdx.x >> 3)
                                            : blockIdx.x;
  const uint32_t wave = __builtin_amdgcn_readfirstlane(blk * (TB / 64) + (threadIdx.x >> 6));
  if (wave >= nwave) return;  // wave-uniform
  const uint32_t lane = threadIdx.x & 63u;
  const uint32_t b = __builtin_amdgcn_readfirstlane(seg_find(woff, B, wave));
  const uint32_t n = L.nel[b], base = L.eoff[b];
  const uint32_t s0 = slot[L.big[b]], nown = L.nown[b];
  const uint32_t e = base + (wave - woff[b]) * 64u + lane;
  const bool in = e < base + n;
  const uint32_t q = in ? pidx[e] : 0xFFFFFFFFu;
  const bool target = in && (q - s0) < nown;
  if (__ballot(target) == 0ull) return;  // wave-uniform
  const double x = in ? px[e] : 0.0, y = in ? py[e] : 0.0, z = in ? pz[e] : 0.0;
  const float xf = (float)x, yf = (float)y, zf = (float)z, eps2f = (float)eps2;
  // the wave's first element and its target lanes: the lanes a cell holds
  // follow from its range alone
  const uint32_t e0 = __builtin_amdgcn_readfirstlane(base + (wave - woff[b]) * 64u);
  const unsigned long long tmask = __ballot(target);
  // the F32 leaf sum's term of the target itself (the same expression at d = 0)
  const float self_f = __builtin_amdgcn_rsqf(
      __fmaf_rn(0.0f, 0.0f, __fmaf_rn(0.0f, 0.0f, __fmaf_rn(0.0f, 0.0f, eps2f))));
  uint32_t u = __builtin_amdgcn_readfirstlane(troot[b]);
  const uint32_t end = __builtin_amdgcn_readfirstlane(troot[b + 1]);
  double acc = 0.0;
  uint32_t ncell = 0, nterm = 0;  // work counts (profiling), the same in every lane
  // the next record is read while this one is processed: entering a cell (the
  // next record) is the common step; a skip reads its target afresh
  BhRec c = R[u];
  while (u < end) {
    const BhRec nx = R[u + 1];
    uint32_t v;
    double d2 = 0.0;
    float d2f = 0.0f;
    bool near;
    if constexpr (F32) {
      const float dx = xf - c.a.f.cx, dy = yf - c.a.f.cy, dz = zf - c.a.f.cz;
      d2f = __fmaf_rn(dz, dz, __fmaf_rn(dy, dy, dx * dx));
      near = d2f <= c.a.f.crit2;
    } else {
      d2 = sq3(x - c.cx, y - c.cy, z - c.cz);
      near = d2 <= c.a.d.crit2;
    }
    // a cell is a monopole for a target outside it beyond the acceptance
    // distance; the cell holding the target itself is always opened (a cell of
    // coincident particles has a zero acceptance distance)
    const unsigned long long inside = lane_span(c.lo, c.hi, e0);
    if (COUNT) ++ncell;
    if (((__builtin_amdgcn_ballot_w64(near) | inside) & tmask) == 0ull) {
      if (COUNT) ++nterm;
      // every lane adds the monopole; lanes without a target discard their sums
      if constexpr (F32)
        acc += c.cm * (double)__builtin_amdgcn_rsqf(d2f + eps2f);
      else
        acc += c.cm * rsqrt_f64(d2 + eps2);
      v = c.skip;
    } else if (c.leaf) {
      if (COUNT) nterm += c.hi - c.lo;
      // every lane evaluates each term and keeps it by a select, so the loads of a
      // leaf particle are not behind a branch and several can be in flight at once
      if constexpr (F32) {
        // every term is summed, the target's own (distance zero: the softening
        // alone) included, and that one is taken back after the leaf; lanes
        // without a target discard their sums
        float sf = 0.0f;
#pragma unroll 4
        for (uint32_t f = c.lo; f < c.hi; ++f) {
          const float4 p4 = reinterpret_cast<const float4*>(pf)[f];
          const float fx = p4.x, fy = p4.y, fz = p4.z;
          const float dx = xf - fx, dy = yf - fy, dz = zf - fz;
          sf += __builtin_amdgcn_rsqf(
              __fmaf_rn(dz, dz, __fmaf_rn(dy, dy, __fmaf_rn(dx, dx, eps2f))));
        }
        if ((inside >> lane) & 1ull) sf -= self_f;
        acc += (double)sf;
      } else {
#pragma unroll 4
        for (uint32_t f = c.lo; f < c.hi; ++f) {
          const double fx = px[f], fy = py[f], fz = pz[f];
          const uint32_t qf = pidx[f];
          const double tf = rsqrt_f64(sq3(x - fx, y - fy, z - fz) + eps2);
          acc = (target && qf != q) ? acc + tf : acc;
        }
      }
      v = c.skip;
    } else {
      v = u + 1u;
    }
    if (v == u + 1u)
      c = nx;
    else if (v < end)
      c = R[v];
    u = v;
  }
  if (target && acc > 0.0) atomic_add_i128(pacc + q, fixed128(acc, kFrac));
  if (COUNT) {  // per target particle: cells tested, terms added
    const unsigned long long nt = (unsigned long long)__popcll(__ballot(target));
    if (lane == 0) {  // the waves spread their adds over kBhSlots lines
      unsigned long long* w = work + 8u * (wave % (uint32_t)kBhSlots);
      atomicAdd(w, nt * ncell);
      atomicAdd(w + 1, nt * nterm);
    }
  }
}

// The step workspace past the unbinding's own carve is idle while the tree runs:
// the tree takes it when it fits and its own workspace only when it does not.
template <class F>
void carve2(Ctx& ctx, F&& carve) {
  Arena dry;
  dry.counting = true;
  carve(dry);
  const size_t need = dry.off + 4096;
  const size_t start = (ctx.ws.off + 255) & ~size_t(255);
  if (ctx.ws.base && start <= ctx.ws.cap && need <= ctx.ws.cap - start) {
    Arena tail;
    tail.base = ctx.ws.base + start;
    tail.cap = ctx.ws.cap - start;
    carve(tail);
    return;
  }
  ctx.ensure_ws2(need);
  ctx.ws2.reset();
  carve(ctx.ws2);
}

}  // namespace

void bh_potential(Ctx& ctx, const libhalo_halos& h, uint32_t S, const uint32_t* nS,
                  const uint32_t* slot, const double* ux, const double* uy, const double* uz,
                  double eps2, double theta, uint32_t bh_min, I128* pacc, hipStream_t s) {
  uint32_t* hb = ctx.host_slot<uint32_t>(4);
  struct W {
    uint32_t *flag, *pos, *cnt, *stmp;
    BhList L;
    unsigned long long* bb;
  } w;
  auto take_list = [&](Arena& A) {
    w.flag = A.take<uint32_t>(S + 2);
    w.pos = A.take<uint32_t>(S + 2);
    w.cnt = A.take<uint32_t>(16);
    w.stmp = A.take<uint32_t>(scan_tmp_elems<uint32_t>(S + 2));
    w.L.big = A.take<uint32_t>(S + 2);
    w.L.nel = A.take<uint32_t>(S + 2);
    w.L.nown = A.take<uint32_t>(S + 2);
    w.L.eoff = A.take<uint32_t>(S + 2);
    w.bb = A.take<unsigned long long>(6ull * (S + 2));
  };
  auto build_list = [&]() {
    k_bh_flags<<<blocks_for(S, TB), TB, 0, s>>>(h, S, nS, theta, bh_min, w.flag);
    exclusive_scan<uint32_t>(w.flag, w.pos, S, w.cnt, w.stmp, s);
    k_bh_list<<<blocks_for(S, TB), TB, 0, s>>>(w.flag, w.pos, S, h, nS, w.L);
  };
  carve2(ctx, take_list);
  build_list();
  HALO_HIP(hipMemcpyAsync(hb, w.cnt, 4, hipMemcpyDeviceToHost, s));
  HALO_HIP(hipStreamSynchronize(s));
  const uint32_t B = hb[0];
  if (B == 0) return;
  HALO_CHECK(B < 65536u, LIBHALO_EINVAL, "more than 65535 haloes take the tree (raise bh_min)");
  exclusive_scan<uint32_t>(w.L.nel, w.L.eoff, B, w.cnt + 1, w.stmp, s);
  std::vector<uint32_t> nel(B);
  HALO_HIP(hipMemcpyAsync(hb + 1, w.cnt + 1, 4, hipMemcpyDeviceToHost, s));
  HALO_HIP(hipMemcpyAsync(nel.data(), w.L.nel, 4ull * B, hipMemcpyDeviceToHost, s));
  HALO_HIP(hipStreamSynchronize(s));
  unsigned long long E64 = 0;
  for (uint32_t b = 0; b < B; ++b) E64 += nel[b];
  HALO_CHECK(E64 < 0x7FFFFFFFull, LIBHALO_EINVAL,
             "tree elements exceed 31-bit indices (raise bh_min)");
  const uint32_t E = hb[1];
  // cells: leaves of at most L particles use about 3.2 / L cells per particle; the
  // capacity bounds memory, not results (a cell without room for its children
  // stays a leaf)
  const uint32_t leaf = ctx.p.bh_leaf > 0 ? (uint32_t)ctx.p.bh_leaf : kLeaf;
  const uint32_t cap = (uint32_t)((4ull * E) / leaf) + B + 64;
  // second carve with the element and cell arrays; the list is rebuilt in it
  unsigned long long *k0, *k1, *rmx;
  uint32_t *v0, *v1;
  double* pz;
  BhRec* R;
  float* pf;  // FP32 sorted positions (mixed form)
  const bool f32 = ctx.p.prec == LIBHALO_PREC_MIXED;
  MTree t;
  void* rtmp;
  carve2(ctx, [&](Arena& A) {
    take_list(A);
    k0 = A.take<unsigned long long>(E + 1);
    k1 = A.take<unsigned long long>(E + 1);
    v0 = A.take<uint32_t>(E + 1);
    v1 = A.take<uint32_t>(E + 1);
    pz = A.take<double>(E + 1);
    mtree_take(A, t, cap, B + 1);
    R = A.take<BhRec>(cap + 1);  // the walk reads one record ahead
    pf = f32 ? A.take<float>(4ull * (E + 1)) : nullptr;
    rmx = A.take<unsigned long long>(cap);
    rtmp = A.take<char>(radix_tmp_bytes(E + 1));
  });
  build_list();
  exclusive_scan<uint32_t>(w.L.nel, w.L.eoff, B, w.cnt + 1, w.stmp, s);
  k_bh_bbox_init<<<blocks_for(B, TB), TB, 0, s>>>(w.bb, B);
  k_bh_bbox<<<blocks_for((E + kBoxTile - 1) / kBoxTile, TB / 64), TB, 0, s>>>(ux, uy, uz, w.L,
                                                                               slot, B, E, w.bb);
  k_bh_keys<<<blocks_for(E, TB), TB, 0, s>>>(ux, uy, uz, w.L, slot, B, E, w.bb, k0, v0);
  const bool f = radix_sort_pairs<unsigned long long>(k0, v0, k1, v1, E,
                                                      48 + bits_for(B > 1 ? B - 1 : 1), rtmp, s);
  const uint32_t* pidx = f ? v1 : v0;
  // the cells over each halo's sorted range; the sorted keys are read by the build
  // only, so afterwards x and y of the sorted positions take their place
  mtree_build(t, f ? k1 : k0, w.L.eoff, w.L.nel, B, leaf, kMaxDepth, hb + 2, s);
  double* px = reinterpret_cast<double*>(k0);
  double* py = reinterpret_cast<double*>(k1);
  k_bh_gather<<<blocks_for(E, TB), TB, 0, s>>>(ux, uy, uz, pidx, E, px, py, pz, pf);
  const uint32_t T = t.NN;
  for (int d = (int)t.lev.size() - 2; d >= 0; --d) {
    const uint32_t nu = t.lev[d + 1] - t.lev[d];
    k_bh_records<<<blocks_for(nu, TB), TB, 0, s>>>(t.bnode, t.pre, t.lev[d], nu, px, py, pz, R);
  }
  // exact r_max, then the acceptance distances
  k_fill_u64<<<blocks_for(T, TB), TB, 0, s>>>(rmx, T, 0ull);
  k_bh_rmax<<<blocks_for(E, TB), TB, 0, s>>>(w.L, B, E, px, py, pz, t.bnode, t.pre, R, rmx);
  k_bh_crit<<<blocks_for(T, TB), TB, 0, s>>>(T, theta, rmx, f32 ? 1 : 0, R);
  // wave units: runs of 64 sorted elements within each halo
  k_bh_wave_counts<<<blocks_for(B, TB), TB, 0, s>>>(w.L, B, w.flag);
  exclusive_scan<uint32_t>(w.flag, w.pos, B, w.cnt + 3, w.stmp, s);
  HALO_HIP(hipMemcpyAsync(hb + 4, w.cnt + 3, 4, hipMemcpyDeviceToHost, s));
  HALO_HIP(hipStreamSynchronize(s));
  const uint32_t nwave = hb[4];
  const unsigned wg = blocks_for((int64_t)nwave * 64, TB);
  unsigned long long* work = ctx.count ? ctx.bh_counters() : nullptr;
  auto walk = [&](auto f32c, auto countc) {
    k_bh_walk<decltype(f32c)::value, decltype(countc)::value><<<wg, TB, 0, s>>>(
        w.L, B, w.pos, nwave, slot, px, py, pz, f32 ? pf : nullptr, pidx, R, t.troot, eps2,
        pacc, work);
  };
  using T1 = std::true_type;
  using F0 = std::false_type;
  HALO_PROF(ctx, "k_bh_walk", s,
            f32 ? (work ? walk(T1{}, T1{}) : walk(T1{}, F0{}))
                : (work ? walk(F0{}, T1{}) : walk(F0{}, F0{})));
  HALO_HIP(hipStreamSynchronize(s));
}

}  // namespace halo
