// Tree potential for the largest haloes on gfx950 (Appendix B of the paper:
// a binary space-partitioning tree whose cells are accepted as monopoles
// beyond the Salmon-Warren distance).
//
// Per halo the particles of S(h) are sorted along a 48-bit Morton curve over
// their bounding box, and the tree is implicit over that order: heap node k
// at level l covers the sorted range [floor(i n / 2^l), floor((i+1) n / 2^l))
// with i = k - 2^l, down to leaves of at most 17 particles.  A cell's mass
// centre x0, its dispersion sigma^2 about x0 and r_max (the largest distance
// of its particles from x0, found by a pass over the particles) give the
// acceptance distance d >= r_max / 2 + sqrt((r_max / 2)^2 + sigma^2 / theta),
// beyond which the monopole's relative error is at most theta.  One wavefront
// per 64 Morton-consecutive particles walks the tree depth first: a cell
// acceptable for every target lane adds m / sqrt(d^2 + eps^2) to each, any
// other cell is opened for all, and opened leaves add their particles one by
// one.  Each lane sums in the wave's fixed order, so the result does not
// depend on scheduling.
#include <algorithm>
#include <cmath>
#include <vector>

#include "bh.hpp"
#include "primitives.hpp"

namespace halo {

namespace {

constexpr int TB = 256;
constexpr uint32_t kLeaf = 16;
constexpr int kStack = 64;
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

__host__ __device__ __forceinline__ uint32_t depth_for(uint32_t n) {
  uint32_t d = 0;
  while ((n >> d) > kLeaf) ++d;
  return d;
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
  uint32_t *big, *nel, *nnode, *depth, *nown, *eoff, *noff;
};

__global__ void k_bh_list(const uint32_t* flag, const uint32_t* pos, uint32_t S,
                          const libhalo_halos h, const uint32_t* nS, BhList L) {
  const uint32_t s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= S || !flag[s]) return;
  const uint32_t b = pos[s];
  const uint32_t n = nS[s];
  const uint32_t d = depth_for(n);
  L.big[b] = s;
  L.nel[b] = n;
  L.depth[b] = d;
  L.nnode[b] = 2u << d;
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

// Bounding box per halo as ordered-integer min / max; a wave whose elements
// all belong to one halo sends one set of atomics.
__global__ void k_bh_bbox(const double* ux, const double* uy, const double* uz, BhList L,
                          const uint32_t* slot, uint32_t B, uint32_t E,
                          unsigned long long* bb) {
  const uint32_t e = blockIdx.x * blockDim.x + threadIdx.x;
  const bool ok = e < E;
  uint32_t b = 0xFFFFFFFFu;
  unsigned long long mn[3] = {~0ull, ~0ull, ~0ull}, mx[3] = {0ull, 0ull, 0ull};
  if (ok) {
    b = seg_find(L.eoff, B, e);
    const uint32_t q = slot[L.big[b]] + (e - L.eoff[b]);
    const double p[3] = {ux[q], uy[q], uz[q]};
    for (int c = 0; c < 3; ++c) mn[c] = mx[c] = f64_ord(p[c]);
  }
  const uint32_t b0 = __shfl(b, 0);
  if (__all(b == b0) && b0 != 0xFFFFFFFFu) {
    for (int o = 32; o > 0; o >>= 1)
      for (int c = 0; c < 3; ++c) {
        const unsigned long long a = __shfl_xor(mn[c], o), z = __shfl_xor(mx[c], o);
        mn[c] = a < mn[c] ? a : mn[c];
        mx[c] = z > mx[c] ? z : mx[c];
      }
    if ((threadIdx.x & 63u) == 0)
      for (int c = 0; c < 3; ++c) {
        atomicMin(bb + 6 * (size_t)b0 + c, mn[c]);
        atomicMax(bb + 6 * (size_t)b0 + 3 + c, mx[c]);
      }
  } else if (ok) {
    for (int c = 0; c < 3; ++c) {
      atomicMin(bb + 6 * (size_t)b + c, mn[c]);
      atomicMax(bb + 6 * (size_t)b + 3 + c, mx[c]);
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

__global__ void k_bh_gather(const double* ux, const double* uy, const double* uz,
                            const uint32_t* sval, uint32_t E, double* px, double* py,
                            double* pz) {
  const uint32_t e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= E) return;
  const uint32_t q = sval[e];
  px[e] = ux[q];
  py[e] = uy[q];
  pz[e] = uz[q];
}

// Node records, one 64-byte line per node: the walk reads a node's centre,
// mass and acceptance distance in one scalar fetch.
struct BhNodes {
  double* r;
  __device__ __forceinline__ double& cx(uint32_t g) const { return r[8ull * g + 0]; }
  __device__ __forceinline__ double& cy(uint32_t g) const { return r[8ull * g + 1]; }
  __device__ __forceinline__ double& cz(uint32_t g) const { return r[8ull * g + 2]; }
  __device__ __forceinline__ double& cm(uint32_t g) const { return r[8ull * g + 3]; }
  __device__ __forceinline__ double& crit2(uint32_t g) const { return r[8ull * g + 4]; }
  __device__ __forceinline__ double& sig2(uint32_t g) const { return r[8ull * g + 5]; }
  __device__ __forceinline__ double& rmax(uint32_t g) const { return r[8ull * g + 6]; }
  // exact r_max as an ordered integer, raised by atomicMax
  __device__ __forceinline__ unsigned long long* rmx(uint32_t g) const {
    return reinterpret_cast<unsigned long long*>(r + 8ull * g + 7);
  }
};

__device__ __forceinline__ void node_range(uint32_t k, uint32_t n, uint32_t& lo, uint32_t& hi) {
  const uint32_t l = 31u - (uint32_t)__builtin_clz(k);
  const unsigned long long i = (unsigned long long)(k - (1u << l));
  lo = (uint32_t)((i * n) >> l);
  hi = (uint32_t)(((i + 1ull) * n) >> l);
}

// Cell statistics of every node at `level` (leaves directly, others from
// their children, which the previous launch filled).
__global__ void k_bh_level(BhList L, uint32_t B, uint32_t T, uint32_t level, double theta,
                           const double* px, const double* py, const double* pz, BhNodes N) {
  const uint32_t t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= T) return;
  const uint32_t b = seg_find(L.noff, B, t);
  const uint32_t k = t - L.noff[b];
  if (k == 0) return;
  const uint32_t l = 31u - (uint32_t)__builtin_clz(k);
  const uint32_t D = L.depth[b];
  if (l != level || l > D) return;
  double x0[3], m, s2, r;
  if (l == D) {
    uint32_t lo, hi;
    node_range(k, L.nel[b], lo, hi);
    const uint32_t base = L.eoff[b];
    double sx = 0.0, sy = 0.0, sz = 0.0;
    for (uint32_t e = base + lo; e < base + hi; ++e) {
      sx += px[e];
      sy += py[e];
      sz += pz[e];
    }
    m = (double)(hi - lo);
    x0[0] = sx / m;
    x0[1] = sy / m;
    x0[2] = sz / m;
    s2 = 0.0;
    r = 0.0;
    for (uint32_t e = base + lo; e < base + hi; ++e) {
      const double d2 = sq3(px[e] - x0[0], py[e] - x0[1], pz[e] - x0[2]);
      s2 += d2;
      r = fmax(r, d2);
    }
    s2 /= m;
    r = sqrt(r);
  } else {
    const uint32_t g1 = L.noff[b] + 2u * k, g2 = g1 + 1u;
    const double m1 = N.cm(g1), m2 = N.cm(g2);
    m = m1 + m2;
    x0[0] = (m1 * N.cx(g1) + m2 * N.cx(g2)) / m;
    x0[1] = (m1 * N.cy(g1) + m2 * N.cy(g2)) / m;
    x0[2] = (m1 * N.cz(g1) + m2 * N.cz(g2)) / m;
    const double d1 = sq3(N.cx(g1) - x0[0], N.cy(g1) - x0[1], N.cz(g1) - x0[2]);
    const double d2 = sq3(N.cx(g2) - x0[0], N.cy(g2) - x0[1], N.cz(g2) - x0[2]);
    s2 = (m1 * (N.sig2(g1) + d1) + m2 * (N.sig2(g2) + d2)) / m;
    r = fmax(sqrt(d1) + N.rmax(g1), sqrt(d2) + N.rmax(g2));
  }
  const uint32_t g = t;
  N.cx(g) = x0[0];
  N.cy(g) = x0[1];
  N.cz(g) = x0[2];
  N.cm(g) = m;
  N.sig2(g) = s2;
  N.rmax(g) = r;
  const double dc = 0.5 * r + sqrt(0.25 * r * r + s2 / theta);
  N.crit2(g) = dc * dc;
}

// Node of level l holding sorted position p of a halo of n particles: the i
// with floor(i n / 2^l) <= p < floor((i + 1) n / 2^l).
__device__ __forceinline__ uint32_t node_at(uint32_t p, uint32_t n, uint32_t l) {
  unsigned long long i = (((unsigned long long)p) << l) / n;
  while (((i + 1ull) * n >> l) <= p) ++i;
  while (i > 0 && ((i * n) >> l) > p) --i;
  return (1u << l) + (uint32_t)i;
}

// Exact r_max of every cell: each particle raises the maximum of its cell on
// every level (as ordered integers; a wave whose particles share a cell sends
// one atomic for it).
__global__ void k_bh_rmax_init(BhNodes N, uint32_t T) {
  const uint32_t t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t < T) *N.rmx(t) = 0ull;
}

__global__ void k_bh_rmax(BhList L, uint32_t B, uint32_t E, const double* px, const double* py,
                          const double* pz, BhNodes N) {
  const uint32_t e = blockIdx.x * blockDim.x + threadIdx.x;
  const bool ok = e < E;
  const uint32_t b = ok ? seg_find(L.eoff, B, e) : 0u;
  const uint32_t D = ok ? L.depth[b] : 0u;
  // every lane runs the same number of levels (the wave maximum) for the
  // wave-wide exchanges; lanes past their own depth or range stay idle
  uint32_t Dm = D;
  for (int o = 32; o > 0; o >>= 1) Dm = max(Dm, (uint32_t)__shfl_xor((int)Dm, o));
  for (uint32_t l = 0; l <= Dm; ++l) {
    const bool act = ok && l <= D;
    uint32_t g = 0xFFFFFFFFu;
    unsigned long long v = 0ull;
    if (act) {
      const uint32_t k = node_at(e - L.eoff[b], L.nel[b], l);
      g = L.noff[b] + k;
      v = f64_ord(sqrt(sq3(px[e] - N.cx(g), py[e] - N.cy(g), pz[e] - N.cz(g))));
    }
    const uint32_t g0 = __shfl(g, 0);
    if (__all(g == g0) && g0 != 0xFFFFFFFFu) {
      for (int o = 32; o > 0; o >>= 1) {
        const unsigned long long w2 = __shfl_xor(v, o);
        v = w2 > v ? w2 : v;
      }
      if ((threadIdx.x & 63u) == 0) atomicMax(N.rmx(g0), v);
    } else if (act) {
      atomicMax(N.rmx(g), v);
    }
  }
}

// Acceptance distances from the exact r_max.
__global__ void k_bh_crit(uint32_t T, double theta, BhNodes N) {
  const uint32_t t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= T || *N.rmx(t) == 0ull) return;  // index 0 of each heap is unused
  const double r = ord_f64(*N.rmx(t));
  N.rmax(t) = r;
  const double dc = 0.5 * r + sqrt(0.25 * r * r + N.sig2(t) / theta);
  N.crit2(t) = dc * dc;
}

// Wave units of each tree halo: its sorted elements in runs of 64.
__global__ void k_bh_wave_counts(BhList L, uint32_t B, uint32_t* wcnt) {
  const uint32_t b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= B) return;
  wcnt[b] = (L.nel[b] + 63u) / 64u;
}

// The walk, one wavefront per 64 consecutive sorted elements of one halo
// (spatially close along the curve); lanes holding an own particle are the
// targets, the others only ride along.  The wave walks one tree: a cell is
// taken as a monopole when it is acceptable for every target lane, else it
// is opened for all (which only makes the others more exact).  Node data are
// wave-uniform (scalar loads), the stack is the wave's own in LDS, and each lane sums
// its terms in the wave's fixed order.
__global__ void __launch_bounds__(TB)
    k_bh_walk(BhList L, uint32_t B, const uint32_t* woff, uint32_t nwave, const uint32_t* slot,
              const double* __restrict__ px, const double* __restrict__ py,
              const double* __restrict__ pz, const uint32_t* __restrict__ pidx,
              const double* __restrict__ nrec, double eps2, I128* __restrict__ pacc,
              uint32_t* __restrict__ err) {
  // read-only inputs that no pointer of the kernel writes: wave-uniform reads of
  // them can take the scalar data cache
  const BhNodes N{const_cast<double*>(nrec)};
  __shared__ uint32_t wstack[TB / 64][kStack];
  const uint32_t wave = __builtin_amdgcn_readfirstlane(blockIdx.x * (TB / 64) +
                                                       (threadIdx.x >> 6));
  if (wave >= nwave) return;  // wave-uniform
  const uint32_t lane = threadIdx.x & 63u;
  const uint32_t b = __builtin_amdgcn_readfirstlane(seg_find(woff, B, wave));
  const uint32_t n = L.nel[b], D = L.depth[b], nb = L.noff[b], base = L.eoff[b];
  const uint32_t s0 = slot[L.big[b]], nown = L.nown[b];
  const uint32_t e = base + (wave - woff[b]) * 64u + lane;
  const bool in = e < base + n;
  const uint32_t q = in ? pidx[e] : 0xFFFFFFFFu;
  const bool target = in && (q - s0) < nown;
  if (__ballot(target) == 0ull) return;  // wave-uniform
  const double x = in ? px[e] : 0.0, y = in ? py[e] : 0.0, z = in ? pz[e] : 0.0;
  uint32_t* stack = wstack[threadIdx.x >> 6];  // the wave's own LDS stack
  // Depth-first, left child first: an opened cell goes on to its left child at
  // once and leaves only the right one on the stack (at most one entry per level).
  int sp = 0;
  uint32_t k = 1u;
  double acc = 0.0;
  for (;;) {
    const uint32_t g = nb + k;
    const double cx = N.cx(g), cy = N.cy(g), cz = N.cz(g), cm = N.cm(g), c2 = N.crit2(g);
    const double d2 = sq3(x - cx, y - cy, z - cz);
    const uint32_t l = 31u - (uint32_t)__builtin_clz(k);
    if (__ballot(target && d2 < c2) == 0ull) {
      if (target) acc += cm * rsqrt_f64(d2 + eps2);
    } else if (l == D) {
      uint32_t lo, hi;
      node_range(k, n, lo, hi);
      // every lane evaluates each term and keeps it by a select, so the loads of a
      // leaf particle are not behind a branch and several can be in flight at once
#pragma unroll 4
      for (uint32_t f = base + lo; f < base + hi; ++f) {
        const double fx = px[f], fy = py[f], fz = pz[f];
        const uint32_t qf = pidx[f];
        const double tf = rsqrt_f64(sq3(x - fx, y - fy, z - fz) + eps2);
        acc = (target && qf != q) ? acc + tf : acc;
      }
    } else {
      if (sp + 1 > kStack) {  // cannot happen for depth <= 31; reported, not faulted
        if (lane == 0) atomicOr(err, 1u);
        break;
      }
      stack[sp++] = 2u * k + 1u;
      k = 2u * k;
      continue;
    }
    if (sp == 0) break;
    k = __builtin_amdgcn_readfirstlane(stack[--sp]);
  }
  if (target && acc > 0.0) atomic_add_i128(pacc + q, fixed128(acc, kFrac));
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
    w.L.nnode = A.take<uint32_t>(S + 2);
    w.L.depth = A.take<uint32_t>(S + 2);
    w.L.nown = A.take<uint32_t>(S + 2);
    w.L.eoff = A.take<uint32_t>(S + 2);
    w.L.noff = A.take<uint32_t>(S + 2);
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
  exclusive_scan<uint32_t>(w.L.nnode, w.L.noff, B, w.cnt + 2, w.stmp, s);
  std::vector<uint32_t> dep(B), nel(B);
  HALO_HIP(hipMemcpyAsync(hb + 1, w.cnt + 1, 8, hipMemcpyDeviceToHost, s));
  HALO_HIP(hipMemcpyAsync(dep.data(), w.L.depth, 4ull * B, hipMemcpyDeviceToHost, s));
  HALO_HIP(hipMemcpyAsync(nel.data(), w.L.nel, 4ull * B, hipMemcpyDeviceToHost, s));
  HALO_HIP(hipStreamSynchronize(s));
  uint32_t Dmax = 0;
  unsigned long long E64 = 0, T64 = 0;
  for (uint32_t b = 0; b < B; ++b) {
    Dmax = std::max(Dmax, dep[b]);
    E64 += nel[b];
    T64 += 2ull << dep[b];
  }
  HALO_CHECK(E64 < 0xFFFFFFFFull && T64 < 0xFFFFFFFFull, LIBHALO_EINVAL,
             "tree elements exceed 32-bit indices (raise bh_min)");
  const uint32_t E = hb[1], T = hb[2];
  HALO_CHECK(Dmax <= 31u, LIBHALO_EINVAL, "tree deeper than 31 levels");
  // second carve with the element and node arrays; the list is rebuilt in it
  unsigned long long *k0, *k1;
  uint32_t *v0, *v1;
  double* pz;
  BhNodes N;
  void* rtmp;
  carve2(ctx, [&](Arena& A) {
    take_list(A);
    k0 = A.take<unsigned long long>(E + 1);
    k1 = A.take<unsigned long long>(E + 1);
    v0 = A.take<uint32_t>(E + 1);
    v1 = A.take<uint32_t>(E + 1);
    pz = A.take<double>(E + 1);
    N.r = A.take<double>(8ull * (T + 1));
    rtmp = A.take<char>(radix_tmp_bytes(E + 1));
  });
  build_list();
  exclusive_scan<uint32_t>(w.L.nel, w.L.eoff, B, w.cnt + 1, w.stmp, s);
  exclusive_scan<uint32_t>(w.L.nnode, w.L.noff, B, w.cnt + 2, w.stmp, s);
  k_bh_bbox_init<<<blocks_for(B, TB), TB, 0, s>>>(w.bb, B);
  k_bh_bbox<<<blocks_for(E, TB), TB, 0, s>>>(ux, uy, uz, w.L, slot, B, E, w.bb);
  k_bh_keys<<<blocks_for(E, TB), TB, 0, s>>>(ux, uy, uz, w.L, slot, B, E, w.bb, k0, v0);
  const bool f = radix_sort_pairs<unsigned long long>(k0, v0, k1, v1, E,
                                                      48 + bits_for(B > 1 ? B - 1 : 1), rtmp, s);
  // after the sort the keys are dead: x and y of the sorted positions take their place, and
  // the sorted values are the particle slots
  const uint32_t* pidx = f ? v1 : v0;
  double* px = reinterpret_cast<double*>(k0);
  double* py = reinterpret_cast<double*>(k1);
  k_bh_gather<<<blocks_for(E, TB), TB, 0, s>>>(ux, uy, uz, pidx, E, px, py, pz);
  for (int l = (int)Dmax; l >= 0; --l)
    k_bh_level<<<blocks_for(T, TB), TB, 0, s>>>(w.L, B, T, (uint32_t)l, theta, px, py, pz, N);
  // exact r_max in place of the children's bound: a tighter acceptance distance
  k_bh_rmax_init<<<blocks_for(T, TB), TB, 0, s>>>(N, T);
  k_bh_rmax<<<blocks_for(E, TB), TB, 0, s>>>(w.L, B, E, px, py, pz, N);
  k_bh_crit<<<blocks_for(T, TB), TB, 0, s>>>(T, theta, N);
  // wave units: runs of 64 sorted elements within each halo
  k_bh_wave_counts<<<blocks_for(B, TB), TB, 0, s>>>(w.L, B, w.flag);
  exclusive_scan<uint32_t>(w.flag, w.pos, B, w.cnt + 3, w.stmp, s);
  HALO_HIP(hipMemcpyAsync(hb + 4, w.cnt + 3, 4, hipMemcpyDeviceToHost, s));
  HALO_HIP(hipMemsetAsync(w.cnt + 8, 0, 4, s));
  HALO_HIP(hipStreamSynchronize(s));
  const uint32_t nwave = hb[4];
  HALO_PROF(ctx, "k_bh_walk", s,
            k_bh_walk<<<blocks_for((int64_t)nwave * 64, TB), TB, 0, s>>>(
                w.L, B, w.pos, nwave, slot, px, py, pz, pidx, N.r, eps2, pacc, w.cnt + 8));
  HALO_HIP(hipMemcpyAsync(hb + 3, w.cnt + 8, 4, hipMemcpyDeviceToHost, s));
  HALO_HIP(hipStreamSynchronize(s));
  HALO_CHECK(hb[3] == 0, LIBHALO_EINVAL, "tree walk stack exhausted");
}

}  // namespace halo
