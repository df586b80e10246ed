// Single-pass unbinding (Section 3.5.3) with an exact direct-sum potential in
// place of the paper's tree code (Appendix B), on gfx950.
//
// Layout: the kept halos of each FOF group are laid out in depth-first
// preorder of the host/subhalo forest, each halo's own particles in input
// order, so S(h) -- the halo with all its subhaloes -- is one contiguous range
// [slot_h, slot_h + |S(h)|) and its own particles are the range's head.
// Coordinates are unwrapped once about the FOF group's anchor particle, so
// pair separations need no minimum image (groups span less than L/2).
//
// Potential: one work item = 256 own particles of a halo; the block streams
// the halo's S(h) through LDS in tiles and each thread sums its particle's
// terms in a fixed order.  FP64 form: FP64 terms 1/sqrt(r^2 + eps^2).  Mixed
// form: FP32 halo-local coordinates and compensated FP32 sums, FP64 recheck
// of particles whose energy lies within e_recheck of zero.
#include <algorithm>
#include <cmath>

#include <type_traits>

#include "lanes.hpp"
#include "bh.hpp"
#include "primitives.hpp"
#include "stages.hpp"

namespace halo {

namespace {

constexpr int TB = 256;
constexpr unsigned kPersist = 4096;
constexpr unsigned kSideGrid = 3 * 256;  // three blocks of 256 on each of 256 CUs

__global__ void k_kept_host_keys(const libhalo_halos h, uint32_t S, uint32_t* flag) {
  uint32_t s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= S) return;
  flag[s] = (h.merged_into[s] == (int32_t)s && h.host[s] >= 0) ? 1u : 0u;
}

__global__ void k_child_compact(const libhalo_halos h, uint32_t S, const uint32_t* flag,
                                const uint32_t* pos, uint32_t* key, uint32_t* val,
                                uint32_t* ccnt) {
  uint32_t s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= S || !flag[s]) return;
  key[pos[s]] = (uint32_t)h.host[s];
  val[pos[s]] = s;
  atomicAdd(ccnt + h.host[s], 1u);
}

// nS[a] += n_assigned[h] for h and every ancestor a of h; depth[h].
__global__ void k_subtree_sizes(const libhalo_halos h, uint32_t S, uint32_t* nS,
                                uint32_t* depth) {
  uint32_t s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= S) return;
  if (h.merged_into[s] != (int32_t)s) {
    depth[s] = 0xFFFFFFFFu;
    return;
  }
  const uint32_t na = h.n_assigned[s];
  uint32_t d = 0;
  atomicAdd(nS + s, na);
  for (int32_t a = h.host[s]; a >= 0; a = h.host[a]) {
    atomicAdd(nS + a, na);
    ++d;
  }
  depth[s] = d;
}

__global__ void k_root_flags(const uint32_t* depth, const uint32_t* nS, uint32_t S,
                             uint32_t* val) {
  uint32_t s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s < S) val[s] = depth[s] == 0 ? nS[s] : 0u;
}

__global__ void k_root_slots(const uint32_t* depth, const uint32_t* scan, uint32_t S,
                             uint32_t* slot) {
  uint32_t s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s < S && depth[s] == 0) slot[s] = scan[s];
}

// Children of halos at depth d get their slots: after the parent's own
// particles, siblings in increasing id.
__global__ void k_child_slots(const libhalo_halos h, const uint32_t* depth, uint32_t S,
                              uint32_t d, const uint32_t* coff, const uint32_t* cids,
                              const uint32_t* nS, uint32_t* slot) {
  uint32_t s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= S || depth[s] != d) return;
  uint32_t o = slot[s] + h.n_assigned[s];
  for (uint32_t q = coff[s]; q < coff[s + 1]; ++q) {
    uint32_t c = cids[q];
    slot[c] = o;
    o += nS[c];
  }
}

__global__ void k_assigned_flags(const int32_t* halo_of, uint32_t n, uint32_t* flag) {
  uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) flag[i] = halo_of[i] >= 0 ? 1u : 0u;
}

__global__ void k_assigned_compact(const int32_t* halo_of, const uint32_t* flag,
                                   const uint32_t* pos, uint32_t n, uint32_t* key,
                                   uint32_t* val) {
  uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n || !flag[i]) return;
  key[pos[i]] = (uint32_t)halo_of[i];
  val[pos[i]] = i;
}

__global__ void k_group_first(const uint32_t* key, uint32_t m, uint32_t* gfirst) {
  uint32_t q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= m) return;
  if (q == 0 || key[q] != key[q - 1]) gfirst[key[q]] = q;
}

// Layout arrays: particle index, unwrapped FP64 coordinates, velocities.
template <class T>
__global__ void k_layout(const T* x, const T* y, const T* z, const float* vx, const float* vy,
                         const float* vz, double box, const libhalo_halos h,
                         const uint32_t* key, const uint32_t* val, const uint32_t* gfirst,
                         const uint32_t* slot, uint32_t m, uint32_t* lp, double* ux, double* uy,
                         double* uz, float* lvx, float* lvy, float* lvz, uint32_t* lhalo) {
  uint32_t q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= m) return;
  const uint32_t hh = key[q], i = val[q];
  const uint32_t p = slot[hh] + (q - gfirst[hh]);
  const uint32_t a = h.fof[hh];
  lp[p] = i;
  lhalo[p] = hh;
  ux[p] = min_image((double)x[i] - (double)x[a], box);
  uy[p] = min_image((double)y[i] - (double)y[a], box);
  uz[p] = min_image((double)z[i] - (double)z[a], box);
  lvx[p] = vx[i];
  lvy[p] = vy[i];
  lvz[p] = vz[i];
}

__global__ void k_zero_acc(I128* acc, uint32_t* nb, uint32_t S) {
  uint32_t s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= S) return;
  for (int c = 0; c < 3; ++c) acc[3 * (size_t)s + c] = I128{0ull, 0ll};
  nb[s] = 0;
}

// Exact velocity sums of each halo's own particles.
__global__ void k_own_vsum(const float* lvx, const float* lvy, const float* lvz,
                           const uint32_t* lhalo, uint32_t m, I128* acc) {
  uint32_t q = blockIdx.x * blockDim.x + threadIdx.x;
  const bool ok = q < m;
  const uint32_t hh = ok ? lhalo[q] : 0xFFFFFFFFu;
  I128 v[3];
  v[0] = i128_from(ok ? quantise((double)lvx[q], kVelShift) : 0);
  v[1] = i128_from(ok ? quantise((double)lvy[q], kVelShift) : 0);
  v[2] = i128_from(ok ? quantise((double)lvz[q], kVelShift) : 0);
  const uint32_t h0 = __shfl(hh, 0);
  if (__all(hh == h0) && h0 != 0xFFFFFFFFu) {
    for (int c = 0; c < 3; ++c) v[c] = wave_sum_i128(v[c]);
    if ((threadIdx.x & 63) == 0)
      for (int c = 0; c < 3; ++c) atomic_add_i128(acc + 3 * (size_t)h0 + c, v[c]);
  } else if (ok) {
    for (int c = 0; c < 3; ++c) atomic_add_i128(acc + 3 * (size_t)hh + c, v[c]);
  }
}

// Adds each halo's own sums to every ancestor's S(h) sums.
__global__ void k_chain_vsum(const libhalo_halos h, uint32_t S, const I128* own, I128* accS) {
  uint32_t s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= S || h.merged_into[s] != (int32_t)s) return;
  for (int c = 0; c < 3; ++c) {
    I128 v = own[3 * (size_t)s + c];
    atomic_add_i128(accS + 3 * (size_t)s + c, v);
    for (int32_t a = h.host[s]; a >= 0; a = h.host[a]) atomic_add_i128(accS + 3 * (size_t)a + c, v);
  }
}

__global__ void k_vbulk(const I128* accS, const uint32_t* nS, uint32_t S, double* vb) {
  uint32_t s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= S) return;
  double n = (double)nS[s];
  for (int c = 0; c < 3; ++c)
    vb[3 * (size_t)s + c] =
        nS[s] ? ldexp(i128_to_f64(accS[3 * (size_t)s + c]) / n, -kVelShift) : 0.0;
}

__device__ __forceinline__ uint32_t seg_of(const uint32_t* off, uint32_t K, uint32_t w) {
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

// ------------------------------------------------------------ potentials --
// Work unit: kPotI own particles of a halo (a block of four wavefronts; each
// lane holds kPotK particles i = t0 + lane + 64 k of its wave's tile of
// kPotTile) against one j-chunk of J particles of its S(h) (J one of the
// instantiated chunk sizes, kPotJ by default; the libhalo_params pot_chunk).  S(h) starts
// with the halo's own particles, followed by its subhaloes' S.  A pair of two
// own particles is evaluated once: the wave owning the lower tile adds the
// term to its particle's sum and, summed over the wave's kPotTile particles,
// to the other particle's sum, which collects in LDS for the unit.  The wave's
// own tile and the subhalo particles are evaluated from the i side only.
//
// Every partial sum goes into a 128-bit fixed-point accumulator (value x 2^32,
// integer atomics): integer addition is associative, so the result does not
// depend on which block ran which unit, or when.
constexpr uint32_t kPotK = 4;
constexpr uint32_t kPotTile = 64 * kPotK;  // particles per wave
constexpr uint32_t kPotI = 4 * kPotTile;   // particles per unit
constexpr uint32_t kPotJ = 2048;           // default j-chunk, a multiple of kPotTile
constexpr int kPotFrac = 32;               // fractional bits of the accumulators
constexpr double kFar = 1e150;             // coordinate of a lane slot without a particle

// round(v 2^32) for v >= 0 (below 2^63) as a 128-bit integer; every step is
// exact: s is an integer, and its 2^64 and 2^32 words are split off by floor
// and fma.
__device__ __forceinline__ I128 pot_fixed(double v) {
  const double s = rint(ldexp(v, kPotFrac));
  const double h = floor(s * 0x1p-64);
  const double m = __fma_rn(-h, 0x1p64, s);
  const double mh = floor(m * 0x1p-32);
  const double ml = __fma_rn(-mh, 0x1p32, m);
  I128 r;
  r.lo = ((unsigned long long)(uint32_t)mh << 32) | (uint32_t)ml;
  r.hi = (long long)(int32_t)h;
  return r;
}

template <uint32_t J>
__host__ __device__ __forceinline__ uint32_t pot_units(uint32_t nown, uint32_t ns) {
  return ((nown + kPotI - 1u) / kPotI) * ((ns + J - 1u) / J);
}

// Calls f with the j-chunk size of pot_chunk (0: kPotJ) as a type.
template <class F>
void with_pot_chunk(int32_t pc, F&& f) {
  if (pc == 1024)
    f(std::integral_constant<uint32_t, 1024>{});
  else if (pc == 4096)
    f(std::integral_constant<uint32_t, 4096>{});
  else
    f(std::integral_constant<uint32_t, kPotJ>{});
}

// Per kept halo: the unit count, and a sort key ordering halos by their cost
// (~ nown |S(h)|), largest first.
template <uint32_t J>
__global__ void k_pot_counts(const libhalo_halos h, uint32_t S, const uint32_t* nS,
                             double bh_theta, uint32_t bh_min, uint32_t* ucnt, uint32_t* key,
                             uint32_t* val) {
  uint32_t s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= S) return;
  const uint32_t nown = h.n_assigned[s], ns = nS[s];
  const bool kept = h.merged_into[s] == (int32_t)s;
  // haloes taking the tree potential get no direct-sum units
  const bool on = kept && nown > 0 && !bh_takes(kept, nown, ns, bh_theta, bh_min);
  const unsigned long long cost = ((unsigned long long)nown * ns) >> 16;
  ucnt[s] = on ? pot_units<J>(nown, ns) : 0u;
  key[s] = on ? ~(uint32_t)min(cost, 0xFFFFFFFEull) : 0xFFFFFFFFu;
  val[s] = s;
}

__global__ void k_gather_u32(const uint32_t* src, const uint32_t* idx, uint32_t n,
                             uint32_t* dst) {
  uint32_t k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k < n) dst[k] = src[idx[k]];
}

struct PotUnit {
  uint32_t base, nown, ns, b, j0, j1;
};

// Decodes unit u: the units of halo order[k] are [uoff[k], uoff[k+1]),
// chunk-major so that concurrent blocks share a j-chunk.
template <uint32_t J>
__device__ __forceinline__ PotUnit pot_unit(const libhalo_halos& h, const uint32_t* order,
                                            const uint32_t* uoff, uint32_t K,
                                            const uint32_t* slot, const uint32_t* nS,
                                            uint32_t u) {
  PotUnit r;
  const uint32_t k = seg_of(uoff, K, u);
  const uint32_t hh = order[k];
  const uint32_t local = u - uoff[k];
  r.nown = h.n_assigned[hh];
  r.ns = nS[hh];
  r.base = slot[hh];
  const uint32_t nb = (r.nown + kPotI - 1u) / kPotI;
  const uint32_t c = local / nb;
  r.b = local - c * nb;
  r.j0 = c * J;
  r.j1 = min(r.j0 + J, r.ns);
  return r;
}

// Next unit of this block: from the shared counter (dynamic) or by striding
// over the grid (static).  readfirstlane marks the result wave-uniform for the
// compiler, which then keeps the unit's bounds and the j loads scalar.
__device__ __forceinline__ uint32_t pot_next(uint32_t* ctr, uint32_t u0, uint32_t t,
                                             uint32_t* su) {
  __syncthreads();  // the previous unit's LDS sums are flushed
  uint32_t v;
  if (ctr) {
    if (threadIdx.x == 0) *su = atomicAdd(ctr, 1u);
    __syncthreads();
    v = *su;
  } else {
    v = blockIdx.x + t * gridDim.x;
  }
  return u0 + __builtin_amdgcn_readfirstlane(v);
}

// jacc[q] += v (fixed point, LDS; lo and hi words in separate arrays).
__device__ __forceinline__ void lds_add_fixed(unsigned long long* jlo, unsigned long long* jhi,
                                              uint32_t q, double v) {
  const I128 f = pot_fixed(v);
  const unsigned long long old = atomicAdd(jlo + q, f.lo);
  const long long add_hi = f.hi + ((old + f.lo) < old ? 1ll : 0ll);
  if (add_hi != 0) atomicAdd(jhi + q, (unsigned long long)add_hi);
}

// Sum over the wave's 64 lanes, in every lane (a fixed tree).
template <class F, F (*X1)(F), F (*X2)(F), F (*X4)(F), F (*X8)(F), F (*X16)(F), F (*X32)(F)>
__device__ __forceinline__ F wave_sum1(F r) {
  r = r + X1(r);
  r = r + X2(r);
  r = r + X4(r);
  r = r + X8(r);
  r = r + X16(r);
  r = r + X32(r);
  return r;
}

// Sum over the wave's 64 lanes of each of d[0..7], transposed, with lane-half
// swaps: v_permlane32_swap exchanges the upper half of one register with the
// lower half of another, so adding the two results sums lanes l and l ^ 32 of
// one value in the lower half and of the other value in the upper half (no
// selects); v_permlane16_swap does the same for l ^ 16 within each half, a
// keep/send exchange for l ^ 8 halves the values once more, and three
// exchanges sum the lanes l ^ 1, l ^ 2, l ^ 4.  Lane l with l & 7 == 0 returns
// the sum of d[u] with u = 4 b3 + 2 b4 + b5 (b3..b5 bits 3..5 of l).  The tree
// is fixed, so the result is deterministic.
template <void (*SW)(uint32_t&, uint32_t&)>
__device__ __forceinline__ double swap_add_f64(double x, double y) {
  unsigned long long ux = (unsigned long long)__double_as_longlong(x);
  unsigned long long uy = (unsigned long long)__double_as_longlong(y);
  uint32_t xl = (uint32_t)ux, xh = (uint32_t)(ux >> 32), yl = (uint32_t)uy,
           yh = (uint32_t)(uy >> 32);
  SW(xl, yl);
  SW(xh, yh);
  const double a = __longlong_as_double((long long)(((unsigned long long)xh << 32) | xl));
  const double b = __longlong_as_double((long long)(((unsigned long long)yh << 32) | yl));
  return a + b;
}
template <void (*SW)(uint32_t&, uint32_t&)>
__device__ __forceinline__ float swap_add_f32(float x, float y) {
  uint32_t ux = __float_as_uint(x), uy = __float_as_uint(y);
  SW(ux, uy);
  return __uint_as_float(ux) + __uint_as_float(uy);
}

__device__ __forceinline__ double wave_sum8_f64(const double* d) {
  const bool b3 = threadIdx.x & 8u;
  double s[4], t[2];
#pragma unroll
  for (int m = 0; m < 4; ++m) s[m] = swap_add_f64<swap_halves32>(d[2 * m], d[2 * m + 1]);
  t[0] = swap_add_f64<swap_halves16>(s[0], s[1]);
  t[1] = swap_add_f64<swap_halves16>(s[2], s[3]);
  double r = (b3 ? t[1] : t[0]) + lane_xor_f64<lane_xor8>(b3 ? t[0] : t[1]);
  r = r + lane_xor_f64<lane_xor1>(r);
  r = r + lane_xor_f64<lane_xor2>(r);
  r = r + lane_xor_f64<lane_xor4>(r);
  return r;
}

__device__ __forceinline__ float wave_sum8_f32(const float* d) {
  const bool b3 = threadIdx.x & 8u;
  float s[4], t[2];
#pragma unroll
  for (int m = 0; m < 4; ++m) s[m] = swap_add_f32<swap_halves32>(d[2 * m], d[2 * m + 1]);
  t[0] = swap_add_f32<swap_halves16>(s[0], s[1]);
  t[1] = swap_add_f32<swap_halves16>(s[2], s[3]);
  float r = (b3 ? t[1] : t[0]) + lane_xor_f32<lane_xor8>(b3 ? t[0] : t[1]);
  r = r + lane_xor_f32<lane_xor1>(r);
  r = r + lane_xor_f32<lane_xor2>(r);
  r = r + lane_xor_f32<lane_xor4>(r);
  return r;
}

#define HALO_XORS(F, f)                                                                   \
  F, lane_xor_##f<lane_xor1>, lane_xor_##f<lane_xor2>, lane_xor_##f<lane_xor4>,         \
      lane_xor_##f<lane_xor8>, lane_xor_##f<lane_xor16>, lane_xor_##f<lane_xor32>


// The unit's LDS j sums into the particles' accumulators.
__device__ __forceinline__ void pot_flush(const unsigned long long* jlo,
                                          const unsigned long long* jhi, uint32_t n,
                                          I128* __restrict__ acc) {
  for (uint32_t q = threadIdx.x; q < n; q += blockDim.x) {
    const I128 v{jlo[q], (long long)jhi[q]};
    if (v.lo != 0 || v.hi != 0) atomic_add_i128(acc + q, v);
  }
}

__device__ __forceinline__ void pot_clear(unsigned long long* jlo, unsigned long long* jhi,
                                          uint32_t n) {
  for (uint32_t q = threadIdx.x; q < n; q += blockDim.x) {
    jlo[q] = 0ull;
    jhi[q] = 0ull;
  }
}

// Twice the FP64 term 1/sqrt(r^2 + eps^2) of particle (x, y, z) and j is
// c y0: with y0 the hardware rsqrt estimate (about 2^-24 relative), one Newton
// step gives y0 (3 - r y0^2) / 2, so c = 3 - r y0^2 (a mul and an fma).  The
// kernels add c y0 with an fma and halve the sums, exactly, when they convert
// them.
__device__ __forceinline__ void pot_term2_f64(double bx, double by, double bz, double x,
                                              double y, double z, double eps2, double& c,
                                              double& y0) {
  const double dx = bx - x, dy = by - y, dz = bz - z;
  const double r = __fma_rn(dz, dz, __fma_rn(dy, dy, __fma_rn(dx, dx, eps2)));
  y0 = __builtin_amdgcn_rsq(r);
  c = __fma_rn(-(r * y0), y0, 3.0);
}

// FP64 terms (doubled) for j in [j0, j1) of the layout, i side only.  The j
// coordinates are wave-uniform and come in through scalar loads as operands of
// the vector ops.  kSelf: skip j == the slot's own particle (the span holding
// the wave's tile).
template <bool kSelf>
__device__ __forceinline__ void pot_span_f64(const double* __restrict__ ux,
                                             const double* __restrict__ uy,
                                             const double* __restrict__ uz, uint32_t j0,
                                             uint32_t j1, const uint32_t* self, const double* x,
                                             const double* y, const double* z, double eps2,
                                             double* A) {
  uint32_t j = j0;
  for (; j + 4 <= j1; j += 4) {
    double bx[4], by[4], bz[4];
    const double* __restrict__ px = ux + j;
    const double* __restrict__ py = uy + j;
    const double* __restrict__ pz = uz + j;
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      bx[u] = px[u];
      by[u] = py[u];
      bz[u] = pz[u];
    }
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
      for (uint32_t k = 0; k < kPotK; ++k) {
        double c, y0;
        pot_term2_f64(bx[u], by[u], bz[u], x[k], y[k], z[k], eps2, c, y0);
        A[k] = __fma_rn(c, (!kSelf || j + u != self[k]) ? y0 : 0.0, A[k]);
      }
  }
  for (; j < j1; ++j)
#pragma unroll
    for (uint32_t k = 0; k < kPotK; ++k) {
      double c, y0;
      pot_term2_f64(ux[j], uy[j], uz[j], x[k], y[k], z[k], eps2, c, y0);
      A[k] = __fma_rn(c, (!kSelf || j != self[k]) ? y0 : 0.0, A[k]);
    }
}

// FP64 terms (doubled) of the pairs (slot, j) for own j in [j0, j1), all
// above the wave's tile, each evaluated once: the term goes to the slot's A
// and, summed over the wave's slots, to jacc[j - jc].  Slots without a
// particle sit at kFar, where the term is ~1e-150: below half an ulp of any
// real term (>= 1 / the group's extent), so it changes no sum.
__device__ __forceinline__ void pot_sym_f64(const double* __restrict__ ux,
                                            const double* __restrict__ uy,
                                            const double* __restrict__ uz, uint32_t j0,
                                            uint32_t j1, uint32_t jc, const double* x,
                                            const double* y, const double* z, double eps2,
                                            double* A, unsigned long long* jlo,
                                            unsigned long long* jhi) {
  const uint32_t l = threadIdx.x & 63u, ul = swap8_index();
  uint32_t j = j0;
  for (; j + 8 <= j1; j += 8) {
    double bx[8], by[8], bz[8], tj[8];
    const double* __restrict__ px = ux + j;
    const double* __restrict__ py = uy + j;
    const double* __restrict__ pz = uz + j;
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      bx[u] = px[u];
      by[u] = py[u];
      bz[u] = pz[u];
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) {
#pragma unroll
      for (uint32_t k = 0; k < kPotK; ++k) {
        double c, y0;
        pot_term2_f64(bx[u], by[u], bz[u], x[k], y[k], z[k], eps2, c, y0);
        const double t = c * y0;  // one live value per pair (fmas of c and y0 spill here)
        A[k] += t;
        tj[u] = k == 0 ? t : tj[u] + t;
      }
    }
    const double s = wave_sum8_f64(tj);
    if ((l & 7u) == 0u) lds_add_fixed(jlo, jhi, j - jc + ul, 0.5 * s);
  }
  for (; j < j1; ++j) {
    double tj = 0.0;
#pragma unroll
    for (uint32_t k = 0; k < kPotK; ++k) {
      double c, y0;
      pot_term2_f64(ux[j], uy[j], uz[j], x[k], y[k], z[k], eps2, c, y0);
      const double t = c * y0;
      A[k] += t;
      tj = k == 0 ? t : tj + t;
    }
    const double s = wave_sum1<HALO_XORS(double, f64)>(tj);
    if (l == 0u) lds_add_fixed(jlo, jhi, j - jc, 0.5 * s);
  }
}

// FP64 form.
template <uint32_t J>
__global__ void __launch_bounds__(TB, 4)
    k_potential_f64(const double* __restrict__ ux, const double* __restrict__ uy,
                    const double* __restrict__ uz, const libhalo_halos h,
                    const uint32_t* __restrict__ order, const uint32_t* __restrict__ uoff,
                    uint32_t K, const uint32_t* __restrict__ slot,
                    const uint32_t* __restrict__ nS, uint32_t u0, uint32_t u1, uint32_t* ctr,
                    double eps2, I128* __restrict__ acc) {
  __shared__ unsigned long long jlo[J], jhi[J];
  __shared__ uint32_t su;
  for (uint32_t t = 0;; ++t) {
    const uint32_t u = pot_next(ctr, u0, t, &su);
    if (u >= u1) break;
    const PotUnit w = pot_unit<J>(h, order, uoff, K, slot, nS, u);
    const uint32_t ib = w.b * kPotI;
    const uint32_t je = min(w.j1, w.nown);  // end of the chunk's own part
    if (w.j1 <= ib && w.j1 <= w.nown) continue;  // pairs taken from the other side
    const uint32_t nj = je > w.j0 ? je - w.j0 : 0u;
    pot_clear(jlo, jhi, nj);
    __syncthreads();
    const uint32_t t0 =
        __builtin_amdgcn_readfirstlane(ib + (threadIdx.x >> 6) * kPotTile);
    if (t0 < w.nown) {
      const uint32_t b = w.base;
      uint32_t qi[kPotK];
      double x[kPotK], y[kPotK], z[kPotK], A[kPotK];
#pragma unroll
      for (uint32_t k = 0; k < kPotK; ++k) {
        const uint32_t li = t0 + (threadIdx.x & 63u) + 64u * k;
        const bool ok = li < w.nown;
        const uint32_t q = b + (ok ? li : 0u);  // an in-range load either way
        qi[k] = ok ? q : 0xFFFFFFFFu;
        x[k] = ok ? ux[q] : kFar;
        y[k] = ok ? uy[q] : kFar;
        z[k] = ok ? uz[q] : kFar;
        A[k] = 0.0;
      }
      if (t0 >= w.j0 && t0 < w.j1)
        pot_span_f64<true>(ux, uy, uz, b + t0, b + min(t0 + kPotTile, w.nown), qi, x, y, z,
                           eps2, A);
      const uint32_t js = max(w.j0, t0 + kPotTile);
      if (js < je)
        pot_sym_f64(ux, uy, uz, b + js, b + je, b + w.j0, x, y, z, eps2, A, jlo, jhi);
      const uint32_t ss = max(w.j0, w.nown);
      if (ss < w.j1)
        pot_span_f64<false>(ux, uy, uz, b + ss, b + w.j1, qi, x, y, z, eps2, A);
#pragma unroll
      for (uint32_t k = 0; k < kPotK; ++k) {
        const double v = 0.5 * A[k];
        if (qi[k] != 0xFFFFFFFFu && v > 0.0) atomic_add_i128(acc + qi[k], pot_fixed(v));
      }
    }
    __syncthreads();
    pot_flush(jlo, jhi, nj, acc + w.base + w.j0);
  }
}

// FP32 form: coordinates relative to the tree's origin, hardware FP32 rsqrt;
// the i-side terms of each slot go into a partial sum folded every 64 j into
// a compensated sum.
struct Comp32 {
  float acc = 0.0f, comp = 0.0f;
  __device__ __forceinline__ void add(float s) {
    const float yk = s - comp;
    const float tk = acc + yk;
    comp = (tk - acc) - yk;
    acc = tk;
  }
};

__device__ __forceinline__ float pot_term_f32(float bx, float by, float bz, float x, float y,
                                              float z, float eps2) {
  const float dx = bx - x, dy = by - y, dz = bz - z;
  return __builtin_amdgcn_rsqf(__fmaf_rn(dz, dz, __fmaf_rn(dy, dy, __fmaf_rn(dx, dx, eps2))));
}

template <bool kSelf>
__device__ __forceinline__ void pot_span_f32(const float* __restrict__ fx,
                                             const float* __restrict__ fy,
                                             const float* __restrict__ fz, uint32_t j0,
                                             uint32_t j1, const uint32_t* self, const float* x,
                                             const float* y, const float* z, float eps2,
                                             Comp32* A) {
  uint32_t j = j0;
  while (j < j1) {
    const uint32_t je = min(j + 64u, j1);
    float p[kPotK];
#pragma unroll
    for (uint32_t k = 0; k < kPotK; ++k) p[k] = 0.0f;
    for (; j + 8 <= je; j += 8) {
      float bx[8], by[8], bz[8];
      const float* __restrict__ px = fx + j;
      const float* __restrict__ py = fy + j;
      const float* __restrict__ pz = fz + j;
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        bx[u] = px[u];
        by[u] = py[u];
        bz[u] = pz[u];
      }
#pragma unroll
      for (int u = 0; u < 8; ++u)
#pragma unroll
        for (uint32_t k = 0; k < kPotK; ++k) {
          float t = pot_term_f32(bx[u], by[u], bz[u], x[k], y[k], z[k], eps2);
          if (kSelf) t = (j + u != self[k]) ? t : 0.0f;
          p[k] += t;
        }
    }
    for (; j < je; ++j)
#pragma unroll
      for (uint32_t k = 0; k < kPotK; ++k) {
        float t = pot_term_f32(fx[j], fy[j], fz[j], x[k], y[k], z[k], eps2);
        if (kSelf) t = (j != self[k]) ? t : 0.0f;
        p[k] += t;
      }
#pragma unroll
    for (uint32_t k = 0; k < kPotK; ++k) A[k].add(p[k]);
  }
}

// FP32 terms of the pairs (slot, j) for own j in [j0, j1) above the wave's
// tile, each evaluated once: i side as in pot_span_f32, j side summed over the
// wave's slots in FP32 (a fixed tree) and added to jacc[j - jc] in fixed
// point.  Slots without a particle sit at 1e18, where the term (~6e-19) is
// below half an ulp of any real term.
__device__ __forceinline__ void pot_sym_f32(const float* __restrict__ fx,
                                            const float* __restrict__ fy,
                                            const float* __restrict__ fz, uint32_t j0,
                                            uint32_t j1, uint32_t jc, const float* x,
                                            const float* y, const float* z, float eps2,
                                            Comp32* A, unsigned long long* jlo,
                                            unsigned long long* jhi) {
  const uint32_t l = threadIdx.x & 63u, ul = swap8_index();
  uint32_t j = j0;
  while (j < j1) {
    const uint32_t je = min(j + 64u, j1);
    float p[kPotK];
#pragma unroll
    for (uint32_t k = 0; k < kPotK; ++k) p[k] = 0.0f;
    for (; j + 8 <= je; j += 8) {
      float bx[8], by[8], bz[8], tj[8];
      const float* __restrict__ px = fx + j;
      const float* __restrict__ py = fy + j;
      const float* __restrict__ pz = fz + j;
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        bx[u] = px[u];
        by[u] = py[u];
        bz[u] = pz[u];
      }
#pragma unroll
      for (int u = 0; u < 8; ++u)
#pragma unroll
        for (uint32_t k = 0; k < kPotK; ++k) {
          const float t = pot_term_f32(bx[u], by[u], bz[u], x[k], y[k], z[k], eps2);
          p[k] += t;
          tj[u] = k == 0 ? t : tj[u] + t;
        }
      const float s = wave_sum8_f32(tj);
      if ((l & 7u) == 0u) lds_add_fixed(jlo, jhi, j - jc + ul, (double)s);
    }
    for (; j < je; ++j) {
      float tj = 0.0f;
#pragma unroll
      for (uint32_t k = 0; k < kPotK; ++k) {
        const float t = pot_term_f32(fx[j], fy[j], fz[j], x[k], y[k], z[k], eps2);
        p[k] += t;
        tj = k == 0 ? t : tj + t;
      }
      const float s = wave_sum1<HALO_XORS(float, f32)>(tj);
      if (l == 0u) lds_add_fixed(jlo, jhi, j - jc, (double)s);
    }
#pragma unroll
    for (uint32_t k = 0; k < kPotK; ++k) A[k].add(p[k]);
  }
}

// Mixed form: FP32 coordinates relative to the first particle of the
// outermost host of the halo's tree (one origin per contiguous tree range).
__global__ void k_rel_f32(const double* ux, const double* uy, const double* uz,
                          const libhalo_halos h, const uint32_t* slot, const uint32_t* lhalo,
                          uint32_t m, float* fx, float* fy, float* fz) {
  uint32_t q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= m) return;
  int32_t r = (int32_t)lhalo[q];
  while (h.host[r] >= 0) r = h.host[r];
  const uint32_t o = slot[r];
  fx[q] = (float)(ux[q] - ux[o]);
  fy[q] = (float)(uy[q] - uy[o]);
  fz[q] = (float)(uz[q] - uz[o]);
}

template <uint32_t J>
__global__ void __launch_bounds__(TB, 4)
    k_potential_f32(const float* __restrict__ fx, const float* __restrict__ fy,
                    const float* __restrict__ fz, const libhalo_halos h,
                    const uint32_t* __restrict__ order, const uint32_t* __restrict__ uoff,
                    uint32_t K, const uint32_t* __restrict__ slot,
                    const uint32_t* __restrict__ nS, uint32_t u0, uint32_t u1, uint32_t* ctr,
                    float eps2, I128* __restrict__ acc) {
  __shared__ unsigned long long jlo[J], jhi[J];
  __shared__ uint32_t su;
  for (uint32_t t = 0;; ++t) {
    const uint32_t u = pot_next(ctr, u0, t, &su);
    if (u >= u1) break;
    const PotUnit w = pot_unit<J>(h, order, uoff, K, slot, nS, u);
    const uint32_t ib = w.b * kPotI;
    const uint32_t je = min(w.j1, w.nown);
    if (w.j1 <= ib && w.j1 <= w.nown) continue;
    const uint32_t nj = je > w.j0 ? je - w.j0 : 0u;
    pot_clear(jlo, jhi, nj);
    __syncthreads();
    const uint32_t t0 =
        __builtin_amdgcn_readfirstlane(ib + (threadIdx.x >> 6) * kPotTile);
    if (t0 < w.nown) {
      const uint32_t b = w.base;
      uint32_t qi[kPotK];
      float x[kPotK], y[kPotK], z[kPotK];
      Comp32 A[kPotK];
#pragma unroll
      for (uint32_t k = 0; k < kPotK; ++k) {
        const uint32_t li = t0 + (threadIdx.x & 63u) + 64u * k;
        const bool ok = li < w.nown;
        const uint32_t q = b + (ok ? li : 0u);
        qi[k] = ok ? q : 0xFFFFFFFFu;
        x[k] = ok ? fx[q] : 1e18f;
        y[k] = ok ? fy[q] : 1e18f;
        z[k] = ok ? fz[q] : 1e18f;
      }
      if (t0 >= w.j0 && t0 < w.j1)
        pot_span_f32<true>(fx, fy, fz, b + t0, b + min(t0 + kPotTile, w.nown), qi, x, y, z,
                           eps2, A);
      const uint32_t js = max(w.j0, t0 + kPotTile);
      if (js < je) pot_sym_f32(fx, fy, fz, b + js, b + je, b + w.j0, x, y, z, eps2, A, jlo, jhi);
      const uint32_t ss = max(w.j0, w.nown);
      if (ss < w.j1) pot_span_f32<false>(fx, fy, fz, b + ss, b + w.j1, qi, x, y, z, eps2, A);
#pragma unroll
      for (uint32_t k = 0; k < kPotK; ++k) {
        const double v = (double)A[k].acc - (double)A[k].comp;
        if (qi[k] != 0xFFFFFFFFu && v > 0.0) atomic_add_i128(acc + qi[k], pot_fixed(v));
      }
    }
    __syncthreads();
    pot_flush(jlo, jhi, nj, acc + w.base + w.j0);
  }
}

// Major mergers (Section 3.5.3): the halo whose S decides the potential of
// h's particles, following host links while |S(h)| >= mp |S(host)| (the
// identity when mp <= 0 and for merged seeds).
__global__ void k_merge_target(const libhalo_halos h, uint32_t S, const uint32_t* nS, double mp,
                               uint32_t* tgt) {
  const uint32_t s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= S) return;
  int32_t t = (int32_t)s;
  if (mp > 0.0 && h.merged_into[s] == (int32_t)s)
    while (h.host[t] >= 0 && (double)nS[t] >= mp * (double)nS[h.host[t]]) t = h.host[t];
  tgt[s] = (uint32_t)t;
}

// Units of the merger term: h's own particles (kPotI per unit) against the
// particles of S(target) outside S(h) (kPotJ per unit); entry S stays 0.
__global__ void k_ext_counts(const libhalo_halos h, uint32_t S, const uint32_t* tgt,
                             const uint32_t* nS, uint32_t* ucnt) {
  const uint32_t s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s > S) return;
  uint32_t u = 0;
  if (s < S && tgt[s] != s) {
    const uint32_t nown = h.n_assigned[s], e = nS[tgt[s]] - nS[s];
    u = ((nown + kPotI - 1u) / kPotI) * ((e + kPotJ - 1u) / kPotJ);
  }
  ucnt[s] = u;
}

// The merger term, FP64, i side only: S(target) lies in the layout as one
// range holding S(h) as a sub-range, so the external particles are the two
// ranges around it.  Terms go to the particles' fixed-point sums next to the
// ones of S(h); the sum does not depend on which unit ran when.
__global__ void __launch_bounds__(TB, 4)
    k_potential_ext_f64(const double* __restrict__ ux, const double* __restrict__ uy,
                        const double* __restrict__ uz, const libhalo_halos h,
                        const uint32_t* __restrict__ tgt, const uint32_t* __restrict__ slot,
                        const uint32_t* __restrict__ nS, const uint32_t* __restrict__ uoff,
                        uint32_t S, double eps2, I128* __restrict__ acc) {
  const uint32_t total = uoff[S];
  for (uint32_t u0 = blockIdx.x; u0 < total; u0 += gridDim.x) {
    const uint32_t u = __builtin_amdgcn_readfirstlane(u0);
    const uint32_t hh = seg_of(uoff, S, u);
    const uint32_t nown = h.n_assigned[hh], t = tgt[hh];
    const uint32_t b = slot[hh], bt = slot[t];
    const uint32_t e = nS[t] - nS[hh], pre = b - bt;
    const uint32_t nb = (nown + kPotI - 1u) / kPotI;
    const uint32_t local = u - uoff[hh];
    const uint32_t c = local / nb;
    const uint32_t t0 =
        __builtin_amdgcn_readfirstlane((local - c * nb) * kPotI + (threadIdx.x >> 6) * kPotTile);
    if (t0 >= nown) continue;  // wave-uniform
    const uint32_t e0 = c * kPotJ, e1 = min(e0 + kPotJ, e);
    uint32_t qi[kPotK];
    double x[kPotK], y[kPotK], z[kPotK], A[kPotK];
#pragma unroll
    for (uint32_t k = 0; k < kPotK; ++k) {
      const uint32_t li = t0 + (threadIdx.x & 63u) + 64u * k;
      const bool ok = li < nown;
      const uint32_t q = b + (ok ? li : 0u);
      qi[k] = ok ? q : 0xFFFFFFFFu;
      x[k] = ok ? ux[q] : kFar;
      y[k] = ok ? uy[q] : kFar;
      z[k] = ok ? uz[q] : kFar;
      A[k] = 0.0;
    }
    if (e0 < min(e1, pre)) pot_span_f64<false>(ux, uy, uz, bt + e0, bt + min(e1, pre), qi, x, y, z, eps2, A);
    if (max(e0, pre) < e1)
      pot_span_f64<false>(ux, uy, uz, bt + nS[hh] + max(e0, pre), bt + nS[hh] + e1, qi, x, y,
                          z, eps2, A);
#pragma unroll
    for (uint32_t k = 0; k < kPotK; ++k) {
      const double v = 0.5 * A[k];
      if (qi[k] != 0xFFFFFFFFu && v > 0.0) atomic_add_i128(acc + qi[k], pot_fixed(v));
    }
  }
}

__global__ void k_zero_i128(I128* a, uint32_t m) {
  uint32_t q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q < m) a[q] = I128{0ull, 0ll};
}

// sum[q] = the particle's fixed-point potential sum as FP64.
__global__ void k_pot_finish(const I128* acc, uint32_t m, double* sum) {
  uint32_t q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q < m) sum[q] = ldexp(i128_to_f64(acc[q]), -kPotFrac);
}

// FP64 recheck of one particle's potential (mixed form), one block per particle,
// over S(h) or, for a major merger, S of the merging system.
__global__ void __launch_bounds__(TB)
    k_recheck(const double* ux, const double* uy, const double* uz, const uint32_t* lhalo,
              const uint32_t* tgt, const uint32_t* slot, const uint32_t* nS,
              const uint32_t* list, const uint32_t* nlist, double eps2, double* sum) {
  __shared__ double red[TB];
  const uint32_t L = nlist[0];
  for (uint32_t t = blockIdx.x; t < L; t += gridDim.x) {
    const uint32_t qi = list[t];
    const uint32_t hh = tgt[lhalo[qi]];  // S(h), or the merging system's S
    const uint32_t base = slot[hh], ns = nS[hh];
    const double xi = ux[qi], yi = uy[qi], zi = uz[qi];
    double acc = 0.0;
    for (uint32_t j = threadIdx.x; j < ns; j += TB) {
      if (base + j == qi) continue;
      double dx = ux[base + j] - xi, dy = uy[base + j] - yi, dz = uz[base + j] - zi;
      acc += rsqrt_f64(sq3(dx, dy, dz) + eps2);  // hardware estimate + one Newton step
    }
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int o = TB / 2; o > 0; o >>= 1) {
      if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
      __syncthreads();
    }
    if (threadIdx.x == 0) sum[qi] = red[0];
    __syncthreads();
  }
}

// Energies and bound flags.  Mixed form: a particle whose energy lies within
// e_rel of zero is listed for the FP64 recheck instead, unless its halo took
// the tree potential, whose error (set by theta) dwarfs FP32 rounding: its
// flag is the tree's, as in the FP64 form with the tree.
__global__ void k_energy(const double* sum, const float* lvx, const float* lvy,
                         const float* lvz, const uint32_t* lhalo, const uint32_t* lp,
                         const double* vb, uint32_t m, double mGm, double e_rel, int mixed,
                         const libhalo_halos h, const uint32_t* nS, double bh_theta,
                         uint32_t bh_min, uint8_t* bound, double* phi, uint32_t* nb_own,
                         uint32_t* rlist, uint32_t* nr) {
  const uint32_t q = blockIdx.x * blockDim.x + threadIdx.x;
  const bool ok = q < m;
  uint32_t hh = 0;
  bool b = false;
  if (ok) {
    hh = lhalo[q];
    const uint32_t i = lp[q];
    const double ph = mGm * sum[q];
    const double ux = (double)lvx[q] - vb[3 * (size_t)hh],
                 uy = (double)lvy[q] - vb[3 * (size_t)hh + 1],
                 uz = (double)lvz[q] - vb[3 * (size_t)hh + 2];
    const double k = 0.5 * sq3(ux, uy, uz);
    const double e = k + ph;
    const bool tree = bh_takes(h.merged_into[hh] == (int32_t)hh, h.n_assigned[hh], nS[hh],
                               bh_theta, bh_min);
    if (mixed && !tree && fabs(e) < e_rel * (k + fabs(ph))) {
      rlist[atomicAdd(nr, 1u)] = q;  // decided after the FP64 recheck
    } else {
      b = e < 0.0;
      bound[i] = b;
      if (phi) phi[i] = ph;
    }
  }
  agg_add_u32(nb_own, hh, 1u, b);
}

__global__ void k_energy_list(const double* sum, const float* lvx, const float* lvy,
                              const float* lvz, const uint32_t* lhalo, const uint32_t* lp,
                              const double* vb, const uint32_t* list, const uint32_t* nlist,
                              double mGm, uint8_t* bound, double* phi, uint32_t* nb_own) {
  uint32_t t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= nlist[0]) return;
  const uint32_t q = list[t];
  const uint32_t hh = lhalo[q], i = lp[q];
  const double ph = mGm * sum[q];
  const double ux = (double)lvx[q] - vb[3 * (size_t)hh], uy = (double)lvy[q] - vb[3 * (size_t)hh + 1],
               uz = (double)lvz[q] - vb[3 * (size_t)hh + 2];
  const double e = 0.5 * sq3(ux, uy, uz) + ph;
  const uint8_t b = e < 0.0;
  bound[i] = b;
  if (phi) phi[i] = ph;
  if (b) atomicAdd(nb_own + hh, 1u);
}

__global__ void k_unbind_out(const libhalo_halos h, uint32_t S, const uint32_t* nS,
                             const uint32_t* nb_own, const double* vb, double ut,
                             libhalo_unbound o, uint32_t* nbS) {
  uint32_t s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= S) return;
  const bool kept = h.merged_into[s] == (int32_t)s;
  o.n_bound_own[s] = kept ? nb_own[s] : 0u;
  o.n_s[s] = kept ? nS[s] : 0u;
  o.vbx[s] = kept ? vb[3 * (size_t)s] : 0.0;
  o.vby[s] = kept ? vb[3 * (size_t)s + 1] : 0.0;
  o.vbz[s] = kept ? vb[3 * (size_t)s + 2] : 0.0;
  if (kept) {
    uint32_t b = nb_own[s];
    atomicAdd(nbS + s, b);
    for (int32_t a = h.host[s]; a >= 0; a = h.host[a]) atomicAdd(nbS + a, b);
  }
}

__global__ void k_valid(const libhalo_halos h, uint32_t S, const uint32_t* nS,
                        const uint32_t* nbS, double ut, libhalo_unbound o) {
  uint32_t s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= S) return;
  const bool kept = h.merged_into[s] == (int32_t)s;
  o.n_bound_s[s] = kept ? nbS[s] : 0u;
  o.valid[s] = kept && ((double)nbS[s] >= ut * (double)nS[s]) ? 1 : 0;
}

__global__ void k_init_particles(uint8_t* bound, double* phi, uint32_t n) {
  uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  bound[i] = 0;
  if (phi) phi[i] = 0.0;
}

template <class T>
void unbind_impl(Ctx& ctx, int64_t n, const T* x, const T* y, const T* z, const float* vx,
                 const float* vy, const float* vz, const libhalo_halos& h, int64_t S64,
                 const int32_t* halo_of, uint8_t* bound, double* phi, libhalo_unbound& o,
                 hipStream_t s) {
  const libhalo_params& P = ctx.p;
  const uint32_t S = (uint32_t)S64;
  const double box = P.box;
  const double eps2 = P.softening * P.softening;
  const double mGm = -P.G * P.particle_mass;
  const bool mixed = P.prec == LIBHALO_PREC_MIXED;
  const bool plain = P.mode == LIBHALO_PLAIN;
  uint32_t* hb = ctx.host_slot<uint32_t>(0);
  auto readu = [&](const uint32_t* d, int slot) {
    HALO_HIP(hipMemcpyAsync(hb + slot, d, 4, hipMemcpyDeviceToHost, s));
    HALO_HIP(hipStreamSynchronize(s));
    return hb[slot];
  };
  if (S == 0) {
    k_init_particles<<<blocks_for(n, TB), TB, 0, s>>>(bound, phi, (uint32_t)n);
    HALO_HIP(hipStreamSynchronize(s));
    return;
  }
  struct W {
    uint32_t *flag, *pos, *ck0, *cv0, *ck1, *cv1, *ccnt, *coff, *nS, *depth, *slot, *rootv,
        *dcnt, *stmp, *ak0, *av0, *ak1, *av1, *gfirst, *lp, *lhalo, *nb_own, *nbS, *rlist,
        *ucnt, *uoff, *pk0, *pv0, *pk1, *pv1, *tgt, *ecnt, *eoff;
    double *ux, *uy, *uz, *vb, *sum;
    float *lvx, *lvy, *lvz, *fx, *fy, *fz;
    I128 *accO, *accS, *pacc;
    void *rtmp;
  } w;
  carve_workspace(ctx, [&](Arena& A) {
    const int64_t S2 = S + 2, N2 = n + 2;
    w.flag = A.take<uint32_t>(std::max(S2, N2));
    w.pos = A.take<uint32_t>(std::max(S2, N2));
    w.ck0 = A.take<uint32_t>(S2);
    w.cv0 = A.take<uint32_t>(S2);
    w.ck1 = A.take<uint32_t>(S2);
    w.cv1 = A.take<uint32_t>(S2);
    w.ccnt = A.take<uint32_t>(S2);
    w.coff = A.take<uint32_t>(S2);
    w.nS = A.take<uint32_t>(S2);
    w.depth = A.take<uint32_t>(S2);
    w.slot = A.take<uint32_t>(S2);
    w.rootv = A.take<uint32_t>(S2);
    w.dcnt = A.take<uint32_t>(16);
    w.stmp = A.take<uint32_t>(scan_tmp_elems<uint32_t>(std::max(S2, N2)));
    w.ak0 = A.take<uint32_t>(N2);
    w.av0 = A.take<uint32_t>(N2);
    w.ak1 = A.take<uint32_t>(N2);
    w.av1 = A.take<uint32_t>(N2);
    w.gfirst = A.take<uint32_t>(S2);
    w.lp = A.take<uint32_t>(N2);
    w.lhalo = A.take<uint32_t>(N2);
    w.ucnt = A.take<uint32_t>(S2);
    w.uoff = A.take<uint32_t>(S2);
    w.pk0 = A.take<uint32_t>(S2);
    w.pv0 = A.take<uint32_t>(S2);
    w.pk1 = A.take<uint32_t>(S2);
    w.pv1 = A.take<uint32_t>(S2);
    w.nb_own = A.take<uint32_t>(S2);
    w.nbS = A.take<uint32_t>(S2);
    w.tgt = A.take<uint32_t>(S2);
    w.ecnt = A.take<uint32_t>(S2);
    w.eoff = A.take<uint32_t>(S2);
    w.rlist = A.take<uint32_t>(N2);
    w.ux = A.take<double>(N2);
    w.uy = A.take<double>(N2);
    w.uz = A.take<double>(N2);
    w.vb = A.take<double>(3 * S2);
    w.sum = A.take<double>(N2);
    w.lvx = A.take<float>(N2);
    w.lvy = A.take<float>(N2);
    w.lvz = A.take<float>(N2);
    w.fx = mixed ? A.take<float>(N2) : nullptr;
    w.fy = mixed ? A.take<float>(N2) : nullptr;
    w.fz = mixed ? A.take<float>(N2) : nullptr;
    w.accO = A.take<I128>(3 * S2);
    w.accS = A.take<I128>(3 * S2);
    w.pacc = A.take<I128>(N2);
    w.rtmp = A.take<char>(radix_tmp_bytes(std::max(S2, N2)));
  });
  // outputs are written only once the workspace is in place
  k_init_particles<<<blocks_for(n, TB), TB, 0, s>>>(bound, phi, (uint32_t)n);
  // children lists of the host/sub forest, ascending ids per host
  k_kept_host_keys<<<blocks_for(S, TB), TB, 0, s>>>(h, S, w.flag);
  exclusive_scan<uint32_t>(w.flag, w.pos, S, w.dcnt, w.stmp, s);
  k_fill_u32<<<blocks_for(S + 1, TB), TB, 0, s>>>(w.ccnt, S + 1, 0u);
  k_child_compact<<<blocks_for(S, TB), TB, 0, s>>>(h, S, w.flag, w.pos, w.ck0, w.cv0, w.ccnt);
  const uint32_t NC = readu(w.dcnt, 0);
  bool fc = radix_sort_pairs<uint32_t>(w.ck0, w.cv0, w.ck1, w.cv1, NC, bits_for(S), w.rtmp, s);
  uint32_t* cids = fc ? w.cv1 : w.cv0;
  exclusive_scan<uint32_t>(w.ccnt, w.coff, S, w.coff + S, w.stmp, s);
  // subtree sizes, depths, preorder slots
  k_fill_u32<<<blocks_for(S, TB), TB, 0, s>>>(w.nS, S, 0u);
  k_subtree_sizes<<<blocks_for(S, TB), TB, 0, s>>>(h, S, w.nS, w.depth);
  k_root_flags<<<blocks_for(S, TB), TB, 0, s>>>(w.depth, w.nS, S, w.rootv);
  exclusive_scan<uint32_t>(w.rootv, w.rootv, S, w.dcnt + 1, w.stmp, s);
  k_root_slots<<<blocks_for(S, TB), TB, 0, s>>>(w.depth, w.rootv, S, w.slot);
  // deepest host chain: bounded by the number of kept halos; stop when no child
  uint32_t maxd = 0;
  {
    std::vector<uint32_t> hd(S);
    HALO_HIP(hipMemcpyAsync(hd.data(), w.depth, 4ull * S, hipMemcpyDeviceToHost, s));
    HALO_HIP(hipStreamSynchronize(s));
    for (uint32_t v : hd)
      if (v != 0xFFFFFFFFu && v > maxd) maxd = v;
  }
  for (uint32_t d = 0; d < maxd; ++d)
    k_child_slots<<<blocks_for(S, TB), TB, 0, s>>>(h, w.depth, S, d, w.coff, cids, w.nS, w.slot);
  // particles in layout order
  k_assigned_flags<<<blocks_for(n, TB), TB, 0, s>>>(halo_of, (uint32_t)n, w.flag);
  exclusive_scan<uint32_t>(w.flag, w.pos, n, w.dcnt + 2, w.stmp, s);
  k_assigned_compact<<<blocks_for(n, TB), TB, 0, s>>>(halo_of, w.flag, w.pos, (uint32_t)n,
                                                      w.ak0, w.av0);
  const uint32_t m = readu(w.dcnt + 2, 1);
  bool fa = radix_sort_pairs<uint32_t>(w.ak0, w.av0, w.ak1, w.av1, m, bits_for(S), w.rtmp, s);
  uint32_t* akey = fa ? w.ak1 : w.ak0;
  uint32_t* aval = fa ? w.av1 : w.av0;
  if (m > 0) {
    k_group_first<<<blocks_for(m, TB), TB, 0, s>>>(akey, m, w.gfirst);
    k_layout<T><<<blocks_for(m, TB), TB, 0, s>>>(x, y, z, vx, vy, vz, box, h, akey, aval,
                                                 w.gfirst, w.slot, m, w.lp, w.ux, w.uy, w.uz,
                                                 w.lvx, w.lvy, w.lvz, w.lhalo);
  }
  // bulk velocities of S(h)
  k_zero_acc<<<blocks_for(S, TB), TB, 0, s>>>(w.accO, w.nb_own, S);
  k_zero_acc<<<blocks_for(S, TB), TB, 0, s>>>(w.accS, w.nbS, S);
  if (m > 0) k_own_vsum<<<blocks_for(m, TB), TB, 0, s>>>(w.lvx, w.lvy, w.lvz, w.lhalo, m, w.accO);
  k_chain_vsum<<<blocks_for(S, TB), TB, 0, s>>>(h, S, w.accO, w.accS);
  k_vbulk<<<blocks_for(S, TB), TB, 0, s>>>(w.accS, w.nS, S, w.vb);
  k_merge_target<<<blocks_for(S, TB), TB, 0, s>>>(h, S, w.nS, P.major_merger, w.tgt);
  // potentials: work units ordered largest first, one partial per particle
  // and j-chunk, partials added in chunk order
  const uint32_t bh_min = P.bh_min > 0 ? (uint32_t)P.bh_min : 32768u;
  with_pot_chunk(P.pot_chunk, [&](auto Jc) {
    k_pot_counts<decltype(Jc)::value><<<blocks_for(S, TB), TB, 0, s>>>(
        h, S, w.nS, P.bh_theta, bh_min, w.ucnt, w.pk0, w.pv0);
  });
  const bool fo = radix_sort_pairs<uint32_t>(w.pk0, w.pv0, w.pk1, w.pv1, S, 32, w.rtmp, s);
  const uint32_t* order = fo ? w.pv1 : w.pv0;
  k_gather_u32<<<blocks_for(S, TB), TB, 0, s>>>(w.ucnt, order, S, w.uoff);
  exclusive_scan<uint32_t>(w.uoff, w.uoff, S, w.uoff + S, w.stmp, s);
  const uint32_t U = readu(w.uoff + S, 2);
  if (m > 0) {
    k_zero_i128<<<blocks_for(m, TB), TB, 0, s>>>(w.pacc, m);
    if (mixed)
      k_rel_f32<<<blocks_for(m, TB), TB, 0, s>>>(w.ux, w.uy, w.uz, h, w.slot, w.lhalo, m, w.fx,
                                                 w.fy, w.fz);
    // With the tree potential on, the direct sums of the other haloes run on
    // the side stream beside it: both add into the fixed-point sums of
    // disjoint particles.
    const bool tree = P.bh_theta > 0.0;
    hipStream_t sp = s;  // stream of the direct sums
    auto launch = [&](uint32_t u0, uint32_t u1, uint32_t* ctr, unsigned grid) {
      with_pot_chunk(P.pot_chunk, [&](auto Jc) {
        constexpr uint32_t J = decltype(Jc)::value;
        if (mixed)
          HALO_PROF(ctx, "k_potential_f32", sp,
                    k_potential_f32<J><<<grid, TB, 0, sp>>>(w.fx, w.fy, w.fz, h, order, w.uoff,
                                                            S, w.slot, w.nS, u0, u1, ctr,
                                                            (float)eps2, w.pacc));
        else
          HALO_PROF(ctx, "k_potential_f64", sp,
                    k_potential_f64<J><<<grid, TB, 0, sp>>>(w.ux, w.uy, w.uz, h, order, w.uoff,
                                                            S, w.slot, w.nS, u0, u1, ctr, eps2,
                                                            w.pacc));
      });
    };
    if (plain) {
      // one launch per halo, in halo order, each over that halo's units
      std::vector<uint32_t> ho(S + 1), ord(S);
      HALO_HIP(hipMemcpyAsync(ho.data(), w.uoff, 4ull * (S + 1), hipMemcpyDeviceToHost, s));
      HALO_HIP(hipMemcpyAsync(ord.data(), order, 4ull * S, hipMemcpyDeviceToHost, s));
      HALO_HIP(hipStreamSynchronize(s));
      std::vector<uint32_t> pos(S);
      for (uint32_t k = 0; k < S; ++k) pos[ord[k]] = k;
      if (tree) sp = ctx.fork(s);
      for (uint32_t hh = 0; hh < S; ++hh) {
        const uint32_t k = pos[hh], nu = ho[k + 1] - ho[k];
        if (nu) launch(ho[k], ho[k + 1], nullptr, nu);
      }
    } else if (U > 0) {
      k_fill_u32<<<1, 64, 0, s>>>(w.dcnt + 4, 1, 0u);
      if (tree) sp = ctx.fork(s);
      // beside the tree, the persistent grid leaves one block slot per CU
      // (of the four its registers allow) to the tree's build kernels, which
      // would otherwise wait for it to drain
      launch(0, U, w.dcnt + 4, std::min<uint32_t>(tree ? kSideGrid : kPersist, U));
    }
    if (tree)
      bh_potential(ctx, h, S, w.nS, w.slot, w.ux, w.uy, w.uz, eps2, P.bh_theta, bh_min, w.pacc,
                   s);
    if (sp != s) ctx.join(s);
    if (P.major_merger > 0.0) {
      k_ext_counts<<<blocks_for(S + 1, TB), TB, 0, s>>>(h, S, w.tgt, w.nS, w.ecnt);
      exclusive_scan<uint32_t>(w.ecnt, w.eoff, S + 1, w.dcnt + 5, w.stmp, s);
      HALO_PROF(ctx, "k_potential_ext_f64", s,
                k_potential_ext_f64<<<kPersist, TB, 0, s>>>(w.ux, w.uy, w.uz, h, w.tgt, w.slot,
                                                             w.nS, w.eoff, S, eps2, w.pacc));
    }
    k_pot_finish<<<blocks_for(m, TB), TB, 0, s>>>(w.pacc, m, w.sum);
    k_fill_u32<<<1, 64, 0, s>>>(w.dcnt + 3, 1, 0u);
    k_energy<<<blocks_for(m, TB), TB, 0, s>>>(w.sum, w.lvx, w.lvy, w.lvz, w.lhalo, w.lp, w.vb, m,
                                             mGm, P.e_recheck, mixed ? 1 : 0, h, w.nS,
                                             P.bh_theta, bh_min, bound, phi, w.nb_own,
                                             w.rlist, w.dcnt + 3);
    if (mixed) {
      k_recheck<<<1024, TB, 0, s>>>(w.ux, w.uy, w.uz, w.lhalo, w.tgt, w.slot, w.nS, w.rlist,
                                    w.dcnt + 3, eps2, w.sum);
      k_energy_list<<<blocks_for(m, TB), TB, 0, s>>>(w.sum, w.lvx, w.lvy, w.lvz, w.lhalo, w.lp,
                                                     w.vb, w.rlist, w.dcnt + 3, mGm, bound,
                                                     phi, w.nb_own);
    }
  }
  k_unbind_out<<<blocks_for(S, TB), TB, 0, s>>>(h, S, w.nS, w.nb_own, w.vb,
                                                P.unbound_threshold, o, w.nbS);
  k_valid<<<blocks_for(S, TB), TB, 0, s>>>(h, S, w.nS, w.nbS, P.unbound_threshold, o);
  HALO_HIP(hipStreamSynchronize(s));
}

}  // namespace

void unbind(Ctx& ctx, int64_t n, int pos_dtype, const void* x, const void* y, const void* z,
            const float* vx, const float* vy, const float* vz, const libhalo_halos* halos,
            int64_t n_halos, const int32_t* halo_of, uint8_t* bound, double* phi,
            libhalo_unbound* out, hipStream_t s) {
  if (pos_dtype == LIBHALO_F64)
    unbind_impl<double>(ctx, n, (const double*)x, (const double*)y, (const double*)z, vx, vy,
                        vz, *halos, n_halos, halo_of, bound, phi, *out, s);
  else
    unbind_impl<float>(ctx, n, (const float*)x, (const float*)y, (const float*)z, vx, vy, vz,
                       *halos, n_halos, halo_of, bound, phi, *out, s);
}

}  // namespace halo
