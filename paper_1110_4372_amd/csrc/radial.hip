// Segmented radial sort and per-halo velocity dispersion / vmax.
#include "primitives.hpp"
#include "radial.hpp"

namespace halo {

namespace {
constexpr int TB = 256;

template <class T>
__global__ void k_r2(const T* x, const T* y, const T* z, double box, const double* cx,
                     const double* cy, const double* cz, const uint32_t* seg,
                     const uint32_t* pidx, uint32_t m, double* r2, uint32_t* key,
                     uint32_t* val) {
  const uint32_t e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= m) return;
  const uint32_t h = seg[e];
  const uint32_t i = pidx[e];
  double dx = min_image((double)x[i] - cx[h], box);
  double dy = min_image((double)y[i] - cy[h], box);
  double dz = min_image((double)z[i] - cz[h], box);
  double d = sq3(dx, dy, dz);
  r2[e] = d;
  // FP32 rounding is monotone, so this key orders like r^2 up to runs of
  // equal keys, which k_radial_fix puts in exact order
  key[e] = __float_as_uint((float)d);
  val[e] = e;
}

// start[s] = first position of segment s in the segment-sorted keys.
__global__ void k_seg_starts(const uint32_t* skey, uint32_t m, uint32_t nseg, uint32_t* start) {
  uint32_t s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s > nseg) return;
  uint32_t lo = 0, hi = m;
  while (lo < hi) {
    const uint32_t mid = (lo + hi) >> 1;
    if (skey[mid] < s)
      lo = mid + 1;
    else
      hi = mid;
  }
  start[s] = lo;
}

__global__ void k_seg_keys(const uint32_t* seg, const uint32_t* perm, uint32_t m,
                           uint32_t* key) {
  uint32_t q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q < m) key[q] = seg[perm[q]];
}

__global__ void k_radial_out(const uint32_t* perm, const uint32_t* seg, const uint32_t* pidx,
                             const double* r2, uint32_t m, uint32_t* s_seg, uint32_t* s_pidx,
                             double* s_r2, uint32_t* s_e) {
  uint32_t q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= m) return;
  uint32_t e = perm[q];
  s_seg[q] = seg[e];
  s_pidx[q] = pidx[e];
  s_r2[q] = r2[e];
  s_e[q] = e;
}

// Elements sorted by (segment, FP32-rounded r^2), equal keys in input order:
// the first element of each run of equal keys sorts its run by (exact r^2,
// input position), which gives the order of a stable sort on the exact r^2.
// Runs are rare and short; a run of identical values is already in order.
__global__ void k_radial_fix(const uint32_t* s_seg, uint32_t* s_pidx, double* s_r2,
                             uint32_t* s_e, uint32_t m) {
  const uint32_t q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= m) return;
  const uint32_t h = s_seg[q];
  const float f = (float)s_r2[q];
  if (q > 0 && s_seg[q - 1] == h && (float)s_r2[q - 1] == f) return;  // not a run head
  uint32_t end = q + 1;
  while (end < m && s_seg[end] == h && (float)s_r2[end] == f) ++end;
  for (uint32_t a = q + 1; a < end; ++a) {
    const double r = s_r2[a];
    const uint32_t pe = s_e[a], pp = s_pidx[a];
    uint32_t b = a;
    while (b > q && (s_r2[b - 1] > r || (s_r2[b - 1] == r && s_e[b - 1] > pe))) {
      s_r2[b] = s_r2[b - 1];
      s_e[b] = s_e[b - 1];
      s_pidx[b] = s_pidx[b - 1];
      --b;
    }
    s_r2[b] = r;
    s_e[b] = pe;
    s_pidx[b] = pp;
  }
}

__global__ void k_zero_sv(I128* acc, unsigned long long* vm, uint32_t nseg) {
  uint32_t h = blockIdx.x * blockDim.x + threadIdx.x;
  if (h >= nseg) return;
  for (int q = 0; q < 4; ++q) acc[4 * (size_t)h + q] = I128{0ull, 0ll};
  vm[h] = 0ull;
}

constexpr int kSvTB = 256;  // block of the accumulation (4 waves)

// Exact velocity sums and max of k^2 / max(r^2, eps^2) per segment over the
// sorted elements, one element per thread.
__global__ void __launch_bounds__(kSvTB)
    k_sigma_vmax_accum(const float* vx, const float* vy, const float* vz,
                       const uint32_t* s_seg, const uint32_t* s_pidx, const double* s_r2,
                       const uint32_t* start, uint32_t m, double eps2, I128* acc,
                       unsigned long long* vm) {
  __shared__ SegMerge<4, kSvTB / 64> L;
  const uint32_t q = blockIdx.x * blockDim.x + threadIdx.x;
  const bool ok = q < m;
  const uint32_t h = ok ? s_seg[q] : 0xFFFFFFFFu;
  long long w[3] = {0, 0, 0};
  double t = 0.0;
  if (ok) {
    const uint32_t i = s_pidx[q];
    w[0] = quantise((double)vx[i], kVelShift);
    w[1] = quantise((double)vy[i], kVelShift);
    w[2] = quantise((double)vz[i], kVelShift);
    const double kk = (double)(q - start[h] + 1);
    t = (kk * kk) / fmax(s_r2[q], eps2);
  }
  I128 v[4];
  for (int c = 0; c < 3; ++c) v[c] = i128_from(w[c]);
  v[3] = i128_add(i128_sqr(w[0]), i128_add(i128_sqr(w[1]), i128_sqr(w[2])));
  seg_merge_add<4, kSvTB / 64>(L, h, v, t, 0u, acc, vm, nullptr);
}

__global__ void k_sigma_vmax_final(const I128* acc, const unsigned long long* vm,
                                   const uint32_t* start, uint32_t nseg, double Gm,
                                   double* sv2, double* vmax2) {
  uint32_t h = blockIdx.x * blockDim.x + threadIdx.x;
  if (h >= nseg) return;
  uint32_t n = start[h + 1] - start[h];
  if (n == 0) {
    sv2[h] = 0.0;
    vmax2[h] = 0.0;
    return;
  }
  const I128* s = acc + 4 * (size_t)h;
  double nn = (double)n;
  double mq[3];
  for (int c = 0; c < 3; ++c) mq[c] = i128_to_f64(s[c]) / nn;
  double s2q = i128_to_f64(s[3]) / nn;
  double t = mq[0] * mq[0];
  t = __fma_rn(mq[1], mq[1], t);
  t = __fma_rn(mq[2], mq[2], t);
  double vq = s2q - t;
  if (!(vq > 0.0)) vq = 0.0;
  sv2[h] = ldexp(vq, -2 * kVelShift);
  vmax2[h] = Gm * sqrt(__longlong_as_double((long long)vm[h]));
}

}  // namespace

size_t radial_bytes(int64_t m, int64_t nseg) {
  size_t b = 0;
  auto add = [&](size_t x) { b += (x + 255) & ~size_t(255); };
  add(4 * m); add(4 * m);                 // seg, pidx
  add(4 * m); add(4 * m); add(8 * m);     // sorted
  add(4 * (nseg + 2));                    // start
  add(4 * m);                             // s_e
  add(4 * m); add(4 * m); add(4 * m); add(4 * m);
  add(8 * m);                             // r2
  add(radix_tmp_bytes(m));
  add(4 * scan_tmp_elems<uint32_t>(m + nseg + 2));
  return b;
}

RadialBufs radial_take(Arena& A, int64_t m, int64_t nseg) {
  RadialBufs b;
  b.seg = A.take<uint32_t>(m);
  b.pidx = A.take<uint32_t>(m);
  b.s_seg = A.take<uint32_t>(m);
  b.s_pidx = A.take<uint32_t>(m);
  b.s_r2 = A.take<double>(m);
  b.start = A.take<uint32_t>(nseg + 2);
  b.s_e = A.take<uint32_t>(m);
  b.va = A.take<uint32_t>(m);
  b.vb = A.take<uint32_t>(m);
  b.k32a = A.take<uint32_t>(m);
  b.k32b = A.take<uint32_t>(m);
  b.r2 = A.take<double>(m);
  b.rtmp = A.take<char>(radix_tmp_bytes(m));
  b.stmp = A.take<uint32_t>(scan_tmp_elems<uint32_t>(m + nseg + 2));
  return b;
}

void radial_sort(int pos_dtype, const void* x, const void* y, const void* z, double box,
                 const double* cx, const double* cy, const double* cz, int64_t m,
                 int64_t nseg, RadialBufs& b, hipStream_t s) {
  if (m == 0) {
    k_fill_u32<<<blocks_for(nseg + 1, TB), TB, 0, s>>>(b.start, nseg + 1, 0u);
    return;
  }
  if (pos_dtype == LIBHALO_F64)
    k_r2<double><<<blocks_for(m, TB), TB, 0, s>>>((const double*)x, (const double*)y,
                                                  (const double*)z, box, cx, cy, cz, b.seg,
                                                  b.pidx, (uint32_t)m, b.r2, b.k32a, b.va);
  else
    k_r2<float><<<blocks_for(m, TB), TB, 0, s>>>((const float*)x, (const float*)y,
                                                 (const float*)z, box, cx, cy, cz, b.seg,
                                                 b.pidx, (uint32_t)m, b.r2, b.k32a, b.va);
  // by FP32-rounded r^2 (non-negative floats order as their bit patterns), then
  // stably by segment; equal keys keep the input order until k_radial_fix
  bool f1 = radix_sort_pairs<uint32_t>(b.k32a, b.va, b.k32b, b.vb, m, 32, b.rtmp, s);
  uint32_t* p1 = f1 ? b.vb : b.va;
  uint32_t* p1o = f1 ? b.va : b.vb;
  k_seg_keys<<<blocks_for(m, TB), TB, 0, s>>>(b.seg, p1, (uint32_t)m, b.k32a);
  bool f2 = radix_sort_pairs<uint32_t>(b.k32a, p1, b.k32b, p1o, m,
                                       bits_for((uint64_t)(nseg > 0 ? nseg - 1 : 0)), b.rtmp,
                                       s);
  uint32_t* perm = f2 ? p1o : p1;
  uint32_t* skey = f2 ? b.k32b : b.k32a;
  k_seg_starts<<<blocks_for(nseg + 1, TB), TB, 0, s>>>(skey, (uint32_t)m, (uint32_t)nseg,
                                                       b.start);
  k_radial_out<<<blocks_for(m, TB), TB, 0, s>>>(perm, b.seg, b.pidx, b.r2, (uint32_t)m,
                                                b.s_seg, b.s_pidx, b.s_r2, b.s_e);
  k_radial_fix<<<blocks_for(m, TB), TB, 0, s>>>(b.s_seg, b.s_pidx, b.s_r2, b.s_e,
                                                (uint32_t)m);
}

void radial_sigma_vmax(const float* vx, const float* vy, const float* vz, int64_t m,
                       int64_t nseg, const RadialBufs& b, double Gm, double eps2, I128* acc,
                       unsigned long long* vm, double* sv2, double* vmax2, hipStream_t s) {
  if (nseg <= 0) return;
  k_zero_sv<<<blocks_for(nseg, TB), TB, 0, s>>>(acc, vm, (uint32_t)nseg);
  if (m > 0)
    k_sigma_vmax_accum<<<blocks_for(m, kSvTB), kSvTB, 0, s>>>(
        vx, vy, vz, b.s_seg, b.s_pidx, b.s_r2, b.start, (uint32_t)m, eps2, acc, vm);
  k_sigma_vmax_final<<<blocks_for(nseg, TB), TB, 0, s>>>(acc, vm, b.start, (uint32_t)nseg, Gm,
                                                         sv2, vmax2);
}

}  // namespace halo
