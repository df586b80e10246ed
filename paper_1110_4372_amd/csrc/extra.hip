// Additional halo properties on gfx950 (Sections 3.5.2 and 3.5.4).
//
// V(h), the set behind M_vir, is the prefix of length k* of the halo's
// segment in the radially sorted list that the basic properties build.  Over
// it, one segmented pass sums (in 128-bit fixed point, so the result does not
// depend on scheduling) the offsets from the centre, the angular momentum,
// |v - v_bulk|^2 and, over the halo's own particles, the Eq. 11 tensor.  The
// potential energy is a triangular pair sum per halo, FP64, one wavefront per
// 256 particles against 2048-particle chunks.  A last per-halo pass derives
// the spins (Eqs. 9-10), the Klypin concentration (Eqs. 7-8, bisection), the
// axis ratios (Jacobi eigenvalues of the 3x3 tensor) and the SO masses at the
// further thresholds (first downcrossing, as for M_vir).
#include <cmath>

#include "extra.hpp"
#include "lanes.hpp"
#include "primitives.hpp"

namespace halo {

namespace {

constexpr int TB = 256;
constexpr int kAccTB = 1024;
constexpr int kExtraSums = 13;  // 3 offsets, 3 angular momentum, 1 kinetic, 6 tensor

// Pair-energy work unit: kEI particles of V(h) (four wavefronts, kEK per
// lane) against a chunk of kEJ particles.
constexpr uint32_t kEK = 4;
constexpr uint32_t kETile = 64 * kEK;
constexpr uint32_t kEI = 4 * kETile;
constexpr uint32_t kEJ = 2048;
constexpr int kEFrac = 32;        // fractional bits of the pair-sum accumulators
constexpr unsigned kEGrid = 2048; // blocks of the pair kernel (grid-stride over units)

// Klypin concentration (Eqs. 5-8): NFW radius of v_max in units of R_s as the
// paper prints it, and the upper clamp of the root.
constexpr double kKlypinX = 2.1626;
constexpr double kKlypinCMax = 1.0e4;

struct SoThresholds {
  double C[LIBHALO_MAX_SO];  // 3 m / (4 pi rho_t)
  int n;
};

struct Shifts {
  int x, j, t, q;  // fixed-point fractions of offsets, J terms, |dv|^2, tensor terms
};

// Fractions keeping every quantised term below 2^62 (64-bit terms: |dx| <=
// L/2, each velocity component below 2^17 km/s after the bulk is removed),
// and the tensor's below 2^93 (128-bit terms, so that the sum of 2^32 of them
// still fits): its small eigenvalues are differences of its entries, which
// need the finer grid.
Shifts shifts_for(double box) {
  const int lh = (int)std::ceil(std::log2(0.5 * box));
  Shifts s;
  s.x = 62 - lh;
  s.j = 62 - (lh + 1 + 17);
  s.t = 62 - 36;
  s.q = 93 - 2 * lh;
  return s;
}

// round(v 2^frac) for 0 <= v 2^frac < 2^94 as a 128-bit integer: s is an
// integer; its 2^64 and 2^32 words are split off exactly by floor and fma.
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

// round(v 2^frac) for |v| 2^frac < 2^94, signed.
__device__ __forceinline__ I128 fixed128_signed(double v, int frac) {
  const I128 a = fixed128(fabs(v), frac);
  if (v >= 0.0) return a;
  I128 r;  // two's complement negation
  r.lo = ~a.lo + 1ull;
  r.hi = (long long)(~(unsigned long long)a.hi + (r.lo == 0ull ? 1ull : 0ull));
  return r;
}

__global__ void k_extra_init(I128* acc, I128* accU, uint32_t* nown, uint32_t* kfail,
                             uint32_t S, int n_so) {
  const uint32_t s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= S) return;
  for (int c = 0; c < kExtraSums; ++c) acc[kExtraSums * (size_t)s + c] = I128{0ull, 0ll};
  accU[s] = I128{0ull, 0ll};
  nown[s] = 0u;
  for (int t = 0; t < n_so; ++t) kfail[(size_t)t * S + s] = 0xFFFFFFFFu;
}

// First j (1-based) of each halo's sorted bound list whose enclosed density
// falls below threshold t: r_j^6 > (j C_t)^2.  Elements of one halo are
// contiguous, so a wave sends one atomic per halo and threshold.
__global__ void k_so_fail_multi(const uint32_t* s_seg, const double* s_r2,
                                const uint32_t* start, uint32_t m, uint32_t S,
                                SoThresholds th, uint32_t* kfail) {
  const uint32_t q = blockIdx.x * blockDim.x + threadIdx.x;
  const bool ok = q < m;
  const uint32_t hh = ok ? s_seg[q] : 0u;
  const uint32_t j = ok ? q - start[hh] + 1 : 0u;
  const double r2 = ok ? s_r2[q] : 0.0;
  const double r6 = r2 * r2 * r2;
  for (int t = 0; t < th.n; ++t) {
    const double jc = (double)j * th.C[t];
    agg_min_u32(kfail + (size_t)t * S, hh, j, ok && !(r6 <= jc * jc));
  }
}

// One element of the sorted list per thread: the sums over V(h), and the
// FP64 offsets from the centre of V(h)'s particles for the pair pass.
template <class T>
__global__ void __launch_bounds__(kAccTB)
    k_extra_accum(const T* x, const T* y, const T* z, double box, const float* vx,
                  const float* vy, const float* vz, const int32_t* halo_of,
                  const uint32_t* s_seg, const uint32_t* s_pidx, const uint32_t* start,
                  uint32_t m, const uint32_t* kstar, const libhalo_props_out o, Shifts sh,
                  I128* acc, uint32_t* nown, double* ux, double* uy, double* uz) {
  __shared__ SegMerge<kExtraSums, kAccTB / 64> L;
  const uint32_t q = blockIdx.x * blockDim.x + threadIdx.x;
  uint32_t hh = 0xFFFFFFFFu, own = 0;
  I128 v[kExtraSums];
  for (int c = 0; c < kExtraSums; ++c) v[c] = i128_from(0);
  if (q < m) {
    hh = s_seg[q];
    const uint32_t j = q - start[hh] + 1;
    if (j <= kstar[hh]) {
      const uint32_t i = s_pidx[q];
      const double dx = min_image(ld_pos(x, i) - o.px[hh], box);
      const double dy = min_image(ld_pos(y, i) - o.py[hh], box);
      const double dz = min_image(ld_pos(z, i) - o.pz[hh], box);
      ux[q] = dx;
      uy[q] = dy;
      uz[q] = dz;
      const double wx = (double)vx[i] - o.vbx[hh];
      const double wy = (double)vy[i] - o.vby[hh];
      const double wz = (double)vz[i] - o.vbz[hh];
      v[0] = i128_from(quantise(dx, sh.x));
      v[1] = i128_from(quantise(dy, sh.x));
      v[2] = i128_from(quantise(dz, sh.x));
      v[3] = i128_from(quantise(dy * wz - dz * wy, sh.j));
      v[4] = i128_from(quantise(dz * wx - dx * wz, sh.j));
      v[5] = i128_from(quantise(dx * wy - dy * wx, sh.j));
      v[6] = i128_from(quantise(sq3(wx, wy, wz), sh.t));
      if (halo_of[i] == (int32_t)hh) {
        own = 1;
        v[7] = fixed128_signed(dx * dx, sh.q);
        v[8] = fixed128_signed(dy * dy, sh.q);
        v[9] = fixed128_signed(dz * dz, sh.q);
        v[10] = fixed128_signed(dx * dy, sh.q);
        v[11] = fixed128_signed(dx * dz, sh.q);
        v[12] = fixed128_signed(dy * dz, sh.q);
      }
    }
  }
  seg_merge_add<kExtraSums, kAccTB / 64>(L, hh, v, 0.0, own, acc, nullptr, nown);
}

// Units of each kept halo with |V(h)| >= 2 (entry S stays 0 for the scan).
__global__ void k_energy_counts(const libhalo_halos h, const uint32_t* kstar, uint32_t S,
                                uint32_t* ucnt) {
  const uint32_t s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s > S) return;
  uint32_t u = 0;
  if (s < S && h.merged_into[s] == (int32_t)s && kstar[s] >= 2) {
    const uint32_t k = kstar[s];
    u = ((k + kEI - 1) / kEI) * ((k + kEJ - 1) / kEJ);
  }
  ucnt[s] = u;
}

// The halo owning unit u: the largest s with uoff[s] <= u.
__device__ __forceinline__ uint32_t unit_halo(const uint32_t* uoff, uint32_t S, uint32_t u) {
  uint32_t lo = 0, hi = S;
  while (hi - lo > 1) {
    const uint32_t mid = (lo + hi) >> 1;
    if (uoff[mid] <= u)
      lo = mid;
    else
      hi = mid;
  }
  return lo;
}

// Doubled pair term 2/sqrt(r^2 + eps^2) as c y: y the hardware rsqrt
// estimate, c = 3 - r y^2 (one Newton step, halved when the sums convert).
__device__ __forceinline__ void energy_term2(double bx, double by, double bz, double x,
                                             double y, double z, double eps2, double& c,
                                             double& r0) {
  const double dx = bx - x, dy = by - y, dz = bz - z;
  const double r = __fma_rn(dz, dz, __fma_rn(dy, dy, __fma_rn(dx, dx, eps2)));
  r0 = __builtin_amdgcn_rsq(r);
  c = __fma_rn(-(r * r0), r0, 3.0);
}

// Sum over the pairs i < j of V(h) of 1/sqrt(r_ij^2 + eps^2).  A wave takes
// the 256 particles i of its tile against j >= its tile start: inside the
// tile only j > i counts, beyond it every pair.  The wave's FP64 total (fixed
// loop order, fixed lane tree) goes to the halo in fixed point.
__global__ void __launch_bounds__(TB, 4)
    k_pair_energy(const double* __restrict__ ux, const double* __restrict__ uy,
                  const double* __restrict__ uz, const uint32_t* __restrict__ start,
                  const uint32_t* __restrict__ kstar, const uint32_t* __restrict__ uoff,
                  uint32_t S, double eps2, I128* __restrict__ accU) {
  const uint32_t total = uoff[S];
  const uint32_t lane = threadIdx.x & 63u;
  for (uint32_t u0 = blockIdx.x; u0 < total; u0 += gridDim.x) {
    const uint32_t u = __builtin_amdgcn_readfirstlane(u0);
    const uint32_t hh = unit_halo(uoff, S, u);
    const uint32_t k = kstar[hh];
    const uint32_t b0 = start[hh];
    const uint32_t nb = (k + kEI - 1) / kEI;
    const uint32_t local = u - uoff[hh];
    const uint32_t c = local / nb;
    const uint32_t t0 =
        __builtin_amdgcn_readfirstlane((local - c * nb) * kEI + (threadIdx.x >> 6) * kETile);
    const uint32_t j0 = c * kEJ;
    const uint32_t j1 = min(j0 + kEJ, k);
    if (t0 >= k || j1 <= t0 + 1) continue;  // wave-uniform: no pair i < j here
    uint32_t li[kEK];
    double x[kEK], y[kEK], z[kEK], A[kEK];
#pragma unroll
    for (uint32_t e = 0; e < kEK; ++e) {
      li[e] = t0 + lane + 64u * e;
      const bool ok = li[e] < k;
      const uint32_t qi = b0 + (ok ? li[e] : 0u);
      x[e] = ok ? ux[qi] : 0.0;
      y[e] = ok ? uy[qi] : 0.0;
      z[e] = ok ? uz[qi] : 0.0;
      A[e] = 0.0;
    }
    // inside the tile: j > i only (also drops the empty slots i >= k > j)
    const uint32_t ja = max(j0, t0), jb = min(j1, t0 + kETile);
    for (uint32_t j = ja; j < jb; ++j) {
      const double bx = ux[b0 + j], by = uy[b0 + j], bz = uz[b0 + j];
#pragma unroll
      for (uint32_t e = 0; e < kEK; ++e) {
        double cc, r0;
        energy_term2(bx, by, bz, x[e], y[e], z[e], eps2, cc, r0);
        A[e] = __fma_rn(cc, j > li[e] ? r0 : 0.0, A[e]);
      }
    }
    // beyond the tile: every slot holds a particle i < j
    uint32_t j = max(j0, t0 + kETile);
    for (; j + 4 <= j1; j += 4) {
      double bx[4], by[4], bz[4];
      const double* __restrict__ px = ux + b0 + j;
      const double* __restrict__ py = uy + b0 + j;
      const double* __restrict__ pz = uz + b0 + j;
#pragma unroll
      for (int w = 0; w < 4; ++w) {
        bx[w] = px[w];
        by[w] = py[w];
        bz[w] = pz[w];
      }
#pragma unroll
      for (int w = 0; w < 4; ++w)
#pragma unroll
        for (uint32_t e = 0; e < kEK; ++e) {
          double cc, r0;
          energy_term2(bx[w], by[w], bz[w], x[e], y[e], z[e], eps2, cc, r0);
          A[e] = __fma_rn(cc, r0, A[e]);
        }
    }
    for (; j < j1; ++j)
#pragma unroll
      for (uint32_t e = 0; e < kEK; ++e) {
        double cc, r0;
        energy_term2(ux[b0 + j], uy[b0 + j], uz[b0 + j], x[e], y[e], z[e], eps2, cc, r0);
        A[e] = __fma_rn(cc, r0, A[e]);
      }
    double t = (A[0] + A[1]) + (A[2] + A[3]);
    t = t + lane_xor_f64<lane_xor1>(t);
    t = t + lane_xor_f64<lane_xor2>(t);
    t = t + lane_xor_f64<lane_xor4>(t);
    t = t + lane_xor_f64<lane_xor8>(t);
    t = t + lane_xor_f64<lane_xor16>(t);
    t = t + lane_xor_f64<lane_xor32>(t);
    if (lane == 0 && t > 0.0) atomic_add_i128(accU + hh, fixed128(0.5 * t, kEFrac));
  }
}

__device__ __forceinline__ double nfw_f(double x) { return log1p(x) - x / (1.0 + x); }

// Root c >= X of c / f(c) = rhs by bisection to adjacent doubles, clamped to
// [X, kKlypinCMax] (c / f(c) increases on that branch).
__device__ double klypin_c(double vmax, double mvir, double rvir, double G) {
  if (!(mvir > 0.0 && rvir > 0.0 && vmax > 0.0)) return 0.0;
  const double rhs = vmax * vmax * rvir / (G * mvir) * (kKlypinX / nfw_f(kKlypinX));
  if (kKlypinX / nfw_f(kKlypinX) - rhs >= 0.0) return kKlypinX;
  if (kKlypinCMax / nfw_f(kKlypinCMax) - rhs <= 0.0) return kKlypinCMax;
  double lo = kKlypinX, hi = kKlypinCMax;
  for (int it = 0; it < 200; ++it) {
    const double mid = 0.5 * (lo + hi);
    if (mid <= lo || mid >= hi) break;
    if (mid / nfw_f(mid) - rhs < 0.0)
      lo = mid;
    else
      hi = mid;
  }
  return 0.5 * (lo + hi);
}

// Eigenvalues (descending) and the leading eigenvector of a symmetric 3x3
// matrix by cyclic Jacobi rotations (Golub & Van Loan, symmetric Schur
// decomposition of 2x2 blocks).
__device__ void sym3_eigen(double a[3][3], double w[3], double e1[3]) {
  double V[3][3] = {{1, 0, 0}, {0, 1, 0}, {0, 0, 1}};
  for (int sweep = 0; sweep < 50; ++sweep) {
    const double off = a[0][1] * a[0][1] + a[0][2] * a[0][2] + a[1][2] * a[1][2];
    const double dia = a[0][0] * a[0][0] + a[1][1] * a[1][1] + a[2][2] * a[2][2];
    if (!(off > 1e-36 * dia)) break;
    for (int pq = 0; pq < 3; ++pq) {
      const int p = pq == 2 ? 1 : 0, q = pq == 0 ? 1 : 2;
      if (a[p][q] == 0.0) continue;
      const double theta = (a[q][q] - a[p][p]) / (2.0 * a[p][q]);
      const double t = (theta >= 0.0 ? 1.0 : -1.0) / (fabs(theta) + sqrt(theta * theta + 1.0));
      const double c = 1.0 / sqrt(t * t + 1.0), s = t * c;
      for (int r = 0; r < 3; ++r) {  // columns p, q of a J
        const double arp = a[r][p], arq = a[r][q];
        a[r][p] = c * arp - s * arq;
        a[r][q] = s * arp + c * arq;
      }
      for (int r = 0; r < 3; ++r) {  // rows p, q of J^T (a J)
        const double apr = a[p][r], aqr = a[q][r];
        a[p][r] = c * apr - s * aqr;
        a[q][r] = s * apr + c * aqr;
      }
      for (int r = 0; r < 3; ++r) {
        const double vrp = V[r][p], vrq = V[r][q];
        V[r][p] = c * vrp - s * vrq;
        V[r][q] = s * vrp + c * vrq;
      }
    }
  }
  int idx[3] = {0, 1, 2};
  for (int i = 0; i < 3; ++i)
    for (int j = i + 1; j < 3; ++j)
      if (a[idx[j]][idx[j]] > a[idx[i]][idx[i]]) {
        const int t = idx[i];
        idx[i] = idx[j];
        idx[j] = t;
      }
  for (int i = 0; i < 3; ++i) w[i] = fmax(a[idx[i]][idx[i]], 0.0);
  for (int r = 0; r < 3; ++r) e1[r] = V[r][idx[0]];
}

__global__ void k_extra_out(const libhalo_halos h, uint32_t S, const uint32_t* start,
                            const uint32_t* kstar, const I128* acc, const I128* accU,
                            const uint32_t* nown, const uint32_t* kfail, SoThresholds th,
                            const libhalo_props_out o, Shifts sh, double m, double G,
                            libhalo_props_extra_out e) {
  const uint32_t s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= S) return;
  const bool kept = h.merged_into[s] == (int32_t)s;
  const uint32_t k = kept ? kstar[s] : 0u;
  const I128* a = acc + kExtraSums * (size_t)s;
  double xoff = 0, J[3] = {0, 0, 0}, T = 0, U = 0, tu = 0, spin = 0, spinb = 0, ck = 0, rs = 0;
  double ba = 0, ca = 0, A[3] = {0, 0, 0};
  uint32_t nsh = 0;
  if (k > 0) {
    const double kd = (double)k;
    const double cm[3] = {ldexp(i128_to_f64(a[0]), -sh.x) / kd,
                          ldexp(i128_to_f64(a[1]), -sh.x) / kd,
                          ldexp(i128_to_f64(a[2]), -sh.x) / kd};
    xoff = sqrt(sq3(cm[0], cm[1], cm[2]));
    for (int c = 0; c < 3; ++c) J[c] = m * ldexp(i128_to_f64(a[3 + c]), -sh.j);
    T = 0.5 * m * ldexp(i128_to_f64(a[6]), -sh.t);
    U = -G * m * m * ldexp(i128_to_f64(accU[s]), -kEFrac);
    tu = U != 0.0 ? T / fabs(U) : 0.0;
    const double M = o.mvir[s], R = o.rvir[s];
    const double Jm = sqrt(sq3(J[0], J[1], J[2]));
    if (M > 0.0) {
      spin = Jm * sqrt(fabs(T + U)) / (G * M * M * sqrt(M));
      if (R > 0.0) spinb = Jm / sqrt(2.0 * G * M * M * M * R);
    }
    ck = klypin_c(o.vmax[s], M, R, G);
    rs = ck > 0.0 ? R / ck : 0.0;
    nsh = nown[s];
    if (nsh > 0) {
      const double nd = (double)nsh;
      double q[6];
      for (int c = 0; c < 6; ++c) q[c] = ldexp(i128_to_f64(a[7 + c]), -sh.q) / nd;
      double M3[3][3] = {{q[0], q[3], q[4]}, {q[3], q[1], q[5]}, {q[4], q[5], q[2]}};
      double w[3], ev[3];
      sym3_eigen(M3, w, ev);
      if (w[0] > 0.0) {
        ba = sqrt(w[1] / w[0]);
        ca = sqrt(w[2] / w[0]);
        int im = 0;
        for (int c = 1; c < 3; ++c)
          if (fabs(ev[c]) > fabs(ev[im])) im = c;
        const double sg = ev[im] < 0.0 ? -1.0 : 1.0;
        const double al = sqrt(w[0]);
        for (int c = 0; c < 3; ++c) A[c] = sg * al * ev[c];
      }
    }
  }
  e.xoff[s] = xoff;
  e.jx[s] = J[0];
  e.jy[s] = J[1];
  e.jz[s] = J[2];
  e.kin[s] = T;
  e.pot[s] = U;
  e.t_u[s] = tu;
  e.spin[s] = spin;
  e.spin_bullock[s] = spinb;
  e.c_klypin[s] = ck;
  e.rs_klypin[s] = rs;
  e.b_to_a[s] = ba;
  e.c_to_a[s] = ca;
  e.ax[s] = A[0];
  e.ay[s] = A[1];
  e.az[s] = A[2];
  e.n_shape[s] = nsh;
  const uint32_t nb = start[s + 1] - start[s];
  for (int t = 0; t < th.n; ++t) {
    const uint32_t f = kfail[(size_t)t * S + s];
    const uint32_t kt = !kept ? 0u : (f == 0xFFFFFFFFu ? nb : f - 1u);
    e.m_so[(size_t)t * e.cap + s] = (double)kt * m;
    e.r_so[(size_t)t * e.cap + s] = cbrt((double)kt * th.C[t]);
  }
}

}  // namespace

ExtraBufs extra_take(Arena& A, uint32_t S, uint32_t m, int n_so) {
  ExtraBufs b;
  b.acc = A.take<I128>((size_t)kExtraSums * (S + 2));
  b.accU = A.take<I128>(S + 2);
  b.nown = A.take<uint32_t>(S + 2);
  b.kfail = A.take<uint32_t>((size_t)std::max(n_so, 1) * (S + 2));
  b.ucnt = A.take<uint32_t>(S + 2);
  b.uoff = A.take<uint32_t>(S + 2);
  b.total = A.take<uint32_t>(16);
  b.stmp = A.take<uint32_t>(scan_tmp_elems<uint32_t>(S + 2));
  b.ux = A.take<double>(std::max<uint32_t>(m, 1));
  b.uy = A.take<double>(std::max<uint32_t>(m, 1));
  b.uz = A.take<double>(std::max<uint32_t>(m, 1));
  return b;
}

void props_extra_run(Ctx& ctx, const ExtraArgs& ea, const ExtraBufs& eb, int pos_dtype,
                     const void* x, const void* y, const void* z, const float* vx,
                     const float* vy, const float* vz, const int32_t* halo_of,
                     const libhalo_halos& h, uint32_t S, const RadialBufs& rb, uint32_t m,
                     const uint32_t* kstar, const libhalo_props_out& out, hipStream_t s) {
  const libhalo_params& P = ctx.p;
  const double mp = P.particle_mass;
  SoThresholds th{};
  th.n = ea.n_so;
  for (int t = 0; t < ea.n_so; ++t) th.C[t] = (3.0 * mp) / (4.0 * M_PI * ea.rho[t]);
  const Shifts sh = shifts_for(P.box);
  k_extra_init<<<blocks_for(S, TB), TB, 0, s>>>(eb.acc, eb.accU, eb.nown, eb.kfail, S,
                                                 ea.n_so);
  if (m > 0) {
    if (ea.n_so > 0)
      k_so_fail_multi<<<blocks_for(m, TB), TB, 0, s>>>(rb.s_seg, rb.s_r2, rb.start, m, S, th,
                                                       eb.kfail);
    if (pos_dtype == LIBHALO_F64)
      k_extra_accum<double><<<blocks_for(m, kAccTB), kAccTB, 0, s>>>(
          (const double*)x, (const double*)y, (const double*)z, P.box, vx, vy, vz, halo_of,
          rb.s_seg, rb.s_pidx, rb.start, m, kstar, out, sh, eb.acc, eb.nown, eb.ux, eb.uy,
          eb.uz);
    else
      k_extra_accum<float><<<blocks_for(m, kAccTB), kAccTB, 0, s>>>(
          (const float*)x, (const float*)y, (const float*)z, P.box, vx, vy, vz, halo_of,
          rb.s_seg, rb.s_pidx, rb.start, m, kstar, out, sh, eb.acc, eb.nown, eb.ux, eb.uy,
          eb.uz);
    k_energy_counts<<<blocks_for(S + 1, TB), TB, 0, s>>>(h, kstar, S, eb.ucnt);
    exclusive_scan<uint32_t>(eb.ucnt, eb.uoff, S + 1, eb.total, eb.stmp, s);
    const double eps2 = P.softening * P.softening;
    HALO_PROF(ctx, "k_pair_energy", s,
              k_pair_energy<<<kEGrid, TB, 0, s>>>(eb.ux, eb.uy, eb.uz, rb.start, kstar, eb.uoff,
                                                  S, eps2, eb.accU));
  }
  k_extra_out<<<blocks_for(S, TB), TB, 0, s>>>(h, S, rb.start, kstar, eb.acc, eb.accU, eb.nown,
                                               eb.kfail, th, out, sh, mp, P.G, *ea.ext);
  HALO_HIP(hipGetLastError());
}

}  // namespace halo
