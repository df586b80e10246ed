// Halo properties from bound particles (Sections 3.5.1-3.5.4) on gfx950:
// centre from the hierarchy, virial spherical overdensity (first downcrossing
// of 360 rho_m), vmax, bulk and core velocities and their offset.
//
// B(h) -- the bound particles of h and of all its subhaloes -- is built as
// (halo, particle) pairs, one per particle and host-chain ancestor, sorted
// by (halo, r^2 from the centre) with the segmented radial sort; every
// property is then an order-free segmented reduction (exact min / max and
// fixed-point sums).
#include <cmath>

#include "extra.hpp"
#include "primitives.hpp"
#include "radial.hpp"
#include "stages.hpp"

namespace halo {

namespace {

constexpr int TB = 256;

__global__ void k_seed_range_init(uint32_t* mn, uint32_t* mx, uint32_t NN) {
  uint32_t k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= NN) return;
  mn[k] = 0xFFFFFFFFu;
  mx[k] = 0u;
}

// Smallest and largest merged halo id among the leaves below each node.
__global__ void k_seed_range(const libhalo_halos h, const libhalo_nodes nd, uint32_t S,
                             uint32_t* mn, uint32_t* mx) {
  uint32_t s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= S) return;
  uint32_t m = (uint32_t)h.merged_into[s];
  for (int32_t k = h.seed_node[s]; k >= 0; k = nd.parent[k]) {
    atomicMin(mn + k, m);
    atomicMax(mx + k, m);
  }
}

__global__ void k_centres(const libhalo_halos h, const libhalo_nodes nd, uint32_t S,
                          const uint32_t* mn, const uint32_t* mx, double* cx, double* cy,
                          double* cz) {
  uint32_t s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= S) return;
  if (h.merged_into[s] != (int32_t)s) {
    cx[s] = cy[s] = cz[s] = 0.0;
    return;
  }
  int32_t k = h.seed_node[s], best = k;
  double bv = nd.sx2[k] / (double)nd.count[k];
  for (int32_t q = nd.parent[k]; q >= 0; q = nd.parent[q]) {
    if (mn[q] != s || mx[q] != s) break;
    double v = nd.sx2[q] / (double)nd.count[q];
    if (v < bv) {
      bv = v;
      best = q;
    }
  }
  cx[s] = nd.cx[best];
  cy[s] = nd.cy[best];
  cz[s] = nd.cz[best];
}

__global__ void k_chain_count(const int32_t* halo_of, const uint8_t* bound,
                              const libhalo_halos h, uint32_t n, uint32_t* cnt) {
  uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  int32_t hh = halo_of[i];
  uint32_t c = 0;
  if (hh >= 0 && bound[i])
    for (int32_t a = hh; a >= 0; a = h.host[a]) ++c;
  cnt[i] = c;
}

__global__ void k_chain_emit(const int32_t* halo_of, const uint8_t* bound, const libhalo_halos h,
                             uint32_t n, const uint32_t* off, uint32_t* seg, uint32_t* pidx) {
  uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  int32_t hh = halo_of[i];
  if (hh < 0 || !bound[i]) return;
  uint32_t o = off[i];
  for (int32_t a = hh; a >= 0; a = h.host[a]) {
    seg[o] = (uint32_t)a;
    pidx[o] = i;
    ++o;
  }
}

__global__ void k_prop_init(uint32_t* kfail, I128* acc, unsigned long long* vm, uint32_t* ncore,
                            uint32_t S) {
  uint32_t s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= S) return;
  kfail[s] = 0xFFFFFFFFu;
  for (int q = 0; q < 6; ++q) acc[6 * (size_t)s + q] = I128{0ull, 0ll};
  vm[s] = 0ull;
  ncore[s] = 0;
}

// First j (1-based) whose enclosed density 3 j m / (4 pi r_j^3) falls below
// rho_vir, tested as r_j^6 > (j C)^2 with C = 3 m / (4 pi rho_vir).  A halo's
// elements are contiguous: one atomic per wave and halo.
__global__ void k_so_fail(const uint32_t* s_seg, const double* s_r2, const uint32_t* start,
                          uint32_t m, double C, uint32_t* kfail) {
  const uint32_t q = blockIdx.x * blockDim.x + threadIdx.x;
  const bool ok = q < m;
  const uint32_t hh = ok ? s_seg[q] : 0u;
  const uint32_t j = ok ? q - start[hh] + 1 : 0u;
  const double r2 = ok ? s_r2[q] : 0.0;
  const double r6 = r2 * r2 * r2;
  const double jc = (double)j * C;
  agg_min_u32(kfail, hh, j, ok && !(r6 <= jc * jc));
}

__global__ void k_so_radius(const uint32_t* kfail, const uint32_t* start, uint32_t S, double C,
                            double core_frac, uint32_t* kstar, double* rvir, double* rc2) {
  uint32_t s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= S) return;
  uint32_t n = start[s + 1] - start[s];
  uint32_t ks = kfail[s] == 0xFFFFFFFFu ? n : kfail[s] - 1;
  kstar[s] = ks;
  double r = cbrt((double)ks * C);
  rvir[s] = r;
  double rc = core_frac * r;
  rc2[s] = rc * rc;
}

constexpr int kSoTB = 1024;

__global__ void __launch_bounds__(kSoTB)
    k_so_accum(const float* vx, const float* vy, const float* vz, const uint32_t* s_seg,
               const uint32_t* s_pidx, const double* s_r2, const uint32_t* start, uint32_t m,
               const uint32_t* kstar, const double* rc2, double eps2, I128* acc,
               unsigned long long* vm, uint32_t* ncore) {
  __shared__ SegMerge<6, kSoTB / 64> L;
  const uint32_t q = blockIdx.x * blockDim.x + threadIdx.x;
  const bool ok = q < m;
  uint32_t hh = 0xFFFFFFFFu;
  I128 v[6];
  for (int c = 0; c < 6; ++c) v[c] = i128_from(0);
  double t = 0.0;
  uint32_t in_core = 0;
  if (ok) {
    hh = s_seg[q];
    const uint32_t i = s_pidx[q];
    const uint32_t j = q - start[hh] + 1;
    const double r2 = s_r2[q];
    const long long w[3] = {quantise((double)vx[i], kVelShift),
                            quantise((double)vy[i], kVelShift),
                            quantise((double)vz[i], kVelShift)};
    if (j <= kstar[hh]) {
      const double jj = (double)j;
      t = (jj * jj) / fmax(r2, eps2);
      for (int c = 0; c < 3; ++c) v[c] = i128_from(w[c]);
    }
    if (r2 < rc2[hh]) {
      in_core = 1;
      for (int c = 0; c < 3; ++c) v[3 + c] = i128_from(w[c]);
    }
  }
  seg_merge_add<6, kSoTB / 64>(L, hh, v, t, in_core, acc, vm, ncore);
}

__global__ void k_prop_out(const libhalo_halos h, uint32_t S, const uint32_t* start,
                           const uint32_t* s_pidx, const float* vx, const float* vy,
                           const float* vz, const uint32_t* kstar, const double* rvir,
                           const I128* acc, const unsigned long long* vm, const uint32_t* ncore,
                           const double* cx, const double* cy, const double* cz, double m,
                           double Gm, libhalo_props_out o) {
  uint32_t s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= S) return;
  const bool kept = h.merged_into[s] == (int32_t)s;
  const uint32_t nb = start[s + 1] - start[s];
  o.px[s] = cx[s];
  o.py[s] = cy[s];
  o.pz[s] = cz[s];
  o.n_bound[s] = kept ? nb : 0u;
  double vb[3] = {0, 0, 0}, vc[3] = {0, 0, 0};
  double mvir = 0, rv = 0, vmax = 0;
  if (kept && nb > 0) {
    const uint32_t ks = kstar[s];
    const uint32_t i0 = s_pidx[start[s]];  // innermost bound particle
    const double v0[3] = {(double)vx[i0], (double)vy[i0], (double)vz[i0]};
    if (ks > 0) {
      for (int c = 0; c < 3; ++c)
        vb[c] = ldexp(i128_to_f64(acc[6 * (size_t)s + c]) / (double)ks, -kVelShift);
      mvir = (double)ks * m;
      rv = rvir[s];
      vmax = sqrt(Gm * sqrt(__longlong_as_double((long long)vm[s])));
    } else {
      for (int c = 0; c < 3; ++c) vb[c] = v0[c];
    }
    if (ncore[s] > 0) {
      for (int c = 0; c < 3; ++c)
        vc[c] = ldexp(i128_to_f64(acc[6 * (size_t)s + 3 + c]) / (double)ncore[s], -kVelShift);
    } else {
      for (int c = 0; c < 3; ++c) vc[c] = v0[c];
    }
  }
  o.vbx[s] = vb[0];
  o.vby[s] = vb[1];
  o.vbz[s] = vb[2];
  o.vcx[s] = vc[0];
  o.vcy[s] = vc[1];
  o.vcz[s] = vc[2];
  o.mvir[s] = mvir;
  o.rvir[s] = rv;
  o.vmax[s] = vmax;
  o.voff[s] = sqrt(sq3(vc[0] - vb[0], vc[1] - vb[1], vc[2] - vb[2]));
}

}  // namespace

void props(Ctx& ctx, int64_t n, int pos_dtype, const void* x, const void* y, const void* z,
           const float* vx, const float* vy, const float* vz, const libhalo_nodes* nodes,
           int64_t n_nodes, const libhalo_halos* halos, int64_t n_halos,
           const int32_t* halo_of, const uint8_t* bound, libhalo_props_out* out,
           hipStream_t s, const ExtraArgs* extra) {
  const libhalo_params& P = ctx.p;
  const libhalo_nodes& nd = *nodes;
  const libhalo_halos& h = *halos;
  const uint32_t S = (uint32_t)n_halos, NN = (uint32_t)n_nodes;
  if (S == 0) return;
  const double C = (3.0 * P.particle_mass) / (4.0 * M_PI * P.rho_vir);
  const double eps2 = P.softening * P.softening;
  const double Gm = P.G * P.particle_mass;
  uint32_t* hb = ctx.host_slot<uint32_t>(0);
  // total pairs: bounded by n times the deepest host chain (checked below)
  struct W {
    uint32_t *mn, *mx, *cnt, *off, *dcnt, *stmp, *kfail, *kstar, *ncore;
    double *cx, *cy, *cz, *rvir, *rc2;
    I128* acc;
    unsigned long long* vm;
  } w;
  // the number of (halo, particle) pairs is known only after a count pass;
  // size the radial buffers for it in a second carve.
  carve_workspace(ctx, [&](Arena& A) {
    w.mn = A.take<uint32_t>(NN + 2);
    w.mx = A.take<uint32_t>(NN + 2);
    w.cnt = A.take<uint32_t>(n + 2);
    w.off = A.take<uint32_t>(n + 2);
    w.dcnt = A.take<uint32_t>(16);
    w.stmp = A.take<uint32_t>(scan_tmp_elems<uint32_t>(n + 2));
  });
  k_chain_count<<<blocks_for(n, TB), TB, 0, s>>>(halo_of, bound, h, (uint32_t)n, w.cnt);
  exclusive_scan<uint32_t>(w.cnt, w.off, n, w.dcnt, w.stmp, s);
  HALO_HIP(hipMemcpyAsync(hb, w.dcnt, 4, hipMemcpyDeviceToHost, s));
  HALO_HIP(hipStreamSynchronize(s));
  const uint32_t m = hb[0];
  RadialBufs rb;
  ExtraBufs eb{};
  carve_workspace(ctx, [&](Arena& A) {
    w.mn = A.take<uint32_t>(NN + 2);
    w.mx = A.take<uint32_t>(NN + 2);
    w.cnt = A.take<uint32_t>(n + 2);
    w.off = A.take<uint32_t>(n + 2);
    w.dcnt = A.take<uint32_t>(16);
    w.stmp = A.take<uint32_t>(scan_tmp_elems<uint32_t>(n + 2));
    w.kfail = A.take<uint32_t>(S + 2);
    w.kstar = A.take<uint32_t>(S + 2);
    w.ncore = A.take<uint32_t>(S + 2);
    w.cx = A.take<double>(S + 2);
    w.cy = A.take<double>(S + 2);
    w.cz = A.take<double>(S + 2);
    w.rvir = A.take<double>(S + 2);
    w.rc2 = A.take<double>(S + 2);
    w.acc = A.take<I128>(6ull * (S + 2));
    w.vm = A.take<unsigned long long>(S + 2);
    rb = radial_take(A, std::max<uint32_t>(m, 1), S + 2);
    if (extra) eb = extra_take(A, S, m, extra->n_so);
  });
  // the second carve may have moved the workspace: redo the pair offsets
  k_chain_count<<<blocks_for(n, TB), TB, 0, s>>>(halo_of, bound, h, (uint32_t)n, w.cnt);
  exclusive_scan<uint32_t>(w.cnt, w.off, n, w.dcnt, w.stmp, s);
  k_seed_range_init<<<blocks_for(NN, TB), TB, 0, s>>>(w.mn, w.mx, NN);
  k_seed_range<<<blocks_for(S, TB), TB, 0, s>>>(h, nd, S, w.mn, w.mx);
  k_centres<<<blocks_for(S, TB), TB, 0, s>>>(h, nd, S, w.mn, w.mx, w.cx, w.cy, w.cz);
  k_chain_emit<<<blocks_for(n, TB), TB, 0, s>>>(halo_of, bound, h, (uint32_t)n, w.off, rb.seg,
                                                rb.pidx);
  radial_sort(pos_dtype, x, y, z, P.box, w.cx, w.cy, w.cz, m, S, rb, s);
  k_prop_init<<<blocks_for(S, TB), TB, 0, s>>>(w.kfail, w.acc, w.vm, w.ncore, S);
  if (m > 0)
    k_so_fail<<<blocks_for(m, TB), TB, 0, s>>>(rb.s_seg, rb.s_r2, rb.start, m, C, w.kfail);
  k_so_radius<<<blocks_for(S, TB), TB, 0, s>>>(w.kfail, rb.start, S, C, P.core_frac, w.kstar,
                                               w.rvir, w.rc2);
  if (m > 0)
    k_so_accum<<<blocks_for(m, kSoTB), kSoTB, 0, s>>>(vx, vy, vz, rb.s_seg, rb.s_pidx, rb.s_r2,
                                                rb.start, m, w.kstar, w.rc2, eps2, w.acc, w.vm,
                                                w.ncore);
  k_prop_out<<<blocks_for(S, TB), TB, 0, s>>>(h, S, rb.start, rb.s_pidx, vx, vy, vz, w.kstar,
                                              w.rvir, w.acc, w.vm, w.ncore, w.cx, w.cy, w.cz,
                                              P.particle_mass, Gm, *out);
  if (extra)
    props_extra_run(ctx, *extra, eb, pos_dtype, x, y, z, vx, vy, vz, halo_of, h, S, rb, m,
                    w.kstar, *out, s);
  HALO_HIP(hipStreamSynchronize(s));
}

}  // namespace halo
