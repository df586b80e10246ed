// C ABI of libhalo: context, parameter validation, error capture, dispatch.
#include <cmath>
#include <cstring>
#include <mutex>
#include <new>
#include <vector>

#include "common.hpp"
#include "fof3d.hpp"
#include "extra.hpp"
#include "stages.hpp"

struct libhalo_ctx {
  halo::Ctx c;
};

namespace halo {

// Fixed device scratch of the no-alloc entry point: one copy per device that
// loads the library, held until the process ends.  Host code never uses the
// array's name as an address: each device's copy is looked up once, with that
// device current, and kept in scratch_dev.
constexpr size_t kScratchBytes = size_t(LIBHALO_NOALLOC_SCRATCH_BYTES);
static __device__ __align__(256) char scratch[kScratchBytes];

static std::mutex scratch_mu;
static std::vector<void*> scratch_dev;  // per device, null until looked up

// The calling thread's current device is `device`.
static hipError_t scratch_setup(int device, void** out) {
  std::lock_guard<std::mutex> lk(scratch_mu);
  if ((int)scratch_dev.size() <= device) scratch_dev.resize(device + 1, nullptr);
  if (!scratch_dev[device]) {
    void* ptr = nullptr;
    hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    scratch_dev[device] = ptr;
  }
  *out = scratch_dev[device];
  return hipSuccess;
}

void* Ctx::dev_alloc(size_t bytes, const char* what) {
  void* p = alloc_fn(bytes, user, (void*)stream);
  if (!p)
    throw Error{LIBHALO_ENOMEM, std::string(what) + " of " + std::to_string(bytes) +
                                    " bytes: the allocator returned NULL"};
  HALO_CHECK((reinterpret_cast<uintptr_t>(p) & 255u) == 0, LIBHALO_EINVAL,
             "the allocator returned memory not aligned to 256 bytes");
  return p;
}

// A workspace grows by returning the old block (once the stream's work on it
// is done) and taking a larger one, with an eighth of slack.
static void grow(Ctx& c, Arena& a, size_t bytes, const char* what) {
  if (bytes <= a.cap) return;
  if (a.base) {
    HALO_HIP(hipStreamSynchronize(c.stream));
    c.free_fn(a.base, c.user, (void*)c.stream);
    a.base = nullptr;
    a.cap = 0;
  }
  const size_t want = bytes + bytes / 8;
  a.base = static_cast<char*>(c.dev_alloc(want, what));
  a.cap = want;
}

void Ctx::ensure_ws(size_t bytes) { grow(*this, ws, bytes, "workspace"); }

void Ctx::ensure_ws2(size_t bytes) { grow(*this, ws2, bytes, "tree workspace"); }

hipEvent_t Ctx::event() {
  if (!spare.empty()) {
    hipEvent_t e = spare.back();
    spare.pop_back();
    return e;
  }
  hipEvent_t e;
  HALO_HIP(hipEventCreate(&e));
  return e;
}

void Ctx::release() {
  for (auto& r : recs) {
    (void)hipEventDestroy(r.e0);
    (void)hipEventDestroy(r.e1);
  }
  for (auto e : spare) (void)hipEventDestroy(e);
  recs.clear();
  spare.clear();
  // the caller has synchronised the device: every block is idle
  if (ws.base) free_fn(ws.base, user, (void*)stream);
  if (ws2.base) free_fn(ws2.base, user, (void*)stream);
  if (d_err) free_fn(d_err, user, nullptr);
  if (h_pinned) (void)hipHostFree(h_pinned);
  if (ev_fork) (void)hipEventDestroy(ev_fork);
  if (ev_join) (void)hipEventDestroy(ev_join);
  if (side) (void)hipStreamDestroy(side);
  ev_fork = ev_join = nullptr;
  side = nullptr;
  ws.base = ws2.base = nullptr;
  ws.cap = ws2.cap = 0;
  d_err = nullptr;
  h_pinned = nullptr;
}

static std::string validate(const libhalo_params& p) {
  if (!(p.box > 0.0) || !std::isfinite(p.box)) return "box must be positive";
  if (!(p.b > 0.0)) return "b must be positive";
  if (!(p.f > 0.0 && p.f <= 1.0)) return "f must lie in (0, 1]";
  if (p.min_members < 2) return "min_members must be >= 2";
  if (p.max_levels < 1 || p.max_levels > 4096) return "max_levels must lie in [1, 4096]";
  if (!(p.merge_q2 >= 0.0)) return "merge_q2 must be >= 0";
  if (!(p.particle_mass > 0.0)) return "particle_mass must be positive";
  if (!(p.G > 0.0)) return "G must be positive";
  if (!(p.rho_vir > 0.0)) return "rho_vir must be positive";
  if (!(p.softening > 0.0)) return "softening must be positive";
  if (!(p.core_frac > 0.0)) return "core_frac must be positive";
  if (!(p.unbound_threshold >= 0.0 && p.unbound_threshold <= 1.0))
    return "unbound_threshold must lie in [0, 1]";
  if (!(p.major_merger >= 0.0 && std::isfinite(p.major_merger)))
    return "major_merger must be finite and >= 0";
  if (p.fof_dense < 0) return "fof_dense must be >= 0";
  if (p.bh_min < 0) return "bh_min must be >= 0";
  if (!(p.bh_theta >= 0.0 && std::isfinite(p.bh_theta))) return "bh_theta must be finite and >= 0";
  if (!(p.e_recheck >= 0.0)) return "e_recheck must be >= 0";
  if (p.mode != LIBHALO_PLAIN && p.mode != LIBHALO_BATCHED) return "unknown mode";
  if (p.prec != LIBHALO_PREC_FP64 && p.prec != LIBHALO_PREC_MIXED) return "unknown prec";
  if (p.grid_min != 0 && p.grid_min < 64) return "grid_min must be 0 or >= 64";
  if (p.ell_subset < 0) return "ell_subset must be >= 0";
  if (p.nn_chunk != 0 && (p.nn_chunk < 256 || p.nn_chunk > 4096 || p.nn_chunk % 256 != 0))
    return "nn_chunk must be 0 or a multiple of 256 in [256, 4096]";
  if (p.fof_chunk != 0 &&
      (p.fof_chunk < 256 || p.fof_chunk > 16384 || p.fof_chunk % 256 != 0))
    return "fof_chunk must be 0 or a multiple of 256 in [256, 16384]";
  if (p.pot_chunk != 0 && p.pot_chunk != 1024 && p.pot_chunk != 2048 && p.pot_chunk != 4096)
    return "pot_chunk must be 0, 1024, 2048 or 4096";
  if (p.kd_leaf != 0 && (p.kd_leaf < 4 || p.kd_leaf > 64)) return "kd_leaf must be 0 or in [4, 64]";
  if (p.bh_leaf != 0 && (p.bh_leaf < 4 || p.bh_leaf > 64)) return "bh_leaf must be 0 or in [4, 64]";
  if (!std::isfinite(p.nn_bracket)) return "nn_bracket must be finite";
  return "";
}

}  // namespace halo

template <class F>
static int guarded(libhalo_ctx* ctx, F&& f, void* stream = nullptr) {
  if (!ctx) return LIBHALO_EINVAL;
  try {
    ctx->c.stream = (hipStream_t)stream;
    HALO_HIP(hipSetDevice(ctx->c.device));
    f(ctx->c);
    ctx->c.err.clear();
    return LIBHALO_OK;
  } catch (const halo::Error& e) {
    ctx->c.err = e.msg;
    // an error between a fork and its join leaves side work queued: let it end
    // before anything can grow or free the workspace it uses
    (void)hipStreamSynchronize(ctx->c.side);
    return e.code;
  } catch (const std::bad_alloc&) {
    ctx->c.err = "host allocation failed";
    (void)hipStreamSynchronize(ctx->c.side);
    return LIBHALO_ENOMEM;
  }
}

extern "C" {

const char* libhalo_version(void) { return "libhalo 0.1 (gfx950)"; }

int libhalo_ctx_create(const libhalo_params* p, int device, libhalo_alloc_fn alloc_fn,
                       libhalo_free_fn free_fn, void* user, libhalo_ctx** out) {
  if (!p || !out || !alloc_fn || !free_fn) return LIBHALO_EINVAL;
  *out = nullptr;
  if (!halo::validate(*p).empty()) return LIBHALO_EINVAL;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev)
    return LIBHALO_EINVAL;
  libhalo_ctx* c = new (std::nothrow) libhalo_ctx();
  if (!c) return LIBHALO_ENOMEM;
  c->c.p = *p;
  c->c.device = device;
  c->c.alloc_fn = alloc_fn;
  c->c.free_fn = free_fn;
  c->c.user = user;
  int rc = LIBHALO_OK;
  if (hipSetDevice(device) != hipSuccess ||
      hipHostMalloc(&c->c.h_pinned, 4096, hipHostMallocDefault) != hipSuccess) {
    rc = LIBHALO_EHIP;
  } else if (halo::scratch_setup(device, &c->c.scratch) != hipSuccess) {
    rc = LIBHALO_EHIP;
  } else if (hipStreamCreateWithFlags(&c->c.side, hipStreamNonBlocking) != hipSuccess ||
             hipEventCreateWithFlags(&c->c.ev_fork, hipEventDisableTiming) != hipSuccess ||
             hipEventCreateWithFlags(&c->c.ev_join, hipEventDisableTiming) != hipSuccess) {
    rc = LIBHALO_EHIP;
  } else {
    c->c.d_err = static_cast<uint32_t*>(alloc_fn(halo::kErrBlockBytes, user, nullptr));
    if (!c->c.d_err) rc = LIBHALO_ENOMEM;
  }
  if (rc != LIBHALO_OK) {
    c->c.release();
    delete c;
    return rc;
  }
  *out = c;
  return LIBHALO_OK;
}

int libhalo_ctx_destroy(libhalo_ctx* ctx) {
  if (!ctx) return LIBHALO_EINVAL;
  (void)hipSetDevice(ctx->c.device);
  (void)hipDeviceSynchronize();
  ctx->c.release();
  delete ctx;
  return LIBHALO_OK;
}

const char* libhalo_last_error(const libhalo_ctx* ctx) {
  return ctx ? ctx->c.err.c_str() : "null context";
}

int libhalo_set_params(libhalo_ctx* ctx, const libhalo_params* p) {
  if (!ctx || !p) return LIBHALO_EINVAL;
  std::string m = halo::validate(*p);
  if (!m.empty()) {
    ctx->c.err = m;
    return LIBHALO_EINVAL;
  }
  ctx->c.p = *p;
  return LIBHALO_OK;
}

static bool dtype_ok(int d) { return d == LIBHALO_F32 || d == LIBHALO_F64; }

int libhalo_profile(libhalo_ctx* ctx, int enable) {
  return guarded(ctx, [&](halo::Ctx& c) {
    c.prof = (enable & 1) != 0;
    c.count = (enable & 2) != 0;
  });
}

int libhalo_profile_reset(libhalo_ctx* ctx) {
  return guarded(ctx, [&](halo::Ctx& c) {
    for (auto& r : c.recs) {
      c.spare.push_back(r.e0);
      c.spare.push_back(r.e1);
    }
    c.recs.clear();
    HALO_HIP(hipDeviceSynchronize());
    HALO_HIP(hipMemset(reinterpret_cast<char*>(c.d_err) + 64, 0, halo::kErrBlockBytes - 64));
  });
}

int libhalo_profile_work(libhalo_ctx* ctx, const char* kernel, double* tests, double* evals) {
  return guarded(ctx, [&](halo::Ctx& c) {
    HALO_CHECK(kernel && tests && evals, LIBHALO_EINVAL, "null pointer argument");
    int slot = -1;
    if (std::strcmp(kernel, "k_kd_walk_nn") == 0) slot = 0;
    if (std::strcmp(kernel, "k_kd_walk_fof") == 0) slot = 2;
    if (std::strcmp(kernel, "k_bh_walk") == 0) slot = 4;
    HALO_CHECK(slot >= 0, LIBHALO_EINVAL, "no work counters for this kernel");
    HALO_HIP(hipDeviceSynchronize());
    if (slot < 4) {
      unsigned long long w[4];
      HALO_HIP(hipMemcpy(w, reinterpret_cast<char*>(c.d_err) + 64, sizeof w,
                         hipMemcpyDeviceToHost));
      *tests = (double)w[slot];
      *evals = (double)w[slot + 1];
    } else {  // the tree potential's counters, spread over kBhSlots cache lines
      unsigned long long w[8 * halo::kBhSlots];
      HALO_HIP(hipMemcpy(w, c.bh_counters(), sizeof w, hipMemcpyDeviceToHost));
      double t = 0.0, e = 0.0;
      for (int k = 0; k < halo::kBhSlots; ++k) {
        t += (double)w[8 * k];
        e += (double)w[8 * k + 1];
      }
      *tests = t;
      *evals = e;
    }
  });
}

int libhalo_profile_read(libhalo_ctx* ctx, const char* kernel, double* total_ms,
                         int64_t* launches) {
  return guarded(ctx, [&](halo::Ctx& c) {
    HALO_CHECK(kernel && total_ms && launches, LIBHALO_EINVAL, "null pointer argument");
    double t = 0.0;
    int64_t k = 0;
    for (auto& r : c.recs) {
      if (std::strcmp(r.name, kernel) != 0) continue;
      HALO_HIP(hipEventSynchronize(r.e1));
      float ms = 0.f;
      HALO_HIP(hipEventElapsedTime(&ms, r.e0, r.e1));
      t += ms;
      ++k;
    }
    *total_ms = t;
    *launches = k;
  });
}

int libhalo_fof3d(libhalo_ctx* ctx, int64_t n, int pos_dtype, const void* x, const void* y,
                  const void* z, uint32_t* fof_label, uint32_t* perm, uint32_t* grp_first,
                  uint32_t* grp_count, int64_t grp_cap, int64_t* n_groups,
                  int64_t* n_members, void* stream) {
  return guarded(ctx, [&](halo::Ctx& c) {
    HALO_CHECK(n >= 1 && n < 0xFFFFFFFFll, LIBHALO_EINVAL, "n must lie in [1, 2^32-1)");
    HALO_CHECK(dtype_ok(pos_dtype), LIBHALO_EINVAL, "pos_dtype must be F32 or F64");
    HALO_CHECK(x && y && z && fof_label && perm && n_groups && n_members, LIBHALO_EINVAL,
               "null pointer argument");
    HALO_CHECK(grp_cap == 0 || (grp_first && grp_count), LIBHALO_EINVAL,
               "null group table");
    c.ensure_ws(halo::fof3d_workspace(c.p, n, pos_dtype));
    halo::fof3d(c, n, pos_dtype, x, y, z, fof_label, perm, grp_first, grp_count, grp_cap,
                n_groups, n_members, (hipStream_t)stream);
  }, stream);
}

int libhalo_fof3d_noalloc(libhalo_ctx* ctx, int64_t n, int pos_dtype, const void* x,
                          const void* y, const void* z, uint32_t* fof_label, uint32_t* perm,
                          uint32_t* grp_first, uint32_t* grp_count, int64_t grp_cap,
                          int64_t* n_groups, int64_t* n_members, void* stream) {
  return guarded(ctx, [&](halo::Ctx& c) {
    HALO_CHECK(n >= 1 && n < 0xFFFFFFFFll, LIBHALO_EINVAL, "n must lie in [1, 2^32-1)");
    HALO_CHECK(dtype_ok(pos_dtype), LIBHALO_EINVAL, "pos_dtype must be F32 or F64");
    HALO_CHECK(x && y && z && fof_label && perm && n_groups && n_members, LIBHALO_EINVAL,
               "null pointer argument");
    HALO_CHECK(grp_cap == 0 || (grp_first && grp_count), LIBHALO_EINVAL,
               "null group table");
    HALO_CHECK(c.scratch != nullptr, LIBHALO_EHIP, "no scratch array on this device");
    const size_t need = halo::fof3d_workspace(c.p, n, pos_dtype);
    if (need > halo::kScratchBytes)
      throw halo::Error{LIBHALO_ENOMEM,
                        "libhalo_fof3d_noalloc: these particles need " + std::to_string(need) +
                            " bytes of scratch; the fixed array holds " +
                            std::to_string(halo::kScratchBytes)};
    // the call's workspace is the device's scratch array, not the context's
    halo::Arena own = c.ws;
    c.ws = halo::Arena{};
    c.ws.base = static_cast<char*>(c.scratch);
    c.ws.cap = halo::kScratchBytes;
    try {
      halo::fof3d(c, n, pos_dtype, x, y, z, fof_label, perm, grp_first, grp_count, grp_cap,
                  n_groups, n_members, (hipStream_t)stream);
    } catch (...) {
      c.ws = own;
      throw;
    }
    c.ws = own;
  }, stream);
}

int libhalo_refine6d(libhalo_ctx* ctx, int64_t n, int pos_dtype, const void* x,
                     const void* y, const void* z, const float* vx, const float* vy,
                     const float* vz, const uint32_t* perm, const uint32_t* grp_first,
                     const uint32_t* grp_count, int64_t n_groups, libhalo_nodes* nodes,
                     int32_t* deepest, int64_t* n_nodes, void* stream) {
  return guarded(ctx, [&](halo::Ctx& c) {
    HALO_CHECK(n >= 1 && n < 0xFFFFFFFFll, LIBHALO_EINVAL, "n must lie in [1, 2^32-1)");
    HALO_CHECK(dtype_ok(pos_dtype), LIBHALO_EINVAL, "pos_dtype must be F32 or F64");
    HALO_CHECK(x && y && z && vx && vy && vz && nodes && deepest && n_nodes, LIBHALO_EINVAL,
               "null pointer argument");
    HALO_CHECK(n_groups >= 0 && (n_groups == 0 || (perm && grp_first && grp_count)),
               LIBHALO_EINVAL, "bad group table");
    halo::refine6d(c, n, pos_dtype, x, y, z, vx, vy, vz, perm, grp_first, grp_count,
                   n_groups, nodes, deepest, n_nodes, (hipStream_t)stream);
  }, stream);
}

int libhalo_assign(libhalo_ctx* ctx, int64_t n, int pos_dtype, const void* x, const void* y,
                   const void* z, const float* vx, const float* vy, const float* vz,
                   const libhalo_nodes* nodes, int64_t n_nodes, const int32_t* deepest,
                   libhalo_halos* halos, int32_t* halo_of, int64_t* n_halos, void* stream) {
  return guarded(ctx, [&](halo::Ctx& c) {
    HALO_CHECK(n >= 1 && n < 0xFFFFFFFFll, LIBHALO_EINVAL, "n must lie in [1, 2^32-1)");
    HALO_CHECK(dtype_ok(pos_dtype), LIBHALO_EINVAL, "pos_dtype must be F32 or F64");
    HALO_CHECK(x && y && z && vx && vy && vz && nodes && deepest && halos && halo_of &&
                   n_halos,
               LIBHALO_EINVAL, "null pointer argument");
    HALO_CHECK(n_nodes >= 0, LIBHALO_EINVAL, "n_nodes must be >= 0");
    halo::assign(c, n, pos_dtype, x, y, z, vx, vy, vz, nodes, n_nodes, deepest, halos,
                 halo_of, n_halos, (hipStream_t)stream);
  }, stream);
}

int libhalo_unbind(libhalo_ctx* ctx, int64_t n, int pos_dtype, const void* x, const void* y,
                   const void* z, const float* vx, const float* vy, const float* vz,
                   const libhalo_halos* halos, int64_t n_halos, const int32_t* halo_of,
                   uint8_t* bound, double* phi, libhalo_unbound* out, void* stream) {
  return guarded(ctx, [&](halo::Ctx& c) {
    HALO_CHECK(n >= 1 && n < 0xFFFFFFFFll, LIBHALO_EINVAL, "n must lie in [1, 2^32-1)");
    HALO_CHECK(dtype_ok(pos_dtype), LIBHALO_EINVAL, "pos_dtype must be F32 or F64");
    HALO_CHECK(x && y && z && vx && vy && vz && halos && halo_of && bound && out,
               LIBHALO_EINVAL, "null pointer argument");
    HALO_CHECK(n_halos >= 0, LIBHALO_EINVAL, "n_halos must be >= 0");
    halo::unbind(c, n, pos_dtype, x, y, z, vx, vy, vz, halos, n_halos, halo_of, bound, phi,
                 out, (hipStream_t)stream);
  }, stream);
}

int libhalo_props(libhalo_ctx* ctx, int64_t n, int pos_dtype, const void* x, const void* y,
                  const void* z, const float* vx, const float* vy, const float* vz,
                  const libhalo_nodes* nodes, int64_t n_nodes, const libhalo_halos* halos,
                  int64_t n_halos, const int32_t* halo_of, const uint8_t* bound,
                  libhalo_props_out* out, void* stream) {
  return guarded(ctx, [&](halo::Ctx& c) {
    HALO_CHECK(n >= 1 && n < 0xFFFFFFFFll, LIBHALO_EINVAL, "n must lie in [1, 2^32-1)");
    HALO_CHECK(dtype_ok(pos_dtype), LIBHALO_EINVAL, "pos_dtype must be F32 or F64");
    HALO_CHECK(x && y && z && vx && vy && vz && nodes && halos && halo_of && bound && out,
               LIBHALO_EINVAL, "null pointer argument");
    HALO_CHECK(n_nodes >= 0 && n_halos >= 0, LIBHALO_EINVAL, "negative table size");
    halo::props(c, n, pos_dtype, x, y, z, vx, vy, vz, nodes, n_nodes, halos, n_halos, halo_of,
                bound, out, (hipStream_t)stream);
  }, stream);
}

int libhalo_props_extra(libhalo_ctx* ctx, int64_t n, int pos_dtype, const void* x,
                        const void* y, const void* z, const float* vx, const float* vy,
                        const float* vz, const libhalo_nodes* nodes, int64_t n_nodes,
                        const libhalo_halos* halos, int64_t n_halos, const int32_t* halo_of,
                        const uint8_t* bound, libhalo_props_out* out, int n_so,
                        const double* so_rho, libhalo_props_extra_out* ext, void* stream) {
  return guarded(ctx, [&](halo::Ctx& c) {
    HALO_CHECK(n >= 1 && n < 0xFFFFFFFFll, LIBHALO_EINVAL, "n must lie in [1, 2^32-1)");
    HALO_CHECK(dtype_ok(pos_dtype), LIBHALO_EINVAL, "pos_dtype must be F32 or F64");
    HALO_CHECK(x && y && z && vx && vy && vz && nodes && halos && halo_of && bound && out && ext,
               LIBHALO_EINVAL, "null pointer argument");
    HALO_CHECK(n_nodes >= 0 && n_halos >= 0, LIBHALO_EINVAL, "negative table size");
    HALO_CHECK(n_so >= 0 && n_so <= LIBHALO_MAX_SO, LIBHALO_EINVAL,
               "n_so must lie in [0, LIBHALO_MAX_SO]");
    HALO_CHECK(n_so == 0 || so_rho, LIBHALO_EINVAL, "so_rho is null");
    HALO_CHECK(ext->cap >= n_halos, LIBHALO_EINVAL, "ext->cap is below n_halos");
    halo::ExtraArgs ea;
    ea.n_so = n_so;
    ea.ext = ext;
    for (int t = 0; t < n_so; ++t) {
      HALO_CHECK(so_rho[t] > 0.0 && std::isfinite(so_rho[t]), LIBHALO_EINVAL,
                 "SO thresholds must be positive and finite");
      ea.rho[t] = so_rho[t];
    }
    HALO_CHECK(ext->xoff && ext->jx && ext->jy && ext->jz && ext->kin && ext->pot && ext->t_u &&
                   ext->spin && ext->spin_bullock && ext->c_klypin && ext->rs_klypin &&
                   ext->b_to_a && ext->c_to_a && ext->ax && ext->ay && ext->az &&
                   ext->n_shape && (n_so == 0 || (ext->m_so && ext->r_so)),
               LIBHALO_EINVAL, "null output array in ext");
    halo::props(c, n, pos_dtype, x, y, z, vx, vy, vz, nodes, n_nodes, halos, n_halos, halo_of,
                bound, out, (hipStream_t)stream, &ea);
  }, stream);
}

}  // extern "C"
