// Additional halo properties (Sections 3.5.2 and 3.5.4), computed after the
// basic properties on the same radially sorted bound particles of S(h).
#pragma once
#include "common.hpp"
#include "radial.hpp"

namespace halo {

struct ExtraArgs {
  int n_so = 0;
  double rho[LIBHALO_MAX_SO] = {};
  libhalo_props_extra_out* ext = nullptr;
};

struct ExtraBufs {
  I128* acc;        // kExtraSums per halo
  I128* accU;       // 1 per halo
  uint32_t* nown;   // own particles of V(h)
  uint32_t* kfail;  // n_so per halo
  uint32_t* ucnt;   // S + 1
  uint32_t* uoff;   // S + 1
  uint32_t* total;
  uint32_t* stmp;
  double *ux, *uy, *uz;  // m: positions about the centre (first k* of each halo)
};

ExtraBufs extra_take(Arena& A, uint32_t S, uint32_t m, int n_so);

// Runs after the basic properties: `out` holds the centre, bulk velocity,
// M_vir, R_vir and v_max; kstar the size of V(h) per halo.
void props_extra_run(Ctx& ctx, const ExtraArgs& ea, const ExtraBufs& eb, int pos_dtype,
                     const void* x, const void* y, const void* z, const float* vx,
                     const float* vy, const float* vz, const int32_t* halo_of,
                     const libhalo_halos& h, uint32_t S, const RadialBufs& rb, uint32_t m,
                     const uint32_t* kstar, const libhalo_props_out& out, hipStream_t s);

}  // namespace halo
