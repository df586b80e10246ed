// Segmented radial sort: particles grouped by segment (a halo), each segment
// ordered by FP64 squared distance from its centre (ties: list order), plus
// the per-segment reductions that both assignment and properties use.
#pragma once
#include "common.hpp"

namespace halo {

struct RadialBufs {
  // inputs (m elements): segment id and particle index
  uint32_t* seg;
  uint32_t* pidx;
  // outputs in sorted order
  uint32_t* s_seg;
  uint32_t* s_pidx;
  double* s_r2;
  uint32_t* start;  // nseg + 1
  // scratch
  uint32_t* s_e;  // input position of each sorted element
  uint32_t* va;
  uint32_t* vb;
  uint32_t* k32a;
  uint32_t* k32b;
  double* r2;
  void* rtmp;
  uint32_t* stmp;
};

size_t radial_bytes(int64_t m, int64_t nseg);
RadialBufs radial_take(Arena& A, int64_t m, int64_t nseg);

// Sort elements (seg[e], pidx[e]) by (seg, r^2 from centre[seg]); fills
// s_seg, s_pidx, s_r2 and start[].
void radial_sort(int pos_dtype, const void* x, const void* y, const void* z, double box,
                 const double* cx, const double* cy, const double* cz, int64_t m,
                 int64_t nseg, RadialBufs& b, hipStream_t s);

// Per segment: sv2 = 3D velocity variance (exact fixed-point sums) and
// vmax2 = G m sqrt(max_k k^2 / max(r_k^2, eps^2)) over the sorted segment.
// Segments with no element keep sv2 = vmax2 = 0.  acc: 4 I128 per segment,
// vm: 1 u64 per segment (scratch).
void radial_sigma_vmax(const float* vx, const float* vy, const float* vz, int64_t m,
                       int64_t nseg, const RadialBufs& b, double Gm, double eps2, I128* acc,
                       unsigned long long* vm, double* sv2, double* vmax2, hipStream_t s);

}  // namespace halo
