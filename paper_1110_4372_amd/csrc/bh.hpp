// Tree potential of the largest haloes (Appendix B), used by unbinding.
#pragma once
#include "common.hpp"

namespace halo {

// Halo s takes the tree when it is kept, has own particles and |S(h)| >= bh_min.
__host__ __device__ inline bool bh_takes(bool kept, uint32_t nown, uint32_t ns, double theta,
                                         uint32_t bh_min) {
  return theta > 0.0 && kept && nown > 0 && ns >= bh_min;
}

// Adds sum_j 1/sqrt(r_ij^2 + eps^2) over S(h), by the tree, to the fixed-point
// potential sums (2^-32, 128-bit) of the own particles of every halo that
// takes the tree.  Layout: S(h) = [slot[h], slot[h] + nS[h]) of (ux, uy, uz),
// its own particles first.
void bh_potential(Ctx& ctx, const libhalo_halos& h, uint32_t S, const uint32_t* nS,
                  const uint32_t* slot, const double* ux, const double* uy, const double* uz,
                  double eps2, double theta, uint32_t bh_min, I128* pacc, hipStream_t s);

}  // namespace halo
