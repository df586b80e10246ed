// 3D friends-of-friends stage.
#pragma once
#include "common.hpp"

namespace halo {
size_t fof3d_workspace(const libhalo_params& P, int64_t n, int pos_dtype);
void fof3d(Ctx& ctx, int64_t n, int pos_dtype, const void* x, const void* y, const void* z,
           uint32_t* label, uint32_t* perm, uint32_t* grp_first, uint32_t* grp_count,
           int64_t grp_cap, int64_t* n_groups, int64_t* n_members, hipStream_t s);
}  // namespace halo
