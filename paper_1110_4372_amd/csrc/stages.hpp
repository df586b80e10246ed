// Hierarchy, assignment, unbinding and property stages.
#pragma once
#include "common.hpp"

namespace halo {
struct ExtraArgs;
void refine6d(Ctx& ctx, int64_t n, int pos_dtype, const void* x, const void* y, const void* z,
              const float* vx, const float* vy, const float* vz, const uint32_t* perm,
              const uint32_t* grp_first, const uint32_t* grp_count, int64_t n_groups,
              libhalo_nodes* nodes, int32_t* deepest, int64_t* n_nodes, hipStream_t s);
void assign(Ctx& ctx, int64_t n, int pos_dtype, const void* x, const void* y, const void* z,
            const float* vx, const float* vy, const float* vz, const libhalo_nodes* nodes,
            int64_t n_nodes, const int32_t* deepest, libhalo_halos* halos, int32_t* halo_of,
            int64_t* n_halos, hipStream_t s);
void unbind(Ctx& ctx, int64_t n, int pos_dtype, const void* x, const void* y, const void* z,
            const float* vx, const float* vy, const float* vz, const libhalo_halos* halos,
            int64_t n_halos, const int32_t* halo_of, uint8_t* bound, double* phi,
            libhalo_unbound* out, hipStream_t s);
void props(Ctx& ctx, int64_t n, int pos_dtype, const void* x, const void* y, const void* z,
           const float* vx, const float* vy, const float* vz, const libhalo_nodes* nodes,
           int64_t n_nodes, const libhalo_halos* halos, int64_t n_halos,
           const int32_t* halo_of, const uint8_t* bound, libhalo_props_out* out,
           hipStream_t s, const ExtraArgs* extra = nullptr);
}  // namespace halo
