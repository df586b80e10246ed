// Stages not yet built report an error.
#include "stages.hpp"
namespace halo {
void assign(Ctx&, int64_t, int, const void*, const void*, const void*, const float*,
            const float*, const float*, const libhalo_nodes*, int64_t, const int32_t*,
            libhalo_halos*, int32_t*, int64_t*, hipStream_t) {
  throw Error{LIBHALO_EINVAL, "assign not built"};
}
void unbind(Ctx&, int64_t, int, const void*, const void*, const void*, const float*,
            const float*, const float*, const libhalo_halos*, int64_t, const int32_t*,
            uint8_t*, double*, libhalo_unbound*, hipStream_t) {
  throw Error{LIBHALO_EINVAL, "unbind not built"};
}
void props(Ctx&, int64_t, int, const void*, const void*, const void*, const float*,
           const float*, const float*, const libhalo_nodes*, int64_t, const libhalo_halos*,
           int64_t, const int32_t*, const uint8_t*, libhalo_props_out*, hipStream_t) {
  throw Error{LIBHALO_EINVAL, "props not built"};
}
}  // namespace halo
