// Shared device helpers and the context of the libhalo HIP library (gfx950).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "libhalo.h"

namespace halo {

constexpr int kWave = 64;
constexpr int kVelShift = 24;  // velocity fixed point: 2^-24 km/s

// ------------------------------------------------------------ errors -----
struct Error {
  int code;
  std::string msg;
};

#define HALO_HIP(call)                                                        \
  do {                                                                        \
    hipError_t e_ = (call);                                                   \
    if (e_ != hipSuccess)                                                     \
      throw ::halo::Error{LIBHALO_EHIP, std::string(#call) + ": " +           \
                                            hipGetErrorString(e_)};           \
  } while (0)

#define HALO_CHECK(cond, code, msg)                       \
  do {                                                    \
    if (!(cond)) throw ::halo::Error{(code), (msg)};      \
  } while (0)

// Device error word bits, set by kernels, read back by the host.
enum : uint32_t {
  kErrPosRange = 1u,   // a position outside [0, L) or NaN
  kErrGeometry = 2u,   // group extent >= L/2
  kErrVelRange = 4u,   // |v| >= 2^16 km/s or NaN
};

// The device error block: error words, then the walks' work counters.
constexpr size_t kErrBlockBytes = 4096;
constexpr int kBhSlots = 32;  // tree-potential counter pairs (one per 64-byte line)

// ------------------------------------------------------------ workspace --
// Grow-only device arena over a block from the context's allocator callback.
// Each entry point resets it and carves buffers.
struct Arena {
  char* base = nullptr;
  size_t cap = 0, off = 0;
  bool counting = false;  // dry run: only sums the sizes of the takes
  void reset() { off = 0; }
  template <class T>
  T* take(size_t count) {
    size_t bytes = (count * sizeof(T) + 255) & ~size_t(255);
    if (counting) {
      off += bytes;
      return reinterpret_cast<T*>(uintptr_t(256));
    }
    if (off + bytes > cap) throw Error{LIBHALO_ENOMEM, "workspace exhausted"};
    T* p = reinterpret_cast<T*>(base + off);
    off += bytes;
    return p;
  }
};

// Runs carve(arena) once to size the workspace, grows it, then carves for real.
template <class Ctx_, class F>
void carve_workspace(Ctx_& ctx, F&& carve) {
  Arena dry;
  dry.counting = true;
  carve(dry);
  ctx.ensure_ws(dry.off + 4096);
  ctx.ws.reset();
  carve(ctx.ws);
}

// Kernel timing: when enabled, instrumented launches are bracketed by HIP
// events on their stream; read back and summed per kernel name on request.
struct ProfRec {
  const char* name;
  hipEvent_t e0, e1;
};

struct Ctx {
  libhalo_params p{};
  bool prof = false;
  std::vector<ProfRec> recs;
  std::vector<hipEvent_t> spare;
  hipEvent_t event();
  int device = 0;
  std::string err;
  Arena ws;
  Arena ws2;                       // second arena: the tree potential, inside unbinding
  uint32_t* d_err = nullptr;       // device error word; its block (kErrBlockBytes)
                                   // also holds the walks' work counters: the 6D
                                   // walks' 4 u64 at byte 64, the tree potential's
                                   // kBhSlots pairs at byte 1024, 64 bytes apart
  void* h_pinned = nullptr;        // small pinned host buffer for read-backs
  hipStream_t stream = nullptr;    // stream of the entry point being run
  // A second stream of the context (default priority) for work that is
  // independent of what runs meanwhile on the entry point's stream: fork()
  // starts it after the work queued so far on s, join() makes s wait for it.
  // Every fork is joined before the entry point returns.
  hipStream_t side = nullptr;
  hipEvent_t ev_fork = nullptr, ev_join = nullptr;
  hipStream_t fork(hipStream_t s) {
    HALO_HIP(hipEventRecord(ev_fork, s));
    HALO_HIP(hipStreamWaitEvent(side, ev_fork, 0));
    return side;
  }
  void join(hipStream_t s) {
    HALO_HIP(hipEventRecord(ev_join, side));
    HALO_HIP(hipStreamWaitEvent(s, ev_join, 0));
  }
  libhalo_alloc_fn alloc_fn = nullptr;  // workspace provider (caller's callbacks)
  libhalo_free_fn free_fn = nullptr;
  void* user = nullptr;
  void* scratch = nullptr;         // this device's fixed scratch array (no-alloc entry)
  void* dev_alloc(size_t bytes, const char* what);  // ENOMEM on NULL
  bool count = false;  // the tree walks count their work (a slower form of them)
  // device work counters of the 6D tree walks while counting, else null
  unsigned long long* work_counters() {
    return count ? reinterpret_cast<unsigned long long*>(reinterpret_cast<char*>(d_err) + 64)
                 : nullptr;
  }
  unsigned long long* bh_counters() {
    return reinterpret_cast<unsigned long long*>(reinterpret_cast<char*>(d_err) + 1024);
  }
  void ensure_ws(size_t bytes);
  void ensure_ws2(size_t bytes);
  void release();
  template <class T>
  T* host_slot(int i) { return reinterpret_cast<T*>(static_cast<char*>(h_pinned) + 64 * i); }
};

// Bracket a launch with events when profiling is on.
#define HALO_PROF(ctx, nm, strm, ...)                               \
  do {                                                              \
    if ((ctx).prof) {                                               \
      ::halo::ProfRec r_{nm, (ctx).event(), (ctx).event()};         \
      HALO_HIP(hipEventRecord(r_.e0, strm));                        \
      __VA_ARGS__;                                                  \
      HALO_HIP(hipEventRecord(r_.e1, strm));                        \
      (ctx).recs.push_back(r_);                                     \
    } else {                                                        \
      __VA_ARGS__;                                                  \
    }                                                               \
  } while (0)

// ------------------------------------------------------------ launch -----
// Blocks are dispatched to the eight XCDs in turn (block b to XCD b mod 8).
// This index gives the blocks of one XCD a contiguous eighth of the grid, so
// neighbouring items, which read the same data, share an L2.  A bijection on
// [0, gridDim.x); the last gridDim.x mod 8 blocks keep their own index.
__device__ __forceinline__ uint32_t xcd_block() {
  const uint32_t g8 = gridDim.x >> 3;
  return blockIdx.x < 8u * g8 ? (blockIdx.x & 7u) * g8 + (blockIdx.x >> 3) : blockIdx.x;
}

inline unsigned blocks_for(int64_t n, int threads) {
  int64_t b = (n + threads - 1) / threads;
  return (unsigned)(b < 1 ? 1 : b);
}

// ------------------------------------------------------------ device math -
__device__ __forceinline__ double min_image(double d, double box) {
  double h = 0.5 * box;
  if (d > h) return d - box;
  if (d < -h) return d + box;
  return d;
}

// |(a, b, c)|^2 evaluated as fma(c, c, fma(b, b, a * a)).
__device__ __forceinline__ double sq3(double a, double b, double c) {
  return __fma_rn(c, c, __fma_rn(b, b, a * a));
}

template <class T>
__device__ __forceinline__ double ld_pos(const T* p, int64_t i) {
  return (double)p[i];
}

// Signed 128-bit integer as two 64-bit words (value = hi * 2^64 + lo).
struct I128 {
  unsigned long long lo;
  long long hi;
};

__device__ __forceinline__ I128 i128_from(long long v) {
  I128 r;
  r.lo = (unsigned long long)v;
  r.hi = v < 0 ? -1ll : 0ll;
  return r;
}

__device__ __forceinline__ I128 i128_add(I128 a, I128 b) {
  I128 r;
  r.lo = a.lo + b.lo;
  r.hi = a.hi + b.hi + (r.lo < a.lo ? 1 : 0);
  return r;
}

__device__ __forceinline__ I128 i128_sqr(long long v) {
  __int128 s = (__int128)v * (__int128)v;
  I128 r;
  r.lo = (unsigned long long)s;
  r.hi = (long long)(s >> 64);
  return r;
}

// Double of a 128-bit integer by one fixed sequence of roundings, within an
// ulp: the magnitude's words are converted (each correctly rounded) and
// combined by one fma, then the sign is applied.  Converting the signed words
// directly would cancel: a small negative value has hi = -1 and lo near 2^64,
// whose rounding loses up to 2^10 units.
__device__ __forceinline__ double i128_to_f64(I128 v) {
  const bool neg = v.hi < 0;
  unsigned long long ml = v.lo, mh = (unsigned long long)v.hi;
  if (neg) {  // two's complement negation of the 128-bit value
    ml = ~ml + 1ull;
    mh = ~mh + (ml == 0ull ? 1ull : 0ull);
  }
  const double d = __fma_rn((double)mh, 18446744073709551616.0, (double)ml);
  return neg ? -d : d;
}

__device__ __forceinline__ I128 wave_sum_i128(I128 v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    I128 w;
    w.lo = __shfl_xor(v.lo, o);
    w.hi = __shfl_xor(v.hi, o);
    v = i128_add(v, w);
  }
  return v;
}

// Exact 128-bit accumulation into global memory with two 64-bit atomics:
// carries out of the low word are added to the high word.
__device__ __forceinline__ void atomic_add_i128(I128* acc, I128 v) {
  unsigned long long old = atomicAdd(&acc->lo, v.lo);
  unsigned long long carry = (old + v.lo) < old ? 1ull : 0ull;
  long long add_hi = v.hi + (long long)carry;
  if (add_hi != 0) atomicAdd((unsigned long long*)&acc->hi, (unsigned long long)add_hi);
}

__device__ __forceinline__ long long quantise(double v, int shift) {
  return (long long)rint(ldexp(v, shift));
}

// Order-preserving u64 image of a double (for atomic min/max).
__device__ __forceinline__ unsigned long long f64_ord(double d) {
  unsigned long long u = (unsigned long long)__double_as_longlong(d);
  return (u >> 63) ? ~u : (u | 0x8000000000000000ull);
}
__device__ __forceinline__ double ord_f64(unsigned long long u) {
  u = (u >> 63) ? (u & 0x7FFFFFFFFFFFFFFFull) : ~u;
  return __longlong_as_double((long long)u);
}

// Canonical FP32 squared 6D distance: s = d0*d0, then fmaf of the other five
// components in the order d1, d2, e0, e1, e2, with d = b - a.
__device__ __forceinline__ float d2_6(float a0, float a1, float a2, float a3, float a4,
                                      float a5, float b0, float b1, float b2, float b3,
                                      float b4, float b5) {
  float d0 = b0 - a0, d1 = b1 - a1, d2 = b2 - a2;
  float e0 = b3 - a3, e1 = b4 - a4, e2 = b5 - a5;
  float s = d0 * d0;
  s = __fmaf_rn(d1, d1, s);
  s = __fmaf_rn(d2, d2, s);
  s = __fmaf_rn(e0, e0, s);
  s = __fmaf_rn(e1, e1, s);
  s = __fmaf_rn(e2, e2, s);
  return s;
}

// 1/sqrt(x) in FP64: the hardware estimate (relative error ~2^-23) refined
// by one Newton step y <- y (3/2 - (x/2) y^2), which squares the error
// (~2^-46, below the rounding of the potential sums it feeds).
__device__ __forceinline__ double rsqrt_f64(double x) {
  double y = __builtin_amdgcn_rsq(x);
  const double h = 0.5 * x;
  y = y * __fma_rn(-h * y, y, 1.5);
  return y;
}

// Per-segment accumulation over segment-sorted elements, one element per
// thread, whole block active: NC exact sums at acc[NC * h + c], a max of
// non-negative doubles at vm[h] (as bits) and an optional count at cnt[h].
// A wave whose elements share one segment reduces them into LDS; thread 0
// then merges runs of equal segment across the block's NW waves, so a large
// segment costs one set of atomics per block.  A wave spanning several
// segments adds per element.  h = 0xFFFFFFFF marks an absent element.
template <int NC, int NW>
struct SegMerge {
  uint32_t h[NW];
  I128 v[NW][NC];
  double t[NW];
  uint32_t c[NW];
};

template <int NC, int NW>
__device__ __forceinline__ void seg_merge_add(SegMerge<NC, NW>& L, uint32_t h, I128* v,
                                              double t, uint32_t c, I128* acc,
                                              unsigned long long* vm, uint32_t* cnt) {
  const uint32_t none = 0xFFFFFFFFu;
  const uint32_t wave = threadIdx.x >> 6;
  const uint32_t h0 = __builtin_amdgcn_readfirstlane(h);
  if (__all(h == h0) && h0 != none) {
    for (int o = 32; o > 0; o >>= 1) {
      t = fmax(t, __shfl_xor(t, o));
      c += __shfl_xor(c, o);
    }
    for (int k = 0; k < NC; ++k) v[k] = wave_sum_i128(v[k]);
    if ((threadIdx.x & 63) == 0) {
      L.h[wave] = h0;
      for (int k = 0; k < NC; ++k) L.v[wave][k] = v[k];
      L.t[wave] = t;
      L.c[wave] = c;
    }
  } else {
    if ((threadIdx.x & 63) == 0) L.h[wave] = none;
    if (h != none) {
      for (int k = 0; k < NC; ++k)
        if (v[k].lo != 0 || v[k].hi != 0) atomic_add_i128(acc + NC * (size_t)h + k, v[k]);
      if (t > 0.0) atomicMax(vm + h, (unsigned long long)__double_as_longlong(t));
      if (cnt && c) atomicAdd(cnt + h, c);
    }
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    uint32_t cur = none, sc = 0;
    I128 s[NC];
    double sm = 0.0;
    for (int w = 0; w <= NW; ++w) {
      const uint32_t hw = w < NW ? L.h[w] : none;
      if (hw != none && hw == cur) {
        for (int k = 0; k < NC; ++k) s[k] = i128_add(s[k], L.v[w][k]);
        sm = fmax(sm, L.t[w]);
        sc += L.c[w];
        continue;
      }
      if (cur != none) {
        for (int k = 0; k < NC; ++k)
          if (s[k].lo != 0 || s[k].hi != 0) atomic_add_i128(acc + NC * (size_t)cur + k, s[k]);
        if (sm > 0.0) atomicMax(vm + cur, (unsigned long long)__double_as_longlong(sm));
        if (cnt && sc) atomicAdd(cnt + cur, sc);
      }
      cur = hw;
      if (hw != none) {
        for (int k = 0; k < NC; ++k) s[k] = L.v[w][k];
        sm = L.t[w];
        sc = L.c[w];
      }
    }
  }
}

// Wave-aggregated atomic min at base[key] (same contract as agg_add_u32).
__device__ __forceinline__ void agg_min_u32(uint32_t* base, uint32_t key, uint32_t val,
                                            bool active) {
  unsigned long long pending = __ballot(active);
  const int lane = threadIdx.x & 63;
  while (pending) {
    const int leader = __ffsll((long long)pending) - 1;
    const uint32_t k = __shfl(key, leader);
    const unsigned long long same = __ballot(active && key == k) & pending;
    uint32_t v = (same >> lane) & 1ull ? val : 0xFFFFFFFFu;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = min(v, (uint32_t)__shfl_xor(v, o));
    if (lane == leader) atomicMin(base + k, v);
    pending &= ~same;
  }
}

// Wave-aggregated atomic add of `val` at base[key]: lanes sharing a key send
// one atomic (the leader's).  Cheap when a wave holds few distinct keys, as
// for data grouped by key.  Every lane of the wave must call it (inactive
// work is passed as active = false): the reduction reads all 64 lanes.
__device__ __forceinline__ void agg_add_u32(uint32_t* base, uint32_t key, uint32_t val,
                                            bool active) {
  unsigned long long pending = __ballot(active);
  const int lane = threadIdx.x & 63;
  while (pending) {
    const int leader = __ffsll((long long)pending) - 1;
    const uint32_t k = __shfl(key, leader);
    const unsigned long long same = __ballot(active && key == k) & pending;
    uint32_t v = (same >> lane) & 1ull ? val : 0u;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    if (lane == leader) atomicAdd(base + k, v);
    pending &= ~same;
  }
}

// ------------------------------------------------------------ union-find --
// Parents always point to smaller indices, so a root is its set's minimum.
__device__ __forceinline__ uint32_t uf_load(const uint32_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void uf_store(uint32_t* p, uint32_t v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ uint32_t uf_find(uint32_t* par, uint32_t x) {
  uint32_t cur = uf_load(par + x);
  if (cur == x) return x;
  uint32_t prev = x, next;
  while (cur > (next = uf_load(par + cur))) {
    uf_store(par + prev, next);  // path halving; next is an ancestor of prev
    prev = cur;
    cur = next;
  }
  return cur;
}

// Root of x without touching the forest.  Compression kernels must use this:
// a path-halving find running in another thread could otherwise overwrite a
// pointer just set to the root with a lower ancestor.
__device__ __forceinline__ uint32_t uf_root(const uint32_t* par, uint32_t x) {
  uint32_t p = uf_load(par + x);
  while (p != x) {
    x = p;
    p = uf_load(par + x);
  }
  return x;
}

// Join the sets of a and b; returns the root of the joined set.
__device__ __forceinline__ uint32_t uf_union(uint32_t* par, uint32_t a, uint32_t b) {
  uint32_t ra = uf_find(par, a), rb = uf_find(par, b);
  while (ra != rb) {
    if (ra < rb) {
      uint32_t t = ra;
      ra = rb;
      rb = t;
    }
    // hook the larger root ra under rb
    uint32_t old = atomicCAS(par + ra, ra, rb);
    if (old == ra) return rb;
    ra = uf_find(par, old);
    rb = uf_find(par, rb);
  }
  return ra;
}

}  // namespace halo
