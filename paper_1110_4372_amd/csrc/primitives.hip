// Device-wide exclusive scan and stable LSD radix sort for gfx950 (wave64).
#include "primitives.hpp"

namespace halo {

namespace {

constexpr int kScanThreads = 256;
constexpr int kScanItems = 8;
constexpr int kScanTile = kScanThreads * kScanItems;

// Exclusive scan of one value per thread across the block; *total receives
// the block sum.  lds needs (blockDim/64 + 1) elements.
template <class T>
__device__ T block_exclusive_scan(T v, T* total, T* lds) {
  const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave;
  const int nw = blockDim.x / kWave;
  T inc = v;
#pragma unroll
  for (int o = 1; o < kWave; o <<= 1) {
    T t = __shfl_up(inc, o);
    if (lane >= o) inc += t;
  }
  if (lane == kWave - 1) lds[wid] = inc;
  __syncthreads();
  if (threadIdx.x == 0) {
    T run = 0;
    for (int w = 0; w < nw; ++w) {
      T t = lds[w];
      lds[w] = run;
      run += t;
    }
    lds[nw] = run;
  }
  __syncthreads();
  T excl = inc - v + lds[wid];
  *total = lds[nw];
  __syncthreads();
  return excl;
}

template <class T>
__global__ void __launch_bounds__(kScanThreads) k_scan_reduce(const T* in, int64_t n, T* part) {
  __shared__ T lds[kScanThreads / kWave + 1];
  int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
  T s = 0;
#pragma unroll
  for (int i = 0; i < kScanItems; ++i)
    if (base + i < n) s += in[base + i];
  T tot;
  block_exclusive_scan(s, &tot, lds);
  if (threadIdx.x == 0) part[blockIdx.x] = tot;
}

// Scans a tile of NT x ITEMS elements per block; adds offset part[blockIdx.x]
// if part.
template <class T, int NT = kScanThreads, int ITEMS = kScanItems>
__global__ void __launch_bounds__(NT) k_scan_down(const T* in, T* out, int64_t n,
                                                  const T* part, T* total) {
  __shared__ T lds[NT / kWave + 1];
  int64_t base = (int64_t)blockIdx.x * (NT * ITEMS) + (int64_t)threadIdx.x * ITEMS;
  T v[ITEMS];
  T s = 0;
#pragma unroll
  for (int i = 0; i < ITEMS; ++i) {
    v[i] = (base + i < n) ? in[base + i] : T(0);
    s += v[i];
  }
  T tot;
  T run = block_exclusive_scan(s, &tot, lds);
  if (part) run += part[blockIdx.x];
#pragma unroll
  for (int i = 0; i < ITEMS; ++i) {
    if (base + i < n) out[base + i] = run;
    run += v[i];
  }
  if (total && blockIdx.x == gridDim.x - 1 && threadIdx.x == blockDim.x - 1) *total = run;
}

// One block of 1024 threads scans up to kScanOneBlock elements in one launch.
constexpr int kScanOneThreads = 1024;
constexpr int kScanOneItems = 16;
constexpr int64_t kScanOneBlock = (int64_t)kScanOneThreads * kScanOneItems;

}  // namespace

template <class T>
size_t scan_tmp_elems(int64_t n) {
  size_t total = 0;
  while (n > kScanTile) {
    n = (n + kScanTile - 1) / kScanTile;
    total += (size_t)n + 64;
  }
  return total + 64;
}

template <class T>
void exclusive_scan(const T* in, T* out, int64_t n, T* total, T* tmp, hipStream_t s) {
  if (n <= 0) {
    if (total) (void)hipMemsetAsync(total, 0, sizeof(T), s);
    return;
  }
  if (n <= kScanTile) {
    k_scan_down<T><<<1, kScanThreads, 0, s>>>(in, out, n, nullptr, total);
    return;
  }
  if (n <= kScanOneBlock) {
    k_scan_down<T, kScanOneThreads, kScanOneItems>
        <<<1, kScanOneThreads, 0, s>>>(in, out, n, nullptr, total);
    return;
  }
  int64_t nb = (n + kScanTile - 1) / kScanTile;
  T* part = tmp;
  T* rest = tmp + nb + 64;
  k_scan_reduce<T><<<(unsigned)nb, kScanThreads, 0, s>>>(in, n, part);
  exclusive_scan<T>(part, part, nb, nullptr, rest, s);
  k_scan_down<T><<<(unsigned)nb, kScanThreads, 0, s>>>(in, out, n, part, total);
}

template size_t scan_tmp_elems<uint32_t>(int64_t);
template size_t scan_tmp_elems<unsigned long long>(int64_t);
template void exclusive_scan<uint32_t>(const uint32_t*, uint32_t*, int64_t, uint32_t*,
                                       uint32_t*, hipStream_t);
template void exclusive_scan<unsigned long long>(const unsigned long long*,
                                                 unsigned long long*, int64_t,
                                                 unsigned long long*, unsigned long long*,
                                                 hipStream_t);

// ------------------------------------------------------------ radix sort --
namespace {

constexpr int kRsThreads = 256;
constexpr int kRsWaves = kRsThreads / kWave;
constexpr int kRsItems = 8;
constexpr int kRsTile = kRsThreads * kRsItems;  // 2048 keys per block

template <class K>
__global__ void __launch_bounds__(kRsThreads) k_rs_hist(const K* keys, int64_t n, int shift,
                                                        uint32_t* hist, int nblocks) {
  __shared__ uint32_t h[kRsWaves][256];
  const int wid = threadIdx.x / kWave;
  for (int i = threadIdx.x; i < kRsWaves * 256; i += kRsThreads) (&h[0][0])[i] = 0;
  __syncthreads();
  int64_t base = (int64_t)blockIdx.x * kRsTile;
#pragma unroll
  for (int i = 0; i < kRsItems; ++i) {
    int64_t k = base + (int64_t)i * kRsThreads + threadIdx.x;
    if (k < n) atomicAdd(&h[wid][(uint32_t)(keys[k] >> shift) & 255u], 1u);
  }
  __syncthreads();
  uint32_t t = 0;
#pragma unroll
  for (int w = 0; w < kRsWaves; ++w) t += h[w][threadIdx.x];
  hist[(int64_t)threadIdx.x * nblocks + blockIdx.x] = t;
}

// Stable scatter: each wave ranks its keys with a ballot-based match of the
// 8-bit digit, the block places keys in LDS in digit order, then writes each
// digit run to its global offset.
template <class K>
__global__ void __launch_bounds__(kRsThreads) k_rs_scatter(const K* kin, const uint32_t* vin,
                                                           K* kout, uint32_t* vout, int64_t n,
                                                           int shift, const uint32_t* offs,
                                                           int nblocks) {
  __shared__ uint32_t wcnt[kRsWaves][256];
  __shared__ uint32_t dstart[256];
  __shared__ uint32_t scan_lds[kRsWaves + 1];
  __shared__ K skey[kRsTile];
  __shared__ uint32_t sval[kRsTile];
  const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave;
  for (int i = threadIdx.x; i < kRsWaves * 256; i += kRsThreads) (&wcnt[0][0])[i] = 0;
  __syncthreads();
  const int64_t base = (int64_t)blockIdx.x * kRsTile;
  K key[kRsItems];
  uint32_t val[kRsItems], rank[kRsItems], dig[kRsItems];
  const unsigned long long lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
#pragma unroll
  for (int c = 0; c < kRsItems; ++c) {
    int64_t idx = base + ((int64_t)wid * kRsItems + c) * kWave + lane;
    bool ok = idx < n;
    key[c] = ok ? kin[idx] : (K)~(K)0;
    val[c] = ok ? vin[idx] : 0u;
    uint32_t d = ok ? ((uint32_t)(key[c] >> shift) & 255u) : 255u;
    dig[c] = d;
    unsigned long long mask = ~0ull;
#pragma unroll
    for (int b = 0; b < 8; ++b) {
      unsigned long long bb = __ballot((d >> b) & 1u);
      mask &= ((d >> b) & 1u) ? bb : ~bb;
    }
    int leader = __ffsll((long long)mask) - 1;
    uint32_t cnt = (uint32_t)__popcll(mask);
    uint32_t pre = (uint32_t)__popcll(mask & lt);
    uint32_t old = 0;
    if (lane == leader) old = atomicAdd(&wcnt[wid][d], cnt);
    old = __shfl(old, leader);
    rank[c] = old + pre;
  }
  __syncthreads();
  // wave prefix within each digit, then block-wide digit starts
  {
    const int d = threadIdx.x;
    uint32_t run = 0;
#pragma unroll
    for (int w = 0; w < kRsWaves; ++w) {
      uint32_t t = wcnt[w][d];
      wcnt[w][d] = run;
      run += t;
    }
    uint32_t tot;
    uint32_t ex = block_exclusive_scan<uint32_t>(run, &tot, scan_lds);
    dstart[d] = ex;
  }
  __syncthreads();
#pragma unroll
  for (int c = 0; c < kRsItems; ++c) {
    uint32_t lp = dstart[dig[c]] + wcnt[wid][dig[c]] + rank[c];
    skey[lp] = key[c];
    sval[lp] = val[c];
  }
  __syncthreads();
  int64_t valid = n - base;
  if (valid > kRsTile) valid = kRsTile;
#pragma unroll
  for (int i = 0; i < kRsItems; ++i) {
    int lp = i * kRsThreads + threadIdx.x;
    if (lp < valid) {
      K k = skey[lp];
      uint32_t d = (uint32_t)(k >> shift) & 255u;
      int64_t g = (int64_t)offs[(int64_t)d * nblocks + blockIdx.x] + (lp - dstart[d]);
      kout[g] = k;
      vout[g] = sval[lp];
    }
  }
}

}  // namespace

size_t radix_tmp_bytes(int64_t n) {
  int64_t nb = (n + kRsTile - 1) / kRsTile;
  if (nb < 1) nb = 1;
  size_t hist = (size_t)nb * 256;
  return (hist + scan_tmp_elems<uint32_t>((int64_t)hist) + 128) * sizeof(uint32_t);
}

template <class K>
bool radix_sort_pairs(K* k0, uint32_t* v0, K* k1, uint32_t* v1, int64_t n, int bits,
                      void* tmp, hipStream_t s) {
  if (n <= 1 || bits <= 0) return false;
  int64_t nb = (n + kRsTile - 1) / kRsTile;
  uint32_t* hist = static_cast<uint32_t*>(tmp);
  uint32_t* stmp = hist + (size_t)nb * 256 + 64;
  bool flip = false;
  for (int shift = 0; shift < bits; shift += 8) {
    K* ki = flip ? k1 : k0;
    K* ko = flip ? k0 : k1;
    uint32_t* vi = flip ? v1 : v0;
    uint32_t* vo = flip ? v0 : v1;
    k_rs_hist<K><<<(unsigned)nb, kRsThreads, 0, s>>>(ki, n, shift, hist, (int)nb);
    exclusive_scan<uint32_t>(hist, hist, nb * 256, nullptr, stmp, s);
    k_rs_scatter<K><<<(unsigned)nb, kRsThreads, 0, s>>>(ki, vi, ko, vo, n, shift, hist, (int)nb);
    flip = !flip;
  }
  return flip;
}

template bool radix_sort_pairs<uint32_t>(uint32_t*, uint32_t*, uint32_t*, uint32_t*, int64_t,
                                         int, void*, hipStream_t);
template bool radix_sort_pairs<unsigned long long>(unsigned long long*, uint32_t*,
                                                   unsigned long long*, uint32_t*, int64_t,
                                                   int, void*, hipStream_t);

void build_worklist(const uint32_t* item_count, int64_t K, uint32_t* off, uint32_t* item_seg,
                    uint32_t* item_idx, int64_t max_items, uint32_t* tmp, hipStream_t s) {
  (void)item_seg;
  (void)item_idx;
  (void)max_items;
  exclusive_scan<uint32_t>(item_count, off, K, off + K, tmp, s);
}

__global__ void k_iota(uint32_t* a, int64_t n) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) a[i] = (uint32_t)i;
}

__global__ void k_fill_u32(uint32_t* a, int64_t n, uint32_t v) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) a[i] = v;
}

__global__ void k_fill_u64(unsigned long long* a, int64_t n, unsigned long long v) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) a[i] = v;
}

}  // namespace halo
