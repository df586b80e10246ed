// Device-wide primitives: exclusive scan, stable LSD radix sort, worklists.
#pragma once

#include "common.hpp"

namespace halo {

// out[i] = sum_{j<i} in[i]; returns nothing; *total (device) = sum of all.
// in and out may alias.  tmp needs scan_tmp_elems(n) elements of T.
template <class T>
size_t scan_tmp_elems(int64_t n);
template <class T>
void exclusive_scan(const T* in, T* out, int64_t n, T* total, T* tmp, hipStream_t s);

// Stable LSD radix sort of (key, value) pairs on the low `bits` bits of the
// keys, 8 bits per pass.  Sorts (k0, v0) using (k1, v1) as ping-pong buffers;
// returns true if the result lies in (k1, v1), false if in (k0, v0).
// tmp needs radix_tmp_bytes(n) bytes.
size_t radix_tmp_bytes(int64_t n);
template <class K>
bool radix_sort_pairs(K* k0, uint32_t* v0, K* k1, uint32_t* v1, int64_t n, int bits,
                      void* tmp, hipStream_t s);

// Worklist of fixed-size items over segments: segment k of length len[k]
// contributes items[k] = f(len[k]) items (f chosen by the caller through
// item_count[]), item w -> (segment, index within segment).
// off[] receives the exclusive scan of item_count (K+1 entries, off[K] = total).
void build_worklist(const uint32_t* item_count, int64_t K, uint32_t* off, uint32_t* item_seg,
                    uint32_t* item_idx, int64_t max_items, uint32_t* tmp, hipStream_t s);

__global__ void k_iota(uint32_t* a, int64_t n);
__global__ void k_fill_u32(uint32_t* a, int64_t n, uint32_t v);
__global__ void k_fill_u64(unsigned long long* a, int64_t n, unsigned long long v);

inline int bits_for(uint64_t maxval) {
  int b = 0;
  while (b < 64 && (maxval >> b) != 0) ++b;
  return b;
}

}  // namespace halo
