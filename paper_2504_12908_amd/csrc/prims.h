// Device-wide primitives: exclusive scan of int32 and a stable LSD radix sort of
// (uint64 key, int32 value) pairs.  Both are deterministic.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace tc {

// Scratch sizes (bytes) needed by the primitives for n elements.
size_t scan_scratch_bytes(int n);
size_t sort_scratch_bytes(int n);

// out[i] = sum_{k<i} in[i]; *d_total (device) = sum of all.  in and out may alias.
hipError_t exclusive_scan(const int* in, int* out, int n, int* d_total, void* scratch,
                          hipStream_t s);

// Sorts keys[0..n) ascending (bits [0, end_bit) are significant) carrying vals; stable.
// keys/vals are overwritten with the result; tmp_keys/tmp_vals hold n elements each.
hipError_t radix_sort_pairs(uint64_t* keys, int* vals, uint64_t* tmp_keys, int* tmp_vals,
                            int n, int end_bit, void* scratch, hipStream_t s);

}  // namespace tc
