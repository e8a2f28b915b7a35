// Device-wide exclusive scan and stable LSD radix sort (wave64, 256-thread workgroups).
#include "prims.h"

namespace tc {

namespace {

constexpr int kThreads = 256;
constexpr int kItems = 4;
constexpr int kTile = kThreads * kItems;

// Exclusive scan of one int per thread over a 256-thread workgroup.
__device__ int block_exclusive_scan(int v, int* lds, int* total) {
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  int x = v;
  for (int off = 1; off < 64; off <<= 1) {
    const int y = __shfl_up(x, off, 64);
    if (lane >= off) x += y;
  }
  if (lane == 63) lds[wid] = x;
  __syncthreads();
  int prefix = 0, tot = 0;
  for (int w = 0; w < kThreads / 64; ++w) {
    if (w < wid) prefix += lds[w];
    tot += lds[w];
  }
  __syncthreads();
  if (total) *total = tot;
  return prefix + x - v;
}

__global__ void __launch_bounds__(kThreads) k_tile_sums(const int* in, int n, int* sums) {
  __shared__ int lds[kThreads / 64];
  const int base = blockIdx.x * kTile + threadIdx.x * kItems;
  int s = 0;
  for (int k = 0; k < kItems; ++k)
    if (base + k < n) s += in[base + k];
  int tot;
  block_exclusive_scan(s, lds, &tot);
  if (threadIdx.x == 0) sums[blockIdx.x] = tot;
}

__global__ void __launch_bounds__(kThreads) k_tile_scan(const int* in, int* out, int n,
                                                        const int* offsets, int* d_total) {
  __shared__ int lds[kThreads / 64];
  const int base = blockIdx.x * kTile + threadIdx.x * kItems;
  int v[kItems];
  int s = 0;
  for (int k = 0; k < kItems; ++k) {
    v[k] = base + k < n ? in[base + k] : 0;
    s += v[k];
  }
  int tot;
  int run = block_exclusive_scan(s, lds, &tot) + (offsets ? offsets[blockIdx.x] : 0);
  for (int k = 0; k < kItems; ++k) {
    if (base + k < n) out[base + k] = run;
    run += v[k];
  }
  if (d_total && blockIdx.x == gridDim.x - 1 && threadIdx.x == kThreads - 1) *d_total = run;
}

__global__ void k_zero_total(int* d_total) { *d_total = 0; }

// ---------------------------------------------------------------- radix sort
__global__ void __launch_bounds__(kThreads) k_digit_hist(const uint64_t* keys, int n, int shift,
                                                         int ntiles, int* counts) {
  __shared__ int hist[256];
  hist[threadIdx.x] = 0;
  __syncthreads();
  for (int r = 0; r < kItems; ++r) {
    const int e = blockIdx.x * kTile + r * kThreads + threadIdx.x;
    if (e < n) atomicAdd(&hist[(int)((keys[e] >> shift) & 255u)], 1);
  }
  __syncthreads();
  counts[threadIdx.x * ntiles + blockIdx.x] = hist[threadIdx.x];
}

__global__ void __launch_bounds__(kThreads) k_digit_scatter(const uint64_t* keys, const int* vals,
                                                            uint64_t* okeys, int* ovals, int n,
                                                            int shift, int ntiles,
                                                            const int* offsets) {
  __shared__ int wcount[kThreads / 64][256];
  __shared__ int running[256];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  running[threadIdx.x] = offsets[threadIdx.x * ntiles + blockIdx.x];
  const unsigned long long lt = lane == 0 ? 0ull : (~0ull >> (64 - lane));
  for (int r = 0; r < kItems; ++r) {
    for (int w = 0; w < kThreads / 64; ++w) wcount[w][threadIdx.x] = 0;
    __syncthreads();
    const int e = blockIdx.x * kTile + r * kThreads + threadIdx.x;
    const bool valid = e < n;
    uint64_t key = 0;
    int val = 0;
    int d = 0;
    if (valid) {
      key = keys[e];
      val = vals[e];
      d = (int)((key >> shift) & 255u);
    }
    unsigned long long peers = __ballot(valid);
    for (int b = 0; b < 8; ++b) {
      const bool bit = (d >> b) & 1;
      const unsigned long long m = __ballot(bit);
      peers &= bit ? m : ~m;
    }
    const int rank = __popcll(peers & lt);
    if (valid && rank == 0) wcount[wid][d] = __popcll(peers);
    __syncthreads();
    if (valid) {
      int pos = running[d] + rank;
      for (int w = 0; w < wid; ++w) pos += wcount[w][d];
      okeys[pos] = key;
      ovals[pos] = val;
    }
    __syncthreads();
    int add = 0;
    for (int w = 0; w < kThreads / 64; ++w) add += wcount[w][threadIdx.x];
    running[threadIdx.x] += add;
    __syncthreads();
  }
}

}  // namespace

size_t scan_scratch_bytes(int n) {
  size_t bytes = 0;
  int m = n;
  while (true) {
    const int tiles = (m + kTile - 1) / kTile;
    bytes += sizeof(int) * (size_t)(tiles + 1);
    if (tiles <= 1) break;
    m = tiles;
  }
  return bytes + 256;
}

hipError_t exclusive_scan(const int* in, int* out, int n, int* d_total, void* scratch,
                          hipStream_t s) {
  if (n <= 0) {
    if (d_total) hipLaunchKernelGGL(k_zero_total, dim3(1), dim3(1), 0, s, d_total);
    return hipGetLastError();
  }
  const int tiles = (n + kTile - 1) / kTile;
  if (tiles == 1) {
    hipLaunchKernelGGL(k_tile_scan, dim3(1), dim3(kThreads), 0, s, in, out, n, nullptr, d_total);
    return hipGetLastError();
  }
  int* sums = static_cast<int*>(scratch);
  hipLaunchKernelGGL(k_tile_sums, dim3(tiles), dim3(kThreads), 0, s, in, n, sums);
  hipError_t e = exclusive_scan(sums, sums, tiles, nullptr, sums + tiles + 1, s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_tile_scan, dim3(tiles), dim3(kThreads), 0, s, in, out, n, sums, d_total);
  return hipGetLastError();
}

size_t sort_scratch_bytes(int n) {
  const int tiles = (n + kTile - 1) / kTile;
  const int m = 256 * (tiles > 0 ? tiles : 1);
  return sizeof(int) * (size_t)m + scan_scratch_bytes(m) + 256;
}

hipError_t radix_sort_pairs(uint64_t* keys, int* vals, uint64_t* tmp_keys, int* tmp_vals, int n,
                            int end_bit, void* scratch, hipStream_t s) {
  if (n <= 1) return hipSuccess;
  const int tiles = (n + kTile - 1) / kTile;
  int* counts = static_cast<int*>(scratch);
  void* scan_tmp = counts + 256 * tiles;
  uint64_t* ka = keys;
  uint64_t* kb = tmp_keys;
  int* va = vals;
  int* vb = tmp_vals;
  int passes = 0;
  for (int shift = 0; shift < end_bit; shift += 8, ++passes) {
    hipLaunchKernelGGL(k_digit_hist, dim3(tiles), dim3(kThreads), 0, s, ka, n, shift, tiles, counts);
    hipError_t e = exclusive_scan(counts, counts, 256 * tiles, nullptr, scan_tmp, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_digit_scatter, dim3(tiles), dim3(kThreads), 0, s, ka, va, kb, vb, n, shift,
                       tiles, counts);
    uint64_t* tk = ka; ka = kb; kb = tk;
    int* tv = va; va = vb; vb = tv;
  }
  if (passes & 1) {
    hipError_t e = hipMemcpyAsync(keys, ka, sizeof(uint64_t) * n, hipMemcpyDeviceToDevice, s);
    if (e != hipSuccess) return e;
    e = hipMemcpyAsync(vals, va, sizeof(int) * n, hipMemcpyDeviceToDevice, s);
    if (e != hipSuccess) return e;
  }
  return hipGetLastError();
}

}  // namespace tc
