// Small device utilities: fills, the box table, and a multi-level exclusive scan.
#include <map>
#include <mutex>
#include <tuple>

#include "nf_internal.h"

namespace anf {

__global__ void k_write_box_table(BoxChunk chunk, DevBox* __restrict__ dev) {
  const int i = threadIdx.x;
  if (i < chunk.count) dev[chunk.offset + i] = chunk.b[i];
}

hipError_t write_box_table(const DevBox* host_boxes, int nboxes, DevBox* dev, hipStream_t s) {
  for (int off = 0; off < nboxes; off += kBoxChunk) {
    BoxChunk c;
    c.count = nboxes - off < kBoxChunk ? nboxes - off : kBoxChunk;
    c.offset = off;
    for (int i = 0; i < c.count; ++i) c.b[i] = host_boxes[off + i];
    hipLaunchKernelGGL(k_write_box_table, dim3(1), dim3(64), 0, s, c, dev);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

__global__ void k_fill_i32(int32_t* __restrict__ p, int32_t v, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = v;
}

__global__ void k_fill_i64(int64_t* __restrict__ p, int64_t v, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = v;
}

static dim3 fill_grid(int64_t n) {
  int64_t b = (n + 255) / 256;
  if (b < 1) b = 1;
  if (b > 8192) b = 8192;
  return dim3((unsigned)b);
}

hipError_t fill_i32(int32_t* p, int32_t v, int64_t n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill_i32, fill_grid(n), dim3(256), 0, s, p, v, n);
  return hipGetLastError();
}

hipError_t fill_i64(int64_t* p, int64_t v, int64_t n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill_i64, fill_grid(n), dim3(256), 0, s, p, v, n);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Exclusive scan of m = n + 1 values (the virtual in[n] is 0) so that out[n]
// is the total.  Level 1 scans tiles of kScanTile values inside a block and
// writes each tile's total; the totals are scanned recursively and added back.
// ---------------------------------------------------------------------------

__device__ __forceinline__ int wave_inclusive_scan(int v) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const int t = __shfl_up(v, d, 64);
    if (lane >= d) v += t;
  }
  return v;
}

__global__ __launch_bounds__(kScanThreads) void k_scan_tiles(const int32_t* __restrict__ in,
                                                             int32_t* __restrict__ out,
                                                             int64_t n, int64_t m,
                                                             int32_t* __restrict__ tile_sums) {
  __shared__ int wave_tot[kScanThreads / 64];
  const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
  const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)t * kScanItems;
  int v[kScanItems];
  int sum = 0;
#pragma unroll
  for (int k = 0; k < kScanItems; ++k) {
    const int64_t i = base + k;
    v[k] = (i < n) ? in[i] : 0;
    sum += v[k];
  }
  const int incl = wave_inclusive_scan(sum);
  if (lane == 63) wave_tot[wv] = incl;
  __syncthreads();
  int before = 0;
  for (int w = 0; w < wv; ++w) before += wave_tot[w];
  int run = before + incl - sum;
#pragma unroll
  for (int k = 0; k < kScanItems; ++k) {
    const int64_t i = base + k;
    if (i < m) out[i] = run;
    run += v[k];
  }
  if (t == kScanThreads - 1) {
    int tot = 0;
    for (int w = 0; w < kScanThreads / 64; ++w) tot += wave_tot[w];
    tile_sums[blockIdx.x] = tot;
  }
}

__global__ __launch_bounds__(kScanThreads) void k_scan_add(int32_t* __restrict__ out, int64_t m,
                                                           const int32_t* __restrict__ tile_pref) {
  const int32_t add = tile_pref[blockIdx.x];
  if (add == 0) return;
  const int64_t base = (int64_t)blockIdx.x * kScanTile;
  for (int k = threadIdx.x; k < kScanTile; k += kScanThreads) {
    const int64_t i = base + k;
    if (i < m) out[i] += add;
  }
}

int64_t scan_tmp_ints(int64_t n) {
  int64_t total = 0, m = n + 1;
  while (true) {
    const int64_t tiles = (m + kScanTile - 1) / kScanTile;
    if (tiles <= 1) { total += 2; break; }
    total += tiles + (tiles + 1);
    m = tiles + 1;
  }
  return total + 64;
}

hipError_t exclusive_scan(const int32_t* in, int32_t* out, int64_t n, int32_t* tmp,
                          hipStream_t s) {
  const int64_t m = n + 1;
  const int64_t tiles = (m + kScanTile - 1) / kScanTile;
  int32_t* sums = tmp;
  hipLaunchKernelGGL(k_scan_tiles, dim3((unsigned)tiles), dim3(kScanThreads), 0, s, in, out, n, m,
                     sums);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || tiles <= 1) return e;
  int32_t* pref = sums + tiles;
  e = exclusive_scan(sums, pref, tiles, pref + tiles + 1, s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_scan_add, dim3((unsigned)tiles), dim3(kScanThreads), 0, s, out, m, pref);
  return hipGetLastError();
}

int persistent_blocks(const void* kernel, int threads) {
  static std::mutex mu;
  static std::map<std::tuple<int, const void*, int>, int> cache;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 1024;
  const auto key = std::make_tuple(dev, kernel, threads);
  {
    std::lock_guard<std::mutex> lock(mu);
    auto it = cache.find(key);
    if (it != cache.end()) return it->second;
  }
  int cus = 0, per_cu = 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
      cus <= 0)
    cus = 256;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, threads, 0) != hipSuccess ||
      per_cu <= 0)
    per_cu = 4;
  std::lock_guard<std::mutex> lock(mu);
  cache[key] = cus * per_cu;
  return cus * per_cu;
}

int resident_wave_capacity() {
  int dev = 0, cus = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
      cus <= 0)
    cus = 256;
  return cus * 32;
}

}  // namespace anf
