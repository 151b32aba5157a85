// Cell binning: FP64 cell assignment, a stable LSD radix sort of (cell,
// particle), the cell offsets read off the sorted keys, and the gather of FP32
// cell-relative offsets.
//
// Sec. 2.2: particles live on a K^3 grid of cells, slabs along x, pencils
// along z, so the linear cell id is (x K + y) K + z.  Sec. 3.5.1: positions are
// kept as FP32 offsets from their cell centre.  The sort is stable (ascending
// original index inside a cell), which makes the sorted order unique and the
// binning bit-reproducible.
//
// All arithmetic that decides a cell or an offset is FP64 and written as single
// IEEE operations (this file is built without FP contraction):
//   t = x * (K/L);  c = floor(t) mod K;  offset = (float)(t - (floor(t) + 0.5)).
#include "nf_internal.h"

namespace anf {

// The box of particle (or sorted slot) i.  A block covers consecutive indices;
// it stages the boxes' first indices in LDS once (up to kLdsBoxes boxes), and
// each thread's binary search then reads LDS instead of walking a chain of
// dependent global loads (six of them for 64 boxes).  Larger batches search
// the box table itself.
constexpr int kLdsBoxes = 1024;

__device__ __forceinline__ void stage_box_firsts(const DevBox* __restrict__ boxes, int nboxes,
                                                 int64_t* s_first) {
  if (nboxes > 1 && nboxes <= kLdsBoxes) {  // uniform over the block
    for (int k = threadIdx.x; k < nboxes; k += blockDim.x) s_first[k] = boxes[k].first;
    __syncthreads();
  }
}

__device__ __forceinline__ int box_of(const DevBox* __restrict__ boxes, int nboxes,
                                      const int64_t* s_first, int64_t i) {
  if (nboxes == 1) return 0;
  if (nboxes > kLdsBoxes) return find_box_by_first(boxes, nboxes, i);
  int lo = 0, hi = nboxes - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (s_first[mid] <= i) lo = mid; else hi = mid - 1;
  }
  return lo;
}

// Pass 1: global cell id per particle and key/value init.  (No per-cell
// counting here: device-wide atomics on the counts of crowded cells cost more
// than the whole radix sort; the offsets are found in the sorted keys instead.)
__global__ __launch_bounds__(256) void k_bin_assign(const DevBox* __restrict__ boxes, int nboxes,
                                                    int64_t n_total, const float* __restrict__ pos,
                                                    int32_t* __restrict__ keys,
                                                    int32_t* __restrict__ vals,
                                                    int32_t* __restrict__ status) {
  __shared__ int64_t s_first[kLdsBoxes];
  stage_box_firsts(boxes, nboxes, s_first);
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n_total) return;
  const int b = box_of(boxes, nboxes, s_first, i);
  const double cpl = boxes[b].cells_per_len;
  const int K = boxes[b].K;
  const CellCoord x = cell_coord(pos[3 * i + 0], cpl, K);
  const CellCoord y = cell_coord(pos[3 * i + 1], cpl, K);
  const CellCoord z = cell_coord(pos[3 * i + 2], cpl, K);
  if (!(x.ok && y.ok && z.ok)) atomicOr(status, ABACUS_NF_STATUS_BADPOS);
  const int cell = boxes[b].cell_base + (x.c * K + y.c) * K + z.c;
  keys[i] = cell;
  vals[i] = (int32_t)i;
}

// Cell offsets from the sorted keys: offsets[c] is the first slot whose key is
// at least c (a lower bound found by binary search), so offsets[cells] = n and
// an empty cell gets the start of the next occupied one.  One thread per cell:
// the work is balanced however the particles are spread (a scan over slots
// would hand a long run of empty cells to a single thread).
__global__ __launch_bounds__(256) void k_cell_offsets(const int32_t* __restrict__ sorted_keys,
                                                      int64_t n, int64_t cells,
                                                      int32_t* __restrict__ offsets,
                                                      int32_t* __restrict__ status) {
  const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c > cells) return;
  int64_t lo = 0, hi = n;
  while (lo < hi) {
    const int64_t mid = (lo + hi) >> 1;
    if (sorted_keys[mid] < c) lo = mid + 1; else hi = mid;
  }
  offsets[c] = (int32_t)lo;
  // cell c holds more than kMaxCellParticles iff its key is still found that
  // many slots on (a load only when the array reaches that far)
  if (lo + kMaxCellParticles < n && sorted_keys[lo + kMaxCellParticles] == c)
    atomicOr(status, ABACUS_NF_STATUS_CELLFULL);
}

// Radix pass, step 1: per-block digit histogram, stored digit-major so that one
// exclusive scan gives every (digit, block) its first output slot.
__global__ __launch_bounds__(kRadixThreads) void k_radix_hist(const int32_t* __restrict__ keys,
                                                              int64_t n, int shift,
                                                              int32_t* __restrict__ hist,
                                                              int nblocks) {
  __shared__ int h[256];
  const int t = threadIdx.x;
  h[t] = 0;
  __syncthreads();
  const int64_t base = (int64_t)blockIdx.x * kRadixTile;
#pragma unroll
  for (int k = 0; k < kRadixItems; ++k) {
    const int64_t i = base + (int64_t)k * kRadixThreads + t;
    if (i < n) atomicAdd(&h[(keys[i] >> shift) & 255], 1);
  }
  __syncthreads();
  hist[(int64_t)t * nblocks + blockIdx.x] = h[t];
}

// Radix pass, step 2: stable scatter.  The block first ranks its tile in LDS:
// walking its keys in index order, 256 at a time, the rank of a key among equal
// digits comes from eight ballots inside a wave and from per-wave digit counts
// across waves; each key lands at its digit's local start (an exclusive scan of
// the block's digit histogram) plus that rank.  The tile, now grouped by digit
// and stable inside each digit, is then written out so that consecutive
// threads write consecutive slots of a digit's run (coalesced, instead of one
// scattered word per key).
__global__ __launch_bounds__(kRadixThreads) void k_radix_scatter(
    const int32_t* __restrict__ keys_in, const int32_t* __restrict__ vals_in, int64_t n, int shift,
    const int32_t* __restrict__ hist, const int32_t* __restrict__ hist_scan, int nblocks,
    int32_t* __restrict__ keys_out, int32_t* __restrict__ vals_out) {
  constexpr int kWaves = kRadixThreads / 64;
  static_assert(kRadixThreads == 256, "one thread per digit");
  __shared__ int base[256], lstart[256], gbase[256];
  __shared__ int wcount[kWaves][256];
  __shared__ int32_t skey[kRadixTile], sval[kRadixTile];
  const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
  // local digit starts: exclusive scan of this block's digit counts
  const int cnt = hist[(int64_t)t * nblocks + blockIdx.x];
  lstart[t] = cnt;
  __syncthreads();
  for (int d = 1; d < 256; d <<= 1) {  // inclusive Hillis-Steele scan
    const int a = t >= d ? lstart[t - d] : 0;
    __syncthreads();
    lstart[t] += a;
    __syncthreads();
  }
  const int excl = lstart[t] - cnt;
  __syncthreads();
  lstart[t] = excl;
  base[t] = excl;
  gbase[t] = hist_scan[(int64_t)t * nblocks + blockIdx.x];
  const uint64_t below = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
  const int64_t block0 = (int64_t)blockIdx.x * kRadixTile;
  for (int k = 0; k < kRadixItems; ++k) {
    for (int w = 0; w < kWaves; ++w) wcount[w][t] = 0;
    __syncthreads();
    const int64_t i = block0 + (int64_t)k * kRadixThreads + t;
    const bool valid = i < n;
    int key = 0, val = 0, d = 0;
    if (valid) {
      key = keys_in[i];
      val = vals_in[i];
      d = (key >> shift) & 255;
    }
    uint64_t peers = __ballot(valid);
#pragma unroll
    for (int bit = 0; bit < kRadixBits; ++bit) {
      const bool on = (d >> bit) & 1;
      const uint64_t m = __ballot(on);
      peers &= on ? m : ~m;
    }
    const int rank = __popcll(peers & below);
    if (valid && rank == 0) wcount[wv][d] = __popcll(peers);
    __syncthreads();
    if (valid) {
      int pos = base[d] + rank;
      for (int w = 0; w < wv; ++w) pos += wcount[w][d];
      skey[pos] = key;
      sval[pos] = val;
    }
    __syncthreads();
    int add = 0;
    for (int w = 0; w < kWaves; ++w) add += wcount[w][t];
    base[t] += add;
    // base[] and wcount[] are read again only after the barrier at the top
    // of the next round.
  }
  __syncthreads();
  const int64_t left = n - block0;
  const int ntile = left < kRadixTile ? (int)left : kRadixTile;
  for (int j = t; j < ntile; j += kRadixThreads) {
    const int key = skey[j];
    const int d = (key >> shift) & 255;
    const int g = gbase[d] + (j - lstart[d]);
    keys_out[g] = key;
    vals_out[g] = sval[j];
  }
}

// Sorted slot -> FP32 cell-relative offsets (same FP64 formula as assignment).
__global__ __launch_bounds__(256) void k_gather_rel(const DevBox* __restrict__ boxes, int nboxes,
                                                    int64_t n_total, const float* __restrict__ pos,
                                                    const int32_t* __restrict__ perm,
                                                    float4* __restrict__ rel) {
  __shared__ int64_t s_first[kLdsBoxes];
  stage_box_firsts(boxes, nboxes, s_first);
  const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= n_total) return;
  const int b = box_of(boxes, nboxes, s_first, s);
  const double cpl = boxes[b].cells_per_len;
  const int K = boxes[b].K;
  const int64_t i = perm[s];
  const CellCoord x = cell_coord(pos[3 * i + 0], cpl, K);
  const CellCoord y = cell_coord(pos[3 * i + 1], cpl, K);
  const CellCoord z = cell_coord(pos[3 * i + 2], cpl, K);
  rel[s] = make_float4(x.off, y.off, z.off, 0.0f);
}

__global__ void k_iota(int32_t* __restrict__ p, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = (int32_t)i;
}

int64_t radix_blocks(int64_t n) { return n <= 0 ? 1 : (n + kRadixTile - 1) / kRadixTile; }

static int key_bits(int64_t cells_total) {
  int bits = 0;
  while (bits < 31 && (int64_t(1) << bits) < cells_total) ++bits;
  return bits;
}

#define ANF_TRY(x)                      \
  do {                                  \
    hipError_t e_ = (x);                \
    if (e_ != hipSuccess) return e_;    \
  } while (0)

hipError_t launch_bin(const DevBox* boxes, int nboxes, int64_t n_total, int64_t cells_total,
                      const float* pos, const abacus_nf_binned* out, const BinWork& w,
                      hipStream_t s) {
  ANF_TRY(fill_i32(out->status, 0, 1, s));
  if (n_total == 0) return fill_i32(out->cell_offsets, 0, cells_total + 1, s);
  {
    const unsigned g = (unsigned)((n_total + 255) / 256);
    hipLaunchKernelGGL(k_bin_assign, dim3(g), dim3(256), 0, s, boxes, nboxes, n_total, pos,
                       w.keys[0], w.vals[0], out->status);
    ANF_TRY(hipGetLastError());
  }

  const int bits = key_bits(cells_total);
  const int passes = (bits + kRadixBits - 1) / kRadixBits;
  const int nb = (int)radix_blocks(n_total);
  const int32_t* kin = w.keys[0];
  const int32_t* vin = w.vals[0];
  if (passes == 0) {
    hipLaunchKernelGGL(k_iota, dim3((unsigned)((n_total + 255) / 256)), dim3(256), 0, s, out->perm,
                       n_total);
    ANF_TRY(hipGetLastError());
  }
  for (int p = 0; p < passes; ++p) {
    const int shift = p * kRadixBits;
    const bool last = p == passes - 1;
    int32_t* kout = w.keys[(p + 1) & 1];
    int32_t* vout = last ? out->perm : w.vals[(p + 1) & 1];
    hipLaunchKernelGGL(k_radix_hist, dim3(nb), dim3(kRadixThreads), 0, s, kin, n_total, shift,
                       w.hist, nb);
    ANF_TRY(hipGetLastError());
    ANF_TRY(exclusive_scan(w.hist, w.hist_scan, (int64_t)256 * nb, w.scan_tmp, s));
    hipLaunchKernelGGL(k_radix_scatter, dim3(nb), dim3(kRadixThreads), 0, s, kin, vin, n_total,
                       shift, w.hist, w.hist_scan, nb, kout, vout);
    ANF_TRY(hipGetLastError());
    kin = kout;
    vin = vout;
  }
  // kin holds the sorted keys (the unsorted ones when no pass ran: a single cell)
  hipLaunchKernelGGL(k_cell_offsets, dim3((unsigned)((cells_total + 1 + 255) / 256)), dim3(256), 0,
                     s, kin, n_total, cells_total, out->cell_offsets, out->status);
  ANF_TRY(hipGetLastError());
  hipLaunchKernelGGL(k_gather_rel, dim3((unsigned)((n_total + 255) / 256)), dim3(256), 0, s, boxes,
                     nboxes, n_total, pos, out->perm, reinterpret_cast<float4*>(out->rel));
  return hipGetLastError();
}

}  // namespace anf
