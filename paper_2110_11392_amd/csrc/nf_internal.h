// Internal declarations shared by the HIP translation units of libabacus_nf.
// Nothing here is part of the public ABI (include/abacus_nf.h is).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

#include "abacus_nf.h"

namespace anf {

// Sinks handled by one wavefront work item: one sink per lane of a wave64.
constexpr int kTile = 64;
// Largest number of sources summed into one FP32 partial before it is folded
// into the sink's accumulator (CHUNKED / COMPENSATED accumulation).
constexpr int kChunk = 64;
// Most cells one work item's 64 sinks may span along its pencil (the planner's
// span parameter is 1..kMaxSpan; kDefaultSpan unless the autotuner chose another).
constexpr int kMaxSpan = 3;
constexpr int kDefaultSpan = 2;
// Cost buckets for the longest-first work queue (floor(log2 cost) descending).
constexpr int kBuckets = 64;
// Radix sort: 8-bit digits, 256 threads x 16 keys per block.
constexpr int kRadixBits = 8;
constexpr int kRadixThreads = 256;
constexpr int kRadixItems = 16;
constexpr int kRadixTile = kRadixThreads * kRadixItems;
// Device scan: 256 threads x 8 elements per block.
constexpr int kScanThreads = 256;
constexpr int kScanItems = 8;
constexpr int kScanTile = kScanThreads * kScanItems;
// Momentum reduction: chunks per box.
constexpr int kMomChunks = 64;
// r^2 guard: added to every squared separation so that coincident particles
// (r = 0, including a particle with itself) give a finite f and zero force.
constexpr float kTinyR2 = 1e-24f;

// Per-box parameters resolved on the host (step a1 of the path) and kept in
// device memory.  Lengths in the kernels are in cell widths w = L/K.
struct DevBox {
  int64_t first;        // first particle of the box (global index, also first sorted slot)
  int64_t n;            // particles in the box
  int32_t cell_base;    // first global cell id
  int32_t K;            // cells per dimension
  int32_t R;            // near-field radius in cells
  int32_t pencil_base;  // first global pencil id (pencils are (x, y) columns along z)
  double cells_per_len; // K / L: global coordinate -> cell units
  float inv_w2;         // 1/w^2: cell-unit acceleration -> box units
  float inv_w3;         // 1/w^3: cell-unit gradient -> box units
  float c0, c1, c2;     // f(r) = c0 + c1 r + c2 r^2 for r < eps (cell units), Eq. 3
  float eps;            // eps_s / w
  float ha, hb;         // h(r) = f'(r)/r = ha + hb / r for r < eps (cell units)
  int32_t far_newton;   // 1 if eps < 1/2 cell: cells >= 2 apart on an axis hold only r > eps pairs
  int32_t pad_;
};

constexpr int kBoxChunk = 24;  // boxes per table-writing launch (kernel argument size)
struct BoxChunk {
  DevBox b[kBoxChunk];
  int count;
  int offset;
};

// Locate the box owning a value v among nb boxes given a monotone key.
__device__ __forceinline__ int find_box_by_first(const DevBox* __restrict__ boxes, int nb,
                                                 int64_t i) {
  int lo = 0, hi = nb - 1;
  while (lo < hi) {
    int mid = (lo + hi + 1) >> 1;
    if (boxes[mid].first <= i) lo = mid; else hi = mid - 1;
  }
  return lo;
}

__device__ __forceinline__ int find_box_by_pencil(const DevBox* __restrict__ boxes, int nb,
                                                  int p) {
  int lo = 0, hi = nb - 1;
  while (lo < hi) {
    int mid = (lo + hi + 1) >> 1;
    if (boxes[mid].pencil_base <= p) lo = mid; else hi = mid - 1;
  }
  return lo;
}

// ---- launch helpers implemented in the .hip files (host side) -------------

// common.hip
hipError_t write_box_table(const DevBox* host_boxes, int nboxes, DevBox* dev, hipStream_t s);
hipError_t fill_i32(int32_t* p, int32_t v, int64_t n, hipStream_t s);
hipError_t fill_i64(int64_t* p, int64_t v, int64_t n, hipStream_t s);
// Exclusive scan of in[0..n) into out[0..n]; out[n] = total.  tmp must hold
// scan_tmp_ints(n) ints.
int64_t scan_tmp_ints(int64_t n);
hipError_t exclusive_scan(const int32_t* in, int32_t* out, int64_t n, int32_t* tmp,
                          hipStream_t s);

// bin.hip
struct BinWork {
  int32_t* counts;   // cells_total
  int32_t* keys[2];  // n_total each
  int32_t* vals[2];  // n_total each
  int32_t* hist;     // 256 * radix blocks
  int32_t* hist_scan;// 256 * radix blocks + 1
  int32_t* scan_tmp;
};
int64_t radix_blocks(int64_t n);
hipError_t launch_bin(const DevBox* boxes, int nboxes, int64_t n_total, int64_t cells_total,
                      const float* pos, const abacus_nf_binned* out, const BinWork& w,
                      hipStream_t s);

// plan.hip
struct PlanWork {
  int32_t* pencil_counts;  // pencils_total
  int32_t* item_base;      // pencils_total + 1 (item_base[pencils_total] = item count)
  int4* items;             // max_items
  int32_t* item_bucket;    // max_items: cost bucket of each item
  int32_t* item_slot;      // max_items: position of the item inside its bucket
  int32_t* queue;          // max_items
  int32_t* ctrl;           // kBuckets*3 + 8: counts, bases, cursors, head
  int32_t* scan_tmp;
  int64_t max_items;
};
int64_t plan_max_items(int64_t n_total, int64_t cells_total, int64_t pencils_total);
hipError_t launch_plan(const DevBox* boxes, int nboxes, int64_t pencils_total,
                       const int32_t* cell_offsets, int span, const PlanWork& w, hipStream_t s);
inline int32_t* plan_head(const PlanWork& w) { return w.ctrl + 3 * kBuckets; }
inline const int32_t* plan_n_items(const PlanWork& w, int64_t pencils_total) {
  return w.item_base + pencils_total;
}

// Tunable launch shape of a pair kernel (chosen by the autotuner in tune.hip).
struct KernelConfig {
  int unroll;     // sources per step of the inner loop (2, 4 or 8)
  int pipeline;   // 1: request the next step's sources before using the current ones
  int span;       // most cells one work item may span (1..3); a planner parameter
  int grid_mult;  // persistent workgroups per resident slot (1 or 2)
};
KernelConfig default_config(int kernel);  // kernel 0: forward, 1: adjoint
bool config_valid(int kernel, const KernelConfig& c);

// Problem signature under which a tuned shape is stored (tune.hip).
struct TuneKey {
  int kernel;           // 0 forward, 1 adjoint
  uint32_t mode;        // accumulation flags
  int nboxes;
  int64_t n_total, cells_total;
  uint64_t shape_hash;  // FNV-1a over the box list
};
KernelConfig lookup_config(const TuneKey& k);
void store_config(const TuneKey& k, const KernelConfig& c, bool persist);
void clear_config(const TuneKey& k);

// pairs.hip
enum AccMode { kAccSingle = 0, kAccChunked = 1, kAccCompensated = 2 };
hipError_t launch_forward(AccMode mode, bool count_pairs, const KernelConfig& cfg,
                          const DevBox* boxes, const PlanWork& w, int64_t pencils_total,
                          const int32_t* cell_offsets, const float* rel, const int32_t* perm,
                          float* acc, int64_t* pair_count, hipStream_t s);

// vjp.hip
hipError_t launch_vjp(AccMode mode, const KernelConfig& cfg, const DevBox* boxes,
                      const PlanWork& w, int64_t pencils_total, const int32_t* cell_offsets,
                      const float* rel, const int32_t* perm, const float* wvec, float4* src_w,
                      int64_t n_total, float* grad, hipStream_t s);

// reduce.hip
hipError_t launch_momentum(const DevBox* boxes, int nboxes, int64_t max_box_n, const float* acc,
                           double* partials, double* momentum, hipStream_t s);

// Occupancy-sized persistent grid for a kernel (cached per device and kernel).
int persistent_blocks(const void* kernel, int threads);

}  // namespace anf
