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
// Largest cells per dimension of a box (larger K is rejected with ERANGE).
constexpr int kMaxCellsPerDim = 2000;
constexpr int kMaxSpan = 3;
constexpr int kDefaultSpan = 2;
// Cost buckets for the longest-first work queue, descending: four per octave
// (floor(log2 cost) and the next two bits of the cost), so the queue's order
// is within 19% of exact longest-first.
constexpr int kBuckets = 128;
// ctrl layout (int32): bucket counts [kBuckets], bucket bases [kBuckets], then
// the task head, task count, whole-item tasks, split items and slices per item.
constexpr int kCtrlHead = 2 * kBuckets;
constexpr int kCtrlNTasks = kCtrlHead + 1;
constexpr int kCtrlNWhole = kCtrlHead + 2;
constexpr int kCtrlNSplit = kCtrlHead + 3;
constexpr int kCtrlSlices = kCtrlHead + 4;
constexpr int kCtrlInts = kCtrlHead + 8;
// Most particles one cell may hold: the pair kernels form record offsets
// inside a cell (up to 6 floats per particle) in 32 bits.
constexpr int64_t kMaxCellParticles = int64_t(1) << 28;
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
constexpr int kMomChunks = 1024;  // a multiple of 64 (the final pass: one wave per box)
// r^2 guard: added to every squared separation so that coincident particles
// (r = 0, including a particle with itself) give a finite f and zero force.
constexpr float kTinyR2 = 1e-24f;

// Accumulation of a sink's sum (see ABACUS_NF_SINGLE_ACC / CHUNKED / COMPENSATED).
enum AccMode { kAccSingle = 0, kAccChunked = 1, kAccCompensated = 2 };

// Error-free TwoSum of (a, t): a <- fl(a + t), e accumulates the rounding error.
__device__ __forceinline__ void two_sum_fold(float& a, float& e, float t) {
  const float s = a + t;
  const float bp = s - a;
  const float ap = s - bp;
  e += (a - ap) + (t - bp);
  a = s;
}

// Fold an x-offset slice (a, e) of a sink's sum into the total (A, E).  The
// pair kernels and k_combine_slices run this same function in the same slice
// order, so a sink's bits do not depend on whether its work item was split.
template <int kAcc>
__device__ __forceinline__ void slice_fold(float& A, float& E, float a, float e) {
  if (kAcc == kAccCompensated) {
    two_sum_fold(A, E, a);
    E += e;
  } else {
    A += a;
  }
}

// Work tasks: task = item << kTaskShift | code; code 0 runs the whole item,
// code c > 0 runs only x offset c - 1 - R (a slice of a split tail item).
constexpr int kTaskShift = 3;
constexpr int kTaskCodeMask = 7;
constexpr int kMaxSlices = 7;      // 2R + 1 for R <= 3; larger R is never split
constexpr int kMaxSplit = 8192;    // most tail items split per launch
// Floats kept per lane and slice of a split item: sum and error per axis, density.
constexpr int kPartialStride = 7;

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
  // Which source cells may use the plain f = (r^2 + guard)^(-3/2) branch:
  // kFarNone every cell needs the spline select; kFarApart cells >= 2 apart on
  // some axis (eps < 1/2 cell, so they hold only r > eps pairs); kFarAll every
  // cell (the Plummer law, Eq. 2).
  int32_t far_mode;
  float guard;          // added to every r^2 (cell units): tiny for Eq. 3, eps_p^2 for Eq. 2
  float b2;             // b^2 + guard, b the top-hat density radius (cell units); 0 if unused
  float inv_b2;         // 1 / b^2
  int32_t dens_far;     // 1 if b < 1/2 cell: cells >= 2 apart on an axis hold no pair within b
  int32_t chunk_base;   // first reduction chunk of the box (kick-drift statistics)
  double width;         // w = L / K (box units per cell width)
  double box_len;       // L
  double kick, drift;   // kick-drift step factors of this call
  double eps_cells64;   // the FP64 kernel's softening in cell widths: eps_s (Eq. 3) or eps_p (Eq. 2)
  float near2;          // (1.1 eps)^2 in cell units: pairs beyond it take 1/r^3 without the select
  int32_t sink_x0, sink_x1;  // the work plan takes sinks of the slabs x in [sink_x0, sink_x1) only
  int32_t pad2_;
};
constexpr int kFarNone = 0, kFarApart = 1, kFarAll = 2;

constexpr int kBoxChunk = 24;  // boxes per table-writing launch (kernel argument size)
struct BoxChunk {
  DevBox b[kBoxChunk];
  int count;
  int offset;
};
static_assert(sizeof(BoxChunk) <= 4096, "a box chunk is passed as one kernel argument");

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

__device__ __forceinline__ int find_box_by_cell(const DevBox* __restrict__ boxes, int nb,
                                                int64_t c) {
  int lo = 0, hi = nb - 1;
  while (lo < hi) {
    int mid = (lo + hi + 1) >> 1;
    if (boxes[mid].cell_base <= c) lo = mid; else hi = mid - 1;
  }
  return lo;
}

// Cell assignment of one FP32 coordinate (the binning's rule, also used by the
// kick-drift statistics to find a sorted slot's cell): t = x * (K/L) in FP64,
// the periodic index floor(t) mod K and the offset t - (floor(t) + 1/2)
// rounded once to FP32.  |t| must stay below 2^30 so the unwrapped cell fits
// comfortably in int32.  Files including this are built without contraction.
constexpr double kMaxCellCoord = 1073741824.0;

struct CellCoord {
  int c;        // periodic cell index in [0, K)
  float off;    // offset from the cell centre, cell units
  bool ok;
};

__device__ __forceinline__ CellCoord cell_coord(float x, double cpl, int K) {
  CellCoord r;
  const double t = (double)x * cpl;
  r.ok = (t == t) && fabs(t) < kMaxCellCoord;  // false for NaN, +-inf, huge
  if (!r.ok) { r.c = 0; r.off = 0.0f; return r; }
  const double fl = floor(t);
  int c = (int)fl;
  if ((unsigned)c >= (unsigned)K) {  // outside [0, K): the periodic image (rare)
    c %= K;
    if (c < 0) c += K;
  }
  r.c = c;
  r.off = (float)(t - (fl + 0.5));
  return r;
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

// multipoles.hip
constexpr int kMaxMultipoleOrder = 8;
constexpr int kMpBuckets = 240;  // bucket table entries (the kernel uses 234)
struct MpWork {
  int64_t cells;
  int32_t* keys;          // cells: bucket of each cell
  int32_t* hist;          // kMpBuckets: cells per bucket
  int32_t* bucket_base;   // kMpBuckets: first sorted slot of each bucket (+ total)
  int32_t* cursor;        // kMpBuckets: scatter cursors
  int32_t* bucket_waves;  // kMpBuckets: first work wave of each bucket (+ total)
  int32_t* sorted;        // cells: cell ids sorted by bucket
  int2* span;             // cells: (first particle, count) of each sorted cell
  double* full;           // cells_total x complete terms (only for the reduced basis)
  double* red_coef;       // 81 x 16 reduction coefficients (reduced basis only)
  int32_t* red_src;       // 81 x 16 complete-basis sources of each reduced term
  int32_t* red_cnt;       // 81 sources per reduced term
};
int64_t multipole_terms(int p, bool reduced);
hipError_t launch_multipoles(const DevBox* boxes, int nboxes, int64_t cells_total, int order,
                             bool reduced, const MpWork& w, const int32_t* cell_offsets,
                             const float* rel, double* out, hipStream_t s);

// kdk.hip
constexpr int kKdkChunk = 512;   // cells per statistics chunk
constexpr int kKdkTile = 512;   // sorted slots per block of the update
struct KdkRec {  // what one particle's update leaves for the statistics (32 bytes)
  double v2, a2;  // |v'|^2 and |a|^2
  int32_t cell;   // its cell in the binning
  int32_t pad[3];
};
static_assert(sizeof(KdkRec) == 32, "one 32-byte record per particle");
struct KdkWork {
  double* cell_sumsq;   // cells_total: sum |v'|^2 per occupied cell
  double* cell_amax;    // cells_total: max |a| per occupied cell
  double* chunk_part;   // chunks x 3: min ratio, sum |v'|^2, max |a|
  double* tile_part;    // tiles x 4: (sum |v|^2, max |a|^2) of the first and of the last run
  int32_t* mode;        // 1: which way the update runs (chosen on the device)
  KdkRec* rec;          // n_total: per-particle records of the gather way
  int64_t chunks;
  int64_t tiles;
};
hipError_t launch_kick_drift(const DevBox* boxes, int nboxes, int64_t n_total,
                             int64_t cells_total,
                             const KdkWork& w, const int32_t* cell_offsets, const int32_t* perm,
                             float* pos, float* vel, const float* acc, double* cell_stats,
                             double* box_stats, hipStream_t s);

// bin.hip
struct BinWork {
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

// One DPP move of a double (two 32-bit halves).  With every row enabled each
// lane reads its source lane; with a partial row mask the lanes of the other
// rows read 0.
template <int kCtrl, int kRowMask>
__device__ __forceinline__ double dpp_f64(double v) {
  const unsigned long long b = __builtin_bit_cast(unsigned long long, v);
  int lo, hi;
  if constexpr (kRowMask == 0xF) {
    lo = __builtin_amdgcn_mov_dpp((int)(unsigned)b, kCtrl, 0xF, 0xF, true);
    hi = __builtin_amdgcn_mov_dpp((int)(unsigned)(b >> 32), kCtrl, 0xF, 0xF, true);
  } else {
    lo = __builtin_amdgcn_update_dpp(0, (int)(unsigned)b, kCtrl, kRowMask, 0xF, false);
    hi = __builtin_amdgcn_update_dpp(0, (int)(unsigned)(b >> 32), kCtrl, kRowMask, 0xF, false);
  }
  return __builtin_bit_cast(double, ((unsigned long long)(unsigned)hi << 32) | (unsigned)lo);
}

// Task index for a wave of a persistent pair kernel.  The first n_static waves
// of the grid (those that are resident from the start) take their own grid
// index as their first task -- no atomic: every resident wave starts at once,
// and 8192 atomics on one counter would hand out the last first task tens of
// microseconds late.  Every other task comes from the shared counter, offset
// by n_static; a grid larger than the resident set (the autotuner's grid
// multiplier) thus leaves no task waiting for a late wave.  `first` is
// wave-uniform, and every lane takes part in the atomic (lane 0 adds 1, the
// others 0) so no divergent branch precedes the caller's wave-uniform exit test.
__device__ __forceinline__ int next_task(int32_t* head, bool& first, int n_static) {
  const int wave = (int)blockIdx.x * (int)(blockDim.x >> 6) + (int)(threadIdx.x >> 6);
  int t;
  if (first && wave < n_static) {
    t = wave;
  } else {
    t = atomicAdd(head, (threadIdx.x & 63) == 0 ? 1 : 0);
    t = __shfl(t, 0, 64) + n_static;
  }
  first = false;
  return __builtin_amdgcn_readfirstlane(t);
}

// Wave priority from the work left in the wave's current task (sources still
// to visit), so the SIMD's instruction arbiter favours the waves with the most
// work left instead of the oldest waves.  With age order alone the last waves
// dispatched to a SIMD barely advance while older ones run, and the heavy
// first items they took finish long after the queue is empty.  `left` must be
// wave-uniform.
__device__ __forceinline__ void set_wave_priority(int left) {
  if (left >= 8192)
    __builtin_amdgcn_s_setprio(3);
  else if (left >= 4096)
    __builtin_amdgcn_s_setprio(2);
  else if (left >= 2048)
    __builtin_amdgcn_s_setprio(1);
  else
    __builtin_amdgcn_s_setprio(0);
}

// plan.hip
struct PlanWork {
  int32_t* pencil_counts;  // pencils_total
  int32_t* item_base;      // pencils_total + 1 (item_base[pencils_total] = item count)
  int4* items;             // max_items
  int32_t* item_bucket;    // max_items: cost bucket of each item
  int32_t* item_slot;      // max_items: position of the item inside its bucket
  int32_t* item_cost;      // max_items: sources the item's wave visits (all x offsets)
  int32_t* tasks;          // max_tasks: item << kTaskShift | code, longest first
  int32_t* ctrl;           // kCtrlInts
  int32_t* scan_tmp;
  float* partial;          // split slices: [slot][slice][6][64] (sum and error per axis)
  int64_t max_items;
  int64_t max_tasks;
  int64_t max_split;       // capacity of partial in split items
  int64_t split_items;     // items to split in this launch (0: none)
};
int64_t plan_max_tasks(int64_t max_items, int64_t max_split);
int64_t plan_max_items(int64_t n_total, int64_t cells_total, int64_t pencils_total);
// w.split_items of the cheapest items are split into `slices` = 2R+1 x-offset
// tasks (every box must share R <= 3 when w.split_items > 0).
// status: the binning's status word; with ABACUS_NF_STATUS_CELLFULL set the
// task list is empty.
hipError_t launch_plan(const DevBox* boxes, int nboxes, int64_t pencils_total,
                       const int32_t* cell_offsets, const int32_t* status, int span, int slices,
                       const PlanWork& w, hipStream_t s);
// Combine the slices of split items into final outputs (adjoint: 1/w^3 scale;
// density: NULL or the density output of the forward kernel).
hipError_t launch_combine(AccMode mode, bool adjoint, const DevBox* boxes, const PlanWork& w,
                          const int32_t* perm, float* out, float* density, hipStream_t s);

// Tunable launch shape of a pair kernel (chosen by the autotuner in tune.hip).
struct KernelConfig {
  int unroll;     // sources per step of the inner loop (2, 4 or 8)
  int pipeline;   // 1: request the next step's sources before using the current ones
  int span;       // most cells one work item may span (1..3); a planner parameter
  int grid_mult;  // persistent workgroups per resident slot (1 or 2)
  int split;      // 1: split the cheapest tail items into x-offset slices
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
// src3: workspace for n_total packed (x, y, z) source records.
// pairs64.hip: the FP64 forward kernel (whole tasks only: plan it with no splits);
// src3: workspace for n_total (x, y, z) FP64 source records (the 24-byte region)
hipError_t launch_forward_f64(const DevBox* boxes, const PlanWork& w, const int32_t* off,
                              const float* rel, const int32_t* perm, double* acc, double* src3,
                              int64_t n_total, hipStream_t s);
// vjp64.hip: the FP64 adjoint (whole tasks only); w64 is workspace for n_total x 3
// FP64 cotangents in sorted order.
hipError_t launch_vjp_f64(const DevBox* boxes, const PlanWork& w, const int32_t* off,
                          const float* rel, const int32_t* perm, const double* wvec,
                          double* w64, int64_t n_total, double* grad, hipStream_t s);
hipError_t launch_forward(AccMode mode, bool count_pairs, const KernelConfig& cfg,
                          const DevBox* boxes, const PlanWork& w, int64_t pencils_total,
                          const int32_t* cell_offsets, const float* rel, const int32_t* perm,
                          float* acc, float* density, int64_t* pair_count, float* src3,
                          int64_t n_total, hipStream_t s);

// vjp.hip
// src6: workspace for n_total packed (x, y, z, w_x, w_y, w_z) source records.
hipError_t launch_vjp(AccMode mode, const KernelConfig& cfg, const DevBox* boxes,
                      const PlanWork& w, int64_t pencils_total, const int32_t* cell_offsets,
                      const float* rel, const int32_t* perm, const float* wvec, float* src6,
                      int64_t n_total, float* grad, hipStream_t s);

// reduce.hip
hipError_t launch_momentum(const DevBox* boxes, int nboxes, int64_t max_box_n, const float* acc,
                           double* partials, double* momentum, hipStream_t s);

// Occupancy-sized persistent grid for a kernel (cached per device and kernel).
int persistent_blocks(const void* kernel, int threads);
// Wavefronts the current device can hold at full occupancy (CUs x 32).
int resident_wave_capacity();

}  // namespace anf
