// Work plan for the pair kernels: which sinks each wavefront work item owns,
// and the order in which a persistent grid takes the items.
//
// An item is up to 64 consecutive sinks (one per lane) of one pencil -- an
// (x, y) column of cells along z, the sink-pencil direction of Sec. 3.4.2.  All
// sinks of a pencil are contiguous in the cell-sorted arrays, so each pencil's
// sink sequence is simply cut into chunks of 64 that span at most `span`
// cells (default 2, tunable 1..3).  Every sink of an item shares the item's (2R+1)^2 source columns; a
// chunk spanning two cells costs one extra z-layer of source cells but keeps
// all 64 lanes busy where cells hold fewer than 64 particles.
//
// Items are queued longest first (bucketed by quarter octaves of cost, cost = number
// of sources the wave visits) so the persistent grid drains evenly; the
// cheapest items at the end are split into one task per x offset so the last
// tasks are short and the grid's tail shrinks.
#include "nf_internal.h"

namespace anf {

// item = {box | count << 16, cx | cy << 16, za | zb << 16, first sink}.
// The walk reads the pencil's K + 1 cell offsets from `po` (LDS): po[z] is the
// first sorted slot of cell z of the pencil, po[K] one past its last.
template <bool kEmit>
__device__ int walk_pencil(const int32_t* po, int K, int b, int cx, int cy, int span,
                           int4* __restrict__ out) {
  int nitems = 0;
  int i = po[0];
  const int end = po[K];
  int z = 0;
  while (i < end) {
    while (po[z + 1] <= i) ++z;  // cell of sink i (skips empty cells)
    const int za = z;
    const int span_end = po[za + span < K ? za + span : K];
    int stop = i + kTile;
    stop = stop < span_end ? stop : span_end;
    int zb = za;
    while (po[zb + 1] < stop) ++zb;  // cell of sink stop-1
    if (kEmit) out[nitems] = make_int4(b | ((stop - i) << 16), cx | (cy << 16), za | (zb << 16), i);
    ++nitems;
    i = stop;
  }
  return nitems;
}

// One wave per pencil: the lanes copy the pencil's offsets into LDS with
// coalesced loads, then lane 0 walks it (a chain of LDS reads instead of a
// chain of dependent global loads).
template <bool kEmit>
__device__ void plan_pencil(const DevBox* __restrict__ boxes, int nboxes, int64_t p,
                            const int32_t* __restrict__ off, int span, int32_t* __restrict__ counts,
                            const int32_t* __restrict__ base, int4* __restrict__ items) {
  __shared__ int32_t po[kMaxCellsPerDim + 1];
  const int b = nboxes == 1 ? 0 : find_box_by_pencil(boxes, nboxes, (int)p);
  const int K = boxes[b].K;
  const int local = (int)p - boxes[b].pencil_base;
  const int cx = local / K, cy = local - (local / K) * K;
  if (cx < boxes[b].sink_x0 || cx >= boxes[b].sink_x1) {  // outside the sink slabs: no items
    if (!kEmit && threadIdx.x == 0) counts[p] = 0;
    return;
  }
  const int cell0 = boxes[b].cell_base + local * K;
  for (int z = threadIdx.x; z <= K; z += blockDim.x) po[z] = off[cell0 + z];
  __syncthreads();
  if (threadIdx.x == 0) {
    if (kEmit)
      walk_pencil<true>(po, K, b, cx, cy, span, items + base[p]);
    else
      counts[p] = walk_pencil<false>(po, K, b, cx, cy, span, nullptr);
  }
}

__global__ __launch_bounds__(64) void k_plan_count(const DevBox* __restrict__ boxes, int nboxes,
                                                   int64_t pencils, const int32_t* __restrict__ off,
                                                   int span, int32_t* __restrict__ counts) {
  plan_pencil<false>(boxes, nboxes, blockIdx.x, off, span, counts, nullptr, nullptr);
}

__global__ __launch_bounds__(64) void k_plan_emit(const DevBox* __restrict__ boxes, int nboxes,
                                                  int64_t pencils, const int32_t* __restrict__ off,
                                                  int span, const int32_t* __restrict__ base,
                                                  int4* __restrict__ items) {
  plan_pencil<true>(boxes, nboxes, blockIdx.x, off, span, nullptr, base, items);
}

// Sources in cells z = lo..hi (unwrapped, periodic) of one column.
__device__ __forceinline__ int64_t column_range_count(const int32_t* __restrict__ off, int col,
                                                      int K, int lo, int hi) {
  int64_t total = 0;
  while (lo <= hi) {
    int zl = lo % K;
    zl += zl < 0 ? K : 0;
    int len = hi - lo + 1;
    len = len < K - zl ? len : K - zl;
    total += off[col + zl + len] - off[col + zl];
    lo += len;
  }
  return total;
}

// Cost of an item = source visits of its wave: the sources in the (2R+1)^2
// columns over z in [za-R, zb+R], with a two-cell item's paired far edge
// cells counted once at the longer one's length.
__global__ __launch_bounds__(256) void k_item_cost(const DevBox* __restrict__ boxes,
                                                   const int4* __restrict__ items,
                                                   const int32_t* __restrict__ n_items_ptr,
                                                   const int32_t* __restrict__ off,
                                                   int32_t* __restrict__ bucket_of,
                                                   int32_t* __restrict__ slot_of,
                                                   int32_t* __restrict__ cost_of,
                                                   int32_t* __restrict__ bucket_count) {
  __shared__ int local[kBuckets];
  __shared__ int base[kBuckets];
  if (threadIdx.x < kBuckets) local[threadIdx.x] = 0;
  __syncthreads();
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  const bool valid = q < *n_items_ptr;
  int bucket = 0, rank = 0;
  if (valid) {
    const int4 it = items[q];
    const DevBox& B = boxes[it.x & 0xffff];
    const int K = B.K, R = B.R;
    const int cx = it.y & 0xffff, cy = it.y >> 16, za = it.z & 0xffff, zb = it.z >> 16;
    // two-cell items walk their far edge cells together: the longer one counts
    const bool paired = zb == za + 1 && R >= 2 && B.far_mode != kFarNone;
    int64_t cost = 0;
    for (int ox = -R; ox <= R; ++ox) {
      int x = cx + ox;
      x += x < 0 ? K : 0;
      x -= x >= K ? K : 0;
      for (int oy = -R; oy <= R; ++oy) {
        int y = cy + oy;
        y += y < 0 ? K : 0;
        y -= y >= K ? K : 0;
        const int col = B.cell_base + (x * K + y) * K;
        cost += column_range_count(off, col, K, za - R, zb + R);
        if (paired) {  // the shorter edge run costs nothing extra
          int zl = za - R, zh = zb + R;
          zl += zl < 0 ? K : 0;
          zh -= zh >= K ? K : 0;
          const int lo = off[col + zl + 1] - off[col + zl];
          const int hi = off[col + zh + 1] - off[col + zh];
          cost -= lo < hi ? lo : hi;
        }
      }
    }
    const int lg = cost > 0 ? 63 - __clzll((unsigned long long)cost) : 0;
    cost_of[q] = cost < 0x7fffffff ? (int32_t)cost : 0x7fffffff;
    const int quarter = lg >= 2 ? (int)((cost >> (lg - 2)) & 3) : 0;
    const int key = 4 * lg + quarter;  // costs reach 25 * 2^31 at most: clamp to the last bucket
    bucket = kBuckets - 1 - (key < kBuckets - 1 ? key : kBuckets - 1);
    rank = atomicAdd(&local[bucket], 1);  // LDS atomic: cheap, order irrelevant
  }
  __syncthreads();
  // one global atomic per (block, non-empty bucket) reserves a run of slots
  if (threadIdx.x < kBuckets) {
    const int c = local[threadIdx.x];
    base[threadIdx.x] = c ? atomicAdd(&bucket_count[threadIdx.x], c) : 0;
  }
  __syncthreads();
  if (valid) {
    bucket_of[q] = bucket;
    slot_of[q] = base[bucket] + rank;
  }
}

// Bucket bases (longest first) and the task-list layout: the cheapest
// split_items items of the queue are split into `slices` x-offset tasks each.
// A binning that found a cell beyond kMaxCellParticles leaves no task at all.
__global__ void k_bucket_scan(int32_t* __restrict__ ctrl, const int32_t* __restrict__ n_items_ptr,
                              const int32_t* __restrict__ status, int split_items, int slices) {
  if (threadIdx.x != 0) return;
  int run = 0;
  for (int k = 0; k < kBuckets; ++k) {
    ctrl[kBuckets + k] = run;
    run += ctrl[k];
  }
  const int n_items = (*status & ABACUS_NF_STATUS_CELLFULL) ? 0 : *n_items_ptr;
  int split = slices >= 2 ? split_items : 0;
  split = split < n_items / 2 ? split : n_items / 2;
  ctrl[kCtrlHead] = 0;
  ctrl[kCtrlNWhole] = n_items - split;
  ctrl[kCtrlNSplit] = split;
  ctrl[kCtrlSlices] = split > 0 ? slices : 1;
  ctrl[kCtrlNTasks] = n_items - split + split * (split > 0 ? slices : 1);
}

// Item q goes to queue position bases[bucket] + slot; whole items keep their
// position as a task, split items fan out to one task per slice (slice-major,
// so the slices of one item are spread over the end of the list).
__global__ __launch_bounds__(256) void k_task_scatter(const int32_t* __restrict__ n_items_ptr,
                                                      const int32_t* __restrict__ bucket_of,
                                                      const int32_t* __restrict__ slot_of,
                                                      const int32_t* __restrict__ ctrl,
                                                      int32_t* __restrict__ tasks) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= *n_items_ptr) return;
  const int pos = ctrl[kBuckets + bucket_of[q]] + slot_of[q];
  const int n_whole = ctrl[kCtrlNWhole];
  if (pos < n_whole) {
    tasks[pos] = q << kTaskShift;
    return;
  }
  const int split = ctrl[kCtrlNSplit], slices = ctrl[kCtrlSlices];
  const int slot = pos - n_whole;
  for (int c = 1; c <= slices; ++c) tasks[n_whole + (c - 1) * split + slot] = (q << kTaskShift) | c;
}

// Final outputs of split items: fold the slices in x-offset order with the
// same slice_fold the pair kernels use for whole items.
template <int kAcc>
__global__ __launch_bounds__(64) void k_combine_slices(const DevBox* __restrict__ boxes,
                                                       const int4* __restrict__ items,
                                                       const int32_t* __restrict__ tasks,
                                                       const int32_t* __restrict__ ctrl,
                                                       const int32_t* __restrict__ perm,
                                                       const float* __restrict__ partial,
                                                       int adjoint, float* __restrict__ out,
                                                       float* __restrict__ density) {
  const int slot = blockIdx.x;
  const int split = ctrl[kCtrlNSplit];
  if (slot >= split) return;
  const int slices = ctrl[kCtrlSlices];
  const int task = tasks[ctrl[kCtrlNWhole] + slot];
  const int4 it = items[task >> kTaskShift];
  const int lane = threadIdx.x;
  const int count = it.x >> 16;
  if (lane >= count) return;
  const DevBox& B = boxes[it.x & 0xffff];
  float A[3] = {0.f, 0.f, 0.f}, E[3] = {0.f, 0.f, 0.f}, rho = 0.f;
  for (int c = 0; c < slices; ++c) {
    const float* src = partial + (int64_t)(slot * slices + c) * kPartialStride * kTile + lane;
    for (int k = 0; k < 3; ++k) slice_fold<kAcc>(A[k], E[k], src[k * kTile], src[(3 + k) * kTile]);
    rho += src[6 * kTile];
  }
  const float scale = adjoint ? B.inv_w3 : B.inv_w2;
  const int64_t i = perm[it.w + lane];
  for (int k = 0; k < 3; ++k) out[3 * i + k] = (A[k] + E[k]) * scale;
  if (density) density[i] = rho * B.inv_b2;
}

hipError_t launch_combine(AccMode mode, bool adjoint, const DevBox* boxes, const PlanWork& w,
                          const int32_t* perm, float* out, float* density, hipStream_t s) {
  if (w.split_items <= 0 || mode == kAccSingle) return hipSuccess;
  const dim3 grid((unsigned)w.split_items);
  if (mode == kAccChunked)
    hipLaunchKernelGGL(k_combine_slices<kAccChunked>, grid, dim3(kTile), 0, s, boxes, w.items,
                       w.tasks, w.ctrl, perm, w.partial, adjoint ? 1 : 0, out, density);
  else
    hipLaunchKernelGGL(k_combine_slices<kAccCompensated>, grid, dim3(kTile), 0, s, boxes, w.items,
                       w.tasks, w.ctrl, perm, w.partial, adjoint ? 1 : 0, out, density);
  return hipGetLastError();
}

int64_t plan_max_tasks(int64_t max_items, int64_t max_split) {
  return max_items + max_split * (kMaxSlices - 1);
}

int64_t plan_max_items(int64_t n_total, int64_t cells_total, int64_t pencils_total) {
  // In a pencil of m sinks and K cells an item ends after 64 sinks, at the end
  // of its span (the next item then starts at least one cell further on), or at
  // the pencil's end: at most m/64 + K + 1 items for any span >= 1.
  return n_total / kTile + cells_total + 2 * pencils_total + 1;
}

#define ANF_TRY(x)                      \
  do {                                  \
    hipError_t e_ = (x);                \
    if (e_ != hipSuccess) return e_;    \
  } while (0)

hipError_t launch_plan(const DevBox* boxes, int nboxes, int64_t pencils, const int32_t* off,
                       const int32_t* status, int span, int slices, const PlanWork& w,
                       hipStream_t s) {
  span = span < 1 ? 1 : (span > kMaxSpan ? kMaxSpan : span);
  const unsigned gp = (unsigned)pencils;  // one wave per pencil
  hipLaunchKernelGGL(k_plan_count, dim3(gp), dim3(64), 0, s, boxes, nboxes, pencils, off, span,
                     w.pencil_counts);
  ANF_TRY(hipGetLastError());
  ANF_TRY(exclusive_scan(w.pencil_counts, w.item_base, pencils, w.scan_tmp, s));
  hipLaunchKernelGGL(k_plan_emit, dim3(gp), dim3(64), 0, s, boxes, nboxes, pencils, off, span,
                     w.item_base, w.items);
  ANF_TRY(hipGetLastError());
  ANF_TRY(fill_i32(w.ctrl, 0, kBuckets, s));
  const int32_t* n_items = w.item_base + pencils;
  const unsigned gi = (unsigned)((w.max_items + 255) / 256);
  hipLaunchKernelGGL(k_item_cost, dim3(gi), dim3(256), 0, s, boxes, w.items, n_items, off,
                     w.item_bucket, w.item_slot, w.item_cost, w.ctrl);
  ANF_TRY(hipGetLastError());
  const int split = (int)(w.split_items < w.max_split ? w.split_items : w.max_split);
  hipLaunchKernelGGL(k_bucket_scan, dim3(1), dim3(64), 0, s, w.ctrl, n_items, status,
                     slices >= 2 && slices <= kMaxSlices ? split : 0, slices);
  ANF_TRY(hipGetLastError());
  hipLaunchKernelGGL(k_task_scatter, dim3(gi), dim3(256), 0, s, n_items, w.item_bucket,
                     w.item_slot, w.ctrl, w.tasks);
  return hipGetLastError();
}

}  // namespace anf
