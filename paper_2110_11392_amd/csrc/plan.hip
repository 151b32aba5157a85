// Work plan for the pair kernels: which sinks each wavefront work item owns,
// and the order in which a persistent grid takes the items.
//
// An item is 64 sinks (one per lane).  Each pencil (an (x, y) column of cells
// along z, the sink-pencil direction of Sec. 3.4.2) is walked in z: every full
// tile of 64 sinks of a cell becomes a FULL item; the partial tile left in each
// cell is packed with the partial tiles of the next few cells along z into a
// PACKED item while they fit in 64 lanes.  All sinks of an item share the
// source columns of their pencil, so a packed item sums one extra z-layer of
// source cells per extra cell instead of leaving lanes idle.
//
// Items are queued longest first (bucketed by floor(log2 cost), cost = number
// of sources the wave visits) so the persistent grid drains evenly.
#include "nf_internal.h"

namespace anf {

// item = {box, cx | cy << 16, za | zb << 16, tile}; tile >= 0: FULL tile of cell
// (cx, cy, za); tile < 0: PACKED partial tiles of cells za..zb.
template <bool kEmit>
__device__ int walk_pencil(const int32_t* __restrict__ off, int cell0, int K, int b, int cx, int cy,
                           int4* __restrict__ out) {
  int nitems = 0;
  int open_z0 = -1, open_z1 = -1, open_sinks = 0;
  for (int z = 0; z < K; ++z) {
    const int m = off[cell0 + z + 1] - off[cell0 + z];
    const int full = m / kTile;
    const int rem = m - full * kTile;
    for (int t = 0; t < full; ++t) {
      if (kEmit) out[nitems] = make_int4(b, cx | (cy << 16), z | (z << 16), t);
      ++nitems;
    }
    if (rem == 0) continue;
    if (open_z0 >= 0 && open_sinks + rem <= kTile && z - open_z0 + 1 <= kMaxPack) {
      open_z1 = z;
      open_sinks += rem;
    } else {
      if (open_z0 >= 0) {
        if (kEmit) out[nitems] = make_int4(b, cx | (cy << 16), open_z0 | (open_z1 << 16), -1);
        ++nitems;
      }
      open_z0 = open_z1 = z;
      open_sinks = rem;
    }
  }
  if (open_z0 >= 0) {
    if (kEmit) out[nitems] = make_int4(b, cx | (cy << 16), open_z0 | (open_z1 << 16), -1);
    ++nitems;
  }
  return nitems;
}

__global__ __launch_bounds__(64) void k_plan_count(const DevBox* __restrict__ boxes, int nboxes,
                                                   int64_t pencils, const int32_t* __restrict__ off,
                                                   int32_t* __restrict__ counts) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= pencils) return;
  const int b = nboxes == 1 ? 0 : find_box_by_pencil(boxes, nboxes, (int)p);
  const int K = boxes[b].K;
  const int local = (int)p - boxes[b].pencil_base;
  const int cx = local / K, cy = local - (local / K) * K;
  const int cell0 = boxes[b].cell_base + local * K;
  counts[p] = walk_pencil<false>(off, cell0, K, b, cx, cy, nullptr);
}

__global__ __launch_bounds__(64) void k_plan_emit(const DevBox* __restrict__ boxes, int nboxes,
                                                  int64_t pencils, const int32_t* __restrict__ off,
                                                  const int32_t* __restrict__ base,
                                                  int4* __restrict__ items) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= pencils) return;
  const int b = nboxes == 1 ? 0 : find_box_by_pencil(boxes, nboxes, (int)p);
  const int K = boxes[b].K;
  const int local = (int)p - boxes[b].pencil_base;
  const int cx = local / K, cy = local - (local / K) * K;
  const int cell0 = boxes[b].cell_base + local * K;
  walk_pencil<true>(off, cell0, K, b, cx, cy, items + base[p]);
}

// Cost of an item = sources in the (2R+1)^2 columns over z in [za-R, zb+R].
__global__ __launch_bounds__(256) void k_item_cost(const DevBox* __restrict__ boxes,
                                                   const int4* __restrict__ items,
                                                   const int32_t* __restrict__ n_items_ptr,
                                                   const int32_t* __restrict__ off,
                                                   int32_t* __restrict__ bucket_of,
                                                   int32_t* __restrict__ bucket_count) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= *n_items_ptr) return;
  const int4 it = items[q];
  const DevBox& B = boxes[it.x];
  const int K = B.K, R = B.R;
  const int cx = it.y & 0xffff, cy = it.y >> 16, za = it.z & 0xffff, zb = it.z >> 16;
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
      for (int zu = za - R; zu <= zb + R; ++zu) {
        int z = zu;
        z += z < 0 ? K : 0;
        z -= z >= K ? K : 0;
        cost += off[col + z + 1] - off[col + z];
      }
    }
  }
  const int lg = cost > 0 ? 63 - __clzll((unsigned long long)cost) : 0;
  const int bucket = kBuckets - 1 - lg;
  bucket_of[q] = bucket;
  atomicAdd(&bucket_count[bucket], 1);
}

// ctrl layout: [0, B) counts, [B, 2B) bases, [2B, 3B) cursors, [3B] queue head.
__global__ void k_bucket_scan(int32_t* __restrict__ ctrl) {
  if (threadIdx.x != 0) return;
  int run = 0;
  for (int k = 0; k < kBuckets; ++k) {
    ctrl[kBuckets + k] = run;
    run += ctrl[k];
    ctrl[2 * kBuckets + k] = 0;
  }
  ctrl[3 * kBuckets] = 0;
}

__global__ __launch_bounds__(256) void k_bucket_scatter(const int32_t* __restrict__ n_items_ptr,
                                                        const int32_t* __restrict__ bucket_of,
                                                        int32_t* __restrict__ ctrl,
                                                        int32_t* __restrict__ queue) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= *n_items_ptr) return;
  const int bk = bucket_of[q];
  const int pos = ctrl[kBuckets + bk] + atomicAdd(&ctrl[2 * kBuckets + bk], 1);
  queue[pos] = q;
}

int64_t plan_max_items(int64_t n_total, int64_t cells_total) {
  // FULL items <= n/64; PACKED items hold >= 1 sink and <= 1 per non-empty cell.
  const int64_t packed = n_total < cells_total ? n_total : cells_total;
  return n_total / kTile + packed + 1;
}

#define ANF_TRY(x)                      \
  do {                                  \
    hipError_t e_ = (x);                \
    if (e_ != hipSuccess) return e_;    \
  } while (0)

hipError_t launch_plan(const DevBox* boxes, int nboxes, int64_t pencils, const int32_t* off,
                       const PlanWork& w, hipStream_t s) {
  const unsigned gp = (unsigned)((pencils + 63) / 64);
  hipLaunchKernelGGL(k_plan_count, dim3(gp), dim3(64), 0, s, boxes, nboxes, pencils, off,
                     w.pencil_counts);
  ANF_TRY(hipGetLastError());
  ANF_TRY(exclusive_scan(w.pencil_counts, w.item_base, pencils, w.scan_tmp, s));
  hipLaunchKernelGGL(k_plan_emit, dim3(gp), dim3(64), 0, s, boxes, nboxes, pencils, off,
                     w.item_base, w.items);
  ANF_TRY(hipGetLastError());
  ANF_TRY(fill_i32(w.ctrl, 0, kBuckets, s));
  const int32_t* n_items = w.item_base + pencils;
  const unsigned gi = (unsigned)((w.max_items + 255) / 256);
  hipLaunchKernelGGL(k_item_cost, dim3(gi), dim3(256), 0, s, boxes, w.items, n_items, off,
                     w.item_bucket, w.ctrl);
  ANF_TRY(hipGetLastError());
  hipLaunchKernelGGL(k_bucket_scan, dim3(1), dim3(64), 0, s, w.ctrl);
  ANF_TRY(hipGetLastError());
  hipLaunchKernelGGL(k_bucket_scatter, dim3(gi), dim3(256), 0, s, n_items, w.item_bucket, w.ctrl,
                     w.queue);
  return hipGetLastError();
}

}  // namespace anf
