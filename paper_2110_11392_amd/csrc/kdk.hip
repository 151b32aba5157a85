// Leapfrog kick and drift with the time-step statistics of Eq. 1 (Sec. 3.1).
//
// What it computes, per particle (FP32 state; each update formed in FP64 with
// separate multiply and add, rounded once to FP32):
//   v' = v + kick a,   x' = wrap(x + drift v') into [0, L)
// and per cell of the binning (the positions before the drift): the sum of
// |v'|^2 and the maximum |a|; per box: min over cells of v_rms/a_max, the
// global v_rms and a_max, and N.  The velocity rms keeps the mean (the paper
// does not subtract it).
//
// How it maps to CDNA4: the step is HBM-bound (64 bytes per particle), so what
// matters is that every wave keeps many independent loads in flight.  The
// update runs one of two ways, chosen on the device from a sample of the
// permutation.  Particles kept in cell order (as the slabs of the paper's code
// keep them): the update is flat over the sorted slots, a block owning a tile
// of kKdkTile consecutive slots, each thread kKdkPer of them at a stride of
// the block size, with all of its gathers through the permutation (contiguous
// here) issued before any arithmetic.  Particles in any other order: a first
// pass updates them in their own order, with coalesced loads and stores, and
// leaves one 32-byte record per particle (cell, |v'|^2, |a|^2); the tile
// kernel then gathers one record per slot instead of three 12-byte state
// records from three random lines.  Small tiles keep the block's registers
// and LDS low, so that many blocks per CU have loads in flight while others
// reduce.  Cells are runs of consecutive
// slots; a slot's cell is recomputed from its position before the drift with
// the binning's own rule.  The per-cell statistics are a segmented reduction
// in a fixed order: inside the tile each run is summed by one wave (lanes
// strided over the run, then a fixed DPP tree), and a run cut by tile
// boundaries leaves its pieces' partials per tile, which the statistics pass
// adds in tile order afterwards.  No atomics, so every result is run-to-run
// identical, whichever way the update ran.  The per-box statistics
// are a two-level, fixed-order reduction over chunks of 512 cells.
#include "nf_internal.h"

namespace anf {

constexpr int kKdkThreads = 256;
constexpr int kKdkPer = kKdkTile / kKdkThreads;  // slots per thread

__device__ __forceinline__ int find_box_by_chunk(const DevBox* __restrict__ boxes, int nb,
                                                 int64_t k) {
  int lo = 0, hi = nb - 1;
  while (lo < hi) {
    int mid = (lo + hi + 1) >> 1;
    if (boxes[mid].chunk_base <= k) lo = mid; else hi = mid - 1;
  }
  return lo;
}

// Periodic wrap of an FP64 coordinate into [0, L), rounded to FP32 (a value
// that rounds up to L becomes 0).  Inside (0, L) the reduction below returns t
// itself (q is 0, or 1 when t / L rounds up, and then t - L + L is exact), so
// only coordinates that left the box take the division.
__device__ __forceinline__ float wrap_coord(double t, double L) {
  double r = t;
  if (!(t > 0.0 && t < L)) {
    const double q = floor(t / L);
    r = t - q * L;
    if (r < 0.0) r += L;
    if (r >= L) r -= L;
  }
  float f = (float)r;
  if (f >= (float)L) f = 0.0f;
  return f;
}

// Sum and maximum over the wave with DPP moves in a fixed pattern (quad
// permutes, half-row and row mirrors, then the row broadcasts into rows 1 and
// 3 and into rows 2 and 3); lane 63 ends with both totals.  Lanes of rows a
// broadcast does not write add 0, and 0 <= |a|^2 leaves the maximum.
__device__ __forceinline__ void wave_sum_max(double& s2, double& am2) {
  double o;
  o = dpp_f64<0xB1, 0xF>(s2); s2 += o; o = dpp_f64<0xB1, 0xF>(am2); am2 = o > am2 ? o : am2;
  o = dpp_f64<0x4E, 0xF>(s2); s2 += o; o = dpp_f64<0x4E, 0xF>(am2); am2 = o > am2 ? o : am2;
  o = dpp_f64<0x141, 0xF>(s2); s2 += o; o = dpp_f64<0x141, 0xF>(am2); am2 = o > am2 ? o : am2;
  o = dpp_f64<0x140, 0xF>(s2); s2 += o; o = dpp_f64<0x140, 0xF>(am2); am2 = o > am2 ? o : am2;
  o = dpp_f64<0x142, 0xA>(s2); s2 += o; o = dpp_f64<0x142, 0xA>(am2); am2 = o > am2 ? o : am2;
  o = dpp_f64<0x143, 0xC>(s2); s2 += o; o = dpp_f64<0x143, 0xC>(am2); am2 = o > am2 ? o : am2;
}

__device__ __forceinline__ void write_cell(int64_t c, int64_t n, double s2, double am2,
                                           double* __restrict__ cell_sumsq,
                                           double* __restrict__ cell_amax,
                                           double* __restrict__ cell_stats) {
  const double am = sqrt(am2);
  cell_sumsq[c] = s2;
  cell_amax[c] = am;
  if (cell_stats) {
    cell_stats[2 * c] = sqrt(s2 / (double)n);
    cell_stats[2 * c + 1] = am;
  }
}

// One particle: the kick, the drift and its wrap (stored in place), and what
// the statistics need of it: its cell in the binning (from the position before
// the drift), |v'|^2 and |a|^2 (the square root is monotonic, so a cell's max
// |a| is the root of its max |a|^2, taken once per cell).
__device__ __forceinline__ void update_one(const DevBox& B, int64_t i, float px, float py,
                                           float pz, float vx, float vy, float vz, float ax,
                                           float ay, float az, float* __restrict__ pos,
                                           float* __restrict__ vel, int& cell, double& v2,
                                           double& a2) {
  const double kick = B.kick, drift = B.drift, L = B.box_len, cpl = B.cells_per_len;
  const int K = B.K;
  const CellCoord cx = cell_coord(px, cpl, K), cy = cell_coord(py, cpl, K),
                  cz = cell_coord(pz, cpl, K);
  cell = B.cell_base + (cx.c * K + cy.c) * K + cz.c;
  const float nvx = (float)((double)vx + kick * (double)ax);
  const float nvy = (float)((double)vy + kick * (double)ay);
  const float nvz = (float)((double)vz + kick * (double)az);
  vel[3 * i] = nvx;
  vel[3 * i + 1] = nvy;
  vel[3 * i + 2] = nvz;
  pos[3 * i] = wrap_coord((double)px + drift * (double)nvx, L);
  pos[3 * i + 1] = wrap_coord((double)py + drift * (double)nvy, L);
  pos[3 * i + 2] = wrap_coord((double)pz + drift * (double)nvz, L);
  v2 = ((double)nvx * (double)nvx + (double)nvy * (double)nvy) + (double)nvz * (double)nvz;
  a2 = ((double)ax * (double)ax + (double)ay * (double)ay) + (double)az * (double)az;
}

// Which way the update runs, chosen on the device from the permutation: when
// most of kKdkThreads sampled neighbouring slots hold consecutive particles
// (particles kept in cell order), the tile kernel updates each slot's particle
// itself; else the particles are updated in their own order (coalesced) and
// each leaves a record that the tile kernel gathers through the permutation
// (one 32-byte record per slot instead of three 12-byte ones from three
// random lines).  Both ways give the same bits.  Every block of the update
// kernel takes the same samples and so the same decision; the tile kernel
// reads it from `mode`.
constexpr int kKdkSorted = 0, kKdkGather = 1;

__device__ __forceinline__ int kdk_way(const int32_t* __restrict__ perm, int64_t n_total) {
  const int64_t pairs = n_total > 1 ? n_total - 1 : 0;
  const int samples = pairs < kKdkThreads ? (int)pairs : kKdkThreads;
  const int64_t stride = samples > 0 ? pairs / samples : 0;  // k stride < pairs for k < samples
  const int64_t at = (int64_t)threadIdx.x * stride;
  const bool run = (int)threadIdx.x < samples && perm[at + 1] == perm[at] + 1;
  const int runs = __syncthreads_count(run);
  return 2 * runs >= samples ? kKdkSorted : kKdkGather;
}

// The gather way's update: particles in their own order, kKdkPer per thread
// at a stride of the block size, persistent blocks over chunks of kKdkTile.
__global__ __launch_bounds__(kKdkThreads) void k_kdk_update(
    const DevBox* __restrict__ boxes, int nboxes, int64_t n_total,
    const int32_t* __restrict__ perm, int32_t* __restrict__ mode, float* __restrict__ pos,
    float* __restrict__ vel, const float* __restrict__ acc, KdkRec* __restrict__ rec) {
  const int way = kdk_way(perm, n_total);
  if (blockIdx.x == 0 && threadIdx.x == 0) *mode = way;
  if (way != kKdkGather) return;
  __shared__ int s_box[2];
  const int t = threadIdx.x;
  const int64_t chunks = (n_total + kKdkTile - 1) / kKdkTile;
  for (int64_t ch = blockIdx.x; ch < chunks; ch += gridDim.x) {
    const int64_t c0 = ch * kKdkTile;
    const int len = n_total - c0 < kKdkTile ? (int)(n_total - c0) : kKdkTile;
    __syncthreads();  // the previous chunk's box range has been read
    if (t == 0) {
      s_box[0] = nboxes == 1 ? 0 : find_box_by_first(boxes, nboxes, c0);
      s_box[1] = nboxes == 1 ? 0 : find_box_by_first(boxes, nboxes, c0 + len - 1);
    }
    __syncthreads();
    const int box_lo = s_box[0], box_hi = s_box[1];
    float ax[kKdkPer], ay[kKdkPer], az[kKdkPer], vx[kKdkPer], vy[kKdkPer], vz[kKdkPer];
    float px[kKdkPer], py[kKdkPer], pz[kKdkPer];
#pragma unroll
    for (int k = 0; k < kKdkPer; ++k) {
      const int j = k * kKdkThreads + t;
      const int64_t i = c0 + (j < len ? j : 0);
      ax[k] = acc[3 * i]; ay[k] = acc[3 * i + 1]; az[k] = acc[3 * i + 2];
      vx[k] = vel[3 * i]; vy[k] = vel[3 * i + 1]; vz[k] = vel[3 * i + 2];
      px[k] = pos[3 * i]; py[k] = pos[3 * i + 1]; pz[k] = pos[3 * i + 2];
    }
#pragma unroll
    for (int k = 0; k < kKdkPer; ++k) {
      const int j = k * kKdkThreads + t;
      if (j >= len) continue;
      const int64_t i = c0 + j;
      const int b = box_lo == box_hi ? box_lo : find_box_by_first(boxes, nboxes, i);
      int cell;
      double v2, a2;
      update_one(boxes[b], i, px[k], py[k], pz[k], vx[k], vy[k], vz[k], ax[k], ay[k], az[k], pos,
                 vel, cell, v2, a2);
      KdkRec r;
      r.v2 = v2;
      r.a2 = a2;
      r.cell = cell;
      r.pad[0] = r.pad[1] = r.pad[2] = 0;
      rec[i] = r;
    }
  }
}

__global__ __launch_bounds__(kKdkThreads) void k_kick_drift(
    const DevBox* __restrict__ boxes, int nboxes, int64_t n_total,
    const int32_t* __restrict__ off, const int32_t* __restrict__ perm, float* __restrict__ pos,
    float* __restrict__ vel, const float* __restrict__ acc, double* __restrict__ cell_sumsq,
    double* __restrict__ cell_amax, double* __restrict__ cell_stats,
    double* __restrict__ tile_part, const int32_t* __restrict__ mode,
    const KdkRec* __restrict__ rec) {
  __shared__ double s_v2[kKdkTile], s_am[kKdkTile];
  __shared__ int s_cell[kKdkTile];
  __shared__ int s_run[kKdkTile + 1];
  __shared__ int s_edge[2];  // begin of the first slot's cell, end of the last slot's cell
  __shared__ int s_wave_runs[kKdkThreads / 64];
  __shared__ int s_box[2];
  const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
  const int64_t tile = blockIdx.x;
  const int64_t tile0 = tile * kKdkTile;
  const int len = n_total - tile0 < kKdkTile ? (int)(n_total - tile0) : kKdkTile;
  if (t == 0) {
    s_box[0] = nboxes == 1 ? 0 : find_box_by_first(boxes, nboxes, tile0);
    s_box[1] = nboxes == 1 ? 0 : find_box_by_first(boxes, nboxes, tile0 + len - 1);
  }
  __syncthreads();
  const int box_lo = s_box[0], box_hi = s_box[1];

  // ---- each slot's cell, |v'|^2 and |a|^2 -----------------------------------
  // Either the update of the slot's particle (every gather first, then the
  // arithmetic) or, when the particles were updated in their own order, the
  // record the particle left.
  int64_t idx[kKdkPer];
#pragma unroll
  for (int k = 0; k < kKdkPer; ++k) {
    const int j = k * kKdkThreads + t;
    idx[k] = j < len ? (int64_t)perm[tile0 + j] : 0;
  }
  int cell[kKdkPer];
  if (*mode == kKdkGather) {
    KdkRec r[kKdkPer];
#pragma unroll
    for (int k = 0; k < kKdkPer; ++k) r[k] = rec[idx[k]];
#pragma unroll
    for (int k = 0; k < kKdkPer; ++k) {
      const int j = k * kKdkThreads + t;
      cell[k] = r[k].cell;
      s_cell[j] = r[k].cell;
      s_v2[j] = r[k].v2;
      s_am[j] = r[k].a2;
    }
  } else {
    float ax[kKdkPer], ay[kKdkPer], az[kKdkPer], vx[kKdkPer], vy[kKdkPer], vz[kKdkPer];
    float px[kKdkPer], py[kKdkPer], pz[kKdkPer];
#pragma unroll
    for (int k = 0; k < kKdkPer; ++k) {
      const int64_t i = idx[k];
      ax[k] = acc[3 * i]; ay[k] = acc[3 * i + 1]; az[k] = acc[3 * i + 2];
      vx[k] = vel[3 * i]; vy[k] = vel[3 * i + 1]; vz[k] = vel[3 * i + 2];
      px[k] = pos[3 * i]; py[k] = pos[3 * i + 1]; pz[k] = pos[3 * i + 2];
    }
#pragma unroll
    for (int k = 0; k < kKdkPer; ++k) {
      const int j = k * kKdkThreads + t;
      cell[k] = 0;
      if (j >= len) continue;
      const int b = box_lo == box_hi ? box_lo : find_box_by_first(boxes, nboxes, tile0 + j);
      double v2, a2;
      update_one(boxes[b], idx[k], px[k], py[k], pz[k], vx[k], vy[k], vz[k], ax[k], ay[k], az[k],
                 pos, vel, cell[k], v2, a2);
      s_cell[j] = cell[k];
      s_v2[j] = v2;
      s_am[j] = a2;
    }
  }
  // Only the tile's first and last runs can belong to cells that continue
  // past the tile: the begin of the first slot's cell and the end of the last
  // slot's cell tell.
#pragma unroll
  for (int k = 0; k < kKdkPer; ++k) {
    const int j = k * kKdkThreads + t;
    if (j == 0) s_edge[0] = off[cell[k]];
    if (j == len - 1) s_edge[1] = off[cell[k] + 1];
  }
  __syncthreads();

  // ---- runs of equal cells: their starts, compacted in slot order ----------
  // Thread t owns slots [kKdkPer t, kKdkPer t + kKdkPer) of the tile here.
  const int j0 = kKdkPer * t;
  int starts = 0;
#pragma unroll
  for (int k = 0; k < kKdkPer; ++k) {
    const int j = j0 + k;
    starts += (j < len && (j == 0 || s_cell[j] != s_cell[j - 1])) ? 1 : 0;
  }
  int incl = starts;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const int o = __shfl_up(incl, d, 64);
    if (lane >= d) incl += o;
  }
  if (lane == 63) s_wave_runs[wv] = incl;
  __syncthreads();
  int base = 0, nruns = 0;
#pragma unroll
  for (int w = 0; w < kKdkThreads / 64; ++w) {
    base += w < wv ? s_wave_runs[w] : 0;
    nruns += s_wave_runs[w];
  }
  int at = base + incl - starts;
#pragma unroll
  for (int k = 0; k < kKdkPer; ++k) {
    const int j = j0 + k;
    if (j < len && (j == 0 || s_cell[j] != s_cell[j - 1])) s_run[at++] = j;
  }
  if (t == 0) s_run[nruns] = len;
  __syncthreads();
  // ---- each run summed by one wave; whole cells written, cut ones kept ----
  for (int r = wv; r < nruns; r += kKdkThreads / 64) {
    const int rb = s_run[r], re = s_run[r + 1];
    double s2 = 0.0, am2 = 0.0;
    for (int j = rb + lane; j < re; j += 64) {
      s2 += s_v2[j];
      am2 = s_am[j] > am2 ? s_am[j] : am2;
    }
    wave_sum_max(s2, am2);
    if (lane == 63) {
      // a run between two others is a whole cell of re - rb particles
      const bool head = r == 0 && s_edge[0] < tile0;
      const bool tail = r == nruns - 1 && s_edge[1] > tile0 + len;
      if (!head && !tail) write_cell(s_cell[rb], re - rb, s2, am2, cell_sumsq, cell_amax, cell_stats);
      if (head) {
        tile_part[4 * tile] = s2;
        tile_part[4 * tile + 1] = am2;
      }
      if (tail) {
        tile_part[4 * tile + 2] = s2;
        tile_part[4 * tile + 3] = am2;
      }
    }
  }
}

// Stage 1: chunk k of a box -> (min over its cells of v_rms/a_max, sum |v'|^2,
// max |a|), reduced across the block in a fixed tree order.  Empty cells count
// as zero and get their zero statistics here.  A cell that spans tiles of the
// update is finished here: its piece in its first tile (that tile's last run),
// then its pieces in the following tiles (their first runs), in tile order.
__global__ __launch_bounds__(256) void k_kdk_chunks(const DevBox* __restrict__ boxes, int nboxes,
                                                    const int32_t* __restrict__ off,
                                                    const double* __restrict__ cell_sumsq,
                                                    const double* __restrict__ cell_amax,
                                                    const double* __restrict__ tile_part,
                                                    double* __restrict__ cell_stats,
                                                    double* __restrict__ part) {
  __shared__ double s_min[256], s_sum[256], s_max[256];
  const int64_t k = blockIdx.x;
  const int b = nboxes == 1 ? 0 : find_box_by_chunk(boxes, nboxes, k);
  const int64_t K = boxes[b].K;
  const int64_t first = boxes[b].cell_base + (k - boxes[b].chunk_base) * (int64_t)kKdkChunk;
  const int64_t box_end = boxes[b].cell_base + K * K * K;
  const int64_t last = first + kKdkChunk < box_end ? first + kKdkChunk : box_end;
  double mn = __builtin_inf(), sm = 0.0, mx = 0.0;
  for (int64_t c = first + threadIdx.x; c < last; c += blockDim.x) {
    const int64_t cb = off[c], ce = off[c + 1];
    const int n = (int)(ce - cb);
    double s2 = 0.0, am = 0.0;
    if (n > 0) {
      const int64_t tb = cb / kKdkTile, te = (ce - 1) / kKdkTile;
      if (tb == te) {  // written by the update
        s2 = cell_sumsq[c];
        am = cell_amax[c];
      } else {
        s2 = tile_part[4 * tb + 2];
        double am2 = tile_part[4 * tb + 3];
        for (int64_t u = tb + 1; u <= te; ++u) {
          s2 += tile_part[4 * u];
          const double m = tile_part[4 * u + 1];
          am2 = m > am2 ? m : am2;
        }
        am = sqrt(am2);
        if (cell_stats) {
          cell_stats[2 * c] = sqrt(s2 / (double)n);
          cell_stats[2 * c + 1] = am;
        }
      }
    } else if (cell_stats) {
      cell_stats[2 * c] = 0.0;
      cell_stats[2 * c + 1] = 0.0;
    }
    sm += s2;
    mx = am > mx ? am : mx;
    if (n > 0 && am > 0.0) {
      const double r = sqrt(s2 / (double)n) / am;
      mn = r < mn ? r : mn;
    }
  }
  s_min[threadIdx.x] = mn;
  s_sum[threadIdx.x] = sm;
  s_max[threadIdx.x] = mx;
  __syncthreads();
  for (int h = 128; h >= 1; h >>= 1) {
    if ((int)threadIdx.x < h) {
      const int o = threadIdx.x + h;
      s_min[threadIdx.x] = s_min[o] < s_min[threadIdx.x] ? s_min[o] : s_min[threadIdx.x];
      s_sum[threadIdx.x] += s_sum[o];
      s_max[threadIdx.x] = s_max[o] > s_max[threadIdx.x] ? s_max[o] : s_max[threadIdx.x];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    part[3 * k] = s_min[0];
    part[3 * k + 1] = s_sum[0];
    part[3 * k + 2] = s_max[0];
  }
}

// Stage 2: one block per box folds its chunks, strided over the threads and
// then through a fixed tree.
__global__ __launch_bounds__(256) void k_kdk_boxes(const DevBox* __restrict__ boxes,
                                                   const double* __restrict__ part,
                                                   double* __restrict__ box_stats) {
  __shared__ double s_min[256], s_sum[256], s_max[256];
  const int b = blockIdx.x;
  const int64_t K = boxes[b].K;
  const int64_t nchunks = (K * K * K + kKdkChunk - 1) / kKdkChunk;
  double mn = __builtin_inf(), sm = 0.0, mx = 0.0;
  for (int64_t j = threadIdx.x; j < nchunks; j += blockDim.x) {
    const double* p = part + 3 * (boxes[b].chunk_base + j);
    mn = p[0] < mn ? p[0] : mn;
    sm += p[1];
    mx = p[2] > mx ? p[2] : mx;
  }
  s_min[threadIdx.x] = mn;
  s_sum[threadIdx.x] = sm;
  s_max[threadIdx.x] = mx;
  __syncthreads();
  for (int h = 128; h >= 1; h >>= 1) {
    if ((int)threadIdx.x < h) {
      const int o = threadIdx.x + h;
      s_min[threadIdx.x] = s_min[o] < s_min[threadIdx.x] ? s_min[o] : s_min[threadIdx.x];
      s_sum[threadIdx.x] += s_sum[o];
      s_max[threadIdx.x] = s_max[o] > s_max[threadIdx.x] ? s_max[o] : s_max[threadIdx.x];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const int64_t n = boxes[b].n;
    box_stats[4 * b] = s_min[0];
    box_stats[4 * b + 1] = n > 0 ? sqrt(s_sum[0] / (double)n) : 0.0;
    box_stats[4 * b + 2] = s_max[0];
    box_stats[4 * b + 3] = (double)n;
  }
}

hipError_t launch_kick_drift(const DevBox* boxes, int nboxes, int64_t n_total,
                             int64_t cells_total, const KdkWork& w, const int32_t* off,
                             const int32_t* perm, float* pos, float* vel, const float* acc,
                             double* cell_stats, double* box_stats, hipStream_t s) {
  hipError_t e;
  if (w.tiles > 0) {
    // the update kernel also decides the way (and idles, cheaply, in cell order)
    const int upd_blocks =
        persistent_blocks(reinterpret_cast<const void*>(&k_kdk_update), kKdkThreads) / 2;
    const int64_t ub = w.tiles < upd_blocks ? w.tiles : upd_blocks;
    hipLaunchKernelGGL(k_kdk_update, dim3((unsigned)(ub > 0 ? ub : 1)), dim3(kKdkThreads), 0, s,
                       boxes, nboxes, n_total, perm, w.mode, pos, vel, acc, w.rec);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(k_kick_drift, dim3((unsigned)w.tiles), dim3(kKdkThreads), 0, s, boxes,
                       nboxes, n_total, off, perm, pos, vel, acc, w.cell_sumsq, w.cell_amax,
                       cell_stats, w.tile_part, w.mode, w.rec);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  if (!cell_stats && !box_stats) return hipSuccess;
  hipLaunchKernelGGL(k_kdk_chunks, dim3((unsigned)w.chunks), dim3(256), 0, s, boxes, nboxes, off,
                     w.cell_sumsq, w.cell_amax, w.tile_part, cell_stats, w.chunk_part);
  if ((e = hipGetLastError()) != hipSuccess || !box_stats) return e;
  hipLaunchKernelGGL(k_kdk_boxes, dim3((unsigned)nboxes), dim3(256), 0, s, boxes, w.chunk_part,
                     box_stats);
  return hipGetLastError();
}

}  // namespace anf
