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
// How it maps to CDNA4: the step is HBM-bound (about 64 bytes per particle),
// so the layout of the traffic is what matters.  One wave per cell (a
// persistent loop over cells): lanes stride over the cell's sorted slots and
// gather the particle through the permutation, so every lane of a cell adds to
// the same statistics and the wave reduces them with DPP moves in a fixed
// order -- no atomics, and run-to-run identical results.  When the caller keeps particles
// in cell order (as the slabs of the paper's code do), the gathers are
// contiguous.  The per-box statistics are a two-level, fixed-order reduction
// over chunks of 512 cells.
#include "nf_internal.h"

namespace anf {

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
// that rounds up to L becomes 0).
__device__ __forceinline__ float wrap_coord(double t, double L) {
  const double q = floor(t / L);
  double r = t - q * L;
  if (r < 0.0) r += L;
  if (r >= L) r -= L;
  float f = (float)r;
  if (f >= (float)L) f = 0.0f;
  return f;
}

__global__ __launch_bounds__(256) void k_kick_drift(const DevBox* __restrict__ boxes, int nboxes,
                                                    int64_t cells_total,
                                                    const int32_t* __restrict__ off,
                                                    const int32_t* __restrict__ perm,
                                                    float* __restrict__ pos,
                                                    float* __restrict__ vel,
                                                    const float* __restrict__ acc,
                                                    double* __restrict__ cell_sumsq,
                                                    double* __restrict__ cell_amax,
                                                    double* __restrict__ cell_stats) {
  const int lane = threadIdx.x & 63;
  const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) >> 6;
  // The next cell's slot range is requested before this cell's particles are
  // processed, so its latency overlaps them.
  int nbeg = 0, nend = 0;
  if (wave < cells_total) {
    nbeg = __builtin_amdgcn_readfirstlane(off[wave]);
    nend = __builtin_amdgcn_readfirstlane(off[wave + 1]);
  }
  for (int64_t c = wave; c < cells_total; c += nwaves) {
    const int beg = nbeg, end = nend;
    if (c + nwaves < cells_total) {
      nbeg = __builtin_amdgcn_readfirstlane(off[c + nwaves]);
      nend = __builtin_amdgcn_readfirstlane(off[c + nwaves + 1]);
    }
    const int b = nboxes == 1 ? 0 : find_box_by_cell(boxes, nboxes, c);
    const double kick = boxes[b].kick, drift = boxes[b].drift, L = boxes[b].box_len;
    double s2 = 0.0, am = 0.0;
    for (int s = beg + lane; s < end; s += 64) {
      const int64_t i = perm[s];
      const float ax = acc[3 * i], ay = acc[3 * i + 1], az = acc[3 * i + 2];
      const float vx = (float)((double)vel[3 * i] + kick * (double)ax);
      const float vy = (float)((double)vel[3 * i + 1] + kick * (double)ay);
      const float vz = (float)((double)vel[3 * i + 2] + kick * (double)az);
      vel[3 * i] = vx;
      vel[3 * i + 1] = vy;
      vel[3 * i + 2] = vz;
      pos[3 * i] = wrap_coord((double)pos[3 * i] + drift * (double)vx, L);
      pos[3 * i + 1] = wrap_coord((double)pos[3 * i + 1] + drift * (double)vy, L);
      pos[3 * i + 2] = wrap_coord((double)pos[3 * i + 2] + drift * (double)vz, L);
      s2 += ((double)vx * (double)vx + (double)vy * (double)vy) + (double)vz * (double)vz;
      const double a2 = ((double)ax * (double)ax + (double)ay * (double)ay) + (double)az * (double)az;
      const double a = sqrt(a2);
      am = a > am ? a : am;
    }
    // Sum and maximum over the wave with DPP moves in a fixed pattern (quad
    // permutes, half-row and row mirrors, then the row broadcasts into rows 1
    // and 3 and into rows 2 and 3); lane 63 ends with both totals.  Lanes of
    // rows a broadcast does not write add 0, and 0 <= |a| leaves the maximum.
    {
      double o;
      o = dpp_f64<0xB1, 0xF>(s2); s2 += o; o = dpp_f64<0xB1, 0xF>(am); am = o > am ? o : am;
      o = dpp_f64<0x4E, 0xF>(s2); s2 += o; o = dpp_f64<0x4E, 0xF>(am); am = o > am ? o : am;
      o = dpp_f64<0x141, 0xF>(s2); s2 += o; o = dpp_f64<0x141, 0xF>(am); am = o > am ? o : am;
      o = dpp_f64<0x140, 0xF>(s2); s2 += o; o = dpp_f64<0x140, 0xF>(am); am = o > am ? o : am;
      o = dpp_f64<0x142, 0xA>(s2); s2 += o; o = dpp_f64<0x142, 0xA>(am); am = o > am ? o : am;
      o = dpp_f64<0x143, 0xC>(s2); s2 += o; o = dpp_f64<0x143, 0xC>(am); am = o > am ? o : am;
    }
    if (lane == 63) {
      cell_sumsq[c] = s2;
      cell_amax[c] = am;
      if (cell_stats) {
        const int n = end - beg;
        cell_stats[2 * c] = n > 0 ? sqrt(s2 / (double)n) : 0.0;
        cell_stats[2 * c + 1] = am;
      }
    }
  }
}

// Stage 1: chunk k of a box -> (min over its cells of v_rms/a_max, sum |v'|^2,
// max |a|), reduced across the block in a fixed tree order.
__global__ __launch_bounds__(256) void k_kdk_chunks(const DevBox* __restrict__ boxes, int nboxes,
                                                    const int32_t* __restrict__ off,
                                                    const double* __restrict__ cell_sumsq,
                                                    const double* __restrict__ cell_amax,
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
    const int n = off[c + 1] - off[c];
    const double s2 = cell_sumsq[c], am = cell_amax[c];
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

hipError_t launch_kick_drift(const DevBox* boxes, int nboxes, int64_t cells_total,
                             const KdkWork& w, const int32_t* off, const int32_t* perm,
                             float* pos, float* vel, const float* acc, double* cell_stats,
                             double* box_stats, hipStream_t s) {
  const void* fn = reinterpret_cast<const void*>(&k_kick_drift);
  int64_t blocks = persistent_blocks(fn, 256);
  const int64_t need = (cells_total + 3) / 4;  // four waves (cells) per block
  if (blocks > need) blocks = need > 0 ? need : 1;
  hipLaunchKernelGGL(k_kick_drift, dim3((unsigned)blocks), dim3(256), 0, s, boxes, nboxes,
                     cells_total, off, perm, pos, vel, acc, w.cell_sumsq, w.cell_amax,
                     cell_stats);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || !box_stats) return e;
  hipLaunchKernelGGL(k_kdk_chunks, dim3((unsigned)w.chunks), dim3(256), 0, s, boxes, nboxes, off,
                     w.cell_sumsq, w.cell_amax, w.chunk_part);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  hipLaunchKernelGGL(k_kdk_boxes, dim3((unsigned)nboxes), dim3(256), 0, s, boxes, w.chunk_part,
                     box_stats);
  return hipGetLastError();
}

}  // namespace anf
