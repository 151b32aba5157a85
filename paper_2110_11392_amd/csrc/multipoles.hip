// Cell multipoles in the complete basis of order p (Eq. 4), and their
// reduction to (p+1)^2 values per cell.
//
// What it computes: for every cell, M^{a,b,c} = sum_q x_q^a y_q^b z_q^c over
// the cell's particles, (x, y, z) the displacement from the cell centre in box
// units, for a + b + c <= p (enumerated a outermost, c innermost).  The sums
// are FP64 (the paper keeps every far-field computation in double precision),
// formed from the stored FP32 cell-relative offsets.
//
// How it maps to CDNA4:
//   * a work wave covers a run of consecutive cells of one pencil; each cell
//     gets min(64, ceil(n/8)) lanes and each lane sums a contiguous segment of
//     the cell's particles, so every lane works on at least a few particles and
//     no cell is split across waves;
//   * a lane keeps its partial moments in VGPRs (two passes over the segment
//     when the basis is too large for the register file, split by the power
//     of x), then the wave reduces the lanes of each cell through LDS, a chunk
//     of terms at a time, with one lane per (cell, term) adding its cell's rows
//     in lane order -- a fixed order, so results are run-to-run deterministic;
//   * each (cell, term) result is scaled by w^(a+b+c) and written once; the
//     writes of one cell row are contiguous across lanes.
// The reduced basis is a second, HBM-bound pass over the complete rows.
#include "nf_internal.h"

namespace anf {

constexpr int kMpMinSeg = 8;   // particles per lane before a cell gets another lane
constexpr int kMpChunk = 16;   // terms reduced per LDS round
constexpr int kMpStride = kMpChunk + 1;

__host__ __device__ constexpr int mp_terms_a(int p, int a0, int a1) {
  int t = 0;
  for (int a = a0; a <= a1; ++a) t += (p - a + 1) * (p - a + 2) / 2;
  return t;
}

// First power of x of the second pass: the split that keeps the larger pass
// smallest (one pass when every term fits in 96 accumulators).
__host__ __device__ constexpr int mp_split(int p) {
  if (mp_terms_a(p, 0, p) <= 96) return p + 1;
  int best = p + 1, best_max = mp_terms_a(p, 0, p);
  for (int a1 = 1; a1 <= p; ++a1) {
    const int lo = mp_terms_a(p, 0, a1 - 1), hi = mp_terms_a(p, a1, p);
    const int m = lo > hi ? lo : hi;
    if (m < best_max) {
      best_max = m;
      best = a1;
    }
  }
  return best;
}

int64_t multipole_terms(int p, bool reduced) {
  if (p < 0) return 0;
  return reduced ? (int64_t)(p + 1) * (p + 1) : (int64_t)mp_terms_a(p, 0, p);
}

__device__ __forceinline__ int mp_nseg(int n) {
  if (n <= 0) return 0;
  const int s = (n + kMpMinSeg - 1) / kMpMinSeg;
  return s < 64 ? s : 64;
}

// ---- work waves ------------------------------------------------------------
// wave = {first global cell, end cell, box, 0}: consecutive cells of one pencil
// with at most 64 lanes' worth of segments and at most 64 cells.
template <bool kEmit>
__device__ int mp_walk_pencil(const int32_t* __restrict__ off, int cell0, int K, int b,
                              int4* __restrict__ out) {
  int nw = 0, lo = 0, lanes = 0;
  for (int z = 0; z < K; ++z) {
    const int ns = mp_nseg(off[cell0 + z + 1] - off[cell0 + z]);
    if (z > lo && (lanes + ns > 64 || z - lo >= 64)) {
      if (kEmit) out[nw] = make_int4(cell0 + lo, cell0 + z, b, 0);
      ++nw;
      lo = z;
      lanes = 0;
    }
    lanes += ns;
  }
  if (kEmit) out[nw] = make_int4(cell0 + lo, cell0 + K, b, 0);
  return nw + 1;
}

__global__ __launch_bounds__(64) void k_mp_count(const DevBox* __restrict__ boxes, int nboxes,
                                                 int64_t pencils, const int32_t* __restrict__ off,
                                                 int32_t* __restrict__ counts) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= pencils) return;
  const int b = nboxes == 1 ? 0 : find_box_by_pencil(boxes, nboxes, (int)p);
  const int K = boxes[b].K;
  const int local = (int)p - boxes[b].pencil_base;
  counts[p] = mp_walk_pencil<false>(off, boxes[b].cell_base + local * K, K, b, nullptr);
}

__global__ __launch_bounds__(64) void k_mp_emit(const DevBox* __restrict__ boxes, int nboxes,
                                                int64_t pencils, const int32_t* __restrict__ off,
                                                const int32_t* __restrict__ base,
                                                int4* __restrict__ waves) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= pencils) return;
  const int b = nboxes == 1 ? 0 : find_box_by_pencil(boxes, nboxes, (int)p);
  const int K = boxes[b].K;
  const int local = (int)p - boxes[b].pencil_base;
  mp_walk_pencil<true>(off, boxes[b].cell_base + local * K, K, b, waves + base[p]);
}

// ---- the moment kernel ----------------------------------------------------

struct MpShared {
  double rows[64 * kMpStride];   // one chunk of every lane's partial moments
  double wpow[20];               // w^n, n = 0..p
  int cell_row[65];              // first lane (row) of each cell of the wave; [ncells] = rows
  unsigned char order[1024];     // a + b + c of each complete term
};

// Sum the terms with x power in [A0, A1] of this lane's particles, then reduce
// each cell's lanes and write the scaled results.
template <int P, int A0, int A1>
__device__ __forceinline__ void mp_pass(const float4* __restrict__ rel, int beg, int end,
                                        MpShared& sh, int lane, int ncells, int64_t cell_lo,
                                        double* __restrict__ out) {
  constexpr int T = mp_terms_a(P, A0, A1);
  constexpr int TT = mp_terms_a(P, 0, P);
  constexpr int base = A0 == 0 ? 0 : mp_terms_a(P, 0, A0 - 1);
  double acc[T];
#pragma unroll
  for (int t = 0; t < T; ++t) acc[t] = 0.0;
  for (int j = beg; j < end; ++j) {
    const float4 r = rel[j];
    const double x = r.x, y = r.y, z = r.z;
    double yp[P + 1], zp[P + 1];
    yp[0] = 1.0;
    zp[0] = 1.0;
#pragma unroll
    for (int k = 1; k <= P; ++k) {
      yp[k] = yp[k - 1] * y;
      zp[k] = zp[k - 1] * z;
    }
    double xa = 1.0;
#pragma unroll
    for (int a = 0; a < A0; ++a) xa *= x;
    int k = 0;
#pragma unroll
    for (int a = A0; a <= A1; ++a) {
#pragma unroll
      for (int b = 0; b <= P - a; ++b) {
        const double m = a == 0 ? yp[b] : xa * yp[b];
#pragma unroll
        for (int c = 0; c <= P - a - b; ++c) {
          acc[k] = c == 0 ? acc[k] + m : __builtin_fma(m, zp[c], acc[k]);
          ++k;
        }
      }
      xa *= x;
    }
  }
  // Reduce chunk by chunk: lane rows go to LDS, then lane q adds the rows of
  // cell q / CH for term q % CH, in row order.
#pragma unroll
  for (int t0 = 0; t0 < T; t0 += kMpChunk) {
    constexpr int kCh = kMpChunk;
#pragma unroll
    for (int t = 0; t < kCh; ++t)
      if (t0 + t < T) sh.rows[lane * kMpStride + t] = acc[t0 + t];
    __syncthreads();
    const int ch = T - t0 < kCh ? T - t0 : kCh;
    for (int q = lane; q < ncells * ch; q += 64) {
      const int ci = q / ch, t = q - (q / ch) * ch;
      const int r0 = sh.cell_row[ci], r1 = sh.cell_row[ci + 1];
      double s = 0.0;
      for (int r = r0; r < r1; ++r) s += sh.rows[r * kMpStride + t];
      const int g = base + t0 + t;
      out[(cell_lo + ci) * TT + g] = s * sh.wpow[sh.order[g]];
    }
    __syncthreads();
  }
}

template <int P>
__global__ __launch_bounds__(64) void k_multipoles(const DevBox* __restrict__ boxes,
                                                   const int4* __restrict__ waves,
                                                   const int32_t* __restrict__ n_waves_ptr,
                                                   const int32_t* __restrict__ off,
                                                   const float4* __restrict__ rel,
                                                   double* __restrict__ out) {
  __shared__ MpShared sh;
  constexpr int A1 = mp_split(P);
  const int lane = threadIdx.x;
  {
    int k = 0;
#pragma unroll
    for (int a = 0; a <= P; ++a)
#pragma unroll
      for (int b = 0; b <= P - a; ++b)
#pragma unroll
        for (int c = 0; c <= P - a - b; ++c) {
          if ((k & 63) == lane) sh.order[k] = (unsigned char)(a + b + c);
          ++k;
        }
  }
  const int n_waves = __builtin_amdgcn_readfirstlane(*n_waves_ptr);
  for (int wv = blockIdx.x; wv < n_waves; wv += gridDim.x) {
    const int4 rec = waves[wv];
    const int c_lo = __builtin_amdgcn_readfirstlane(rec.x);
    const int c_hi = __builtin_amdgcn_readfirstlane(rec.y);
    const int b = __builtin_amdgcn_readfirstlane(rec.z);
    const int ncells = c_hi - c_lo;
    // lane -> (cell, segment of that cell's particles)
    int beg = 0, end = 0, rows = 0;
    for (int c = c_lo; c < c_hi; ++c) {
      const int cb = __builtin_amdgcn_readfirstlane(off[c]);
      const int ce = __builtin_amdgcn_readfirstlane(off[c + 1]);
      const int ns = mp_nseg(ce - cb);
      if (lane == c - c_lo) sh.cell_row[lane] = rows;
      if (lane >= rows && lane < rows + ns) {
        const int per = (ce - cb + ns - 1) / ns;
        beg = cb + (lane - rows) * per;
        end = beg + per < ce ? beg + per : ce;
      }
      rows += ns;
    }
    if (lane == 0) sh.cell_row[ncells] = rows;
    if (lane <= P) {
      const double w = boxes[b].width;
      double v = 1.0;
      for (int k = 0; k < lane; ++k) v *= w;
      sh.wpow[lane] = v;
    }
    __syncthreads();
    mp_pass<P, 0, A1 - 1>(rel, beg, end, sh, lane, ncells, c_lo, out);
    if constexpr (A1 <= P) mp_pass<P, A1, P>(rel, beg, end, sh, lane, ncells, c_lo, out);
  }
}

// ---- reduction to (p+1)^2 values -------------------------------------------
// R^{a,b,c0} = sum_{m, i} (-1)^m C(m, i) a! b! c0! / ((a-2i)! (b-2m+2i)! (c0+2m)!)
//              M^{a-2i, b-2m+2i, c0+2m},
// so that the exterior expansion sum (-1)^n M^{abc}/(a!b!c!) D_{abc} keeps its
// value with D_{a,b,c+2} = -D_{a+2,b,c} - D_{a,b+2,c} (1/r is harmonic).

__device__ __forceinline__ int mp_index(int p, int a, int b, int c) {
  // position of (a, b, c) in the complete enumeration (a outermost)
  int k = 0;
  for (int aa = 0; aa < a; ++aa) k += (p - aa + 1) * (p - aa + 2) / 2;
  for (int bb = 0; bb < b; ++bb) k += p - a - bb + 1;
  return k + c;
}

__device__ __forceinline__ double mp_fact(int n) {
  double f = 1.0;
  for (int i = 2; i <= n; ++i) f *= (double)i;
  return f;
}

__global__ __launch_bounds__(256) void k_mp_reduce(const double* __restrict__ full, int p,
                                                   int64_t cells, double* __restrict__ out) {
  const int RT = (p + 1) * (p + 1);
  const int TT = mp_terms_a(p, 0, p);
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= cells * RT) return;
  const int64_t cell = idx / RT;
  int r = (int)(idx - cell * RT);
  // decode reduced term r -> (a, b, c0), enumerated a, b, then c0 in {0, 1}
  int a = 0, b = 0, c0 = 0;
  for (a = 0; a <= p; ++a) {
    int here = 0;
    for (int bb = 0; bb <= p - a; ++bb) here += (p - a - bb >= 1) ? 2 : 1;
    if (r < here) break;
    r -= here;
  }
  for (b = 0; b <= p - a; ++b) {
    const int here = (p - a - b >= 1) ? 2 : 1;
    if (r < here) break;
    r -= here;
  }
  c0 = r;
  const double* row = full + cell * TT;
  double sum = 0.0;
  for (int m = 0; 2 * m <= a + b; ++m)
    for (int i = 0; i <= m; ++i) {
      const int sa = a - 2 * i, sb = b - 2 * (m - i), sc = c0 + 2 * m;
      if (sa < 0 || sb < 0) continue;
      const double coef = ((m & 1) ? -1.0 : 1.0) * (mp_fact(m) / (mp_fact(i) * mp_fact(m - i))) *
                          mp_fact(a) * mp_fact(b) * mp_fact(c0) /
                          (mp_fact(sa) * mp_fact(sb) * mp_fact(sc));
      sum += coef * row[mp_index(p, sa, sb, sc)];
    }
  out[idx] = sum;
}

// ---- host launch -------------------------------------------------------------

template <int P>
static hipError_t launch_mp_t(const DevBox* boxes, const MpWork& w, const int32_t* off,
                              const float* rel, double* full, hipStream_t s) {
  const void* fn = reinterpret_cast<const void*>(&k_multipoles<P>);
  int blocks = persistent_blocks(fn, 64);
  if ((int64_t)blocks > w.max_waves) blocks = (int)(w.max_waves > 0 ? w.max_waves : 1);
  hipLaunchKernelGGL(k_multipoles<P>, dim3(blocks), dim3(64), 0, s, boxes, w.waves,
                     w.wave_base + w.pencils, off, reinterpret_cast<const float4*>(rel), full);
  return hipGetLastError();
}

hipError_t launch_multipoles(const DevBox* boxes, int nboxes, int64_t cells_total, int order,
                             bool reduced, const MpWork& w, const int32_t* off, const float* rel,
                             double* out, hipStream_t s) {
  const unsigned pg = (unsigned)((w.pencils + 63) / 64);
  hipLaunchKernelGGL(k_mp_count, dim3(pg), dim3(64), 0, s, boxes, nboxes, w.pencils, off,
                     w.wave_count);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  if ((e = exclusive_scan(w.wave_count, w.wave_base, w.pencils, w.scan_tmp, s)) != hipSuccess)
    return e;
  hipLaunchKernelGGL(k_mp_emit, dim3(pg), dim3(64), 0, s, boxes, nboxes, w.pencils, off,
                     w.wave_base, w.waves);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  double* full = reduced ? w.full : out;
  switch (order) {
    case 0: e = launch_mp_t<0>(boxes, w, off, rel, full, s); break;
    case 1: e = launch_mp_t<1>(boxes, w, off, rel, full, s); break;
    case 2: e = launch_mp_t<2>(boxes, w, off, rel, full, s); break;
    case 3: e = launch_mp_t<3>(boxes, w, off, rel, full, s); break;
    case 4: e = launch_mp_t<4>(boxes, w, off, rel, full, s); break;
    case 5: e = launch_mp_t<5>(boxes, w, off, rel, full, s); break;
    case 6: e = launch_mp_t<6>(boxes, w, off, rel, full, s); break;
    case 7: e = launch_mp_t<7>(boxes, w, off, rel, full, s); break;
    default: e = launch_mp_t<8>(boxes, w, off, rel, full, s); break;
  }
  if (e != hipSuccess || !reduced) return e;
  const int64_t threads = cells_total * (int64_t)(order + 1) * (order + 1);
  hipLaunchKernelGGL(k_mp_reduce, dim3((unsigned)((threads + 255) / 256)), dim3(256), 0, s, w.full,
                     order, cells_total, out);
  return hipGetLastError();
}

}  // namespace anf
