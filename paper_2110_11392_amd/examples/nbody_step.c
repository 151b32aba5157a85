/*
 * nbody_step.c -- the near field through the C ABI alone, from plain C99.
 *
 * A periodic box of uniformly placed particles goes through a few leapfrog
 * steps: binning (Sec. 2.2), near-field accelerations with the per-box FP64
 * momentum sums (Eq. 3, Sec. 3.4.1), the adjoint for a fixed cotangent, the
 * kick and drift with the Eq. 1 statistics (Sec. 3.1) and the resulting time
 * step.  Every device buffer and the workspace are the caller's (hipMalloc
 * here); the library only enqueues work on the stream.
 *
 * Usage: nbody_step [n] [cells per dimension] [steps]   (defaults 262144 16 3)
 * Exit status 0 when every call succeeds and the momentum residual
 * |sum a| / sum |a| of every step stays below 1e-5 (pair antisymmetry).
 */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

#include <hip/hip_runtime_api.h>

#include "abacus_nf.h"

#define CHECK_NF(call)                                                         \
  do {                                                                         \
    int rc_ = (call);                                                          \
    if (rc_ != ABACUS_NF_OK) {                                                 \
      fprintf(stderr, "%s: %s\n", #call, abacus_nf_strerror(rc_));             \
      return 1;                                                                \
    }                                                                          \
  } while (0)

#define CHECK_HIP(call)                                                        \
  do {                                                                         \
    hipError_t e_ = (call);                                                    \
    if (e_ != hipSuccess) {                                                    \
      fprintf(stderr, "%s: %s\n", #call, hipGetErrorString(e_));               \
      return 1;                                                                \
    }                                                                          \
  } while (0)

/* 64-bit linear congruential generator, top 24 bits as a float in [0, 1). */
static float uniform01(uint64_t *s) {
  *s = *s * 6364136223846793005ull + 1442695040888963407ull;
  return (float)(*s >> 40) * (1.0f / 16777216.0f);
}

int main(int argc, char **argv) {
  const int64_t n = argc > 1 ? atoll(argv[1]) : 262144;
  const int cpd = argc > 2 ? atoi(argv[2]) : 16;
  const int steps = argc > 3 ? atoi(argv[3]) : 3;
  abacus_nf_box box = {n, 1.0, cpd, 2, 1.0 / (40.0 * cbrt((double)n)), 0.0};

  int64_t n_total = 0, cells_total = 0;
  CHECK_NF(abacus_nf_layout(&box, 1, &n_total, &cells_total));
  size_t ws_bytes = 0, kdk_bytes = 0;
  CHECK_NF(abacus_nf_workspace_bytes(&box, 1, &ws_bytes));
  CHECK_NF(abacus_nf_kick_drift_workspace_bytes(&box, 1, &kdk_bytes));
  printf("n = %lld, K = %d (%lld cells), workspace %.1f MB + %.1f MB\n", (long long)n_total, cpd,
         (long long)cells_total, ws_bytes / 1e6, kdk_bytes / 1e6);

  /* host state: uniform positions, zero velocities, a fixed cotangent */
  const size_t bytes3 = (size_t)n_total * 3 * sizeof(float);
  float *h_pos = (float *)malloc(bytes3), *h_w = (float *)malloc(bytes3);
  if (!h_pos || !h_w) return 1;
  uint64_t seed = 2110113920ull;
  for (int64_t i = 0; i < 3 * n_total; ++i) {
    h_pos[i] = uniform01(&seed);
    h_w[i] = uniform01(&seed) - 0.5f;
  }

  float *pos, *vel, *acc, *grad, *w, *rel;
  int32_t *offsets, *perm, *status;
  double *momentum, *box_stats;
  void *ws, *kdk_ws;
  CHECK_HIP(hipMalloc((void **)&pos, bytes3));
  CHECK_HIP(hipMalloc((void **)&vel, bytes3));
  CHECK_HIP(hipMalloc((void **)&acc, bytes3));
  CHECK_HIP(hipMalloc((void **)&grad, bytes3));
  CHECK_HIP(hipMalloc((void **)&w, bytes3));
  CHECK_HIP(hipMalloc((void **)&rel, (size_t)n_total * 4 * sizeof(float)));
  CHECK_HIP(hipMalloc((void **)&offsets, (size_t)(cells_total + 1) * sizeof(int32_t)));
  CHECK_HIP(hipMalloc((void **)&perm, (size_t)n_total * sizeof(int32_t)));
  CHECK_HIP(hipMalloc((void **)&status, sizeof(int32_t)));
  CHECK_HIP(hipMalloc((void **)&momentum, 4 * sizeof(double)));
  CHECK_HIP(hipMalloc((void **)&box_stats, 4 * sizeof(double)));
  CHECK_HIP(hipMalloc(&ws, ws_bytes));
  CHECK_HIP(hipMalloc(&kdk_ws, kdk_bytes));
  CHECK_HIP(hipMemcpy(pos, h_pos, bytes3, hipMemcpyHostToDevice));
  CHECK_HIP(hipMemcpy(w, h_w, bytes3, hipMemcpyHostToDevice));
  CHECK_HIP(hipMemset(vel, 0, bytes3));

  hipStream_t stream;
  CHECK_HIP(hipStreamCreate(&stream));
  hipEvent_t t0, t1;
  CHECK_HIP(hipEventCreate(&t0));
  CHECK_HIP(hipEventCreate(&t1));
  const abacus_nf_binned binned = {offsets, perm, rel, status};
  const double kick = 1e-6, drift = 1e-6;
  int ok = 1;
  for (int step = 0; step < steps; ++step) {
    double m[4], stats[4];
    int32_t st = 0;
    CHECK_HIP(hipEventRecord(t0, stream));
    CHECK_NF(abacus_nf_bin(&box, 1, pos, &binned, ws, ws_bytes, stream));
    CHECK_NF(abacus_nf_forces(&box, 1, &binned, acc, NULL, momentum, NULL,
                              ABACUS_NF_COMPENSATED, ws, ws_bytes, stream));
    CHECK_NF(abacus_nf_forces_vjp(&box, 1, &binned, w, grad, ABACUS_NF_COMPENSATED, ws,
                                  ws_bytes, stream));
    CHECK_NF(abacus_nf_kick_drift(&box, 1, &binned, &kick, &drift, pos, vel, acc, NULL,
                                  box_stats, kdk_ws, kdk_bytes, stream));
    CHECK_HIP(hipEventRecord(t1, stream));
    CHECK_HIP(hipMemcpyAsync(m, momentum, sizeof m, hipMemcpyDeviceToHost, stream));
    CHECK_HIP(hipMemcpyAsync(stats, box_stats, sizeof stats, hipMemcpyDeviceToHost, stream));
    CHECK_HIP(hipMemcpyAsync(&st, status, sizeof st, hipMemcpyDeviceToHost, stream));
    CHECK_HIP(hipStreamSynchronize(stream));
    float ms = 0.f;
    CHECK_HIP(hipEventElapsedTime(&ms, t0, t1));
    const double resid = sqrt(m[0] * m[0] + m[1] * m[1] + m[2] * m[2]) / m[3];
    const double da = abacus_nf_timestep(stats, 1.0, 1.0, 0.25, 0.03);
    printf("step %d: %.3f ms, momentum residual %.2e, v_rms %.3e, a_max %.3e, Eq. 1 step %.3e, "
           "status %d\n",
           step, ms, resid, stats[1], stats[2], da, st);
    if (!(resid < 1e-5) || st != 0) ok = 0;
  }
  hipFree(pos); hipFree(vel); hipFree(acc); hipFree(grad); hipFree(w); hipFree(rel);
  hipFree(offsets); hipFree(perm); hipFree(status); hipFree(momentum); hipFree(box_stats);
  hipFree(ws); hipFree(kdk_ws);
  hipStreamDestroy(stream);
  free(h_pos);
  free(h_w);
  printf(ok ? "ok\n" : "FAILED\n");
  return ok ? 0 : 1;
}
