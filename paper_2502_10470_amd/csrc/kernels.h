// Host-side launch interface of the gfx950 kernels (internal to the library).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "device.h"

namespace mde {

struct TraceArgs {
  float *u;        // [sum N*D] trial vectors, or null
  float *fu;       // [sum N] trial fitness, or null
  int32_t *desc;   // [sum N][16] descriptors, or null
};

struct LaunchArgs {
  const RunDev *runs;
  const ProbDev *probs;
  const unsigned char *tab;
  float *pop;
  float *fit;
  float *pending;
  uint32_t n_runs;
  uint32_t lds_bytes;
  uint32_t init_lds_bytes;
  uint32_t mfma_lds_bytes;
  uint32_t k0, k1;
  uint32_t mfma_rows;   // row tiles per plain rotation item of the matrix-core kernel: 2 or 4
  int lane_kind;        // the function kind of every lane-kernel run, or -1 if they differ
  hipStream_t stream;
};

// Hidden widths of the control policies: 32 (the MLPs of Table VII) or CT_H = 64;
// both hidden layers have the same width, and all control runs of a context too.
// Lanes per policy in the evaluation: 32, or 16 for width 32 when every control
// problem has at most CT_OBS_L16 observations.
constexpr int CT_H_SMALL = 32;
constexpr int CT_OBS_L16 = 16;

// Control runs (two individuals per wavefront, several launches per generation).
struct CtrlArgs {
  const uint32_t *list;   // run ids
  uint32_t n, max_n;      // number of control runs, their largest N
  uint32_t hidden;        // hidden width of their policies (CT_H_SMALL or CT_H)
  uint32_t lanes;         // lanes per policy in the evaluation (32, or 16 for CT_H_SMALL)
  uint32_t mx;            // 1: every problem has a multiple of 16 rollouts, matrix-core evaluation
  uint32_t *order;        // [sum N] top-p lists at the runs' fitness offsets
  float *fu;              // [sum N] trial fitness
  uint32_t *acc;          // [sum N] selection decisions
};

#ifdef MDE_STAGE_CLOCKS
hipError_t read_stage_clocks(void *dst, size_t bytes);
hipError_t read_stage_clocks_mfma(void *dst, size_t bytes);
#endif
hipError_t set_lds_limits();
hipError_t launch_tables64(const float *R, double *Rt, uint32_t D, hipStream_t s);
hipError_t launch_init(const LaunchArgs &a, double lb, double ub);
hipError_t launch_generations(const LaunchArgs &a, const uint32_t *list, uint32_t n,
                              uint32_t g0, uint32_t n_gens, float lb, float ub, TraceArgs tr);
hipError_t set_lds_limits_mfma();
// padded float32 rotation [Rs][Rs] and R o in float64 for the matrix-core kernel
hipError_t launch_tables_mfma(const float *R, const float *o, float *R32, double *ro64, uint32_t D,
                              hipStream_t s);
hipError_t launch_generations_mfma(const LaunchArgs &a, const uint32_t *list, uint32_t n,
                                   bool bf16, uint32_t g0, uint32_t n_gens, float lb, float ub,
                                   unsigned long long *counters, TraceArgs tr);
hipError_t launch_ctrl_init(const LaunchArgs &a, const CtrlArgs &c, double lb, double ub);
// control runs: generation sequences read and advance the device counter gen
hipError_t launch_ctrl_set_gen(uint32_t *gen, uint32_t v, hipStream_t s);
hipError_t launch_ctrl_generations(const LaunchArgs &a, const CtrlArgs &c, uint32_t *gen,
                                   uint32_t n_gens, float lb, float ub, TraceArgs tr);
hipError_t launch_ctrl_finalize(const LaunchArgs &a, const CtrlArgs &c, double *best_y,
                                float *best_x);
hipError_t launch_finalize(const LaunchArgs &a, double *best_y, float *best_x);
hipError_t launch_decode(RunDev *runs, float *theta, uint32_t n, uint32_t n_cs, hipStream_t s);
hipError_t launch_outer_init(float *X, double *y, uint32_t P, uint32_t stream, uint32_t k0,
                             uint32_t k1, uint32_t n_cs, hipStream_t s);
hipError_t launch_outer_trial(const float *X, float *U, RunDev *runs, uint32_t P, uint32_t g_o,
                              uint32_t stream, uint32_t k0, uint32_t k1, uint32_t n_cs,
                              hipStream_t s);
hipError_t launch_outer_select(float *X, double *y, const float *U, const double *y_run,
                               double *y_trial, float *bxo, const float *best_x,
                               const RunDev *runs, uint32_t P, bool take_all, hipStream_t s);
hipError_t launch_cso_move(float *X, float *V, float *U, const double *y, RunDev *runs,
                           uint32_t P, uint32_t g_o, uint32_t stream, uint32_t k0, uint32_t k1,
                           uint32_t n_cs, hipStream_t s);
hipError_t launch_nes_init(float *V, uint32_t n_cs, hipStream_t s);
hipError_t launch_nes_sample(float *U, const float *V, RunDev *runs, uint32_t P, uint32_t g_o,
                             uint32_t stream, uint32_t k0, uint32_t k1, uint32_t n_cs,
                             hipStream_t s);
hipError_t launch_nes_update(const double *y, float *V, uint32_t P, uint32_t g_o, uint32_t stream,
                             uint32_t k0, uint32_t k1, double eta_sigma, hipStream_t s);
hipError_t launch_outer_best(const double *y, uint32_t P, int32_t *out, hipStream_t s);
hipError_t launch_pso_move(float *U, float *V, const float *X, const int32_t *gbest, RunDev *runs,
                           uint32_t P, uint32_t g_o, uint32_t stream, uint32_t k0, uint32_t k1,
                           uint32_t n_cs, hipStream_t s);

}  // namespace mde
