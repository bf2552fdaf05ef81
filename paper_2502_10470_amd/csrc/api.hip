// C ABI of the MetaDE inner-DE library: validation, device tables, launch
// sequencing of the executor and evolver kernels, checkpointing and timing.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <mutex>
#include <sstream>
#include <string>
#include <vector>

#include "metade.h"
#include "device.h"
#include "kernels.h"

using mde::LaunchArgs;
using mde::ProbDev;
using mde::RunDev;

// Workspace of metade_inner_step_static: the matrix-core kernel's trial rows
// of every run, at the run offsets the context
// uses for its own trial buffer.  One copy per GPU, held until the process
// ends.  In host code this name is only a stand-in for the symbol: kernels
// get the per-device address that hipGetSymbolAddress returns at init.
static __device__ __align__(256) float scratch[METADE_STATIC_SCRATCH_BYTES / sizeof(float)];

namespace {

thread_local std::string g_init_error = "no error";

// Device address of `scratch` on each GPU, looked up once per device (with
// that device current) by metade_init.
constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mu;
float *g_scratch_dev[MAX_DEVICES] = {};

// Device counters of a context: [0] trials re-evaluated exactly by the bf16
// mode; [1..5] the bound check of traced bf16 generations (checked, outside
// the bound, screened out, screened out but accepted by the exact value, and
// the largest deviation / bound as double bits).
constexpr size_t N_COUNTERS = 8;

struct EventPair {
  hipEvent_t a, b;
};

}  // namespace

struct metade_ctx {
  hipStream_t stream = nullptr;
  uint32_t n_runs = 0, n_cs = 2, precision = 0, evolver = 0;
  uint64_t seed = 0;
  float lb = 0, ub = 0;
  float *pop = nullptr, *fit = nullptr, *best_x = nullptr;
  double *best_y = nullptr;
  std::vector<RunDev> runs_h;
  std::vector<ProbDev> probs_h;
  RunDev *runs_d = nullptr;
  ProbDev *probs_d = nullptr;
  float *theta_d = nullptr;
  float *pend_d = nullptr;
  size_t pop_floats = 0, fit_n = 0, bx_n = 0, pend_floats = 0;
  uint32_t lds_bytes = 0, init_lds_bytes = 0, mfma_lds_bytes = 0;
  int lane_kind = -1;   // one kind for every lane-kernel run: its own kernel (else -1)
  uint32_t n_lane = 0, n_mfma = 0, n_ctrl = 0, ctrl_max_n = 0, ctrl_hidden = 0, ctrl_lanes = 32;
  uint32_t ctrl_mx = 0;
  uint32_t *lane_list_d = nullptr, *mfma_list_d = nullptr, *ctrl_list_d = nullptr;
  uint32_t *order_d = nullptr, *cacc_d = nullptr;  // control runs: top-p lists, decisions
  float *cfu_d = nullptr;                          // control runs: trial fitness
  unsigned long long *counters_d = nullptr;
  int device = 0;
  float *scratch_d = nullptr;   // this device's copy of the static workspace
  // tuning: row tiles per plain rotation item (matrix-core kernel) and parts
  // per trial in the lane kernel's fitness stage (0 = as many as fit)
  uint32_t mfma_rows = 4, lane_parts = 0;
  uint32_t gen = 0;
  // control runs: device copy of the generation counter, and the generation
  // loop captured as HIP graphs (one per sequence length, replayed on stream)
  uint32_t *gen_d = nullptr;
  bool graph = false;
  hipStream_t cap_stream = nullptr;
  std::vector<std::pair<uint32_t, hipGraphExec_t>> graphs;
  // evolver
  float *Xo = nullptr, *Uo = nullptr, *Vo = nullptr, *bxo = nullptr;  // Vo: PSO velocities
  double *yo = nullptr, *yt = nullptr;
  int32_t *bidx = nullptr;
  unsigned char *tab = nullptr; // read-only problem tables (shift, float64 rotation, weights)
  uint32_t outer_gen = 0;
  bool outer_ready = false;
  // measurement
  bool timing = false;
  std::vector<EventPair> events;
  uint64_t trials = 0, refined = 0;
  std::string err = "no error";
};

namespace {

metade_status fail(metade_ctx *c, metade_status s, const std::string &msg) {
  if (c) c->err = msg; else g_init_error = msg;
  return s;
}

#define HIP_TRY(ctx, expr)                                                              \
  do {                                                                                  \
    hipError_t e_ = (expr);                                                             \
    if (e_ != hipSuccess)                                                               \
      return fail((ctx), METADE_EDEVICE, std::string(#expr) + ": " + hipGetErrorString(e_)); \
  } while (0)

uint32_t round4(uint32_t d) { return (d + 3u) & ~3u; }

struct Plan {
  std::vector<RunDev> runs;
  std::vector<ProbDev> probs;
  size_t tab_bytes = 0;
  uint32_t init_lds_bytes = 0, mfma_lds_bytes = 0;
  std::vector<uint32_t> lane_list, mfma_list, ctrl_list;
  uint32_t ctrl_max_n = 0, ctrl_hidden = 0, ctrl_max_obs = 0;
  bool ctrl_roll16 = true;   // every control problem has a multiple of 16 rollouts
  size_t pop_floats = 0, fit_n = 0, bx_n = 0, pend_floats = 0;
  uint32_t lds_bytes = 0;
  int lane_kind = -1;        // the kind of every lane-kernel run, -1 if they differ
};

metade_status plan_config(const metade_config *cfg, Plan &pl, std::string &msg) {
  if (!cfg) { msg = "cfg is NULL"; return METADE_EINVAL; }
  if (cfg->n_runs == 0) { msg = "n_runs must be >= 1"; return METADE_EINVAL; }
  if (!cfg->N || !cfg->problem || !cfg->stream_id) { msg = "N, problem and stream_id host arrays are required"; return METADE_EINVAL; }
  if (cfg->n_problems == 0 || !cfg->problems) { msg = "at least one problem is required"; return METADE_EINVAL; }
  if (!(cfg->lb < cfg->ub) || std::fabs(cfg->lb) > 1e30f || std::fabs(cfg->ub) > 1e30f) {
    msg = "search box must satisfy lb < ub and |lb|, |ub| <= 1e30"; return METADE_EINVAL;
  }
  if (cfg->n_cs != 2 && cfg->n_cs != 3) { msg = "n_cs must be 2 or 3"; return METADE_EINVAL; }
  if (cfg->precision != METADE_FP32 && cfg->precision != METADE_BF16_REFINE) {
    msg = "precision must be METADE_FP32 or METADE_BF16_REFINE"; return METADE_EINVAL;
  }
  if (cfg->evolver != METADE_EVOLVER_DE && cfg->evolver != METADE_EVOLVER_PSO &&
      cfg->evolver != METADE_EVOLVER_CSO && cfg->evolver != METADE_EVOLVER_NES) {
    msg = "evolver must be METADE_EVOLVER_DE, METADE_EVOLVER_PSO, METADE_EVOLVER_CSO or "
          "METADE_EVOLVER_NES";
    return METADE_EINVAL;
  }
  if (cfg->evolver == METADE_EVOLVER_CSO && cfg->n_runs > 1024) {
    msg = "the CSO evolver pairs at most 1024 particles (n_runs <= 1024)"; return METADE_EINVAL;
  }
  if (cfg->evolver == METADE_EVOLVER_NES && cfg->n_runs > 1024) {
    msg = "the NES evolver ranks at most 1024 samples (n_runs <= 1024)"; return METADE_EINVAL;
  }
  pl.probs.resize(cfg->n_problems);
  const double zs = mde::SCHWEFEL_ZSTAR;
  const double cs = zs * std::sin(std::sqrt(zs));
  for (uint32_t k = 0; k < cfg->n_problems; ++k) {
    const metade_problem &q = cfg->problems[k];
    ProbDev p;
    std::memset(&p, 0, sizeof(p));
    p.kind = q.kind;
    p.D = q.D;
    p.bias = q.bias;
    p.cs_d = cs;
    p.cs_f = (float)cs;
    const double cond = q.cond > 0 ? (double)q.cond : 1e6;
    if (q.kind < METADE_FN_RASTRIGIN || q.kind > METADE_FN_LQR_MLP) {
      msg = "problem " + std::to_string(k) + ": unsupported kind " + std::to_string(q.kind);
      return METADE_EINVAL;
    }
    auto take = [&](size_t bytes) {
      const uint64_t off = pl.tab_bytes;
      pl.tab_bytes += (bytes + 255) & ~(size_t)255;
      return off;
    };
    if (q.kind == METADE_FN_LQR_MLP) {
      const std::string pk = "problem " + std::to_string(k) + ": ";
      const uint32_t H = q.hidden1;
      if ((H != (uint32_t)mde::CT_H_SMALL && H != (uint32_t)mde::CT_H) || q.hidden2 != H) {
        msg = pk + "control policy hidden layers must both have 32 or both 64 units";
        return METADE_EINVAL;
      }
      if (pl.ctrl_hidden != 0 && pl.ctrl_hidden != H) {
        msg = pk + "all control policies of a context must have the same hidden width";
        return METADE_EINVAL;
      }
      pl.ctrl_hidden = H;
      pl.ctrl_max_obs = std::max(pl.ctrl_max_obs, q.obs);
      pl.ctrl_roll16 = pl.ctrl_roll16 && q.n_rollouts % 16 == 0;
      if (q.obs < 1 || q.obs > (uint32_t)mde::CT_MAX_OBS || q.act < 1 || q.act > (uint32_t)mde::CT_MAX_ACT) {
        msg = pk + "control workload needs 1 <= obs <= 20 and 1 <= act <= 8"; return METADE_EINVAL;
      }
      if (q.steps < 1 || q.n_rollouts < 1) { msg = pk + "steps and n_rollouts must be >= 1"; return METADE_EINVAL; }
      if (!q.A || !q.B || !q.x0) { msg = pk + "A, B and x0 are required"; return METADE_EINVAL; }
      if (!std::isfinite(q.ctrl_weight)) { msg = pk + "ctrl_weight must be finite"; return METADE_EINVAL; }
      const uint64_t Dm = (uint64_t)H * q.obs + H + (uint64_t)H * H + H + (uint64_t)H * q.act + q.act;
      if (q.D != Dm) {
        msg = pk + "D must equal the policy's weight count " + std::to_string(Dm); return METADE_EINVAL;
      }
      p.obs = q.obs;
      p.act = q.act;
      p.h1 = q.hidden1;
      p.h2 = q.hidden2;
      p.steps = q.steps;
      p.nroll = q.n_rollouts;
      p.cw = q.ctrl_weight;
      p.A_off = take((size_t)q.obs * q.obs * sizeof(float));
      p.B_off = take((size_t)q.obs * q.act * sizeof(float));
      p.x0_off = take((size_t)q.n_rollouts * q.obs * sizeof(float));
      pl.probs[k] = p;
      continue;
    }
    if (q.D == 0 || q.D > (uint32_t)mde::MAX_D) {
      msg = "problem " + std::to_string(k) + ": D must be in 1..128"; return METADE_EINVAL;
    }
    if (!q.o || !q.R) { msg = "problem " + std::to_string(k) + ": o and R are required"; return METADE_EINVAL; }
    if (q.kind == METADE_FN_HYBRID &&
        (!q.perm || (uint64_t)q.split[0] + q.split[1] + q.split[2] != q.D)) {
      msg = "problem " + std::to_string(k) + ": hybrid needs perm and split summing to D";
      return METADE_EINVAL;
    }
    (void)cond;
    // read-only table layout of this problem
    p.o_off = take((size_t)q.D * sizeof(float));
    // transposed float64 rotation [D][rt_stride]; the row-major float32 one
    // zero padded to whole 16-wide tiles, and R o, that the matrix-core kernel reads
    p.r64t_off = take((size_t)q.D * mde::rt_stride(q.D) * sizeof(double));
    p.r32_off = take((size_t)mde::r32_stride(q.D) * mde::r32_stride(q.D) * sizeof(float));
    p.ro64_off = take((size_t)mde::r32_stride(q.D) * sizeof(double));
    p.ew_off = take((size_t)q.D * sizeof(float));
    p.ew64_off = take((size_t)q.D * sizeof(double));
    p.ek_off = take((size_t)q.D * sizeof(uint32_t));
    pl.probs[k] = p;
  }
  pl.runs.resize(cfg->n_runs);
  for (uint32_t r = 0; r < cfg->n_runs; ++r) {
    RunDev &d = pl.runs[r];
    std::memset(&d, 0, sizeof(d));
    const uint32_t N = cfg->N[r];
    if (cfg->problem[r] >= cfg->n_problems) {
      msg = "run " + std::to_string(r) + ": problem index out of range"; return METADE_EINVAL;
    }
    const uint32_t D = pl.probs[cfg->problem[r]].D;
    if (pl.probs[cfg->problem[r]].kind == mde::FN_LQR_MLP) {
      if (N < 10 || N > (uint32_t)mde::CT_MAX_N) {
        msg = "run " + std::to_string(r) + ": N must be in 10..1024 for the control workload";
        return METADE_EINVAL;
      }
      d.N = N;
      d.D = D;
      d.Dp = round4(D);
      d.prob = cfg->problem[r];
      d.stream = cfg->stream_id[r];
      d.kp = std::max<uint32_t>(1, (N * 10 + 99) / 100);
      d.kern = 2;
      d.pop_off = pl.pop_floats;
      d.pend_off = pl.pend_floats;
      d.fit_off = (uint32_t)pl.fit_n;
      d.bx_off = (uint32_t)pl.bx_n;
      pl.pend_floats += (size_t)N * d.Dp;   // pending trial rows, 16-byte aligned
      pl.pop_floats += (size_t)N * D;
      pl.fit_n += N;
      pl.bx_n += D;
      pl.ctrl_list.push_back(r);
      pl.ctrl_max_n = std::max(pl.ctrl_max_n, N);
      d.F = 0.5f;
      d.CR = 0.9f;
      d.bl = d.br = mde::RAND;
      d.dn = 1;
      d.cs = mde::BIN;
      continue;
    }
    if (N < 10 || N > (uint32_t)mde::MAX_N) {
      msg = "run " + std::to_string(r) + ": N must be in 10..256 (9 distinct draws plus the target)";
      return METADE_EINVAL;
    }
    d.N = N;
    d.D = D;
    d.Dp = round4(D);
    d.prob = cfg->problem[r];
    d.stream = cfg->stream_id[r];
    d.kp = std::max<uint32_t>(1, (N * 10 + 99) / 100);
    // lanes per part: whole waves covering N; parts: as many as fit the
    // consumer lanes of the kernel the run goes to
    d.Np = ((N + 63u) / 64u) * 64u;
    const uint32_t L_lane = std::max<uint32_t>(1, std::min<uint32_t>(8, mde::GEN_CONSUMERS / d.Np));
    const uint32_t L_mf = std::max<uint32_t>(1, std::min<uint32_t>(8, mde::MF_CONSUMERS / d.Np));
    d.Dk = ((D + 31u) / 32u) * 32u;
    d.NCT = (D + 15u) / 16u;
    const bool rosen = pl.probs[d.prob].kind == mde::FN_ROSENBROCK;
    const uint32_t lane_bytes = mde::lds_layout(N, d.Dp, L_lane, d.Np, true).total;
    const uint32_t mf_bytes = mde::mfma_layout(N, d.Dp, d.Dk, L_mf, d.Np, d.NCT, rosen,
                                               cfg->precision == METADE_BF16_REFINE).total;
    if (cfg->precision == METADE_FP32 && lane_bytes <= mde::LDS_BUDGET) {
      d.kern = 0;
      d.t_lds = 1;
      d.L = L_lane;
      pl.lds_bytes = std::max(pl.lds_bytes, lane_bytes);
      pl.lane_list.push_back(r);
    } else if (mf_bytes <= mde::LDS_BUDGET) {
      d.kern = 1;
      d.t_lds = 0;
      d.L = L_mf;
      pl.mfma_lds_bytes = std::max(pl.mfma_lds_bytes, mf_bytes);
      pl.mfma_list.push_back(r);
    } else {
      msg = "run " + std::to_string(r) + ": population does not fit in LDS (N*D too large)";
      return METADE_EINVAL;
    }
    pl.init_lds_bytes = std::max(pl.init_lds_bytes, mde::init_lds_bytes(N, d.Dp, d.Np));
    d.pop_off = pl.pop_floats;
    d.pend_off = pl.pend_floats;
    d.fit_off = (uint32_t)pl.fit_n;
    d.bx_off = (uint32_t)pl.bx_n;
    // matrix-core runs: trial rows [N][Dk] float32 (both precisions; the bf16
    // mode splits them in registers), each run's rows 4 KB after the previous
    // run's end.  Without the skew the runs that share an XCD (every eighth
    // workgroup) start their rows at the same offset within the L2's set
    // period, and the sets they share overflow: at D = 100 the rotation's
    // re-reads of the rows then came from memory (7.8 GB per launch instead of
    // 37 MB) with no change in time.
    if (d.kern == 1) pl.pend_floats += (size_t)N * d.Dk + 1024;
    pl.pop_floats += (size_t)N * D;
    pl.fit_n += N;
    pl.bx_n += D;
    d.F = 0.5f;
    d.CR = 0.9f;
    d.bl = d.br = mde::RAND;
    d.dn = 1;
    d.cs = mde::BIN;
  }
  // one function kind for every lane-kernel run: the kernel of that kind
  for (size_t k = 0; k < pl.lane_list.size(); ++k) {
    const int kind = (int)pl.probs[pl.runs[pl.lane_list[k]].prob].kind;
    pl.lane_kind = k == 0 ? kind : (pl.lane_kind == kind ? kind : -1);
  }
  return METADE_OK;
}

LaunchArgs largs(metade_ctx *c) {
  LaunchArgs a;
  a.runs = c->runs_d;
  a.probs = c->probs_d;
  a.tab = c->tab;
  a.pop = c->pop;
  a.fit = c->fit;
  a.pending = c->pend_d;
  a.n_runs = c->n_runs;
  a.lds_bytes = c->lds_bytes;
  a.init_lds_bytes = c->init_lds_bytes;
  a.mfma_lds_bytes = c->mfma_lds_bytes;
  a.k0 = (uint32_t)(c->seed & 0xFFFFFFFFu);
  a.k1 = (uint32_t)(c->seed >> 32);
  a.mfma_rows = c->mfma_rows;
  a.lane_kind = c->lane_kind;
  a.stream = c->stream;
  return a;
}

mde::CtrlArgs cargs(metade_ctx *c) {
  return mde::CtrlArgs{c->ctrl_list_d, c->n_ctrl,  c->ctrl_max_n, c->ctrl_hidden, c->ctrl_lanes,
                       c->ctrl_mx,     c->order_d, c->cfu_d,      c->cacc_d};
}

// Capture n generations of the control runs (rank, trials, rollouts, commit,
// then the counter advance) on a private stream and instantiate the graph.
// Replays read the generation from the device counter, so one graph serves
// every starting generation.  The sequence holds kernels only.
metade_status capture_ctrl(metade_ctx *c, uint32_t n, hipGraphExec_t *out) {
  if (!c->cap_stream) HIP_TRY(c, hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking));
  mde::LaunchArgs a = largs(c);
  a.stream = c->cap_stream;
  HIP_TRY(c, hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeThreadLocal));
  const hipError_t e1 = mde::launch_ctrl_generations(a, cargs(c), c->gen_d, n, c->lb, c->ub,
                                                     mde::TraceArgs{nullptr, nullptr, nullptr});
  hipGraph_t gph = nullptr;
  const hipError_t e2 = hipStreamEndCapture(c->cap_stream, &gph);
  if (e1 != hipSuccess || e2 != hipSuccess) {
    if (gph) (void)hipGraphDestroy(gph);
    return fail(c, METADE_EDEVICE, std::string("capturing the control generations: ") +
                                       hipGetErrorString(e1 != hipSuccess ? e1 : e2));
  }
  hipGraphExec_t ex = nullptr;
  const hipError_t e3 = hipGraphInstantiate(&ex, gph, nullptr, nullptr, 0);
  (void)hipGraphDestroy(gph);
  if (e3 != hipSuccess)
    return fail(c, METADE_EDEVICE, std::string("hipGraphInstantiate: ") + hipGetErrorString(e3));
  if (c->graphs.size() >= 8) {  // a handful of sequence lengths is all a caller uses
    (void)hipGraphExecDestroy(c->graphs.front().second);
    c->graphs.erase(c->graphs.begin());
  }
  c->graphs.emplace_back(n, ex);
  *out = ex;
  return METADE_OK;
}

metade_status run_generations(metade_ctx *c, uint32_t n, mde::TraceArgs tr) {
  if (n == 0) return METADE_OK;
  EventPair ev{nullptr, nullptr};
  if (c->timing) {
    HIP_TRY(c, hipEventCreate(&ev.a));
    HIP_TRY(c, hipEventCreate(&ev.b));
    HIP_TRY(c, hipEventRecord(ev.a, c->stream));
  }
  HIP_TRY(c, mde::launch_generations(largs(c), c->lane_list_d, c->n_lane, c->gen, n, c->lb, c->ub, tr));
  HIP_TRY(c, mde::launch_generations_mfma(largs(c), c->mfma_list_d, c->n_mfma,
                                          c->precision == METADE_BF16_REFINE, c->gen, n, c->lb,
                                          c->ub, c->counters_d, tr));
  if (c->n_ctrl && c->graph && !tr.u) {
    hipGraphExec_t ex = nullptr;
    for (const auto &e : c->graphs)
      if (e.first == n) ex = e.second;
    if (!ex) {
      const metade_status st = capture_ctrl(c, n, &ex);
      if (st != METADE_OK) return st;
    }
    HIP_TRY(c, hipGraphLaunch(ex, c->stream));
  } else {
    HIP_TRY(c, mde::launch_ctrl_generations(largs(c), cargs(c), c->gen_d, n, c->lb, c->ub, tr));
  }
  if (c->timing) {
    HIP_TRY(c, hipEventRecord(ev.b, c->stream));
    c->events.push_back(ev);
  }
  c->gen += n;
  for (const RunDev &r : c->runs_h) c->trials += (uint64_t)r.N * n;
  return METADE_OK;
}

metade_status reinit(metade_ctx *c) {
  HIP_TRY(c, mde::launch_init(largs(c), (double)c->lb, (double)c->ub));
  HIP_TRY(c, mde::launch_ctrl_init(largs(c), cargs(c), (double)c->lb, (double)c->ub));
  c->gen = 0;
  if (c->n_ctrl) HIP_TRY(c, mde::launch_ctrl_set_gen(c->gen_d, 0, c->stream));
  return METADE_OK;
}

metade_status finalize(metade_ctx *c) {
  HIP_TRY(c, mde::launch_finalize(largs(c), c->best_y, c->best_x));
  HIP_TRY(c, mde::launch_ctrl_finalize(largs(c), cargs(c), c->best_y, c->best_x));
  return METADE_OK;
}

template <typename T>
metade_status dalloc(metade_ctx *c, T **p, size_t n) {
  if (n == 0) { *p = nullptr; return METADE_OK; }
  hipError_t e = hipMalloc((void **)p, n * sizeof(T));
  if (e != hipSuccess) return fail(c, METADE_ENOMEM, std::string("hipMalloc: ") + hipGetErrorString(e));
  return METADE_OK;
}

#define TRY(expr)                       \
  do {                                  \
    metade_status s_ = (expr);          \
    if (s_ != METADE_OK) return s_;     \
  } while (0)

}  // namespace

extern "C" {

metade_status metade_query_sizes(const metade_config *cfg, size_t *pop_bytes, size_t *fit_bytes,
                                 size_t *best_y_bytes, size_t *best_x_bytes,
                                 size_t *scratch_bytes) {
  Plan pl;
  std::string msg;
  metade_status s = plan_config(cfg, pl, msg);
  if (s != METADE_OK) return fail(nullptr, s, msg);
  if (pop_bytes) *pop_bytes = pl.pop_floats * sizeof(float);
  if (fit_bytes) *fit_bytes = pl.fit_n * sizeof(float);
  if (best_y_bytes) *best_y_bytes = (size_t)cfg->n_runs * sizeof(double);
  if (best_x_bytes) *best_x_bytes = pl.bx_n * sizeof(float);
  if (scratch_bytes)
    *scratch_bytes = pl.runs.size() * sizeof(RunDev) + pl.probs.size() * sizeof(ProbDev) +
                     pl.pend_floats * sizeof(float) + (size_t)cfg->n_runs * (6 * 4 * 3 + 16) +
                     pl.bx_n * sizeof(float) + 16;
  if (scratch_bytes) *scratch_bytes += pl.tab_bytes;
  if (scratch_bytes && !pl.ctrl_list.empty())
    *scratch_bytes += pl.fit_n * 12 + pl.ctrl_list.size() * 4;
  return METADE_OK;
}

metade_status metade_init(const metade_config *cfg, metade_ctx **out) {
  if (!out) return fail(nullptr, METADE_EINVAL, "out is NULL");
  *out = nullptr;
  Plan pl;
  std::string msg;
  metade_status s = plan_config(cfg, pl, msg);
  if (s != METADE_OK) return fail(nullptr, s, msg);
  if (!cfg->pop || !cfg->fit || !cfg->best_y || !cfg->best_x)
    return fail(nullptr, METADE_EINVAL, "pop, fit, best_y and best_x device buffers are required");
  metade_ctx *c = new metade_ctx();
  c->stream = (hipStream_t)cfg->stream;
  c->n_runs = cfg->n_runs;
  c->n_cs = cfg->n_cs;
  c->precision = cfg->precision;
  c->evolver = cfg->evolver;
  c->graph = cfg->graph != 0;
  c->seed = cfg->seed;
  c->lb = cfg->lb;
  c->ub = cfg->ub;
  c->pop = cfg->pop;
  c->fit = cfg->fit;
  c->best_y = cfg->best_y;
  c->best_x = cfg->best_x;
  c->runs_h = pl.runs;
  c->probs_h = pl.probs;
  c->pop_floats = pl.pop_floats;
  c->fit_n = pl.fit_n;
  c->bx_n = pl.bx_n;
  c->pend_floats = pl.pend_floats;
  c->lds_bytes = pl.lds_bytes;
  c->lane_kind = pl.lane_kind;
  c->init_lds_bytes = pl.init_lds_bytes;
  c->mfma_lds_bytes = pl.mfma_lds_bytes;
  c->n_lane = (uint32_t)pl.lane_list.size();
  c->n_mfma = (uint32_t)pl.mfma_list.size();
  c->n_ctrl = (uint32_t)pl.ctrl_list.size();
  c->ctrl_max_n = pl.ctrl_max_n;
  c->ctrl_hidden = pl.ctrl_hidden;
  // width-32 policies with few observations: 16 lanes each, four per wavefront
  c->ctrl_lanes = (pl.ctrl_hidden == (uint32_t)mde::CT_H_SMALL &&
                   pl.ctrl_max_obs <= (uint32_t)mde::CT_OBS_L16) ? 16u : 32u;
  // 16 rollouts per policy or a multiple: one policy per wavefront on the matrix cores
  c->ctrl_mx = (pl.ctrl_hidden != 0 && pl.ctrl_roll16) ? 1u : 0u;
  auto bail = [&](metade_status st) {
    g_init_error = c->err;
    metade_destroy(c);
    return st;
  };
  metade_status st;
  {
    // the static workspace's address on this device (the current one)
    hipError_t e0 = hipGetDevice(&c->device);
    if (e0 == hipSuccess && (c->device < 0 || c->device >= MAX_DEVICES)) e0 = hipErrorInvalidDevice;
    if (e0 == hipSuccess) {
      std::lock_guard<std::mutex> lk(g_scratch_mu);
      if (!g_scratch_dev[c->device]) {
        void *ptr = nullptr;
        e0 = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e0 == hipSuccess) g_scratch_dev[c->device] = static_cast<float *>(ptr);
      }
      c->scratch_d = g_scratch_dev[c->device];
    }
    if (e0 != hipSuccess) {
      c->err = std::string("static workspace address: ") + hipGetErrorString(e0);
      return bail(METADE_EDEVICE);
    }
  }
  std::vector<std::vector<uint32_t>> perms(c->probs_h.size());
  for (size_t k = 0; k < c->probs_h.size(); ++k) {
    const metade_problem &q = cfg->problems[k];
    if (q.kind != METADE_FN_HYBRID) continue;
    // the element tables are built from the permutation: it must be one
    std::vector<uint32_t> &perm = perms[k];
    perm.resize(q.D);
    hipError_t e = hipMemcpy(perm.data(), q.perm, q.D * sizeof(uint32_t), hipMemcpyDeviceToHost);
    if (e != hipSuccess) { c->err = std::string("reading hybrid permutation: ") + hipGetErrorString(e); return bail(METADE_EDEVICE); }
    std::vector<char> seen(q.D, 0);
    for (uint32_t v : perm) {
      if (v >= q.D || seen[v]) { c->err = "problem " + std::to_string(k) + ": perm is not a permutation of 0..D-1"; return bail(METADE_EINVAL); }
      seen[v] = 1;
    }
  }
  if ((st = dalloc(c, &c->tab, pl.tab_bytes)) != METADE_OK) return bail(st);
  if ((st = dalloc(c, &c->runs_d, c->n_runs)) != METADE_OK) return bail(st);
  if ((st = dalloc(c, &c->probs_d, c->probs_h.size())) != METADE_OK) return bail(st);
  if ((st = dalloc(c, &c->theta_d, (size_t)c->n_runs * 6)) != METADE_OK) return bail(st);
  if ((st = dalloc(c, &c->pend_d, c->pend_floats)) != METADE_OK) return bail(st);
  if ((st = dalloc(c, &c->Xo, (size_t)c->n_runs * 6)) != METADE_OK) return bail(st);
  if ((st = dalloc(c, &c->Uo, (size_t)c->n_runs * 6)) != METADE_OK) return bail(st);
  if ((st = dalloc(c, &c->Vo, (size_t)c->n_runs * 6)) != METADE_OK) return bail(st);
  if ((st = dalloc(c, &c->yo, c->n_runs)) != METADE_OK) return bail(st);
  if ((st = dalloc(c, &c->yt, c->n_runs)) != METADE_OK) return bail(st);
  if ((st = dalloc(c, &c->bxo, c->bx_n)) != METADE_OK) return bail(st);
  if ((st = dalloc(c, &c->bidx, 4)) != METADE_OK) return bail(st);
  if ((st = dalloc(c, &c->counters_d, N_COUNTERS)) != METADE_OK) return bail(st);
  if ((st = dalloc(c, &c->gen_d, 1)) != METADE_OK) return bail(st);
  if ((st = dalloc(c, &c->lane_list_d, pl.lane_list.size())) != METADE_OK) return bail(st);
  if ((st = dalloc(c, &c->mfma_list_d, pl.mfma_list.size())) != METADE_OK) return bail(st);
  if ((st = dalloc(c, &c->ctrl_list_d, pl.ctrl_list.size())) != METADE_OK) return bail(st);
  if (c->n_ctrl) {
    if ((st = dalloc(c, &c->order_d, c->fit_n)) != METADE_OK) return bail(st);
    if ((st = dalloc(c, &c->cfu_d, c->fit_n)) != METADE_OK) return bail(st);
    if ((st = dalloc(c, &c->cacc_d, c->fit_n)) != METADE_OK) return bail(st);
  }
  {
    hipError_t e5 = hipMemset(c->counters_d, 0, N_COUNTERS * sizeof(unsigned long long));
    if (e5 == hipSuccess && !pl.lane_list.empty())
      e5 = hipMemcpy(c->lane_list_d, pl.lane_list.data(), pl.lane_list.size() * 4, hipMemcpyHostToDevice);
    if (e5 == hipSuccess && !pl.mfma_list.empty())
      e5 = hipMemcpy(c->mfma_list_d, pl.mfma_list.data(), pl.mfma_list.size() * 4, hipMemcpyHostToDevice);
    if (e5 == hipSuccess && !pl.ctrl_list.empty())
      e5 = hipMemcpy(c->ctrl_list_d, pl.ctrl_list.data(), pl.ctrl_list.size() * 4, hipMemcpyHostToDevice);
    if (e5 != hipSuccess) { c->err = std::string("run lists: ") + hipGetErrorString(e5); return bail(METADE_EDEVICE); }
  }
  for (size_t k = 0; k < c->probs_h.size(); ++k) {
    // per-output element tables: elliptic weights cond^(idx/(n-1)) and, for
    // the hybrid, the block each rotated output falls in after permutation
    const ProbDev &p = c->probs_h[k];
    const metade_problem &q = cfg->problems[k];
    if (p.kind == mde::FN_LQR_MLP) {
      // plant and initial states, copied so that the context does not depend on them
      unsigned char *t = c->tab;
      hipError_t e6 = hipMemcpy(t + p.A_off, q.A, (size_t)p.obs * p.obs * sizeof(float), hipMemcpyDeviceToDevice);
      if (e6 == hipSuccess) e6 = hipMemcpy(t + p.B_off, q.B, (size_t)p.obs * p.act * sizeof(float), hipMemcpyDeviceToDevice);
      if (e6 == hipSuccess) e6 = hipMemcpy(t + p.x0_off, q.x0, (size_t)p.nroll * p.obs * sizeof(float), hipMemcpyDeviceToDevice);
      if (e6 != hipSuccess) { c->err = std::string("control tables: ") + hipGetErrorString(e6); return bail(METADE_EDEVICE); }
      continue;
    }
    const double cond = q.cond > 0 ? (double)q.cond : 1e6;
    std::vector<float> ew(p.D, 0.0f);
    std::vector<double> ew64(p.D, 0.0);
    std::vector<uint32_t> ek(p.D, 0);
    if (p.kind == mde::FN_ELLIPTIC) {
      for (uint32_t j = 0; j < p.D; ++j) {
        ew64[j] = p.D > 1 ? std::pow(cond, (double)j / (double)(p.D - 1)) : 1.0;
        ew[j] = (float)ew64[j];
      }
    } else if (p.kind == mde::FN_HYBRID) {
      const uint32_t n1 = q.split[0], n2 = q.split[1], n3 = q.split[2];
      for (uint32_t pos = 0; pos < p.D; ++pos) {
        const uint32_t j = perms[k][pos];
        if (pos < n1) {
          ek[j] = 0;
        } else if (pos < n1 + n2) {
          ek[j] = 1;
        } else {
          ek[j] = 2;
          const uint32_t idx = pos - n1 - n2;
          ew64[j] = n3 > 1 ? std::pow(cond, (double)idx / (double)(n3 - 1)) : 1.0;
          ew[j] = (float)ew64[j];
        }
      }
    }
    unsigned char *t = c->tab;
    hipError_t e4 = hipMemcpy(t + p.ew_off, ew.data(), p.D * sizeof(float), hipMemcpyHostToDevice);
    if (e4 == hipSuccess) e4 = hipMemcpy(t + p.ew64_off, ew64.data(), p.D * sizeof(double), hipMemcpyHostToDevice);
    if (e4 == hipSuccess) e4 = hipMemcpy(t + p.ek_off, ek.data(), p.D * sizeof(uint32_t), hipMemcpyHostToDevice);
    if (e4 == hipSuccess) e4 = hipMemcpy(t + p.o_off, q.o, p.D * sizeof(float), hipMemcpyDeviceToDevice);
    if (e4 == hipSuccess)
      e4 = mde::launch_tables64(q.R, reinterpret_cast<double *>(t + p.r64t_off), p.D, c->stream);
    if (e4 == hipSuccess)
      e4 = mde::launch_tables_mfma(q.R, q.o, reinterpret_cast<float *>(t + p.r32_off),
                                   reinterpret_cast<double *>(t + p.ro64_off), p.D, c->stream);
    if (e4 != hipSuccess) { c->err = std::string("problem tables: ") + hipGetErrorString(e4); return bail(METADE_EDEVICE); }
  }
  hipError_t e = mde::set_lds_limits();
  if (e != hipSuccess) { c->err = std::string("set_lds_limits: ") + hipGetErrorString(e); return bail(METADE_EDEVICE); }
  e = hipMemcpyAsync(c->runs_d, c->runs_h.data(), c->n_runs * sizeof(RunDev), hipMemcpyHostToDevice, c->stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(c->probs_d, c->probs_h.data(), c->probs_h.size() * sizeof(ProbDev), hipMemcpyHostToDevice, c->stream);
  if (e != hipSuccess) { c->err = std::string("table upload: ") + hipGetErrorString(e); return bail(METADE_EDEVICE); }
  std::vector<float> th((size_t)c->n_runs * 6);
  for (uint32_t r = 0; r < c->n_runs; ++r) {
    const float d[6] = {0.5f, 0.9f, 1.0f, 1.0f, 1.0f, 1.0f};
    std::memcpy(&th[(size_t)r * 6], d, sizeof(d));
  }
  e = hipMemcpyAsync(c->theta_d, th.data(), th.size() * sizeof(float), hipMemcpyHostToDevice, c->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  if (e != hipSuccess) { c->err = std::string("theta upload: ") + hipGetErrorString(e); return bail(METADE_EDEVICE); }
  if ((st = reinit(c)) != METADE_OK) return bail(st);
  if ((st = finalize(c)) != METADE_OK) return bail(st);
  *out = c;
  return METADE_OK;
}

metade_status metade_reset(metade_ctx *c) {
  if (!c) return fail(nullptr, METADE_EINVAL, "ctx is NULL");
  TRY(reinit(c));
  return finalize(c);
}

metade_status metade_set_theta(metade_ctx *c, const float *theta) {
  if (!c || !theta) return fail(c, METADE_EINVAL, "ctx and theta are required");
  HIP_TRY(c, hipMemcpyAsync(c->theta_d, theta, (size_t)c->n_runs * 6 * sizeof(float),
                            hipMemcpyHostToDevice, c->stream));
  HIP_TRY(c, mde::launch_decode(c->runs_d, c->theta_d, c->n_runs, c->n_cs, c->stream));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  return METADE_OK;
}

metade_status metade_inner_step(metade_ctx *c, uint32_t n) {
  if (!c) return fail(nullptr, METADE_EINVAL, "ctx is NULL");
  TRY(run_generations(c, n, mde::TraceArgs{nullptr, nullptr, nullptr}));
  return finalize(c);
}

metade_status metade_inner_step_static(metade_ctx *c, uint32_t n) {
  if (!c) return fail(nullptr, METADE_EINVAL, "ctx is NULL");
  if (c->n_ctrl)
    return fail(c, METADE_EINVAL,
                "metade_inner_step_static takes no control runs (their pending rows exceed the "
                "static workspace)");
  const size_t need = c->pend_floats * sizeof(float);
  if (need > (size_t)METADE_STATIC_SCRATCH_BYTES)
    return fail(c, METADE_EINVAL,
                "the runs' trial rows need " + std::to_string(need) +
                    " bytes, more than the static workspace's " +
                    std::to_string((size_t)METADE_STATIC_SCRATCH_BYTES));
  int dev = -1;
  HIP_TRY(c, hipGetDevice(&dev));
  if (dev != c->device)
    return fail(c, METADE_EINVAL, "call metade_inner_step_static with the context's device current");
  if (!c->scratch_d) return fail(c, METADE_EDEVICE, "static workspace address unknown");
  if (n) {
    // the same kernels as metade_inner_step, with the trial rows in the
    // static workspace; no events, no graphs, no allocation
    LaunchArgs a = largs(c);
    a.pending = c->scratch_d;
    const mde::TraceArgs none{nullptr, nullptr, nullptr};
    HIP_TRY(c, mde::launch_generations(a, c->lane_list_d, c->n_lane, c->gen, n, c->lb, c->ub, none));
    HIP_TRY(c, mde::launch_generations_mfma(a, c->mfma_list_d, c->n_mfma,
                                            c->precision == METADE_BF16_REFINE, c->gen, n, c->lb,
                                            c->ub, c->counters_d, none));
    c->gen += n;
    for (const RunDev &r : c->runs_h) c->trials += (uint64_t)r.N * n;
  }
  return finalize(c);
}

metade_status metade_trace_sizes(metade_ctx *c, size_t *u_bytes, size_t *fu_bytes,
                                 size_t *desc_bytes) {
  if (!c) return fail(nullptr, METADE_EINVAL, "ctx is NULL");
  if (u_bytes) *u_bytes = c->pop_floats * sizeof(float);
  if (fu_bytes) *fu_bytes = c->fit_n * sizeof(float);
  if (desc_bytes) *desc_bytes = c->fit_n * 16 * sizeof(int32_t);
  return METADE_OK;
}

metade_status metade_inner_step_trace(metade_ctx *c, float *u, float *fu, int32_t *desc) {
  if (!c || !u || !fu || !desc) return fail(c, METADE_EINVAL, "ctx and all trace buffers are required");
  TRY(run_generations(c, 1, mde::TraceArgs{u, fu, desc}));
  return finalize(c);
}

metade_status metade_outer_reset(metade_ctx *c) {
  if (!c) return fail(nullptr, METADE_EINVAL, "ctx is NULL");
  if (c->n_runs < 4) return fail(c, METADE_EINVAL, "the evolver needs at least 4 individuals");
  HIP_TRY(c, mde::launch_outer_init(c->Xo, c->yo, c->n_runs, c->runs_h[0].stream,
                                    (uint32_t)(c->seed & 0xFFFFFFFFu), (uint32_t)(c->seed >> 32),
                                    c->n_cs, c->stream));
  HIP_TRY(c, hipMemsetAsync(c->bxo, 0, c->bx_n * sizeof(float), c->stream));
  if (c->evolver == METADE_EVOLVER_PSO || c->evolver == METADE_EVOLVER_CSO) {
    // particles start at the initial population, at rest
    HIP_TRY(c, hipMemcpyAsync(c->Uo, c->Xo, (size_t)c->n_runs * 6 * sizeof(float),
                              hipMemcpyDeviceToDevice, c->stream));
    HIP_TRY(c, hipMemsetAsync(c->Vo, 0, (size_t)c->n_runs * 6 * sizeof(float), c->stream));
  }
  if (c->evolver == METADE_EVOLVER_NES) HIP_TRY(c, mde::launch_nes_init(c->Vo, c->n_cs, c->stream));
  c->outer_gen = 0;
  c->outer_ready = true;
  return METADE_OK;
}

metade_status metade_outer_step(metade_ctx *c, uint32_t G_inner, uint32_t power_up) {
  if (!c) return fail(nullptr, METADE_EINVAL, "ctx is NULL");
  if (!c->outer_ready) return fail(c, METADE_ESTATE, "metade_outer_reset must come first");
  if (power_up > 1 && G_inner > UINT32_MAX / power_up)
    return fail(c, METADE_EINVAL, "G_inner * power_up exceeds 2^32 - 1");
  const uint32_t G = G_inner * (power_up > 1 ? power_up : 1);
  const uint32_t k0 = (uint32_t)(c->seed & 0xFFFFFFFFu), k1 = (uint32_t)(c->seed >> 32);
  if (c->evolver == METADE_EVOLVER_PSO) {
    if (c->outer_gen == 0) {
      HIP_TRY(c, mde::launch_decode(c->runs_d, c->Uo, c->n_runs, c->n_cs, c->stream));
    } else {
      HIP_TRY(c, mde::launch_outer_best(c->yo, c->n_runs, c->bidx, c->stream));
      HIP_TRY(c, mde::launch_pso_move(c->Uo, c->Vo, c->Xo, c->bidx, c->runs_d, c->n_runs,
                                      c->outer_gen, c->runs_h[0].stream, k0, k1, c->n_cs,
                                      c->stream));
    }
  } else if (c->evolver == METADE_EVOLVER_NES) {
    HIP_TRY(c, mde::launch_nes_sample(c->Uo, c->Vo, c->runs_d, c->n_runs, c->outer_gen,
                                      c->runs_h[0].stream, k0, k1, c->n_cs, c->stream));
  } else if (c->evolver == METADE_EVOLVER_CSO) {
    if (c->outer_gen == 0) {
      HIP_TRY(c, mde::launch_decode(c->runs_d, c->Uo, c->n_runs, c->n_cs, c->stream));
    } else {
      HIP_TRY(c, mde::launch_cso_move(c->Xo, c->Vo, c->Uo, c->yo, c->runs_d, c->n_runs,
                                      c->outer_gen, c->runs_h[0].stream, k0, k1, c->n_cs,
                                      c->stream));
    }
  } else {
    HIP_TRY(c, mde::launch_outer_trial(c->Xo, c->Uo, c->runs_d, c->n_runs, c->outer_gen,
                                       c->runs_h[0].stream, k0, k1, c->n_cs, c->stream));
  }
  TRY(reinit(c));
  TRY(run_generations(c, G, mde::TraceArgs{nullptr, nullptr, nullptr}));
  TRY(finalize(c));
  HIP_TRY(c, mde::launch_outer_select(c->Xo, c->yo, c->Uo, c->best_y, c->yt, c->bxo, c->best_x,
                                      c->runs_d, c->n_runs,
                                      c->evolver == METADE_EVOLVER_CSO ||
                                          c->evolver == METADE_EVOLVER_NES,
                                      c->stream));
  if (c->evolver == METADE_EVOLVER_NES) {
    const double eta_sigma = (3.0 + std::log(6.0)) / (5.0 * std::sqrt(6.0));
    HIP_TRY(c, mde::launch_nes_update(c->yt, c->Vo, c->n_runs, c->outer_gen, c->runs_h[0].stream,
                                      k0, k1, eta_sigma, c->stream));
  }
  ++c->outer_gen;
  return METADE_OK;
}

metade_status metade_get_outer(metade_ctx *c, float *X, double *y, float *U, double *y_trial) {
  if (!c) return fail(nullptr, METADE_EINVAL, "ctx is NULL");
  if (!c->outer_ready) return fail(c, METADE_ESTATE, "evolver not initialised");
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  const size_t n6 = (size_t)c->n_runs * 6;
  if (X) HIP_TRY(c, hipMemcpy(X, c->Xo, n6 * sizeof(float), hipMemcpyDeviceToHost));
  if (y) HIP_TRY(c, hipMemcpy(y, c->yo, c->n_runs * sizeof(double), hipMemcpyDeviceToHost));
  if (U) HIP_TRY(c, hipMemcpy(U, c->Uo, n6 * sizeof(float), hipMemcpyDeviceToHost));
  if (y_trial) HIP_TRY(c, hipMemcpy(y_trial, c->yt, c->n_runs * sizeof(double), hipMemcpyDeviceToHost));
  return METADE_OK;
}

metade_status metade_set_outer(metade_ctx *c, const float *X, const double *y, uint32_t gen) {
  if (!c || !X || !y) return fail(c, METADE_EINVAL, "ctx, X and y are required");
  if (c->evolver != METADE_EVOLVER_DE && !c->outer_ready)
    return fail(c, METADE_ESTATE,
                "metade_outer_reset must come first for this evolver: its positions, "
                "velocities or search distribution are not part of X and y");
  HIP_TRY(c, hipMemcpyAsync(c->Xo, X, (size_t)c->n_runs * 6 * sizeof(float), hipMemcpyHostToDevice, c->stream));
  HIP_TRY(c, hipMemcpyAsync(c->yo, y, c->n_runs * sizeof(double), hipMemcpyHostToDevice, c->stream));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  c->outer_gen = gen;
  c->outer_ready = true;
  return METADE_OK;
}

metade_status metade_run(metade_ctx *c, uint32_t outer_gens, uint32_t G_inner, uint32_t power_up,
                         double *best_y, float *best_theta, float *best_x) {
  if (!c) return fail(nullptr, METADE_EINVAL, "ctx is NULL");
  if (outer_gens == 0) return fail(c, METADE_EINVAL, "outer_gens must be >= 1");
  TRY(metade_outer_reset(c));
  for (uint32_t g = 0; g < outer_gens; ++g)
    TRY(metade_outer_step(c, G_inner, g + 1 == outer_gens ? power_up : 1));
  HIP_TRY(c, mde::launch_outer_best(c->yo, c->n_runs, c->bidx, c->stream));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  int32_t b = 0;
  HIP_TRY(c, hipMemcpy(&b, c->bidx, sizeof(b), hipMemcpyDeviceToHost));
  if (best_y) HIP_TRY(c, hipMemcpy(best_y, c->yo + b, sizeof(double), hipMemcpyDeviceToHost));
  if (best_theta) HIP_TRY(c, hipMemcpy(best_theta, c->Xo + (size_t)b * 6, 6 * sizeof(float), hipMemcpyDeviceToHost));
  if (best_x)
    HIP_TRY(c, hipMemcpy(best_x, c->bxo + c->runs_h[b].bx_off, c->runs_h[b].D * sizeof(float),
                         hipMemcpyDeviceToHost));
  return METADE_OK;
}

metade_status metade_get_best(metade_ctx *c, double *y) {
  if (!c || !y) return fail(c, METADE_EINVAL, "ctx and y are required");
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  HIP_TRY(c, hipMemcpy(y, c->best_y, c->n_runs * sizeof(double), hipMemcpyDeviceToHost));
  return METADE_OK;
}

namespace {
constexpr uint32_t STATE_MAGIC = 0x3245444Du;  // "MDE2"
struct StateHeader {
  uint32_t magic, n_runs, gen, outer_gen, outer_ready, n_cs;
  uint64_t pop_floats, fit_n, bx_n;
};
// The decoded theta of a run: the only part of the run table a checkpoint
// carries.  Sizes, offsets and the kernel choice always come from the context
// the blob is restored into (they depend on its precision), so a blob taken
// from a context of another precision restores safely.
struct RunTheta {
  float F, CR;
  int32_t bl, br, dn, cs;
};
}  // namespace

metade_status metade_get_state(metade_ctx *c, void *blob, size_t *bytes) {
  if (!c || !bytes) return fail(c, METADE_EINVAL, "ctx and bytes are required");
  const size_t n = c->n_runs;
  const size_t need = sizeof(StateHeader) + c->pop_floats * 4 + c->fit_n * 4 + n * 6 * 4 +
                      n * sizeof(RunTheta) + n * 8 + c->bx_n * 4 + n * 6 * 4 * 3 + n * 8 * 2 +
                      c->bx_n * 4;
  if (!blob) { *bytes = need; return METADE_OK; }
  if (*bytes < need) return fail(c, METADE_EINVAL, "state buffer too small");
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  unsigned char *p = (unsigned char *)blob;
  StateHeader h{STATE_MAGIC, c->n_runs, c->gen, c->outer_gen, c->outer_ready ? 1u : 0u, c->n_cs,
                c->pop_floats, c->fit_n, c->bx_n};
  std::vector<RunDev> runs(n);
  HIP_TRY(c, hipMemcpy(runs.data(), c->runs_d, n * sizeof(RunDev), hipMemcpyDeviceToHost));
  std::vector<RunTheta> th(n);
  for (size_t r = 0; r < n; ++r)
    th[r] = RunTheta{runs[r].F, runs[r].CR, runs[r].bl, runs[r].br, runs[r].dn, runs[r].cs};
  std::memcpy(p, &h, sizeof(h));
  p += sizeof(h);
  auto d2h = [&](const void *src, size_t nb) -> hipError_t {
    hipError_t e = nb ? hipMemcpy(p, src, nb, hipMemcpyDeviceToHost) : hipSuccess;
    p += nb;
    return e;
  };
  HIP_TRY(c, d2h(c->pop, c->pop_floats * 4));
  HIP_TRY(c, d2h(c->fit, c->fit_n * 4));
  HIP_TRY(c, d2h(c->theta_d, n * 6 * 4));
  std::memcpy(p, th.data(), n * sizeof(RunTheta));
  p += n * sizeof(RunTheta);
  HIP_TRY(c, d2h(c->best_y, n * 8));
  HIP_TRY(c, d2h(c->best_x, c->bx_n * 4));
  HIP_TRY(c, d2h(c->Xo, n * 6 * 4));
  HIP_TRY(c, d2h(c->Uo, n * 6 * 4));
  HIP_TRY(c, d2h(c->Vo, n * 6 * 4));
  HIP_TRY(c, d2h(c->yo, n * 8));
  HIP_TRY(c, d2h(c->yt, n * 8));
  HIP_TRY(c, d2h(c->bxo, c->bx_n * 4));
  *bytes = need;
  return METADE_OK;
}

metade_status metade_set_state(metade_ctx *c, const void *blob, size_t bytes) {
  if (!c || !blob) return fail(c, METADE_EINVAL, "ctx and blob are required");
  size_t need = 0;
  TRY(metade_get_state(c, nullptr, &need));
  if (bytes != need) return fail(c, METADE_EINVAL, "state size does not match this context");
  const unsigned char *p = (const unsigned char *)blob;
  StateHeader h;
  std::memcpy(&h, p, sizeof(h));
  if (h.magic != STATE_MAGIC || h.n_runs != c->n_runs || h.pop_floats != c->pop_floats ||
      h.fit_n != c->fit_n || h.bx_n != c->bx_n || h.n_cs != c->n_cs)
    return fail(c, METADE_EINVAL, "state blob does not belong to this configuration");
  p += sizeof(h);
  const size_t n = c->n_runs;
  // only the decoded theta comes from the blob; the run layout (offsets, the
  // kernel choice and the trial-row area, which depend on the precision) is
  // this context's own
  std::vector<RunTheta> th(n);
  std::memcpy(th.data(), p + c->pop_floats * 4 + c->fit_n * 4 + n * 6 * 4, n * sizeof(RunTheta));
  std::vector<RunDev> runs = c->runs_h;
  for (size_t r = 0; r < n; ++r) {
    const RunTheta &t = th[r];
    const bool cat_ok = t.bl >= 1 && t.bl <= 4 && t.br >= 1 && t.br <= 4 && t.dn >= 1 &&
                        t.dn <= 4 && t.cs >= 1 && t.cs <= (int32_t)c->n_cs;
    if (!cat_ok || !(t.F >= 0.0f && t.F <= 1.0f) || !(t.CR >= 0.0f && t.CR <= 1.0f))
      return fail(c, METADE_EINVAL, "state blob holds a theta outside the decoded domain");
    runs[r].F = t.F;
    runs[r].CR = t.CR;
    runs[r].bl = t.bl;
    runs[r].br = t.br;
    runs[r].dn = t.dn;
    runs[r].cs = t.cs;
  }
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  auto h2d = [&](void *dst, size_t nb) -> hipError_t {
    hipError_t e = nb ? hipMemcpy(dst, p, nb, hipMemcpyHostToDevice) : hipSuccess;
    p += nb;
    return e;
  };
  HIP_TRY(c, h2d(c->pop, c->pop_floats * 4));
  HIP_TRY(c, h2d(c->fit, c->fit_n * 4));
  HIP_TRY(c, h2d(c->theta_d, n * 6 * 4));
  HIP_TRY(c, hipMemcpy(c->runs_d, runs.data(), n * sizeof(RunDev), hipMemcpyHostToDevice));
  p += n * sizeof(RunTheta);
  HIP_TRY(c, h2d(c->best_y, n * 8));
  HIP_TRY(c, h2d(c->best_x, c->bx_n * 4));
  HIP_TRY(c, h2d(c->Xo, n * 6 * 4));
  HIP_TRY(c, h2d(c->Uo, n * 6 * 4));
  HIP_TRY(c, h2d(c->Vo, n * 6 * 4));
  HIP_TRY(c, h2d(c->yo, n * 8));
  HIP_TRY(c, h2d(c->yt, n * 8));
  HIP_TRY(c, h2d(c->bxo, c->bx_n * 4));
  c->gen = h.gen;
  if (c->n_ctrl) HIP_TRY(c, mde::launch_ctrl_set_gen(c->gen_d, c->gen, c->stream));
  c->outer_gen = h.outer_gen;
  c->outer_ready = h.outer_ready != 0;
  return METADE_OK;
}

metade_status metade_kernel_timing(metade_ctx *c, int enable) {
  if (!c) return fail(nullptr, METADE_EINVAL, "ctx is NULL");
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  for (EventPair &ev : c->events) {
    (void)hipEventDestroy(ev.a);
    (void)hipEventDestroy(ev.b);
  }
  c->events.clear();
  c->timing = enable != 0;
  return METADE_OK;
}

metade_status metade_kernel_time(metade_ctx *c, double *ms, uint64_t *launches) {
  if (!c) return fail(nullptr, METADE_EINVAL, "ctx is NULL");
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  double total = 0.0;
  for (EventPair &ev : c->events) {
    float t = 0.0f;
    HIP_TRY(c, hipEventElapsedTime(&t, ev.a, ev.b));
    total += t;
  }
  if (ms) *ms = total;
  if (launches) *launches = c->events.size();
  return METADE_OK;
}

metade_status metade_get_counters(metade_ctx *c, uint64_t *trials, uint64_t *refined) {
  if (!c) return fail(nullptr, METADE_EINVAL, "ctx is NULL");
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  if (trials) *trials = c->trials;
  if (refined) {
    unsigned long long r = 0;
    HIP_TRY(c, hipMemcpy(&r, c->counters_d, sizeof(r), hipMemcpyDeviceToHost));
    *refined = r;
  }
  return METADE_OK;
}

metade_status metade_get_bound_check(metade_ctx *c, uint64_t *checked, uint64_t *outside,
                                     uint64_t *screened, uint64_t *screen_wrong,
                                     double *max_ratio) {
  if (!c) return fail(nullptr, METADE_EINVAL, "ctx is NULL");
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  unsigned long long v[N_COUNTERS];
  HIP_TRY(c, hipMemcpy(v, c->counters_d, sizeof(v), hipMemcpyDeviceToHost));
  if (checked) *checked = v[1];
  if (outside) *outside = v[2];
  if (screened) *screened = v[3];
  if (screen_wrong) *screen_wrong = v[4];
  if (max_ratio) {
    double r;
    std::memcpy(&r, &v[5], sizeof(r));
    *max_ratio = r;
  }
  return METADE_OK;
}

#ifdef MDE_STAGE_CLOCKS
// Diagnostic builds only: per-(block, wave, stage) cycle totals of the last
// launch of the lane kernel (which = 0) or the matrix-core kernel (which = 1).
int metade_debug_stage_clocks(int which, void *dst, size_t bytes) {
  const hipError_t e = which ? mde::read_stage_clocks_mfma(dst, bytes)
                             : mde::read_stage_clocks(dst, bytes);
  return e == hipSuccess ? 0 : -1;
}
#endif

metade_status metade_get_tuning(metade_ctx *c, metade_tuning *t) {
  if (!c || !t) return fail(c, METADE_EINVAL, "ctx and t are required");
  t->lane_parts = c->lane_parts;
  t->mfma_rows = c->mfma_rows;
  return METADE_OK;
}

metade_status metade_set_tuning(metade_ctx *c, const metade_tuning *t) {
  if (!c || !t) return fail(c, METADE_EINVAL, "ctx and t are required");
  const uint32_t rows = t->mfma_rows ? t->mfma_rows : 4u;
  if (rows != 2 && rows != 4) return fail(c, METADE_EINVAL, "mfma_rows must be 0, 2 or 4");
  const uint32_t lp = t->lane_parts;
  if (lp != 0 && lp != 1 && lp != 2 && lp != 4 && lp != 8)
    return fail(c, METADE_EINVAL, "lane_parts must be 0, 1, 2, 4 or 8");
  if (c->n_lane) {
    // parts per trial of the lane runs (the device table also holds the decoded
    // theta, so only L is changed there)
    std::vector<RunDev> runs(c->n_runs);
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    HIP_TRY(c, hipMemcpy(runs.data(), c->runs_d, c->n_runs * sizeof(RunDev), hipMemcpyDeviceToHost));
    uint32_t lds = 0;
    for (uint32_t r = 0; r < c->n_runs; ++r) {
      RunDev &d = runs[r];
      if (d.kern != 0) continue;
      const uint32_t lmax = std::max<uint32_t>(1, std::min<uint32_t>(8, mde::GEN_CONSUMERS / d.Np));
      d.L = lp ? std::min(lp, lmax) : lmax;
      c->runs_h[r].L = d.L;
      lds = std::max(lds, mde::lds_layout(d.N, d.Dp, d.L, d.Np, true).total);
    }
    HIP_TRY(c, hipMemcpy(c->runs_d, runs.data(), c->n_runs * sizeof(RunDev), hipMemcpyHostToDevice));
    c->lds_bytes = lds;
  }
  c->lane_parts = lp;
  c->mfma_rows = rows;
  return METADE_OK;
}

namespace {
// Key of a tuning choice: the shapes of the runs (as a multiset), the
// precision and the generation count the choice was measured with.
uint64_t tuning_key(const metade_ctx *c, uint32_t n_gens) {
  std::vector<uint64_t> shapes;
  for (const RunDev &r : c->runs_h)
    shapes.push_back(((uint64_t)r.N << 40) | ((uint64_t)r.D << 16) |
                     (uint64_t)c->probs_h[r.prob].kind);
  std::sort(shapes.begin(), shapes.end());
  uint64_t h = 0xcbf29ce484222325ull;
  auto mix = [&](uint64_t v) {
    for (int b = 0; b < 8; ++b) {
      h ^= (v >> (8 * b)) & 0xffu;
      h *= 0x100000001b3ull;
    }
  };
  mix(0x6766783935300000ull);  // tag of this library's kernels on gfx950
  mix(c->precision);
  mix(n_gens);
  for (uint64_t v : shapes) mix(v);
  return h;
}
}  // namespace

metade_status metade_autotune(metade_ctx *c, uint32_t n_gens, const char *cache_path,
                              metade_tuning *chosen, double *best_ms) {
  if (!c) return fail(nullptr, METADE_EINVAL, "ctx is NULL");
  if (n_gens == 0) return fail(c, METADE_EINVAL, "n_gens must be >= 1");
  const uint64_t key = tuning_key(c, n_gens);
  char keyhex[17];
  std::snprintf(keyhex, sizeof(keyhex), "%016llx", (unsigned long long)key);
  if (cache_path) {
    std::ifstream in(cache_path);
    std::string line;
    while (std::getline(in, line)) {
      std::istringstream ls(line);
      std::string k;
      metade_tuning t{0, 0};
      double ms = 0.0;
      if ((ls >> k >> t.lane_parts >> t.mfma_rows >> ms) && k == keyhex) {
        TRY(metade_set_tuning(c, &t));
        if (chosen) *chosen = t;
        if (best_ms) *best_ms = ms;
        return METADE_OK;
      }
    }
  }
  // candidates: only the knobs of the kernels this context runs
  std::vector<uint32_t> rows = {4};
  if (c->n_mfma && c->precision == METADE_FP32) rows.push_back(2);
  std::vector<uint32_t> parts = {0};
  if (c->n_lane) parts.insert(parts.end(), {4, 2, 1});
  // the search runs the context's own generations from a checkpoint, which is
  // restored after every candidate and at the end: the context's results do
  // not depend on it
  size_t bytes = 0;
  TRY(metade_get_state(c, nullptr, &bytes));
  std::vector<unsigned char> blob(bytes);
  TRY(metade_get_state(c, blob.data(), &bytes));
  const uint64_t trials0 = c->trials;
  unsigned long long cnt0[N_COUNTERS];
  HIP_TRY(c, hipMemcpy(cnt0, c->counters_d, sizeof(cnt0), hipMemcpyDeviceToHost));
  const bool timing0 = c->timing;
  c->timing = false;
  const metade_tuning orig{c->lane_parts, c->mfma_rows};
  metade_tuning best = orig;
  double best_t = 1e300;
  hipEvent_t ea = nullptr, eb = nullptr;
  metade_status st = METADE_OK;
  {
    hipError_t e = hipEventCreate(&ea);
    if (e == hipSuccess) e = hipEventCreate(&eb);
    if (e != hipSuccess) st = fail(c, METADE_EDEVICE, std::string("autotune events: ") + hipGetErrorString(e));
  }
  for (uint32_t r : rows) {
    if (st != METADE_OK) break;
    for (uint32_t lp : parts) {
      const metade_tuning t{lp, r};
      if ((st = metade_set_tuning(c, &t)) != METADE_OK) break;
      double tmin = 1e300;
      for (int rep = 0; rep < 3 && st == METADE_OK; ++rep) {   // first run warms up
        if ((st = metade_set_state(c, blob.data(), bytes)) != METADE_OK) break;
        hipError_t e = hipEventRecord(ea, c->stream);
        if (e == hipSuccess && (st = run_generations(c, n_gens, mde::TraceArgs{nullptr, nullptr, nullptr})) != METADE_OK) break;
        if (e == hipSuccess) e = hipEventRecord(eb, c->stream);
        if (e == hipSuccess) e = hipEventSynchronize(eb);
        float ms = 0.0f;
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, ea, eb);
        if (e != hipSuccess) { st = fail(c, METADE_EDEVICE, std::string("autotune timing: ") + hipGetErrorString(e)); break; }
        if (rep > 0) tmin = std::min(tmin, (double)ms);
      }
      if (st != METADE_OK) break;
      if (tmin < best_t) { best_t = tmin; best = t; }
    }
    if (st != METADE_OK) break;
  }
  if (ea) (void)hipEventDestroy(ea);
  if (eb) (void)hipEventDestroy(eb);
  c->timing = timing0;
  if (st != METADE_OK) {
    // best effort: the launch shape and the state the context had before the
    // search, keeping the search's own error message
    const std::string err = c->err;
    (void)metade_set_tuning(c, &orig);
    (void)metade_set_state(c, blob.data(), bytes);
    c->trials = trials0;
    (void)hipMemcpy(c->counters_d, cnt0, sizeof(cnt0), hipMemcpyHostToDevice);
    c->err = err;
    return st;
  }
  TRY(metade_set_tuning(c, &best));
  TRY(metade_set_state(c, blob.data(), bytes));
  c->trials = trials0;
  HIP_TRY(c, hipMemcpy(c->counters_d, cnt0, sizeof(cnt0), hipMemcpyHostToDevice));
  if (cache_path) {
    std::ofstream out(cache_path, std::ios::app);
    if (out) out << keyhex << " " << best.lane_parts << " " << best.mfma_rows << " " << best_t << "\n";
  }
  if (chosen) *chosen = best;
  if (best_ms) *best_ms = best_t;
  return METADE_OK;
}

const char *metade_last_error(const metade_ctx *c) {
  return c ? c->err.c_str() : g_init_error.c_str();
}

void metade_destroy(metade_ctx *c) {
  if (!c) return;
  if (c->stream) (void)hipStreamSynchronize(c->stream);
  else (void)hipDeviceSynchronize();
  for (EventPair &ev : c->events) {
    (void)hipEventDestroy(ev.a);
    (void)hipEventDestroy(ev.b);
  }
  (void)hipFree(c->runs_d);
  (void)hipFree(c->probs_d);
  (void)hipFree(c->theta_d);
  (void)hipFree(c->pend_d);
  (void)hipFree(c->Xo);
  (void)hipFree(c->Uo);
  (void)hipFree(c->Vo);
  (void)hipFree(c->yo);
  (void)hipFree(c->yt);
  (void)hipFree(c->bxo);
  (void)hipFree(c->bidx);
  (void)hipFree(c->tab);
  for (auto &e : c->graphs) (void)hipGraphExecDestroy(e.second);
  if (c->cap_stream) (void)hipStreamDestroy(c->cap_stream);
  (void)hipFree(c->counters_d);
  (void)hipFree(c->gen_d);
  (void)hipFree(c->lane_list_d);
  (void)hipFree(c->mfma_list_d);
  (void)hipFree(c->ctrl_list_d);
  (void)hipFree(c->order_d);
  (void)hipFree(c->cfu_d);
  (void)hipFree(c->cacc_d);
  delete c;
}

}  // extern "C"
