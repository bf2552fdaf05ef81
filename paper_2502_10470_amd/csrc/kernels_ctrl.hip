// Control-shaped workload: each individual is the flattened weight vector of
// a tanh policy obs -> 64 -> 64 -> act, scored by a rollout of a linear
// system x_{t+1} = A x_t + B u_t with cost sum_t |x_t|^2 + cw |u_t|^2.  This
// is the paper's neural-control setting (Sec. IV-D, policy MLPs of Table VII)
// on a synthetic plant, with the PDE generation of Alg. 2 around it.
//
// One wavefront owns one individual.  Lane o holds, in registers, row o of
// W1 and of W2, the biases b1[o], b2[o] and an 8-weight slice of W3; the
// rollout's activations are exchanged through LDS.  The closed loop of a
// random policy is chaotic (rounding differences grow by many orders of
// magnitude over the horizon), so the rollout is computed in float64: on
// gfx950 a float64 FMA issues at the same rate as a non-packed float32 FMA.
//
// Per generation three launches: rank (top-p list per run), generation
// (draws, Eq. 12 mutation, Eqs. 8-10 crossover, clip, rollout, selection
// decision; the trial goes to a pending row) and commit (accepted rows).
#include <hip/hip_runtime.h>

#include "gen_common.h"
#include "kernels.h"

namespace mde {

namespace {

// ---------------------------------------------------------------- geometry

struct CtGeom {
  uint32_t O, A, D;                 // obs, act, decision dimension
  uint32_t b1, w2, b2, w3, b3;      // flat offsets of the parameter blocks
};

__device__ __forceinline__ CtGeom ct_geom(const ProbDev &p) {
  CtGeom g;
  g.O = p.obs;
  g.A = p.act;
  g.b1 = CT_H * g.O;
  g.w2 = g.b1 + CT_H;
  g.b2 = g.w2 + CT_H * CT_H;
  g.w3 = g.b2 + CT_H;
  g.b3 = g.w3 + CT_H * g.A;
  g.D = g.b3 + g.A;
  return g;
}

// ---------------------------------------------------------------- float64 tanh
//
// tanh|x| = 1 - 2 / (e^{2|x|} + 1).  e^y: Cody-Waite reduction y = n ln2 + r
// with ln2 split in a 32-bit head (n ln2_hi exact for the n that occur) and a
// tail, |r| <= ln2 / 2, then the Taylor series of e^r to degree 13 (remainder
// below 1e-17 relative) and a scaling by 2^n.  The reciprocal is the hardware
// estimate refined by two Newton steps.  The absolute error is a few units of
// 2^-53, which is what the rollout needs (activations enter sums of O(1)).
// For |x| >= 20, tanh rounds to +-1 in float64; the argument is clamped there.

constexpr double CT_LN2_HI = 0x1.62e42ff000000p-1;
constexpr double CT_LN2_LO = -0x1.718432a1b0e26p-35;
constexpr double CT_LOG2E = 0x1.71547652b82fep+0;

__device__ __forceinline__ double tanh_f64(double x) {
  const double y = fmin(2.0 * fabs(x), 40.0);
  const double n = rint(y * CT_LOG2E);
  double r = fma(-n, CT_LN2_HI, y);
  r = fma(-n, CT_LN2_LO, r);
  double p = 1.0 / 6227020800.0;          // 1/13!
  p = fma(p, r, 1.0 / 479001600.0);
  p = fma(p, r, 1.0 / 39916800.0);
  p = fma(p, r, 1.0 / 3628800.0);
  p = fma(p, r, 1.0 / 362880.0);
  p = fma(p, r, 1.0 / 40320.0);
  p = fma(p, r, 1.0 / 5040.0);
  p = fma(p, r, 1.0 / 720.0);
  p = fma(p, r, 1.0 / 120.0);
  p = fma(p, r, 1.0 / 24.0);
  p = fma(p, r, 1.0 / 6.0);
  p = fma(p, r, 0.5);
  p = fma(p, r, 1.0);
  p = fma(p, r, 1.0);
  const double E = ldexp(p, (int)n);
  const double d = E + 1.0;
  double q = __builtin_amdgcn_rcp(d);
  q = fma(q, fma(-d, q, 1.0), q);
  q = fma(q, fma(-d, q, 1.0), q);
  const double t = fma(-2.0, q, 1.0);
  return copysign(t, x);
}

// ---------------------------------------------------------------- weights and rollout

// The lane's share of one policy (see the file comment); slots past the
// geometry are zero so that they contribute nothing.
struct Wts {
  float w1[CT_MAX_OBS];
  double b1;
  double w2[CT_H];
  double b2;
  double w3[8];
  double b3;
};

// LDS of one wavefront: the plant's coefficients by lane (at[k][lane] =
// A[lane][k], bt[a][lane] = B[lane][a], zero for lanes >= obs) and the
// vectors exchanged between the lanes in a step.
struct CtLds {
  float at[CT_MAX_OBS][CT_H];
  float bt[CT_MAX_ACT][CT_H];
  double x[CT_MAX_OBS];
  double h1[CT_H];
  double h2[CT_H];
  double u[CT_MAX_ACT];
};

__device__ __forceinline__ void load_plant(const unsigned char *tab, const ProbDev &p,
                                           const CtGeom &G, uint32_t lane, CtLds &S) {
  const float *A = tab_ptr<float>(tab, p.A_off);
  const float *B = tab_ptr<float>(tab, p.B_off);
  const bool own = lane < G.O;
  for (uint32_t k = 0; k < (uint32_t)CT_MAX_OBS; ++k) S.at[k][lane] = (own && k < G.O) ? A[lane * G.O + k] : 0.0f;
  for (uint32_t a = 0; a < (uint32_t)CT_MAX_ACT; ++a) S.bt[a][lane] = (own && a < G.A) ? B[lane * G.A + a] : 0.0f;
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int s = 32; s > 0; s >>= 1) v += __shfl_xor(v, s);
  return v;
}

// Mean over the rollouts of J = sum_{t < steps} (|x_t|^2 + cw |u_t|^2),
// u_t = tanh(W3 tanh(W2 tanh(W1 x_t + b1) + b2) + b3), x_{t+1} = A x_t + B u_t.
// Called by the whole wavefront (a one-wave block); returns J in every lane.
__device__ __forceinline__ double rollout(const Wts &W, const float *x0, const CtGeom &G,
                                          uint32_t steps, uint32_t E, double cw, uint32_t lane,
                                          CtLds &S) {
  const uint32_t ga = lane >> 3, gc = lane & 7;
  double jx = 0.0, ju = 0.0;
  for (uint32_t e = 0; e < E; ++e) {
    __syncthreads();
    if (lane < CT_MAX_OBS) {
      const double v = lane < G.O ? (double)x0[e * G.O + lane] : 0.0;
      S.x[lane] = v;
      jx = fma(v, v, jx);
    }
    __syncthreads();
    for (uint32_t t = 0; t < steps; ++t) {
      // layer 1 and the A x_t part of the plant update
      double a1 = W.b1, ax = 0.0;
#pragma unroll
      for (int k = 0; k < CT_MAX_OBS; k += 2) {
        if ((uint32_t)k < G.O) {
          const double2 xv = *reinterpret_cast<const double2 *>(S.x + k);
          a1 = fma((double)W.w1[k], xv.x, a1);
          ax = fma((double)S.at[k][lane], xv.x, ax);
          a1 = fma((double)W.w1[k + 1], xv.y, a1);
          ax = fma((double)S.at[k + 1][lane], xv.y, ax);
        }
      }
      S.h1[lane] = tanh_f64(a1);
      __syncthreads();
      // layer 2: four partial sums
      double c0 = W.b2, c1 = 0.0, c2 = 0.0, c3 = 0.0;
#pragma unroll
      for (int k = 0; k < CT_H; k += 4) {
        const double2 p = *reinterpret_cast<const double2 *>(S.h1 + k);
        const double2 q = *reinterpret_cast<const double2 *>(S.h1 + k + 2);
        c0 = fma(W.w2[k], p.x, c0);
        c1 = fma(W.w2[k + 1], p.y, c1);
        c2 = fma(W.w2[k + 2], q.x, c2);
        c3 = fma(W.w2[k + 3], q.y, c3);
      }
      S.h2[lane] = tanh_f64((c0 + c1) + (c2 + c3));
      __syncthreads();
      // layer 3: lane (ga, gc) sums W3[ga][8gc .. 8gc+7] h2[...], then 8 lanes combine
      double pz = 0.0;
#pragma unroll
      for (int s = 0; s < 8; s += 2) {
        const double2 v = *reinterpret_cast<const double2 *>(S.h2 + 8 * gc + s);
        pz = fma(W.w3[s], v.x, pz);
        pz = fma(W.w3[s + 1], v.y, pz);
      }
      pz += __shfl_xor(pz, 1);
      pz += __shfl_xor(pz, 2);
      pz += __shfl_xor(pz, 4);
      if (gc == 0 && ga < G.A) {
        const double u = tanh_f64(pz + W.b3);
        S.u[ga] = u;
        ju = fma(u, u, ju);
      }
      __syncthreads();
      // plant update; every lane has finished reading x_t (before the first barrier)
      double xn = ax;
#pragma unroll
      for (int a = 0; a < CT_MAX_ACT; ++a)
        if ((uint32_t)a < G.A) xn = fma((double)S.bt[a][lane], S.u[a], xn);
      if (lane < G.O) {
        S.x[lane] = xn;
        if (t + 1 < steps) jx = fma(xn, xn, jx);
      }
      __syncthreads();
    }
  }
  return (wave_sum(jx) + cw * wave_sum(ju)) / (double)E;
}

// Gene index of the lane's slots.
__device__ __forceinline__ uint32_t w1_gene(const CtGeom &G, uint32_t lane, uint32_t k) { return lane * G.O + k; }
__device__ __forceinline__ uint32_t w2_gene(const CtGeom &G, uint32_t lane, uint32_t k) { return G.w2 + lane * CT_H + k; }
__device__ __forceinline__ uint32_t w3_gene(const CtGeom &G, uint32_t lane, uint32_t s) {
  return G.w3 + (lane >> 3) * CT_H + 8 * (lane & 7) + s;
}
__device__ __forceinline__ bool w3_owned(const CtGeom &G, uint32_t lane) { return (lane >> 3) < G.A; }
__device__ __forceinline__ bool b3_owned(const CtGeom &G, uint32_t lane) {
  return (lane >> 3) < G.A && (lane & 7) == 0;
}

// Fill the lane's slots from a per-gene function val(j) -> float.
template <typename Val>
__device__ __forceinline__ void fill_wts(const CtGeom &G, uint32_t lane, Wts &W, Val val) {
#pragma unroll
  for (int k = 0; k < CT_MAX_OBS; ++k) W.w1[k] = (uint32_t)k < G.O ? val(w1_gene(G, lane, k)) : 0.0f;
  W.b1 = (double)val(G.b1 + lane);
#pragma unroll
  for (int k = 0; k < CT_H; ++k) W.w2[k] = (double)val(w2_gene(G, lane, k));
  W.b2 = (double)val(G.b2 + lane);
  const bool o3 = w3_owned(G, lane);
#pragma unroll
  for (int s = 0; s < 8; ++s) W.w3[s] = o3 ? (double)val(w3_gene(G, lane, s)) : 0.0;
  W.b3 = b3_owned(G, lane) ? (double)val(G.b3 + (lane >> 3)) : 0.0;
}

// ---------------------------------------------------------------- trial construction

// Everything one trial needs besides its gene index (uniform over the wave).
struct TrialSrc {
  const float *xi, *xb, *xr;
  const float *pa[4], *pb[4];
  float F, CR, K, lb, ub;
  int dn, cs;
  bool two_base;
  uint32_t D, jn, L;
};

// Mutation (Eq. 12) of gene j, float32 with the operation order of the other
// generation kernels: base = x_bl + F (x_br - x_bl); d = sum of differences
// left to right; v = base + F d.
__device__ __forceinline__ float mutant(const TrialSrc &s, uint32_t j) {
  const float xb = s.xb[j];
  float base = xb;
  if (s.two_base) base = xb + s.F * (s.xr[j] - xb);
  float d = s.pa[0][j] - s.pb[0][j];
#pragma unroll
  for (int k = 1; k < 4; ++k)
    if (k < s.dn) d = d + (s.pa[k][j] - s.pb[k][j]);
  return base + s.F * d;
}

// Trial gene j given the binomial bit of its uniform (r_j <= CR): crossover
// (Eqs. 8-10) and clip to the box.
__device__ __forceinline__ float trial_gene(const TrialSrc &s, uint32_t j, bool bin_bit) {
  const float v = mutant(s, j);
  const float x = s.xi[j];
  float u;
  if (s.cs == ARITH) {
    u = x + s.K * (v - x);
  } else if (s.cs == BIN) {
    u = (bin_bit || j == s.jn) ? v : x;
  } else {
    const uint32_t off = (j + s.D - s.jn) % s.D;
    u = off < s.L ? v : x;
  }
  return fminf(fmaxf(u, s.lb), s.ub);
}

// Binomial bits of genes j0 .. j0+len-1 (len <= 64): bit t is (r_{j0+t} <= CR)
// with r_j the uniform of Philox word 12 + j.
__device__ __forceinline__ uint64_t bin_bits(uint32_t j0, uint32_t len, uint32_t i, uint32_t g,
                                             uint32_t stream, float CR, uint32_t k0, uint32_t k1) {
  uint64_t bits = 0;
  const uint32_t w0 = W_GENE0 + j0, w1 = W_GENE0 + j0 + len;  // words [w0, w1)
  for (uint32_t blk = w0 / 4; 4 * blk < w1; ++blk) {
    const uint4 w = philox(blk, i, g, stream, k0, k1);
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const uint32_t wi = 4 * blk + t;
      if (wi >= w0 && wi < w1 && unit_oc(word_of(w, t)) <= CR) bits |= 1ull << (wi - w0);
    }
  }
  return bits;
}

}  // namespace

// ---------------------------------------------------------------- kernels

// Initial population (Alg. 2 initialisation: word j of the INIT phase gives
// gene j, x = lb + (ub - lb) (w >> 8) 2^-24 in float64 rounded once) and its
// fitness.  Grid (max N, control runs), one wavefront per individual.
__global__ __launch_bounds__(64) void k_ctrl_init(const RunDev *__restrict__ runs,
                                                  const uint32_t *__restrict__ list,
                                                  const ProbDev *__restrict__ probs,
                                                  const unsigned char *__restrict__ tab,
                                                  float *__restrict__ pop, float *__restrict__ fit,
                                                  uint32_t k0, uint32_t k1, double lb, double ub) {
  __shared__ CtLds S;
  const RunDev run = runs[list[blockIdx.y]];
  const uint32_t i = blockIdx.x;
  if (i >= run.N) return;
  const ProbDev p = probs[run.prob];
  const CtGeom G = ct_geom(p);
  const uint32_t lane = threadIdx.x;
  float *row = pop + run.pop_off + (size_t)i * G.D;
  auto val = [&](uint32_t j) -> float {
    const uint4 w = philox(j / 4, i, INIT_PHASE, run.stream, k0, k1);
    const double u0 = (double)(word_of(w, j & 3) >> 8) * 0x1p-24;
    const float x = (float)(lb + (ub - lb) * u0);
    row[j] = x;
    return x;
  };
  Wts W;
  fill_wts(G, lane, W, val);
  load_plant(tab, p, G, lane, S);
  const double J = rollout(W, tab_ptr<float>(tab, p.x0_off), G, p.steps, p.nroll, (double)p.cw,
                           lane, S);
  if (lane == 0) fit[run.fit_off + i] = (float)J;
}

// Top-p list of every control run: order[fit_off + rank] = individual for
// rank < kp, ranking by (fitness, index) with NaN as +inf.  One block per run.
__global__ __launch_bounds__(CT_MAX_N) void k_ctrl_rank(const RunDev *__restrict__ runs,
                                                        const uint32_t *__restrict__ list,
                                                        const float *__restrict__ fit,
                                                        uint32_t *__restrict__ order) {
  __shared__ uint64_t keys[CT_MAX_N];
  const RunDev run = runs[list[blockIdx.x]];
  const uint32_t N = run.N, i = threadIdx.x;
  if (i < N) keys[i] = mkkey(fit[run.fit_off + i], i);
  __syncthreads();
  if (i < N) {
    const uint64_t ki = keys[i];
    uint32_t rank = 0;
    for (uint32_t k = 0; k < N; ++k) rank += keys[k] < ki ? 1u : 0u;
    if (rank < run.kp) order[run.fit_off + rank] = i;
  }
}

// One generation of every control run.  Grid (max N, control runs), one
// wavefront per target i.  Writes the trial to its pending row, its fitness
// and the selection decision (Alg. 1 rule: accept iff f(u) <= f(x)).
template <bool TRACE>
__global__ __launch_bounds__(64) void k_ctrl_gen(
    const RunDev *__restrict__ runs, const uint32_t *__restrict__ list,
    const ProbDev *__restrict__ probs, const unsigned char *__restrict__ tab,
    const float *__restrict__ pop, const float *__restrict__ fit, float *__restrict__ pend,
    float *__restrict__ fu_out, uint32_t *__restrict__ acc_out, const uint32_t *__restrict__ order,
    uint32_t g, float lb, float ub, uint32_t k0, uint32_t k1, TraceArgs tr) {
  __shared__ CtLds S;
  const RunDev run = runs[list[blockIdx.y]];
  const uint32_t i = blockIdx.x;
  if (i >= run.N) return;
  const ProbDev p = probs[run.prob];
  const CtGeom G = ct_geom(p);
  const uint32_t lane = threadIdx.x, N = run.N, D = G.D;

  // random draws of (i, g): words 0..11
  const int use_rand = (run.bl == RAND || run.br == RAND) ? 1 : 0;
  const int dn = run.dn;
  const int m = use_rand + 2 * dn;
  uint32_t w[12];
  {
    const uint4 a = philox(0, i, g, run.stream, k0, k1);
    const uint4 b = philox(1, i, g, run.stream, k0, k1);
    const uint4 c = philox(2, i, g, run.stream, k0, k1);
    w[0] = a.x; w[1] = a.y; w[2] = a.z; w[3] = a.w;
    w[4] = b.x; w[5] = b.y; w[6] = b.z; w[7] = b.w;
    w[8] = c.x; w[9] = c.y; w[10] = c.z; w[11] = c.w;
  }
  uint32_t dr[9];
#pragma unroll
  for (int k = 0; k < 9; ++k) dr[k] = 0;
  sample_distinct(w, m, i, N, dr);
  const uint32_t r0 = use_rand ? dr[0] : 0u;
  const uint32_t pbr = lemire(w[W_PBEST], run.kp);
  const uint32_t jn = lemire(w[W_JRAND], D);
  const float K = unit_oc(w[W_K]);
  // exponential length: 1 + the number of leading uniforms r_0, r_1, ... <= CR, at most D
  uint32_t L = 1;
  if (run.cs == EXP) {
    L = D;
    for (uint32_t c = 0; 256 * c + 1 < D; ++c) {
      const uint4 wr = philox(W_GENE0 / 4 + 64 * c + lane, i, g, run.stream, k0, k1);
      uint32_t first = 4;
#pragma unroll
      for (int t = 3; t >= 0; --t)
        if (unit_oc(word_of(wr, t)) > run.CR) first = (uint32_t)t;
      const uint64_t fail = __ballot(first < 4);
      if (fail) {
        const uint32_t fl = __ffsll((unsigned long long)fail) - 1;
        const uint32_t ft = __shfl(first, (int)fl);
        L = min(D, 4 * (64 * c + fl) + ft + 1);
        break;
      }
    }
  }
  const uint32_t ibest = order[run.fit_off], ipb = order[run.fit_off + pbr];
  auto pick = [&](int code) {
    return code == RAND ? r0 : (code == BEST ? ibest : (code == PBEST ? ipb : i));
  };
  const uint32_t ibl = pick(run.bl), ibr = pick(run.br);
  if (TRACE && lane == 0) {
    int32_t *o = tr.desc + (size_t)(run.fit_off + i) * 16;
    o[0] = (int32_t)ibl;
    o[1] = (int32_t)ibr;
    for (int k = 0; k < 8; ++k) o[2 + k] = (k / 2) < dn ? (int32_t)dr[use_rand + k] : -1;
    o[10] = (int32_t)jn;
    o[11] = run.cs == EXP ? (int32_t)L : -1;
    o[12] = (int32_t)pbr;
    o[13] = use_rand ? (int32_t)r0 : -1;
    o[14] = run.cs == ARITH ? (int32_t)__float_as_uint(K) : -1;
    o[15] = 0;
  }

  const float *P0 = pop + run.pop_off;
  TrialSrc s;
  s.xi = P0 + (size_t)i * D;
  s.xb = P0 + (size_t)ibl * D;
  s.xr = P0 + (size_t)ibr * D;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const uint32_t a = k < dn ? dr[use_rand + 2 * k] : 0u;
    const uint32_t b = k < dn ? dr[use_rand + 2 * k + 1] : 0u;
    s.pa[k] = P0 + (size_t)a * D;
    s.pb[k] = P0 + (size_t)b * D;
  }
  s.F = run.F;
  s.CR = run.CR;
  s.K = K;
  s.lb = lb;
  s.ub = ub;
  s.dn = dn;
  s.cs = run.cs;
  s.two_base = run.bl != run.br;
  s.D = D;
  s.jn = jn;
  s.L = L;

  // binomial bits of the lane's gene segments
  const bool bin = run.cs == BIN;
  const uint32_t st = run.stream;
  const uint64_t m1 = bin ? bin_bits(w1_gene(G, lane, 0), G.O, i, g, st, run.CR, k0, k1) : 0;
  const uint64_t m2 = bin ? bin_bits(w2_gene(G, lane, 0), CT_H, i, g, st, run.CR, k0, k1) : 0;
  const uint64_t m3 = (bin && w3_owned(G, lane)) ? bin_bits(w3_gene(G, lane, 0), 8, i, g, st, run.CR, k0, k1) : 0;
  const uint64_t mb = bin ? bin_bits(G.b1 + lane, 1, i, g, st, run.CR, k0, k1) |
                                (bin_bits(G.b2 + lane, 1, i, g, st, run.CR, k0, k1) << 1) |
                                ((b3_owned(G, lane) ? bin_bits(G.b3 + (lane >> 3), 1, i, g, st, run.CR, k0, k1) : 0ull) << 2)
                          : 0;
  float *U = pend + run.pend_off + (size_t)i * D;
  float *Ut = TRACE ? tr.u + run.pop_off + (size_t)i * D : nullptr;
  auto put = [&](uint32_t j, float u) {
    U[j] = u;
    if (TRACE) Ut[j] = u;
    return u;
  };
  Wts W;
#pragma unroll
  for (int k = 0; k < CT_MAX_OBS; ++k) {
    float u = 0.0f;
    if ((uint32_t)k < G.O) {
      const uint32_t j = w1_gene(G, lane, k);
      u = put(j, trial_gene(s, j, (m1 >> k) & 1));
    }
    W.w1[k] = u;
  }
  W.b1 = (double)put(G.b1 + lane, trial_gene(s, G.b1 + lane, mb & 1));
#pragma unroll
  for (int k = 0; k < CT_H; ++k) {
    const uint32_t j = w2_gene(G, lane, k);
    W.w2[k] = (double)put(j, trial_gene(s, j, (m2 >> k) & 1));
  }
  W.b2 = (double)put(G.b2 + lane, trial_gene(s, G.b2 + lane, (mb >> 1) & 1));
  const bool o3 = w3_owned(G, lane);
#pragma unroll
  for (int t = 0; t < 8; ++t) {
    double v = 0.0;
    if (o3) {
      const uint32_t j = w3_gene(G, lane, t);
      v = (double)put(j, trial_gene(s, j, (m3 >> t) & 1));
    }
    W.w3[t] = v;
  }
  W.b3 = b3_owned(G, lane) ? (double)put(G.b3 + (lane >> 3), trial_gene(s, G.b3 + (lane >> 3), (mb >> 2) & 1)) : 0.0;

  load_plant(tab, p, G, lane, S);
  const double J = rollout(W, tab_ptr<float>(tab, p.x0_off), G, p.steps, p.nroll, (double)p.cw,
                           lane, S);
  if (lane == 0) {
    const float f = (float)J;
    const float fx = fit[run.fit_off + i];
    const bool a = accept_trial(f, fx);
    fu_out[run.fit_off + i] = f;
    acc_out[run.fit_off + i] = a ? 1u : 0u;
    if (TRACE) {
      tr.fu[run.fit_off + i] = f;
      tr.desc[(size_t)(run.fit_off + i) * 16 + 15] = a ? 1 : 0;
    }
  }
}

// Greedy selection commit: accepted pending rows replace their targets.
// Grid (max N, control runs).
__global__ __launch_bounds__(256) void k_ctrl_commit(const RunDev *__restrict__ runs,
                                                     const uint32_t *__restrict__ list,
                                                     float *__restrict__ pop, float *__restrict__ fit,
                                                     const float *__restrict__ pend,
                                                     const float *__restrict__ fu,
                                                     const uint32_t *__restrict__ acc) {
  const RunDev run = runs[list[blockIdx.y]];
  const uint32_t i = blockIdx.x;
  if (i >= run.N || !acc[run.fit_off + i]) return;
  const uint32_t D = run.D;
  const float *src = pend + run.pend_off + (size_t)i * D;
  float *dst = pop + run.pop_off + (size_t)i * D;
  for (uint32_t j = threadIdx.x; j < D; j += 256) dst[j] = src[j];
  if (threadIdx.x == 0) fit[run.fit_off + i] = fu[run.fit_off + i];
}

// Best record of every control run: the first individual in (fitness, index)
// order, its float64 cost (the rollout is float64 already) and its weights.
__global__ __launch_bounds__(64) void k_ctrl_finalize(const RunDev *__restrict__ runs,
                                                      const uint32_t *__restrict__ list,
                                                      const ProbDev *__restrict__ probs,
                                                      const unsigned char *__restrict__ tab,
                                                      const float *__restrict__ pop,
                                                      const float *__restrict__ fit,
                                                      double *__restrict__ best_y,
                                                      float *__restrict__ best_x) {
  __shared__ CtLds S;
  const uint32_t r = list[blockIdx.x];
  const RunDev run = runs[r];
  const ProbDev p = probs[run.prob];
  const CtGeom G = ct_geom(p);
  const uint32_t lane = threadIdx.x;
  uint64_t best = ~0ull;
  for (uint32_t i = lane; i < run.N; i += 64) best = min(best, mkkey(fit[run.fit_off + i], i));
#pragma unroll
  for (int s = 32; s > 0; s >>= 1) {
    const uint64_t o = __shfl_xor(best, s);
    best = min(best, o);
  }
  const uint32_t b = (uint32_t)(best & 0xFFFFFFFFu);
  const float *x = pop + run.pop_off + (size_t)b * G.D;
  for (uint32_t j = lane; j < G.D; j += 64) best_x[run.bx_off + j] = x[j];
  Wts W;
  fill_wts(G, lane, W, [&](uint32_t j) { return x[j]; });
  load_plant(tab, p, G, lane, S);
  const double J = rollout(W, tab_ptr<float>(tab, p.x0_off), G, p.steps, p.nroll, (double)p.cw,
                           lane, S);
  if (lane == 0) best_y[r] = J;
}

// ---------------------------------------------------------------- launchers

hipError_t launch_ctrl_init(const LaunchArgs &a, const CtrlArgs &c, double lb, double ub) {
  if (c.n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_ctrl_init, dim3(c.max_n, c.n), dim3(64), 0, a.stream, a.runs, c.list,
                     a.probs, a.tab, a.pop, a.fit, a.k0, a.k1, lb, ub);
  return hipGetLastError();
}

hipError_t launch_ctrl_generations(const LaunchArgs &a, const CtrlArgs &c, uint32_t g0,
                                   uint32_t n_gens, float lb, float ub, TraceArgs tr) {
  if (c.n == 0) return hipSuccess;
  for (uint32_t g = g0; g < g0 + n_gens; ++g) {
    hipLaunchKernelGGL(k_ctrl_rank, dim3(c.n), dim3(CT_MAX_N), 0, a.stream, a.runs, c.list, a.fit,
                       c.order);
    if (tr.u)
      hipLaunchKernelGGL(HIP_KERNEL_NAME(k_ctrl_gen<true>), dim3(c.max_n, c.n), dim3(64), 0,
                         a.stream, a.runs, c.list, a.probs, a.tab, a.pop, a.fit, a.pending, c.fu,
                         c.acc, c.order, g, lb, ub, a.k0, a.k1, tr);
    else
      hipLaunchKernelGGL(HIP_KERNEL_NAME(k_ctrl_gen<false>), dim3(c.max_n, c.n), dim3(64), 0,
                         a.stream, a.runs, c.list, a.probs, a.tab, a.pop, a.fit, a.pending, c.fu,
                         c.acc, c.order, g, lb, ub, a.k0, a.k1, tr);
    hipLaunchKernelGGL(k_ctrl_commit, dim3(c.max_n, c.n), dim3(256), 0, a.stream, a.runs, c.list,
                       a.pop, a.fit, a.pending, c.fu, c.acc);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t launch_ctrl_finalize(const LaunchArgs &a, const CtrlArgs &c, double *best_y,
                                float *best_x) {
  if (c.n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_ctrl_finalize, dim3(c.n), dim3(64), 0, a.stream, a.runs, c.list, a.probs,
                     a.tab, a.pop, a.fit, best_y, best_x);
  return hipGetLastError();
}

}  // namespace mde
