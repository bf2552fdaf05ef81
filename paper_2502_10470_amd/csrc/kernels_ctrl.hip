// Control-shaped workload: each individual is the flattened weight vector of
// a tanh policy obs -> H -> H -> act (H = 32, the MLPs of Table VII, or 64),
// scored by a rollout of a linear system x_{t+1} = A x_t + B u_t with cost
// sum_t |x_t|^2 + cw |u_t|^2.  This is the paper's neural-control setting
// (Sec. IV-D) on a synthetic plant, with the PDE generation of Alg. 2 around
// it.
//
// One wavefront evaluates 64 / L individuals of one run, L lanes each (L = 32;
// L = 16 for H = 32 when obs <= 16, which halves the number of wavefronts
// and keeps two rows per lane).  Lane l of a group holds, in registers,
// hidden rows l + L r of W2 (r < H / L; the float32 values of the population,
// widened at use), their biases and a slice of W3; its rows of W1 sit in LDS
// next to each other.  The activations are exchanged through LDS; with two
// rows per lane every float64 value read from LDS feeds two FMAs, which
// halves the LDS traffic per multiply-add.  The rollout is float64: the
// closed loop of a policy amplifies rounding differences (by orders of
// magnitude for weights of order one), and on gfx950 a float64 FMA issues at
// the rate of a non-packed float32 FMA.
//
// Per generation four launches: rank (top-p list per run); trials (draws,
// Eq. 12 mutation, Eqs. 8-10 crossover, clip: one block per trial reading
// the population rows with coalesced loads and writing the trial to a
// 16-byte aligned pending row); evaluation (rollout and selection decision);
// commit (accepted rows replace their targets).  The trial kernel reads the
// generation from a device counter that the last launch of a sequence
// advances, so a captured sequence replays at any starting generation.
#include <hip/hip_runtime.h>

#include <type_traits>

#include "gen_common.h"
#include "kernels.h"

namespace mde {

namespace {

constexpr uint32_t CT_TRIAL_THREADS = 256;       // trial construction: threads per trial
constexpr uint32_t CT_TRIAL_THREADS_INIT = 256;  // initialisation: threads per individual

// Layout of a policy of hidden width H over L lanes of a wavefront (a group):
// lane l holds hidden rows l + L r, r < RPL; for layer 3 lane l is part
// c = l % LPA of output a = l / LPA (LPA = L / 8 lanes per output, so up to 8
// outputs) and holds W3[a][c W3 .. (c+1) W3 - 1]; observation l of the plant
// update sits on lane l, so obs <= MAXO.
template <int H, int L>
struct Ct {
  static_assert((H == CT_H_SMALL || H == CT_H) && (L == 16 || L == 32) && H >= L, "layout");
  static constexpr int RPL = H / L;    // hidden rows per lane
  static constexpr int IPW = 64 / L;   // individuals per wavefront
  static constexpr int LPA = L / 8;    // lanes per output of layer 3
  static constexpr int W3 = H / LPA;   // W3 weights per lane
  static constexpr int MAXO = L < CT_MAX_OBS ? L : CT_MAX_OBS;
};

// ---------------------------------------------------------------- geometry

struct CtGeom {
  uint32_t O, A, D;                 // obs, act, decision dimension
  uint32_t b1, w2, b2, w3, b3;      // flat offsets of the parameter blocks
};

template <int H>
__device__ __forceinline__ CtGeom ct_geom(const ProbDev &p) {
  CtGeom g;
  g.O = p.obs;
  g.A = p.act;
  g.b1 = H * g.O;
  g.w2 = g.b1 + H;
  g.b2 = g.w2 + H * H;
  g.w3 = g.b2 + H;
  g.b3 = g.w3 + H * g.A;
  g.D = g.b3 + g.A;
  return g;
}

// Gene index of each register slot of lane l (0..L-1 within its group).
template <int L>
__device__ __forceinline__ uint32_t row_of(uint32_t l, int r) { return l + L * r; }
template <int L>
__device__ __forceinline__ uint32_t w1_gene(const CtGeom &G, uint32_t l, int r, uint32_t k) {
  return row_of<L>(l, r) * G.O + k;
}
template <int H, int L>
__device__ __forceinline__ uint32_t w2_gene(const CtGeom &G, uint32_t l, int r, uint32_t k) {
  return G.w2 + row_of<L>(l, r) * H + k;
}
template <int H, int L>
__device__ __forceinline__ uint32_t w3_gene(const CtGeom &G, uint32_t l, uint32_t s) {
  using C = Ct<H, L>;
  return G.w3 + (l / C::LPA) * H + C::W3 * (l % C::LPA) + s;
}
template <int H, int L>
__device__ __forceinline__ bool w3_owned(const CtGeom &G, uint32_t l) {
  return l / Ct<H, L>::LPA < G.A;
}
template <int H, int L>
__device__ __forceinline__ bool b3_owned(const CtGeom &G, uint32_t l) {
  return l / Ct<H, L>::LPA < G.A && l % Ct<H, L>::LPA == 0;
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
  // sum_{k<=13} r^k / k! by Estrin's scheme (dependency depth 4 instead of 13)
  const double r2 = r * r, r4 = r2 * r2, r8 = r4 * r4;
  const double q0 = fma(r, 1.0, 1.0);
  const double q1 = fma(r, 1.0 / 6.0, 0.5);
  const double q2 = fma(r, 1.0 / 120.0, 1.0 / 24.0);
  const double q3 = fma(r, 1.0 / 5040.0, 1.0 / 720.0);
  const double q4 = fma(r, 1.0 / 362880.0, 1.0 / 40320.0);
  const double q5 = fma(r, 1.0 / 39916800.0, 1.0 / 3628800.0);
  const double q6 = fma(r, 1.0 / 6227020800.0, 1.0 / 479001600.0);
  const double s0 = fma(r2, q1, q0);
  const double s1 = fma(r2, q3, q2);
  const double s2 = fma(r2, q5, q4);
  const double t0 = fma(r4, s1, s0);
  const double t1 = fma(r4, q6, s2);
  const double p = fma(r8, t1, t0);
  const double E = ldexp(p, (int)n);
  const double d = E + 1.0;
  double q = __builtin_amdgcn_rcp(d);
  q = fma(q, fma(-d, q, 1.0), q);
  q = fma(q, fma(-d, q, 1.0), q);
  const double t = fma(-2.0, q, 1.0);
  return copysign(t, x);
}

// ---------------------------------------------------------------- weights and rollout

// The lane's share of one policy (see the file comment), kept as the float32
// values the population holds; slots past the geometry are zero so that they
// contribute nothing.
template <int H, int L>
struct Wts {
  float b1[Ct<H, L>::RPL];
  float w2[Ct<H, L>::RPL][H];
  float b2[Ct<H, L>::RPL];
  float w3[Ct<H, L>::W3];
  float b3;
};

// LDS of one wavefront: the plant's coefficients by lane (at[k][l] = A[l][k],
// bt[a][l] = B[l][a], zero for l >= obs; all groups belong to one run) and
// per group the vectors exchanged between the lanes in a step.
// The groups' vectors are padded by 16 bytes so that the addresses of one
// broadcast read fall in different LDS banks; every vector starts at a
// multiple of 16 bytes (they are read in double2).
template <int H, int L>
struct alignas(16) CtLds {
  using C = Ct<H, L>;
  float w1[C::MAXO][C::IPW][C::RPL * L];  // W1[l + L r][k] of group h at [k][h][RPL l + r]
  float at[C::MAXO][L];
  float bt[CT_MAX_ACT][L];
  double x[C::IPW][C::MAXO + 2];
  double h1[C::IPW][H + 2];
  double h2[C::IPW][H + 2];
  double u[C::IPW][CT_MAX_ACT + 2];
};

template <int H, int L>
__device__ __forceinline__ void load_plant(const unsigned char *tab, const ProbDev &p,
                                           const CtGeom &G, uint32_t lane, CtLds<H, L> &S) {
  if (lane >= (uint32_t)L) return;
  const float *A = tab_ptr<float>(tab, p.A_off);
  const float *B = tab_ptr<float>(tab, p.B_off);
  const bool own = lane < G.O;
  for (uint32_t k = 0; k < (uint32_t)Ct<H, L>::MAXO; ++k) S.at[k][lane] = (own && k < G.O) ? A[lane * G.O + k] : 0.0f;
  for (uint32_t a = 0; a < (uint32_t)CT_MAX_ACT; ++a) S.bt[a][lane] = (own && a < G.A) ? B[lane * G.A + a] : 0.0f;
}

// Sum over the L lanes of a group.
template <int L>
__device__ __forceinline__ double group_sum(double v) {
#pragma unroll
  for (int s = L / 2; s > 0; s >>= 1) v += __shfl_xor(v, s);
  return v;
}

// Mean over the rollouts of J = sum_{t < steps} (|x_t|^2 + cw |u_t|^2),
// u_t = tanh(W3 tanh(W2 tanh(W1 x_t + b1) + b2) + b3), x_{t+1} = A x_t + B u_t,
// for the individual of this lane's group.  Called by the whole wavefront (a
// one-wave block); returns J in every lane of the group.
template <int H, int L>
__device__ __forceinline__ double rollout(Wts<H, L> &W, const float *x0, const CtGeom &G,
                                          uint32_t steps, uint32_t E, double cw, uint32_t lane,
                                          CtLds<H, L> &S) {
  using C = Ct<H, L>;
  constexpr int RPL = C::RPL, W3N = C::W3, LPA = C::LPA, MAXO = C::MAXO;
  const uint32_t h = lane / L, l = lane % L;
  const uint32_t ga = l / LPA, gc = l % LPA;
  double *X = S.x[h], *H1 = S.h1[h], *H2 = S.h2[h], *U = S.u[h];
  double jx = 0.0, ju = 0.0;
  for (uint32_t e = 0; e < E; ++e) {
    __syncthreads();
    if (l < (uint32_t)MAXO) {
      const double v = l < G.O ? (double)x0[e * G.O + l] : 0.0;
      X[l] = v;
      jx = fma(v, v, jx);
    }
    __syncthreads();
    for (uint32_t t = 0; t < steps; ++t) {
      // Keep the weights as float32 across steps: an empty asm that "modifies"
      // them stops the compiler from hoisting the float64 widening out of the
      // loop (which would double their registers).
#pragma unroll
      for (int k = 0; k < H; ++k) {
        if constexpr (RPL == 2) asm volatile("" : "+v"(W.w2[0][k]), "+v"(W.w2[1][k]));
        else asm volatile("" : "+v"(W.w2[0][k]));
      }
#pragma unroll
      for (int k = 0; k < W3N; ++k) asm volatile("" : "+v"(W.w3[k]));
      // layer 1 (the lane's rows) and the A x_t part of the plant update
      double y1[RPL], y1b[RPL];
#pragma unroll
      for (int r = 0; r < RPL; ++r) {
        y1[r] = (double)W.b1[r];
        y1b[r] = 0.0;
      }
      double ax = 0.0, axb = 0.0;
#pragma unroll
      for (int k = 0; k < MAXO; k += 2) {
        if ((uint32_t)k < G.O) {
          const double2 xv = *reinterpret_cast<const double2 *>(X + k);
          if constexpr (RPL == 2) {
            const float2 wa = *reinterpret_cast<const float2 *>(&S.w1[k][h][2 * l]);
            const float2 wb = *reinterpret_cast<const float2 *>(&S.w1[k + 1][h][2 * l]);
            y1[0] = fma((double)wa.x, xv.x, y1[0]);
            y1[1] = fma((double)wa.y, xv.x, y1[1]);
            y1b[0] = fma((double)wb.x, xv.y, y1b[0]);
            y1b[1] = fma((double)wb.y, xv.y, y1b[1]);
          } else {
            y1[0] = fma((double)S.w1[k][h][l], xv.x, y1[0]);
            y1b[0] = fma((double)S.w1[k + 1][h][l], xv.y, y1b[0]);
          }
          ax = fma((double)S.at[k][l], xv.x, ax);
          axb = fma((double)S.at[k + 1][l], xv.y, axb);
        }
      }
      ax += axb;
#pragma unroll
      for (int r = 0; r < RPL; ++r) H1[l + L * r] = tanh_f64(y1[r] + y1b[r]);
      __syncthreads();
      // layer 2: the lane's rows, four partial sums each
      double c[RPL][4];
#pragma unroll
      for (int r = 0; r < RPL; ++r)
#pragma unroll
        for (int q = 0; q < 4; ++q) c[r][q] = q == 0 ? (double)W.b2[r] : 0.0;
#pragma unroll
      for (int k = 0; k < H; k += 2) {
        const double2 v = *reinterpret_cast<const double2 *>(H1 + k);
#pragma unroll
        for (int r = 0; r < RPL; ++r) {
          c[r][k & 3] = fma((double)W.w2[r][k], v.x, c[r][k & 3]);
          c[r][(k + 1) & 3] = fma((double)W.w2[r][k + 1], v.y, c[r][(k + 1) & 3]);
        }
      }
#pragma unroll
      for (int r = 0; r < RPL; ++r)
        H2[l + L * r] = tanh_f64((c[r][0] + c[r][1]) + (c[r][2] + c[r][3]));
      __syncthreads();
      // layer 3: lane (ga, gc) sums its W3N weights of W3 row ga against the
      // matching slice of h2, then the LPA lanes of the row combine
      double pz = 0.0, pzb = 0.0;
#pragma unroll
      for (int s = 0; s < W3N; s += 2) {
        const double2 v = *reinterpret_cast<const double2 *>(H2 + W3N * gc + s);
        pz = fma((double)W.w3[s], v.x, pz);
        pzb = fma((double)W.w3[s + 1], v.y, pzb);
      }
      pz += pzb;
#pragma unroll
      for (int o = 1; o < LPA; o <<= 1) pz += __shfl_xor(pz, o);
      if (gc == 0 && ga < G.A) {
        const double u = tanh_f64(pz + (double)W.b3);
        U[ga] = u;
        ju = fma(u, u, ju);
      }
      __syncthreads();
      // plant update; every lane has finished reading x_t (before the first barrier)
      double xn = ax;
#pragma unroll
      for (int a = 0; a < CT_MAX_ACT; ++a)
        if ((uint32_t)a < G.A) xn = fma((double)S.bt[a][l], U[a], xn);
      if (l < G.O) {
        X[l] = xn;
        if (t + 1 < steps) jx = fma(xn, xn, jx);
      }
      __syncthreads();
    }
  }
  return (group_sum<L>(jx) + cw * group_sum<L>(ju)) / (double)E;
}

// Fill the lane's slots from a per-gene function val(j) -> float.
template <int H, int L, typename Val>
__device__ __forceinline__ void fill_wts(const CtGeom &G, uint32_t h, uint32_t l, Wts<H, L> &W,
                                         CtLds<H, L> &S, Val val) {
  using C = Ct<H, L>;
#pragma unroll
  for (int r = 0; r < C::RPL; ++r) {
    for (uint32_t k = 0; k < (uint32_t)C::MAXO; ++k)
      S.w1[k][h][C::RPL * l + r] = k < G.O ? val(w1_gene<L>(G, l, r, k)) : 0.0f;
    W.b1[r] = val(G.b1 + row_of<L>(l, r));
#pragma unroll
    for (int k = 0; k < H; ++k) W.w2[r][k] = val(w2_gene<H, L>(G, l, r, k));
    W.b2[r] = val(G.b2 + row_of<L>(l, r));
  }
  const bool o3 = w3_owned<H, L>(G, l);
#pragma unroll
  for (int s = 0; s < C::W3; ++s) W.w3[s] = o3 ? val(w3_gene<H, L>(G, l, s)) : 0.0f;
  W.b3 = b3_owned<H, L>(G, l) ? val(G.b3 + l / C::LPA) : 0.0f;
}

// ---------------------------------------------------------------- trial construction

// Genes j0 .. j0+3 of a population row (stride D floats; rows are 8-byte
// aligned when D is even); genes >= D read as 0.
__device__ __forceinline__ float4 row_quad(const float *row, uint32_t j0, uint32_t D, bool even) {
  if (j0 + 4 <= D) {
    if (even) {
      const float2 a = *reinterpret_cast<const float2 *>(row + j0);
      const float2 b = *reinterpret_cast<const float2 *>(row + j0 + 2);
      return make_float4(a.x, a.y, b.x, b.y);
    }
    return make_float4(row[j0], row[j0 + 1], row[j0 + 2], row[j0 + 3]);
  }
  float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
#pragma unroll
  for (int t = 0; t < 4; ++t)
    if (j0 + t < D) set_comp(v, t, row[j0 + t]);
  return v;
}

}  // namespace

// ---------------------------------------------------------------- kernels

// Initial population (Alg. 2 initialisation: word j of the INIT phase gives
// gene j, x = lb + (ub - lb) (w >> 8) 2^-24 in float64 rounded once), written
// to the population and to the pending row the evaluation kernel reads.  One
// block per individual, grid (max N, control runs).
__global__ __launch_bounds__(CT_TRIAL_THREADS_INIT) void k_ctrl_init_pop(
    const RunDev *__restrict__ runs, const uint32_t *__restrict__ list, float *__restrict__ pop,
    float *__restrict__ pend, uint32_t k0, uint32_t k1, double lb, double ub) {
  const RunDev run = runs[list[blockIdx.y]];
  const uint32_t i = blockIdx.x;
  if (i >= run.N) return;
  const uint32_t D = run.D;
  float *row = pop + run.pop_off + (size_t)i * D;
  float *Urow = pend + run.pend_off + (size_t)i * run.Dp;
  for (uint32_t q = threadIdx.x; 4 * q < D; q += CT_TRIAL_THREADS_INIT) {
    const uint4 w = philox(q, i, INIT_PHASE, run.stream, k0, k1);
    float4 x;
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const double u0 = (double)(word_of(w, t) >> 8) * 0x1p-24;
      const float v = 4 * q + t < D ? (float)(lb + (ub - lb) * u0) : 0.0f;
      set_comp(x, t, v);
      if (4 * q + t < D) row[4 * q + t] = v;
    }
    *reinterpret_cast<float4 *>(Urow + 4 * q) = x;
  }
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

// Trial vectors of one generation of every control run: one block per target
// i, grid (max N, control runs).  Index draws, the pbest rank, j_rand / n, K
// and the exponential length come from Philox words of (i, g); mutation
// (Eq. 12, float32, the operation order of the other generation kernels:
// base = x_bl + F (x_br - x_bl), differences summed left to right,
// v = base + F d), crossover (Eqs. 8-10) and clip run over gene quads with
// coalesced loads.  The trial goes to its pending row (stride Dp).

template <bool TRACE>
__global__ __launch_bounds__(CT_TRIAL_THREADS) void k_ctrl_trials(
    const RunDev *__restrict__ runs, const uint32_t *__restrict__ list,
    const float *__restrict__ pop, float *__restrict__ pend, const uint32_t *__restrict__ order,
    const uint32_t *__restrict__ gen, uint32_t gg, float lb, float ub, uint32_t k0, uint32_t k1,
    TraceArgs tr) {
  const RunDev run = runs[list[blockIdx.y]];
  const uint32_t i = blockIdx.x;
  const uint32_t g = gen[0] + gg;  // generation counter kept on the device
  if (i >= run.N) return;
  const uint32_t N = run.N, D = run.D, tid = threadIdx.x, lane = tid % 64;
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
  const float F = run.F, CR = run.CR;
  // exponential length: 1 + the number of leading uniforms r_0, r_1, ... <= CR,
  // at most D; every wavefront scans 256 uniforms per round (4 per lane)
  uint32_t L = 1;
  if (run.cs == EXP) {
    L = D;
    for (uint32_t c = 0; 256 * c + 1 < D; ++c) {
      const uint4 wr = philox(W_GENE0 / 4 + 64 * c + lane, i, g, run.stream, k0, k1);
      uint32_t first = 4;
#pragma unroll
      for (int t = 3; t >= 0; --t)
        if (unit_oc(word_of(wr, t)) > CR) first = (uint32_t)t;
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
  if (TRACE && tid == 0) {
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
  const float *xi = P0 + (size_t)i * D, *xb = P0 + (size_t)ibl * D, *xr = P0 + (size_t)ibr * D;
  const float *pa[4], *pb[4];
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    pa[k] = P0 + (size_t)(k < dn ? dr[use_rand + 2 * k] : 0u) * D;
    pb[k] = P0 + (size_t)(k < dn ? dr[use_rand + 2 * k + 1] : 0u) * D;
  }
  // float2 loads when every row is 8-byte aligned
  const bool even = ((reinterpret_cast<uintptr_t>(P0) & 7u) == 0) && (D & 1u) == 0;
  const bool two_base = run.bl != run.br;
  float *Urow = pend + run.pend_off + (size_t)i * run.Dp;
  float *Ut = TRACE ? tr.u + run.pop_off + (size_t)i * D : nullptr;
  for (uint32_t q = tid; 4 * q < D; q += CT_TRIAL_THREADS) {
    const uint32_t j0 = 4 * q;
    const float4 x = row_quad(xi, j0, D, even);
    const float4 b = row_quad(xb, j0, D, even);
    float4 base = b;
    if (two_base) {
      const float4 rr = row_quad(xr, j0, D, even);
      base.x = b.x + F * (rr.x - b.x);
      base.y = b.y + F * (rr.y - b.y);
      base.z = b.z + F * (rr.z - b.z);
      base.w = b.w + F * (rr.w - b.w);
    }
    float4 d;
    {
      const float4 a0 = row_quad(pa[0], j0, D, even), b0 = row_quad(pb[0], j0, D, even);
      d.x = a0.x - b0.x; d.y = a0.y - b0.y; d.z = a0.z - b0.z; d.w = a0.w - b0.w;
    }
#pragma unroll
    for (int k = 1; k < 4; ++k) {
      if (k < dn) {
        const float4 ak = row_quad(pa[k], j0, D, even), bk = row_quad(pb[k], j0, D, even);
        d.x = d.x + (ak.x - bk.x);
        d.y = d.y + (ak.y - bk.y);
        d.z = d.z + (ak.z - bk.z);
        d.w = d.w + (ak.w - bk.w);
      }
    }
    float4 v;
    v.x = base.x + F * d.x;
    v.y = base.y + F * d.y;
    v.z = base.z + F * d.z;
    v.w = base.w + F * d.w;
    float4 u;
    if (run.cs == ARITH) {
      u.x = x.x + K * (v.x - x.x);
      u.y = x.y + K * (v.y - x.y);
      u.z = x.z + K * (v.z - x.z);
      u.w = x.w + K * (v.w - x.w);
    } else if (run.cs == BIN) {
      // words 12 + j0 .. 12 + j0 + 3 are exactly Philox block 3 + q
      const uint4 wr = philox(W_GENE0 / 4 + q, i, g, run.stream, k0, k1);
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const bool take = unit_oc(word_of(wr, t)) <= CR || j0 + t == jn;
        set_comp(u, t, take ? comp(v, t) : comp(x, t));
      }
    } else {
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const uint32_t off = (j0 + t + D - jn) % D;
        set_comp(u, t, off < L ? comp(v, t) : comp(x, t));
      }
    }
#pragma unroll
    for (int t = 0; t < 4; ++t)
      set_comp(u, t, j0 + t < D ? fminf(fmaxf(comp(u, t), lb), ub) : 0.0f);
    *reinterpret_cast<float4 *>(Urow + j0) = u;
    if (TRACE) {
#pragma unroll
      for (int t = 0; t < 4; ++t)
        if (j0 + t < D) Ut[j0 + t] = comp(u, t);
    }
  }
}

// Rollout and selection decision of every control trial (INIT: the first
// evaluation of the initial population, written as its fitness).  Grid
// (ceil(max N / IPW), control runs), one wavefront per IPW = 64 / L targets
// (the obs <= MAXO of the layout is checked at set-up); each lane loads its
// weight slots from the pending row (float4 where aligned).
template <int H, int L, bool TRACE, bool INIT>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(2))) void k_ctrl_eval(
    const RunDev *__restrict__ runs, const uint32_t *__restrict__ list,
    const ProbDev *__restrict__ probs, const unsigned char *__restrict__ tab,
    float *__restrict__ fit, const float *__restrict__ pend, float *__restrict__ fu_out,
    uint32_t *__restrict__ acc_out, TraceArgs tr) {
  using C = Ct<H, L>;
  constexpr int RPL = C::RPL;
  __shared__ CtLds<H, L> S;
  const RunDev run = runs[list[blockIdx.y]];
  const uint32_t lane = threadIdx.x, h = lane / L, l = lane % L;
  const uint32_t i0 = C::IPW * blockIdx.x;
  if (i0 >= run.N) return;
  const uint32_t N = run.N;
  const uint32_t i = min(i0 + h, N - 1);   // past the end: a copy of the last target
  const bool writer = i0 + h < N;
  const ProbDev p = probs[run.prob];
  const CtGeom G = ct_geom<H>(p);
  const float *U = pend + run.pend_off + (size_t)i * run.Dp;
  Wts<H, L> W;
  // W1 rows (stride obs, not aligned in general) into LDS, biases
#pragma unroll
  for (int r = 0; r < RPL; ++r) {
    for (uint32_t k = 0; k < (uint32_t)C::MAXO; ++k)
      S.w1[k][h][RPL * l + r] = k < G.O ? U[w1_gene<L>(G, l, r, k)] : 0.0f;
    W.b1[r] = U[G.b1 + row_of<L>(l, r)];
    W.b2[r] = U[G.b2 + row_of<L>(l, r)];
  }
  // W2 rows: 16-byte aligned (pending rows are, the block starts at H (obs + 1)
  // and H is a multiple of 4)
#pragma unroll
  for (int r = 0; r < RPL; ++r) {
#pragma unroll
    for (int k = 0; k < H; k += 4) {
      const float4 a = *reinterpret_cast<const float4 *>(U + w2_gene<H, L>(G, l, r, k));
      W.w2[r][k] = a.x; W.w2[r][k + 1] = a.y; W.w2[r][k + 2] = a.z; W.w2[r][k + 3] = a.w;
    }
  }
  const bool o3 = w3_owned<H, L>(G, l);
#pragma unroll
  for (int t = 0; t < C::W3; t += 4) {
    float4 a = make_float4(0.f, 0.f, 0.f, 0.f);
    if (o3) a = *reinterpret_cast<const float4 *>(U + w3_gene<H, L>(G, l, t));
    W.w3[t] = a.x; W.w3[t + 1] = a.y; W.w3[t + 2] = a.z; W.w3[t + 3] = a.w;
  }
  W.b3 = b3_owned<H, L>(G, l) ? U[G.b3 + l / C::LPA] : 0.0f;

  load_plant<H, L>(tab, p, G, lane, S);
  const double J = rollout(W, tab_ptr<float>(tab, p.x0_off), G, p.steps, p.nroll, (double)p.cw,
                           lane, S);
  if (writer && l == 0) {
    const float f = (float)J;
    if (INIT) {
      fit[run.fit_off + i] = f;
    } else {
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
}

// ---------------------------------------------------------------- matrix-core evaluation
//
// With 16 rollouts per policy (or a multiple of 16, taken 16 at a time) every
// layer of a step is a product [rows x k] x [k x 16 rollouts], so one
// wavefront evaluates one policy on v_mfma_f64_16x16x4f64.  That
// instruction takes A[i][k] from lane i + 16 k and B[k][j] from lane j + 16 k
// and leaves result element v of lane l at row l/16 + 4 v, column l % 16.  A
// result tile therefore already holds in every lane what the next product
// needs as its B operand: k-step s = 4 t + v (rows 4 s + l/16) is element v
// of tile t.  State, activations and actions stay in registers for the whole
// rollout (no LDS, no shuffles, no barriers); the weights are the A operands,
// float32 values of the population widened at use: W1, W3 and the plant in
// registers, W2 and the hidden biases read from the (L2-resident) row at every
// step, which leaves room for two wavefronts per SIMD.

typedef double ct_d4 __attribute__((ext_vector_type(4)));

constexpr int CT_MX_S1 = (CT_MAX_OBS + 3) / 4;  // k-steps over the observations
constexpr int CT_MX_SA = (CT_MAX_ACT + 3) / 4;  // k-steps over the actions

__device__ __forceinline__ ct_d4 mx(float a, double b, ct_d4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64((double)a, b, c, 0, 0, 0);
}
__device__ __forceinline__ ct_d4 tanh4(ct_d4 x) {
  ct_d4 y;
#pragma unroll
  for (int v = 0; v < 4; ++v) y[v] = tanh_f64(x[v]);
  return y;
}

// Mean cost J of the policy with weights U (D floats) over the problem's
// rollouts, on the matrix cores; called by a whole wavefront, returns J in
// every lane.  The problem has obs <= 20, act <= 8 and a multiple of 16
// rollouts (checked at set-up).
// Physical order of the hidden units: result row p of a hidden layer holds
// unit (H/4)(p mod 4) + p/4, so that a lane's A operands of the next layer
// (k-steps s = 0 .. H/4-1 of lane group g: units (H/4) g + s) and its biases
// (rows 16 t + g + 4 v: units 16 g + 4 t + v for H = 64) are contiguous.
template <int H>
__device__ __forceinline__ uint32_t unit_of(uint32_t p) {
  return (H / 4) * (p % 4) + p / 4;
}

template <bool VEC>
__device__ __forceinline__ float4 ld4w(const float *__restrict__ q) {
  if (VEC) return *reinterpret_cast<const float4 *>(q);
  return make_float4(q[0], q[1], q[2], q[3]);
}

// Mean cost J of the policy with weights U (D floats; 16-byte aligned rows
// when VEC) over the problem's rollouts, on the matrix cores; called by a
// whole wavefront, returns J in every lane.  The problem has obs <= 20,
// act <= 8 and a multiple of 16 rollouts (checked at set-up).  W2 and the
// hidden biases are read from the row at every step (L2-resident), one block
// of four k-steps ahead; the rest of the weights stay in registers.
template <int H, bool VEC>
__device__ __forceinline__ double rollout_mx(const float *__restrict__ U, const ProbDev &p,
                                             const unsigned char *__restrict__ tab,
                                             uint32_t lane) {
  constexpr int T = H / 16;  // row tiles of a hidden layer
  constexpr int S = H / 4;   // k-steps over a hidden layer
  const uint32_t c = lane % 16, g = lane / 16;
  const CtGeom G = ct_geom<H>(p);
  const float *Ap = tab_ptr<float>(tab, p.A_off);
  const float *Bp = tab_ptr<float>(tab, p.B_off);
  const float *x0 = tab_ptr<float>(tab, p.x0_off);
  // registers: W1[unit(16 t + c)][4 s + g], W3[c][unit(4 s + g)], plant A and B
  float w1[T][CT_MX_S1], w3[S], pa[2][CT_MX_S1], pb[2][CT_MX_SA], b3[4];
#pragma unroll
  for (int t = 0; t < T; ++t) {
    const uint32_t row = unit_of<H>(16 * t + c);
#pragma unroll
    for (int s = 0; s < CT_MX_S1; ++s) {
      const uint32_t col = 4 * s + g;
      w1[t][s] = col < G.O ? U[row * G.O + col] : 0.0f;
    }
  }
#pragma unroll
  for (int s = 0; s < S; ++s) w3[s] = c < G.A ? U[G.w3 + c * H + (H / 4) * g + s] : 0.0f;
#pragma unroll
  for (int v = 0; v < 4; ++v) b3[v] = g + 4 * v < G.A ? U[G.b3 + g + 4 * v] : 0.0f;
#pragma unroll
  for (int t = 0; t < 2; ++t) {
    const uint32_t row = 16 * t + c;
#pragma unroll
    for (int s = 0; s < CT_MX_S1; ++s) {
      const uint32_t col = 4 * s + g;
      pa[t][s] = (row < G.O && col < G.O) ? Ap[row * G.O + col] : 0.0f;
    }
#pragma unroll
    for (int s = 0; s < CT_MX_SA; ++s) {
      const uint32_t col = 4 * s + g;
      pb[t][s] = (row < G.O && col < G.A) ? Bp[row * G.A + col] : 0.0f;
    }
  }
  // streamed: row t of the lane's W2 operands (units (H/4) g .. +H/4-1 of row
  // unit(16 t + c)); biases of the lane's result rows, tile t element v = unit
  // (H/4) g + 4 t + v: four consecutive floats per tile
  const float *w2r[T];
#pragma unroll
  for (int t = 0; t < T; ++t) w2r[t] = U + G.w2 + unit_of<H>(16 * t + c) * H + (H / 4) * g;
  const float *b1r = U + G.b1 + (H / 4) * g;
  const float *b2r = U + G.b2 + (H / 4) * g;

  const uint32_t E = p.nroll, steps = p.steps;
  double jx = 0.0, ju = 0.0;
  for (uint32_t e0 = 0; e0 < E; e0 += 16) {
    ct_d4 X[2];
#pragma unroll
    for (int t = 0; t < 2; ++t)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const uint32_t o = 16 * t + g + 4 * v;
        const double xv = o < G.O ? (double)x0[(e0 + c) * G.O + o] : 0.0;
        X[t][v] = xv;
        jx = fma(xv, xv, jx);
      }
    for (uint32_t st = 0; st < steps; ++st) {
      // keep the register weights as float32 across steps (an empty asm that
      // "modifies" them stops the widening from being hoisted out of the loop,
      // which would double their registers)
#pragma unroll
      for (int t = 0; t < T; ++t)
#pragma unroll
        for (int s = 0; s < CT_MX_S1; ++s) asm volatile("" : "+v"(w1[t][s]));
#pragma unroll
      for (int s = 0; s < S; ++s) asm volatile("" : "+v"(w3[s]));
#pragma unroll
      for (int t = 0; t < 2; ++t) {
#pragma unroll
        for (int s = 0; s < CT_MX_S1; ++s) asm volatile("" : "+v"(pa[t][s]));
#pragma unroll
        for (int s = 0; s < CT_MX_SA; ++s) asm volatile("" : "+v"(pb[t][s]));
      }
      // first W2 block of this step and the biases, in flight during layer 1
      float4 wb[T];
#pragma unroll
      for (int t = 0; t < T; ++t) wb[t] = ld4w<VEC>(w2r[t]);
      ct_d4 H1[T];
#pragma unroll
      for (int t = 0; t < T; ++t) {
        const float4 bb = ld4w<VEC>(b1r + 4 * t);
        H1[t] = ct_d4{(double)bb.x, (double)bb.y, (double)bb.z, (double)bb.w};
      }
#pragma unroll
      for (int s = 0; s < CT_MX_S1; ++s)
#pragma unroll
        for (int t = 0; t < T; ++t) H1[t] = mx(w1[t][s], X[s / 4][s % 4], H1[t]);
#pragma unroll
      for (int t = 0; t < T; ++t) H1[t] = tanh4(H1[t]);
      // layer 2: blocks j of four k-steps, the next block's loads in flight
      ct_d4 H2[T];
#pragma unroll
      for (int t = 0; t < T; ++t) {
        const float4 bb = ld4w<VEC>(b2r + 4 * t);
        H2[t] = ct_d4{(double)bb.x, (double)bb.y, (double)bb.z, (double)bb.w};
      }
#pragma unroll
      for (int j = 0; j < S / 4; ++j) {
        float4 wn[T];
        if (j + 1 < S / 4) {
#pragma unroll
          for (int t = 0; t < T; ++t) wn[t] = ld4w<VEC>(w2r[t] + 4 * (j + 1));
        }
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const int s = 4 * j + e;
#pragma unroll
          for (int t = 0; t < T; ++t) H2[t] = mx(comp(wb[t], e), H1[s / 4][s % 4], H2[t]);
        }
        if (j + 1 < S / 4) {
#pragma unroll
          for (int t = 0; t < T; ++t) wb[t] = wn[t];
        }
      }
#pragma unroll
      for (int t = 0; t < T; ++t) H2[t] = tanh4(H2[t]);
      ct_d4 u = ct_d4{(double)b3[0], (double)b3[1], (double)b3[2], (double)b3[3]};
#pragma unroll
      for (int s = 0; s < S; ++s) u = mx(w3[s], H2[s / 4][s % 4], u);
      u = tanh4(u);
#pragma unroll
      for (int v = 0; v < 4; ++v) ju = fma(u[v], u[v], ju);
      ct_d4 Xn[2];
#pragma unroll
      for (int t = 0; t < 2; ++t) {
        Xn[t] = ct_d4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int s = 0; s < CT_MX_S1; ++s) Xn[t] = mx(pa[t][s], X[s / 4][s % 4], Xn[t]);
#pragma unroll
        for (int s = 0; s < CT_MX_SA; ++s) Xn[t] = mx(pb[t][s], u[s], Xn[t]);
      }
#pragma unroll
      for (int t = 0; t < 2; ++t) X[t] = Xn[t];
      if (st + 1 < steps) {
#pragma unroll
        for (int t = 0; t < 2; ++t)
#pragma unroll
          for (int v = 0; v < 4; ++v) jx = fma(X[t][v], X[t][v], jx);
      }
    }
  }
  double jsum = jx + (double)p.cw * ju;
#pragma unroll
  for (int s2 = 32; s2 > 0; s2 >>= 1) jsum += __shfl_xor(jsum, s2);
  return jsum / (double)E;
}

// Rollout and selection decision of every control trial, one wavefront per
// target (INIT: the first evaluation).  Grid (max N, control runs).
template <int H, bool TRACE, bool INIT>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(2))) void k_ctrl_eval_mx(
    const RunDev *__restrict__ runs, const uint32_t *__restrict__ list,
    const ProbDev *__restrict__ probs, const unsigned char *__restrict__ tab,
    float *__restrict__ fit, const float *__restrict__ pend, float *__restrict__ fu_out,
    uint32_t *__restrict__ acc_out, TraceArgs tr) {
  const RunDev run = runs[list[blockIdx.y]];
  const uint32_t i = blockIdx.x;
  if (i >= run.N) return;
  const uint32_t lane = threadIdx.x;
  const ProbDev p = probs[run.prob];
  const double J = rollout_mx<H, true>(pend + run.pend_off + (size_t)i * run.Dp, p, tab, lane);
  if (lane == 0) {
    const float f = (float)J;
    if (INIT) {
      fit[run.fit_off + i] = f;
    } else {
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
  const float *src = pend + run.pend_off + (size_t)i * run.Dp;
  float *dst = pop + run.pop_off + (size_t)i * D;
  for (uint32_t j = threadIdx.x; j < D; j += 256) dst[j] = src[j];
  if (threadIdx.x == 0) fit[run.fit_off + i] = fu[run.fit_off + i];
}

// Best record of every control run: the first individual in (fitness, index)
// order, its float64 cost (the rollout is float64 already) and its weights.
// Every group of the wavefront evaluates it; the first writes.
template <int H, int L>
__global__ __launch_bounds__(64) void k_ctrl_finalize(const RunDev *__restrict__ runs,
                                                      const uint32_t *__restrict__ list,
                                                      const ProbDev *__restrict__ probs,
                                                      const unsigned char *__restrict__ tab,
                                                      const float *__restrict__ pop,
                                                      const float *__restrict__ fit,
                                                      double *__restrict__ best_y,
                                                      float *__restrict__ best_x) {
  __shared__ CtLds<H, L> S;
  const uint32_t r = list[blockIdx.x];
  const RunDev run = runs[r];
  const ProbDev p = probs[run.prob];
  const CtGeom G = ct_geom<H>(p);
  const uint32_t lane = threadIdx.x, h = lane / L, l = lane % L;
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
  Wts<H, L> W;
  fill_wts<H, L>(G, h, l, W, S, [&](uint32_t j) { return x[j]; });
  load_plant<H, L>(tab, p, G, lane, S);
  const double J = rollout(W, tab_ptr<float>(tab, p.x0_off), G, p.steps, p.nroll, (double)p.cw,
                           lane, S);
  if (lane == 0) best_y[r] = J;
}

// Best record with the matrix-core rollout (runs with a multiple of 16
// rollouts): as k_ctrl_finalize, one wavefront per run.
template <int H>
__global__ __launch_bounds__(64) void k_ctrl_finalize_mx(const RunDev *__restrict__ runs,
                                                         const uint32_t *__restrict__ list,
                                                         const ProbDev *__restrict__ probs,
                                                         const unsigned char *__restrict__ tab,
                                                         const float *__restrict__ pop,
                                                         const float *__restrict__ fit,
                                                         double *__restrict__ best_y,
                                                         float *__restrict__ best_x) {
  const uint32_t r = list[blockIdx.x];
  const RunDev run = runs[r];
  const ProbDev p = probs[run.prob];
  const uint32_t lane = threadIdx.x;
  uint64_t best = ~0ull;
  for (uint32_t i = lane; i < run.N; i += 64) best = min(best, mkkey(fit[run.fit_off + i], i));
#pragma unroll
  for (int s = 32; s > 0; s >>= 1) {
    const uint64_t o = __shfl_xor(best, s);
    best = min(best, o);
  }
  const uint32_t b = (uint32_t)(best & 0xFFFFFFFFu);
  const float *x = pop + run.pop_off + (size_t)b * run.D;
  for (uint32_t j = lane; j < run.D; j += 64) best_x[run.bx_off + j] = x[j];
  const double J = rollout_mx<H, false>(x, p, tab, lane);
  if (lane == 0) best_y[r] = J;
}

// ---------------------------------------------------------------- launchers

namespace {

// The three layouts: (H, L) = (64, 32), (32, 32), (32, 16).
bool layout_ok(const CtrlArgs &c) {
  return (c.hidden == (uint32_t)CT_H && c.lanes == 32) ||
         (c.hidden == (uint32_t)CT_H_SMALL && (c.lanes == 32 || c.lanes == 16));
}

// Evaluation launch for the context's layout.
template <bool TRACE, bool INIT>
void launch_eval(const LaunchArgs &a, const CtrlArgs &c, TraceArgs tr) {
  if (c.mx) {
    const dim3 mgrid(c.max_n, c.n);
    if (c.hidden == (uint32_t)CT_H)
      hipLaunchKernelGGL(HIP_KERNEL_NAME(k_ctrl_eval_mx<CT_H, TRACE, INIT>), mgrid, dim3(64), 0,
                         a.stream, a.runs, c.list, a.probs, a.tab, a.fit, a.pending, c.fu, c.acc,
                         tr);
    else
      hipLaunchKernelGGL(HIP_KERNEL_NAME(k_ctrl_eval_mx<CT_H_SMALL, TRACE, INIT>), mgrid, dim3(64),
                         0, a.stream, a.runs, c.list, a.probs, a.tab, a.fit, a.pending, c.fu,
                         c.acc, tr);
    return;
  }
  const uint32_t ipw = 64 / c.lanes;
  const dim3 egrid((c.max_n + ipw - 1) / ipw, c.n);
  if (c.hidden == (uint32_t)CT_H)
    hipLaunchKernelGGL(HIP_KERNEL_NAME(k_ctrl_eval<CT_H, 32, TRACE, INIT>), egrid, dim3(64), 0,
                       a.stream, a.runs, c.list, a.probs, a.tab, a.fit, a.pending, c.fu, c.acc, tr);
  else if (c.lanes == 32)
    hipLaunchKernelGGL(HIP_KERNEL_NAME(k_ctrl_eval<CT_H_SMALL, 32, TRACE, INIT>), egrid, dim3(64),
                       0, a.stream, a.runs, c.list, a.probs, a.tab, a.fit, a.pending, c.fu, c.acc,
                       tr);
  else
    hipLaunchKernelGGL(HIP_KERNEL_NAME(k_ctrl_eval<CT_H_SMALL, 16, TRACE, INIT>), egrid, dim3(64),
                       0, a.stream, a.runs, c.list, a.probs, a.tab, a.fit, a.pending, c.fu, c.acc,
                       tr);
}

}  // namespace

hipError_t launch_ctrl_init(const LaunchArgs &a, const CtrlArgs &c, double lb, double ub) {
  if (c.n == 0) return hipSuccess;
  if (!layout_ok(c)) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_ctrl_init_pop, dim3(c.max_n, c.n), dim3(CT_TRIAL_THREADS_INIT), 0, a.stream,
                     a.runs, c.list, a.pop, a.pending, a.k0, a.k1, lb, ub);
  launch_eval<false, true>(a, c, TraceArgs{nullptr, nullptr, nullptr});
  return hipGetLastError();
}

// Generation counter of the control runs: set from the host's count, and
// advanced by the last launch of every generation sequence, so that a
// captured sequence (HIP graph) can be replayed at any starting generation.
__global__ void k_ctrl_set_gen(uint32_t *gen, uint32_t v) {
  if (threadIdx.x == 0) gen[0] = v;
}
__global__ void k_ctrl_add_gen(uint32_t *gen, uint32_t n) {
  if (threadIdx.x == 0) gen[0] += n;
}

hipError_t launch_ctrl_set_gen(uint32_t *gen, uint32_t v, hipStream_t s) {
  hipLaunchKernelGGL(k_ctrl_set_gen, dim3(1), dim3(64), 0, s, gen, v);
  return hipGetLastError();
}

hipError_t launch_ctrl_generations(const LaunchArgs &a, const CtrlArgs &c, uint32_t *gen,
                                   uint32_t n_gens, float lb, float ub, TraceArgs tr) {
  if (c.n == 0) return hipSuccess;
  if (!layout_ok(c)) return hipErrorInvalidValue;
  const dim3 tgrid(c.max_n, c.n);
  for (uint32_t g = 0; g < n_gens; ++g) {
    hipLaunchKernelGGL(k_ctrl_rank, dim3(c.n), dim3(CT_MAX_N), 0, a.stream, a.runs, c.list, a.fit,
                       c.order);
    if (tr.u) {
      hipLaunchKernelGGL(HIP_KERNEL_NAME(k_ctrl_trials<true>), tgrid, dim3(CT_TRIAL_THREADS), 0,
                         a.stream, a.runs, c.list, a.pop, a.pending, c.order, gen, g, lb, ub,
                         a.k0, a.k1, tr);
      launch_eval<true, false>(a, c, tr);
    } else {
      hipLaunchKernelGGL(HIP_KERNEL_NAME(k_ctrl_trials<false>), tgrid, dim3(CT_TRIAL_THREADS), 0,
                         a.stream, a.runs, c.list, a.pop, a.pending, c.order, gen, g, lb, ub,
                         a.k0, a.k1, tr);
      launch_eval<false, false>(a, c, tr);
    }
    hipLaunchKernelGGL(k_ctrl_commit, dim3(c.max_n, c.n), dim3(256), 0, a.stream, a.runs, c.list,
                       a.pop, a.fit, a.pending, c.fu, c.acc);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(k_ctrl_add_gen, dim3(1), dim3(64), 0, a.stream, gen, n_gens);
  return hipGetLastError();
}

hipError_t launch_ctrl_finalize(const LaunchArgs &a, const CtrlArgs &c, double *best_y,
                                float *best_x) {
  if (c.n == 0) return hipSuccess;
  if (!layout_ok(c)) return hipErrorInvalidValue;
  if (c.mx) {
    if (c.hidden == (uint32_t)CT_H)
      hipLaunchKernelGGL(HIP_KERNEL_NAME(k_ctrl_finalize_mx<CT_H>), dim3(c.n), dim3(64), 0,
                         a.stream, a.runs, c.list, a.probs, a.tab, a.pop, a.fit, best_y, best_x);
    else
      hipLaunchKernelGGL(HIP_KERNEL_NAME(k_ctrl_finalize_mx<CT_H_SMALL>), dim3(c.n), dim3(64), 0,
                         a.stream, a.runs, c.list, a.probs, a.tab, a.pop, a.fit, best_y, best_x);
    return hipGetLastError();
  }
  if (c.hidden == (uint32_t)CT_H)
    hipLaunchKernelGGL(HIP_KERNEL_NAME(k_ctrl_finalize<CT_H, 32>), dim3(c.n), dim3(64), 0,
                       a.stream, a.runs, c.list, a.probs, a.tab, a.pop, a.fit, best_y, best_x);
  else if (c.lanes == 32)
    hipLaunchKernelGGL(HIP_KERNEL_NAME(k_ctrl_finalize<CT_H_SMALL, 32>), dim3(c.n), dim3(64), 0,
                       a.stream, a.runs, c.list, a.probs, a.tab, a.pop, a.fit, best_y, best_x);
  else
    hipLaunchKernelGGL(HIP_KERNEL_NAME(k_ctrl_finalize<CT_H_SMALL, 16>), dim3(c.n), dim3(64), 0,
                       a.stream, a.runs, c.list, a.probs, a.tab, a.pop, a.fit, best_y, best_x);
  return hipGetLastError();
}

}  // namespace mde
