// HIP kernels of the MetaDE inner-DE path for gfx950.
//
// One workgroup owns one executor run for the whole launch: its population,
// fitness, ranking state, random draws and the generation's trial rows live
// in LDS, and the generation loop of Alg. 2 runs inside the kernel (no
// grid-wide synchronisation).  Runs whose population and trials do not fit
// in LDS go to the matrix-core kernel.
#include "device.h"
#include "gen_common.h"
#include "kernels.h"

namespace mde {

MDE_STAGE_ARRAY;

// ---------------------------------------------------------------- fitness of one row, split by output

// acc[q] = sum_k R[jc+q][k] u_k in float64 for q < J, from the transposed
// rotation Rt[k][j]: the J coefficients of one k are contiguous and
// wave-uniform, so they arrive by wide scalar loads and feed the FMAs as
// scalar operands.  u_k = t[k*ts] is the lane's own trial.  The products of
// two float32 values are exact in float64; R o is subtracted per output
// afterwards (z = R u - R o, R o precomputed in float64), which spares a
// subtraction and a load per k.  Outputs past D read the padding columns of
// Rt (zero) and are not used.
template <int J, typename TP>
__device__ __forceinline__ void rot_block(const double *__restrict__ Rt, uint32_t D, uint32_t Dr,
                                          uint32_t jc, TP t, uint32_t ts, double (&acc)[J]) {
#pragma unroll
  for (int q = 0; q < J; ++q) acc[q] = 0.0;
  const double *col = Rt + jc;
  uint32_t k = 0;
  for (; k + 8 <= D; k += 8) {
    float tv[8];
#pragma unroll
    for (int kk = 0; kk < 8; ++kk) tv[kk] = t[(k + kk) * ts];
#pragma unroll
    for (int kk = 0; kk < 8; ++kk) {
      const double yk = (double)tv[kk];
      const double *c = col + (size_t)(k + kk) * Dr;
#pragma unroll
      for (int q = 0; q < J; ++q) acc[q] = fma(c[q], yk, acc[q]);
    }
  }
  for (; k < D; ++k) {
    const double yk = (double)t[k * ts];
    const double *c = col + (size_t)k * Dr;
#pragma unroll
    for (int q = 0; q < J; ++q) acc[q] = fma(c[q], yk, acc[q]);
  }
}

struct TermAcc {
  double s0, s1;
  float prevz;
  bool have;
};

template <int J>
__device__ __forceinline__ void consume(const unsigned char *tab, const ProbDev &p,
                                        const double (&a)[J], uint32_t jc, uint32_t n,
                                        uint32_t j1, TermAcc &ta) {
#pragma unroll
  for (int q = 0; q < J; ++q) {
    if ((uint32_t)q < n) {
      const uint32_t j = jc + q;
      const float z = (float)(a[q] - tab_ptr<double>(tab, p.ro64_off)[j]);
      if (p.kind == FN_ROSENBROCK) {
        if (ta.have && j - 1 < j1) ta.s0 += (double)h_rosenbrock<float>(ta.prevz, z);
        ta.prevz = z;
        ta.have = true;
      } else {
        float t0, t1;
        elem_term<float>(tab, p, j, z, t0, t1);
        ta.s0 += (double)t0;
        ta.s1 += (double)t1;
      }
    }
  }
}

// Sum of the element terms of outputs [j0, j1) of the row at t (gene stride
// ts).  Plain path: z = R u - R o accumulated in float64 -- the products are
// exact and the sums round at 2^-53 of |R| |u|, so a small z_j that cancels
// between large terms still comes out far below float32 resolution -- z
// rounded once to float32, element terms in float32, sums in float64.
template <typename TP>
__device__ __forceinline__ void eval_part(const unsigned char *__restrict__ tab, const ProbDev &p,
                                          uint32_t D, uint32_t j0, uint32_t j1, TP t, uint32_t ts,
                                          double &s0, double &s1) {
  const double *Rt = tab_ptr<double>(tab, p.r64t_off);
  const uint32_t Dr = rt_stride(D);
  TermAcc ta{0.0, 0.0, 0.0f, false};
  const uint32_t jend = p.kind == FN_ROSENBROCK ? min(j1 + 1, D) : j1;
  uint32_t jc = j0;
  while (jc < jend) {
    const uint32_t rem = jend - jc;
#define MDE_BLOCK(JJ)                                        \
  {                                                          \
    double a[JJ];                                            \
    rot_block<JJ>(Rt, D, Dr, jc, t, ts, a);                  \
    consume<JJ>(tab, p, a, jc, min(rem, (uint32_t)JJ), j1, ta); \
    jc += JJ;                                                \
  }
    if (rem > 10) MDE_BLOCK(12)
    else if (rem > 8) MDE_BLOCK(10)
    else if (rem > 6) MDE_BLOCK(8)
    else if (rem == 6) MDE_BLOCK(6)
    else if (rem == 5) MDE_BLOCK(5)
    else if (rem > 2) MDE_BLOCK(4)
    else MDE_BLOCK(2)
#undef MDE_BLOCK
  }
  s0 = ta.s0;
  s1 = ta.s1;
}

// ---------------------------------------------------------------- init (Alg. 2 initialisation)

__global__ __launch_bounds__(INIT_THREADS) void k_init(const RunDev *__restrict__ runs,
                                                       const ProbDev *__restrict__ probs,
                                                       const unsigned char *__restrict__ tab,
                                                       float *__restrict__ pop,
                                                       float *__restrict__ fit, uint32_t k0,
                                                       uint32_t k1, double lb, double ub) {
  extern __shared__ __align__(16) unsigned char smem[];
  const RunDev run = runs[blockIdx.x];
  if (run.kern == 2) return;  // control runs have their own initialisation kernel
  const ProbDev p = probs[run.prob];
  const uint32_t N = run.N, D = run.D, Dp = run.Dp, Q = Dp / 4;
  const uint32_t Np = ((N + 63u) / 64u) * 64u, L = init_parts(Np);
  float *pop_s = reinterpret_cast<float *>(smem);
  double2 *Ps = reinterpret_cast<double2 *>(smem + al16(N * Dp * 4));
  const uint32_t tid = threadIdx.x;
  const uint32_t l = __builtin_amdgcn_readfirstlane(tid / Np);
  const uint32_t i = tid - l * Np;
  const bool act = l < L && i < N;

  // x = lb + (ub - lb) u0, u0 = (w >> 8) 2^-24, in float64, rounded once.
  for (uint32_t u = tid; u < N * Q; u += INIT_THREADS) {
    const uint32_t r = u / Q, q = u - r * Q;
    const uint4 w = philox(q, r, INIT_PHASE, run.stream, k0, k1);
    float4 x;
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const uint32_t j = 4 * q + t;
      const double u0 = (double)(word_of(w, t) >> 8) * 0x1p-24;
      set_comp(x, t, j < D ? (float)(lb + (ub - lb) * u0) : 0.0f);
    }
    st4(pop_s, r * Dp + 4 * q, x);
  }
  __syncthreads();
  if (act) {
    double s0, s1;
    eval_part(tab, p, D, l * D / L, (l + 1) * D / L, pop_s + i * Dp, 1u, s0, s1);
    Ps[l * Np + i] = make_double2(s0, s1);
  }
  __syncthreads();
  if (act && l == 0) {
    double s0 = 0.0, s1 = 0.0;
    for (uint32_t ll = 0; ll < L; ++ll) {
      const double2 v = Ps[ll * Np + i];
      s0 += v.x;
      s1 += v.y;
    }
    fit[run.fit_off + i] = finish_f32(p, s0, s1);
  }
  for (uint32_t u = tid; u < N * D; u += INIT_THREADS) {
    const uint32_t r = u / D, j = u - r * D;
    pop[run.pop_off + u] = pop_s[r * Dp + j];
  }
}

// ---------------------------------------------------------------- generations (Alg. 2 main loop)
//
// Consumer lanes build the trials by (trial, gene quad) items and write them
// gene-major to LDS; for the fitness, lane i of part l takes outputs
// [l D / L, (l+1) D / L) of trial i, and the parts' partial sums meet in LDS.
// Per generation (four barriers):
//   S0 ranks and top-p list | S2 mutation + crossover (producers: the
//   crossover-test nibbles of g+1, into the other buffer, and Philox block 2
//   of g+1's draws) | S3 fitness (producers: the rest of g+1's draws: index
//   draws, pbest rank, j_rand, K, exponential length from the nibbles) |
//   S4 selection + commit by the items of S2.

// Producer waves: the random draws of generation g + 1 while the consumers
// work on generation g.  Runs the same barrier sequence as gen_consumers
// (one before the loop, four per generation, one after it), so the two roles
// keep separate loops and neither holds the other's registers.
__device__ __forceinline__ void gen_producers(const Lds &lay, unsigned char *smem,
                                              const RunDev &run, uint32_t g0, uint32_t n_gens,
                                              uint32_t k0, uint32_t k1, uint32_t ptid) {
  const uint32_t N = run.N, D = run.D, Q = run.Dp / 4, kp = run.kp;
  uint8_t *msk = reinterpret_cast<uint8_t *>(smem + lay.msk);
  uint4 *dsc = reinterpret_cast<uint4 *>(smem + lay.dsc);
  constexpr uint32_t NP = GEN_THREADS - GEN_CONSUMERS;
  produce_masks(ptid, NP, run, N, Q, g0, k0, k1, msk + (g0 & 1u) * N * Q);
  __syncthreads();
  produce_desc_direct(ptid, NP, run, N, D, kp, g0, k0, k1, msk + (g0 & 1u) * N * Q, dsc);
  MDE_STAGE_BEGIN
  for (uint32_t gg = 0; gg < n_gens; ++gg) {
    const uint32_t g = g0 + gg;
    __syncthreads();   // generation g starts (consumers rank)
    MDE_STAGE(0)
    __syncthreads();   // consumers build the trials of g
    MDE_STAGE(1)
    uint8_t *mn = msk + ((g + 1) & 1u) * N * Q;
    produce_masks(ptid, NP, run, N, Q, g + 1, k0, k1, mn);
    // block 2 of the next generation's draws now, the rest during the
    // fitness (N <= 256: one trial per producer lane)
    uint4 wc_next = uint4{};
    if (ptid < N) wc_next = philox(2, ptid, g + 1, run.stream, k0, k1);
    MDE_STAGE_WORK(6)
    __syncthreads();   // consumers evaluate g
    MDE_STAGE(2)
    produce_desc_direct<true>(ptid, NP, run, N, D, kp, g + 1, k0, k1, mn, dsc, wc_next);
    MDE_STAGE_WORK(7)
    __syncthreads();   // consumers select and commit g
    MDE_STAGE(3)
  }
  __syncthreads();
  MDE_STAGE(0)
  MDE_STAGE_END
}

// Consumer waves: ranking, trial construction, fitness, selection and commit
// of every generation (barrier sequence as gen_producers).
template <bool TRACE>
__device__ __forceinline__ void gen_consumers(const Lds &lay, unsigned char *smem,
                                              const RunDev &run, const ProbDev &p,
                                              const unsigned char *__restrict__ tab,
                                              uint32_t g0, uint32_t n_gens, float lb, float ub,
                                              const TraceArgs &tr, uint32_t tid) {
  const uint32_t N = run.N, D = run.D, Dp = run.Dp, Q = Dp / 4, kp = run.kp, L = run.L,
                 Np = run.Np;
  float *pop_s = reinterpret_cast<float *>(smem + lay.pop);
  uint64_t *key_s = reinterpret_cast<uint64_t *>(smem + lay.key);
  float *fit_s = reinterpret_cast<float *>(smem + lay.fit);
  float *fx_s = reinterpret_cast<float *>(smem + lay.fx);
  uint32_t *topk = reinterpret_cast<uint32_t *>(smem + lay.topk);
  double2 *Ps = reinterpret_cast<double2 *>(smem + lay.ps);
  const uint8_t *msk = reinterpret_cast<const uint8_t *>(smem + lay.msk);
  const uint4 *dsc = reinterpret_cast<const uint4 *>(smem + lay.dsc);
  float *T = reinterpret_cast<float *>(smem + lay.T);
  const uint32_t ts = Np;
  const uint32_t l = __builtin_amdgcn_readfirstlane(tid / Np);
  const uint32_t i = tid - l * Np;
  const bool act = l < L && i < N;
  const uint32_t j0 = l * D / L, j1 = (l + 1) * D / L;
  const int use_rand = (run.bl == RAND || run.br == RAND) ? 1 : 0;

  __syncthreads();   // draws of the first generation are being made
  MDE_STAGE_BEGIN
  for (uint32_t gg = 0; gg < n_gens; ++gg) {
    const uint32_t g = g0 + gg;
    MDE_STAGE_WORK(4)
    __syncthreads();
    MDE_STAGE(0)
    // S0: ranks and the top-p list (first is the best).  Four consumer lanes
    // per individual each count the keys below it in a quarter of the
    // population; lane shuffles add the four counts.
    for (uint32_t base = 0; base < N; base += GEN_CONSUMERS / 4) {
      const uint32_t ri = base + (tid >> 2), rq = tid & 3u;
      uint32_t cnt = 0;
      if (ri < N) {
        const uint64_t ki = key_s[ri];
        const uint32_t a = rq * N / 4, b = (rq + 1) * N / 4;
        uint32_t j = a;
        for (; j + 8 <= b; j += 8) {
          uint64_t kv[8];
#pragma unroll
          for (int q = 0; q < 8; ++q) kv[q] = key_s[j + q];
#pragma unroll
          for (int q = 0; q < 8; ++q) cnt += kv[q] < ki ? 1u : 0u;
        }
        for (; j < b; ++j) cnt += key_s[j] < ki ? 1u : 0u;
      }
      // the four counts of an individual sit in one lane quad: two DPP quad
      // permutes (lane ^ 1, lane ^ 2) add them without an LDS round trip
      cnt += (uint32_t)__builtin_amdgcn_mov_dpp((int)cnt, 0xB1, 0xF, 0xF, false);
      cnt += (uint32_t)__builtin_amdgcn_mov_dpp((int)cnt, 0x4E, 0xF, 0xF, false);
      if (ri < N && rq == 0 && cnt < kp) topk[cnt] = ri;
    }
    MDE_STAGE_WORK(5)
    __syncthreads();
    MDE_STAGE(1)
    // S2: mutation, crossover, clip.  Consumer lane c builds quads it = c,
    // c + 512, ... of the generation's N x Q quads (trial it / Q, genes
    // 4 (it mod Q) .. +3): every lane has at most one quad more than any
    // other, and lanes of one trial read neighbouring parts of the same
    // source rows.  A lane's first quad stays in registers for the commit.
    float4 keep = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
    uint32_t ki = 0, kq = 0;
    float kfx = 0.0f;
    if (tid < N * Q) {
      ki = tid / Q;
      kq = tid - ki * Q;
      kfx = fit_s[ki];
    }
    {
      const uint8_t *mg = msk + (g & 1u) * N * Q;
      for (uint32_t it = tid; it < N * Q; it += GEN_CONSUMERS) {
        const uint32_t ti = it == tid ? ki : it / Q, q = it == tid ? kq : it - (it / Q) * Q;
        const uint4 d = dsc[ti];
        const uint32_t r0 = byte_of(d.z, 0), pb = byte_of(d.z, 1);
        const uint32_t ibest = topk[0], ipb = topk[pb];
        const uint32_t ibl = run.bl == RAND ? r0 : (run.bl == BEST ? ibest : (run.bl == PBEST ? ipb : ti));
        const uint32_t ibr = run.br == RAND ? r0 : (run.br == BEST ? ibest : (run.br == PBEST ? ipb : ti));
        if (TRACE && q == 0) {
          int32_t *o = tr.desc + (size_t)(run.fit_off + ti) * 16;
          o[0] = (int32_t)ibl;
          o[1] = (int32_t)ibr;
#pragma unroll
          for (int k = 0; k < 8; ++k) {
            const uint32_t word = k < 4 ? d.x : d.y;
            o[2 + k] = (k / 2) < run.dn ? (int32_t)byte_of(word, k & 3) : -1;
          }
          o[10] = (int32_t)byte_of(d.z, 2);
          o[11] = run.cs == EXP ? (int32_t)(d.z >> 24) : -1;
          o[12] = (int32_t)pb;
          o[13] = use_rand ? (int32_t)r0 : -1;
          o[14] = run.cs == ARITH ? (int32_t)d.w : -1;
          o[15] = 0;
        }
        if (q == 0) fx_s[ti] = fit_s[ti];
        const uint32_t nib = run.cs == BIN ? mg[it] : 0u;
        const float4 uu = trial_quad(pop_s, Dp, D, ti, q, ibl, ibr, d, nib, run, lb, ub);
#pragma unroll
        for (int t = 0; t < 4; ++t) {
          const uint32_t j = 4 * q + t;
          if (j < D) {
            T[j * ts + ti] = comp(uu, t);
            if (TRACE) tr.u[run.pop_off + (size_t)ti * D + j] = comp(uu, t);
          }
        }
        if (it == tid) keep = uu;
      }
    }
    MDE_STAGE_WORK(6)
    __syncthreads();
    MDE_STAGE(2)
    // S3: this part's share of the fitness (producers draw generation g+1)
    if (act) {
      double s0, s1;
      eval_part(tab, p, D, j0, j1, T + i, ts, s0, s1);
      Ps[l * Np + i] = make_double2(s0, s1);
    }
    MDE_STAGE_WORK(7)
    __syncthreads();
    MDE_STAGE(3)
    // S4: greedy selection and commit, by the lanes of S2: each lane sums the
    // parts of its trial (all lanes of a trial take the same decision) and
    // writes its quad back; the quad-0 lane updates fitness and key.
    for (uint32_t it = tid; it < N * Q; it += GEN_CONSUMERS) {
      const uint32_t ti = it == tid ? ki : it / Q, q = it == tid ? kq : it - (it / Q) * Q;
      const float fx = it == tid ? kfx : fx_s[ti];
      double s0 = 0.0, s1 = 0.0;
      for (uint32_t ll = 0; ll < L; ++ll) {
        const double2 v = Ps[ll * Np + ti];
        s0 += v.x;
        s1 += v.y;
      }
      const float f = finish_f32(p, s0, s1);
      const bool a = accept_trial(f, fx);
      if (a) {
        float4 x = keep;
        if (it != tid) {
#pragma unroll
          for (int t = 0; t < 4; ++t) {
            const uint32_t j = 4 * q + t;
            set_comp(x, t, j < D ? T[j * ts + ti] : 0.0f);
          }
        }
        st4(pop_s, ti * Dp + 4 * q, x);
      }
      if (q == 0) {
        if (a) {
          fit_s[ti] = f;
          key_s[ti] = mkkey(f, ti);
        }
        if (TRACE) {
          tr.fu[run.fit_off + ti] = f;
          tr.desc[(size_t)(run.fit_off + ti) * 16 + 15] = a ? 1 : 0;
        }
      }
    }
  }
  MDE_STAGE_WORK(4)
  __syncthreads();
  MDE_STAGE(0)
  MDE_STAGE_END
}

// Persistent generation loop of one run (one workgroup): load the run into
// LDS, run the consumer and producer roles side by side, write the run back.
template <bool TRACE>
__device__ __forceinline__ void gen_body(unsigned char *smem, const RunDev &run, const ProbDev &p,
                                         const unsigned char *__restrict__ tab,
                                         float *__restrict__ pop, float *__restrict__ fit,
                                         uint32_t g0, uint32_t n_gens, uint32_t k0, uint32_t k1,
                                         float lb, float ub,
                                         const TraceArgs &tr) {
  const uint32_t N = run.N, D = run.D, Dp = run.Dp;
  const Lds lay = lds_layout(N, Dp, run.L, run.Np, true);
  float *pop_s = reinterpret_cast<float *>(smem + lay.pop);
  uint64_t *key_s = reinterpret_cast<uint64_t *>(smem + lay.key);
  float *fit_s = reinterpret_cast<float *>(smem + lay.fit);
  const uint32_t tid = threadIdx.x;
  for (uint32_t u = tid; u < N * Dp; u += GEN_THREADS) {
    const uint32_t r = u / Dp, j = u - r * Dp;
    pop_s[u] = j < D ? pop[run.pop_off + (size_t)r * D + j] : 0.0f;
  }
  for (uint32_t r = tid; r < N; r += GEN_THREADS) {
    const float f = fit[run.fit_off + r];
    fit_s[r] = f;
    key_s[r] = mkkey(f, r);
  }
  // the role is uniform per wave (whole waves on either side of GEN_CONSUMERS)
  const bool producer = __builtin_amdgcn_readfirstlane(tid >> 6) >= GEN_CONSUMERS / 64;
  if (producer)
    gen_producers(lay, smem, run, g0, n_gens, k0, k1, tid - GEN_CONSUMERS);
  else
    gen_consumers<TRACE>(lay, smem, run, p, tab, g0, n_gens, lb, ub, tr, tid);
  for (uint32_t u = tid; u < N * D; u += GEN_THREADS) {
    const uint32_t r = u / D, j = u - r * D;
    pop[run.pop_off + u] = pop_s[r * Dp + j];
  }
  for (uint32_t r = tid; r < N; r += GEN_THREADS) fit[run.fit_off + r] = fit_s[r];
}

template <bool TRACE>
__global__ __launch_bounds__(GEN_THREADS) void k_generations(
    const RunDev *__restrict__ runs, const uint32_t *__restrict__ list,
    const ProbDev *__restrict__ probs, const unsigned char *__restrict__ tab,
    float *__restrict__ pop, float *__restrict__ fit, uint32_t g0, uint32_t n_gens, uint32_t k0,
    uint32_t k1, float lb, float ub, TraceArgs tr) {
  extern __shared__ __align__(16) unsigned char smem[];
  const RunDev run = runs[list[blockIdx.x]];
  ProbDev p = probs[run.prob];
  // One copy of the generation loop per function kind: inside each case the
  // kind is a constant, so the loop a workgroup runs holds only its own
  // fitness code (a far smaller instruction footprint than one loop that
  // branches over every kind at every output).
#define MDE_KIND(K)                                                                   \
  case K:                                                                             \
    p.kind = K;                                                                       \
    gen_body<TRACE>(smem, run, p, tab, pop, fit, g0, n_gens, k0, k1, lb, ub, tr);     \
    break;
  switch (p.kind) {
    MDE_KIND(FN_RASTRIGIN)
    MDE_KIND(FN_ROSENBROCK)
    MDE_KIND(FN_ACKLEY)
    MDE_KIND(FN_ELLIPTIC)
    MDE_KIND(FN_SCHWEFEL)
    MDE_KIND(FN_HYBRID)
    default: break;
  }
#undef MDE_KIND
}

// The same generation loop for launches whose runs all have one function
// kind: a kernel that holds a single loop gets a register allocation of its
// own, where the six loops of k_generations share one (for the hybrid, 71
// scalar-register spills against 392).
template <bool TRACE, int KIND>
__global__ __launch_bounds__(GEN_THREADS) void k_generations_kind(
    const RunDev *__restrict__ runs, const uint32_t *__restrict__ list,
    const ProbDev *__restrict__ probs, const unsigned char *__restrict__ tab,
    float *__restrict__ pop, float *__restrict__ fit, uint32_t g0, uint32_t n_gens, uint32_t k0,
    uint32_t k1, float lb, float ub, TraceArgs tr) {
  extern __shared__ __align__(16) unsigned char smem[];
  const RunDev run = runs[list[blockIdx.x]];
  ProbDev p = probs[run.prob];
  p.kind = KIND;
  gen_body<TRACE>(smem, run, p, tab, pop, fit, g0, n_gens, k0, k1, lb, ub, tr);
}

#ifdef MDE_STAGE_CLOCKS
hipError_t read_stage_clocks(void *dst, size_t bytes) {
  return hipMemcpyFromSymbol(dst, HIP_SYMBOL(mde_stage_clk), bytes, 0, hipMemcpyDeviceToHost);
}
#endif

// ---------------------------------------------------------------- best record in float64

constexpr int FIN_BLOCK = 128;

__global__ __launch_bounds__(FIN_BLOCK) void k_finalize(const RunDev *__restrict__ runs,
                                                        const ProbDev *__restrict__ probs,
                                                        const unsigned char *__restrict__ tab,
                                                        const float *__restrict__ pop,
                                                        const float *__restrict__ fit,
                                                        double *__restrict__ best_y,
                                                        float *__restrict__ best_x) {
  __shared__ uint32_t sk[FIN_BLOCK], si[FIN_BLOCK];
  __shared__ double z[MAX_D], t0s[MAX_D], t1s[MAX_D];
  const RunDev run = runs[blockIdx.x];
  if (run.kern == 2) return;  // control runs have their own record kernel
  const ProbDev p = probs[run.prob];
  const uint32_t N = run.N, D = run.D, tid = threadIdx.x;
  uint32_t bk = 0xFFFFFFFFu, bi = 0xFFFFFFFFu;
  for (uint32_t i = tid; i < N; i += FIN_BLOCK) {
    const uint32_t k = okey(fit[run.fit_off + i]);
    if (k < bk || (k == bk && i < bi)) { bk = k; bi = i; }
  }
  sk[tid] = bk;
  si[tid] = bi;
  __syncthreads();
  for (int s = FIN_BLOCK / 2; s > 0; s >>= 1) {
    if (tid < (uint32_t)s) {
      const uint32_t k2 = sk[tid + s], i2 = si[tid + s];
      if (k2 < sk[tid] || (k2 == sk[tid] && i2 < si[tid])) { sk[tid] = k2; si[tid] = i2; }
    }
    __syncthreads();
  }
  const uint32_t b = si[0];
  const float *x = pop + run.pop_off + (size_t)b * D;
  const double *Rt = tab_ptr<double>(tab, p.r64t_off);
  const uint32_t Dr = rt_stride(D);
  const float *o = tab_ptr<float>(tab, p.o_off);
  for (uint32_t j = tid; j < D; j += FIN_BLOCK) {
    double acc = 0.0;
    for (uint32_t k = 0; k < D; ++k) acc = fma(Rt[(size_t)k * Dr + j], (double)x[k] - (double)o[k], acc);
    z[j] = acc;
  }
  __syncthreads();
  for (uint32_t j = tid; j < D; j += FIN_BLOCK) {
    if (p.kind == FN_ROSENBROCK) {
      t0s[j] = j + 1 < D ? h_rosenbrock<double>(z[j], z[j + 1]) : 0.0;
      t1s[j] = 0.0;
    } else {
      elem_term<double>(tab, p, j, z[j], t0s[j], t1s[j]);
    }
  }
  __syncthreads();
  if (tid == 0) {
    double s0 = 0.0, s1 = 0.0;
    for (uint32_t j = 0; j < D; ++j) { s0 += t0s[j]; s1 += t1s[j]; }
    best_y[blockIdx.x] = fn_finish<double>(p, s0, s1);
  }
  for (uint32_t j = tid; j < D; j += FIN_BLOCK) best_x[run.bx_off + j] = x[j];
}

// ---------------------------------------------------------------- theta decode (Alg. 3 decode step)

__device__ __forceinline__ void theta_box(uint32_t n_cs, int k, float &lo, float &hi) {
  lo = k < 2 ? 0.0f : 1.0f;
  hi = k < 2 ? 1.0f : (k < 5 ? 5.0f : 1.0f + (float)n_cs);
}

__device__ __forceinline__ void decode_into(RunDev &r, const float *t, uint32_t n_cs) {
  r.F = t[0];
  r.CR = t[1];
  r.bl = min((int)floorf(t[2]), 4);
  r.br = min((int)floorf(t[3]), 4);
  r.dn = min((int)floorf(t[4]), 4);
  r.cs = min((int)floorf(t[5]), (int)n_cs);
}

__global__ void k_decode(RunDev *__restrict__ runs, float *__restrict__ theta, uint32_t n,
                         uint32_t n_cs) {
  const uint32_t r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= n) return;
  float t[6];
#pragma unroll
  for (int k = 0; k < 6; ++k) {
    float lo, hi;
    theta_box(n_cs, k, lo, hi);
    float v = theta[r * 6 + k];
    if (v != v) v = lo;
    v = fminf(fmaxf(v, lo), hi);
    t[k] = v;
    theta[r * 6 + k] = v;
  }
  decode_into(runs[r], t, n_cs);
}

// ---------------------------------------------------------------- evolver (Alg. 3)

__global__ void k_outer_init(float *__restrict__ X, double *__restrict__ y, uint32_t P,
                             uint32_t stream, uint32_t k0, uint32_t k1, uint32_t n_cs) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= P) return;
  const uint4 w0 = philox(0, i, INIT_PHASE, stream | OUTER_BIT, k0, k1);
  const uint4 w1 = philox(1, i, INIT_PHASE, stream | OUTER_BIT, k0, k1);
  const uint32_t w[8] = {w0.x, w0.y, w0.z, w0.w, w1.x, w1.y, w1.z, w1.w};
#pragma unroll
  for (int k = 0; k < 6; ++k) {
    float lo, hi;
    theta_box(n_cs, k, lo, hi);
    const double u0 = (double)(w[k] >> 8) * 0x1p-24;
    X[i * 6 + k] = (float)((double)lo + ((double)hi - (double)lo) * u0);
  }
  y[i] = __longlong_as_double(0x7FF0000000000000ll);
}

// DE/rand/1/bin trial of the evolver: F = 0.5, CR = 0.9, same word map as an
// executor with theta = (0.5, 0.9, rand, rand, 1, bin).
__global__ void k_outer_trial(const float *__restrict__ X, float *__restrict__ U,
                              RunDev *__restrict__ runs, uint32_t P, uint32_t g_o,
                              uint32_t stream, uint32_t k0, uint32_t k1, uint32_t n_cs, float F,
                              float CR) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= P) return;
  const uint32_t st = stream | OUTER_BIT;
  const uint4 wa = philox(0, i, g_o, st, k0, k1);
  const uint4 wc = philox(2, i, g_o, st, k0, k1);
  const uint4 g0w = philox(3, i, g_o, st, k0, k1);
  const uint4 g1w = philox(4, i, g_o, st, k0, k1);
  uint32_t w[12] = {wa.x, wa.y, wa.z, wa.w, 0, 0, 0, 0, wc.x, wc.y, wc.z, wc.w};
  uint32_t dr[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
  sample_distinct(w, 3, i, P, dr);
  const uint32_t jr = lemire(w[W_JRAND], 6);
  const uint32_t gw[8] = {g0w.x, g0w.y, g0w.z, g0w.w, g1w.x, g1w.y, g1w.z, g1w.w};
  float t[6];
#pragma unroll
  for (int k = 0; k < 6; ++k) {
    const float v = X[dr[0] * 6 + k] + F * (X[dr[1] * 6 + k] - X[dr[2] * 6 + k]);
    const bool take = (unit_oc(gw[k]) <= CR) || ((uint32_t)k == jr);
    float u = take ? v : X[i * 6 + k];
    float lo, hi;
    theta_box(n_cs, k, lo, hi);
    u = fminf(fmaxf(u, lo), hi);
    t[k] = u;
    U[i * 6 + k] = u;
  }
  decode_into(runs[i], t, n_cs);
}

__global__ void k_outer_select(float *__restrict__ X, double *__restrict__ y,
                               const float *__restrict__ U, const double *__restrict__ y_run,
                               double *__restrict__ y_trial, float *__restrict__ bxo,
                               const float *__restrict__ best_x, const RunDev *__restrict__ runs,
                               uint32_t P, uint32_t take_all) {
  const uint32_t i = blockIdx.x;
  if (i >= P) return;
  const double yt = y_run[i];
  const bool acc = take_all != 0 || accept_trial_d(yt, y[i]);
  __syncthreads();
  const RunDev run = runs[i];
  if (acc) {
    for (uint32_t j = threadIdx.x; j < run.D; j += blockDim.x) bxo[run.bx_off + j] = best_x[run.bx_off + j];
    if (threadIdx.x < 6) X[i * 6 + threadIdx.x] = U[i * 6 + threadIdx.x];
  }
  if (threadIdx.x == 0) {
    y_trial[i] = yt;
    if (acc) y[i] = yt;
  }
}

// Particle-swarm evolver (the paper's supplement, S.III): move every particle
// from its position U, velocity V, personal best X and the swarm's best X[g],
// v = w v + c1 r1 (p - x) + c2 r2 (g - x), x = clip(x + v) in float32 in that
// order; r1, r2 are Philox words k and 6 + k of (particle, g_o).  The new
// position is decoded into the particle's executor.
constexpr float PSO_W = 0.729f, PSO_C1 = 1.49f, PSO_C2 = 1.49f;

__global__ void k_pso_move(float *__restrict__ U, float *__restrict__ V,
                           const float *__restrict__ X, const int32_t *__restrict__ gbest,
                           RunDev *__restrict__ runs, uint32_t P, uint32_t g_o, uint32_t stream,
                           uint32_t k0, uint32_t k1, uint32_t n_cs) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= P) return;
  const uint32_t st = stream | OUTER_BIT;
  const uint4 a = philox(0, i, g_o, st, k0, k1);
  const uint4 b = philox(1, i, g_o, st, k0, k1);
  const uint4 c = philox(2, i, g_o, st, k0, k1);
  const uint32_t w[12] = {a.x, a.y, a.z, a.w, b.x, b.y, b.z, b.w, c.x, c.y, c.z, c.w};
  const uint32_t g = (uint32_t)gbest[0];
  float t[6];
#pragma unroll
  for (int k = 0; k < 6; ++k) {
    const float r1 = (float)(w[k] >> 8) * 0x1p-24f;
    const float r2 = (float)(w[6 + k] >> 8) * 0x1p-24f;
    const float x = U[i * 6 + k];
    const float pa = (PSO_C1 * r1) * (X[i * 6 + k] - x);
    const float ga = (PSO_C2 * r2) * (X[g * 6 + k] - x);
    const float v = ((PSO_W * V[i * 6 + k]) + pa) + ga;
    float lo, hi;
    theta_box(n_cs, k, lo, hi);
    const float xn = fminf(fmaxf(x + v, lo), hi);
    V[i * 6 + k] = v;
    U[i * 6 + k] = xn;
    t[k] = xn;
  }
  decode_into(runs[i], t, n_cs);
}

// Competitive swarm evolver (the paper's supplement, S.III; Cheng and Jin's
// optimiser without the mean-position term): one workgroup pairs the P
// particles by sorting Philox word 12 of (particle, g_o) with the index
// breaking ties, pairing sorted positions 2k and 2k + 1; in each pair the
// particle first in (score, index) order wins and stays, the loser moves
// v = r1 v + r2 (x_w - x_l), x = clip(x + v) in float32 in that order (r1, r2:
// Philox words k and 6 + k of the loser's (particle, g_o)).  Positions X are
// updated in place, copied to U and decoded into the executors.
constexpr uint32_t CSO_MAX_P = 1024;

__global__ __launch_bounds__(CSO_MAX_P) void k_cso_move(
    float *__restrict__ X, float *__restrict__ V, float *__restrict__ U,
    const double *__restrict__ y, RunDev *__restrict__ runs, uint32_t P, uint32_t g_o,
    uint32_t stream, uint32_t k0, uint32_t k1, uint32_t n_cs) {
  __shared__ uint64_t key[CSO_MAX_P];
  __shared__ uint32_t at[CSO_MAX_P];
  const uint32_t i = threadIdx.x;
  const uint32_t st = stream | OUTER_BIT;
  if (i < P) key[i] = ((uint64_t)philox(3, i, g_o, st, k0, k1).x << 32) | i;
  __syncthreads();
  uint32_t pos = 0;
  if (i < P) {
    const uint64_t ki = key[i];
    for (uint32_t j = 0; j < P; ++j) pos += key[j] < ki ? 1u : 0u;
    at[pos] = i;
  }
  __syncthreads();
  bool loser = false;
  uint32_t w = 0;
  if (i < P && (pos ^ 1u) < P && !((P & 1u) && pos == P - 1)) {
    const uint32_t j = at[pos ^ 1u];
    double yi = y[i], yj = y[j];
    if (yi != yi) yi = __longlong_as_double(0x7FF0000000000000LL);
    if (yj != yj) yj = __longlong_as_double(0x7FF0000000000000LL);
    loser = yj < yi || (yj == yi && j < i);
    w = j;
  }
  // every thread has read the positions it needs before any loser writes
  float xw[6];
  if (i < P) {
#pragma unroll
    for (int k = 0; k < 6; ++k) xw[k] = X[w * 6 + k];
  }
  __syncthreads();
  if (i >= P) return;
  float t[6];
  if (loser) {
    const uint4 a = philox(0, i, g_o, st, k0, k1);
    const uint4 b = philox(1, i, g_o, st, k0, k1);
    const uint4 c = philox(2, i, g_o, st, k0, k1);
    const uint32_t wd[12] = {a.x, a.y, a.z, a.w, b.x, b.y, b.z, b.w, c.x, c.y, c.z, c.w};
#pragma unroll
    for (int k = 0; k < 6; ++k) {
      const float r1 = (float)(wd[k] >> 8) * 0x1p-24f;
      const float r2 = (float)(wd[6 + k] >> 8) * 0x1p-24f;
      const float x = X[i * 6 + k];
      const float v = (r1 * V[i * 6 + k]) + (r2 * (xw[k] - x));
      float lo, hi;
      theta_box(n_cs, k, lo, hi);
      t[k] = fminf(fmaxf(x + v, lo), hi);
      V[i * 6 + k] = v;
    }
  } else {
#pragma unroll
    for (int k = 0; k < 6; ++k) t[k] = X[i * 6 + k];
  }
#pragma unroll
  for (int k = 0; k < 6; ++k) {
    X[i * 6 + k] = t[k];
    U[i * 6 + k] = t[k];
  }
  decode_into(runs[i], t, n_cs);
}

// Separable natural evolution strategy (the paper's supplement, S.III;
// Schaul, Glasmachers and Schmidhuber's SNES).  State: mu = V[0..5], sigma =
// V[6..11] (float32).  Normals s of sample k are the Box-Muller transform of
// Philox words 2m, 2m + 1 of (k, g_o) on the evolver's stream, in float64;
// the sample is z = mu + sigma s rounded once to float32, clipped to the
// theta box and decoded into executor k.  The update ranks the samples by
// (score, index), weights them with the rank utilities and moves
// mu += sigma sum_r u_r s_(r), sigma *= exp(eta_sigma / 2 sum_r u_r (s^2 - 1)),
// all in float64 with the sums taken in rank order by one lane per
// coordinate.
constexpr uint32_t NES_MAX_P = 1024;

__device__ __forceinline__ void nes_normals(uint32_t k, uint32_t g_o, uint32_t st, uint32_t k0,
                                            uint32_t k1, double (&s)[6]) {
  const uint4 a = philox(0, k, g_o, st, k0, k1);
  const uint4 b = philox(1, k, g_o, st, k0, k1);
  const uint32_t w[6] = {a.x, a.y, a.z, a.w, b.x, b.y};
#pragma unroll
  for (int m = 0; m < 3; ++m) {
    const double u1 = (double)((w[2 * m] >> 8) + 1u) * 0x1p-24;
    const double u2 = (double)(w[2 * m + 1] >> 8) * 0x1p-24;
    const double rho = sqrt(-2.0 * log(u1));
    const double ang = (2.0 * 3.141592653589793) * u2;
    s[2 * m] = rho * cos(ang);
    s[2 * m + 1] = rho * sin(ang);
  }
}

__global__ void k_nes_init(float *__restrict__ V, uint32_t n_cs) {
  const int k = (int)threadIdx.x;
  if (k >= 6) return;
  float lo, hi;
  theta_box(n_cs, k, lo, hi);
  V[k] = (lo + hi) / 2.0f;
  V[6 + k] = (hi - lo) / 4.0f;
}

__global__ void k_nes_sample(float *__restrict__ U, const float *__restrict__ V,
                             RunDev *__restrict__ runs, uint32_t P, uint32_t g_o,
                             uint32_t stream, uint32_t k0, uint32_t k1, uint32_t n_cs) {
  const uint32_t k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= P) return;
  double s[6];
  nes_normals(k, g_o, stream | OUTER_BIT, k0, k1, s);
  float t[6];
#pragma unroll
  for (int j = 0; j < 6; ++j) {
    const float z = (float)((double)V[j] + (double)V[6 + j] * s[j]);
    float lo, hi;
    theta_box(n_cs, j, lo, hi);
    t[j] = fminf(fmaxf(z, lo), hi);
    U[k * 6 + j] = t[j];
  }
  decode_into(runs[k], t, n_cs);
}

__global__ __launch_bounds__(NES_MAX_P) void k_nes_update(
    const double *__restrict__ y, float *__restrict__ V, uint32_t P, uint32_t g_o,
    uint32_t stream, uint32_t k0, uint32_t k1, double eta_sigma) {
  __shared__ double s_all[NES_MAX_P * 6];
  __shared__ double util[NES_MAX_P];
  __shared__ uint32_t at[NES_MAX_P];
  const uint32_t k = threadIdx.x;
  if (k < P) {
    double s[6];
    nes_normals(k, g_o, stream | OUTER_BIT, k0, k1, s);
#pragma unroll
    for (int j = 0; j < 6; ++j) s_all[k * 6 + j] = s[j];
    double yk = y[k];
    if (yk != yk) yk = __longlong_as_double(0x7FF0000000000000LL);
    uint32_t r = 0;
    for (uint32_t q = 0; q < P; ++q) {
      double yq = y[q];
      if (yq != yq) yq = __longlong_as_double(0x7FF0000000000000LL);
      r += (yq < yk || (yq == yk && q < k)) ? 1u : 0u;
    }
    at[r] = k;
    // utility weight before normalisation of rank r + 1
    util[k] = fmax(0.0, log((double)P / 2.0 + 1.0) - log((double)(k + 1)));
  }
  __syncthreads();
  __shared__ double tot;
  if (k == 0) {
    double t = 0.0;
    for (uint32_t q = 0; q < P; ++q) t = t + util[q];
    tot = t;
  }
  __syncthreads();
  if (k < P) util[k] = util[k] / tot - 1.0 / (double)P;
  __syncthreads();
  if (k < 6) {
    double gmu = 0.0, gsig = 0.0;
    for (uint32_t r = 0; r < P; ++r) {
      const double sk = s_all[at[r] * 6 + k];
      gmu = gmu + util[r] * sk;
      gsig = gsig + util[r] * (sk * sk - 1.0);
    }
    const double mu = (double)V[k], sig = (double)V[6 + k];
    V[k] = (float)(mu + sig * gmu);
    V[6 + k] = (float)(sig * exp((eta_sigma / 2.0) * gsig));
  }
}

__global__ void k_outer_best(const double *__restrict__ y, uint32_t P, int32_t *__restrict__ out) {
  __shared__ double sv[256];
  __shared__ int32_t si[256];
  const uint32_t tid = threadIdx.x;
  double bv = __longlong_as_double(0x7FF0000000000000ll);
  int32_t bi = 0x7FFFFFFF;
  for (uint32_t i = tid; i < P; i += 256) {
    double v = y[i];
    if (v != v) v = __longlong_as_double(0x7FF0000000000000ll);
    if (v < bv || (v == bv && (int32_t)i < bi)) { bv = v; bi = (int32_t)i; }
  }
  sv[tid] = bv;
  si[tid] = bi;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (tid < (uint32_t)s) {
      if (sv[tid + s] < sv[tid] || (sv[tid + s] == sv[tid] && si[tid + s] < si[tid])) {
        sv[tid] = sv[tid + s];
        si[tid] = si[tid + s];
      }
    }
    __syncthreads();
  }
  if (tid == 0) out[0] = si[0] == 0x7FFFFFFF ? 0 : si[0];
}

// Rt[k][j] = R[j][k] in float64, row stride Dr >= D + 16 (zero padding so a
// block of 16 outputs starting anywhere below D stays inside the row).
__global__ void k_tables64(const float *__restrict__ R, double *__restrict__ Rt, uint32_t D,
                           uint32_t Dr) {
  const uint32_t u = blockIdx.x * blockDim.x + threadIdx.x;
  if (u >= D * Dr) return;
  const uint32_t k = u / Dr, j = u - k * Dr;
  Rt[u] = j < D ? (double)R[(size_t)j * D + k] : 0.0;
}

// ---------------------------------------------------------------- launchers

hipError_t launch_tables64(const float *R, double *Rt, uint32_t D, hipStream_t s) {
  const uint32_t n = D * rt_stride(D);
  hipLaunchKernelGGL(k_tables64, dim3((n + 255) / 256), dim3(256), 0, s, R, Rt, D, rt_stride(D));
  return hipGetLastError();
}

#define MDE_KINDS(X)                                                                        \
  X(FN_RASTRIGIN) X(FN_ROSENBROCK) X(FN_ACKLEY) X(FN_ELLIPTIC) X(FN_SCHWEFEL) X(FN_HYBRID)

hipError_t set_lds_limits() {
  const void *ks[14] = {(const void *)k_generations<false>, (const void *)k_generations<true>,
#define MDE_KIND_PTRS(K) (const void *)k_generations_kind<false, K>, \
                         (const void *)k_generations_kind<true, K>,
                        MDE_KINDS(MDE_KIND_PTRS)};
#undef MDE_KIND_PTRS
  hipError_t e = hipSuccess;
  for (const void *k : ks) {
    e = hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, LDS_BUDGET);
    if (e != hipSuccess) return e;
  }
  e = hipFuncSetAttribute((const void *)k_init, hipFuncAttributeMaxDynamicSharedMemorySize,
                          LDS_BUDGET);
  if (e != hipSuccess) return e;
  return set_lds_limits_mfma();
}

hipError_t launch_init(const LaunchArgs &a, double lb, double ub) {
  hipLaunchKernelGGL(k_init, dim3(a.n_runs), dim3(INIT_THREADS), a.init_lds_bytes, a.stream,
                     a.runs, a.probs, a.tab, a.pop, a.fit, a.k0, a.k1, lb, ub);
  return hipGetLastError();
}

hipError_t launch_generations(const LaunchArgs &a, const uint32_t *list, uint32_t n,
                              uint32_t g0, uint32_t n_gens, float lb, float ub, TraceArgs tr) {
  if (n == 0) return hipSuccess;
  const bool trace = tr.u != nullptr;
#define MDE_LAUNCH_KIND(T, K)                                                                   \
  hipLaunchKernelGGL(HIP_KERNEL_NAME(k_generations_kind<T, K>), dim3(n), dim3(GEN_THREADS),     \
                     a.lds_bytes, a.stream, a.runs, list, a.probs, a.tab, a.pop, a.fit, g0,      \
                     n_gens, a.k0, a.k1, lb, ub, tr)
#define MDE_KIND_CASE(K)                      \
  case K:                                     \
    if (trace) MDE_LAUNCH_KIND(true, K);      \
    else MDE_LAUNCH_KIND(false, K);           \
    return hipGetLastError();
  switch (a.lane_kind) {
    MDE_KINDS(MDE_KIND_CASE)
    default: break;
  }
#undef MDE_KIND_CASE
#undef MDE_LAUNCH_KIND
  if (trace)
    hipLaunchKernelGGL(HIP_KERNEL_NAME(k_generations<true>), dim3(n), dim3(GEN_THREADS),
                       a.lds_bytes, a.stream, a.runs, list, a.probs, a.tab, a.pop, a.fit, g0,
                       n_gens, a.k0, a.k1, lb, ub, tr);
  else
    hipLaunchKernelGGL(HIP_KERNEL_NAME(k_generations<false>), dim3(n), dim3(GEN_THREADS),
                       a.lds_bytes, a.stream, a.runs, list, a.probs, a.tab, a.pop, a.fit, g0,
                       n_gens, a.k0, a.k1, lb, ub, tr);
  return hipGetLastError();
}

hipError_t launch_finalize(const LaunchArgs &a, double *best_y, float *best_x) {
  hipLaunchKernelGGL(k_finalize, dim3(a.n_runs), dim3(FIN_BLOCK), 0, a.stream, a.runs, a.probs,
                     a.tab, a.pop, a.fit, best_y, best_x);
  return hipGetLastError();
}

hipError_t launch_decode(RunDev *runs, float *theta, uint32_t n, uint32_t n_cs,
                         hipStream_t s) {
  hipLaunchKernelGGL(k_decode, dim3((n + 63) / 64), dim3(64), 0, s, runs, theta, n, n_cs);
  return hipGetLastError();
}

hipError_t launch_outer_init(float *X, double *y, uint32_t P, uint32_t stream, uint32_t k0,
                             uint32_t k1, uint32_t n_cs, hipStream_t s) {
  hipLaunchKernelGGL(k_outer_init, dim3((P + 63) / 64), dim3(64), 0, s, X, y, P, stream, k0, k1,
                     n_cs);
  return hipGetLastError();
}

hipError_t launch_outer_trial(const float *X, float *U, RunDev *runs, uint32_t P, uint32_t g_o,
                              uint32_t stream, uint32_t k0, uint32_t k1, uint32_t n_cs,
                              hipStream_t s) {
  hipLaunchKernelGGL(k_outer_trial, dim3((P + 63) / 64), dim3(64), 0, s, X, U, runs, P, g_o,
                     stream, k0, k1, n_cs, 0.5f, 0.9f);
  return hipGetLastError();
}

hipError_t launch_outer_select(float *X, double *y, const float *U, const double *y_run,
                               double *y_trial, float *bxo, const float *best_x,
                               const RunDev *runs, uint32_t P, bool take_all, hipStream_t s) {
  hipLaunchKernelGGL(k_outer_select, dim3(P), dim3(64), 0, s, X, y, U, y_run, y_trial, bxo, best_x,
                     runs, P, take_all ? 1u : 0u);
  return hipGetLastError();
}

hipError_t launch_pso_move(float *U, float *V, const float *X, const int32_t *gbest, RunDev *runs,
                           uint32_t P, uint32_t g_o, uint32_t stream, uint32_t k0, uint32_t k1,
                           uint32_t n_cs, hipStream_t s) {
  hipLaunchKernelGGL(k_pso_move, dim3((P + 63) / 64), dim3(64), 0, s, U, V, X, gbest, runs, P, g_o,
                     stream, k0, k1, n_cs);
  return hipGetLastError();
}

hipError_t launch_nes_init(float *V, uint32_t n_cs, hipStream_t s) {
  hipLaunchKernelGGL(k_nes_init, dim3(1), dim3(64), 0, s, V, n_cs);
  return hipGetLastError();
}

hipError_t launch_nes_sample(float *U, const float *V, RunDev *runs, uint32_t P, uint32_t g_o,
                             uint32_t stream, uint32_t k0, uint32_t k1, uint32_t n_cs,
                             hipStream_t s) {
  hipLaunchKernelGGL(k_nes_sample, dim3((P + 63) / 64), dim3(64), 0, s, U, V, runs, P, g_o, stream,
                     k0, k1, n_cs);
  return hipGetLastError();
}

hipError_t launch_nes_update(const double *y, float *V, uint32_t P, uint32_t g_o, uint32_t stream,
                             uint32_t k0, uint32_t k1, double eta_sigma, hipStream_t s) {
  if (P > NES_MAX_P) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_nes_update, dim3(1), dim3(((P + 63) / 64) * 64), 0, s, y, V, P, g_o, stream,
                     k0, k1, eta_sigma);
  return hipGetLastError();
}

hipError_t launch_cso_move(float *X, float *V, float *U, const double *y, RunDev *runs,
                           uint32_t P, uint32_t g_o, uint32_t stream, uint32_t k0, uint32_t k1,
                           uint32_t n_cs, hipStream_t s) {
  if (P > CSO_MAX_P) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_cso_move, dim3(1), dim3(((P + 63) / 64) * 64), 0, s, X, V, U, y, runs, P,
                     g_o, stream, k0, k1, n_cs);
  return hipGetLastError();
}

hipError_t launch_outer_best(const double *y, uint32_t P, int32_t *out, hipStream_t s) {
  hipLaunchKernelGGL(k_outer_best, dim3(1), dim3(256), 0, s, y, P, out);
  return hipGetLastError();
}

}  // namespace mde
