// HIP kernels of the MetaDE inner-DE path for gfx950.
//
// One workgroup owns one executor run for the whole launch: its population,
// fitness, ranking and trial descriptors live in LDS, and the generation loop
// of Alg. 2 runs inside the kernel (no grid-wide synchronisation).  Trials are
// built and evaluated in chunks of C rows when the whole trial matrix does
// not fit beside the population; accepted rows of earlier chunks then wait in
// a global buffer until the synchronous commit at the end of the generation.
#include "device.h"
#include "kernels.h"

namespace mde {

__device__ __forceinline__ float4 ld4(const float *s, uint32_t idx) {
  return *reinterpret_cast<const float4 *>(s + idx);
}
__device__ __forceinline__ void st4(float *s, uint32_t idx, float4 v) {
  *reinterpret_cast<float4 *>(s + idx) = v;
}
__device__ __forceinline__ float comp(const float4 &v, int t) {
  return t == 0 ? v.x : (t == 1 ? v.y : (t == 2 ? v.z : v.w));
}
__device__ __forceinline__ void set_comp(float4 &v, int t, float x) {
  if (t == 0) v.x = x; else if (t == 1) v.y = x; else if (t == 2) v.z = x; else v.w = x;
}

// Fitness of nC staged rows Y (y = u - o in float64, row stride ys) into
// out[il].  Plain path: z = R y accumulated in float64 (y is exact, so a
// small z_j that cancels between large products keeps its relative accuracy),
// z rounded once to float32, element terms in float32 summed four at a time,
// the partial sums accumulated in float64.
template <int BLOCK>
__device__ void eval_rows(const ProbDev &p, uint32_t D, uint32_t Dp, uint32_t ys, uint32_t nC,
                          const double *Y, float *Z, double2 *P, float *out) {
  const uint32_t tid = threadIdx.x;
  const uint32_t Q = Dp / 4;
  for (uint32_t u = tid; u < nC * D; u += BLOCK) {
    const uint32_t j = u / nC, il = u - j * nC;
    const double *Rj = p.R64 + (size_t)j * D;
    const double *y = Y + il * ys;
    double acc = 0.0;
    for (uint32_t k = 0; k < D; ++k) acc = fma(Rj[k], y[k], acc);
    Z[il * Dp + j] = (float)acc;
  }
  __syncthreads();
  for (uint32_t u = tid; u < nC * Q; u += BLOCK) {
    const uint32_t il = u / Q, q = u - il * Q;
    float s0 = 0.0f, s1 = 0.0f;
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const uint32_t j = 4 * q + t;
      if (j < D) {
        float a, b;
        fn_term<float>(p, Z + il * Dp, j, a, b);
        s0 += a;
        s1 += b;
      }
    }
    P[il * Q + q] = make_double2((double)s0, (double)s1);
  }
  __syncthreads();
  for (uint32_t il = tid; il < nC; il += BLOCK) {
    double s0 = 0.0, s1 = 0.0;
    for (uint32_t q = 0; q < Q; ++q) {
      const double2 v = P[il * Q + q];
      s0 += v.x;
      s1 += v.y;
    }
    out[il] = p.kind == FN_ACKLEY ? fn_finish<float>(p, (float)s0, (float)s1)
                                  : (float)(s0 + (double)p.bias);
  }
}

// ---------------------------------------------------------------- init (Alg. 2, lines 1-2)

template <int BLOCK>
__global__ __launch_bounds__(BLOCK) void k_init(const RunDev *__restrict__ runs,
                                                const ProbDev *__restrict__ probs,
                                                float *__restrict__ pop, float *__restrict__ fit,
                                                uint32_t k0, uint32_t k1, double lb, double ub) {
  extern __shared__ __align__(16) unsigned char smem[];
  const RunDev run = runs[blockIdx.x];
  const ProbDev p = probs[run.prob];
  const uint32_t N = run.N, D = run.D, Dp = run.Dp, C = run.C, Q = Dp / 4;
  const Lds L = lds_layout(N, Dp, C);
  float *pop_s = reinterpret_cast<float *>(smem + L.pop);
  double *Y = reinterpret_cast<double *>(smem + L.Y);
  float *Z = reinterpret_cast<float *>(smem + L.Z);
  double2 *P = reinterpret_cast<double2 *>(smem + L.P);
  float *fu_s = reinterpret_cast<float *>(smem + L.fu);
  const uint32_t tid = threadIdx.x;

  // x = lb + (ub - lb) u0, u0 = (w >> 8) 2^-24, in float64, rounded once.
  for (uint32_t u = tid; u < N * Q; u += BLOCK) {
    const uint32_t i = u / Q, q = u - i * Q;
    const uint4 w = philox(q, i, INIT_PHASE, run.stream, k0, k1);
    float4 x;
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const uint32_t j = 4 * q + t;
      const double u0 = (double)(word_of(w, t) >> 8) * 0x1p-24;
      set_comp(x, t, j < D ? (float)(lb + (ub - lb) * u0) : 0.0f);
    }
    st4(pop_s, i * Dp + 4 * q, x);
  }
  __syncthreads();
  for (uint32_t c0 = 0; c0 < N; c0 += C) {
    const uint32_t nC = min(C, N - c0);
    for (uint32_t u = tid; u < nC * Q; u += BLOCK) {
      const uint32_t il = u / Q, q = u - il * Q;
      const float4 x = ld4(pop_s, (c0 + il) * Dp + 4 * q);
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const uint32_t j = 4 * q + t;
        Y[il * L.ys + j] = j < D ? (double)comp(x, t) - (double)p.o[j] : 0.0;
      }
    }
    __syncthreads();
    eval_rows<BLOCK>(p, D, Dp, L.ys, nC, Y, Z, P, fu_s + c0);
    __syncthreads();
  }
  for (uint32_t u = tid; u < N * D; u += BLOCK) {
    const uint32_t i = u / D, j = u - i * D;
    pop[run.pop_off + u] = pop_s[i * Dp + j];
  }
  for (uint32_t i = tid; i < N; i += BLOCK) fit[run.fit_off + i] = fu_s[i];
}

// ---------------------------------------------------------------- generations (Alg. 2, lines 6-12)

template <int BLOCK>
__global__ __launch_bounds__(BLOCK) void k_generations(
    const RunDev *__restrict__ runs, const ProbDev *__restrict__ probs, float *__restrict__ pop,
    float *__restrict__ fit, uint32_t g0, uint32_t n_gens, uint32_t k0, uint32_t k1, float lb,
    float ub, float *__restrict__ pending, TraceArgs tr) {
  extern __shared__ __align__(16) unsigned char smem[];
  const RunDev run = runs[blockIdx.x];
  const ProbDev p = probs[run.prob];
  const uint32_t N = run.N, D = run.D, Dp = run.Dp, C = run.C, Q = Dp / 4, kp = run.kp;
  const Lds L = lds_layout(N, Dp, C);
  float *pop_s = reinterpret_cast<float *>(smem + L.pop);
  float *fit_s = reinterpret_cast<float *>(smem + L.fit);
  uint32_t *topk = reinterpret_cast<uint32_t *>(smem + L.topk);
  uint4 *desc = reinterpret_cast<uint4 *>(smem + L.desc);
  float *T = reinterpret_cast<float *>(smem + L.T);
  double *Y = reinterpret_cast<double *>(smem + L.Y);
  float *Z = reinterpret_cast<float *>(smem + L.Z);
  double2 *P = reinterpret_cast<double2 *>(smem + L.P);
  float *fu_s = reinterpret_cast<float *>(smem + L.fu);
  int *acc_s = reinterpret_cast<int *>(smem + L.acc);
  const uint32_t tid = threadIdx.x;
  const bool chunked = C < N;
  float *pend = pending + run.pend_off;
  const float F = run.F, CR = run.CR;
  const int bl = run.bl, br = run.br, dn = run.dn, cs = run.cs;
  const int use_rand = (bl == RAND || br == RAND) ? 1 : 0;
  const int m = use_rand + 2 * dn;

  for (uint32_t u = tid; u < N * Dp; u += BLOCK) {
    const uint32_t i = u / Dp, j = u - i * Dp;
    pop_s[u] = j < D ? pop[run.pop_off + (size_t)i * D + j] : 0.0f;
  }
  for (uint32_t i = tid; i < N; i += BLOCK) fit_s[i] = fit[run.fit_off + i];

  for (uint32_t gg = 0; gg < n_gens; ++gg) {
    const uint32_t g = g0 + gg;
    __syncthreads();
    // (1) ranking by (fitness, index): best and the top-p set
    for (uint32_t i = tid; i < N; i += BLOCK) {
      const uint32_t ki = okey(fit_s[i]);
      uint32_t rank = 0;
      for (uint32_t j = 0; j < N; ++j) {
        const uint32_t kj = okey(fit_s[j]);
        rank += (kj < ki || (kj == ki && j < i)) ? 1u : 0u;
      }
      if (rank < kp) topk[rank] = i;
    }
    __syncthreads();
    // (2) per-target descriptors: index draws, pbest pick, j_rand / n, K, L
    for (uint32_t i = tid; i < N; i += BLOCK) {
      uint32_t w[12];
      const uint4 wa = philox(0, i, g, run.stream, k0, k1);
      const uint4 wc = philox(2, i, g, run.stream, k0, k1);
      w[0] = wa.x; w[1] = wa.y; w[2] = wa.z; w[3] = wa.w;
      if (m > 4) {
        const uint4 wb = philox(1, i, g, run.stream, k0, k1);
        w[4] = wb.x; w[5] = wb.y; w[6] = wb.z; w[7] = wb.w;
      } else {
        w[4] = w[5] = w[6] = w[7] = 0;
      }
      w[8] = wc.x; w[9] = wc.y; w[10] = wc.z; w[11] = wc.w;
      uint32_t dr[9];
#pragma unroll
      for (int k = 0; k < 9; ++k) dr[k] = 0;
      sample_distinct(w, m, i, N, dr);
      const int r0 = use_rand ? (int)dr[0] : -1;
      uint32_t pr[8];
#pragma unroll
      for (int k = 0; k < 8; ++k) pr[k] = (k < 2 * dn) ? dr[use_rand + k] : 0u;
      const uint32_t pb_rank = lemire(w[W_PBEST], kp);
      const uint32_t ipb = topk[pb_rank];
      const uint32_t ibest = topk[0];
      auto resolve = [&](int code) -> uint32_t {
        return code == RAND ? (uint32_t)r0 : (code == BEST ? ibest : (code == PBEST ? ipb : i));
      };
      const uint32_t ibl = resolve(bl), ibr = resolve(br);
      const uint32_t jn = lemire(w[W_JRAND], D);
      const float K = unit_oc(w[W_K]);
      uint32_t Lx = 1;
      if (cs == EXP) {
        // censored geometric length: continue while the t-th uniform <= CR
        bool go = true;
        uint32_t blk = W_GENE0 / 4;
        while (go && Lx < D) {
          const uint4 wr = philox(blk++, i, g, run.stream, k0, k1);
#pragma unroll
          for (int t = 0; t < 4; ++t) {
            if (go && Lx < D) {
              if (unit_oc(word_of(wr, t)) <= CR) ++Lx; else go = false;
            }
          }
        }
      }
      uint4 d;
      d.x = ibl | (ibr << 8) | (jn << 16) | (Lx << 24);
      d.y = pr[0] | (pr[1] << 8) | (pr[2] << 16) | (pr[3] << 24);
      d.z = pr[4] | (pr[5] << 8) | (pr[6] << 16) | (pr[7] << 24);
      d.w = __float_as_uint(K);
      desc[i] = d;
      if (tr.desc) {
        int32_t *o = tr.desc + (size_t)(run.fit_off + i) * 16;
        o[0] = (int32_t)ibl;
        o[1] = (int32_t)ibr;
#pragma unroll
        for (int k = 0; k < 8; ++k) o[2 + k] = (k < 2 * dn) ? (int32_t)pr[k] : -1;
        o[10] = (int32_t)jn;
        o[11] = cs == EXP ? (int32_t)Lx : -1;
        o[12] = (int32_t)pb_rank;
        o[13] = r0;
        o[14] = cs == ARITH ? (int32_t)__float_as_uint(K) : -1;
        o[15] = 0;
      }
    }
    __syncthreads();
    // (3) trials chunk by chunk: mutation (Eq. 12), crossover (Eqs. 8-10), clip, fitness
    for (uint32_t c0 = 0; c0 < N; c0 += C) {
      const uint32_t nC = min(C, N - c0);
      for (uint32_t u = tid; u < nC * Q; u += BLOCK) {
        const uint32_t il = u / Q, q = u - il * Q, i = c0 + il, j0 = 4 * q;
        const uint4 d = desc[i];
        const uint32_t ibl = d.x & 0xFF, ibr = (d.x >> 8) & 0xFF, jn = (d.x >> 16) & 0xFF,
                       Lx = d.x >> 24;
        const float4 xi = ld4(pop_s, i * Dp + j0);
        const float4 xb = ld4(pop_s, ibl * Dp + j0);
        float4 base = xb;
        if (bl != br) {
          const float4 xr = ld4(pop_s, ibr * Dp + j0);
          base.x = xb.x + F * (xr.x - xb.x);
          base.y = xb.y + F * (xr.y - xb.y);
          base.z = xb.z + F * (xr.z - xb.z);
          base.w = xb.w + F * (xr.w - xb.w);
        }
        float4 dd;
        {
          const float4 a = ld4(pop_s, (d.y & 0xFF) * Dp + j0);
          const float4 b = ld4(pop_s, ((d.y >> 8) & 0xFF) * Dp + j0);
          dd.x = a.x - b.x; dd.y = a.y - b.y; dd.z = a.z - b.z; dd.w = a.w - b.w;
        }
        for (int k = 1; k < dn; ++k) {
          const uint32_t word = k == 1 ? (d.y >> 16) : (k == 2 ? d.z : (d.z >> 16));
          const float4 a = ld4(pop_s, (word & 0xFF) * Dp + j0);
          const float4 b = ld4(pop_s, ((word >> 8) & 0xFF) * Dp + j0);
          dd.x = dd.x + (a.x - b.x);
          dd.y = dd.y + (a.y - b.y);
          dd.z = dd.z + (a.z - b.z);
          dd.w = dd.w + (a.w - b.w);
        }
        float4 v;
        v.x = base.x + F * dd.x;
        v.y = base.y + F * dd.y;
        v.z = base.z + F * dd.z;
        v.w = base.w + F * dd.w;
        float4 uu;
        if (cs == ARITH) {
          const float K = __uint_as_float(d.w);
          uu.x = xi.x + K * (v.x - xi.x);
          uu.y = xi.y + K * (v.y - xi.y);
          uu.z = xi.z + K * (v.z - xi.z);
          uu.w = xi.w + K * (v.w - xi.w);
        } else if (cs == BIN) {
          const uint4 wr = philox(W_GENE0 / 4 + q, i, g, run.stream, k0, k1);
#pragma unroll
          for (int t = 0; t < 4; ++t) {
            const bool take = (unit_oc(word_of(wr, t)) <= CR) || (j0 + t == jn);
            set_comp(uu, t, take ? comp(v, t) : comp(xi, t));
          }
        } else {
#pragma unroll
          for (int t = 0; t < 4; ++t) {
            const uint32_t off = (j0 + t + D - jn) % D;
            set_comp(uu, t, off < Lx ? comp(v, t) : comp(xi, t));
          }
        }
#pragma unroll
        for (int t = 0; t < 4; ++t) {
          const uint32_t j = j0 + t;
          const float c = fminf(fmaxf(comp(uu, t), lb), ub);
          set_comp(uu, t, j < D ? c : 0.0f);
          Y[il * L.ys + j] = j < D ? (double)c - (double)p.o[j] : 0.0;
          if (tr.u && j < D) tr.u[run.pop_off + (size_t)i * D + j] = c;
        }
        st4(T, il * Dp + j0, uu);
      }
      __syncthreads();
      eval_rows<BLOCK>(p, D, Dp, L.ys, nC, Y, Z, P, fu_s + c0);
      __syncthreads();
      // (4) greedy selection decision
      for (uint32_t il = tid; il < nC; il += BLOCK) {
        const uint32_t i = c0 + il;
        const int a = accept_trial(fu_s[i], fit_s[i]) ? 1 : 0;
        acc_s[i] = a;
        if (tr.fu) tr.fu[run.fit_off + i] = fu_s[i];
        if (tr.desc) tr.desc[(size_t)(run.fit_off + i) * 16 + 15] = a;
      }
      if (chunked) {
        __syncthreads();
        for (uint32_t u = tid; u < nC * Q; u += BLOCK) {
          const uint32_t il = u / Q, q = u - il * Q;
          if (acc_s[c0 + il]) st4(pend, (c0 + il) * Dp + 4 * q, ld4(T, il * Dp + 4 * q));
        }
      }
      __syncthreads();
    }
    // (5) synchronous commit of accepted trials
    for (uint32_t u = tid; u < N * Q; u += BLOCK) {
      const uint32_t i = u / Q, q = u - i * Q;
      if (acc_s[i]) {
        const float4 x = chunked ? ld4(pend, i * Dp + 4 * q) : ld4(T, i * Dp + 4 * q);
        st4(pop_s, i * Dp + 4 * q, x);
      }
    }
    for (uint32_t i = tid; i < N; i += BLOCK)
      if (acc_s[i]) fit_s[i] = fu_s[i];
  }
  __syncthreads();
  for (uint32_t u = tid; u < N * D; u += BLOCK) {
    const uint32_t i = u / D, j = u - i * D;
    pop[run.pop_off + u] = pop_s[i * Dp + j];
  }
  for (uint32_t i = tid; i < N; i += BLOCK) fit[run.fit_off + i] = fit_s[i];
}

// ---------------------------------------------------------------- best record in float64

constexpr int FIN_BLOCK = 128;

__global__ __launch_bounds__(FIN_BLOCK) void k_finalize(const RunDev *__restrict__ runs,
                                                        const ProbDev *__restrict__ probs,
                                                        const float *__restrict__ pop,
                                                        const float *__restrict__ fit,
                                                        double *__restrict__ best_y,
                                                        float *__restrict__ best_x) {
  __shared__ uint32_t sk[FIN_BLOCK], si[FIN_BLOCK];
  __shared__ double z[MAX_D], t0s[MAX_D], t1s[MAX_D];
  const RunDev run = runs[blockIdx.x];
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
  for (uint32_t j = tid; j < D; j += FIN_BLOCK) {
    double acc = 0.0;
    for (uint32_t k = 0; k < D; ++k)
      acc = fma(p.R64[(size_t)j * D + k], (double)x[k] - (double)p.o[k], acc);
    z[j] = acc;
  }
  __syncthreads();
  for (uint32_t j = tid; j < D; j += FIN_BLOCK) fn_term<double>(p, z, j, t0s[j], t1s[j]);
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
                               uint32_t P) {
  const uint32_t i = blockIdx.x;
  if (i >= P) return;
  const double yt = y_run[i];
  const bool acc = accept_trial_d(yt, y[i]);
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

__global__ void k_to_f64(const float *__restrict__ src, double *__restrict__ dst, uint32_t n) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) dst[i] = (double)src[i];
}

// ---------------------------------------------------------------- launchers

hipError_t launch_to_f64(const float *src, double *dst, uint32_t n, hipStream_t s) {
  hipLaunchKernelGGL(k_to_f64, dim3((n + 255) / 256), dim3(256), 0, s, src, dst, n);
  return hipGetLastError();
}

hipError_t set_lds_limits() {
  hipError_t e = hipFuncSetAttribute((const void *)k_generations<GEN_BLOCK>,
                                     hipFuncAttributeMaxDynamicSharedMemorySize, LDS_BUDGET);
  if (e != hipSuccess) return e;
  return hipFuncSetAttribute((const void *)k_init<GEN_BLOCK>,
                             hipFuncAttributeMaxDynamicSharedMemorySize, LDS_BUDGET);
}

hipError_t launch_init(const LaunchArgs &a, double lb, double ub) {
  hipLaunchKernelGGL(k_init<GEN_BLOCK>, dim3(a.n_runs), dim3(GEN_BLOCK), a.lds_bytes, a.stream,
                     a.runs, a.probs, a.pop, a.fit, a.k0, a.k1, lb, ub);
  return hipGetLastError();
}

hipError_t launch_generations(const LaunchArgs &a, uint32_t g0, uint32_t n_gens, float lb,
                              float ub, TraceArgs tr) {
  hipLaunchKernelGGL(k_generations<GEN_BLOCK>, dim3(a.n_runs), dim3(GEN_BLOCK), a.lds_bytes,
                     a.stream, a.runs, a.probs, a.pop, a.fit, g0, n_gens, a.k0, a.k1, lb, ub,
                     a.pending, tr);
  return hipGetLastError();
}

hipError_t launch_finalize(const LaunchArgs &a, double *best_y, float *best_x) {
  hipLaunchKernelGGL(k_finalize, dim3(a.n_runs), dim3(FIN_BLOCK), 0, a.stream, a.runs, a.probs,
                     a.pop, a.fit, best_y, best_x);
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
                               const RunDev *runs, uint32_t P, hipStream_t s) {
  hipLaunchKernelGGL(k_outer_select, dim3(P), dim3(64), 0, s, X, y, U, y_run, y_trial, bxo, best_x,
                     runs, P);
  return hipGetLastError();
}

hipError_t launch_outer_best(const double *y, uint32_t P, int32_t *out, hipStream_t s) {
  hipLaunchKernelGGL(k_outer_best, dim3(1), dim3(256), 0, s, y, P, out);
  return hipGetLastError();
}

}  // namespace mde
