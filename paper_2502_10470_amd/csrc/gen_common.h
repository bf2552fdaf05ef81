// Device helpers shared by the generation kernels (lane-per-trial and
// matrix-core variants): vector access, ranking keys, the random draws of a
// generation and the trial construction of Eq. (12) with Eqs. (8)-(10).
#pragma once

#include "device.h"

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

// 64-bit ranking key: order of (fitness, index), NaN as +inf.
__device__ __forceinline__ uint64_t mkkey(float f, uint32_t i) {
  return ((uint64_t)okey(f) << 32) | i;
}

__device__ __forceinline__ float finish_f32(const ProbDev &p, double s0, double s1) {
  return p.kind == FN_ACKLEY ? fn_finish<float>(p, (float)s0, (float)s1)
                             : (float)(s0 + (double)p.bias);
}

// ---------------------------------------------------------------- random draws (producers)
//
// The random part of a generation does not depend on the population: index
// draws, the pbest rank, j_rand / n, K, the exponential length L and the
// binomial mask bits are functions of (seed, stream, generation, individual)
// and theta only.  Producer lanes compute them one generation ahead.

// Crossover-test nibbles of generation g (Philox blocks 3 + q): bit t of
// nibble (i, q) is the test r <= CR of gene uniform 4q + t.  Binomial
// crossover takes gene 4q + t where the bit is set; exponential crossover
// continues its run while consecutive bits (in test order) are set.
// INT_TEST: the same test in integers, r <= CR iff (w >> 8) < floor(CR 2^24)
// (r = ((w >> 8) + 1) 2^-24; CR in [0, 1], so CR 2^24 is exact and the
// conversion is the floor), three instructions fewer per word.  The
// matrix-core kernel uses it (D = 100: 26.05 against 26.44 ms per launch);
// in the lane kernel the float form measured faster (5.37 against 5.45 ms
// per 1000 generations at D = 20), for reasons of code layout rather than
// instruction count, and it keeps that form.
template <bool INT_TEST = false>
__device__ __forceinline__ void produce_masks(uint32_t ptid, uint32_t nprod, const RunDev &run,
                                              uint32_t N, uint32_t Q, uint32_t g, uint32_t k0,
                                              uint32_t k1, uint8_t *msk) {
  if (run.cs != BIN && run.cs != EXP) return;
  const uint32_t thr = (uint32_t)(run.CR * 16777216.0f);
  // item it = i Q + q, stepped by nprod without a division per item
  const uint32_t di = nprod / Q, dq = nprod - di * Q;
  uint32_t i = ptid / Q, q = ptid - i * Q;
  for (uint32_t it = ptid; it < N * Q; it += nprod) {
    const uint4 w = philox(W_GENE0 / 4 + q, i, g, run.stream, k0, k1);
    uint32_t nib = 0;
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const bool pass = INT_TEST ? (word_of(w, t) >> 8) < thr : unit_oc(word_of(w, t)) <= run.CR;
      nib |= (pass ? 1u : 0u) << t;
    }
    msk[it] = (uint8_t)nib;
    i += di;
    q += dq;
    if (q >= Q) {
      q -= Q;
      ++i;
    }
  }
}

// Packed draws of generation g: Philox blocks 0..2 by the lane itself (with
// PRE, block 2 of the lane's one trial comes in wc_pre, drawn in an earlier
// phase); the exponential length from the test nibbles of generation g (mskg,
// written by produce_masks and visible to this lane).
template <bool PRE = false>
__device__ __forceinline__ void produce_desc_direct(uint32_t ptid, uint32_t nprod,
                                                    const RunDev &run, uint32_t N, uint32_t D,
                                                    uint32_t kp, uint32_t g, uint32_t k0,
                                                    uint32_t k1, const uint8_t *mskg,
                                                    uint4 *dsc, uint4 wc_pre = uint4{}) {
  const int use_rand = (run.bl == RAND || run.br == RAND) ? 1 : 0;
  const int dn = run.dn;
  const int m = use_rand + 2 * dn;
  for (uint32_t i = ptid; i < N; i += nprod) {
    uint32_t w[12];
    const uint4 wa = philox(0, i, g, run.stream, k0, k1);
    const uint4 wc = PRE ? wc_pre : philox(2, i, g, run.stream, k0, k1);
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
    uint32_t pr[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) pr[k] = (k < 2 * dn) ? dr[use_rand + k] : 0u;
    const uint32_t r0 = use_rand ? dr[0] : 0u;
    const uint32_t pb = lemire(w[W_PBEST], kp);
    const uint32_t jn = lemire(w[W_JRAND], D);
    // L = 1 + the number of leading passed continuation tests, at most D
    uint32_t Lx = 1;
    if (run.cs == EXP) {
      const uint32_t Q = (D + 3) / 4;
      for (uint32_t q = 0; q < Q && Lx < D; ++q) {
        const uint32_t ones = (uint32_t)__builtin_ctz(~(uint32_t)mskg[i * Q + q]);
        Lx += ones;
        if (ones < 4) break;
      }
      Lx = min(Lx, D);
    }
    uint4 d;
    d.x = pr[0] | (pr[1] << 8) | (pr[2] << 16) | (pr[3] << 24);
    d.y = pr[4] | (pr[5] << 8) | (pr[6] << 16) | (pr[7] << 24);
    d.z = r0 | (pb << 8) | (jn << 16) | (Lx << 24);
    d.w = __float_as_uint(unit_oc(w[W_K]));
    dsc[i] = d;
  }
}

__device__ __forceinline__ uint32_t byte_of(uint32_t w, int k) { return (w >> (8 * k)) & 0xFFu; }

// Genes 4q..4q+3 of trial i: mutation Eq. (12), crossover Eqs. (8)-(10),
// clip to the box.  Genes >= D come back as 0.
__device__ __forceinline__ float4 trial_quad(const float *pop_s, uint32_t Dp, uint32_t D,
                                             uint32_t i, uint32_t q, uint32_t ibl, uint32_t ibr,
                                             const uint4 &d, uint32_t nib, const RunDev &run,
                                             float lb, float ub) {
  const uint32_t j0 = 4 * q;
  const float F = run.F;
  const float4 xi = ld4(pop_s, i * Dp + j0);
  const float4 xb = ld4(pop_s, ibl * Dp + j0);
  float4 base = xb;
  if (run.bl != run.br) {
    const float4 xr = ld4(pop_s, ibr * Dp + j0);
    base.x = xb.x + F * (xr.x - xb.x);
    base.y = xb.y + F * (xr.y - xb.y);
    base.z = xb.z + F * (xr.z - xb.z);
    base.w = xb.w + F * (xr.w - xb.w);
  }
  float4 dd;
  {
    const float4 a = ld4(pop_s, byte_of(d.x, 0) * Dp + j0);
    const float4 b = ld4(pop_s, byte_of(d.x, 1) * Dp + j0);
    dd.x = a.x - b.x; dd.y = a.y - b.y; dd.z = a.z - b.z; dd.w = a.w - b.w;
  }
#pragma unroll
  for (int k = 1; k < 4; ++k) {
    if (k < run.dn) {
      const uint32_t word = k == 1 ? (d.x >> 16) : (k == 2 ? d.y : (d.y >> 16));
      const float4 a = ld4(pop_s, byte_of(word, 0) * Dp + j0);
      const float4 b = ld4(pop_s, byte_of(word, 1) * Dp + j0);
      dd.x = dd.x + (a.x - b.x);
      dd.y = dd.y + (a.y - b.y);
      dd.z = dd.z + (a.z - b.z);
      dd.w = dd.w + (a.w - b.w);
    }
  }
  float4 v;
  v.x = base.x + F * dd.x;
  v.y = base.y + F * dd.y;
  v.z = base.z + F * dd.z;
  v.w = base.w + F * dd.w;
  float4 uu;
  if (run.cs == ARITH) {
    const float K = __uint_as_float(d.w);
    uu.x = xi.x + K * (v.x - xi.x);
    uu.y = xi.y + K * (v.y - xi.y);
    uu.z = xi.z + K * (v.z - xi.z);
    uu.w = xi.w + K * (v.w - xi.w);
  } else if (run.cs == BIN) {
    const uint32_t jn = byte_of(d.z, 2);
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const bool take = ((nib >> t) & 1u) || (j0 + t == jn);
      set_comp(uu, t, take ? comp(v, t) : comp(xi, t));
    }
  } else {
    const uint32_t n0 = byte_of(d.z, 2), Lx = d.z >> 24;
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      // (j0 + t - n0) mod D: for a gene j0 + t < D the sum lies in [1, 2D), so
      // one conditional subtraction is the remainder (padding genes past D
      // take any value; they never reach a fitness)
      uint32_t off = j0 + t + D - n0;
      off = off >= D ? off - D : off;
      set_comp(uu, t, off < Lx ? comp(v, t) : comp(xi, t));
    }
  }
#pragma unroll
  for (int t = 0; t < 4; ++t)
    set_comp(uu, t, j0 + t < D ? fminf(fmaxf(comp(uu, t), lb), ub) : 0.0f);
  return uu;
}

}  // namespace mde
