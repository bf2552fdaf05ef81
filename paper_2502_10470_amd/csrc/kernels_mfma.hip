// Matrix-core generation kernel of the MetaDE inner-DE path (gfx950).
//
// Used for runs whose trial rows do not fit in LDS next to the population
// (large D) and for the bf16 precision mode.  One workgroup of 768 lanes per
// run; lanes 0..511 are consumers, 512..767 producers of the next
// generation's random draws (as in the lane-per-trial kernel).  The rotation
// z = R (u - o) of all trials of a generation is a [N x D] x [D x D] product
// done on the matrix cores, dealt to the waves as (output tile, row tiles)
// items from an LDS counter.  Both modes read a row-major float32 copy of R,
// zero padded to whole tiles, and the float32 trial rows from a global
// buffer.
//
// Plain mode: v_mfma_f64_16x16x4 on y = u - o in float64 (exact), the same
// accuracy as the lane kernel's float64 accumulation.
// bf16 mode: the product is formed from bf16 splits, y R ~ y_hi R_hi +
// y_hi R_lo + y_lo R_hi with v_mfma_f32_16x16x32_bf16 and float32
// accumulation.  Each trial gets a certified bound E on |f_hat - f| (from a
// per-output error radius: a fourth product of the bf16 magnitudes); a trial
// with f_hat - E > f(target) would be rejected by the plain evaluation too, so
// it is rejected at once; every other trial is re-evaluated in plain mode (on
// compacted row tiles) and decided from that value.  Decisions -- hence
// trajectories -- are those of the plain mode as long as the bound holds.
#include <hip/hip_bf16.h>

#include "device.h"
#include "gen_common.h"
#include "kernels.h"

namespace mde {

MDE_STAGE_ARRAY;

typedef double d4v __attribute__((ext_vector_type(4)));
typedef float f4v __attribute__((ext_vector_type(4)));
typedef __bf16 bf8v __attribute__((ext_vector_type(8)));

constexpr int KSB = 4;        // bf16 k-steps of 32 (D <= 128)
// Per-output error radius of the three-product bf16 split with float32
// accumulation: |z_hat_j - z_j| <= E_AB * S_j, S_j = sum_k |R_jk| |y_k|.
// With u_b = 2^-8 the unit roundoff of bf16, the splits y = y_hi + y_lo + dy,
// R = R_hi + R_lo + dR leave |dy| <= u_b^2 |y|, |dR| <= u_b^2 |R|; the products
// y_hi R_hi + y_hi R_lo + y_lo R_hi miss y_lo R_lo + (y_hi + y_lo) dR +
// dy (R_hi + R_lo) + dy dR, at most (3 + 2^-15) 2^-16 |y| |R| per term; the
// float32 sum of the 3 Dk <= 384 exact bf16 products adds at most
// 384 2^-24 (1 + 2^-7) of the same sum, and rounding u - o to float32 2^-24:
// in all below 6.92e-5 S_j.  S_j itself comes from a fourth product of the
// bf16 magnitudes, |R_hi| |y_hi|, summed in float32: each magnitude is within
// a factor 1/(1 - 2^-8) of its rounded value and the float32 sum of
// non-negative terms within 1/(1 - 384 2^-24), so S_j <= 1.0079 S_hat_j.
// E_AB = 6.92e-5 * 1.0079 rounded up.
constexpr float E_AB = 7.0e-5f;

// ---------------------------------------------------------------- rotation tiles

// Plain mode.  The product is formed transposed, z^T = R u^T: the A operand
// is 16 rows of R, the B operand 16 trial rows, so that each lane ends with
// one trial and four of its outputs; R o is subtracted afterwards (z = R u -
// R o; the products of two float32 values are exact in float64, so only the
// float64 sums round).  Any consistent assignment of the physical k to
// (step, lane) slots gives the same product, so the k order is permuted inside
// each block of four steps: lane l feeds steps 4b..4b+3 with k = 16 b +
// 4 (l/16) + 0..3, one contiguous float4 of its trial row and of its row of R.
// Result element v is (R u)[trial 16 rt + l%16][output 16 ct + l/16 + 4v].
// The rotation is zero padded to whole tiles (row stride Rs) and the trial
// rows are zero beyond D, so no operand needs a bounds test.  RR row tiles at
// once (rows given per tile): RR independent accumulator chains sharing the A
// loads, so that consecutive matrix-core instructions do not wait on each
// other's results.  The plain rotation takes two or four row tiles per item
// (a tuning choice, RTF), the bf16 mode's re-evaluation two.  (Storing the operands in float64 to spare
// the conversions was measured slower: the rotation waits on its loads, and
// float64 operands double them.)
constexpr int RT = 2;

template <int RR>
__device__ __forceinline__ void tiles_f64(const float *__restrict__ Tg, uint32_t Dk,
                                          const bool (&row_ok)[RR],
                                          const uint32_t (&row_trial)[RR],
                                          const float *__restrict__ R32, uint32_t Rs, uint32_t j,
                                          uint32_t lane, d4v (&acc)[RR]) {
  const uint32_t kq = lane >> 4;
  const uint32_t nb = Rs / 16;  // blocks of 16 k (four steps of 4)
#pragma unroll
  for (int r = 0; r < RR; ++r) acc[r] = d4v{0.0, 0.0, 0.0, 0.0};
  const float *rrow = R32 + (size_t)j * Rs + 4 * kq;
  // operands of block b: the lane's float4 of each trial row and of its row of R
  auto load = [&](uint32_t b, float4 (&tv)[RR], float4 &bv) {
    const uint32_t kb = 16 * b + 4 * kq;
#pragma unroll
    for (int r = 0; r < RR; ++r)
      tv[r] = row_ok[r] ? *reinterpret_cast<const float4 *>(Tg + (size_t)row_trial[r] * Dk + kb)
                        : make_float4(0.f, 0.f, 0.f, 0.f);
    bv = *reinterpret_cast<const float4 *>(rrow + 16 * b);
  };
  auto products = [&](const float4 (&tv)[RR], const float4 &bv) {
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const double re = (double)comp(bv, e);
#pragma unroll
      for (int r = 0; r < RR; ++r)
        acc[r] = __builtin_amdgcn_mfma_f64_16x16x4f64(re, (double)comp(tv[r], e), acc[r], 0, 0, 0);
    }
  };
  // three operand buffers in turn, the loop unrolled by three so that the
  // turn is a renaming at compile time (no register moves between products);
  // the loads of the next two blocks are in flight while a block's products run
  float4 t0[RR], t1[RR], t2[RR];
  float4 b0, b1, b2;
  load(0, t0, b0);
  if (nb > 1) load(1, t1, b1);
#pragma unroll 1
  for (uint32_t b = 0; b < nb; b += 3) {
    if (b + 2 < nb) load(b + 2, t2, b2);
    products(t0, b0);
    if (b + 1 >= nb) break;
    if (b + 3 < nb) load(b + 3, t0, b0);
    products(t1, b1);
    if (b + 2 >= nb) break;
    if (b + 4 < nb) load(b + 4, t1, b1);
    products(t2, b2);
  }
}

// z = R u - R o of the four outputs a lane holds after a plain tile
// (outputs 16 ct + l/16 + 4 v), rounded once to float32.
__device__ __forceinline__ void tile_z(const d4v &acc, const double *ro, uint32_t ct,
                                       uint32_t lane, float (&z)[4]) {
#pragma unroll
  for (int v = 0; v < 4; ++v) z[v] = (float)(acc[v] - ro[16 * ct + (lane >> 4) + 4 * v]);
}

// The rotation of a generation as (output tiles, group of row tiles) items,
// fetched from a counter in LDS by every wave that calls this (the consumers
// as soon as the trials are built, the producers once the next generation's
// crossover tests are drawn: before the rotation with two mask buffers,
// during it with one), so that one wave's products run while
// another waits for its loads or forms the element terms.  In the plain mode
// items that share row tiles are adjacent in the order, so their trial rows
// come from cache; the bf16 mode orders its items by output-tile group.
template <typename BODY>
__device__ __forceinline__ void rotation_items(uint32_t *ctr, uint32_t n_items, uint32_t lane,
                                               BODY &&body) {
  for (;;) {
    uint32_t it = 0;
    if (lane == 0) it = atomicAdd(ctr, 1u);
    it = __builtin_amdgcn_readfirstlane(it);
    if (it >= n_items) break;
    body(it);
  }
}

// bf16 mode, transposed like the plain mode.  Lane l feeds trial 16 rt + l%16
// with k = 32 s + 8 (l/16) + e; result element v is
// z_hat[trial 16 rt + l%16][output 16 ct + 4 (l/16) + v].  The trial operands
// are the bf16 splits of y = u - o (float32 subtraction), formed here from the
// float32 trial rows, which the exact re-evaluation reads as well: one buffer
// per run in the cache instead of three.  ab[c][r] receives
// sum_k |R_hi jk| |y_hi k| for the outputs' error radii.
__device__ __forceinline__ bf8v abs8(const bf8v &x) {
  uint4 u = __builtin_bit_cast(uint4, x);
  u.x &= 0x7FFF7FFFu;
  u.y &= 0x7FFF7FFFu;
  u.z &= 0x7FFF7FFFu;
  u.w &= 0x7FFF7FFFu;
  return __builtin_bit_cast(bf8v, u);
}

// bf16 parts of eight float32 values: hi = bf16(x), lo = bf16(x - hi).
__device__ __forceinline__ void split8(const float4 &a, const float4 &b, bf8v &hi, bf8v &lo) {
#pragma unroll
  for (int e = 0; e < 8; ++e) {
    const float x = e < 4 ? comp(a, e) : comp(b, e - 4);
    const __bf16 h = (__bf16)x;
    hi[e] = h;
    lo[e] = (__bf16)(x - (float)h);
  }
}

// BCT output tiles per call (R rows Rrow0, Rrow0 + 16 Rs, ...; the first ncol
// of them exist), so that the splits of each trial value, the bulk of this
// vector-bound stage, are formed once for all of them.
constexpr int BCT = 4;
__device__ __forceinline__ void tiles_bf16(const float *__restrict__ Tg,
                                           const float *__restrict__ oc, uint32_t Dk,
                                           const bool (&row_ok)[RT],
                                           const uint32_t (&row_trial)[RT],
                                           const float *__restrict__ Rrow0, uint32_t ncol,
                                           uint32_t Rs, uint32_t lane, f4v (&acc)[BCT][RT],
                                           f4v (&ab)[BCT][RT]) {
  const uint32_t Ksb = Dk / 32;
#pragma unroll
  for (int c = 0; c < BCT; ++c)
#pragma unroll
    for (int r = 0; r < RT; ++r) {
      acc[c][r] = f4v{0.0f, 0.0f, 0.0f, 0.0f};
      ab[c][r] = f4v{0.0f, 0.0f, 0.0f, 0.0f};
    }
#pragma unroll
  for (int s = 0; s < KSB; ++s) {
    if ((uint32_t)s < Ksb) {
      const uint32_t k0 = 32 * s + 8 * (lane >> 4);
      const float4 oa = *reinterpret_cast<const float4 *>(oc + k0);
      const float4 ob = *reinterpret_cast<const float4 *>(oc + k0 + 4);
      bf8v ah[RT], al[RT];
#pragma unroll
      for (int r = 0; r < RT; ++r) {
        if (row_ok[r]) {
          const float *t = Tg + (size_t)row_trial[r] * Dk + k0;
          float4 ya = *reinterpret_cast<const float4 *>(t);
          float4 yb = *reinterpret_cast<const float4 *>(t + 4);
          ya.x -= oa.x; ya.y -= oa.y; ya.z -= oa.z; ya.w -= oa.w;
          yb.x -= ob.x; yb.y -= ob.y; yb.z -= ob.z; yb.w -= ob.w;
          split8(ya, yb, ah[r], al[r]);
        } else {
#pragma unroll
          for (int e = 0; e < 8; ++e) ah[r][e] = al[r][e] = (__bf16)0.0f;
        }
      }
      bf8v aab[RT];
#pragma unroll
      for (int r = 0; r < RT; ++r) aab[r] = abs8(ah[r]);
#pragma unroll
      for (int c = 0; c < BCT; ++c) {
        if ((uint32_t)c >= ncol) break;
        bf8v bh, bl;
        {
          const float *Rrow = Rrow0 + (size_t)(16 * c) * Rs;
          float4 ra = make_float4(0.f, 0.f, 0.f, 0.f), rb = ra;
          if (k0 < Rs) {
            ra = *reinterpret_cast<const float4 *>(Rrow + k0);
            rb = *reinterpret_cast<const float4 *>(Rrow + k0 + 4);
          }
          split8(ra, rb, bh, bl);
        }
#pragma unroll
        for (int r = 0; r < RT; ++r) acc[c][r] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(bh, al[r], acc[c][r], 0, 0, 0);
#pragma unroll
        for (int r = 0; r < RT; ++r) acc[c][r] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(bl, ah[r], acc[c][r], 0, 0, 0);
#pragma unroll
        for (int r = 0; r < RT; ++r) acc[c][r] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(bh, ah[r], acc[c][r], 0, 0, 0);
        const bf8v bab = abs8(bh);
#pragma unroll
        for (int r = 0; r < RT; ++r) ab[c][r] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(bab, aab[r], ab[c][r], 0, 0, 0);
      }
    }
  }
}


// ---------------------------------------------------------------- element terms and bounds

// Constants of output j: the element kind (the hybrid's block resolved) and
// the elliptic weight.
struct ColInfo {
  uint32_t kind;
  float w;
};

__device__ __forceinline__ ColInfo col_info(const unsigned char *tab, const ProbDev &p, uint32_t j) {
  ColInfo c{p.kind, 0.0f};
  if (j >= p.D) return c;
  if (p.kind == FN_HYBRID) {
    const uint32_t ek = tab_ptr<uint32_t>(tab, p.ek_off)[j];
    c.kind = ek == 0 ? FN_SCHWEFEL : (ek == 1 ? FN_RASTRIGIN : FN_ELLIPTIC);
  }
  if (c.kind == FN_ELLIPTIC) c.w = tab_ptr<float>(tab, p.ew_off)[j];
  return c;
}

// Element term of kind c.kind (Rosenbrock excluded), as elem_term.
__device__ __forceinline__ void col_term(const ProbDev &p, const ColInfo &c, float v, float &t0,
                                         float &t1) {
  t1 = 0.0f;
  switch (c.kind) {
    case FN_RASTRIGIN: t0 = h_rastrigin<float>(v); break;
    case FN_ELLIPTIC: t0 = c.w * (v * v); break;
    case FN_ACKLEY: t0 = v * v; t1 = Math<float>::cos2pi(v); break;
    case FN_SCHWEFEL: t0 = h_schwefel<float>(p, v); break;
    default: t0 = 0.0f;
  }
}

// Bound on |h(z_hat) - h(z)| for |z_hat - z| <= e, plus an allowance for the
// float32 evaluation of the term t.
__device__ __forceinline__ float term_bound(const ProbDev &p, const ColInfo &c, float zh, float e,
                                            float t) {
  const float az = fabsf(zh) + e;
  float b;
  switch (c.kind) {
    case FN_RASTRIGIN: b = (2.0f * az + 62.83186f) * e; break;
    case FN_ELLIPTIC: b = c.w * e * (2.0f * fabsf(zh) + e); break;
    case FN_SCHWEFEL: b = (1.0f + 0.5f * sqrtf(fabsf(zh + SCHWEFEL_ZSTAR) + e)) * e; break;
    case FN_ACKLEY: b = (4.0f * rsqrtf((float)p.D) + 17.1f / (float)p.D) * e; break;
    default: b = __int_as_float(0x7F800000); break;  // no certified bound: always refine
  }
  return b * 1.0001f + 2.4e-7f * (fabsf(t) + 30.0f);
}

// x + x[lane ^ 16] and x + x[lane ^ 32] with the gfx950 row swaps: called
// with both operands x, v_permlane16_swap leaves in every lane one of its own
// value and its partner's (which one depends on the row's parity), so their
// sum is the butterfly step bit for bit (addition commutes), with no LDS
// round trip.
__device__ __forceinline__ float xsum16(float x) {
  const auto r = __builtin_amdgcn_permlane16_swap(__float_as_uint(x), __float_as_uint(x), false,
                                                  false);
  return __uint_as_float(r[0]) + __uint_as_float(r[1]);
}
__device__ __forceinline__ float xsum32(float x) {
  const auto r = __builtin_amdgcn_permlane32_swap(__float_as_uint(x), __float_as_uint(x), false,
                                                  false);
  return __uint_as_float(r[0]) + __uint_as_float(r[1]);
}

// Terms of the four results a lane holds after a transposed tile (one trial,
// outputs j(v): 16 ct + l/16 + 4 v for the plain tiles (STRIDED), 16 ct +
// 4 (l/16) + v for the bf16 tiles) and their sum over the tile's 16 outputs:
// four local terms, then the four lane groups of the trial (lanes l, l+16,
// l+32, l+48) by two shuffles.  Lanes 0..15 write the trial's partial sum (and
// bound).  Rosenbrock pairs z_j with z_{j+1}; the pair that crosses into the
// next output tile is formed from zl / zf when the tiles are combined.
template <bool BOUND, bool STRIDED>
__device__ __forceinline__ void tile_epilogue(const ProbDev &p, const uint32_t *ek_s,
                                              const float *ew_s, const float (&z)[4],
                                              uint32_t slot, bool ok, const float (&e)[4],
                                              uint32_t D,
                                              uint32_t ct, uint32_t nslot, uint32_t lane,
                                              float2 *Ps, float *Pb, float *zf, float *zl) {
  const uint32_t grp = lane >> 4;
  float t0 = 0.0f, t1 = 0.0f, bd = 0.0f;
  if (p.kind == FN_ROSENBROCK) {
    // successor of each element: the next lane group (same v, or v+1 when
    // wrapping from group 3 to group 0) for STRIDED; the next element, or
    // element 0 of the next lane group, otherwise
    float up[4];
#pragma unroll
    for (int v = 0; v < 4; ++v) up[v] = __shfl(z[v], (int)((lane + 16) & 63));
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const uint32_t j = STRIDED ? 16 * ct + grp + 4 * v : 16 * ct + 4 * grp + v;
      float zn;
      if (STRIDED) zn = grp < 3 ? up[v] : (v < 3 ? up[v + 1] : 0.0f);
      else zn = v < 3 ? z[v + 1] : up[0];
      const bool inner = (j & 15) != 15 && j + 1 < D;
      if (ok && inner) t0 += h_rosenbrock<float>(z[v], zn);
    }
    if (ok && grp == 0) zf[ct * nslot + slot] = z[0];
    if (ok && grp == 3) zl[ct * nslot + slot] = z[3];
    if (BOUND && ok) bd = __int_as_float(0x7F800000);
  } else {
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const uint32_t j = STRIDED ? 16 * ct + grp + 4 * v : 16 * ct + 4 * grp + v;
      if (ok && j < D) {
        // the kind is a constant of the generation loop except for the hybrid,
        // whose outputs fall in different blocks
        const uint32_t kind = p.kind == FN_HYBRID ? ek_s[j] : p.kind;
        const ColInfo c{kind, kind == FN_ELLIPTIC ? ew_s[j] : 0.0f};
        float a0, a1;
        col_term(p, c, z[v], a0, a1);
        t0 += a0;
        t1 += a1;
        if (BOUND) bd += term_bound(p, c, z[v], e[v], a0);
      }
    }
  }
  t0 = xsum32(xsum16(t0));
  if (p.kind == FN_ACKLEY) t1 = xsum32(xsum16(t1));
  if (BOUND) bd = xsum32(xsum16(bd));
  if (ok && grp == 0) {
    Ps[ct * nslot + slot] = make_float2(t0, t1);
    if (BOUND) Pb[ct * nslot + slot] = bd;
  }
}

// Sum of the per-tile partials of slot s (and Rosenbrock's tile-boundary
// terms); returns the float32 fitness.
__device__ __forceinline__ float combine(const ProbDev &p, const float2 *Ps, const float *zf,
                                         const float *zl, uint32_t NCT, uint32_t D, uint32_t nslot,
                                         uint32_t s) {
  double s0 = 0.0, s1 = 0.0;
  for (uint32_t ct = 0; ct < NCT; ++ct) {
    const float2 v = Ps[ct * nslot + s];
    s0 += (double)v.x;
    s1 += (double)v.y;
  }
  if (p.kind == FN_ROSENBROCK)
    for (uint32_t ct = 0; ct + 1 < NCT; ++ct)
      if (16 * ct + 16 < D) s0 += (double)h_rosenbrock<float>(zl[ct * nslot + s], zf[(ct + 1) * nslot + s]);
  return finish_f32(p, s0, s1);
}

// ---------------------------------------------------------------- generation loop

// Check of the bf16 screen in traced generations (every trial re-evaluated):
// trials checked, bf16 values farther than their bound from the plain value,
// trials the screen alone would have rejected, of those the ones the plain
// value accepts (a wrong decision the bound should have prevented), and the
// largest |f_hat - f| / bound seen.
struct BoundCheck {
  unsigned long long checked, outside, screened, screen_wrong;
  double max_ratio;
};

// Producer waves: the random draws of generation g + 1 (crossover-test
// nibbles during the trial construction or the rotation, packed draws after
// the decisions), rotation items, and in the bf16 mode a third of the exact
// re-evaluation's items.  Runs the same barrier sequence as the consumers --
// one before the loop, five per generation (eight in the bf16 mode), one
// after it -- so the two roles keep separate loops.
template <bool BF16, typename BODY, typename REEVAL>
__device__ __forceinline__ void mfma_producers(const MLds &lay, unsigned char *smem,
                                               const RunDev &run, uint32_t g0, uint32_t n_gens,
                                               uint32_t k0, uint32_t k1, uint32_t ptid,
                                               uint32_t *ctr, uint32_t n_items, BODY &&item,
                                               const uint32_t *cnts, REEVAL &&reeval) {
  const uint32_t N = run.N, D = run.D, Q = run.Dp / 4, kp = run.kp;
  uint8_t *const mbuf[2] = {reinterpret_cast<uint8_t *>(smem + lay.msk),
                            reinterpret_cast<uint8_t *>(smem + lay.msk2)};
  const bool two = lay.msk2 != lay.msk;
  uint4 *dsc = reinterpret_cast<uint4 *>(smem + lay.dsc);
  constexpr uint32_t NP = MF_THREADS - MF_CONSUMERS;
  // with two mask buffers the tests of g+1 are drawn during the trial
  // construction, which waits on LDS gathers, instead of during the rotation,
  // whose float64 products the vector work would hold up
  produce_masks<true>(ptid, NP, run, N, Q, g0, k0, k1, mbuf[g0 & 1u]);
  __syncthreads();
  produce_desc_direct(ptid, NP, run, N, D, kp, g0, k0, k1, mbuf[g0 & 1u], dsc);
  MDE_STAGE_BEGIN
  for (uint32_t gg = 0; gg < n_gens; ++gg) {
    const uint32_t g = g0 + gg;
    uint8_t *mn = two ? mbuf[(g + 1) & 1u] : mbuf[0];
    __syncthreads();   // generation g: consumers count ranks
    MDE_STAGE(0)
    __syncthreads();   // top-p list
    MDE_STAGE(1)
    __syncthreads();   // trial construction (reads the masks of g)
    MDE_STAGE(2)
    if (two) produce_masks<true>(ptid, NP, run, N, Q, g + 1, k0, k1, mn);
    MDE_STAGE_WORK(11)
    __syncthreads();   // rotation: the masks of g are free
    MDE_STAGE(3)
    if (!two) produce_masks<true>(ptid, NP, run, N, Q, g + 1, k0, k1, mn);
    rotation_items(ctr, n_items, ptid & 63, item);   // then help with the rotation
    MDE_STAGE_WORK(12)
    __syncthreads();   // decisions (plain) or screen (bf16)
    MDE_STAGE(4)
    if (BF16) {
      __syncthreads(); // candidate counts
      MDE_STAGE(5)
      __syncthreads(); // candidate list
      MDE_STAGE(6)
      {
        // help with the exact re-evaluation: the candidate count from the
        // consumers' per-wave counts, items dealt as to the consumers
        uint32_t total = 0;
        for (uint32_t w = 0; w < MF_CONSUMERS / 64; ++w) total += cnts[w];
        const uint32_t NCT = run.NCT;
        const uint32_t n_re = NCT * (((total + 15) / 16 + RT - 1) / RT);
        for (uint32_t it = MF_CONSUMERS / 64 + ptid / 64; it < n_re; it += MF_THREADS / 64)
          reeval(it, total);
      }
      MDE_STAGE_WORK(15)
      __syncthreads(); // re-evaluation
      MDE_STAGE(7)
    }
    produce_desc_direct(ptid, NP, run, N, D, kp, g + 1, k0, k1, mn, dsc);
    MDE_STAGE_WORK(8)
  }
  __syncthreads();
  MDE_STAGE(0)
  MDE_STAGE_END
}

template <bool BF16, bool TRACE, int RTF>
__device__ __forceinline__ void mfma_body(unsigned char *smem, const RunDev &run,
                                          const ProbDev &p, const unsigned char *__restrict__ tab,
                                          float *__restrict__ pop, float *__restrict__ fit,
                                          uint32_t g0, uint32_t n_gens, uint32_t k0, uint32_t k1,
                                          float lb, float ub, float *__restrict__ Tg,
                                          unsigned long long *__restrict__ counters,
                                          const TraceArgs &tr) {
  const uint32_t N = run.N, D = run.D, Dp = run.Dp, Dk = run.Dk, Q = Dp / 4, kp = run.kp,
                 L = run.L, Np = run.Np, NCT = run.NCT;
  const uint32_t NRT = (N + 15) / 16;
  const bool rosen = p.kind == FN_ROSENBROCK;
  const MLds lay = mfma_layout(N, Dp, Dk, L, Np, NCT, rosen, BF16);
  float *pop_s = reinterpret_cast<float *>(smem + lay.pop);
  uint64_t *key_s = reinterpret_cast<uint64_t *>(smem + lay.key);
  float *fit_s = reinterpret_cast<float *>(smem + lay.fit);
  uint32_t *topk = reinterpret_cast<uint32_t *>(smem + lay.topk);
  uint32_t *rk = reinterpret_cast<uint32_t *>(smem + lay.rk);
  uint8_t *msk = reinterpret_cast<uint8_t *>(smem + lay.msk);
  uint4 *dsc = reinterpret_cast<uint4 *>(smem + lay.dsc);
  float2 *Ps = reinterpret_cast<float2 *>(smem + lay.ps);
  float *Pb = reinterpret_cast<float *>(smem + lay.pb);
  float *zf = reinterpret_cast<float *>(smem + lay.zf);
  float *zl = reinterpret_cast<float *>(smem + lay.zl);
  float *oc = reinterpret_cast<float *>(smem + lay.oc);
  uint32_t *ek_s = reinterpret_cast<uint32_t *>(smem + lay.ek);
  float *ew_s = reinterpret_cast<float *>(smem + lay.ew);
  uint32_t *cl = reinterpret_cast<uint32_t *>(smem + lay.cl);
  uint32_t *cnt = reinterpret_cast<uint32_t *>(smem + lay.cnt);
  const double *Rt = tab_ptr<double>(tab, p.r64t_off);
  const uint32_t Dr = rt_stride(D);
  // row-major float32 rotation, zero padded to Rs x Rs, and R o
  const uint32_t Rs = r32_stride(D);
  const float *R32 = tab_ptr<float>(tab, p.r32_off);
  double *ro_s = reinterpret_cast<double *>(smem + lay.ro);

  const uint32_t tid = threadIdx.x;

  for (uint32_t u = tid; u < N * Dp; u += MF_THREADS) {
    const uint32_t r = u / Dp, j = u - r * Dp;
    pop_s[u] = j < D ? pop[run.pop_off + (size_t)r * D + j] : 0.0f;
  }
  for (uint32_t r = tid; r < N; r += MF_THREADS) {
    const float f = fit[run.fit_off + r];
    fit_s[r] = f;
    key_s[r] = mkkey(f, r);
  }
  const float *og = tab_ptr<float>(tab, p.o_off);
  const double *rog = tab_ptr<double>(tab, p.ro64_off);
  for (uint32_t k = tid; k < Dk; k += MF_THREADS) {
    oc[k] = k < D ? og[k] : 0.0f;
    ro_s[k] = k < Rs ? rog[k] : 0.0;
    const ColInfo c = col_info(tab, p, k);
    ek_s[k] = c.kind;
    ew_s[k] = c.w;
  }
  if (Dk > Dp)
    for (uint32_t u = tid; u < N * (Dk - Dp); u += MF_THREADS) {
      const uint32_t r = u / (Dk - Dp);
      const size_t at = (size_t)r * Dk + Dp + (u - r * (Dk - Dp));
      Tg[at] = 0.0f;
    }
  // the rotation's items, shared by consumers and producers: plain, (output
  // tile, RTF row tiles) in float64; bf16, (output tile, RT row tiles)
  // from the bf16 splits with each output's error radius
  constexpr uint32_t RTI = BF16 ? RT : RTF;
  // bf16 mode: items of BCT output tiles x RT row tiles
  const uint32_t NCP = (NCT + BCT - 1) / BCT;
  const uint32_t n_items = BF16 ? NCP * ((NRT + RT - 1) / RT) : NCT * ((NRT + RTI - 1) / RTI);
  auto item = [&](uint32_t it) {
    const uint32_t lane = tid & 63;
    const uint32_t ci = it % NCT, rt0 = (it / NCT) * RTI;
    bool rok[RTI];
    uint32_t rtr[RTI];
#pragma unroll
    for (int r = 0; r < (int)RTI; ++r) {
      rtr[r] = 16 * (rt0 + r) + (lane & 15);
      rok[r] = rtr[r] < N;
    }
    if constexpr (BF16) {
      // items of the first (full) group of output tiles first: the group that
      // holds the last tiles can be narrower, and its shorter items end the
      // stage with less of a tail
      const uint32_t NRG = (NRT + RT - 1) / RT;
      const uint32_t c0 = BCT * (it / NRG), rb0 = (it % NRG) * RT;
      const uint32_t ncol = min(NCT - c0, (uint32_t)BCT);
      bool rok2[RT];
      uint32_t rtr2[RT];
#pragma unroll
      for (int r = 0; r < RT; ++r) {
        rtr2[r] = 16 * (rb0 + r) + (lane & 15);
        rok2[r] = rtr2[r] < N;
      }
      f4v acc[BCT][RT], ab[BCT][RT];
      tiles_bf16(Tg, oc, Dk, rok2, rtr2, R32 + (size_t)(16 * c0 + (lane & 15)) * Rs, ncol, Rs,
                 lane, acc, ab);
#pragma unroll
      for (int c = 0; c < BCT; ++c) {
        if ((uint32_t)c >= ncol) break;
#pragma unroll
        for (int r = 0; r < RT; ++r) {
          const float z[4] = {acc[c][r][0], acc[c][r][1], acc[c][r][2], acc[c][r][3]};
          const float e[4] = {E_AB * ab[c][r][0], E_AB * ab[c][r][1], E_AB * ab[c][r][2],
                              E_AB * ab[c][r][3]};
          tile_epilogue<true, false>(p, ek_s, ew_s, z, rtr2[r], rok2[r], e, D, c0 + c, N, lane,
                                     Ps, Pb, zf, zl);
        }
      }
    } else {
      d4v acc[RTF];
      tiles_f64(Tg, Dk, rok, rtr, R32, Rs, 16 * ci + (lane & 15), lane, acc);
#pragma unroll
      for (int r = 0; r < RTF; ++r) {
        float z[4];
        tile_z(acc[r], ro_s, ci, lane, z);
        const float e0[4] = {0.0f, 0.0f, 0.0f, 0.0f};
        tile_epilogue<false, true>(p, ek_s, ew_s, z, rtr[r], rok[r], e0, D, ci, N, lane, Ps, Pb,
                                   zf, zl);
      }
    }
  };
  // bf16 mode: one (output tile, row tile group) item of the exact re-evaluation
  // of the candidate list (total candidates, cl), run by consumers and producers
  auto reeval = [&](uint32_t it, uint32_t total) {
    const uint32_t lane = tid & 63;
    const uint32_t ci = it % NCT, rt0 = (it / NCT) * RT;
    bool rok[RT];
    uint32_t rtr[RT];
#pragma unroll
    for (int r = 0; r < RT; ++r) {
      const uint32_t srow = 16 * (rt0 + r) + (lane & 15);
      rok[r] = srow < total;
      rtr[r] = rok[r] ? cl[srow] : 0u;
    }
    d4v acc[RT];
    tiles_f64(Tg, Dk, rok, rtr, R32, Rs, 16 * ci + (lane & 15), lane, acc);
#pragma unroll
    for (int r = 0; r < RT; ++r) {
      float z[4];
      tile_z(acc[r], ro_s, ci, lane, z);
      const uint32_t slot = 16 * (rt0 + r) + (lane & 15);
      const float e0[4] = {0.0f, 0.0f, 0.0f, 0.0f};
      tile_epilogue<false, true>(p, ek_s, ew_s, z, slot, rok[r], e0, D, ci, N, lane, Ps, Pb, zf,
                                 zl);
    }
  };
  // the role is uniform per wave (whole waves on either side of MF_CONSUMERS)
  if (__builtin_amdgcn_readfirstlane(tid >> 6) >= MF_CONSUMERS / 64) {
    mfma_producers<BF16>(lay, smem, run, g0, n_gens, k0, k1, tid - MF_CONSUMERS, cnt + 15,
                         n_items, item, cnt, reeval);
  } else {
  constexpr bool producer = false;
  const uint32_t lane = tid & 63;
  const uint32_t wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  // ranking geometry: L parts of Np lanes
  const uint32_t l = __builtin_amdgcn_readfirstlane(tid / Np);
  const uint32_t ir = tid - l * Np;
  const bool act_r = l < L && ir < N;
  const uint32_t kr0 = l * N / L, kr1 = (l + 1) * N / L;
  // decision lane of trial tid
  const bool dec = tid < N;
  const int use_rand = (run.bl == RAND || run.br == RAND) ? 1 : 0;
  // trial construction: P lanes per trial, the largest power of two <= 32 with N P <= consumers
  uint32_t P = 1;
  while (P < 32 && N * (2 * P) <= MF_CONSUMERS) P *= 2;
  __syncthreads();   // draws of the first generation are being made
  unsigned long long refined = 0;
  BoundCheck chk{0, 0, 0, 0, 0.0};
  MDE_STAGE_BEGIN

  for (uint32_t gg = 0; gg < n_gens; ++gg) {
    const uint32_t g = g0 + gg;
    MDE_STAGE_WORK(8)
    __syncthreads();
    MDE_STAGE(0)
    // S0: partial ranks
    if (act_r) {
      const uint64_t ki = key_s[ir];
      uint32_t c = 0, j = kr0;
      for (; j + 16 <= kr1; j += 16) {
        uint64_t kv[16];
#pragma unroll
        for (int q = 0; q < 16; ++q) kv[q] = key_s[j + q];
#pragma unroll
        for (int q = 0; q < 16; ++q) c += kv[q] < ki ? 1u : 0u;
      }
      for (; j + 8 <= kr1; j += 8) {
        uint64_t kv[8];
#pragma unroll
        for (int q = 0; q < 8; ++q) kv[q] = key_s[j + q];
#pragma unroll
        for (int q = 0; q < 8; ++q) c += kv[q] < ki ? 1u : 0u;
      }
      for (; j < kr1; ++j) c += key_s[j] < ki ? 1u : 0u;
      rk[l * Np + ir] = c;
    }
    MDE_STAGE_WORK(9)
    __syncthreads();
    MDE_STAGE(1)
    // S1: top-p list; the decision lane keeps its target's fitness
    float fx = 0.0f;
    if (dec) fx = fit_s[tid];
    if (act_r && l == 0) {
      uint32_t rank = 0;
      for (uint32_t ll = 0; ll < L; ++ll) rank += rk[ll * Np + ir];
      if (rank < kp) topk[rank] = ir;
    }
    MDE_STAGE_WORK(10)
    __syncthreads();
    MDE_STAGE(2)
    // S2: trial genes -> global trial rows.  P lanes per trial (a power of
    // two, as many as the consumers allow) take its quads in turn.
    if (tid == 0) cnt[15] = 0;   // the rotation's item counter
    const uint8_t *mg = msk + ((g & 1u) && lay.msk2 != lay.msk ? lay.msk2 - lay.msk : 0u);
    if (!producer) {
      const uint32_t lp = tid & (P - 1), per = MF_CONSUMERS / P;
      for (uint32_t i0 = 0; i0 < N; i0 += per) {
        const uint32_t i = i0 + tid / P;
        const bool valid = i < N;
        if (valid) {
          const uint4 d = dsc[i];
          const uint32_t r0 = byte_of(d.z, 0), pb = byte_of(d.z, 1);
          const uint32_t ibest = topk[0], ipb = topk[pb];
          const uint32_t ibl = run.bl == RAND ? r0 : (run.bl == BEST ? ibest : (run.bl == PBEST ? ipb : i));
          const uint32_t ibr = run.br == RAND ? r0 : (run.br == BEST ? ibest : (run.br == PBEST ? ipb : i));
          for (uint32_t q = lp; q < Q; q += P) {
            const uint32_t nib = run.cs == BIN ? mg[i * Q + q] : 0u;
            const float4 uu = trial_quad(pop_s, Dp, D, i, q, ibl, ibr, d, nib, run, lb, ub);
            *reinterpret_cast<float4 *>(Tg + (size_t)i * Dk + 4 * q) = uu;
            if (TRACE) {
#pragma unroll
              for (int t = 0; t < 4; ++t)
                if (4 * q + t < D) tr.u[run.pop_off + (size_t)i * D + 4 * q + t] = comp(uu, t);
            }
          }
          if (TRACE && lp == 0) {
            int32_t *o = tr.desc + (size_t)(run.fit_off + i) * 16;
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
        }
      }
    }
    MDE_STAGE_WORK(11)
    __syncthreads();
    MDE_STAGE(3)
    // S3: rotation on the matrix cores + element terms (the producers join
    // once the masks of g+1 are drawn)
    rotation_items(cnt + 15, n_items, lane, item);
    MDE_STAGE_WORK(12)
    __syncthreads();
    MDE_STAGE(4)
    // S4: plain mode decides and commits; bf16 mode selects the candidates
    bool cand = false, screen = false;
    float fh = 0.0f;
    double bnd = 0.0;
    if (dec) {
      fh = combine(p, Ps, zf, zl, NCT, D, N, tid);
      if (!BF16) {
        const bool a = accept_trial(fh, fx);
        if (a) {
          const float *trow = Tg + (size_t)tid * Dk;
          for (uint32_t q = 0; q < Q; ++q)
            st4(pop_s, tid * Dp + 4 * q, *reinterpret_cast<const float4 *>(trow + 4 * q));
          fit_s[tid] = fh;
          key_s[tid] = mkkey(fh, tid);
        }
        if (TRACE) {
          tr.fu[run.fit_off + tid] = fh;
          tr.desc[(size_t)(run.fit_off + tid) * 16 + 15] = a ? 1 : 0;
        }
      } else {
        for (uint32_t c2 = 0; c2 < NCT; ++c2) bnd += (double)Pb[c2 * N + tid];
        bnd += 9.5367e-7 * (double)fabsf(fh);
        screen = (fh == fh) && !((double)fh - bnd > (double)fx);
        // traced generations re-evaluate every trial, so that each bf16 value
        // can be checked against its bound (the decisions are unchanged)
        cand = TRACE ? true : screen;
      }
    }
    if (BF16) {
      // deterministic compaction of the candidates (ascending trial index)
      const unsigned long long bal = __ballot(cand);
      if (!producer && lane == 0) cnt[wave] = (uint32_t)__popcll(bal);
      MDE_STAGE_WORK(13)
      __syncthreads();
      MDE_STAGE(5)
      uint32_t base = 0, total = 0;
      for (uint32_t w = 0; w < MF_CONSUMERS / 64; ++w) {
        const uint32_t cw = cnt[w];
        if (w < wave) base += cw;
        total += cw;
      }
      if (cand) {
        const uint32_t pos = base + (uint32_t)__popcll(bal & ((1ull << lane) - 1ull));
        cl[pos] = tid;
      }
      MDE_STAGE_WORK(14)
      __syncthreads();
      MDE_STAGE(6)
      // S5: plain re-evaluation of the candidates on compacted row tiles,
      // (output tile, row tile group) items dealt to all twelve waves (the
      // producers take items 8..11, 20..23, ...)
      if (!producer) {
        const uint32_t n_re = NCT * (((total + 15) / 16 + RT - 1) / RT);
        for (uint32_t it = wave; it < n_re; it += MF_THREADS / 64) reeval(it, total);
      }
      MDE_STAGE_WORK(15)
      __syncthreads();
      MDE_STAGE(7)
      // S6: decisions of the candidates from their plain values, commit
      if (!producer && tid < total) {
        const uint32_t t = cl[tid];
        const float f = combine(p, Ps, zf, zl, NCT, D, N, tid);
        const bool a = accept_trial(f, fit_s[t]);
        if (a) {
          const float *trow = Tg + (size_t)t * Dk;
          for (uint32_t q = 0; q < Q; ++q)
            st4(pop_s, t * Dp + 4 * q, *reinterpret_cast<const float4 *>(trow + 4 * q));
          fit_s[t] = f;
          key_s[t] = mkkey(f, t);
        }
        if (TRACE) {
          // every trial is a candidate here and the list is in trial order,
          // so t == tid and fh, bnd, screen of this lane belong to trial t
          tr.fu[run.fit_off + t] = f;
          tr.desc[(size_t)(run.fit_off + t) * 16 + 15] = a ? 1 : 0;
          ++chk.checked;
          if (f == f && fh == fh) {
            const double dev = fabs((double)fh - (double)f);
            if (dev > bnd) ++chk.outside;
            if (bnd > 0.0) chk.max_ratio = fmax(chk.max_ratio, dev / bnd);
          }
          if (!screen) {
            ++chk.screened;
            if (a) ++chk.screen_wrong;
          }
        }
      }
      refined += total;
    }
  }
  MDE_STAGE_WORK(8)
  __syncthreads();
  MDE_STAGE(0)
  MDE_STAGE_END
  if (BF16 && tid == 0) atomicAdd(counters, refined);
  if (BF16 && TRACE) {
    if (chk.checked) atomicAdd(counters + 1, chk.checked);
    if (chk.outside) atomicAdd(counters + 2, chk.outside);
    if (chk.screened) atomicAdd(counters + 3, chk.screened);
    if (chk.screen_wrong) atomicAdd(counters + 4, chk.screen_wrong);
    // non-negative doubles order like their bit patterns
    if (chk.max_ratio > 0.0)
      atomicMax(counters + 5, (unsigned long long)__double_as_longlong(chk.max_ratio));
  }
  }
  for (uint32_t u = tid; u < N * D; u += MF_THREADS) {
    const uint32_t r = u / D, j = u - r * D;
    pop[run.pop_off + u] = pop_s[r * Dp + j];
  }
  for (uint32_t r = tid; r < N; r += MF_THREADS) fit[run.fit_off + r] = fit_s[r];
}

template <bool BF16, bool TRACE, int RTF>
__global__ __launch_bounds__(MF_THREADS) void k_generations_mfma(
    const RunDev *__restrict__ runs, const uint32_t *__restrict__ list,
    const ProbDev *__restrict__ probs, const unsigned char *__restrict__ tab,
    float *__restrict__ pop, float *__restrict__ fit, uint32_t g0, uint32_t n_gens, uint32_t k0,
    uint32_t k1, float lb, float ub, float *__restrict__ tbuf,
    unsigned long long *__restrict__ counters, TraceArgs tr) {
  extern __shared__ __align__(16) unsigned char smem[];
  const RunDev run = runs[list[blockIdx.x]];
  ProbDev p = probs[run.prob];
  // one copy of the generation loop per function kind (the kind is a
  // constant inside each case)
#define MDE_KIND(K)                                                                     \
  case K:                                                                               \
    p.kind = K;                                                                         \
    mfma_body<BF16, TRACE, RTF>(smem, run, p, tab, pop, fit, g0, n_gens, k0, k1, lb, ub, \
                           tbuf + run.pend_off, counters, tr);                          \
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

// Padded float32 rotation [Rs][Rs] (zero outside D x D) and R o in float64
// (k ascending, one fused multiply-add per term; zero past D).
__global__ void k_tables_mfma(const float *__restrict__ R, const float *__restrict__ o,
                              float *__restrict__ R32, double *__restrict__ ro64, uint32_t D,
                              uint32_t Rs) {
  const uint32_t u = blockIdx.x * blockDim.x + threadIdx.x;
  if (u >= Rs * Rs) return;
  const uint32_t j = u / Rs, k = u - j * Rs;
  R32[u] = (j < D && k < D) ? R[(size_t)j * D + k] : 0.0f;
  if (k == 0) {
    double acc = 0.0;
    if (j < D)
      for (uint32_t kk = 0; kk < D; ++kk) acc = fma((double)R[(size_t)j * D + kk], (double)o[kk], acc);
    ro64[j] = acc;
  }
}

hipError_t launch_tables_mfma(const float *R, const float *o, float *R32, double *ro64, uint32_t D,
                              hipStream_t s) {
  const uint32_t Rs = r32_stride(D);
  hipLaunchKernelGGL(k_tables_mfma, dim3((Rs * Rs + 255) / 256), dim3(256), 0, s, R, o, R32, ro64,
                     D, Rs);
  return hipGetLastError();
}

#ifdef MDE_STAGE_CLOCKS
hipError_t read_stage_clocks_mfma(void *dst, size_t bytes) {
  return hipMemcpyFromSymbol(dst, HIP_SYMBOL(mde_stage_clk), bytes, 0, hipMemcpyDeviceToHost);
}
#endif

hipError_t set_lds_limits_mfma() {
  const void *ks[6] = {(const void *)k_generations_mfma<false, false, 2>,
                       (const void *)k_generations_mfma<false, true, 2>,
                       (const void *)k_generations_mfma<false, false, 4>,
                       (const void *)k_generations_mfma<false, true, 4>,
                       (const void *)k_generations_mfma<true, false, RT>,
                       (const void *)k_generations_mfma<true, true, RT>};
  for (const void *k : ks) {
    hipError_t e = hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, LDS_BUDGET);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t launch_generations_mfma(const LaunchArgs &a, const uint32_t *list, uint32_t n,
                                   bool bf16, uint32_t g0, uint32_t n_gens, float lb, float ub,
                                   unsigned long long *counters, TraceArgs tr) {
  if (n == 0) return hipSuccess;
  const bool trace = tr.u != nullptr;
#define MDE_LAUNCH(B, T, R)                                                                    \
  hipLaunchKernelGGL(HIP_KERNEL_NAME(k_generations_mfma<B, T, R>), dim3(n), dim3(MF_THREADS),  \
                     a.mfma_lds_bytes, a.stream, a.runs, list, a.probs, a.tab, a.pop, a.fit, g0, \
                     n_gens, a.k0, a.k1, lb, ub, a.pending, counters, tr)
  if (bf16) {
    if (trace) MDE_LAUNCH(true, true, RT); else MDE_LAUNCH(true, false, RT);
  } else if (a.mfma_rows == 2) {
    if (trace) MDE_LAUNCH(false, true, 2); else MDE_LAUNCH(false, false, 2);
  } else {
    if (trace) MDE_LAUNCH(false, true, 4); else MDE_LAUNCH(false, false, 4);
  }
#undef MDE_LAUNCH
  return hipGetLastError();
}

}  // namespace mde
