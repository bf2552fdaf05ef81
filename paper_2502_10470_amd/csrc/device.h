// Device-side building blocks of the MetaDE inner-DE path (gfx950).
//
// Everything here follows the paper's Parameterized DE (Sec. III-A, Alg. 2)
// and MetaDE (Alg. 3); random numbers come from Philox4x32-10 (Salmon et al.,
// SC'11).  Floating-point DE arithmetic is float32 with one rounding per
// operation and no contraction (the library is compiled with
// -ffp-contract=off), so trial vectors are bit-reproducible.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mde {

// ---------------------------------------------------------------- constants

constexpr uint32_t PH_M0 = 0xD2511F53u;
constexpr uint32_t PH_M1 = 0xCD9E8D57u;
constexpr uint32_t PH_W0 = 0x9E3779B9u;
constexpr uint32_t PH_W1 = 0xBB67AE85u;
constexpr uint32_t INIT_PHASE = 0xFFFFFFFFu;
constexpr uint32_t OUTER_BIT = 0x80000000u;

enum Base { RAND = 1, BEST = 2, PBEST = 3, CURRENT = 4 };
enum Cross { BIN = 1, EXP = 2, ARITH = 3 };
enum Word { W_PBEST = 9, W_JRAND = 10, W_K = 11, W_GENE0 = 12 };
enum Kind { FN_RASTRIGIN = 1, FN_ROSENBROCK = 2, FN_ACKLEY = 3, FN_ELLIPTIC = 4,
            FN_SCHWEFEL = 5, FN_HYBRID = 6, FN_LQR_MLP = 7 };

constexpr int MAX_N = 256;     // LDS-resident kernel: indices fit in 8 bits
constexpr int MAX_D = 128;
constexpr int MAX_KP = 32;     // top-p set size for N <= 256 is at most 26
constexpr uint32_t LDS_BUDGET = 160 * 1024;
// control workload: the larger policy hidden width (the smaller one, 32, is
// declared with the launch interface), bounded observation / action sizes
constexpr int CT_H = 64;
constexpr int CT_MAX_OBS = 20;
constexpr int CT_MAX_ACT = 8;
constexpr int CT_MAX_N = 1024;
constexpr float SCHWEFEL_ZSTAR = 420.96875f;

// ---------------------------------------------------------------- stage clocks
//
// Diagnostic builds only (compiled with MDE_STAGE_CLOCKS): every wave of a
// generation kernel adds the cycles it spends in each stage of every
// generation to a per-(block, wave, stage) total, written once at the end of
// the launch to a device array of the kernel's source file.  In ordinary
// builds the hooks expand to nothing.
#ifdef MDE_STAGE_CLOCKS
constexpr int STAGE_MAX_BLOCKS = 256, STAGE_MAX_WAVES = 16, STAGE_N = 16;
#define MDE_STAGE_ARRAY \
  static __device__ unsigned long long mde_stage_clk[STAGE_MAX_BLOCKS * STAGE_MAX_WAVES * STAGE_N]
#define MDE_STAGE_BEGIN                         \
  unsigned long long mde_st_t = clock64();      \
  unsigned long long mde_st_acc[STAGE_N] = {};
#define MDE_STAGE(k)                            \
  {                                             \
    const unsigned long long t_ = clock64();    \
    mde_st_acc[k] += t_ - mde_st_t;             \
    mde_st_t = t_;                              \
  }
// the cycles since the last MDE_STAGE, without starting a new interval: placed
// just before a barrier, the wave's own work in the stage, its wait left out
#define MDE_STAGE_WORK(k) \
  { mde_st_acc[k] += clock64() - mde_st_t; }
#define MDE_STAGE_END                                                                  \
  if ((threadIdx.x & 63) == 0 && blockIdx.x < (unsigned)STAGE_MAX_BLOCKS)             \
    for (int k_ = 0; k_ < STAGE_N; ++k_)                                               \
      mde_stage_clk[(blockIdx.x * STAGE_MAX_WAVES + threadIdx.x / 64) * STAGE_N + k_] = \
          mde_st_acc[k_];
#else
#define MDE_STAGE_ARRAY
#define MDE_STAGE_BEGIN
#define MDE_STAGE(k)
#define MDE_STAGE_WORK(k)
#define MDE_STAGE_END
#endif

// ---------------------------------------------------------------- tables

// One executor run.  Theta fields are written by the decode kernel.
struct RunDev {
  uint32_t N, D, Dp, prob;      // Dp = D rounded up to a multiple of 4
  uint32_t stream, kp;          // kp = top-p count
  uint32_t L, Np;               // lanes per trial (parts) and lanes per part (multiple of 64)
  uint32_t t_lds, kern;         // trial rows in LDS (1, lane kernel) or global (0); kernel: 0 lanes, 1 matrix cores, 2 control
  uint32_t Dk, NCT;             // matrix-core kernel: D rounded up to 32; 16-wide output tiles
  uint64_t pop_off;             // float offset of the run in pop (N*D packing)
  uint64_t pend_off;            // float offset in the global trial buffer
  uint32_t fit_off, bx_off;     // offsets in fit / best_x
  float F, CR;
  int32_t bl, br, dn, cs;
};

// One problem instance.  Its arrays live in the library's read-only table
// buffer (one allocation for all problems), addressed by byte offsets so that
// every kernel reads them through one const __restrict__ pointer: uniform
// reads then become scalar loads.
struct ProbDev {
  uint32_t kind, D;
  float bias, cs_f;             // cs = Schwefel constant z* sin(sqrt z*)
  double cs_d;
  uint64_t o_off;               // float  [D]    shift
  uint64_t r64t_off;            // double [D][rt_stride] rotation transposed: (k, j) = R[j][k]
  uint64_t r32_off;             // float  [Rs][Rs] row-major R zero padded to Rs = r32_stride(D)
  uint64_t ro64_off;            // double [Rs]   R o (zero past D): z = R u - R o
  uint64_t ew_off;              // float  [D]    elliptic weight of output j
  uint64_t ew64_off;            // double [D]    same in float64
  uint64_t ek_off;              // uint32 [D]    hybrid block of output j (0 Schwefel, 1 Rastrigin, 2 elliptic)
  // control workload
  uint32_t obs, act, h1, h2, steps, nroll;
  float cw, pad0;
  uint64_t A_off, B_off, x0_off;  // float [obs*obs], [obs*act], [nroll*obs], row-major
};

// Row stride of the transposed float64 rotation: D plus zero padding for the
// widest output block (16), rounded to 4 doubles.
__host__ __device__ inline uint32_t rt_stride(uint32_t D) { return ((D + 16u) + 3u) & ~3u; }
// Rows and row stride of the padded float32 rotation the matrix-core kernel
// reads: D rounded up to whole 16-wide tiles in both directions.
__host__ __device__ inline uint32_t r32_stride(uint32_t D) { return (D + 15u) & ~15u; }

template <typename T>
__host__ __device__ __forceinline__ const T *tab_ptr(const unsigned char *tab, uint64_t off) {
  return reinterpret_cast<const T *>(tab + off);
}

// ---------------------------------------------------------------- Philox4x32-10

__device__ __forceinline__ uint4 philox(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                        uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    const uint64_t p0 = (uint64_t)PH_M0 * c0;
    const uint64_t p1 = (uint64_t)PH_M1 * c2;
    const uint32_t n0 = (uint32_t)(p1 >> 32) ^ c1 ^ k0;
    const uint32_t n2 = (uint32_t)(p0 >> 32) ^ c3 ^ k1;
    c1 = (uint32_t)p1;
    c3 = (uint32_t)p0;
    c0 = n0;
    c2 = n2;
    k0 += PH_W0;
    k1 += PH_W1;
  }
  return make_uint4(c0, c1, c2, c3);
}

__device__ __forceinline__ uint32_t word_of(const uint4 &w, int t) {
  return t == 0 ? w.x : (t == 1 ? w.y : (t == 2 ? w.z : w.w));
}

// floor(w * m / 2^32)
__device__ __forceinline__ uint32_t lemire(uint32_t w, uint32_t m) { return __umulhi(w, m); }

// ((w >> 8) + 1) 2^-24 in (0, 1], exact in float32
__device__ __forceinline__ float unit_oc(uint32_t w) {
  return (float)((w >> 8) + 1u) * 0x1p-24f;
}

// ---------------------------------------------------------------- ordering

// Total order key of a fitness value: NaN counts as +inf, -0 as +0.
__device__ __forceinline__ uint32_t okey(float f) {
  if (f != f) f = __int_as_float(0x7F800000);
  if (f == 0.0f) f = 0.0f;
  const uint32_t b = __float_as_uint(f);
  return (b & 0x80000000u) ? ~b : (b | 0x80000000u);
}

// Selection rule: accept iff f(u) <= f(x), never a NaN trial, NaN target = +inf.
__device__ __forceinline__ bool accept_trial(float fu, float fx) {
  return (fu == fu) && ((fx != fx) || fu <= fx);
}
__device__ __forceinline__ bool accept_trial_d(double fu, double fx) {
  return (fu == fu) && ((fx != fx) || fu <= fx);
}

// ---------------------------------------------------------------- LDS layout

// Block shape of the generation kernel: GEN_THREADS lanes, the first half
// consumers (the generation's ranking, mutation, fitness and commit), the
// second half producers (the next generation's random draws).  Consumer lanes
// form L parts of Np lanes (Np a multiple of the wave size, Np >= N).
constexpr uint32_t GEN_THREADS = 1024;
constexpr uint32_t GEN_CONSUMERS = GEN_THREADS / 2;
constexpr uint32_t INIT_THREADS = 256;

// LDS of the generation kernel: population [N][Dp] (row-major, float4 rows
// for the gathers of the mutation), 64-bit ranking keys, fitness, the top-p
// list, per-part partial fitness sums, the producers' binomial mask
// nibbles [2][N][Q] (two generations) and packed draws [N], and -- when it
// fits -- the trial rows stored gene-major ([D][Np]) so that lane i reading
// gene k of its own trial touches consecutive words.
struct Lds {
  uint32_t pop, key, fit, fx, topk, ps, msk, dsc, T, total;
};

__host__ __device__ inline uint32_t al16(uint32_t b) { return (b + 15u) & ~15u; }

__host__ __device__ inline Lds lds_layout(uint32_t N, uint32_t Dp, uint32_t L, uint32_t Np,
                                          bool t_lds) {
  Lds l;
  uint32_t o = 0;
  l.pop = o;  o += al16(N * Dp * 4);
  l.key = o;  o += al16(N * 8);
  l.fit = o;  o += al16(N * 4);
  l.fx = o;   o += al16(N * 4);         // targets' fitness, frozen for the commit
  l.topk = o; o += al16(MAX_KP * 4);
  l.ps = o;   o += al16(L * Np * 16);
  l.msk = o;  o += al16(2 * N * (Dp / 4));   // two generations: read g, write g+1
  l.dsc = o;  o += al16(N * 16);
  l.T = o;    o += t_lds ? al16(Dp * Np * 4) : 0u;
  l.total = o;
  return l;
}

// Matrix-core generation kernel (runs whose trial rows do not fit in LDS, and
// the bf16 precision mode; 512 consumer + 256 producer lanes): trial rows live
// in a global buffer [N][Dk] (Dk = D rounded up to 32, zero padding); LDS
// holds the population, ranking state, the producers' mask
// nibbles and packed draws, per (output tile, trial) partial sums (and
// bounds in the bf16 mode), Rosenbrock
// boundary values, the shift, R o, the element kind and elliptic weight of
// every output, the candidate list of the bf16 mode and per-wave counts.
constexpr uint32_t MF_THREADS = 768;
constexpr uint32_t MF_CONSUMERS = 512;

struct MLds {
  uint32_t pop, key, fit, topk, rk, msk, dsc, ps, pb, zf, zl, oc, ro, ek, ew, cl, cnt, msk2, total;
};

__host__ __device__ inline MLds mfma_layout(uint32_t N, uint32_t Dp, uint32_t Dk, uint32_t L,
                                            uint32_t Np, uint32_t NCT, bool rosen, bool bf16) {
  MLds l;
  uint32_t o = 0;
  l.pop = o;  o += al16(N * Dp * 4);
  l.key = o;  o += al16(N * 8);
  l.fit = o;  o += al16(N * 4);
  l.topk = o; o += al16(MAX_KP * 4);
  l.rk = o;   o += al16(L * Np * 4);
  l.msk = o;  o += al16(N * (Dp / 4));
  l.dsc = o;  o += al16(N * 16);
  l.ps = o;   o += al16(NCT * N * 8);
  l.pb = o;   o += bf16 ? al16(NCT * N * 4) : 0u;
  l.zf = o;   o += rosen ? al16(NCT * N * 4) : 0u;
  l.zl = o;   o += rosen ? al16(NCT * N * 4) : 0u;
  l.oc = o;   o += al16(Dk * 4);
  l.ro = o;   o += al16(Dk * 8);
  l.ek = o;   o += al16(Dk * 4);
  l.ew = o;   o += al16(Dk * 4);
  l.cl = o;   o += bf16 ? al16(N * 4) : 0u;
  l.cnt = o;  o += al16(16 * 4);
  // plain mode: a second mask buffer where it fits, so that the producers
  // draw the next generation's crossover tests while the consumers build this
  // generation's trials (msk2 == msk: one buffer, the tests drawn during the
  // rotation, as in the bf16 mode, whose rotation is not bound by the float64
  // products)
  l.msk2 = l.msk;
  if (!bf16 && o + al16(N * (Dp / 4)) <= LDS_BUDGET) {
    l.msk2 = o;
    o += al16(N * (Dp / 4));
  }
  l.total = o;
  return l;
}

// LDS of the initialisation kernel: population and per-part partial sums.
__host__ __device__ inline uint32_t init_parts(uint32_t Np) {
  const uint32_t L = INIT_THREADS / Np;
  return L < 1 ? 1 : (L > 4 ? 4 : L);
}
__host__ __device__ inline uint32_t init_lds_bytes(uint32_t N, uint32_t Dp, uint32_t Np) {
  return al16(N * Dp * 4) + al16(init_parts(Np) * Np * 16);
}

// ---------------------------------------------------------------- sampler

// Index sampling without rejection: draw k is the t_k-th smallest element of
// {0..N-1} minus {i} minus the earlier draws, t_k = floor(w_k (N-1-k) / 2^32).
// The excluded set is kept sorted; skipping every excluded value <= r in
// ascending order turns the rank t into the element.
__device__ __forceinline__ void sample_distinct(const uint32_t *w, int m, uint32_t i, uint32_t N,
                                                uint32_t *draws) {
  uint32_t ex[10];  // ex[0..k] hold the k+1 excluded values in ascending order
  ex[0] = i;
#pragma unroll
  for (int k = 0; k < 9; ++k) {
    if (k < m) {
      uint32_t r = lemire(w[k], N - 1u - (uint32_t)k);
#pragma unroll
      for (int q = 0; q <= k; ++q) r += (ex[q] <= r) ? 1u : 0u;
      draws[k] = r;
      uint32_t carry = r;
#pragma unroll
      for (int q = 0; q <= k; ++q) {
        const uint32_t lo = min(carry, ex[q]);
        carry = max(carry, ex[q]);
        ex[q] = lo;
      }
      ex[k + 1] = carry;
    }
  }
}

// ---------------------------------------------------------------- math per precision

template <typename T> struct Math;

// sin(x) in float32 for |x| < 2^20 (the Schwefel term takes the sine of a
// square root, which stays far below that for any finite box of practical
// size): quadrant k = rint(2x / pi) and r = x - k pi/2 in float64 (|r| <= pi/4,
// error below 1e-10), then the Taylor series of sin r to degree 13 or of cos r
// to degree 12 in float64 (truncation below 4e-13) and one rounding.  Compact
// enough to inline at every output of a fitness block.
__device__ __forceinline__ float sin_reduced(float xf) {
  const double x = (double)xf;
  const double k = rint(x * 0.63661977236758134308);
  const double r = fma(-k, 1.57079632679489661923, x);
  const double r2 = r * r;
  double ps = 1.0 / 6227020800.0;
  ps = fma(ps, r2, -1.0 / 39916800.0);
  ps = fma(ps, r2, 1.0 / 362880.0);
  ps = fma(ps, r2, -1.0 / 5040.0);
  ps = fma(ps, r2, 1.0 / 120.0);
  ps = fma(ps, r2, -1.0 / 6.0);
  const double sv = fma(ps * r2, r, r);
  double pc = 1.0 / 479001600.0;
  pc = fma(pc, r2, -1.0 / 3628800.0);
  pc = fma(pc, r2, 1.0 / 40320.0);
  pc = fma(pc, r2, -1.0 / 720.0);
  pc = fma(pc, r2, 1.0 / 24.0);
  pc = fma(pc, r2, -0.5);
  const double cv = fma(pc, r2, 1.0);
  const int q = (int)(int64_t)k & 3;
  const double v = (q & 1) ? cv : sv;
  return (float)((q & 2) ? -v : v);
}

template <> struct Math<float> {
  // cos(2 pi z): exact reduction r = z - rint(z) in [-1/2, 1/2], then the
  // hardware cosine, whose argument is in revolutions
  static __device__ __forceinline__ float cos2pi(float z) {
    const float r = z - rintf(z);
    return __builtin_amdgcn_cosf(r);
  }
  static __device__ __forceinline__ float sin_(float x) { return sin_reduced(x); }
  static __device__ __forceinline__ float sqrt_(float x) { return sqrtf(x); }
  static __device__ __forceinline__ float exp_(float x) { return expf(x); }
  static __device__ __forceinline__ float exp2_(float x) { return exp2f(x); }
  static __device__ __forceinline__ float abs_(float x) { return fabsf(x); }
};

template <> struct Math<double> {
  static __device__ __forceinline__ double cos2pi(double z) {
    const double r = z - rint(z);
    return cospi(2.0 * r);
  }
  static __device__ __forceinline__ double sin_(double x) { return sin(x); }
  static __device__ __forceinline__ double sqrt_(double x) { return sqrt(x); }
  static __device__ __forceinline__ double exp_(double x) { return exp(x); }
  static __device__ __forceinline__ double exp2_(double x) { return exp2(x); }
  static __device__ __forceinline__ double abs_(double x) { return fabs(x); }
};

template <typename T> __device__ __forceinline__ T schwefel_cs(const ProbDev &p);
template <> __device__ __forceinline__ float schwefel_cs<float>(const ProbDev &p) { return p.cs_f; }
template <> __device__ __forceinline__ double schwefel_cs<double>(const ProbDev &p) { return p.cs_d; }
template <typename T> __device__ __forceinline__ T ell_w(const unsigned char *tab, const ProbDev &p, uint32_t j);
template <> __device__ __forceinline__ float ell_w<float>(const unsigned char *tab, const ProbDev &p, uint32_t j) {
  return tab_ptr<float>(tab, p.ew_off)[j];
}
template <> __device__ __forceinline__ double ell_w<double>(const unsigned char *tab, const ProbDev &p, uint32_t j) {
  return tab_ptr<double>(tab, p.ew64_off)[j];
}

template <typename T> __device__ __forceinline__ T h_rastrigin(T v) {
  return (v * v - T(10) * Math<T>::cos2pi(v)) + T(10);
}
template <typename T> __device__ __forceinline__ T h_schwefel(const ProbDev &p, T v) {
  using Mt = Math<T>;
  const T x = v + T(SCHWEFEL_ZSTAR);
  return schwefel_cs<T>(p) - x * Mt::sin_(Mt::sqrt_(Mt::abs_(x)));
}
template <typename T> __device__ __forceinline__ T h_rosenbrock(T v, T vn) {
  const T a = v + T(1);
  const T b = vn + T(1);
  const T c = a * a - b;
  const T e = a - T(1);
  return T(100) * (c * c) + e * e;
}

// Term of output j (value v) for every kind but Rosenbrock, whose term pairs
// z_j with z_{j+1} and is formed by the caller.  t1 is Ackley's cosine sum.
template <typename T>
__device__ __forceinline__ void elem_term(const unsigned char *tab, const ProbDev &p, uint32_t j,
                                          T v, T &t0, T &t1) {
  t1 = T(0);
  switch (p.kind) {
    case FN_RASTRIGIN: t0 = h_rastrigin<T>(v); break;
    case FN_ELLIPTIC: t0 = ell_w<T>(tab, p, j) * (v * v); break;
    case FN_ACKLEY: t0 = v * v; t1 = Math<T>::cos2pi(v); break;
    case FN_SCHWEFEL: t0 = h_schwefel<T>(p, v); break;
    case FN_HYBRID: {
      const uint32_t e = tab_ptr<uint32_t>(tab, p.ek_off)[j];
      t0 = e == 0 ? h_schwefel<T>(p, v) : (e == 1 ? h_rastrigin<T>(v) : ell_w<T>(tab, p, j) * (v * v));
      break;
    }
    default: t0 = T(0);
  }
}

// Final value from the summed terms.
template <typename T>
__device__ __forceinline__ T fn_finish(const ProbDev &p, T s0, T s1) {
  using Mt = Math<T>;
  if (p.kind == FN_ACKLEY) {
    const T n = T(p.D);
    const T e = T(2.718281828459045);
    return ((T(-20) * Mt::exp_(T(-0.2) * Mt::sqrt_(s0 / n)) - Mt::exp_(s1 / n)) + T(20) + e) + T(p.bias);
  }
  return s0 + T(p.bias);
}

}  // namespace mde
