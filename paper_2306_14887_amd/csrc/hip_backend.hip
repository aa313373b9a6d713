// HIP/CDNA4 (gfx950) kernels and the device backend of the bpki engine.
//
//  * gemm_kernel: grouped, batched complex GEMM on MFMA (FP64: v_mfma_f64_16x16x4f64; FP32 mode:
//                 v_mfma_f32_16x16x4f32 with FP64 storage and FP64 split-K sums).  Complex
//                 products by the 3M method: three real MFMA accumulators per 16x16 tile,
//                 P1 = sum re*re, P2 = sum im*im, P3 = sum (re+im)*(re+im), combined in the
//                 epilogue as re = P1 - P2, im = P3 - P1 - P2.  Operands are staged
//                 through LDS in split re/im planes; the global loads follow whichever index is
//                 unit-stride so they coalesce for every leg ordering of the site tensors.
//  * eigh: batched Hermitian eigendecomposition in FP64.  n < 32: cyclic Jacobi in LDS with
//          the parallel round-robin ordering (n/2 disjoint rotations per round, all 2x2 block
//          updates of a round in parallel).  32 <= n <= 256: Householder tridiagonalisation
//          and divide and conquer, one workgroup per matrix (matrix in LDS up to n = 128, in
//          an L2-resident work area above), then a column-parallel back-transformation.
//  * small kernels for the X rotations, message square roots, Gram factor, the gate block,
//    truncation, BP normalisation/residual and the site density matrices.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <type_traits>
#include <utility>
#include <vector>

#include "bpki_internal.h"

namespace bpki {

typedef double double4_t __attribute__((ext_vector_type(4)));
typedef float float4_t __attribute__((ext_vector_type(4)));

#define HIPCHK(x)                                                                    \
  do {                                                                               \
    hipError_t e_ = (x);                                                             \
    if (e_ != hipSuccess && err_ == 0) {                                             \
      err_ = -5;                                                                     \
      errmsg_ = std::string(#x) + ": " + hipGetErrorString(e_);                      \
    }                                                                                \
  } while (0)

// ------------------------------------------------------------------------------------------
// GEMM
namespace {
constexpr int BM = 64, BN = 64, BK = 16, PAD = 1;
constexpr int LOADS = (BM * BK) / 256;   // complex elements each thread stages per operand
}

__device__ __forceinline__ long cidx(int i, int inner, long so, long si) {
  return (long)(i / inner) * so + (long)(i % inner) * si;
}

// Offsets of the K part of an operand for a whole K tile starting at k0.  When Ki is a
// multiple of BK the tile never straddles an outer index, so the division happens once per
// tile; otherwise per element.
struct KOff {
  long base;
  long si;
  bool uniform;
};

__device__ __forceinline__ KOff k_tile(int k0, int Ki, long so, long si) {
  KOff r;
  r.uniform = (Ki % BK) == 0;
  r.base = r.uniform ? (long)(k0 / Ki) * so + (long)(k0 % Ki) * si : 0;
  r.si = si;
  return r;
}

// Loads and stores in the global address space.  The kernels reach their operands through device
// arrays of pointers, which the compiler can only treat as generic (flat) addresses; a flat load
// counts against both the vector-memory and the LDS counters, so every wait for an LDS read then
// also waits for all loads in flight (prefetches included).  Accessed through these, the same
// addresses become global loads with their own counter.
#define BPKI_GLOBAL __attribute__((address_space(1)))
typedef double gd2_t __attribute__((ext_vector_type(2)));
typedef float gf2_t __attribute__((ext_vector_type(2)));
__device__ __forceinline__ double2 gld(const double2 *p, long i) {
  const gd2_t v = ((const BPKI_GLOBAL gd2_t *)p)[i];
  return make_double2(v.x, v.y);
}
__device__ __forceinline__ float2 gld(const float2 *p, long i) {
  const gf2_t v = ((const BPKI_GLOBAL gf2_t *)p)[i];
  return make_float2(v.x, v.y);
}
__device__ __forceinline__ double gld(const double *p, long i) {
  return ((const BPKI_GLOBAL double *)p)[i];
}
__device__ __forceinline__ void gst(double *p, long i, double x) { ((BPKI_GLOBAL double *)p)[i] = x; }
__device__ __forceinline__ void gst(double2 *p, long i, double2 x) {
  gd2_t v;
  v.x = x.x;
  v.y = x.y;
  ((BPKI_GLOBAL gd2_t *)p)[i] = v;
}
__device__ __forceinline__ void gst(float2 *p, long i, float2 x) {
  gf2_t v;
  v.x = x.x;
  v.y = x.y;
  ((BPKI_GLOBAL gf2_t *)p)[i] = v;
}

// Complex storage of a GEMM operand: FP64 (double pairs) or FP32 (float pairs), read into and
// written from double2 registers.
template <bool F32>
struct Cx;
template <>
struct Cx<false> {
  typedef double2 t;
  static __device__ __forceinline__ double2 zero() { return make_double2(0.0, 0.0); }
  static __device__ __forceinline__ double2 get(double2 v) { return v; }
  static __device__ __forceinline__ double2 make(double re, double im) {
    return make_double2(re, im);
  }
};
template <>
struct Cx<true> {
  typedef float2 t;
  static __device__ __forceinline__ float2 zero() { return make_float2(0.0f, 0.0f); }
  static __device__ __forceinline__ double2 get(float2 v) { return make_double2(v.x, v.y); }
  static __device__ __forceinline__ float2 make(double re, double im) {
    return make_float2((float)re, (float)im);
  }
};

// Grouped complex GEMM.  grid: x = output tiles, y = batch * ksplit, z = problem.  With
// ksplit > 1 each block sums its K chunk into the partial buffer W (layout
// [prob][batch][kz][M][N]); gemm_reduce_kernel then combines the chunks in a fixed order.
// T = double: FP64 MFMA (v_mfma_f64_16x16x4f64); T = float: operands rounded to FP32 when
// staged, FP32 MFMA (v_mfma_f32_16x16x4f32) with FP32 accumulation over the block's K range.
// A32 / B32 / C32: that operand is stored as complex FP32 (FP32 mode only); the split-K chunk
// sums stay FP64.
template <typename T>
struct MfmaTraits;
template <>
struct MfmaTraits<double> {
  typedef double4_t acc_t;
  static __device__ __forceinline__ acc_t mma(double a, double b, acc_t c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  // result layout: lane l, register r -> row l/16 + 4 r, column l % 16
  static __device__ __forceinline__ int row(int lane, int r) { return (lane >> 4) + 4 * r; }
};
template <>
struct MfmaTraits<float> {
  typedef float4_t acc_t;
  static __device__ __forceinline__ acc_t mma(float a, float b, acc_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  // result layout: lane l, register r -> row 4 (l/16) + r, column l % 16
  static __device__ __forceinline__ int row(int lane, int r) { return 4 * (lane >> 4) + r; }
};

template <typename T, bool HERM, bool A32 = false, bool B32 = false, bool C32 = false>
__global__ __launch_bounds__(256, 2) void gemm_kernel(GemmDesc d, const double *const *Ap,
                                                      const double *const *Bp,
                                                      double *const *Cp, int ksplit,
                                                      int kchunk, double2 *W) {
  typedef MfmaTraits<T> MT;
  typedef typename MT::acc_t acc_t;
  typedef Cx<A32> XA;
  typedef Cx<B32> XB;
  typedef Cx<C32> XC;
  __shared__ T As[2][BK][BM + PAD];
  __shared__ T Bs[2][BK][BN + PAD];
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int tiles_m = (d.M + BM - 1) / BM;
  const int tm = blockIdx.x % tiles_m, tn = blockIdx.x / tiles_m;
  // Hermitian output: tiles above the diagonal are left to the mirror writes of their transposes;
  // a diagonal tile computes its ten 16x16 blocks on or below the diagonal, three or two per wave
  // (block b of wave w is number w + 4 b in the order (0,0) (1,0) (1,1) (2,0) (2,1) ...)
  if (HERM && tm < tn) return;
  const bool dtile = HERM && tm == tn;
  const int wv = __builtin_amdgcn_readfirstlane(wave);     // wave-uniform: scalar registers
  const int nblk = wv < 2 ? 3 : 2;
  int dbi[3], dbj[3];
#pragma unroll
  for (int b = 0; b < 3; ++b) {
    const int q = wv + 4 * b;
    const int bi = q < 1 ? 0 : q < 3 ? 1 : q < 6 ? 2 : 3;
    dbi[b] = bi;
    dbj[b] = min(q - bi * (bi + 1) / 2, bi);
  }
  const int bat = blockIdx.y / ksplit, kz = blockIdx.y % ksplit, prob = blockIdx.z;
  const typename XA::t *A = reinterpret_cast<const typename XA::t *>(Ap[prob]) + (long)bat * d.a_b;
  const typename XB::t *B = reinterpret_cast<const typename XB::t *>(Bp[prob]) + (long)bat * d.b_b;
  const int m0 = tm * BM, n0 = tn * BN;
  const int kbeg = kz * kchunk, kend = min(d.K, kbeg + kchunk);
  const int wm = (wave & 1) * 32, wn = (wave >> 1) * 32;
  const bool a_mfast = (d.a_mi == 1);
  const bool b_nfast = (d.b_ni == 1);
  const T sa = d.conjA ? T(-1) : T(1), sb = d.conjB ? T(-1) : T(1);

  // per-thread staging coordinates and the M / N parts of their offsets (fixed over K)
  int am[LOADS], ak[LOADS], bn[LOADS], bk[LOADS];
  long aoff[LOADS], boff[LOADS];
  bool aok[LOADS], bok[LOADS];
#pragma unroll
  for (int it = 0; it < LOADS; ++it) {
    int e = tid + it * 256;
    if (a_mfast) { am[it] = e % BM; ak[it] = e / BM; } else { ak[it] = e % BK; am[it] = e / BK; }
    if (b_nfast) { bn[it] = e % BN; bk[it] = e / BN; } else { bk[it] = e % BK; bn[it] = e / BK; }
    int mg = m0 + am[it], ng = n0 + bn[it];
    aok[it] = mg < d.M;
    bok[it] = ng < d.N;
    aoff[it] = aok[it] ? cidx(mg, d.Mi, d.a_mo, d.a_mi) : 0;
    boff[it] = bok[it] ? cidx(ng, d.Ni, d.b_no, d.b_ni) : 0;
  }
  // fetched values stay in their storage type until staged (no round trip through FP64)
  typename XA::t ra[LOADS];
  typename XB::t rb[LOADS];
  auto fetch = [&](int k0) {
    KOff ka = k_tile(k0, d.Ki, d.a_ko, d.a_ki), kb = k_tile(k0, d.Ki, d.b_ko, d.b_ki);
#pragma unroll
    for (int it = 0; it < LOADS; ++it) {
      int kga = k0 + ak[it], kgb = k0 + bk[it];
      typename XA::t va = XA::zero();
      typename XB::t vb = XB::zero();
      if (aok[it] && kga < kend) {
        long o = ka.uniform ? ka.base + (long)ak[it] * ka.si : cidx(kga, d.Ki, d.a_ko, d.a_ki);
        va = gld(A, aoff[it] + o);
      }
      if (bok[it] && kgb < kend) {
        long o = kb.uniform ? kb.base + (long)bk[it] * kb.si : cidx(kgb, d.Ki, d.b_ko, d.b_ki);
        vb = gld(B, boff[it] + o);
      }
      ra[it] = va;
      rb[it] = vb;
    }
  };
  auto stage = [&]() {
#pragma unroll
    for (int it = 0; it < LOADS; ++it) {
      As[0][ak[it]][am[it]] = T(ra[it].x);
      As[1][ak[it]][am[it]] = sa * T(ra[it].y);
      Bs[0][bk[it]][bn[it]] = T(rb[it].x);
      Bs[1][bk[it]][bn[it]] = sb * T(rb[it].y);
    }
  };

  acc_t acc[2][2][3];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int t = 0; t < 3; ++t) acc[i][j][t] = (acc_t){T(0), T(0), T(0), T(0)};

  if (kbeg < kend) fetch(kbeg);
  if (HERM && dtile) {
    // blocks 0, 1, 2 of the wave accumulate in acc[0][0], acc[0][1], acc[1][0]
    auto block = [&](int kr, int bi, int bj, acc_t(&a3)[3]) {
      const int ra = 16 * bi + (lane & 15), cb = 16 * bj + (lane & 15);
      const T ar = As[0][kr][ra], ai = As[1][kr][ra], br = Bs[0][kr][cb], bi_ = Bs[1][kr][cb];
      const T as = ar + ai, bs = br + bi_;
      a3[0] = MT::mma(ar, br, a3[0]);
      a3[1] = MT::mma(ai, bi_, a3[1]);
      a3[2] = MT::mma(as, bs, a3[2]);
    };
    for (int k0 = kbeg; k0 < kend; k0 += BK) {
      stage();
      __syncthreads();
      if (k0 + BK < kend) fetch(k0 + BK);
#pragma unroll
      for (int kk = 0; kk < BK / 4; ++kk) {
        const int kr = kk * 4 + (lane >> 4);
        block(kr, dbi[0], dbj[0], acc[0][0]);
        block(kr, dbi[1], dbj[1], acc[0][1]);
        if (nblk > 2) block(kr, dbi[2], dbj[2], acc[1][0]);
      }
      __syncthreads();
    }
  } else
  for (int k0 = kbeg; k0 < kend; k0 += BK) {
    stage();
    __syncthreads();
    if (k0 + BK < kend) fetch(k0 + BK);      // next tile's global loads overlap the MFMAs
#pragma unroll
    for (int kk = 0; kk < BK / 4; ++kk) {
      const int kr = kk * 4 + (lane >> 4);
      T ar[2], ai[2], br[2], bi[2];
#pragma unroll
      for (int t = 0; t < 2; ++t) {
        ar[t] = As[0][kr][wm + t * 16 + (lane & 15)];
        ai[t] = As[1][kr][wm + t * 16 + (lane & 15)];
        br[t] = Bs[0][kr][wn + t * 16 + (lane & 15)];
        bi[t] = Bs[1][kr][wn + t * 16 + (lane & 15)];
      }
      T as[2], bs[2];
#pragma unroll
      for (int t = 0; t < 2; ++t) {
        as[t] = ar[t] + ai[t];
        bs[t] = br[t] + bi[t];
      }
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) {
          acc[i][j][0] = MT::mma(ar[i], br[j], acc[i][j][0]);
          acc[i][j][1] = MT::mma(ai[i], bi[j], acc[i][j][1]);
          acc[i][j][2] = MT::mma(as[i], bs[j], acc[i][j][2]);
        }
    }
    __syncthreads();
  }
  // ---- epilogue ----
  typename XC::t *C = reinterpret_cast<typename XC::t *>(Cp[prob]) + (long)bat * d.c_b;
  double2 *Wp = W ? W + (((size_t)prob * d.batch + bat) * ksplit + kz) * (size_t)d.M * d.N
                  : nullptr;
  if constexpr (HERM) {
    // element (mg, ng) with mg >= ng, and its conjugate at (ng, mg) (single strides, real alpha,
    // no accumulation); split K: the partial sum only, mirrored by the reduction
    auto put = [&](int mg, int ng, double cr, double ci) {
      if (mg >= d.M || ng >= d.N || mg < ng) return;
      if (Wp) {
        Wp[(size_t)mg * d.N + ng] = make_double2(cr, ci);
        return;
      }
      const double vr = d.alpha_re * cr, vi = mg == ng ? 0.0 : d.alpha_re * ci;
      gst(C, (long)mg * d.c_mi + (long)ng * d.c_ni, XC::make(vr, vi));
      if (mg > ng) gst(C, (long)ng * d.c_mi + (long)mg * d.c_ni, XC::make(vr, -vi));
    };
    if (dtile) {
      auto put_block = [&](int bi, int bj, const acc_t(&a3)[3]) {
#pragma unroll
        for (int r = 0; r < 4; ++r)
          put(m0 + 16 * bi + MT::row(lane, r), n0 + 16 * bj + (lane & 15),
              (double)a3[0][r] - (double)a3[1][r],
              (double)a3[2][r] - (double)a3[0][r] - (double)a3[1][r]);
      };
      put_block(dbi[0], dbj[0], acc[0][0]);
      put_block(dbi[1], dbj[1], acc[0][1]);
      if (nblk > 2) put_block(dbi[2], dbj[2], acc[1][0]);
    } else {
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
          for (int r = 0; r < 4; ++r)
            put(m0 + wm + i * 16 + MT::row(lane, r), n0 + wn + j * 16 + (lane & 15),
                (double)acc[i][j][0][r] - (double)acc[i][j][1][r],
                (double)acc[i][j][2][r] - (double)acc[i][j][0][r] - (double)acc[i][j][1][r]);
    }
    return;
  }
  // output offsets: 8 distinct rows and 2 distinct columns per thread
  long roff[2][4], coff[2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int mg = m0 + wm + i * 16 + MT::row(lane, r);
      roff[i][r] = (!Wp && mg < d.M) ? cidx(mg, d.Mi, d.c_mo, d.c_mi) : 0;
    }
#pragma unroll
  for (int j = 0; j < 2; ++j) {
    const int ng = n0 + wn + j * 16 + (lane & 15);
    coff[j] = (!Wp && ng < d.N) ? cidx(ng, d.Ni, d.c_no, d.c_ni) : 0;
  }
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        int mg = m0 + wm + i * 16 + MT::row(lane, r);
        int ng = n0 + wn + j * 16 + (lane & 15);
        if (mg >= d.M || ng >= d.N) continue;
        double cr = (double)acc[i][j][0][r] - (double)acc[i][j][1][r];
        double ci = (double)acc[i][j][2][r] - (double)acc[i][j][0][r] - (double)acc[i][j][1][r];
        if (Wp) {
          Wp[(size_t)mg * d.N + ng] = make_double2(cr, ci);
          continue;
        }
        double vr = d.alpha_re * cr - d.alpha_im * ci;
        double vi = d.alpha_re * ci + d.alpha_im * cr;
        long off = roff[i][r] + coff[j];
        if (d.beta) {
          double2 o = XC::get(gld(C, off));
          vr += o.x;
          vi += o.y;
        }
        gst(C, off, XC::make(vr, vi));
      }
}

// Streaming complex GEMM for K <= 64 and N <= 64 (single-stride K and N): C = A B with the whole
// B (K x N) resident in LDS and the rows of A streamed through registers.  The leg contractions
// of the site tensors (K = N = chi) have this shape: M = chi^2 rows per (site, s), so the tiled
// kernel's short K loop (64 / 16 steps per tile) would leave the loads of a tile exposed.  Each
// wave owns strips of 16 rows: the A fragments of a strip (16 rows x 64 k) are loaded straight into
// the MFMA operand layout in two halves of K, the next strip's half being in flight while the other
// half is multiplied, and the 16 x 64 output strip goes from the accumulators to C.  3M complex
// products as in gemm_kernel.  TR: the MFMA computes the transposed strip (B^T A^T), so that a
// lane's outputs share one row of C and the stores run along M (used when M is C's unit-stride
// index).  grid: x = workgroups per (batch, problem), y = batch, z = problem.
constexpr int SK_MAX = 64;
template <typename T, bool TR, bool A32 = false, bool C32 = false, bool FULL = false>
__global__ __launch_bounds__(256, 2) void gemm_stream_kernel(GemmDesc d, const double *const *Ap,
                                                             const double *const *Bp,
                                                             double *const *Cp) {
  typedef MfmaTraits<T> MT;
  typedef typename MT::acc_t acc_t;
  typedef Cx<A32> XA;
  typedef Cx<C32> XC;
  __shared__ T Bs[2][SK_MAX][SK_MAX + 1];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int bat = blockIdx.y, prob = blockIdx.z;
  const typename XA::t *A = reinterpret_cast<const typename XA::t *>(Ap[prob]) + (long)bat * d.a_b;
  const double2 *B = reinterpret_cast<const double2 *>(Bp[prob]) + (long)bat * d.b_b;
  typename XC::t *C = reinterpret_cast<typename XC::t *>(Cp[prob]) + (long)bat * d.c_b;
  const T sa = d.conjA ? T(-1) : T(1), sb = d.conjB ? T(-1) : T(1);
  // B into LDS, zero outside K x N
  for (int idx = tid; idx < SK_MAX * SK_MAX; idx += 256) {
    const int k = idx / SK_MAX, n = idx % SK_MAX;
    double2 v = make_double2(0.0, 0.0);
    if (k < d.K && n < d.N) v = gld(B, (long)k * d.b_ki + (long)n * d.b_ni);
    Bs[0][k][n] = T(v.x);
    Bs[1][k][n] = sb * T(v.y);
  }
  __syncthreads();
  const int ksteps = FULL ? 16 : (d.K + 3) >> 2;      // 1 .. 16
  const int ntiles = FULL ? 4 : (d.N + 15) >> 4;      // 1 .. 4
  const int strips = (d.M + 15) >> 4;
  const int stride = gridDim.x * 4;
  const int r16 = lane & 15, kq = lane >> 4;
  // A fragment of k-step j for this lane: row (strip * 16 + r16), k = 4 j + kq.  Every load is
  // issued: a row beyond M reads row M - 1 (its products only reach output rows that are not
  // stored), a k beyond K reads k = K - 1 and is replaced by zero.
  auto row_off = [&](int s) -> long { return cidx(min(s * 16 + r16, d.M - 1), d.Mi, d.a_mo, d.a_mi); };
  typedef typename XA::t av_t;            // A values stay in their storage type
  auto load_half = [&](long ro, int h, av_t (&v)[8]) {
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const int k = 4 * (8 * h + q) + kq;
      if constexpr (FULL) {
        v[q] = gld(A, ro + (long)k * d.a_ki);
      } else {
        const av_t x = gld(A, ro + (long)min(k, d.K - 1) * d.a_ki);
        v[q] = k < d.K ? x : XA::zero();
      }
    }
  };
  acc_t acc[4][3];
  auto mma_half = [&](int h, const av_t (&v)[8]) {
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const int j = 8 * h + q;
      if (j >= ksteps) break;
      const int k = 4 * j + kq;
      const T ar = T(v[q].x), ai = sa * T(v[q].y), as = ar + ai;
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        if (t >= ntiles) break;
        const T br = Bs[0][k][16 * t + r16], bi = Bs[1][k][16 * t + r16], bs = br + bi;
        if constexpr (TR) {
          acc[t][0] = MT::mma(br, ar, acc[t][0]);
          acc[t][1] = MT::mma(bi, ai, acc[t][1]);
          acc[t][2] = MT::mma(bs, as, acc[t][2]);
        } else {
          acc[t][0] = MT::mma(ar, br, acc[t][0]);
          acc[t][1] = MT::mma(ai, bi, acc[t][1]);
          acc[t][2] = MT::mma(as, bs, acc[t][2]);
        }
      }
      // one k step at a time: the next step's LDS reads are issued behind these MFMAs, not
      // hoisted all at once (which would exceed the registers of two waves per SIMD)
      if constexpr (FULL) __builtin_amdgcn_sched_barrier(0);
    }
  };
  int s = blockIdx.x * 4 + wave;
  av_t lo[8], hi[8];
  long ro = row_off(s);
  if (s < strips) {
    load_half(ro, 0, lo);
    load_half(ro, 1, hi);
  }
  for (; s < strips; s += stride) {
#pragma unroll
    for (int t = 0; t < 4; ++t)
#pragma unroll
      for (int c = 0; c < 3; ++c) acc[t][c] = (acc_t){T(0), T(0), T(0), T(0)};
    const int sn = s + stride;
    const long ron = row_off(sn);
    mma_half(0, lo);
    if (sn < strips) load_half(ron, 0, lo);     // the next strip's first half is in flight ...
    mma_half(1, hi);                              // ... while this strip's second half is used
    if (sn < strips) load_half(ron, 1, hi);
    // output strip: lane holds rows MT::row(lane, r) and column 16 t + r16 of each n-tile
    // (TR: row s * 16 + r16 and columns 16 t + MT::row(lane, r))
    const int mt = s * 16 + r16;
    const long cot = (TR && mt < d.M) ? cidx(mt, d.Mi, d.c_mo, d.c_mi) : 0;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int m = TR ? mt : s * 16 + MT::row(lane, r);
      if (m >= d.M) continue;
      const long co = TR ? cot : cidx(m, d.Mi, d.c_mo, d.c_mi);
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const int n = 16 * t + (TR ? MT::row(lane, r) : r16);
        if (t >= ntiles || n >= d.N) continue;
        const double cr = (double)acc[t][0][r] - (double)acc[t][1][r];
        const double ci = (double)acc[t][2][r] - (double)acc[t][0][r] - (double)acc[t][1][r];
        double vr = d.alpha_re * cr - d.alpha_im * ci;
        double vi = d.alpha_re * ci + d.alpha_im * cr;
        const long off = co + (long)n * d.c_ni;
        if (d.beta) {
          const double2 o = XC::get(gld(C, off));
          vr += o.x;
          vi += o.y;
        }
        gst(C, off, XC::make(vr, vi));
      }
    }
    ro = ron;
  }
}

// Twelve independent MFMA accumulation chains per wave, no memory traffic: the achievable MFMA
// rate that bounds gemm_kernel.  The final comparison keeps the chains live.
template <typename T>
__global__ __launch_bounds__(256) void mfma_rate_kernel(int iters, double *out) {
  typedef MfmaTraits<T> MT;
  typedef typename MT::acc_t acc_t;
  acc_t acc[12];
#pragma unroll
  for (int i = 0; i < 12; ++i) acc[i] = (acc_t){T(0), T(0), T(0), T(0)};
  const T a = T(threadIdx.x) * T(1e-3), b = T(blockIdx.x) * T(1e-3);
  for (int it = 0; it < iters; ++it)
#pragma unroll
    for (int i = 0; i < 12; ++i) acc[i] = MT::mma(a, b, acc[i]);
  double sum = 0.0;
#pragma unroll
  for (int i = 0; i < 12; ++i) sum += (double)acc[i][0] + (double)acc[i][1] + (double)acc[i][2] + (double)acc[i][3];
  if (sum == -1.0) out[0] = sum;
}

// Sums the K chunks of a split-K GEMM in chunk order and applies alpha / beta.
template <bool C32>
__global__ __launch_bounds__(256) void gemm_reduce_kernel(GemmDesc d, double *const *Cp,
                                                          int ksplit, const double2 *W) {
  typedef Cx<C32> XC;
  const int bat = blockIdx.y, prob = blockIdx.z;
  const size_t mn = (size_t)d.M * d.N;
  const double2 *wp = W + ((size_t)prob * d.batch + bat) * ksplit * mn;
  typename XC::t *C = reinterpret_cast<typename XC::t *>(Cp[prob]) + (long)bat * d.c_b;
  for (size_t idx = blockIdx.x * (size_t)blockDim.x + threadIdx.x; idx < mn;
       idx += (size_t)gridDim.x * blockDim.x) {
    int mg = (int)(idx / d.N), ng = (int)(idx % d.N);
    if (d.herm && mg < ng) continue;              // written as the mirror of (ng, mg)
    double cr = 0, ci = 0;
    for (int kz = 0; kz < ksplit; ++kz) {
      double2 v = wp[kz * mn + idx];
      cr += v.x;
      ci += v.y;
    }
    if (d.herm) {
      const double vr = d.alpha_re * cr, vi = mg == ng ? 0.0 : d.alpha_re * ci;
      gst(C, (long)mg * d.c_mi + (long)ng * d.c_ni, XC::make(vr, vi));
      if (mg > ng) gst(C, (long)ng * d.c_mi + (long)mg * d.c_ni, XC::make(vr, -vi));
      continue;
    }
    double vr = d.alpha_re * cr - d.alpha_im * ci;
    double vi = d.alpha_re * ci + d.alpha_im * cr;
    long off = cidx(mg, d.Mi, d.c_mo, d.c_mi) + cidx(ng, d.Ni, d.c_no, d.c_ni);
    if (d.beta) {
      double2 o = XC::get(gld(C, off));
      vr += o.x;
      vi += o.y;
    }
    gst(C, off, XC::make(vr, vi));
  }
}

// ------------------------------------------------------------------------------------------
// Fused BP closing at chi = CH = 64 or 32 (BpCloseDesc).  The message towards the outgoing leg b
// sums, over chunks (s, x) of the chunk leg (s alone for a degree-2 site),
//   W[b][a] = sum_{a0} Y[b][a0] M[a0][a]          (Y, T: the chunk's CH x CH slices)
//   out[b][b'] += sum_a W[b][a] conj(T[b'][a]).
// A workgroup owns a contiguous range of the chunks of all problems (a problem's 2 xdim chunks may
// be split between two workgroups) and works on G = 64 / CH chunks at a time, NT = CH / 16 waves
// each.  Per chunk, wave wl of its group forms the CH x 16 strip W^T[.][b-block wl] on MFMA:
// A = M^T from LDS, B = Y from registers.  The MFMA accumulator of that strip holds, in lane l and
// register r of tile i, W[16 wl + l % 16][16 i + row(l, r)]: exactly the A operand of the second
// product for k step (i, r) when the k index of that step is taken as 16 i + row(l, r) (the B
// operand, conj(T), uses the same k map).  So W never leaves the registers and the intermediates of
// the chain never reach memory.  The second product covers the 16 x 16 blocks of the Hermitian
// output on or below the diagonal once each: wave wl computes blocks (wl, wl + d mod NT) for
// d = 0 .. NT / 2, the last one only for wl < NT / 2; blocks above the diagonal are stored as their
// mirrors.  The chunks' T slices sit in LDS (transposed, [a][b']), and the next chunks' Y values and
// T slices are loaded into registers while these chunks are multiplied.  Complex products by the
// 3M method as in gemm_kernel.  Each wave group's partial sums (lower triangle) go to
// part[wg][slot][group] (slot 0: the workgroup's first problem, 1: the next);
// bp_close_reduce_kernel adds them in workgroup order.  FP64 at CH = 64: one workgroup per CU (LDS
// and registers); otherwise two.  grid: workgroups, each `per` chunks (a multiple of G).
//
// PAIR: the message from two absorbed copies of the site tensor, Y (Yp) and Y' (Tp), with the
// messages of the two summed legs absorbed one in each: for a Hermitian M',
// sum_{a'} M'[x][a'] conj(T[.., a', ..]) = conj(Y'[.., x, ..]) with Y' = T x M', so
//   out[b][b'] = sum over chunks of sum_a Y[b][a] conj(Y'[b'][a])
// is the same closing without the leg absorption of the chunk: W is Y's slice itself, loaded
// straight into the A-operand layout of the product, and only the Hermitian product runs (Mp is
// not read); the next chunks' W values and T slices are loaded after the product.
template <typename T, int CH, bool PR = false>
struct BpCloseCfg {
  static constexpr bool F64 = std::is_same<T, double>::value;
  static constexpr int PAD = F64 ? 8 : 4;                 // LDS row padding
  // workgroups per CU: one for the FP64 chain at chi = 64 (LDS and registers), else two (the
  // FP64 pair at chi = 64 is HBM-bound: two workgroups keep more loads in flight than the
  // register prefetch of one)
  static constexpr int WGS = (F64 && CH == 64 && !PR) ? 1 : 2;
  static constexpr int NT = CH / 16;                      // 16-row tiles per side
  static constexpr int KS = CH / 4;                       // k steps of the first product
  static constexpr int G = 64 / CH;                       // chunks in flight, NT waves each
  static constexpr int NB = NT / 2 + 1;                   // most output blocks of one wave
};
template <typename T, bool S32, int CH, bool PAIR>
__global__ __launch_bounds__(256, (BpCloseCfg<T, CH, PAIR>::WGS)) void bp_close_kernel(
    BpCloseDesc d, const double *const *Yp, const double *const *Tp, const double *const *Mp,
    int total, int per, double2 *part) {
  typedef MfmaTraits<T> MT;
  typedef typename MT::acc_t acc_t;
  typedef Cx<S32> X;
  typedef typename X::t st_t;
  typedef BpCloseCfg<T, CH> Cfg;
  constexpr int CC = CH * CH, NT = Cfg::NT, KS = Cfg::KS, G = Cfg::G, NB = Cfg::NB;
  constexpr int P = Cfg::PAD;
  const int J = 2 * d.xdim;              // chunks per problem: (s, x)
  __shared__ T Ms[PAIR ? 1 : 2][PAIR ? 1 : CH][PAIR ? 1 : CH + P];   // M[a0][a]
  __shared__ T Ts[G][2][CH][CH + P];     // per chunk in flight: T[b'][a], stored as [a][b']
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int c = lane & 15, g = lane >> 4;
  const int wv = __builtin_amdgcn_readfirstlane(w);
  const int q = G == 1 ? 0 : wv / NT;    // this wave's chunk in flight
  const int wl = G == 1 ? wv : wv % NT;  // and its 16 rows b
  const int nb = NT / 2 + (wl < NT / 2 ? 1 : 0);
  int bj[NB];
#pragma unroll
  for (int jj = 0; jj < NB; ++jj) bj[jj] = (wl + jj) % NT;
  // strides of the current problem (workgroup-uniform), set when a problem starts
  long rs = 0, qs = 0, cs = 0, yrow = 0, toff0 = 0, tstep = 0;
  bool a_fast = true;
  // this thread's TU elements u of a chunk's T slice: tid % CH along whichever of b', a is
  // unit-stride, tid / CH + HS u along the other
  constexpr int TU = CC / 256, HS = 256 / CH;
  const int tlo = tid % CH, thi = tid / CH;
  auto set_strides = [&](int p) {
    const int k = min(p / d.group, d.nsets - 1);
    rs = d.rs[k];
    qs = d.qs[k];
    cs = d.cs[k];
    yrow = (long)(16 * wl + c) * rs;
    a_fast = qs == 1;
    toff0 = a_fast ? (long)thi * rs + tlo : (long)tlo * rs + (long)thi * qs;
    tstep = HS * (a_fast ? rs : qs);
  };
  acc_t acc2[NB][3];
  auto clear2 = [&]() {
#pragma unroll
    for (int jj = 0; jj < NB; ++jj)
#pragma unroll
      for (int t = 0; t < 3; ++t) acc2[jj][t] = (acc_t){T(0), T(0), T(0), T(0)};
  };
  // the lower-triangle partial sum of one problem over this wave group's chunks
  auto flush = [&](int slot) {
    double2 *Pp = part + (((size_t)blockIdx.x * 2 + slot) * G + q) * CC;
#pragma unroll
    for (int jj = 0; jj < NB; ++jj) {
      if (jj >= nb) break;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int b = 16 * wl + MT::row(lane, r), bp = 16 * bj[jj] + c;
        const double re = (double)acc2[jj][0][r] - (double)acc2[jj][1][r];
        const double im = (double)acc2[jj][2][r] - (double)acc2[jj][0][r] - (double)acc2[jj][1][r];
        if (b >= bp) Pp[b * CH + bp] = make_double2(re, im);
        else if (bj[jj] != wl) Pp[bp * CH + b] = make_double2(re, -im);
      }
    }
  };
  auto chunk_base = [&](int k) {
    const int j = k % J;
    return (long)(j / d.xdim) * d.ss + (long)(j % d.xdim) * cs;
  };
  st_t yv[KS], tn[G][TU];
  // this wave's Y values of chunk k + q: the B operand of the first product (Y[b][a0],
  // a0 = 4 t + g), or (PAIR) W itself in the A-operand layout of the product (Y[b][a],
  // a = 16 i + row(lane, r) at t = 4 i + r)
  auto load_y = [&](st_t (&dst)[KS], const st_t *Y, int k) {
    const long base = chunk_base(k + q);
#pragma unroll
    for (int t = 0; t < KS; ++t) {
      const int a = PAIR ? 16 * (t >> 2) + MT::row(lane, t & 3) : 4 * t + g;
      dst[t] = gld(Y, base + yrow + (long)a * qs);
    }
  };
  auto load_t = [&](const st_t *Tt, int k) {     // the T slices of chunks k .. k + G - 1
#pragma unroll
    for (int qq = 0; qq < G; ++qq) {
      const st_t *src = Tt + chunk_base(k + qq) + toff0;
#pragma unroll
      for (int u = 0; u < TU; ++u) tn[qq][u] = gld(src, (long)u * tstep);
    }
  };
  auto store_t = [&]() {
#pragma unroll
    for (int qq = 0; qq < G; ++qq)
#pragma unroll
      for (int u = 0; u < TU; ++u) {
        const int a = a_fast ? tlo : thi + HS * u, b = a_fast ? thi + HS * u : tlo;
        Ts[qq][0][a][b] = T(tn[qq][u].x);
        Ts[qq][1][a][b] = -T(tn[qq][u].y);    // conj(T)
      }
  };
  clear2();
  // a workgroup's run of chunks is a multiple of G long and starts at a multiple of G, and so does
  // every problem (J is even), so the G chunks in flight always belong to one problem
  const int k0 = blockIdx.x * per, k1 = min(k0 + per, total);
  int cur = -1, slot = 0;
  const st_t *Y = nullptr, *Tt = nullptr;
  bool ready = false;                    // this iteration's Y values and T slices are in place
  for (int k = k0; k < k1; k += G) {
    const int p = k / J;
    if (!ready) {                        // first chunks, or a new problem (workgroup-uniform)
      if (cur >= 0) {
        flush(slot++);
        clear2();
      }
      cur = p;
      set_strides(p);
      Y = reinterpret_cast<const st_t *>(Yp[p]);
      Tt = reinterpret_cast<const st_t *>(Tp[p]);
      load_y(yv, Y, k);
      load_t(Tt, k);
      __syncthreads();
      if constexpr (!PAIR) {
        const double2 *M = reinterpret_cast<const double2 *>(Mp[p]);
        for (int idx = tid; idx < CC; idx += 256) {
          const double2 v = gld(M, idx);
          Ms[0][idx / CH][idx % CH] = T(v.x);
          Ms[1][idx / CH][idx % CH] = T(v.y);
        }
      }
      store_t();
      __syncthreads();
    }
    // the next chunks of the same problem: their T slices are loaded while these chunks are
    // multiplied, their Y values once this iteration's first product has used the current ones
    ready = k + G < k1 && (k + G) / J == p;
    if (!PAIR && ready) load_t(Tt, k + G);
    // W^T[a][b] = sum_a0 M[a0][a] Y[b][a0], NT a tiles by this wave's 16 columns b (PAIR: the
    // next chunks' W values are loaded instead)
    acc_t acc1[PAIR ? 1 : NT][3];
    if constexpr (!PAIR) {
#pragma unroll
      for (int i = 0; i < NT; ++i)
#pragma unroll
        for (int t = 0; t < 3; ++t) acc1[i][t] = (acc_t){T(0), T(0), T(0), T(0)};
#pragma unroll
      for (int t = 0; t < KS; ++t) {
        const int a0 = 4 * t + g;
        const T br = T(yv[t].x), bi = T(yv[t].y), bs = br + bi;
#pragma unroll
        for (int i = 0; i < NT; ++i) {
          const T ar = Ms[0][a0][16 * i + c], ai = Ms[1][a0][16 * i + c], as = ar + ai;
          acc1[i][0] = MT::mma(ar, br, acc1[i][0]);
          acc1[i][1] = MT::mma(ai, bi, acc1[i][1]);
          acc1[i][2] = MT::mma(as, bs, acc1[i][2]);
        }
      }
      if (ready) load_y(yv, Y, k + G);
    }
    // out[b][b'] += sum_a W[b][a] conj(T[b'][a]), k step (i, r) <-> a = 16 i + row(lane, r)
#pragma unroll
    for (int i = 0; i < NT; ++i) {
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        T wr, wi;
        if constexpr (PAIR) {
          wr = T(yv[4 * i + r].x);
          wi = T(yv[4 * i + r].y);
        } else {
          wr = acc1[i][0][r] - acc1[i][1][r];
          wi = acc1[i][2][r] - acc1[i][0][r] - acc1[i][1][r];
        }
        const T ws = wr + wi;
        const int a = 16 * i + MT::row(lane, r);
#pragma unroll
        for (int jj = 0; jj < NB; ++jj) {
          if (jj >= nb) break;
          const T br = Ts[q][0][a][16 * bj[jj] + c], bi = Ts[q][1][a][16 * bj[jj] + c];
          const T bs = br + bi;
          acc2[jj][0] = MT::mma(wr, br, acc2[jj][0]);
          acc2[jj][1] = MT::mma(wi, bi, acc2[jj][1]);
          acc2[jj][2] = MT::mma(ws, bs, acc2[jj][2]);
        }
      }
    }
    if constexpr (PAIR) {           // the next chunks' W values and T slices, after this product
      if (ready) {
        load_y(yv, Y, k + G);
        load_t(Tt, k + G);
      }
    }
    if (ready) {
      __syncthreads();                   // every wave is done with these chunks' T slices
      store_t();
      __syncthreads();
    }
  }
  if (cur >= 0) flush(slot);
}

// Message p of a fused BP closing: the partial sums of the workgroups (and their G chunk groups)
// that covered its chunks (J per problem), in workgroup order; lower triangle, its mirror above,
// real diagonal.  grid (ceil(chi^2 / 256), nprob).
__global__ __launch_bounds__(256) void bp_close_reduce_kernel(int ch, int G, int per, int J,
                                                              const double2 *part,
                                                              double *const *Op) {
  const int CC = ch * ch;
  const int p = blockIdx.y;
  const int idx = blockIdx.x * 256 + threadIdx.x;
  if (idx >= CC) return;
  const int b = idx / ch, bp = idx % ch;
  if (b < bp) return;
  const long first = (long)p * J, last = first + J - 1;
  double re = 0.0, im = 0.0;
  for (long wg = first / per; wg <= last / per; ++wg) {
    const int slot = (wg * per) / J == p ? 0 : 1;
    for (int qq = 0; qq < G; ++qq) {
      const double2 v = part[(((size_t)wg * 2 + slot) * G + qq) * CC + idx];
      re += v.x;
      im += v.y;
    }
  }
  double2 *O = reinterpret_cast<double2 *>(Op[p]);
  gst(O, (long)b * ch + bp, make_double2(re, b == bp ? 0.0 : im));
  if (b > bp) gst(O, (long)bp * ch + b, make_double2(re, -im));
}

// ------------------------------------------------------------------------------------------
// Hermitian Jacobi eigensolver
struct Rot {
  double c, s;
  double wr, wi;   // omega = e^{-i phi}
  int p, q;
};

__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ double2 cconj(double2 a) { return make_double2(a.x, -a.y); }
__device__ __forceinline__ double2 cadd(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ double2 cscale(double s, double2 a) { return make_double2(s * a.x, s * a.y); }

// Sum of one value per thread over the whole block; every thread gets the result.
__device__ double block_allsum(double v, double *sh /* >= 16 */) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  const int w = threadIdx.x >> 6, nw = (blockDim.x + 63) >> 6;
  __syncthreads();
  if ((threadIdx.x & 63) == 0) sh[w] = v;
  __syncthreads();
  double r = 0;
  for (int i = 0; i < nw; ++i) r += sh[i];
  __syncthreads();
  return r;
}

// Round-robin pairing (circle method) for np even, m = np-1 odd.
__device__ __forceinline__ void pair_of(int r, int i, int np, int &p, int &q) {
  int m = np - 1;
  if (i == 0) { p = r % m; q = m; }
  else { p = (r + i) % m; q = (r - i + m) % m; }
}

__global__ __launch_bounds__(1024) void eigh_jacobi_kernel(int n, int lda,
                                                           const double *const *in,
                                                           double *const *evals,
                                                           double *const *vecs, int max_sweeps) {
  extern __shared__ double2 smem[];
  __shared__ Rot rot[128];
  __shared__ int any_rot;
  __shared__ double diag_s[256];
  __shared__ double red_s[16];
  const int prob = blockIdx.x;
  const int tid = threadIdx.x, nt = blockDim.x;
  const int np = n + (n & 1);
  const int h = np / 2;
  double2 *A = smem, *V = smem + (size_t)np * np;
  const double2 *src = reinterpret_cast<const double2 *>(in[prob]);
  double fro2 = 0.0;
  for (int idx = tid; idx < np * np; idx += nt) {
    int i = idx / np, j = idx % np;
    double2 v = make_double2(0.0, 0.0);
    if (i < n && j < n) {
      double2 a = src[(size_t)i * lda + j], b = src[(size_t)j * lda + i];
      v = make_double2(0.5 * (a.x + b.x), 0.5 * (a.y - b.y));   // Hermitian part
    }
    A[idx] = v;
    V[idx] = make_double2(i == j ? 1.0 : 0.0, 0.0);
    fro2 += v.x * v.x + v.y * v.y;
  }
  __syncthreads();
  const double eps = 2.220446049250313e-16;
  // couplings below 0.1 eps ||A||_F are at the rounding level of A and are not rotated
  const double thr_abs = 0.1 * eps * sqrt(block_allsum(fro2, red_s));
  for (int sweep = 0; sweep < max_sweeps; ++sweep) {
    if (tid == 0) any_rot = 0;
    __syncthreads();
    for (int r = 0; r < np - 1; ++r) {
      if (tid < h) {
        int p, q;
        pair_of(r, tid, np, p, q);
        double a = A[(size_t)p * np + p].x, dd = A[(size_t)q * np + q].x;
        double2 b = A[(size_t)p * np + q];
        double beta = sqrt(b.x * b.x + b.y * b.y);
        Rot R;
        R.p = p; R.q = q;
        if (beta > 1e-300 && beta > thr_abs && beta > eps * sqrt(fabs(a) * fabs(dd))) {
          double tau = (dd - a) / (2.0 * beta);
          double t = (tau >= 0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
          double c = 1.0 / sqrt(1.0 + t * t);
          R.c = c; R.s = t * c;
          R.wr = b.x / beta; R.wi = -b.y / beta;
          any_rot = 1;
        } else {
          R.c = 1.0; R.s = 0.0; R.wr = 1.0; R.wi = 0.0;
        }
        rot[tid] = R;
      }
      __syncthreads();
      for (int blk = tid; blk < h * h; blk += nt) {
        int I = blk / h, J = blk % h;
        Rot ri = rot[I], rj = rot[J];
        double2 w_j = make_double2(rj.wr, rj.wi), w_i_c = make_double2(ri.wr, -ri.wi);
        size_t o00 = (size_t)ri.p * np + rj.p, o01 = (size_t)ri.p * np + rj.q;
        size_t o10 = (size_t)ri.q * np + rj.p, o11 = (size_t)ri.q * np + rj.q;
        double2 b00 = A[o00], b01 = A[o01], b10 = A[o10], b11 = A[o11];
        // T = B J_J
        double2 sw = cscale(rj.s, w_j), cw = cscale(rj.c, w_j);
        double2 t00 = cadd(cscale(rj.c, b00), cscale(-1.0, cmul(sw, b01)));
        double2 t10 = cadd(cscale(rj.c, b10), cscale(-1.0, cmul(sw, b11)));
        double2 t01 = cadd(cscale(rj.s, b00), cmul(cw, b01));
        double2 t11 = cadd(cscale(rj.s, b10), cmul(cw, b11));
        // B' = J_I^H T
        double2 swc = cscale(ri.s, w_i_c), cwc = cscale(ri.c, w_i_c);
        double2 n00 = cadd(cscale(ri.c, t00), cscale(-1.0, cmul(swc, t10)));
        double2 n01 = cadd(cscale(ri.c, t01), cscale(-1.0, cmul(swc, t11)));
        double2 n10 = cadd(cscale(ri.s, t00), cmul(cwc, t10));
        double2 n11 = cadd(cscale(ri.s, t01), cmul(cwc, t11));
        if (I == J) {
          n00.y = 0.0; n11.y = 0.0;
          if (ri.s != 0.0) { n01 = make_double2(0.0, 0.0); n10 = n01; }
        }
        A[o00] = n00; A[o01] = n01; A[o10] = n10; A[o11] = n11;
      }
      for (int it = tid; it < np * h; it += nt) {
        int row = it / h, J = it % h;
        Rot rj = rot[J];
        if (rj.s == 0.0) continue;
        double2 w_j = make_double2(rj.wr, rj.wi);
        size_t op = (size_t)row * np + rj.p, oq = (size_t)row * np + rj.q;
        double2 vp = V[op], vq = V[oq];
        double2 sw = cscale(rj.s, w_j), cw = cscale(rj.c, w_j);
        V[op] = cadd(cscale(rj.c, vp), cscale(-1.0, cmul(sw, vq)));
        V[oq] = cadd(cscale(rj.s, vp), cmul(cw, vq));
      }
      __syncthreads();
    }
    __syncthreads();
    int stop = (any_rot == 0);
    __syncthreads();
    if (stop) break;
  }
  // sort descending (rank sort over the n real indices) and write out
  for (int i = tid; i < n; i += nt) diag_s[i] = A[(size_t)i * np + i].x;
  __syncthreads();
  double *ev = evals[prob];
  double2 *vo = reinterpret_cast<double2 *>(vecs[prob]);
  for (int i = tid; i < n; i += nt) {
    double li = diag_s[i];
    int rank = 0;
    for (int j = 0; j < n; ++j) {
      double lj = diag_s[j];
      rank += (lj > li) || (lj == li && j < i);
    }
    ev[rank] = li;
    for (int row = 0; row < n; ++row) vo[(size_t)row * n + rank] = V[(size_t)row * np + i];
  }
}

// Packed lower-triangle index (i >= j).
__device__ __forceinline__ size_t pk_idx(int i, int j) {
  return (size_t)i * (i + 1) / 2 + j;
}

// ------------------------------------------------------------------------------------------
// Hermitian eigensolver for 32 <= n <= 256 in three kernels, one workgroup per matrix each.
//
//  1. eigh_tridiag_kernel (1024 threads): Householder reduction to real symmetric
//     tridiagonal form, A = Q T Q^H with
//     Q = H_0 H_1 ... H_{n-2}, H_k = I - tau_k v_k v_k^H (v_k(k+1) = 1, zero above).  Each
//     reflector maps column k below the diagonal onto beta e_1 with beta real, so T is real.
//     The trailing block is updated as A <- A - v w^H - w v^H with x = tau A v and
//     w = x - (1/2) Re(conj(tau) v^H x) v.  Only the lower triangle is kept (packed in LDS for
//     n <= 128, row-major in the workspace above); reflectors go to the workspace.
//     The diagonal d and off-diagonal e go to the workspace (eigenvalue and staging areas).
//  2. eigh_dc_kernel (512 threads): divide and conquer on T (Cuppen's rank-one tearing;
//     eigenvectors by the Gu-Eisenstat construction).  The index range is cut into the binary
//     tree of ranges [floor(q n / 2^D), floor((q+1) n / 2^D)) down to single entries (depth
//     ceil(log2 n)); every coupling beta is torn off at the level whose merge joins its two
//     sides (T = diag(T_1 .. T_L) + sum |beta| u u^T with u = e_{k-1} + sign(beta) e_k and the
//     two diagonal entries lowered by |beta|), and the levels are merged back bottom-up by the
//     whole workgroup, all merges of a level at once.  A merge of two solved halves with
//     eigenvectors Q = diag(Q1, Q2) solves D + rho z z^T (z = Q^T u / sqrt 2, rho = 2|beta|):
//       - deflation: components with rho |z_i| <= tol keep (d_i, q_i); pairs of eigenvalues
//         closer than tol are rotated so that one z component vanishes
//         (tol = 8 eps max(|d|_max, rho));
//       - each remaining root of f = 1 + rho sum z_i^2 / (d_i - lambda) is bracketed between
//         consecutive poles and computed in the variable tau = lambda - d_o from the nearer
//         pole d_o (so that every difference d_i - lambda is formed accurately) by a
//         safeguarded rational iteration: the pole sums on either side of the root are
//         replaced by one-pole models matched in value and slope (as in Bunch, Nielsen and
//         Sorensen, 1978), with bisection whenever the model's root leaves the bracket;
//       - z is recomputed from the roots (Loewner's formula) so that the eigenvectors
//         v_j = (zhat_i / (d_i - lambda_j))_i are numerically orthogonal; the new eigenvector
//         matrix is Q_K V.
//  3. eigh_backtransform_kernel (grid: 16-column blocks x matrices): V = Q Z by applying
//     H_{n-2}, ..., H_0 to each column block in LDS, the columns taken in descending
//     eigenvalue order and only as many as the caller needs.
//
// Workspace per matrix (doubles): reflectors n*n complex (column k = v_k), tau n complex,
// Z n*n real (column-major), eigenvalues n, an n*n staging area for the merges, and for
// n > 128 an n*n complex area that holds the matrix during the reduction (its lower triangle,
// row-major) and the merge coefficient vectors V afterwards, then for n > 256 the blocked
// reduction's panel vectors [V | W] (n x 2 TRD_NB complex, row-major).  For n <= 128 the matrix and Z live in LDS
// and Z's global area holds V during the merges.
constexpr int TRD_NB = 32;
__host__ __device__ __forceinline__ size_t tql_ws_doubles(int n) {
  return (size_t)(n > 128 ? 6 : 4) * n * n + (size_t)3 * n +
         (n > 256 ? (size_t)4 * n * TRD_NB : 0);
}
__host__ __device__ __forceinline__ size_t trd_panel_offset(int n) {   // doubles, for n > 256
  return (size_t)6 * n * n + (size_t)3 * n;
}

// Cross-lane reductions on the DPP network (no LDS round trips).  dpp_d<CTRL> moves a double
// from the lane that the DPP control CTRL names: 0xB1 lane ^ 1, 0x4E lane ^ 2 (quad permutes),
// 0x141 the mirror within 8 lanes, 0x140 the mirror within 16 lanes.  Every lane of the groups
// involved must be active.
template <int CTRL>
__device__ __forceinline__ double dpp_d(double v) {
  const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, 0xF, 0xF, false);
  return __hiloint2double(hi, lo);
}
template <int CTRL>
__device__ __forceinline__ int dpp_i(int v) {
  return __builtin_amdgcn_update_dpp(0, v, CTRL, 0xF, 0xF, false);
}
__device__ __forceinline__ double readlane_d(double v, int l) {
  return __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(v), l),
                          __builtin_amdgcn_readlane(__double2loint(v), l));
}
// sum over the 4 lanes of a quad, the same value in each of them
__device__ __forceinline__ double quad_sum(double v) {
  v += dpp_d<0xB1>(v);
  return v + dpp_d<0x4E>(v);
}
__device__ __forceinline__ double quad_prod(double v) {
  v *= dpp_d<0xB1>(v);
  return v * dpp_d<0x4E>(v);
}
// sum over the 8 lanes of an aligned group of 8
__device__ __forceinline__ double oct_sum(double v) {
  v = quad_sum(v);
  return v + dpp_d<0x141>(v);
}
// sum / max over the wave (all 64 lanes active), the same value in every lane
__device__ __forceinline__ double wave_sum(double v) {
  v = oct_sum(v);
  v += dpp_d<0x140>(v);
  return (readlane_d(v, 0) + readlane_d(v, 16)) + (readlane_d(v, 32) + readlane_d(v, 48));
}
// the largest value over the wave and its index (the smallest index among equal values), in
// every lane
__device__ __forceinline__ void wave_argmax(double &best, int &bj) {
  auto take = [&](double ob, int oj) {
    if (ob > best || (ob == best && oj < bj)) { best = ob; bj = oj; }
  };
  take(dpp_d<0xB1>(best), dpp_i<0xB1>(bj));
  take(dpp_d<0x4E>(best), dpp_i<0x4E>(bj));
  take(dpp_d<0x141>(best), dpp_i<0x141>(bj));
  take(dpp_d<0x140>(best), dpp_i<0x140>(bj));
  const double r0 = readlane_d(best, 0), r1 = readlane_d(best, 16), r2 = readlane_d(best, 32),
               r3 = readlane_d(best, 48);
  const int j0 = __builtin_amdgcn_readlane(bj, 0), j1 = __builtin_amdgcn_readlane(bj, 16),
            j2 = __builtin_amdgcn_readlane(bj, 32), j3 = __builtin_amdgcn_readlane(bj, 48);
  best = r0;
  bj = j0;
  take(r1, j1);
  take(r2, j2);
  take(r3, j3);
}
__device__ __forceinline__ double wave_max(double v) {
  v = fmax(v, dpp_d<0xB1>(v));
  v = fmax(v, dpp_d<0x4E>(v));
  v = fmax(v, dpp_d<0x141>(v));
  v = fmax(v, dpp_d<0x140>(v));
  return fmax(fmax(readlane_d(v, 0), readlane_d(v, 16)), fmax(readlane_d(v, 32), readlane_d(v, 48)));
}

__device__ __forceinline__ int dc_bound(int q, int n, int depth) {
  return (int)(((long)q * n) >> depth);
}

// Scratch of the merges of one level (LDS): per-position arrays indexed by the position i in
// [0, n) (each merge uses the positions of its own range), per-merge values by the merge q.
struct DcScratch {
  double *z, *dd, *zK, *dK, *tau, *dorg, *zh, *lam, *rc, *rs, *tol;
  int *perm, *K, *defl, *ra, *rb, *cnk, *cnr;
};

// Merges, for every q < 2^D at once, the solved ranges [lo, k) and [k, hi) coupled by
// beta = e[k - 1], where lo = floor(q n / 2^D), k = floor((2q + 1) n / 2^(D+1)),
// hi = floor((q + 1) n / 2^D); ranges with lo = k or k = hi are not split at this level.
// All 512 threads; every loop runs over the positions (or position pairs) of all merges of the
// level, so a level costs about what its largest merge costs.  d: eigenvalues (LDS), Z:
// eigenvectors (column-major, leading dimension n; LDS or global); Vg, Wg: n x n global staging
// areas of this matrix.
__device__ void dc_level(int n, int D, const double *e, double *d, double *Z, const DcScratch &S,
                         double *Vg, double *Wg) {
  const double eps = 2.220446049250313e-16;
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  constexpr int NT = 512, NW = 8;
  const int nq = 1 << D;
  const int smax = (n + nq - 1) / nq + 1;        // a bound on the size of a range
  // the merge holding position i: the largest q with floor(q n / 2^D) <= i
  auto merge_of = [&](int i) { return (((i + 1) << D) + n - 1) / n - 1; };
  struct Rg { int lo, k, hi; bool on; };
  auto range = [&](int q) {
    Rg r;
    r.lo = dc_bound(q, n, D);
    r.hi = dc_bound(q + 1, n, D);
    r.k = dc_bound(2 * q + 1, n, D + 1);
    r.on = r.lo < r.k && r.k < r.hi;
    return r;
  };
  // z = (last row of Q1, sign(beta) first row of Q2) / sqrt 2
  for (int i = tid; i < n; i += NT) {
    const Rg g = range(merge_of(i));
    if (!g.on) continue;
    const double sg = e[g.k - 1] >= 0.0 ? 1.0 : -1.0;
    S.z[i] = (i < g.k ? Z[(size_t)i * n + g.k - 1] : sg * Z[(size_t)i * n + g.k]) *
             0.70710678118654752440;
    S.dd[i] = d[i];
  }
  // deflation tolerance of each merge: 8 eps max(|d|_max, rho), one wave per merge
  for (int q = wave; q < nq; q += NW) {
    const Rg g = range(q);
    if (!g.on) continue;
    double m = 0.0;
    for (int i = g.lo + lane; i < g.hi; i += 64) m = fmax(m, fabs(d[i]));
    m = wave_max(m);
    if (lane == 0) S.tol[q] = 8.0 * eps * fmax(m, 2.0 * fabs(e[g.k - 1]));
  }
  __syncthreads();
  // ascending order of dd within each merge (ties by position)
  for (int i = tid; i < n; i += NT) {
    const Rg g = range(merge_of(i));
    if (!g.on) continue;
    const double v = S.dd[i];
    int r = 0;
    for (int u = g.lo; u < g.hi; ++u) {
      const double w = S.dd[u];
      r += (w < v) || (w == v && u < i);
    }
    S.perm[g.lo + r] = i;
    S.zK[g.lo + r] = S.z[i];    // sorted copies for the scan (dK is free until the gather below)
    S.dK[g.lo + r] = v;
  }
  __syncthreads();
  // deflation scan of each merge in ascending order (one thread per merge).  The last kept
  // entry's d and z live in registers and the sorted copies are read one entry ahead, so no
  // iteration waits on a load that depends on the previous one.  K: kept positions, defl:
  // deflated positions, (ra, rb, rc, rs): rotations of close pairs, all at the merge's offset.
  for (int q = tid; q < nq; q += NT) {
    const Rg g = range(q);
    if (!g.on) continue;
    const int lo = g.lo, s = g.hi - g.lo;
    const double rho = 2.0 * fabs(e[g.k - 1]), tol = S.tol[q];
    int nk = 0, nd = 0, nr = 0, prev = -1;
    double zp = 0.0, dp = 0.0;
    int tn = S.perm[lo];
    double zn = S.zK[lo], dn = S.dK[lo];
    for (int r = 0; r < s; ++r) {
      const int t = tn;
      const double zt = zn, dt = dn;
      if (r + 1 < s) {
        tn = S.perm[lo + r + 1];
        zn = S.zK[lo + r + 1];
        dn = S.dK[lo + r + 1];
      }
      if (rho * fabs(zt) <= tol) {
        S.defl[lo + nd++] = t;
        continue;
      }
      if (prev >= 0 && fabs(dt - dp) <= tol) {
        const double rr = sqrt(zp * zp + zt * zt);
        const double c = zt / rr, sn = zp / rr;
        const double dtn = sn * sn * dp + c * c * dt;
        S.dd[prev] = c * c * dp + sn * sn * dt;
        S.dd[t] = dtn;
        S.z[prev] = 0.0;
        S.z[t] = rr;
        S.ra[lo + nr] = prev;
        S.rb[lo + nr] = t;
        S.rc[lo + nr] = c;
        S.rs[lo + nr] = sn;
        ++nr;
        S.defl[lo + nd++] = prev;
        prev = t;
        zp = rr;
        dp = dtn;
        continue;
      }
      if (prev >= 0) S.K[lo + nk++] = prev;
      prev = t;
      zp = zt;
      dp = dt;
    }
    if (prev >= 0) S.K[lo + nk++] = prev;
    S.cnk[q] = nk;
    S.cnr[q] = nr;
  }
  __syncthreads();
  // the deflation rotations act on the columns of Q; each row evolves independently
  for (int r = tid; r < n; r += NT) {
    const int q = merge_of(r);
    const Rg g = range(q);
    if (!g.on) continue;
    const int nr = S.cnr[q];
    for (int p = 0; p < nr; ++p) {
      const size_t ca = (size_t)S.ra[g.lo + p] * n + r, cb = (size_t)S.rb[g.lo + p] * n + r;
      const double c = S.rc[g.lo + p], sn = S.rs[g.lo + p];
      const double qa = Z[ca], qb = Z[cb];
      Z[ca] = c * qa - sn * qb;
      Z[cb] = sn * qa + c * qb;
    }
  }
  __syncthreads();
  // gather: kept columns of Q (in ascending eigenvalue order), then the deflated ones, to Wg;
  // kept z and d contiguous
  for (int idx = tid; idx < n * smax; idx += NT) {
    const int cg = idx / smax, q = merge_of(cg);
    const Rg g = range(q);
    const int r = g.lo + idx % smax;
    if (!g.on || r >= g.hi) continue;
    const int c = cg - g.lo, nk = S.cnk[q];
    const int col = c < nk ? S.K[g.lo + c] : S.defl[g.lo + c - nk];
    Wg[(size_t)cg * n + r] = Z[(size_t)col * n + r];
  }
  for (int i = tid; i < n; i += NT) {
    const int q = merge_of(i);
    const Rg g = range(q);
    if (!g.on || i - g.lo >= S.cnk[q]) continue;
    S.zK[i] = S.z[S.K[i]];
    S.dK[i] = S.dd[S.K[i]];
  }
  __syncthreads();
  // secular roots: four lanes per root, each summing a quarter of the terms (a quad shares its
  // root, so its lanes agree on every branch)
  for (int i = tid >> 2; i < n; i += NT / 4) {
    const int q4 = tid & 3, q = merge_of(i);
    const Rg g = range(q);
    if (!g.on) continue;
    const int nk = S.cnk[q], j = i - g.lo;
    if (j >= nk) continue;
    const double rho = 2.0 * fabs(e[g.k - 1]);
    const double *zK = S.zK + g.lo, *dK = S.dK + g.lo;
    double zs = 0.0;
    for (int t = q4; t < nk; t += 4) zs += zK[t] * zK[t];
    zs = quad_sum(zs);
    const double dj = dK[j];
    int o = j;
    double a, b;
    if (j + 1 < nk) {
      const double half = 0.5 * (dK[j + 1] - dj);
      double f = 0.0;
      for (int t = q4; t < nk; t += 4) f += zK[t] * zK[t] / ((dK[t] - dj) - half);
      f = quad_sum(f);
      f = 1.0 + rho * f;
      if (f >= 0.0) { a = 0.0; b = half; }
      else { o = j + 1; a = -half; b = 0.0; }
    } else {
      a = 0.0;
      b = rho * zs;
    }
    // Safeguarded rational iteration: near tau, the poles at or left of d_j (psi) and right
    // of it (phi) are modelled as p + q/(dL - x) and r + s/(dR - x), matched in value and
    // slope; the model's root (a quadratic) is taken when it lies inside the bracket [a, b],
    // else the bracket midpoint.  Stops when f vanishes to rounding or the bracket closes.
    const double dorg = dK[o];
    const bool hasR = j + 1 < nk;
    const double dL = dK[j] - dorg, dR = hasR ? dK[j + 1] - dorg : 0.0;
    double tau = 0.5 * (a + b);
    for (int it = 0; it < 96; ++it) {
      double psi = 0.0, dpsi = 0.0, phi = 0.0, dphi = 0.0;
      for (int t = q4; t < nk; t += 4) {
        const double r = 1.0 / ((dK[t] - dorg) - tau);
        const double w = zK[t] * zK[t] * r;
        if (t <= j) {
          psi += w;
          dpsi += w * r;
        } else {
          phi += w;
          dphi += w * r;
        }
      }
      psi = rho * quad_sum(psi);
      dpsi = rho * quad_sum(dpsi);
      phi = rho * quad_sum(phi);
      dphi = rho * quad_sum(dphi);
      const double f = 1.0 + psi + phi;
      if (fabs(f) <= eps * (1.0 + fabs(psi) + phi)) break;
      if (f > 0.0) b = tau;
      else a = tau;
      if (!(b - a > 4.0 * eps * fmax(fabs(a), fabs(b)))) break;
      const double hL = dL - tau;
      const double Qm = dpsi * hL * hL, Pm = psi - dpsi * hL;
      double x = 0.5 * (a + b);
      if (hasR) {
        const double hR = dR - tau;
        const double Sm = dphi * hR * hR, Rm = phi - dphi * hR;
        const double C = 1.0 + Pm + Rm;
        const double B = C * (dL + dR) + Qm + Sm, Dq = C * dL * dR + Qm * dR + Sm * dL;
        const double disc = B * B - 4.0 * C * Dq;
        if (C != 0.0 && disc >= 0.0) {
          const double sq = sqrt(disc), den = B >= 0.0 ? B + sq : B - sq;
          const double u1 = den / (2.0 * C);
          const double u2 = den != 0.0 ? 2.0 * Dq / den : u1;
          if (u1 > a && u1 < b) x = u1;
          else if (u2 > a && u2 < b) x = u2;
        }
      } else {
        const double C = 1.0 + Pm + phi;
        if (C > 0.0) {
          const double u = dL + Qm / C;
          if (u > a && u < b) x = u;
        }
      }
      if (x == tau) break;
      tau = x;
    }
    if (q4 == 0) {
      S.dorg[i] = dorg;
      S.tau[i] = tau;
    }
  }
  __syncthreads();
  // zhat_t^2 = (lambda_{nk-1} - d_t)/rho * prod_{j<t} (lambda_j - d_t)/(d_j - d_t)
  //            * prod_{t<=j<nk-1} (lambda_j - d_t)/(d_{j+1} - d_t)      (d = kept, ascending)
  for (int i = tid >> 2; i < n; i += NT / 4) {
    const int q4 = tid & 3, q = merge_of(i);
    const Rg g = range(q);
    if (!g.on) continue;
    const int nk = S.cnk[q], t = i - g.lo;
    if (t >= nk) continue;
    const double rho = 2.0 * fabs(e[g.k - 1]);
    const double *dK = S.dK + g.lo, *tau = S.tau + g.lo, *dorg = S.dorg + g.lo;
    const double dt = dK[t];
    double prod = q4 == 0 ? (tau[nk - 1] - (dt - dorg[nk - 1])) / rho : 1.0;
    for (int j = q4; j < t; j += 4) prod *= (tau[j] - (dt - dorg[j])) / (dK[j] - dt);
    for (int j = t + q4; j < nk - 1; j += 4) prod *= (tau[j] - (dt - dorg[j])) / (dK[j + 1] - dt);
    prod = quad_prod(prod);
    if (q4 == 0) S.zh[i] = copysign(sqrt(fmax(prod, 0.0)), S.zK[i]);
  }
  __syncthreads();
  // coefficient vectors v_j (unnormalised; the norms are taken in the product below), column
  // lo + j at Vg[(lo + j) n + lo ..]
  for (int idx = tid; idx < n * smax; idx += NT) {
    const int jg = idx / smax, q = merge_of(jg);
    const Rg g = range(q);
    if (!g.on) continue;
    const int nk = S.cnk[q], j = jg - g.lo, t = idx % smax;
    if (j >= nk || t >= nk) continue;
    Vg[(size_t)jg * n + g.lo + t] =
        S.zh[g.lo + t] / ((S.dK[g.lo + t] - S.dorg[jg]) - S.tau[jg]);
  }
  for (int i = tid; i < n; i += NT) {
    const int q = merge_of(i);
    const Rg g = range(q);
    if (g.on && i - g.lo < S.cnk[q]) S.lam[i] = S.dorg[i] + S.tau[i];
  }
  __syncthreads();
  // new eigenvectors Q_K V (4 x 4 register tiles), then the deflated columns
  {
    const int tm = (smax + 3) >> 2, tpm = tm * tm;   // tiles per merge, at most
    for (int tile = tid; tile < nq * tpm; tile += NT) {
      const int q = tile / tpm, tl = tile % tpm;
      const Rg g = range(q);
      if (!g.on) continue;
      const int lo = g.lo, hi = g.hi, s = hi - lo, nk = S.cnk[q];
      const int tr = (s + 3) >> 2, tc = (nk + 3) >> 2;
      if (tl >= tr * tc) continue;
      const int r0 = lo + (tl % tr) * 4, j0 = (tl / tr) * 4;
      double acc[4][4];
#pragma unroll
      for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int v = 0; v < 4; ++v) acc[u][v] = 0.0;
      const double *vcol[4];
#pragma unroll
      for (int v = 0; v < 4; ++v) vcol[v] = Vg + (size_t)(lo + min(j0 + v, nk - 1)) * n + lo;
      double nrm[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll 4
      for (int t = 0; t < nk; ++t) {
        const double *wcol = Wg + (size_t)(lo + t) * n;
        double a[4], b[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) a[u] = r0 + u < hi ? wcol[r0 + u] : 0.0;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          b[v] = vcol[v][t];
          nrm[v] += b[v] * b[v];
        }
#pragma unroll
        for (int u = 0; u < 4; ++u)
#pragma unroll
          for (int v = 0; v < 4; ++v) acc[u][v] += a[u] * b[v];
      }
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const double inv = 1.0 / sqrt(nrm[v]);
#pragma unroll
        for (int u = 0; u < 4; ++u)
          if (j0 + v < nk && r0 + u < hi) Z[(size_t)(lo + j0 + v) * n + r0 + u] = acc[u][v] * inv;
      }
    }
    for (int idx = tid; idx < n * smax; idx += NT) {
      const int cg = idx / smax, q = merge_of(cg);
      const Rg g = range(q);
      const int r = g.lo + idx % smax;
      if (!g.on || r >= g.hi || cg - g.lo < S.cnk[q]) continue;
      Z[(size_t)cg * n + r] = Wg[(size_t)cg * n + r];
    }
    for (int i = tid; i < n; i += NT) {
      const int q = merge_of(i);
      const Rg g = range(q);
      if (!g.on) continue;
      const int j = i - g.lo, nk = S.cnk[q];
      d[i] = j < nk ? S.lam[i] : S.dd[S.defl[g.lo + j - nk]];
    }
  }
  __syncthreads();
}

// eigh_tridiag_kernel: stage 1 (Householder reduction), NT threads per matrix; writes the
// reflectors and tau, d to the eigenvalue area and e to the staging area of the workspace.
// NMAX = 128: matrix packed (lower triangle) in LDS.  NMAX = 256: lower triangle of a row-major
// n x n array in this matrix's workspace, which stays in L2 (n > 256: eigh_trd_panel_kernel).
template <int NMAX, int NT>
__global__ __launch_bounds__(NT) void eigh_tridiag_kernel(int n, int lda, const double *const *in,
                                                          double *ws) {
  constexpr bool BIG = NMAX > 128;
  constexpr int HALVES = NT / 256;              // BIG: row slabs of the column pass
  constexpr int TPR = NT / 128;                 // !BIG: threads per row of the matvec
  extern __shared__ double2 smem[];
  __shared__ double d_s[NMAX], e_s[NMAX];
  __shared__ __attribute__((aligned(16))) double sbuf[(6 + 2 * HALVES) * NMAX];
  __shared__ double2 tau_sh;
  __shared__ double2 dot_s[NT / 64];
  double2 *v_s = reinterpret_cast<double2 *>(sbuf), *w_s = v_s + NMAX;
  double2 *x1_s = w_s + NMAX, *x2_s = x1_s + NMAX;   // BIG: row part, HALVES column partials
  const int prob = blockIdx.x;
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  constexpr int nw = NT / 64;
  double *base = ws + (size_t)prob * tql_ws_doubles(n);
  double2 *hh = reinterpret_cast<double2 *>(base);
  double2 *tau_g = hh + (size_t)n * n;
  double *Zg = reinterpret_cast<double *>(tau_g + n);
  double *dg = Zg + (size_t)n * n;
  double *Wg = dg + n;
  double2 *Pg = reinterpret_cast<double2 *>(Wg + (size_t)n * n);
  const double2 *src = reinterpret_cast<const double2 *>(in[prob]);
  // element (i, j), i >= j, of the matrix being reduced
  auto pel = [&](int i, int j) -> double2 & {
    if constexpr (BIG) return Pg[(size_t)i * n + j];
    else return smem[pk_idx(i, j)];
  };

  // Hermitian part of the input, lower triangle
  for (int i = wave; i < n; i += nw)
    for (int j = lane; j <= i; j += 64) {
      double2 a = gld(src, (long)i * lda + j), b = gld(src, (long)j * lda + i);
      pel(i, j) = make_double2(0.5 * (a.x + b.x), i == j ? 0.0 : 0.5 * (a.y - b.y));
    }
  __syncthreads();

  // ---- 1. tridiagonal reduction ----
  if constexpr (!BIG) {
    // n <= 128, matrix packed in LDS, with look-ahead: while waves 1.. apply the rank-2 update
    // of step k to columns k+2.., wave 0 updates column k+1 and forms reflector k+1 from it in
    // registers, so every step has two barriers and no serial reflector phase.  The reflector
    // vector and tau are double buffered: v_s[b VB + i] (b = 0: v_s, b = 1: x1_s) and tau_b[b].
    // (The buffer is chosen by an offset from v_s, not by a pointer picked at run time, which
    // the compiler could not keep in LDS and would access as flat memory.)
    __shared__ double2 tau_b[2];
    constexpr int VB = 2 * NMAX;
    // reflector k from its column col[i] = A(k+1+i, k), i < m (this lane: i = lane + 64 t), and
    // the diagonal dkk = A(k, k); wave 0 only
    auto reflect = [&](int k, const double2 (&col)[2], double dkk, int b) {
      const int m = n - 1 - k;
      double sq = 0.0;
#pragma unroll
      for (int t = 0; t < 2; ++t) {
        const int i = lane + 64 * t;
        if (i >= 1 && i < m) sq += col[t].x * col[t].x + col[t].y * col[t].y;
      }
      sq = wave_sum(sq);
      const double2 alpha = make_double2(readlane_d(col[0].x, 0), readlane_d(col[0].y, 0));
      double2 tau = make_double2(0.0, 0.0), scale = make_double2(0.0, 0.0);
      double beta = alpha.x;
      if (sq > 0.0 || alpha.y != 0.0) {
        beta = -copysign(sqrt(alpha.x * alpha.x + alpha.y * alpha.y + sq), alpha.x);
        tau = make_double2((beta - alpha.x) / beta, -alpha.y / beta);
        const double2 den = make_double2(alpha.x - beta, alpha.y);   // 1 / (alpha - beta)
        const double dn = den.x * den.x + den.y * den.y;
        scale = make_double2(den.x / dn, -den.y / dn);
      }
#pragma unroll
      for (int t = 0; t < 2; ++t) {
        const int i = lane + 64 * t;
        if (i < m) {
          const double2 vi = i == 0 ? make_double2(1.0, 0.0) : cmul(col[t], scale);
          v_s[b * VB + i] = vi;
          hh[(size_t)k * n + k + 1 + i] = vi;
        }
      }
      if (lane == 0) {
        tau_b[b] = tau;
        tau_g[k] = tau;
        e_s[k] = beta;
        d_s[k] = dkk;
      }
    };
    auto reflect_lds = [&](int k, int b) {
      const int m = n - 1 - k;
      double2 col[2];
#pragma unroll
      for (int t = 0; t < 2; ++t) {
        const int i = lane + 64 * t;
        col[t] = i < m ? pel(k + 1 + i, k) : make_double2(0.0, 0.0);
      }
      reflect(k, col, pel(k, k).x, b);
    };
    int b = 0;
    if (n >= 2 && wave == 0) reflect_lds(0, 0);
    __syncthreads();
    for (int k = 0; k + 1 < n; ++k, b ^= 1) {
      const int m = n - 1 - k;          // length of the column below the diagonal
      const double2 tau = tau_b[b];
      if (tau.x == 0.0 && tau.y == 0.0) {   // H_k = I: column k+1 is as it was
        if (k + 2 < n && wave == 0) reflect_lds(k + 1, b ^ 1);
        __syncthreads();
        continue;
      }
      const double2 *v = v_s + b * VB;
      {
        // x = tau S v over the trailing block S (rows / columns k+1 .. n-1): TPR = 8 threads per
        // row; row gi of S is row gi of the packed triangle up to the diagonal, then column gi
        // (packed index of (k+1+c, gi) stepped by c += 8: + 8 (k+1+c) + 36)
        static_assert(TPR == 8, "the row sums are reductions over aligned groups of 8 lanes");
        const int r = tid / TPR, q = tid % TPR;
        double2 acc = make_double2(0.0, 0.0);
        if (r < m) {
          const int gi = k + 1 + r;
          const double2 *prow = smem + pk_idx(gi, k + 1);
#pragma unroll 4
          for (int c = q; c <= r; c += TPR) {
            const double2 a = prow[c], vc = v[c];
            acc.x += a.x * vc.x - a.y * vc.y;
            acc.y += a.x * vc.y + a.y * vc.x;
          }
          int i = gi + 1 + q, idx = i * (i + 1) / 2 + gi;
#pragma unroll 4
          for (int c = r + 1 + q; c < m; c += TPR) {
            const double2 a = smem[idx], vc = v[c];   // conj(a) vc
            acc.x += a.x * vc.x + a.y * vc.y;
            acc.y += a.x * vc.y - a.y * vc.x;
            idx += 8 * i + 36;
            i += 8;
          }
        }
        acc.x = oct_sum(acc.x);
        acc.y = oct_sum(acc.y);
        // this wave's share of v^H x (rows r < m), for a = -(1/2) Re(conj(tau) v^H x)
        double pr = 0.0, pi = 0.0;
        if (r < m && q == 0) {
          const double2 x = cmul(tau, acc), vr = v[r];
          w_s[r] = x;
          pr = vr.x * x.x + vr.y * x.y;
          pi = vr.x * x.y - vr.y * x.x;
        }
        pr = wave_sum(pr);
        pi = wave_sum(pi);
        if (lane == 0) dot_s[wave] = make_double2(pr, pi);
      }
      __syncthreads();
      double dr = 0.0, di = 0.0;
#pragma unroll
      for (int w2 = 0; w2 < nw; ++w2) {          // the waves' shares in a fixed order
        dr += dot_s[w2].x;
        di += dot_s[w2].y;
      }
      const double aw = -0.5 * (tau.x * dr + tau.y * di);
      // S <- S - v w^H - w v^H on the lower triangle, w = x + aw v
      auto wval = [&](int i) {
        const double2 vi = v[i], xi = w_s[i];
        return make_double2(xi.x + aw * vi.x, xi.y + aw * vi.y);
      };
      auto upd = [&](double2 a, double2 vi, double2 wi, double2 vc, double2 wc, bool diag) {
        const double ur = vi.x * wc.x + vi.y * wc.y + wi.x * vc.x + wi.y * vc.y;
        const double ui = vi.y * wc.x - vi.x * wc.y + wi.y * vc.x - wi.x * vc.y;
        return make_double2(a.x - ur, diag ? 0.0 : a.y - ui);
      };
      if (wave == 0) {
        // column k+1 (c = 0): the diagonal by lane 0, rows rr = 1 + lane + 64 t, then the next
        // reflector from these values
        const double2 v0 = v[0], w0 = wval(0);
        double dnext = 0.0;
        if (lane == 0) {
          double2 &a = smem[pk_idx(k + 1, k + 1)];
          const double2 y = upd(a, v0, w0, v0, w0, true);
          a = y;
          dnext = y.x;
        }
        double2 col[2];
#pragma unroll
        for (int t = 0; t < 2; ++t) {
          const int rr = 1 + lane + 64 * t;
          col[t] = make_double2(0.0, 0.0);
          if (rr < m) {
            double2 &a = smem[pk_idx(k + 1 + rr, k + 1)];
            col[t] = upd(a, v[rr], wval(rr), v0, w0, false);
            a = col[t];
          }
        }
        if (k + 2 < n) reflect(k + 1, col, readlane_d(dnext, 0), b ^ 1);
      } else {
        // columns c >= 1 of rows rr (waves 1 .. nw-1 in turn)
        double2 wl[NMAX / 64], vl[NMAX / 64];
#pragma unroll
        for (int t = 0; t < NMAX / 64; ++t) {
          const int c = lane + 64 * t;
          vl[t] = c < m ? v[c] : make_double2(0.0, 0.0);
          wl[t] = c < m ? wval(c) : make_double2(0.0, 0.0);
        }
        for (int rr = wave - 1; rr < m; rr += nw - 1) {
          const double2 vi = v[rr], wi = wval(rr);
          double2 *prow = smem + pk_idx(k + 1 + rr, k + 1);
#pragma unroll
          for (int t = 0; t < NMAX / 64; ++t) {
            const int c = lane + 64 * t;
            if (c >= 1 && c <= rr) prow[c] = upd(prow[c], vi, wi, vl[t], wl[t], c == rr);
          }
        }
      }
      __syncthreads();
    }
  } else
  for (int k = 0; k + 1 < n; ++k) {
    const int m = n - 1 - k;          // length of the column below the diagonal
    if (wave == 0) {
      double sq = 0.0;
      for (int i = 1 + lane; i < m; i += 64) {
        double2 x = pel(k + 1 + i, k);
        sq += x.x * x.x + x.y * x.y;
      }
      sq = wave_sum(sq);
      const double2 alpha = pel(k + 1, k);
      double2 tau = make_double2(0.0, 0.0), scale = make_double2(0.0, 0.0);
      double beta = alpha.x;
      if (sq > 0.0 || alpha.y != 0.0) {
        beta = -copysign(sqrt(alpha.x * alpha.x + alpha.y * alpha.y + sq), alpha.x);
        tau = make_double2((beta - alpha.x) / beta, -alpha.y / beta);
        const double2 den = make_double2(alpha.x - beta, alpha.y);   // 1 / (alpha - beta)
        const double dn = den.x * den.x + den.y * den.y;
        scale = make_double2(den.x / dn, -den.y / dn);
      }
      for (int i = lane; i < m; i += 64) {
        double2 vi = i == 0 ? make_double2(1.0, 0.0) : cmul(pel(k + 1 + i, k), scale);
        v_s[i] = vi;
        hh[(size_t)k * n + k + 1 + i] = vi;
      }
      if (lane == 0) {
        tau_sh = tau;
        tau_g[k] = tau;
        e_s[k] = beta;
        d_s[k] = pel(k, k).x;
      }
    }
    __syncthreads();
    const double2 tau = tau_sh;
    if (tau.x == 0.0 && tau.y == 0.0) continue;   // H_k = I (uniform over the block)
    if constexpr (!BIG) {
      // x = tau S v over the trailing block S (rows / columns k+1 .. n-1): TPR = 8 threads per
      // row; row gi of S is row gi of the packed triangle up to the diagonal, then column gi
      // (packed index of (k+1+c, gi) stepped by c += 8: + 8 (k+1+c) + 36)
      static_assert(TPR == 8, "the row sums are reductions over aligned groups of 8 lanes");
      const int r = tid / TPR, q = tid % TPR;
      double2 acc = make_double2(0.0, 0.0);
      if (r < m) {
        const int gi = k + 1 + r;
        const double2 *prow = smem + pk_idx(gi, k + 1);
#pragma unroll 4
        for (int c = q; c <= r; c += TPR) {
          const double2 a = prow[c], vc = v_s[c];
          acc.x += a.x * vc.x - a.y * vc.y;
          acc.y += a.x * vc.y + a.y * vc.x;
        }
        int i = gi + 1 + q, idx = i * (i + 1) / 2 + gi;
#pragma unroll 4
        for (int c = r + 1 + q; c < m; c += TPR) {
          const double2 a = smem[idx], vc = v_s[c];   // conj(a) vc
          acc.x += a.x * vc.x + a.y * vc.y;
          acc.y += a.x * vc.y - a.y * vc.x;
          idx += 8 * i + 36;
          i += 8;
        }
      }
      acc.x = oct_sum(acc.x);
      acc.y = oct_sum(acc.y);
      // this wave's share of v^H x (rows r < m), for a = -(1/2) Re(conj(tau) v^H x)
      double pr = 0.0, pi = 0.0;
      if (r < m && q == 0) {
        const double2 x = cmul(tau, acc), vr = v_s[r];
        w_s[r] = x;
        pr = vr.x * x.x + vr.y * x.y;
        pi = vr.x * x.y - vr.y * x.x;
      }
      pr = wave_sum(pr);
      pi = wave_sum(pi);
      if (lane == 0) dot_s[wave] = make_double2(pr, pi);
    } else {
      // S v from the lower triangle in two coalesced passes: the row part (diagonal included)
      // with 16 lanes per row, and the strictly upper part as conj(S)^T v with one lane per
      // column and the rows split in HALVES slabs by residue
      const double2 *S0 = Pg + (size_t)(k + 1) * n + k + 1;
      {
        const int q = tid & 15;
        for (int r = tid >> 4; r < m; r += NT / 16) {
          const double2 *prow = S0 + (size_t)r * n;
          double2 acc = make_double2(0.0, 0.0);
          for (int c = q; c <= r; c += 16) {
            const double2 a = prow[c], vc = v_s[c];
            acc.x += a.x * vc.x - a.y * vc.y;
            acc.y += a.x * vc.y + a.y * vc.x;
          }
#pragma unroll
          for (int o = 1; o < 16; o <<= 1) {
            acc.x += __shfl_xor(acc.x, o, 64);
            acc.y += __shfl_xor(acc.y, o, 64);
          }
          if (q == 0) x1_s[r] = acc;
        }
      }
      for (int c = tid & 255; c < NMAX; c += 256) {
        const int half = tid >> 8, c0 = c & ~63;
        if (c0 < m) {
          double2 acc = make_double2(0.0, 0.0);
#pragma unroll 4
          for (int r = c0 + 1 + half; r < m; r += HALVES) {
            if (r > c) {
              const double2 a = S0[(size_t)r * n + c], vr = v_s[r];   // conj(a) v_r
              acc.x += a.x * vr.x + a.y * vr.y;
              acc.y += a.x * vr.y - a.y * vr.x;
            }
          }
          if (c < m) x2_s[half * NMAX + c] = acc;
        }
      }
    }
    __syncthreads();
    // every wave forms a = -(1/2) Re(conj(tau) v^H x) itself; then S <- S - v w^H - w v^H on
    // the lower triangle with w = x + a v formed on the fly
    auto xval = [&](int i) -> double2 {
      if constexpr (BIG) {
        double2 t = x1_s[i];
#pragma unroll
        for (int h = 0; h < HALVES; ++h) {
          const double2 u = x2_s[h * NMAX + i];
          t.x += u.x;
          t.y += u.y;
        }
        return cmul(tau, t);
      } else {
        return w_s[i];
      }
    };
    double dr = 0.0, di = 0.0;
    if constexpr (BIG) {
      for (int i = lane; i < m; i += 64) {
        const double2 vi = v_s[i], xi = xval(i);
        dr += vi.x * xi.x + vi.y * xi.y;
        di += vi.x * xi.y - vi.y * xi.x;
      }
      dr = wave_sum(dr);
      di = wave_sum(di);
    } else {
#pragma unroll
      for (int w2 = 0; w2 < nw; ++w2) {        // the waves' shares in a fixed order
        dr += dot_s[w2].x;
        di += dot_s[w2].y;
      }
    }
    const double aw = -0.5 * (tau.x * dr + tau.y * di);
    // w at this lane's columns (c = lane + 64 t)
    double2 wl[NMAX / 64];
#pragma unroll
    for (int t = 0; t < NMAX / 64; ++t) {
      const int c = lane + 64 * t;
      if (c < m) {
        const double2 vc = v_s[c], xc = xval(c);
        wl[t] = make_double2(xc.x + aw * vc.x, xc.y + aw * vc.y);
      } else {
        wl[t] = make_double2(0.0, 0.0);
      }
    }
    for (int rr = wave; rr < m; rr += nw) {
      const int gi = k + 1 + rr;
      const double2 vi = v_s[rr], xi = xval(rr);
      const double2 wi = make_double2(xi.x + aw * vi.x, xi.y + aw * vi.y);
      double2 *prow = &pel(gi, k + 1);
#pragma unroll
      for (int t = 0; t < NMAX / 64; ++t) {
        const int c = lane + 64 * t;
        if (c <= rr) {
          const double2 vc = v_s[c], wc = wl[t];
          const double2 a = prow[c];
          const double ur = vi.x * wc.x + vi.y * wc.y + wi.x * vc.x + wi.y * vc.y;
          const double ui = vi.y * wc.x - vi.x * wc.y + wi.y * vc.x - wi.x * vc.y;
          prow[c] = make_double2(a.x - ur, c == rr ? 0.0 : a.y - ui);
        }
      }
    }
    __syncthreads();
  }
  if (tid == 0) {
    d_s[n - 1] = pel(n - 1, n - 1).x;
    e_s[n - 1] = 0.0;
  }
  __syncthreads();
  for (int i = tid; i < n; i += NT) {
    dg[i] = d_s[i];
    Wg[i] = e_s[i];
  }
}

// Blocked Householder reduction for n > 256 (the reduction of eigh_tridiag_kernel, reorganised as in
// LAPACK's panel form): a panel of TRD_NB reflectors is generated by one workgroup per matrix
// without touching the stored matrix A_st, whose true trailing part is
// A_st - V W^H - W V^H for the panel's reflector vectors V and w-vectors W so far; the column a
// reflector is taken from and every product S v are corrected on the fly.  After the panel two
// GEMMs apply A_st -= V W^H + W V^H.  The single-workgroup memory traffic per reflector drops from
// four passes over the trailing triangle (two reads for S v, read and write for the rank-2
// update) to two.  Outputs as eigh_tridiag_kernel: reflectors and tau, d to the eigenvalue area
// and e to the staging area.
template <int NMAX, int NT>
__global__ __launch_bounds__(NT) void eigh_trd_panel_kernel(int n, int lda, const double *const *in,
                                                            double *ws, int k0) {
  constexpr int HALVES = NT / 256;
  __shared__ __attribute__((aligned(16))) double sbuf[(6 + 2 * HALVES) * NMAX];
  __shared__ double2 pq_s[2 * TRD_NB];
  __shared__ double2 tau_sh;
  double2 *v_s = reinterpret_cast<double2 *>(sbuf), *a_s = v_s + NMAX;
  double2 *x1_s = a_s + NMAX, *x2_s = x1_s + NMAX;
  const int prob = blockIdx.x;
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  constexpr int nw = NT / 64;
  double *base = ws + (size_t)prob * tql_ws_doubles(n);
  double2 *hh = reinterpret_cast<double2 *>(base);
  double2 *tau_g = hh + (size_t)n * n;
  double *Zg = reinterpret_cast<double *>(tau_g + n);
  double *dg = Zg + (size_t)n * n;
  double *Wg = dg + n;
  double2 *Pg = reinterpret_cast<double2 *>(Wg + (size_t)n * n);
  double2 *U = reinterpret_cast<double2 *>(base + trd_panel_offset(n));   // [n][2 TRD_NB]
  constexpr int UL = 2 * TRD_NB;
  if (k0 == 0) {
    const double2 *src = reinterpret_cast<const double2 *>(in[prob]);
    for (int i = wave; i < n; i += nw)
      for (int j = lane; j <= i; j += 64) {
        const double2 a = src[(size_t)i * lda + j], b = src[(size_t)j * lda + i];
        Pg[(size_t)i * n + j] = make_double2(0.5 * (a.x + b.x), i == j ? 0.0 : 0.5 * (a.y - b.y));
      }
  }
  for (int idx = tid; idx < n * UL; idx += NT) U[idx] = make_double2(0.0, 0.0);
  __syncthreads();
  const int kend = min(n - 1, k0 + TRD_NB);
  for (int k = k0; k < kend; ++k) {
    const int j = k - k0, m = n - 1 - k;
    // 1. column k of the true matrix, rows k..n-1: A_st[i][k] - sum_c V[i][c] conj(W[k][c]) +
    //    W[i][c] conj(V[k][c])
    for (int i = k + tid; i < n; i += NT) {
      double2 a = Pg[(size_t)i * n + k];
      for (int c = 0; c < j; ++c) {
        const double2 vi = U[(size_t)i * UL + c], wi = U[(size_t)i * UL + TRD_NB + c];
        const double2 vk = U[(size_t)k * UL + c], wk = U[(size_t)k * UL + TRD_NB + c];
        // vi conj(wk) + wi conj(vk)
        a.x -= vi.x * wk.x + vi.y * wk.y + wi.x * vk.x + wi.y * vk.y;
        a.y -= vi.y * wk.x - vi.x * wk.y + wi.y * vk.x - wi.x * vk.y;
      }
      a_s[i - k] = a;
    }
    __syncthreads();
    // 2. the reflector (wave 0), as in eigh_tridiag_kernel
    if (wave == 0) {
      double sq = 0.0;
      for (int i = 2 + lane; i <= m; i += 64) {
        const double2 x = a_s[i];
        sq += x.x * x.x + x.y * x.y;
      }
      sq = wave_sum(sq);
      const double2 alpha = a_s[1];
      double2 tau = make_double2(0.0, 0.0), scale = make_double2(0.0, 0.0);
      double beta = alpha.x;
      if (sq > 0.0 || alpha.y != 0.0) {
        beta = -copysign(sqrt(alpha.x * alpha.x + alpha.y * alpha.y + sq), alpha.x);
        tau = make_double2((beta - alpha.x) / beta, -alpha.y / beta);
        const double2 den = make_double2(alpha.x - beta, alpha.y);   // 1 / (alpha - beta)
        const double dn = den.x * den.x + den.y * den.y;
        scale = make_double2(den.x / dn, -den.y / dn);
      }
      for (int i = lane; i < m; i += 64) {
        const double2 vi = i == 0 ? make_double2(1.0, 0.0) : cmul(a_s[1 + i], scale);
        v_s[i] = vi;
        hh[(size_t)k * n + k + 1 + i] = vi;
        U[(size_t)(k + 1 + i) * UL + j] = vi;
      }
      if (lane == 0) {
        tau_sh = tau;
        tau_g[k] = tau;
        Wg[k] = beta;
        dg[k] = a_s[0].x;
      }
    }
    __syncthreads();
    const double2 tau = tau_sh;
    if (tau.x == 0.0 && tau.y == 0.0) continue;   // H_k = I: w = 0 (U's column stays 0)
    // 3. S v over the stored trailing block (two coalesced passes as in eigh_tridiag_kernel) and
    //    the panel scalars p_c = W_c^H v, q_c = V_c^H v (rows k+1..n-1)
    const double2 *S0 = Pg + (size_t)(k + 1) * n + k + 1;
    {
      const int q = tid & 15;
      for (int r = tid >> 4; r < m; r += NT / 16) {
        const double2 *prow = S0 + (size_t)r * n;
        double2 acc = make_double2(0.0, 0.0);
        for (int c = q; c <= r; c += 16) {
          const double2 a = prow[c], vc = v_s[c];
          acc.x += a.x * vc.x - a.y * vc.y;
          acc.y += a.x * vc.y + a.y * vc.x;
        }
#pragma unroll
        for (int o = 1; o < 16; o <<= 1) {
          acc.x += __shfl_xor(acc.x, o, 64);
          acc.y += __shfl_xor(acc.y, o, 64);
        }
        if (q == 0) x1_s[r] = acc;
      }
    }
    for (int c = tid & 255; c < NMAX; c += 256) {
      const int half = tid >> 8, c0 = c & ~63;
      if (c0 < m) {
        double2 acc = make_double2(0.0, 0.0);
#pragma unroll 4
        for (int r = c0 + 1 + half; r < m; r += HALVES) {
          if (r > c) {
            const double2 a = S0[(size_t)r * n + c], vr = v_s[r];   // conj(a) v_r
            acc.x += a.x * vr.x + a.y * vr.y;
            acc.y += a.x * vr.y - a.y * vr.x;
          }
        }
        if (c < m) x2_s[half * NMAX + c] = acc;
      }
    }
    for (int c = wave; c < 2 * j; c += nw) {      // c < j: p_c (W column), else q_{c-j} (V)
      const int col = c < j ? TRD_NB + c : c - j;
      double pr = 0.0, pi = 0.0;
      for (int i = lane; i < m; i += 64) {
        const double2 u = U[(size_t)(k + 1 + i) * UL + col], vi = v_s[i];   // conj(u) v
        pr += u.x * vi.x + u.y * vi.y;
        pi += u.x * vi.y - u.y * vi.x;
      }
      pr = wave_sum(pr);
      pi = wave_sum(pi);
      if (lane == 0) pq_s[c] = make_double2(pr, pi);
    }
    __syncthreads();
    // x_i = tau (S v - sum_c V[i][c] p_c + W[i][c] q_c)
    for (int i = tid; i < m; i += NT) {
      double2 t = x1_s[i];
#pragma unroll
      for (int h = 0; h < HALVES; ++h) {
        const double2 u = x2_s[h * NMAX + i];
        t.x += u.x;
        t.y += u.y;
      }
      for (int c = 0; c < j; ++c) {
        const double2 vi = U[(size_t)(k + 1 + i) * UL + c], wi = U[(size_t)(k + 1 + i) * UL + TRD_NB + c];
        const double2 p = pq_s[c], q = pq_s[j + c];
        t.x -= vi.x * p.x - vi.y * p.y + wi.x * q.x - wi.y * q.y;
        t.y -= vi.x * p.y + vi.y * p.x + wi.x * q.y + wi.y * q.x;
      }
      x1_s[i] = cmul(tau, t);
    }
    __syncthreads();
    // 4. w = x + a v with a = -(1/2) Re(conj(tau) v^H x) (every wave forms a itself)
    double dr = 0.0, di = 0.0;
    for (int i = lane; i < m; i += 64) {
      const double2 vi = v_s[i], xi = x1_s[i];
      dr += vi.x * xi.x + vi.y * xi.y;
      di += vi.x * xi.y - vi.y * xi.x;
    }
    dr = wave_sum(dr);
    di = wave_sum(di);
    const double aw = -0.5 * (tau.x * dr + tau.y * di);
    for (int i = tid; i < m; i += NT) {
      const double2 vi = v_s[i], xi = x1_s[i];
      U[(size_t)(k + 1 + i) * UL + TRD_NB + j] = make_double2(xi.x + aw * vi.x, xi.y + aw * vi.y);
    }
    __syncthreads();
  }
}

// Last diagonal entry after the final panel update (d[n-1]; e[n-1] = 0).  One thread per matrix.
__global__ void eigh_trd_last_kernel(int n, double *ws, int nprob) {
  const int prob = blockIdx.x * blockDim.x + threadIdx.x;
  if (prob >= nprob) return;
  double *base = ws + (size_t)prob * tql_ws_doubles(n);
  double2 *tau_g = reinterpret_cast<double2 *>(base) + (size_t)n * n;
  double *Zg = reinterpret_cast<double *>(tau_g + n);
  double *dg = Zg + (size_t)n * n;
  double *Wg = dg + n;
  const double2 *Pg = reinterpret_cast<const double2 *>(Wg + (size_t)n * n);
  dg[n - 1] = Pg[(size_t)(n - 1) * n + n - 1].x;
  Wg[n - 1] = 0.0;
}

// eigh_dc_kernel: stage 2 (divide and conquer on the tridiagonal d, e left by
// eigh_tridiag_kernel), 512 threads per matrix.  The leaves are single entries (depth
// ceil(log2 n)); every coupling is torn at its level and the levels are merged bottom-up, all
// merges of a level at once (dc_level).  NMAX = 128: Z in LDS; NMAX = 256, 512: Z in the
// workspace.
template <int NMAX>
__global__ __launch_bounds__(512) void eigh_dc_kernel(int n, double *ws) {
  constexpr bool BIG = NMAX > 128;
  extern __shared__ double2 smem[];
  __shared__ double d_s[NMAX], e_s[NMAX];
  // merge scratch: 11 per-position double arrays (10 full, tol per merge), 5 per-position int
  // arrays and 2 per-merge int arrays
  __shared__ __attribute__((aligned(16))) double sbuf[11 * NMAX + 4 * NMAX];
  const int prob = blockIdx.x;
  const int tid = threadIdx.x;
  double *base = ws + (size_t)prob * tql_ws_doubles(n);
  double2 *hh = reinterpret_cast<double2 *>(base);
  double2 *tau_g = hh + (size_t)n * n;
  double *Zg = reinterpret_cast<double *>(tau_g + n);
  double *dg = Zg + (size_t)n * n;
  double *Wg = dg + n;
  double2 *Pg = reinterpret_cast<double2 *>(Wg + (size_t)n * n);
  for (int i = tid; i < n; i += 512) {
    d_s[i] = dg[i];
    e_s[i] = Wg[i];
  }
  int LD = 0;                                   // leaves of at most one entry: n <= 2^LD
  while ((1 << LD) < n) ++LD;
  // Z = I (column-major): the eigenvectors of the single-entry leaves
  double *Z = BIG ? Zg : reinterpret_cast<double *>(smem);
  double *Vg = BIG ? reinterpret_cast<double *>(Pg) : Zg;
  for (int idx = tid; idx < n * n; idx += blockDim.x) Z[idx] = (idx % (n + 1)) == 0 ? 1.0 : 0.0;
  __syncthreads();
  // tear every coupling at the level whose merge it joins: T = diag(T_1 .. T_L) +
  // sum |beta| u u^T with u = e_{k-1} + sign(beta) e_k, the two diagonal entries lowered by |beta|
  if (tid == 0)
    for (int D = 0; D < LD; ++D)
      for (int q = 0; q < (1 << D); ++q) {
        const int lo = dc_bound(q, n, D), hi = dc_bound(q + 1, n, D);
        const int k = dc_bound(2 * q + 1, n, D + 1);
        if (!(lo < k && k < hi)) continue;
        const double r = fabs(e_s[k - 1]);
        d_s[k - 1] -= r;
        d_s[k] -= r;
      }
  __syncthreads();
  {
    DcScratch S;
    double *f = sbuf;
    S.z = f; S.dd = f + NMAX; S.zK = f + 2 * NMAX; S.dK = f + 3 * NMAX;
    S.tau = f + 4 * NMAX; S.dorg = f + 5 * NMAX; S.zh = f + 6 * NMAX;
    S.lam = f + 7 * NMAX; S.rc = f + 8 * NMAX; S.rs = f + 9 * NMAX; S.tol = f + 10 * NMAX;
    int *ib = reinterpret_cast<int *>(f + 11 * NMAX);
    S.perm = ib; S.K = ib + NMAX; S.defl = ib + 2 * NMAX; S.ra = ib + 3 * NMAX;
    S.rb = ib + 4 * NMAX; S.cnk = ib + 5 * NMAX; S.cnr = ib + 6 * NMAX;
    for (int D = LD - 1; D >= 0; --D) dc_level(n, D, e_s, d_s, Z, S, Vg, Wg);
  }
  if constexpr (!BIG)
    for (int idx = tid; idx < n * n; idx += blockDim.x) Zg[idx] = Z[idx];
  for (int i = tid; i < n; i += blockDim.x) dg[i] = d_s[i];
}

template <int NMAX>
__global__ __launch_bounds__(256) void eigh_backtransform_kernel(int n, int ncols, const double *ws,
                                                                 double *const *evals,
                                                                 double *const *vecs) {
  constexpr int CB = NMAX > 256 ? 4 : 16;          // eigenvector columns per workgroup
  __shared__ double2 Vb[NMAX * CB];
  __shared__ double2 vk[2][NMAX];
  __shared__ double2 part[4][CB];
  __shared__ double dsh[NMAX];
  __shared__ int src[NMAX];
  const int prob = blockIdx.y, c0 = blockIdx.x * CB;
  const int tid = threadIdx.x;
  const double *base = ws + (size_t)prob * tql_ws_doubles(n);
  const double2 *hh = reinterpret_cast<const double2 *>(base);
  const double2 *tau_g = hh + (size_t)n * n;
  const double *Zg = reinterpret_cast<const double *>(tau_g + n);
  const double *dg = Zg + (size_t)n * n;
  // descending order (rank sort, ties by index): output column rank holds Z column src[rank];
  // this workgroup's columns are the ranks c0 .. c0 + cols - 1 (ranks below ncols only)
  double *ev = evals[prob];
  for (int i = tid; i < n; i += 256) dsh[i] = dg[i];
  __syncthreads();
  for (int j = tid; j < n; j += 256) {
    const double lj = dsh[j];
    int rank = 0;
    for (int i = 0; i < n; ++i) {
      const double li = dsh[i];
      rank += (li > lj) || (li == lj && i < j);
    }
    src[rank] = j;
    if (blockIdx.x == 0) gst(ev, rank, lj);
  }
  __syncthreads();
  const int cols = min(CB, ncols - c0);
  for (int idx = tid; idx < n * CB; idx += 256) {
    const int r = idx / CB, c = idx % CB;
    Vb[idx] = make_double2(c < cols ? Zg[(size_t)src[c0 + c] * n + r] : 0.0, 0.0);
  }
  __syncthreads();
  constexpr int RG = 256 / CB;                        // row groups per column
  const int c = tid & (CB - 1), part_id = tid / CB;
  // The reflectors are applied in reverse order.  Reflector k - 1's vector (and tau) is loaded
  // from the workspace while reflector k is applied and staged in the other vk buffer at the
  // end of the step, so no step waits on a global load; every thread forms w = tau v^H x for its
  // own column from the four waves' partial sums, so a step has two barriers.
  constexpr int VPT = (NMAX + 255) / 256;           // vector elements per thread
  auto vload = [&](int k, double2 (&dst)[VPT]) {   // reflector k's vector (0 past its end)
#pragma unroll
    for (int e = 0; e < VPT; ++e) {
      const int i = tid + 256 * e;
      dst[e] = (k >= 0 && i < n - 1 - k) ? gld(hh, (long)k * n + k + 1 + i) : make_double2(0.0, 0.0);
    }
  };
  auto vstore = [&](int buf, const double2 (&src)[VPT]) {
#pragma unroll
    for (int e = 0; e < VPT; ++e)
      if (tid + 256 * e < NMAX) vk[buf][tid + 256 * e] = src[e];
  };
  auto tload = [&](int k) -> double2 { return k >= 0 ? gld(tau_g, k) : make_double2(0.0, 0.0); };
  double2 vn[VPT];
  vload(n - 2, vn);
  vstore(0, vn);
  vload(n - 3, vn);
  double2 taun = tload(n - 3), tau = tload(n - 2);
  __syncthreads();
  int b = 0;
  for (int k = n - 2; k >= 0; --k, b ^= 1) {
    const int m = n - 1 - k;
    if (tau.x != 0.0 || tau.y != 0.0) {
      const double2 *v = vk[b];
      double2 acc = make_double2(0.0, 0.0);
      for (int i = part_id; i < m; i += RG) {
        const double2 vv = v[i], x = Vb[(k + 1 + i) * CB + c];
        acc.x += vv.x * x.x + vv.y * x.y;      // conj(v) x
        acc.y += vv.x * x.y - vv.y * x.x;
      }
#pragma unroll
      for (int o = CB; o < 64; o <<= 1) {    // the wave's lanes of this column
        acc.x += __shfl_xor(acc.x, o, 64);
        acc.y += __shfl_xor(acc.y, o, 64);
      }
      if ((tid & 63) < CB) part[tid >> 6][c] = acc;
      __syncthreads();
      const double2 t = make_double2(part[0][c].x + part[1][c].x + part[2][c].x + part[3][c].x,
                                     part[0][c].y + part[1][c].y + part[2][c].y + part[3][c].y);
      const double2 w = cmul(tau, t);
      for (int idx = tid; idx < m * CB; idx += 256) {
        const int i = idx / CB;             // (idx % CB == c: 256 is a multiple of CB)
        const double2 u = cmul(v[i], w);
        double2 &x = Vb[(k + 1 + i) * CB + c];
        x = make_double2(x.x - u.x, x.y - u.y);
      }
    }
    vstore(b ^ 1, vn);
    tau = taun;
    vload(k - 2, vn);
    taun = tload(k - 2);
    __syncthreads();
  }
  double2 *vo = reinterpret_cast<double2 *>(vecs[prob]);
  for (int idx = tid; idx < n * cols; idx += 256) {
    const int r = idx / cols, cc = idx % cols;
    gst(vo, (long)r * n + c0 + cc, Vb[r * CB + cc]);
  }
}

// ------------------------------------------------------------------------------------------
// Pivoted Cholesky factor of a Gram matrix G = A^H A: pivot = largest remaining diagonal entry,
// column of L, update of the trailing Schur complement; stops at the first pivot <= cut * max
// diag.  Then X = L1^{-1}, R = L^H P^T and Wsc = P [L1^{-H}; 0].
//
// For n > 128 it is blocked so that most of the work runs on the GEMM: between launches the workspace
// holds, per matrix, the trailing matrix W, the factor L (row = original index, column = pivot
// order) and X, and the meta block {rank, done, gmax, dg[n], perm[n]} (dg: diagonal of the
// trailing matrix; 16-byte aligned blocks).  chol_init_kernel sets them up; per panel of CHOL_NB columns
// chol_panel_kernel (one workgroup per matrix) picks the pivots and computes the columns with the
// in-panel corrections, and a GEMM applies W -= L_panel L_panel^H.  Then L1^{-1} by blocks: the
// diagonal blocks' inverses (chol_diag_inv_kernel), and for each block row I in turn
// Y = L1[I, :I] X[:I, :I] and X[I, :I] = -X[I, I] Y on the GEMM; chol_out_kernel writes R and Wsc.
constexpr int CHOL_NB = 16;
__host__ __device__ inline size_t chol_meta_bytes(int n) { return (16 + (size_t)n * 12 + 15) & ~size_t(15); }
// per-matrix workspace of the blocked path: W (later L1), L, X (n x n each) and Y (CHOL_NB x n)
__host__ __device__ inline size_t chol_stride(int n) {
  return 3 * (size_t)n * n + (size_t)CHOL_NB * n;
}

__global__ __launch_bounds__(1024) void chol_init_kernel(int n, const double *const *G,
                                                         double2 *ws, char *meta) {
  __shared__ double red[16];
  const int prob = blockIdx.x, tid = threadIdx.x, nt = blockDim.x;
  double2 *W = ws + (size_t)prob * chol_stride(n), *L = W + (size_t)n * n, *X = L + (size_t)n * n;
  char *mb = meta + (size_t)prob * chol_meta_bytes(n);
  double *dg = reinterpret_cast<double *>(mb + 16);
  int *perm = reinterpret_cast<int *>(mb + 16 + (size_t)n * 8);
  const double2 *g = reinterpret_cast<const double2 *>(G[prob]);
  for (int idx = tid; idx < n * n; idx += nt) {
    const int i = idx / n, j = idx % n;
    const double2 x = gld(g, (long)i * n + j), y = gld(g, (long)j * n + i);
    W[idx] = make_double2(0.5 * (x.x + y.x), 0.5 * (x.y - y.y));
    L[idx] = make_double2(0.0, 0.0);
    X[idx] = make_double2(0.0, 0.0);
  }
  double m = 0.0;
  for (int i = tid; i < n; i += nt) {
    perm[i] = i;
    const double d = gld(g, (long)i * n + i).x;
    dg[i] = d;
    m = fmax(m, d);
  }
  for (int o = 32; o > 0; o >>= 1) m = fmax(m, __shfl_xor(m, o, 64));
  if ((tid & 63) == 0) red[tid >> 6] = m;
  __syncthreads();
  if (tid == 0) {
    double gm = 0.0;
    for (int w = 0; w < nt / 64; ++w) gm = fmax(gm, red[w]);
    reinterpret_cast<int *>(mb)[0] = n;         // rank
    reinterpret_cast<int *>(mb)[1] = 0;         // done
    reinterpret_cast<double *>(mb)[1] = gm;     // gmax
  }
}

__global__ __launch_bounds__(1024) void chol_panel_kernel(int n, int k0, double cut, double2 *ws,
                                                          char *meta) {
  extern __shared__ double2 lp[];                // [n][CHOL_NB + 1] (padded rows)
  __shared__ int perm_s[512];
  __shared__ double dg_s[512];
  __shared__ int stop_s;
  constexpr int LD = CHOL_NB + 1;
  const int prob = blockIdx.x, tid = threadIdx.x, nt = blockDim.x;
  const int lane = tid & 63, wave = tid >> 6;
  char *mb = meta + (size_t)prob * chol_meta_bytes(n);
  if (reinterpret_cast<const int *>(mb)[1]) return;          // rank reached in an earlier panel
  const double gmax = reinterpret_cast<const double *>(mb)[1];
  double *dg = reinterpret_cast<double *>(mb + 16);
  int *perm = reinterpret_cast<int *>(mb + 16 + (size_t)n * 8);
  const double2 *W = ws + (size_t)prob * chol_stride(n);
  double2 *L = const_cast<double2 *>(W) + (size_t)n * n;
  for (int i = tid; i < n; i += nt) {
    perm_s[i] = perm[i];
    dg_s[i] = dg[i];
  }
  for (int idx = tid; idx < n * LD; idx += nt) lp[idx] = make_double2(0.0, 0.0);
  if (tid == 0) stop_s = 0;
  __syncthreads();
  int j = 0;
  for (; j < CHOL_NB && k0 + j < n; ++j) {
    const int k = k0 + j;
    if (wave == 0) {
      double best = -1.0;
      int bj = k;
      for (int q = k + lane; q < n; q += 64) {
        const double v = dg_s[perm_s[q]];
        if (v > best) { best = v; bj = q; }
      }
      wave_argmax(best, bj);
      if (lane == 0) {
        if (!(best > cut * gmax) || !(gmax > 0)) {
          stop_s = 1;
        } else {
          const int t = perm_s[k];
          perm_s[k] = perm_s[bj];
          perm_s[bj] = t;
        }
      }
    }
    __syncthreads();
    if (stop_s) break;
    const int pk = perm_s[k];
    const double piv = sqrt(dg_s[pk]);
    const double ipiv = 1.0 / piv;
    for (int q = k + 1 + tid; q < n; q += nt) {
      const int i = perm_s[q];
      double2 v = W[(size_t)i * n + pk];
      for (int c = 0; c < j; ++c) {
        const double2 a = lp[i * LD + c], b = lp[pk * LD + c];
        // v -= a conj(b)
        v.x -= a.x * b.x + a.y * b.y;
        v.y -= a.y * b.x - a.x * b.y;
      }
      lp[i * LD + j] = make_double2(v.x * ipiv, v.y * ipiv);
    }
    if (tid == 0) lp[pk * LD + j] = make_double2(piv, 0.0);
    __syncthreads();
    for (int q = k + 1 + tid; q < n; q += nt) {
      const int i = perm_s[q];
      const double2 l = lp[i * LD + j];
      dg_s[i] -= l.x * l.x + l.y * l.y;
    }
    __syncthreads();
  }
  for (int idx = tid; idx < n * CHOL_NB; idx += nt) {
    const int i = idx / CHOL_NB, c = idx % CHOL_NB;
    if (c < j) L[(size_t)i * n + k0 + c] = lp[i * LD + c];
  }
  for (int i = tid; i < n; i += nt) {
    perm[i] = perm_s[i];
    dg[i] = dg_s[i];
  }
  if (tid == 0 && stop_s) {
    reinterpret_cast<int *>(mb)[0] = k0 + j;
    reinterpret_cast<int *>(mb)[1] = 1;
  }
}

// L1 (pivot order, rows of L permuted; identity rows beyond the rank so that L1 is invertible and
// its leading rank x rank block is the factor's) into the W area; X cleared.
__global__ __launch_bounds__(1024) void chol_l1_kernel(int n, double2 *ws, const char *meta) {
  __shared__ int perm[512];
  const int prob = blockIdx.x, tid = threadIdx.x, nt = blockDim.x;
  double2 *L1 = ws + (size_t)prob * chol_stride(n), *L = L1 + (size_t)n * n, *X = L + (size_t)n * n;
  const char *mb = meta + (size_t)prob * chol_meta_bytes(n);
  const int r = reinterpret_cast<const int *>(mb)[0];
  for (int i = tid; i < n; i += nt) perm[i] = reinterpret_cast<const int *>(mb + 16 + (size_t)n * 8)[i];
  __syncthreads();
  for (int idx = tid; idx < n * n; idx += nt) {
    const int i = idx / n, m = idx % n;
    L1[idx] = i < r ? L[(size_t)perm[i] * n + m] : make_double2(i == m ? 1.0 : 0.0, 0.0);
    X[idx] = make_double2(0.0, 0.0);
  }
}

// Inverses of the CHOL_NB x CHOL_NB diagonal blocks of L1 into X (real positive diagonal): lane j
// solves column j by forward substitution.  Grid (blocks, nprob), one wave.
__global__ __launch_bounds__(64) void chol_diag_inv_kernel(int n, double2 *ws) {
  __shared__ double2 ls[CHOL_NB][CHOL_NB + 1], xs[CHOL_NB][CHOL_NB + 1];
  const int blk = blockIdx.x, prob = blockIdx.y, lane = threadIdx.x;
  const int i0 = blk * CHOL_NB, b = min(CHOL_NB, n - i0);
  double2 *L1 = ws + (size_t)prob * chol_stride(n), *X = L1 + 2 * (size_t)n * n;
  for (int idx = lane; idx < b * b; idx += 64) {
    const int i = idx / b, m = idx % b;
    ls[i][m] = L1[(size_t)(i0 + i) * n + i0 + m];
  }
  __syncthreads();
  if (lane < b) {
    const int j = lane;
    for (int i = j; i < b; ++i) {
      double sr = i == j ? 1.0 : 0.0, si = 0.0;
      for (int m = j; m < i; ++m) {
        const double2 a = ls[i][m], x = xs[m][j];
        sr -= a.x * x.x - a.y * x.y;
        si -= a.x * x.y + a.y * x.x;
      }
      const double inv = 1.0 / ls[i][i].x;
      xs[i][j] = make_double2(sr * inv, si * inv);
    }
    for (int i = j; i < b; ++i) X[(size_t)(i0 + i) * n + i0 + j] = xs[i][j];
  }
}

// Outputs from L, X = L1^{-1} and the pivot order: R = L^H P^T (rows beyond the rank zero) and
// Wsc[perm[kk]][k] = conj(X[k][kk]) for k, kk < rank.
__global__ __launch_bounds__(1024) void chol_out_kernel(int n, double *const *R, double *const *Wsc,
                                                        const double2 *ws, const char *meta) {
  __shared__ int perm[512];
  const int prob = blockIdx.x, tid = threadIdx.x, nt = blockDim.x;
  const double2 *L = ws + (size_t)prob * chol_stride(n) + (size_t)n * n, *X = L + (size_t)n * n;
  const char *mb = meta + (size_t)prob * chol_meta_bytes(n);
  const int r = reinterpret_cast<const int *>(mb)[0];
  for (int i = tid; i < n; i += nt) perm[i] = reinterpret_cast<const int *>(mb + 16 + (size_t)n * 8)[i];
  __syncthreads();
  double2 *Ro = reinterpret_cast<double2 *>(R[prob]);
  double2 *Wo = reinterpret_cast<double2 *>(Wsc[prob]);
  for (int idx = tid; idx < n * n; idx += nt) {
    const int k = idx / n, c = idx % n;
    const double2 l = L[(size_t)c * n + k];
    gst(Ro, idx, k < r ? make_double2(l.x, -l.y) : make_double2(0.0, 0.0));
    gst(Wo, idx, make_double2(0.0, 0.0));
  }
  __syncthreads();
  for (int idx = tid; idx < r * r; idx += nt) {
    const int kk = idx / r, k = idx % r;
    const double2 x = X[(size_t)k * n + kk];
    gst(Wo, (long)perm[kk] * n + k, make_double2(x.x, -x.y));
  }
}

// The same factorisation for n <= 128 with the Gram matrix packed (lower triangle, physical
// indices) in LDS: pivoting permutes logical indices only, each rank-one update touches the
// remaining triangle, and X = L1^{-1} is formed in the LDS that held G.  L goes to the workspace.
__global__ __launch_bounds__(1024) void gram_chol_lds_kernel(int n, const double *const *G,
                                                             double *const *R,
                                                             double *const *Wsc, double cut,
                                                             double2 *ws) {
  extern __shared__ double2 smem[];
  __shared__ int perm[128];
  __shared__ double dg[128];
  __shared__ double2 lk[128];
  __shared__ double2 lrow_s[2 * 128];
  __shared__ int piv_s, rank_s;
  __shared__ double gmax_s;
  const int prob = blockIdx.x, tid = threadIdx.x, nt = blockDim.x;
  const int lane = tid & 63, wave = tid >> 6, nw = nt >> 6;
  double2 *L = ws + (size_t)prob * n * n;
  double2 *P = smem;
  const double2 *g = reinterpret_cast<const double2 *>(G[prob]);
  for (int i = wave; i < n; i += nw)
    for (int j = lane; j <= i; j += 64) {
      const double2 a = gld(g, (long)i * n + j), b = gld(g, (long)j * n + i);
      P[pk_idx(i, j)] = make_double2(0.5 * (a.x + b.x), i == j ? 0.0 : 0.5 * (a.y - b.y));
    }
  for (int idx = tid; idx < n * n; idx += nt) L[idx] = make_double2(0.0, 0.0);
  for (int i = tid; i < n; i += nt) {
    perm[i] = i;
    dg[i] = gld(g, (long)i * n + i).x;
  }
  __syncthreads();
  if (wave == 0) {
    double m = 0;
    for (int i = lane; i < n; i += 64) m = fmax(m, dg[i]);
    m = wave_max(m);
    if (lane == 0) {
      gmax_s = m;
      rank_s = n;
    }
  }
  __syncthreads();
  const double gmax = gmax_s;
  for (int k = 0; k < n; ++k) {
    if (wave == 0) {
      double best = -1.0;
      int bj = k;
      for (int j = k + lane; j < n; j += 64) {
        const double v = dg[perm[j]];
        if (v > best) { best = v; bj = j; }
      }
      wave_argmax(best, bj);
      if (lane == 0) {
        if (!(best > cut * gmax) || !(gmax > 0)) {
          rank_s = k;
          piv_s = -1;
        } else {
          const int t = perm[k];
          perm[k] = perm[bj];
          perm[bj] = t;
          piv_s = bj;
        }
      }
    }
    __syncthreads();
    if (piv_s < 0) break;
    const int pkk = perm[k];
    const double piv = sqrt(dg[pkk]);
    for (int kk = k + 1 + tid; kk < n; kk += nt) {
      const int i = perm[kk];
      const double2 w = i >= pkk ? P[pk_idx(i, pkk)] : cconj(P[pk_idx(pkk, i)]);
      const double2 l = make_double2(w.x / piv, w.y / piv);
      L[(size_t)i * n + k] = l;
      lk[i] = l;
    }
    if (tid == 0) L[(size_t)pkk * n + k] = make_double2(piv, 0.0);
    __syncthreads();
    // W[i][j] -= L[i][k] conj(L[j][k]) over the remaining logical pairs (row >= col)
    const int m = n - k - 1;
    for (int row = wave; row < m; row += nw) {
      const int i = perm[k + 1 + row];
      const double2 li = lk[i];
      for (int col = lane; col <= row; col += 64) {
        const int j = perm[k + 1 + col];
        const double2 lj = lk[j];
        if (i >= j) {
          double2 &w = P[pk_idx(i, j)];
          w = make_double2(w.x - (li.x * lj.x + li.y * lj.y), w.y - (li.y * lj.x - li.x * lj.y));
          if (i == j) dg[i] = w.x;
        } else {
          double2 &w = P[pk_idx(j, i)];
          w = make_double2(w.x - (lj.x * li.x + lj.y * li.y), w.y - (lj.y * li.x - lj.x * li.y));
        }
      }
    }
    __syncthreads();
  }
  const int r = rank_s;
  __syncthreads();
  // X = L1^{-1} (L1[i][m] = L[perm[i]][m], i, m < r), rows in turn, X packed in LDS.  Row i of
  // L1 is staged in LDS (double buffered: row i+1 is fetched while row i is solved).
  double2 *X = P;
  double2(*lrow)[128] = reinterpret_cast<double2(*)[128]>(lrow_s);
  if (r > 0 && tid == 0) lrow[0][0] = L[(size_t)perm[0] * n];
  __syncthreads();
  for (int i = 0; i < r; ++i) {
    const double2 *Li = lrow[i & 1];
    const bool fetch = i + 1 < r && tid <= i + 1;
    double2 nxt = make_double2(0.0, 0.0);
    if (fetch) nxt = L[(size_t)perm[i + 1] * n + tid];
    const double inv = 1.0 / Li[i].x;
    const int q = tid & 7;
    for (int j = tid >> 3; j <= i; j += nt >> 3) {
      double sr = 0.0, si = 0.0;
      for (int mm = j + q; mm < i; mm += 8) {
        const double2 a = Li[mm], x = X[pk_idx(mm, j)];
        sr += a.x * x.x - a.y * x.y;
        si += a.x * x.y + a.y * x.x;
      }
      sr = oct_sum(sr);
      si = oct_sum(si);
      if (q == 0) X[pk_idx(i, j)] = make_double2(((i == j ? 1.0 : 0.0) - sr) * inv, -si * inv);
    }
    if (fetch) lrow[(i + 1) & 1][tid] = nxt;
    __syncthreads();
  }
  double2 *Ro = reinterpret_cast<double2 *>(R[prob]);
  double2 *Wo = reinterpret_cast<double2 *>(Wsc[prob]);
  for (int idx = tid; idx < n * n; idx += nt) {
    const int k = idx / n, c = idx % n;
    const double2 l = L[(size_t)c * n + k];
    gst(Ro, idx, k < r ? make_double2(l.x, -l.y) : make_double2(0.0, 0.0));
    gst(Wo, idx, make_double2(0.0, 0.0));
  }
  __syncthreads();
  for (int idx = tid; idx < r * r; idx += nt) {
    const int kk = idx / r, k = idx % r;     // Wsc[perm[kk]][k] = conj(X[k][kk]), kk <= k
    if (kk > k) continue;
    const double2 x = X[pk_idx(k, kk)];
    gst(Wo, (long)perm[kk] * n + k, make_double2(x.x, -x.y));
  }
}

// ------------------------------------------------------------------------------------------
// small kernels

__global__ void rx_kernel(double *const *T, const int64_t *half, double c, double s) {
  double2 *t = reinterpret_cast<double2 *>(T[blockIdx.y]);
  int64_t h = half[blockIdx.y];
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < h;
       i += (int64_t)gridDim.x * blockDim.x) {
    double2 a = gld(t, i), b = gld(t, h + i);
    // [c, -is; -is, c]
    gst(t, i, make_double2(c * a.x + s * b.y, c * a.y - s * b.x));
    gst(t, h + i, make_double2(s * a.y + c * b.x, -s * a.x + c * b.y));
  }
}

// X = W f(l) W^H and Xp = W g(l) W^H with f = sqrt(max(l, 0)) and g = 1/sqrt(l) above the cutoff
// (0 below); f and g are formed once per message in LDS.  n <= 128.
__global__ __launch_bounds__(256) void msg_sqrt_kernel(int n, const double *const *evals,
                                                       const double *const *vecs,
                                                       double *const *X, double *const *Xp,
                                                       double cut) {
  __shared__ double fs[128], gs[128];
  const double *l = evals[blockIdx.x];
  const double2 *W = reinterpret_cast<const double2 *>(vecs[blockIdx.x]);
  double2 *x = reinterpret_cast<double2 *>(X[blockIdx.x]);
  double2 *xp = reinterpret_cast<double2 *>(Xp[blockIdx.x]);
  const double l0 = gld(l, 0), lmax = l0 > 0 ? l0 : 0.0;
  for (int k = threadIdx.x; k < n; k += blockDim.x) {
    const double lk = gld(l, k);
    fs[k] = lk > 0 ? sqrt(lk) : 0.0;
    gs[k] = (lk > cut * lmax && lk > 0) ? 1.0 / sqrt(lk) : 0.0;
  }
  __syncthreads();
  for (int idx = threadIdx.x; idx < n * n; idx += blockDim.x) {
    const int i = idx / n, j = idx % n;
    const double2 *wi = W + (size_t)i * n, *wj = W + (size_t)j * n;
    double sr = 0, si = 0, pr = 0, pi = 0;
    for (int k = 0; k < n; ++k) {
      const double2 a = gld(wi, k), b = gld(wj, k);
      // a * conj(b)
      const double re = a.x * b.x + a.y * b.y, im = a.y * b.x - a.x * b.y;
      const double f = fs[k], g = gs[k];
      sr += f * re;
      si += f * im;
      pr += g * re;
      pi += g * im;
    }
    gst(x, idx, make_double2(sr, si));
    gst(xp, idx, make_double2(pr, pi));
  }
}

// Theta <- g(s_B, s_S) Theta in place, rows (r_B, s_B), columns (r_S, s_S).
__global__ void theta_phase_kernel(int rB, int rS, double *const *Th, double gsr, double gsi,
                                   double gdr, double gdi) {
  double2 *t = reinterpret_cast<double2 *>(Th[blockIdx.y]);
  const int cols = 2 * rS, tot = 2 * rB * cols;
  for (int idx = blockIdx.x * blockDim.x + threadIdx.x; idx < tot; idx += gridDim.x * blockDim.x) {
    const int row = idx / cols, col = idx - row * cols;
    const bool same = (row & 1) == (col & 1);
    const double gr = same ? gsr : gdr, gi = same ? gsi : gdi;
    const double2 v = gld(t, idx);
    gst(t, idx, make_double2(gr * v.x - gi * v.y, gr * v.y + gi * v.x));
  }
}

__global__ void svd_finish_kernel(int n, int chi, const double *const *evals,
                                  const double *const *vecs, double *const *Vs, double *const *S,
                                  int *kout, double *disc, double *const *mA, double *const *mB,
                                  double cutoff) {
  __shared__ double sig[512], l[512];      // the eigenvalues staged in LDS for the serial scan
  __shared__ int ks;
  __shared__ double nrm, ssum;
  const int p = blockIdx.x;
  const double *lg = evals[p];
  for (int i = threadIdx.x; i < n; i += blockDim.x) {
    l[i] = gld(lg, i);
    sig[i] = sqrt(fmax(l[i], 0.0));
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    // Keep min(chi, #{lambda_i > cutoff * lambda_1}): the cutoff acts on the Schmidt weights
    // lambda = sigma^2, which the FP64 eigenvalues of Theta^H Theta resolve to ~eps * lambda_1
    // (sigma itself only to ~sqrt(eps) * sigma_1).
    const double l0 = fmax(l[0], 0.0);
    int above = 0;
    for (int i = 0; i < n; ++i)
      if (fmax(l[i], 0.0) > cutoff * l0) ++above;
    const int k = above < chi ? above : chi;
    double tot = 0, kept = 0, sum = 0;
    for (int i = 0; i < n; ++i) tot += sig[i] * sig[i];
    for (int i = 0; i < k; ++i) kept += sig[i] * sig[i];
    double nr = sqrt(kept);
    for (int i = 0; i < k; ++i) sum += sig[i] / nr;
    ks = k;
    nrm = nr;
    ssum = sum;
    kout[p] = k;
    disc[2 * p] = tot > 0 ? (tot - kept) / tot : 0.0;
    // gap of a chi-limited cut relative to sigma_1 (infinite when the cutoff set k)
    disc[2 * p + 1] = (above > k && k > 0 && sig[0] > 0.0) ? (sig[k - 1] - sig[k]) / sig[0]
                                                           : INFINITY;
  }
  __syncthreads();
  const int k = ks;
  double *Sp = S[p];
  for (int a = threadIdx.x; a < chi; a += blockDim.x) gst(Sp, a, a < k ? sig[a] / nrm : 0.0);
  const double2 *V = reinterpret_cast<const double2 *>(vecs[p]);
  double2 *vs = reinterpret_cast<double2 *>(Vs[p]);
  for (int idx = threadIdx.x; idx < n * chi; idx += blockDim.x) {
    int c = idx / chi, a = idx % chi;
    double2 v = make_double2(0.0, 0.0);
    if (a < k) { double2 w = gld(V, (long)c * n + a); v = make_double2(w.x / sig[a], w.y / sig[a]); }
    gst(vs, idx, v);
  }
  double2 *ma = reinterpret_cast<double2 *>(mA[p]);
  double2 *mb = reinterpret_cast<double2 *>(mB[p]);
  for (int idx = threadIdx.x; idx < chi * chi; idx += blockDim.x) {
    int i = idx / chi, j = idx % chi;
    double v = (i == j && i < k) ? (sig[i] / nrm) / ssum : 0.0;
    gst(ma, idx, make_double2(v, 0.0));
    gst(mb, idx, make_double2(v, 0.0));
  }
}

__global__ __launch_bounds__(256) void to_f32_kernel(const double2 *src, float2 *dst, size_t n) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n;
       i += (size_t)gridDim.x * blockDim.x) {
    const double2 v = src[i];
    dst[i] = make_float2((float)v.x, (float)v.y);
  }
}

__global__ void split_sqrt_kernel(int rowsB, int rowsS, int n, int chi, const double *const *U,
                                  const double *const *V, const double *const *S,
                                  double *const *RBn, double *const *RSn) {
  const int p = blockIdx.y;
  const double *s = S[p];
  const double2 *u = reinterpret_cast<const double2 *>(U[p]);
  const double2 *v = reinterpret_cast<const double2 *>(V[p]);
  double2 *rb = reinterpret_cast<double2 *>(RBn[p]);
  double2 *rs = reinterpret_cast<double2 *>(RSn[p]);
  int totB = rowsB * chi, totS = rowsS * chi;
  for (int idx = blockIdx.x * blockDim.x + threadIdx.x; idx < totB + totS;
       idx += gridDim.x * blockDim.x) {
    if (idx < totB) {
      int a = idx % chi;
      double q = sqrt(gld(s, a));
      double2 x = gld(u, idx);
      gst(rb, idx, make_double2(q * x.x, q * x.y));
    } else {
      int j = idx - totB;
      int row = j / chi, a = j % chi;
      double2 o = make_double2(0.0, 0.0);
      if (a < n) {
        double q = sqrt(gld(s, a));
        double2 x = gld(v, (long)row * n + a);
        o = make_double2(q * x.x, -q * x.y);
      }
      gst(rs, j, o);
    }
  }
}

template <int NT>
__device__ double block_sum(double v, double *sh) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
  int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  if (l == 0) sh[w] = v;
  __syncthreads();
  double r = 0;
  if (threadIdx.x == 0)
    for (int i = 0; i < NT / 64; ++i) r += sh[i];
  __syncthreads();
  return r;   // valid on thread 0
}

// Message p: divide by its complex trace, then the residual |new - old|_F.  256 threads, wave sums
// by DPP, the four waves' sums added in a fixed order (two barriers in all).
__global__ __launch_bounds__(256) void normalize_residual_kernel(int chi, double *const *Mn,
                                                                const double *const *Mo,
                                                                double *res) {
  __shared__ double sh[3][4];
  const int p = blockIdx.x, tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  double2 *m = reinterpret_cast<double2 *>(Mn[p]);
  const double2 *o = reinterpret_cast<const double2 *>(Mo[p]);
  double tr = 0, ti = 0;
  for (int i = tid; i < chi; i += 256) {
    const double2 v = gld(m, (long)i * chi + i);
    tr += v.x;
    ti += v.y;
  }
  tr = wave_sum(tr);
  ti = wave_sum(ti);
  if (lane == 0) {
    sh[0][w] = tr;
    sh[1][w] = ti;
  }
  __syncthreads();
  const double trr = (sh[0][0] + sh[0][1]) + (sh[0][2] + sh[0][3]);
  const double tri = (sh[1][0] + sh[1][1]) + (sh[1][2] + sh[1][3]);
  const double den = trr * trr + tri * tri;
  const double ir = trr / den, ii = -tri / den;   // 1/tr
  double acc = 0;
#pragma unroll 4
  for (int idx = tid; idx < chi * chi; idx += 256) {
    const double2 v = gld(m, idx), q = gld(o, idx);
    const double2 nw = make_double2(v.x * ir - v.y * ii, v.x * ii + v.y * ir);
    gst(m, idx, nw);
    const double dx = nw.x - q.x, dy = nw.y - q.y;
    acc += dx * dx + dy * dy;
  }
  acc = wave_sum(acc);
  if (lane == 0) sh[2][w] = acc;
  __syncthreads();
  if (tid == 0) {
    const double sq = (sh[2][0] + sh[2][1]) + (sh[2][2] + sh[2][3]);
    res[p] = (trr > 0 && isfinite(sq)) ? sqrt(sq) : INFINITY;
  }
}

// For n > 64 the two products of msg_sqrt_kernel run on the GEMM: this kernel forms
// Wf = W diag(f) and Wg = W diag(g) (f, g as above) into a work area (2 n^2 per message, message p
// at ws + 2 p n^2) and the pointer arrays of the three operands; then X = Wf W^H, Xp = Wg W^H.
__global__ __launch_bounds__(256) void sqrt_scale_kernel(int n, const double *const *evals,
                                                         const double *const *vecs, double cut,
                                                         double2 *ws, double **pf, double **pg) {
  __shared__ double fs[256], gs[256];
  const int p = blockIdx.x;
  const double *l = evals[p];
  const double2 *W = reinterpret_cast<const double2 *>(vecs[p]);
  double2 *wf = ws + (size_t)p * 2 * n * n, *wg = wf + (size_t)n * n;
  const double l0 = gld(l, 0), lmax = l0 > 0 ? l0 : 0.0;
  for (int k = threadIdx.x; k < n; k += blockDim.x) {
    const double lk = gld(l, k);
    fs[k] = lk > 0 ? sqrt(lk) : 0.0;
    gs[k] = (lk > cut * lmax && lk > 0) ? 1.0 / sqrt(lk) : 0.0;
  }
  __syncthreads();
  for (int idx = threadIdx.x; idx < n * n; idx += blockDim.x) {
    const int k = idx % n;
    const double2 w = gld(W, idx);
    wf[idx] = make_double2(w.x * fs[k], w.y * fs[k]);
    wg[idx] = make_double2(w.x * gs[k], w.y * gs[k]);
  }
  if (threadIdx.x == 0) {
    pf[p] = reinterpret_cast<double *>(wf);
    pg[p] = reinterpret_cast<double *>(wg);
  }
}

// Bond entanglement entropy (Eq. "EntanglementEntropy", with the minus sign and the sum over the
// chi weights of one bond): the eigenvalues of the bond matrix X M^T X, clipped at zero and
// normalised to unit sum, give the Schmidt weights p; s = -sum p log2 p.  One workgroup per bond.
__global__ __launch_bounds__(256) void bond_entropy_kernel(int n, const double *const *evals,
                                                           double *out) {
  __shared__ double sh[4];
  __shared__ double tot;
  const double *l = evals[blockIdx.x];
  double acc = 0.0;
  for (int i = threadIdx.x; i < n; i += 256) acc += fmax(l[i], 0.0);
  const double t = block_sum<256>(acc, sh);
  if (threadIdx.x == 0) tot = t;
  __syncthreads();
  const double inv = tot > 0.0 ? 1.0 / tot : 0.0;
  acc = 0.0;
  for (int i = threadIdx.x; i < n; i += 256) {
    const double q = fmax(l[i], 0.0) * inv;
    if (q > 0.0) acc -= q * log2(q);
  }
  const double e = block_sum<256>(acc, sh);
  if (threadIdx.x == 0) out[blockIdx.x] = tot > 0.0 && isfinite(e) ? e : NAN;
}

// Symmetric Vidal gauge (Methods, "The Vidal gauge"), one workgroup per edge (u, v) with
// C = X^T Y, X and Y the square roots of the two messages on the edge.  From the eigenpairs
// (l_i descending, columns of V) of C^H C the singular values are lambda_i = sqrt(l_i); those
// above cut * lambda_1 are kept and normalised to unit 2-norm (s_i), the rest dropped.  With
// w_i = (s_i / sum s)^{1/2}, writes D1 = V diag(w_i / lambda_i) (so C D1 = U W),
// D2 = conj(V) diag(w_i), the BP fixed point diag(s) / sum(s) into both messages of the edge,
// s (zero-padded) and the kept count.  n <= 256.
__global__ __launch_bounds__(256) void vidal_svd_kernel(int n, const double *const *evals,
                                                        const double *const *vecs,
                                                        double *const *D1, double *const *D2,
                                                        double *const *Mu, double *const *Mv,
                                                        double *lam, int *kept, double cut) {
  __shared__ double sv[256], f1[256], f2[256];
  __shared__ double sh[4];
  __shared__ double nrm_s, sum_s, cnt_s;
  const int e = blockIdx.x, tid = threadIdx.x;
  const double *l = evals[e];
  const double l0 = sqrt(fmax(l[0], 0.0));
  double acc = 0.0, cnt = 0.0;
  for (int i = tid; i < n; i += 256) {
    const double li = sqrt(fmax(l[i], 0.0));
    const bool keep = li > 0.0 && li * li > cut * l0 * l0;    // cutoff on the Schmidt weights
    sv[i] = keep ? li : 0.0;
    acc += keep ? li * li : 0.0;
    cnt += keep ? 1.0 : 0.0;
  }
  const double t = block_sum<256>(acc, sh);
  const double c = block_sum<256>(cnt, sh);
  if (tid == 0) {
    nrm_s = sqrt(t);
    cnt_s = c;
  }
  __syncthreads();
  const double inv = nrm_s > 0.0 ? 1.0 / nrm_s : 0.0;
  acc = 0.0;
  for (int i = tid; i < n; i += 256) {
    const double si = sv[i] * inv;
    lam[(size_t)e * n + i] = si;
    acc += si;
  }
  const double ss = block_sum<256>(acc, sh);
  if (tid == 0) sum_s = ss;
  __syncthreads();
  const double isum = sum_s > 0.0 ? 1.0 / sum_s : 0.0;
  // W = (S / sum S)^{1/2}, the root of the new unit-trace message: a state already in this gauge
  // gets P = 1 (idempotent, scale kept)
  for (int i = tid; i < n; i += 256) {
    const double wi = sqrt(sv[i] * inv * isum);
    f1[i] = sv[i] > 0.0 ? wi / sv[i] : 0.0;
    f2[i] = wi;
  }
  __syncthreads();
  const double2 *V = reinterpret_cast<const double2 *>(vecs[e]);
  double2 *d1 = reinterpret_cast<double2 *>(D1[e]), *d2 = reinterpret_cast<double2 *>(D2[e]);
  double2 *mu = reinterpret_cast<double2 *>(Mu[e]), *mv = reinterpret_cast<double2 *>(Mv[e]);
  for (int idx = tid; idx < n * n; idx += 256) {
    const int r = idx / n, q = idx % n;
    const double2 w = V[idx];                  // component r of eigenvector q
    d1[idx] = make_double2(w.x * f1[q], w.y * f1[q]);
    d2[idx] = make_double2(w.x * f2[q], -w.y * f2[q]);
    const double2 m = make_double2(r == q ? sv[q] * inv * isum : 0.0, 0.0);
    mu[idx] = m;
    mv[idx] = m;
  }
  if (tid == 0) kept[e] = (int)cnt_s;
}

// Trace of an n x n complex matrix: out = (Re, Im).  One workgroup.
__global__ __launch_bounds__(256) void trace_kernel(const double *R, int n, double *out) {
  __shared__ double sh[4];
  const double2 *r = reinterpret_cast<const double2 *>(R);
  double re = 0.0, im = 0.0;
  for (int i = threadIdx.x; i < n; i += 256) {
    const double2 v = r[(size_t)i * n + i];
    re += v.x;
    im += v.y;
  }
  const double a = block_sum<256>(re, sh);
  const double b = block_sum<256>(im, sh);
  if (threadIdx.x == 0) {
    out[0] = a;
    out[1] = b;
  }
}

__global__ __launch_bounds__(256) void reduce_max_kernel(const double *x, int n, double *out) {
  __shared__ double sh[256];
  double m = 0;
  for (int i = threadIdx.x; i < n; i += blockDim.x) {
    double v = x[i];
    m = (v > m || v != v) ? v : m;
  }
  sh[threadIdx.x] = m;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (threadIdx.x < s) {
      double a = sh[threadIdx.x], b = sh[threadIdx.x + s];
      sh[threadIdx.x] = (b > a || b != b) ? b : a;
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] = sh[0];
}

// Packed solves: one workgroup per member takes the max (NaN-propagating) of its residual slots
// and clears the member's active flag for the next sweep once the max is below tol.
__global__ __launch_bounds__(256) void member_residual_kernel(const double *res, const int *off,
                                                              const int *idx, const int *act,
                                                              int *act_next, double tol,
                                                              double *out) {
  __shared__ double sh[256];
  const int j = blockIdx.x;
  double m = 0;
  for (int k = off[j] + threadIdx.x; k < off[j + 1]; k += blockDim.x) {
    double v = res[idx[k]];
    m = (v > m || v != v) ? v : m;
  }
  sh[threadIdx.x] = m;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (threadIdx.x < s) {
      double a = sh[threadIdx.x], b = sh[threadIdx.x + s];
      sh[threadIdx.x] = (b > a || b != b) ? b : a;
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    out[j] = sh[0];
    act_next[j] = act[j] && !(sh[0] < tol);
  }
}

// M[m] <- Mn[m] for the messages of active members (elems complex per message).
__global__ __launch_bounds__(256) void commit_messages_kernel(double2 *M, const double2 *Mn,
                                                              long elems, long total,
                                                              const int *msg_member,
                                                              const int *act) {
  for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < total;
       i += (long)gridDim.x * blockDim.x)
    if (act[msg_member[i / elems]]) M[i] = Mn[i];
}

// rho[p][s][s'] = sum_i Y_p[s][i] conj(T_p[s'][i]): RHO_CHUNKS workgroups per problem each sum a
// strided part into partial[p][chunk][8]; rho_sum_kernel adds the chunks in a fixed order.
constexpr int RHO_CHUNKS = 64;
__global__ __launch_bounds__(256) void rho_dot_kernel(const double *const *Y,
                                                      const double *const *T, const int64_t *len,
                                                      double *partial) {
  __shared__ double sh[8];
  const int p = blockIdx.y;
  const double2 *y = reinterpret_cast<const double2 *>(Y[p]);
  const double2 *t = reinterpret_cast<const double2 *>(T[p]);
  const int64_t L = len[p];
  double acc[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < L;
       i += (int64_t)gridDim.x * blockDim.x) {
    const double2 y0 = gld(y, i), y1 = gld(y, L + i), t0 = gld(t, i), t1 = gld(t, L + i);
    // y_s * conj(t_s')
    acc[0] += y0.x * t0.x + y0.y * t0.y; acc[1] += y0.y * t0.x - y0.x * t0.y;
    acc[2] += y0.x * t1.x + y0.y * t1.y; acc[3] += y0.y * t1.x - y0.x * t1.y;
    acc[4] += y1.x * t0.x + y1.y * t0.y; acc[5] += y1.y * t0.x - y1.x * t0.y;
    acc[6] += y1.x * t1.x + y1.y * t1.y; acc[7] += y1.y * t1.x - y1.x * t1.y;
  }
  for (int k = 0; k < 8; ++k) {
    const double s = block_sum<256>(acc[k], sh);
    if (threadIdx.x == 0) partial[((size_t)p * gridDim.x + blockIdx.x) * 8 + k] = s;
  }
}

__global__ void rho_sum_kernel(const double *partial, int chunks, int nprob, double *rho) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= nprob * 8) return;
  const int p = idx / 8, k = idx % 8;
  double s = 0.0;
  for (int c = 0; c < chunks; ++c) s += partial[((size_t)p * chunks + c) * 8 + k];
  rho[idx] = s;
}

__global__ void apply_op_kernel(const double *const *Tin, double *const *Tout,
                                const int64_t *half, const double *ops) {
  const int p = blockIdx.y;
  const double2 *t = reinterpret_cast<const double2 *>(Tin[p]);
  double2 *o = reinterpret_cast<double2 *>(Tout[p]);
  int64_t h = half[p];
  const double2 *O = reinterpret_cast<const double2 *>(ops) + 4 * p;
  double2 o00 = O[0], o01 = O[1], o10 = O[2], o11 = O[3];
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < h;
       i += (int64_t)gridDim.x * blockDim.x) {
    double2 a = t[i], b = t[h + i];
    o[i] = cadd(cmul(o00, a), cmul(o01, b));
    o[h + i] = cadd(cmul(o10, a), cmul(o11, b));
  }
}

// ------------------------------------------------------------------------------------------

class HipBackend : public Backend {
 public:
  HipBackend(int device, void *stream) : dev_(device) {
    HIPCHK(hipSetDevice(device));
    if (stream) {
      s_ = (hipStream_t)stream;
      own_ = false;
    } else {
      HIPCHK(hipStreamCreateWithFlags(&s_, hipStreamNonBlocking));
      own_ = true;
    }
    int cus = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device) == hipSuccess &&
        cus > 0)
      resident_ = 2 * cus;
    else
      (void)hipGetLastError();
    if (hipHostMalloc(&pin_, kPinBytes, hipHostMallocDefault) != hipSuccess) {
      pin_ = nullptr;            // small reads then take the staged path
      (void)hipGetLastError();
    }
    HIPCHK(hipFuncSetAttribute((const void *)eigh_jacobi_kernel,
                               hipFuncAttributeMaxDynamicSharedMemorySize, 140 * 1024));
    HIPCHK(hipFuncSetAttribute((const void *)gram_chol_lds_kernel,
                               hipFuncAttributeMaxDynamicSharedMemorySize, 132096));
    HIPCHK(hipFuncSetAttribute((const void *)chol_panel_kernel,
                               hipFuncAttributeMaxDynamicSharedMemorySize,
                               512 * (CHOL_NB + 1) * (int)sizeof(double2)));
    HIPCHK(hipFuncSetAttribute((const void *)eigh_tridiag_kernel<128, 1024>,
                               hipFuncAttributeMaxDynamicSharedMemorySize, 132096));
    HIPCHK(hipFuncSetAttribute((const void *)eigh_dc_kernel<128>,
                               hipFuncAttributeMaxDynamicSharedMemorySize, 132096));
  }
  ~HipBackend() override {
    for (auto &e : ev_)
      if (e) hipEventDestroy(e);
    for (auto &e : rd_ev_)
      if (e) hipEventDestroy(e);
    if (skws_) HIPCHK(dfree(skws_));
    if (cws_) HIPCHK(dfree(cws_));
    if (cmeta_) HIPCHK(dfree(cmeta_));
    if (sqws_) HIPCHK(dfree(sqws_));
    if (tptr_) HIPCHK(dfree(tptr_));
    if (lws_) HIPCHK(dfree(lws_));
    if (rws_) HIPCHK(dfree(rws_));
    if (pin_) HIPCHK(hipHostFree(pin_));
    if (own_) hipStreamDestroy(s_);
  }
  int set_allocator(DevAlloc a, DevFree f, void *user) override {
    if (touched_ || !a != !f) return -1;
    ua_ = a;
    uf_ = f;
    uu_ = user;
    return 0;
  }
  // Device memory from hipMalloc, or from the caller's allocator: asked for memory used on this
  // backend's stream, which must come 256-byte aligned as hipMalloc's does (correctness needs the
  // 16 bytes of a complex double; the rest keeps a tile row's loads within whole cache lines).
  hipError_t dmalloc(void **p, size_t bytes) {
    touched_ = true;
    if (!ua_) return hipMalloc(p, bytes);
    *p = ua_(bytes, (void *)s_, uu_);
    if (*p && ((uintptr_t)*p & 255)) {
      uf_(*p, (void *)s_, uu_);
      *p = nullptr;
      if (err_ == 0) {
        err_ = -5;
        errmsg_ = "the device allocator returned memory not aligned to 256 bytes";
      }
    }
    return *p ? hipSuccess : hipErrorOutOfMemory;
  }
  // The caller's free runs after this stream has drained: the allocator may hand the memory to
  // other work at once.
  hipError_t dfree(void *p) {
    if (!uf_) return hipFree(p);
    hipError_t e = hipStreamSynchronize(s_);
    uf_(p, (void *)s_, uu_);
    return e;
  }
  // The cached workspaces are dropped without being freed (their memory belongs to an arena
  // that the caller resets); an allocation failure, unlike a device error, is cleared.
  void forget_workspaces() override {
    HIPCHK(hipStreamSynchronize(s_));
    skws_ = cws_ = cmeta_ = sqws_ = tptr_ = lws_ = rws_ = nullptr;
    skws_bytes_ = cws_bytes_ = cmeta_bytes_ = sqws_bytes_ = tptr_bytes_ = lws_bytes_ = rws_bytes_ = 0;
  }
  void clear_alloc_error() override {
    if (err_ == -4) {
      err_ = 0;
      errmsg_.clear();
    }
  }
  void *alloc(size_t bytes) override {
    void *p = nullptr;
    hipError_t e = dmalloc(&p, bytes);
    if (e != hipSuccess) {
      if (err_ == 0) { err_ = -4; errmsg_ = "device allocation failed (out of device memory)"; }
      return nullptr;
    }
    HIPCHK(hipMemsetAsync(p, 0, bytes, s_));
    return p;
  }
  void release(void *p) override {
    if (p) {
      HIPCHK(hipStreamSynchronize(s_));
      HIPCHK(dfree(p));
    }
  }
  // After an error (a failed allocation leaves null buffers behind) no copy is issued.
  void h2d(void *d, const void *h, size_t b) override {
    if (err_) return;
    if (b) HIPCHK(hipMemcpyAsync(d, h, b, hipMemcpyHostToDevice, s_));
    HIPCHK(hipStreamSynchronize(s_));
  }
  // Small reads (residuals, bond dimensions, site densities) go through a pinned buffer and a
  // polling wait on the stream: the host resumes as soon as the stream drains, which shortens
  // the bubble between BP sweeps.
  void d2h(void *h, const void *d, size_t b) override {
    if (err_) return;
    if (b && b <= kPinBytes - kPinAsync && pin_) {
      HIPCHK(hipMemcpyAsync(pin_, d, b, hipMemcpyDeviceToHost, s_));
      hipError_t e;
      while ((e = hipStreamQuery(s_)) == hipErrorNotReady) {
      }
      // a not-ready answer of the query may linger as the last error: clear it
      const hipError_t le = hipGetLastError();
      if (e != hipSuccess) HIPCHK(e);
      if (le != hipSuccess && le != hipErrorNotReady) HIPCHK(le);
      std::memcpy(h, pin_, b);
      return;
    }
    if (b) HIPCHK(hipMemcpyAsync(h, d, b, hipMemcpyDeviceToHost, s_));
    HIPCHK(hipStreamSynchronize(s_));
  }  // One double into slot 0 or 1 at the end of the pinned buffer, in stream order; wait_read spins on
  // the copy's event (the host resumes as soon as the stream reaches it).
  void read_async(const double *d, int slot) override {
    if (err_) return;
    double *h = pin_ ? (double *)((char *)pin_ + kPinBytes - kPinAsync) + (slot & 1) : nullptr;
    if (!h) {
      d2h(&rd_val_[slot & 1], d, 8);
      return;
    }
    if (!rd_ev_[slot & 1]) HIPCHK(hipEventCreateWithFlags(&rd_ev_[slot & 1], hipEventDisableTiming));
    HIPCHK(hipMemcpyAsync(h, d, 8, hipMemcpyDeviceToHost, s_));
    HIPCHK(hipEventRecord(rd_ev_[slot & 1], s_));
  }
  double wait_read(int slot) override {
    if (err_) return NAN;
    if (!pin_) return rd_val_[slot & 1];
    hipError_t e;
    while ((e = hipEventQuery(rd_ev_[slot & 1])) == hipErrorNotReady) {
    }
    const hipError_t le = hipGetLastError();
    if (e != hipSuccess) HIPCHK(e);
    if (le != hipSuccess && le != hipErrorNotReady) HIPCHK(le);
    return ((const double *)((const char *)pin_ + kPinBytes - kPinAsync))[slot & 1];
  }

  void d2d(void *d, const void *s, size_t b) override {
    if (err_) return;
    if (b) HIPCHK(hipMemcpyAsync(d, s, b, hipMemcpyDeviceToDevice, s_));
  }
  void sync() override { HIPCHK(hipStreamSynchronize(s_)); }
  int check(std::string *msg) override {
    HIPCHK(hipGetLastError());
    if (msg) *msg = errmsg_;
    return err_;
  }
  hipStream_t stream() const { return s_; }
  void stale_check(const char *where) {
    hipError_t e = hipGetLastError();
    if (e != hipSuccess && err_ == 0) {
      err_ = -5;
      errmsg_ = std::string("pending error before ") + where + ": " + hipGetErrorString(e);
    }
  }
  void launch_check(const char *name) {
    hipError_t e = hipGetLastError();
    if (e != hipSuccess && err_ == 0) {
      err_ = -5;
      errmsg_ = std::string("launch of ") + name + ": " + hipGetErrorString(e);
    }
  }
  void timer_mark(int slot) override {
    if (slot < 0 || slot >= 8) return;
    if (!ev_[slot]) HIPCHK(hipEventCreate(&ev_[slot]));
    HIPCHK(hipEventRecord(ev_[slot], s_));
  }
  double timer_ms(int a, int b) override {
    if (a < 0 || b < 0 || a >= 8 || b >= 8 || !ev_[a] || !ev_[b]) return 0.0;
    HIPCHK(hipEventSynchronize(ev_[b]));
    float ms = 0;
    HIPCHK(hipEventElapsedTime(&ms, ev_[a], ev_[b]));
    return ms;
  }

  void gemm(const GemmDesc &d, const double *const *A, const double *const *B, double *const *C,
            int nprob) override {
    if (nprob <= 0 || d.M <= 0 || d.N <= 0) return;
    int tiles = ((d.M + BM - 1) / BM) * ((d.N + BN - 1) / BN);
    dim3 grid(tiles, d.batch, nprob);
    hipEvent_t e0 = nullptr, e1 = nullptr;
    // K and N within 64 (one stride each) and enough rows to amortise loading B (at least 16
    // strips): B resident in LDS, rows of A streamed
    const bool stream = d.K <= SK_MAX && d.N <= SK_MAX && d.K == d.Ki && d.N == d.Ni &&
                        d.M >= 256 && !d.herm && !d.b32;
    const bool rec = prof_sample(stream ? 2 : 0, d.prec);
    if (rec) {
      HIPCHK(hipEventCreate(&e0));
      HIPCHK(hipEventCreate(&e1));
      HIPCHK(hipEventRecord(e0, s_));
    }
    // FP32 storage: an absorption into an FP32 buffer (A, C FP32; B FP64) or a closing into an
    // FP64 message (A, B FP32), in FP32 mode only
    const int st = (d.a32 ? 1 : 0) | (d.b32 ? 2 : 0) | (d.c32 ? 4 : 0);
    if (st && (d.prec != 1 || (st != 5 && st != 3))) {
      if (err_ == 0) {
        err_ = -1;
        errmsg_ = "gemm: unsupported combination of FP32 operand storage";
      }
      return;
    }
    if (stream) {
      const int strips = (d.M + 15) / 16;
      const int per = std::max(1, resident_ / std::max(1, d.batch * nprob));
      dim3 g(std::max(1, std::min(per, (strips + 3) / 4)), d.batch, nprob);
      const bool tr = d.c_mi == 1 && d.c_ni != 1;     // C is unit-stride along M
      stale_check("gemm_stream_kernel");
      // K = N = 64 (the leg contractions at chi = 64): loop bounds fixed at compile time
      const bool full = d.K == SK_MAX && d.N == SK_MAX;
#define GSK_LAUNCH(TT, TRV, S32)                                                                  \
  do {                                                                                            \
    if (full)                                                                                     \
      hipLaunchKernelGGL((gemm_stream_kernel<TT, TRV, S32, S32, true>), g, dim3(256), 0, s_, d, A, \
                         B, C);                                                                   \
    else                                                                                          \
      hipLaunchKernelGGL((gemm_stream_kernel<TT, TRV, S32, S32, false>), g, dim3(256), 0, s_, d,   \
                         A, B, C);                                                                \
  } while (0)
      if (d.prec == 1 && st == 5) {
        if (tr) GSK_LAUNCH(float, true, true);
        else GSK_LAUNCH(float, false, true);
      } else if (d.prec == 1) {
        if (tr) GSK_LAUNCH(float, true, false);
        else GSK_LAUNCH(float, false, false);
      } else {
        if (tr) GSK_LAUNCH(double, true, false);
        else GSK_LAUNCH(double, false, false);
      }
#undef GSK_LAUNCH
      launch_check("gemm_stream_kernel");
      if (rec) {
        HIPCHK(hipEventRecord(e1, s_));
        prof_ev_.push_back({e0, e1});
        const int q = 4 + (d.prec & 1);
        prof_prec_.push_back(q);
        prof_flops_ += 8.0 * d.M * d.N * (double)d.K * d.batch * nprob;
        prof_flops_p_[q] += 8.0 * d.M * d.N * (double)d.K * d.batch * nprob;
        prof_bytes_p_[q] += gemm_bytes(d, nprob);
      }
      return;
    }
    // split K when the output alone cannot fill the machine: as many chunks (of at least 32) as
    // keep the grid within one round of resident workgroups (two per CU; a partial second round
    // measured slower than fewer, longer chunks)
    int blocks = tiles * d.batch * nprob;
    int ksplit = 1, kchunk = d.K;
    if (blocks < resident_ && d.K >= 128) {
      int want = std::min(resident_ / blocks, d.K / 32);
      if (want > 1) {
        kchunk = ((d.K + want - 1) / want + BK - 1) / BK * BK;
        ksplit = (d.K + kchunk - 1) / kchunk;
      }
    }
    double2 *W = nullptr;
    if (ksplit > 1) {
      size_t need = (size_t)nprob * d.batch * ksplit * d.M * d.N * sizeof(double2);
      W = (double2 *)splitk_ws(need);
      if (!W) return;
      grid.y = d.batch * ksplit;
    }
    if (d.prec == 1) {
      stale_check("gemm_kernel<float>");
      if (st == 5) {
        if (d.herm)
          hipLaunchKernelGGL((gemm_kernel<float, true, true, false, true>), grid, dim3(256), 0, s_,
                             d, A, B, C, ksplit, kchunk, W);
        else
          hipLaunchKernelGGL((gemm_kernel<float, false, true, false, true>), grid, dim3(256), 0,
                             s_, d, A, B, C, ksplit, kchunk, W);
      } else if (st == 3) {
        if (d.herm)
          hipLaunchKernelGGL((gemm_kernel<float, true, true, true, false>), grid, dim3(256), 0, s_,
                             d, A, B, C, ksplit, kchunk, W);
        else
          hipLaunchKernelGGL((gemm_kernel<float, false, true, true, false>), grid, dim3(256), 0,
                             s_, d, A, B, C, ksplit, kchunk, W);
      } else if (d.herm) {
        hipLaunchKernelGGL((gemm_kernel<float, true>), grid, dim3(256), 0, s_, d, A, B, C, ksplit,
                           kchunk, W);
      } else {
        hipLaunchKernelGGL((gemm_kernel<float, false>), grid, dim3(256), 0, s_, d, A, B, C, ksplit,
                           kchunk, W);
      }
      launch_check("gemm_kernel<float>");
    } else {
      stale_check("gemm_kernel<double>");
      if (d.herm)
        hipLaunchKernelGGL((gemm_kernel<double, true>), grid, dim3(256), 0, s_, d, A, B, C, ksplit,
                           kchunk, W);
      else
        hipLaunchKernelGGL((gemm_kernel<double, false>), grid, dim3(256), 0, s_, d, A, B, C, ksplit,
                           kchunk, W);
      launch_check("gemm_kernel<double>");
    }
    if (rec) {
      HIPCHK(hipEventRecord(e1, s_));
      prof_ev_.push_back({e0, e1});
      const int q = d.prec & 1;
      prof_prec_.push_back(q);
      // algorithmic work: the distinct entries (a Hermitian output has M (M + 1) / 2)
      const double outs = d.herm ? 0.5 * d.M * (d.M + 1.0) : (double)d.M * d.N;
      prof_flops_ += 8.0 * outs * (double)d.K * d.batch * nprob;
      prof_flops_p_[q] += 8.0 * outs * (double)d.K * d.batch * nprob;
      prof_bytes_p_[q] += gemm_bytes(d, nprob);
    }
    if (ksplit > 1) {
      int bx = std::min(64, (int)((d.M * (size_t)d.N + 255) / 256));
      stale_check("gemm_reduce_kernel");
      if (d.c32)
        hipLaunchKernelGGL(gemm_reduce_kernel<true>, dim3(bx, d.batch, nprob), dim3(256), 0, s_, d,
                           C, ksplit, (const double2 *)W);
      else
        hipLaunchKernelGGL(gemm_reduce_kernel<false>, dim3(bx, d.batch, nprob), dim3(256), 0, s_,
                           d, C, ksplit, (const double2 *)W);
      launch_check("gemm_reduce_kernel");
    }
  }
  void bp_close(const BpCloseDesc &d, const double *const *Y, const double *const *T,
                const double *const *M, double *const *out, int nprob) override {
    if (nprob <= 0) return;
    bool bad = (d.chi != 64 && d.chi != 32) || (d.s32 && d.prec != 1) || d.ss < 0 ||
               (d.pair != 0 && d.pair != 1) ||
               d.nsets < 1 || d.nsets > 3 || d.group < 1 || (d.xdim != 1 && d.xdim != d.chi);
    for (int k = 0; k < 3 && !bad; ++k)
      bad = k < d.nsets && (d.rs[k] < 0 || d.qs[k] < 0 || d.cs[k] < 0);
    if (bad) {
      if (err_ == 0) {
        err_ = -1;
        errmsg_ = "bp_close: unsupported descriptor";
      }
      return;
    }
    // one round of resident workgroups (FP64 at chi 64: one per CU, otherwise two), each a
    // contiguous run of `per` chunks: a multiple of the G chunks in flight, and at most one
    // problem's 2 xdim (so a workgroup touches at most two problems)
    const int ch = d.chi, G = 64 / ch;
    const long J = 2L * d.xdim, total = J * nprob;
    if (total > INT_MAX - 256) {
      if (err_ == 0) {
        err_ = -1;
        errmsg_ = "bp_close: too many chunks in one call (2^31 - 257 at most)";
      }
      return;
    }
    const long slots =
        (d.prec == 0 && ch == 64 && !d.pair) ? std::max(1, resident_ / 2) : resident_;
    long per = std::max<long>(1, std::min(J, (total + slots - 1) / slots));
    per = (per + G - 1) / G * G;
    const int nwg = (int)((total + per - 1) / per);
    double2 *W = (double2 *)splitk_ws((size_t)nwg * 2 * G * ch * ch * sizeof(double2));
    if (!W) return;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    const bool rec = prof_sample(1, d.prec);
    if (rec) {
      HIPCHK(hipEventCreate(&e0));
      HIPCHK(hipEventCreate(&e1));
      HIPCHK(hipEventRecord(e0, s_));
    }
    stale_check("bp_close_kernel");
#define BPC_LAUNCH(TT, S, C, PR)                                                                  \
  hipLaunchKernelGGL((bp_close_kernel<TT, S, C, PR>), dim3(nwg), dim3(256), 0, s_, d, Y, T, M,     \
                     (int)total, (int)per, W)
#define BPC_PREC(C, PR)                                                                           \
  do {                                                                                            \
    if (d.prec == 1 && d.s32) BPC_LAUNCH(float, true, C, PR);                                    \
    else if (d.prec == 1) BPC_LAUNCH(float, false, C, PR);                                       \
    else BPC_LAUNCH(double, false, C, PR);                                                       \
  } while (0)
    if (ch == 64) {
      if (d.pair) BPC_PREC(64, true);
      else BPC_PREC(64, false);
    } else {
      if (d.pair) BPC_PREC(32, true);
      else BPC_PREC(32, false);
    }
#undef BPC_PREC
#undef BPC_LAUNCH
    launch_check("bp_close_kernel");
    if (rec) {
      HIPCHK(hipEventRecord(e1, s_));
      prof_ev_.push_back({e0, e1});
      const int q = 2 + (d.prec & 1);
      prof_prec_.push_back(q);
      // algorithmic work per message, per chunk (2 xdim of them): the absorption W = Y M (chi^3,
      // none for a pair) and the distinct entries of the Hermitian closing (chi (chi + 1) / 2 of
      // them, K = chi); a degree-3 site (xdim = chi): 2 chi^4 + chi^3 (chi + 1)
      const double c = ch;
      const double fl =
          8.0 * nprob * 2.0 * d.xdim * ((d.pair ? 0.0 : c * c * c) + 0.5 * c * c * (c + 1.0));
      prof_flops_ += fl;
      prof_flops_p_[q] += fl;
      // algorithmic bytes: both site-sized operands read once (Y and T, or the pair), M, out
      const double esz = d.s32 ? 8.0 : 16.0, cc = c * c;
      prof_bytes_p_[q] += nprob * (2.0 * 2.0 * d.xdim * cc * esz + (d.pair ? 0.0 : 16.0 * cc) +
                                   16.0 * cc);
    }
    stale_check("bp_close_reduce_kernel");
    hipLaunchKernelGGL(bp_close_reduce_kernel, dim3((ch * ch + 255) / 256, nprob), dim3(256), 0,
                       s_, ch, G, (int)per, (int)J, (const double2 *)W, out);
    launch_check("bp_close_reduce_kernel");
  }
  void *splitk_ws(size_t need) {
    if (need > skws_bytes_) {
      HIPCHK(hipStreamSynchronize(s_));
      if (skws_) HIPCHK(dfree(skws_));
      skws_ = nullptr;
      skws_bytes_ = 0;
      if (dmalloc(&skws_, need) != hipSuccess) {
        err_ = -4;
        errmsg_ = "split-K workspace allocation failed";
        return nullptr;
      }
      skws_bytes_ = need;
    }
    return skws_;
  }
  void gemm_profile(int stride) override {
    prof_stride_ = stride > 0 ? stride : 0;
    if (prof_stride_) {
      drain_profile();
      prof_launches_ = 0;
      prof_all_ = 0;
      for (int q = 0; q < kProfBuckets; ++q) prof_all_p_[q] = 0;
      prof_ms_ = 0;
      prof_flops_ = 0;
      for (int q = 0; q < kProfBuckets; ++q) {
        prof_launches_p_[q] = 0;
        prof_ms_p_[q] = prof_flops_p_[q] = prof_bytes_p_[q] = 0;
      }
    }
  }
  void gemm_profile_read(long *sampled, long *all, double *ms, double *flops) override {
    drain_profile();
    if (sampled) *sampled = prof_launches_;
    if (all) *all = prof_all_;
    if (ms) *ms = prof_ms_;
    if (flops) *flops = prof_flops_;
  }
  void gemm_profile_read_prec(int prec, long *sampled, double *ms, double *flops) override {
    drain_profile();
    long l = 0;
    double t = 0, f = 0;
    for (int k = 0; k < kProfBuckets / 2; ++k) {
      l += prof_launches_p_[2 * k + (prec & 1)];
      t += prof_ms_p_[2 * k + (prec & 1)];
      f += prof_flops_p_[2 * k + (prec & 1)];
    }
    if (sampled) *sampled = l;
    if (ms) *ms = t;
    if (flops) *flops = f;
  }
  void gemm_profile_read_kernel(int kernel, int prec, long *sampled, double *ms, double *flops,
                                double *bytes, long *all) override {
    drain_profile();
    const int q = 2 * kernel + (prec & 1);
    if (all) *all = prof_all_p_[q];
    if (sampled) *sampled = prof_launches_p_[q];
    if (ms) *ms = prof_ms_p_[q];
    if (flops) *flops = prof_flops_p_[q];
    if (bytes) *bytes = prof_bytes_p_[q];
  }
  // Profiling: every prof_stride_-th launch of each kernel and arithmetic is bracketed by events
  // (counted per kernel, so every kernel is sampled whatever the launch pattern)
  bool prof_sample(int kernel, int prec) {
    if (prof_stride_ <= 0) return false;
    ++prof_all_;
    return (prof_all_p_[2 * kernel + (prec & 1)]++ % prof_stride_) == 0;
  }
  // algorithmic bytes of a GEMM launch: A, B (once per problem unless batched) and C once each,
  // C twice when accumulated into
  static double gemm_bytes(const GemmDesc &d, int nprob) {
    const double ea = d.a32 ? 8 : 16, eb = d.b32 ? 8 : 16, ec = d.c32 ? 8 : 16;
    return nprob * (ea * d.M * (double)d.K * d.batch + eb * d.K * (double)d.N * (d.b_b ? d.batch : 1) +
                    ec * d.M * (double)d.N * d.batch * (d.beta ? 2 : 1));
  }
  void drain_profile() {
    for (size_t i = 0; i < prof_ev_.size(); ++i) {
      auto &pr = prof_ev_[i];
      HIPCHK(hipEventSynchronize(pr.second));
      float ms = 0;
      HIPCHK(hipEventElapsedTime(&ms, pr.first, pr.second));
      prof_ms_ += ms;
      prof_launches_ += 1;
      const int q = prof_prec_[i];
      prof_ms_p_[q] += ms;
      prof_launches_p_[q] += 1;
      HIPCHK(hipEventDestroy(pr.first));
      HIPCHK(hipEventDestroy(pr.second));
    }
    prof_ev_.clear();
    prof_prec_.clear();
  }
  // Blocked Householder reduction (n > 256): panels of TRD_NB reflectors, each followed by the
  // two GEMMs A_st -= V W^H + W V^H on every matrix, then the last diagonal entry.
  void trd_blocked(int n, int lda, const double *const *in, int nprob) {
    const size_t need = (size_t)6 * nprob * sizeof(void *);
    if (need > tptr_bytes_) {
      HIPCHK(hipStreamSynchronize(s_));
      if (tptr_) HIPCHK(dfree(tptr_));
      tptr_ = nullptr;
      tptr_bytes_ = 0;
      if (dmalloc(&tptr_, need) != hipSuccess) {
        err_ = -4;
        errmsg_ = "eigh pointer table allocation failed";
        return;
      }
      tptr_bytes_ = need;
    }
    std::vector<void *> hp((size_t)6 * nprob);
    for (int q = 0; q < nprob; ++q) {
      double *base = (double *)lws_ + (size_t)q * tql_ws_doubles(n);
      double2 *U = (double2 *)(base + trd_panel_offset(n));
      double2 *P = (double2 *)(base + (size_t)4 * n * n + (size_t)3 * n);   // the stored matrix
      hp[0 * nprob + q] = U;                // V W^H: A = V, B = W
      hp[1 * nprob + q] = U + TRD_NB;
      hp[2 * nprob + q] = P;
      hp[3 * nprob + q] = U + TRD_NB;       // W V^H: A = W, B = V
      hp[4 * nprob + q] = U;
      hp[5 * nprob + q] = P;
    }
    h2d(tptr_, hp.data(), need);
    void **tp = (void **)tptr_;
    GemmDesc d;
    d.M = d.Mi = n; d.N = d.Ni = n; d.K = d.Ki = TRD_NB;
    d.a_mi = 2 * TRD_NB; d.a_ki = 1;
    d.b_ki = 1; d.b_ni = 2 * TRD_NB; d.conjB = 1;
    d.c_mi = n; d.c_ni = 1;
    d.beta = 1; d.alpha_re = -1.0;
    for (int k0 = 0; k0 < n - 1; k0 += TRD_NB) {
      stale_check("eigh_trd_panel_kernel");
      hipLaunchKernelGGL((eigh_trd_panel_kernel<512, 1024>), dim3(nprob), dim3(1024), 0, s_, n,
                         lda, in, (double *)lws_, k0);
      launch_check("eigh_trd_panel_kernel");
      gemm(d, (const double *const *)tp, (const double *const *)(tp + nprob),
           (double *const *)(tp + 2 * nprob), nprob);
      gemm(d, (const double *const *)(tp + 3 * nprob), (const double *const *)(tp + 4 * nprob),
           (double *const *)(tp + 5 * nprob), nprob);
    }
    stale_check("eigh_trd_last_kernel");
    hipLaunchKernelGGL(eigh_trd_last_kernel, dim3((nprob + 63) / 64), dim3(64), 0, s_, n,
                       (double *)lws_, nprob);
    launch_check("eigh_trd_last_kernel");
  }
  void eigh(int n, int lda, const double *const *in, double *const *evals, double *const *vecs,
            int nprob, int ncols) override {
    if (nprob <= 0) return;
    if (n < 1 || n > 512) {
      err_ = -1;
      errmsg_ = "eigh: n must be in 1..512";
      return;
    }
    ncols = std::max(1, std::min(ncols, n));
    int np = n + (n & 1);
    if (n < 32) {
      size_t sm = (size_t)2 * np * np * sizeof(double2);
      stale_check("eigh_jacobi_kernel");
      hipLaunchKernelGGL(eigh_jacobi_kernel, dim3(nprob), dim3(1024), sm, s_, n, lda, in,
                         evals, vecs, 60);
    } else {
      // n <= 512 (the callers' limit)
      size_t need = (size_t)nprob * tql_ws_doubles(n) * sizeof(double);
      if (need > lws_bytes_) {
        HIPCHK(hipStreamSynchronize(s_));
        if (lws_) HIPCHK(dfree(lws_));
        lws_ = nullptr;
        lws_bytes_ = 0;
        if (dmalloc(&lws_, need) != hipSuccess) {
          err_ = -4;
          errmsg_ = "eigh workspace allocation failed";
          return;
        }
        lws_bytes_ = need;
      }
      stale_check("eigh_tridiag_kernel");
      if (n <= 128) {
        hipLaunchKernelGGL((eigh_tridiag_kernel<128, 1024>), dim3(nprob), dim3(1024),
                           (size_t)n * (n + 1) / 2 * sizeof(double2), s_, n, lda, in,
                           (double *)lws_);
        launch_check("eigh_tridiag_kernel");
        hipLaunchKernelGGL(eigh_dc_kernel<128>, dim3(nprob), dim3(512),
                           (size_t)n * n * sizeof(double), s_, n, (double *)lws_);
      } else if (n <= 256) {
        hipLaunchKernelGGL((eigh_tridiag_kernel<256, 1024>), dim3(nprob), dim3(1024), 0, s_, n,
                           lda, in, (double *)lws_);
        launch_check("eigh_tridiag_kernel");
        hipLaunchKernelGGL(eigh_dc_kernel<256>, dim3(nprob), dim3(512), 0, s_, n,
                           (double *)lws_);
      } else {
        // n > 256: the blocked reduction (at n = 256 the single kernel is as fast: ~50 matrices
        // per launch keep enough workgroups busy, and the panels' extra launches cost more)
        trd_blocked(n, lda, in, nprob);
        if (err_) return;
        hipLaunchKernelGGL(eigh_dc_kernel<512>, dim3(nprob), dim3(512), 0, s_, n,
                           (double *)lws_);
      }
      launch_check("eigh_dc_kernel");
      stale_check("eigh_backtransform_kernel");
      if (n <= 128)
        hipLaunchKernelGGL(eigh_backtransform_kernel<128>, dim3((ncols + 15) / 16, nprob),
                           dim3(256), 0, s_, n, ncols, (const double *)lws_, evals, vecs);
      else if (n <= 256)
        hipLaunchKernelGGL(eigh_backtransform_kernel<256>, dim3((ncols + 15) / 16, nprob),
                           dim3(256), 0, s_, n, ncols, (const double *)lws_, evals, vecs);
      else
        hipLaunchKernelGGL(eigh_backtransform_kernel<512>, dim3((ncols + 3) / 4, nprob),
                           dim3(256), 0, s_, n, ncols, (const double *)lws_, evals, vecs);
    }
    launch_check("eigh");
  }
  void rx(double *const *t, const int64_t *half, int nprob, double c, double s) override {
    stale_check("rx_kernel");
    hipLaunchKernelGGL(rx_kernel, dim3(64, nprob), dim3(256), 0, s_, t, half, c, s);
    launch_check("rx_kernel");
  }
  void msg_sqrt(int n, const double *const *ev, const double *const *vec, double *const *X,
                double *const *Xp, double cut, int nprob) override {
    if (nprob <= 0) return;
    if (n < 64) {
      stale_check("msg_sqrt_kernel");
      hipLaunchKernelGGL(msg_sqrt_kernel, dim3(nprob), dim3(256), 0, s_, n, ev, vec, X, Xp, cut);
      launch_check("msg_sqrt_kernel");
      return;
    }
    const size_t need = (size_t)nprob * 2 * n * n * sizeof(double2) + 2 * nprob * sizeof(void *);
    if (need > sqws_bytes_) {
      HIPCHK(hipStreamSynchronize(s_));
      if (sqws_) HIPCHK(dfree(sqws_));
      sqws_ = nullptr;
      sqws_bytes_ = 0;
      if (dmalloc(&sqws_, need) != hipSuccess) {
        err_ = -4;
        errmsg_ = "message square-root workspace allocation failed";
        return;
      }
      sqws_bytes_ = need;
    }
    double2 *w = (double2 *)sqws_;
    double **pf = (double **)(w + (size_t)nprob * 2 * n * n), **pg = pf + nprob;
    stale_check("sqrt_scale_kernel");
    hipLaunchKernelGGL(sqrt_scale_kernel, dim3(nprob), dim3(256), 0, s_, n, ev, vec, cut, w, pf,
                       pg);
    launch_check("sqrt_scale_kernel");
    GemmDesc d;                          // X = (W diag f) W^H, Hermitian
    d.M = d.Mi = n; d.N = d.Ni = n; d.K = d.Ki = n;
    d.a_mi = n; d.a_ki = 1;
    d.b_ki = 1; d.b_ni = n; d.conjB = 1;
    d.c_mi = n; d.c_ni = 1;
    d.herm = 1;
    gemm(d, (const double *const *)pf, vec, X, nprob);
    gemm(d, (const double *const *)pg, vec, Xp, nprob);
  }
  void gram_chol(int n, const double *const *G, double *const *R, double *const *Wsc, double cut,
                 int nprob) override {
    if (nprob <= 0) return;
    size_t need = (size_t)nprob * (n <= 128 ? 3 * (size_t)n * n : chol_stride(n)) * sizeof(double2);
    if (need > cws_bytes_) {
      HIPCHK(hipStreamSynchronize(s_));
      if (cws_) HIPCHK(dfree(cws_));
      cws_ = nullptr;
      cws_bytes_ = 0;
      if (dmalloc(&cws_, need) != hipSuccess) {
        err_ = -4;
        errmsg_ = "Cholesky workspace allocation failed";
        return;
      }
      cws_bytes_ = need;
    }
    if (n <= 128) {
      stale_check("gram_chol_lds_kernel");
      hipLaunchKernelGGL(gram_chol_lds_kernel, dim3(nprob), dim3(1024),
                         (size_t)n * (n + 1) / 2 * sizeof(double2), s_, n, G, R, Wsc, cut,
                         (double2 *)cws_);
      launch_check("gram_chol_lds_kernel");
    } else {
      // blocked: meta blocks and the GEMMs' pointer arrays (panel updates, then the block rows of
      // the triangular inverse)
      const size_t mbytes = (size_t)nprob * chol_meta_bytes(n);
      const int npan = (n + CHOL_NB - 1) / CHOL_NB;
      const size_t nptr = ((size_t)npan * 3 + (size_t)(npan - 1) * 6) * nprob;
      const size_t pbytes = nptr * sizeof(void *);
      const size_t moff = (mbytes + 15) & ~size_t(15);
      if (moff + pbytes > cmeta_bytes_) {
        HIPCHK(hipStreamSynchronize(s_));
        if (cmeta_) HIPCHK(dfree(cmeta_));
        cmeta_ = nullptr;
        cmeta_bytes_ = 0;
        if (dmalloc(&cmeta_, moff + pbytes) != hipSuccess) {
          err_ = -4;
          errmsg_ = "Cholesky workspace allocation failed";
          return;
        }
        cmeta_bytes_ = moff + pbytes;
      }
      char *meta = (char *)cmeta_;
      void **cp = (void **)(meta + moff);
      std::vector<void *> hp(nptr);
      double2 *base = (double2 *)cws_;
      const size_t nn = (size_t)n * n;
      auto slot = [&](size_t gemm, int which, int q) -> void *& {
        return hp[(gemm * 3 + which) * nprob + q];
      };
      for (int q = 0; q < nprob; ++q) {
        double2 *W = base + (size_t)q * chol_stride(n), *L = W + nn, *X = L + nn, *Y = X + nn;
        for (int pn = 0; pn < npan; ++pn) {                   // W -= L_panel L_panel^H
          slot(pn, 0, q) = L + pn * CHOL_NB;
          slot(pn, 1, q) = L + pn * CHOL_NB;
          slot(pn, 2, q) = W;
        }
        for (int I = 1; I < npan; ++I) {                      // W now holds L1
          const size_t g = npan + 2 * (size_t)(I - 1);
          const size_t i0 = (size_t)I * CHOL_NB;
          slot(g, 0, q) = W + i0 * n;                         // Y = L1[I, :I] X[:I, :I]
          slot(g, 1, q) = X;
          slot(g, 2, q) = Y;
          slot(g + 1, 0, q) = X + i0 * n + i0;                // X[I, :I] = -X[I, I] Y
          slot(g + 1, 1, q) = Y;
          slot(g + 1, 2, q) = X + i0 * n;
        }
      }
      h2d(cp, hp.data(), pbytes);
      auto ptrs = [&](size_t gemm, int which) { return cp + (gemm * 3 + which) * nprob; };
      stale_check("chol_init_kernel");
      hipLaunchKernelGGL(chol_init_kernel, dim3(nprob), dim3(1024), 0, s_, n, G, base, meta);
      launch_check("chol_init_kernel");
      GemmDesc up;                       // W -= L_panel L_panel^H
      up.M = up.Mi = n; up.N = up.Ni = n;
      up.K = up.Ki = CHOL_NB;
      up.a_mi = n; up.a_ki = 1;
      up.b_ki = 1; up.b_ni = n; up.conjB = 1;
      up.c_mi = n; up.c_ni = 1;
      up.beta = 1; up.alpha_re = -1.0;
      const size_t lds = (size_t)n * (CHOL_NB + 1) * sizeof(double2);
      for (int pn = 0; pn < npan; ++pn) {
        const int k0 = pn * CHOL_NB;
        stale_check("chol_panel_kernel");
        hipLaunchKernelGGL(chol_panel_kernel, dim3(nprob), dim3(1024), lds, s_, n, k0, cut, base,
                           meta);
        launch_check("chol_panel_kernel");
        if (k0 + CHOL_NB < n)
          gemm(up, (const double *const *)ptrs(pn, 0), (const double *const *)ptrs(pn, 1),
               (double *const *)ptrs(pn, 2), nprob);
      }
      stale_check("chol_l1_kernel");
      hipLaunchKernelGGL(chol_l1_kernel, dim3(nprob), dim3(1024), 0, s_, n, base,
                         (const char *)meta);
      launch_check("chol_l1_kernel");
      stale_check("chol_diag_inv_kernel");
      hipLaunchKernelGGL(chol_diag_inv_kernel, dim3(npan, nprob), dim3(64), 0, s_, n, base);
      launch_check("chol_diag_inv_kernel");
      for (int I = 1; I < npan; ++I) {
        const size_t g = npan + 2 * (size_t)(I - 1);
        const int i0 = I * CHOL_NB, b = std::min(CHOL_NB, n - i0);
        GemmDesc y;                      // Y (b x i0) = L1[i0.., :i0] X[:i0, :i0]
        y.M = y.Mi = b; y.N = y.Ni = i0; y.K = y.Ki = i0;
        y.a_mi = n; y.a_ki = 1;
        y.b_ki = n; y.b_ni = 1;
        y.c_mi = n; y.c_ni = 1;
        gemm(y, (const double *const *)ptrs(g, 0), (const double *const *)ptrs(g, 1),
             (double *const *)ptrs(g, 2), nprob);
        GemmDesc x = y;                  // X[i0.., :i0] = -X[i0.., i0..] Y
        x.K = x.Ki = b;
        x.alpha_re = -1.0;
        gemm(x, (const double *const *)ptrs(g + 1, 0), (const double *const *)ptrs(g + 1, 1),
             (double *const *)ptrs(g + 1, 2), nprob);
      }
      stale_check("chol_out_kernel");
      hipLaunchKernelGGL(chol_out_kernel, dim3(nprob), dim3(1024), 0, s_, n, R, Wsc,
                         (const double2 *)base, (const char *)meta);
      launch_check("chol_out_kernel");
    }
  }
  void theta(int rB, int rS, int chi, const double *const *RB, const double *const *RS,
             double *const *Th, double a, double b, double c, double d, int nprob) override {
    // Theta[(rb,sb)][(rs,ss)] = sum_k RB[rb][sb][k] RS[rs][ss][k] on the MFMA GEMM (rows of RB
    // and RS are contiguous runs of chi), then the gate phases elementwise
    GemmDesc gd;
    gd.M = 2 * rB; gd.Mi = gd.M; gd.a_mi = chi;
    gd.N = 2 * rS; gd.Ni = gd.N; gd.b_ni = chi;
    gd.K = chi; gd.Ki = chi; gd.a_ki = 1; gd.b_ki = 1;
    gd.c_mi = gd.N; gd.c_ni = 1;
    gemm(gd, RB, RS, Th, nprob);
    int tot = 4 * rB * rS;
    int bx = std::min(1024, (tot + 255) / 256);
    stale_check("theta_phase_kernel");
    hipLaunchKernelGGL(theta_phase_kernel, dim3(bx, nprob), dim3(256), 0, s_, rB, rS, Th, a, b, c,
                       d);
    launch_check("theta_phase_kernel");
  }
  void svd_finish(int n, int chi, const double *const *ev, const double *const *vec,
                  double *const *Vs, double *const *S, int *kout, double *disc,
                  double *const *mA, double *const *mB, double cutoff, int nprob) override {
    stale_check("svd_finish_kernel");
    hipLaunchKernelGGL(svd_finish_kernel, dim3(nprob), dim3(256), 0, s_, n, chi, ev, vec, Vs, S,
                       kout, disc, mA, mB, cutoff);
    launch_check("svd_finish_kernel");
  }
  void split_sqrt(int rowsB, int rowsS, int n, int chi, const double *const *U,
                  const double *const *V, const double *const *S, double *const *RBn,
                  double *const *RSn, int nprob) override {
    int tot = (rowsB + rowsS) * chi;
    int bx = std::min(1024, (tot + 255) / 256);
    stale_check("split_sqrt_kernel");
    hipLaunchKernelGGL(split_sqrt_kernel, dim3(bx, nprob), dim3(256), 0, s_, rowsB, rowsS, n,
                       chi, U, V, S, RBn, RSn);
    launch_check("split_sqrt_kernel");
  }
  void to_f32(const double *src, float *dst, size_t n) override {
    if (!n) return;
    const unsigned bx = (unsigned)std::min<size_t>(4 * (size_t)resident_, (n + 255) / 256);
    stale_check("to_f32_kernel");
    hipLaunchKernelGGL(to_f32_kernel, dim3(bx), dim3(256), 0, s_, (const double2 *)src,
                       (float2 *)dst, n);
    launch_check("to_f32_kernel");
  }
  void normalize_residual(int chi, double *const *Mn, const double *const *Mo, double *res,
                          int nprob) override {
    stale_check("normalize_residual_kernel");
    hipLaunchKernelGGL(normalize_residual_kernel, dim3(nprob), dim3(256), 0, s_, chi, Mn, Mo,
                       res);
    launch_check("normalize_residual_kernel");
  }
  double mfma_rate(int prec, int blocks, int iters) override {
    if (blocks < 1 || iters < 1) return 0.0;
    double *out = (double *)alloc(sizeof(double));
    if (!out) return 0.0;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    HIPCHK(hipEventCreate(&e0));
    HIPCHK(hipEventCreate(&e1));
    float ms = 0.0f;
    for (int rep = 0; rep < 2; ++rep) {      // the first launch warms the clocks up
      HIPCHK(hipEventRecord(e0, s_));
      if (prec == 1)
        hipLaunchKernelGGL(mfma_rate_kernel<float>, dim3(blocks), dim3(256), 0, s_, iters, out);
      else
        hipLaunchKernelGGL(mfma_rate_kernel<double>, dim3(blocks), dim3(256), 0, s_, iters, out);
      launch_check("mfma_rate_kernel");
      HIPCHK(hipEventRecord(e1, s_));
      HIPCHK(hipEventSynchronize(e1));
      HIPCHK(hipEventElapsedTime(&ms, e0, e1));
    }
    HIPCHK(hipEventDestroy(e0));
    HIPCHK(hipEventDestroy(e1));
    release(out);
    const double flops = 2048.0 * 12 * (double)iters * (double)blocks * 4;
    return ms > 0.0f ? flops / (ms * 1e-3) / 1e12 : 0.0;
  }
  void bond_entropy(int n, const double *const *evals, double *out, int nprob) override {
    if (nprob <= 0) return;
    stale_check("bond_entropy_kernel");
    hipLaunchKernelGGL(bond_entropy_kernel, dim3(nprob), dim3(256), 0, s_, n, evals, out);
    launch_check("bond_entropy_kernel");
  }
  void vidal_svd(int n, const double *const *evals, const double *const *vecs, double *const *D1,
                 double *const *D2, double *const *Mu, double *const *Mv, double *lam, int *kept,
                 double cut, int nprob) override {
    if (nprob <= 0) return;
    stale_check("vidal_svd_kernel");
    hipLaunchKernelGGL(vidal_svd_kernel, dim3(nprob), dim3(256), 0, s_, n, evals, vecs, D1, D2,
                       Mu, Mv, lam, kept, cut);
    launch_check("vidal_svd_kernel");
  }
  void trace(const double *R, int n, double *out) override {
    stale_check("trace_kernel");
    hipLaunchKernelGGL(trace_kernel, dim3(1), dim3(256), 0, s_, R, n, out);
    launch_check("trace_kernel");
  }
  void reduce_max(const double *x, int n, double *out) override {
    stale_check("reduce_max_kernel");
    hipLaunchKernelGGL(reduce_max_kernel, dim3(1), dim3(256), 0, s_, x, n, out);
    launch_check("reduce_max_kernel");
  }
  void member_residual(const double *res, const int *off, const int *idx, int nmem,
                       const int *act, int *act_next, double tol, double *out) override {
    if (nmem <= 0) return;
    stale_check("member_residual_kernel");
    hipLaunchKernelGGL(member_residual_kernel, dim3(nmem), dim3(256), 0, s_, res, off, idx, act,
                       act_next, tol, out);
    launch_check("member_residual_kernel");
  }
  void commit_messages(double *M, const double *Mn, long elems, int nmsg, const int *msg_member,
                       const int *act) override {
    const long total = elems * nmsg;
    if (total <= 0) return;
    const int blocks = (int)std::min<long>((total + 255) / 256, 4096);
    stale_check("commit_messages_kernel");
    hipLaunchKernelGGL(commit_messages_kernel, dim3(blocks), dim3(256), 0, s_, (double2 *)M,
                       (const double2 *)Mn, elems, total, msg_member, act);
    launch_check("commit_messages_kernel");
  }
  void rho_dot(const double *const *Y, const double *const *T, const int64_t *len, double *rho,
               int nprob) override {
    if (nprob <= 0) return;
    const size_t need = (size_t)nprob * RHO_CHUNKS * 8 * sizeof(double);
    if (need > rws_bytes_) {
      HIPCHK(hipStreamSynchronize(s_));
      if (rws_) HIPCHK(dfree(rws_));
      rws_ = nullptr;
      rws_bytes_ = 0;
      if (dmalloc(&rws_, need) != hipSuccess) {
        err_ = -4;
        errmsg_ = "observable workspace allocation failed";
        return;
      }
      rws_bytes_ = need;
    }
    stale_check("rho_dot_kernel");
    hipLaunchKernelGGL(rho_dot_kernel, dim3(RHO_CHUNKS, nprob), dim3(256), 0, s_, Y, T, len,
                       (double *)rws_);
    launch_check("rho_dot_kernel");
    hipLaunchKernelGGL(rho_sum_kernel, dim3((nprob * 8 + 255) / 256), dim3(256), 0, s_,
                       (const double *)rws_, RHO_CHUNKS, nprob, rho);
    launch_check("rho_sum_kernel");
  }
  void apply_op(const double *const *Tin, double *const *Tout, const int64_t *half,
                const double *ops, int nprob) override {
    stale_check("apply_op_kernel");
    hipLaunchKernelGGL(apply_op_kernel, dim3(64, nprob), dim3(256), 0, s_, Tin, Tout, half, ops);
    launch_check("apply_op_kernel");
  }

  int err_ = 0;
  std::string errmsg_;

 private:
  int dev_;
  hipStream_t s_;
  bool own_;
  hipEvent_t ev_[8] = {};
  void *lws_ = nullptr;
  size_t lws_bytes_ = 0;
  void *rws_ = nullptr;
  size_t rws_bytes_ = 0;
  static constexpr size_t kPinBytes = 16384;
  static constexpr size_t kPinAsync = 64;      // the tail of pin_ holds the read_async slots
  hipEvent_t rd_ev_[2] = {nullptr, nullptr};
  double rd_val_[2] = {0, 0};
  int resident_ = 512;             // gemm_kernel workgroups resident at once (2 per CU)
  void *pin_ = nullptr;
  void *cws_ = nullptr;
  size_t cws_bytes_ = 0;
  void *cmeta_ = nullptr;            // blocked Cholesky: meta blocks + panel pointer arrays
  size_t cmeta_bytes_ = 0;
  void *sqws_ = nullptr;             // message square roots on the GEMM: scaled vectors, pointers
  size_t sqws_bytes_ = 0;
  void *tptr_ = nullptr;             // blocked tridiagonalisation: GEMM pointer table
  size_t tptr_bytes_ = 0;
  void *skws_ = nullptr;
  DevAlloc ua_ = nullptr;            // caller's allocator (null: hipMalloc / hipFree)
  DevFree uf_ = nullptr;
  void *uu_ = nullptr;
  bool touched_ = false;             // device memory has been taken (the allocator is then fixed)
  size_t skws_bytes_ = 0;
  int prof_stride_ = 0;
  std::vector<std::pair<hipEvent_t, hipEvent_t>> prof_ev_;
  long prof_launches_ = 0, prof_all_ = 0;
  double prof_ms_ = 0, prof_flops_ = 0;
  // the same sums by arithmetic of the bracketed launches (0 FP64 MFMA, 1 FP32 MFMA)
  // per bracketed launch: 2 * kernel + FP32 MFMA, kernel 0 gemm_kernel, 1 bp_close_kernel,
  // 2 gemm_stream_kernel
  static constexpr int kProfBuckets = 6;
  std::vector<int> prof_prec_;
  long prof_launches_p_[kProfBuckets] = {}, prof_all_p_[kProfBuckets] = {};
  double prof_ms_p_[kProfBuckets] = {}, prof_flops_p_[kProfBuckets] = {},
         prof_bytes_p_[kProfBuckets] = {};
};

// Device memory of the allocation-free solve (bpki_solve_noalloc): a fixed array in the code
// object, so that every device holds its own copy from module load until the process ends.  Host
// code must not use the array's name as an address; scratch_region looks up each device's copy
// once (with that device current) and hands out that address.
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

int scratch_region(int device, void **ptr, std::string *err) {
  static std::mutex mu;
  static std::map<int, void *> addr;
  std::lock_guard<std::mutex> lk(mu);
  auto it = addr.find(device);
  if (it == addr.end()) {
    int cur = -1;
    if (hipGetDevice(&cur) != hipSuccess || cur != device) {
      (void)hipGetLastError();
      if (err) *err = "scratch: device " + std::to_string(device) + " is not current";
      return -5;
    }
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) {
      (void)hipGetLastError();
      if (err) *err = std::string("scratch: hipGetSymbolAddress: ") + hipGetErrorString(e);
      return -5;
    }
    it = addr.emplace(device, p).first;
  }
  *ptr = it->second;
  return 0;
}

Backend *make_hip_backend(int device, void *stream, std::string *err) {
  int count = 0;
  hipError_t e = hipGetDeviceCount(&count);
  if (e != hipSuccess || count <= device || device < 0) {
    if (err) *err = "no HIP device available (hipGetDeviceCount)";
    return nullptr;
  }
  HipBackend *b = new HipBackend(device, stream);
  if (b->err_) {
    if (err) *err = b->errmsg_;
    delete b;
    return nullptr;
  }
  return b;
}

}  // namespace bpki
