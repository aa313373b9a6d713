// HIP/CDNA4 (gfx950) kernels and the device backend of the bpki engine.
//
//  * gemm_kernel: grouped, batched complex GEMM on MFMA (FP64: v_mfma_f64_16x16x4f64; FP32 mode:
//                 v_mfma_f32_16x16x4f32 with FP64 storage and FP64 split-K sums).  Complex
//                 products in real-split form: four real MFMA accumulators per 16x16 tile
//                 (re*re, im*im, re*im, im*re), combined in the epilogue.  Operands are staged
//                 through LDS in split re/im planes; the global loads follow whichever index is
//                 unit-stride so they coalesce for every leg ordering of the site tensors.
//  * eigh_jacobi: batched Hermitian eigendecomposition, FP64 cyclic Jacobi with the parallel
//                 round-robin ordering (n/2 disjoint rotations per round, all 2x2 block updates
//                 of a round in parallel).  Matrix and eigenvectors live in LDS up to n = 64,
//                 otherwise in a global (L2-resident) work area.
//  * small kernels for the X rotations, message square roots, Gram factor, the gate block,
//    truncation, BP normalisation/residual and the site density matrices.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
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

// Grouped complex GEMM.  grid: x = output tiles, y = batch * ksplit, z = problem.  With
// ksplit > 1 each block sums its K chunk into the partial buffer W (layout
// [prob][batch][kz][M][N]); gemm_reduce_kernel then combines the chunks in a fixed order.
// T = double: FP64 MFMA (v_mfma_f64_16x16x4f64); T = float: operands rounded to FP32 when
// staged, FP32 MFMA (v_mfma_f32_16x16x4f32) with FP32 accumulation over the block's K range.
// Storage and the split-K chunk sums stay FP64.
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

template <typename T>
__global__ __launch_bounds__(256, 2) void gemm_kernel(GemmDesc d, const double *const *Ap,
                                                      const double *const *Bp,
                                                      double *const *Cp, int ksplit,
                                                      int kchunk, double2 *W) {
  typedef MfmaTraits<T> MT;
  typedef typename MT::acc_t acc_t;
  __shared__ T As[2][BK][BM + PAD];
  __shared__ T Bs[2][BK][BN + PAD];
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int tiles_m = (d.M + BM - 1) / BM;
  const int tm = blockIdx.x % tiles_m, tn = blockIdx.x / tiles_m;
  const int bat = blockIdx.y / ksplit, kz = blockIdx.y % ksplit, prob = blockIdx.z;
  const double2 *A = reinterpret_cast<const double2 *>(Ap[prob]) + (long)bat * d.a_b;
  const double2 *B = reinterpret_cast<const double2 *>(Bp[prob]) + (long)bat * d.b_b;
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
  double2 ra[LOADS], rb[LOADS];
  auto fetch = [&](int k0) {
    KOff ka = k_tile(k0, d.Ki, d.a_ko, d.a_ki), kb = k_tile(k0, d.Ki, d.b_ko, d.b_ki);
#pragma unroll
    for (int it = 0; it < LOADS; ++it) {
      int kga = k0 + ak[it], kgb = k0 + bk[it];
      double2 va = make_double2(0.0, 0.0), vb = make_double2(0.0, 0.0);
      if (aok[it] && kga < kend) {
        long o = ka.uniform ? ka.base + (long)ak[it] * ka.si : cidx(kga, d.Ki, d.a_ko, d.a_ki);
        va = A[aoff[it] + o];
      }
      if (bok[it] && kgb < kend) {
        long o = kb.uniform ? kb.base + (long)bk[it] * kb.si : cidx(kgb, d.Ki, d.b_ko, d.b_ki);
        vb = B[boff[it] + o];
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

  acc_t acc[2][2][4];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int t = 0; t < 4; ++t) acc[i][j][t] = (acc_t){T(0), T(0), T(0), T(0)};

  if (kbeg < kend) fetch(kbeg);
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
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) {
          acc[i][j][0] = MT::mma(ar[i], br[j], acc[i][j][0]);
          acc[i][j][1] = MT::mma(ai[i], bi[j], acc[i][j][1]);
          acc[i][j][2] = MT::mma(ar[i], bi[j], acc[i][j][2]);
          acc[i][j][3] = MT::mma(ai[i], br[j], acc[i][j][3]);
        }
    }
    __syncthreads();
  }
  // ---- epilogue ----
  double2 *C = reinterpret_cast<double2 *>(Cp[prob]) + (long)bat * d.c_b;
  double2 *Wp = W ? W + (((size_t)prob * d.batch + bat) * ksplit + kz) * (size_t)d.M * d.N
                  : nullptr;
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
        double ci = (double)acc[i][j][2][r] + (double)acc[i][j][3][r];
        if (Wp) {
          Wp[(size_t)mg * d.N + ng] = make_double2(cr, ci);
          continue;
        }
        double vr = d.alpha_re * cr - d.alpha_im * ci;
        double vi = d.alpha_re * ci + d.alpha_im * cr;
        long off = cidx(mg, d.Mi, d.c_mo, d.c_mi) + cidx(ng, d.Ni, d.c_no, d.c_ni);
        if (d.beta) {
          double2 o = C[off];
          vr += o.x;
          vi += o.y;
        }
        C[off] = make_double2(vr, vi);
      }
}

// Sums the K chunks of a split-K GEMM in chunk order and applies alpha / beta.
__global__ __launch_bounds__(256) void gemm_reduce_kernel(GemmDesc d, double *const *Cp,
                                                          int ksplit, const double2 *W) {
  const int bat = blockIdx.y, prob = blockIdx.z;
  const size_t mn = (size_t)d.M * d.N;
  const double2 *wp = W + ((size_t)prob * d.batch + bat) * ksplit * mn;
  double2 *C = reinterpret_cast<double2 *>(Cp[prob]) + (long)bat * d.c_b;
  for (size_t idx = blockIdx.x * (size_t)blockDim.x + threadIdx.x; idx < mn;
       idx += (size_t)gridDim.x * blockDim.x) {
    double cr = 0, ci = 0;
    for (int kz = 0; kz < ksplit; ++kz) {
      double2 v = wp[kz * mn + idx];
      cr += v.x;
      ci += v.y;
    }
    int mg = (int)(idx / d.N), ng = (int)(idx % d.N);
    double vr = d.alpha_re * cr - d.alpha_im * ci;
    double vi = d.alpha_re * ci + d.alpha_im * cr;
    long off = cidx(mg, d.Mi, d.c_mo, d.c_mi) + cidx(ng, d.Ni, d.c_no, d.c_ni);
    if (d.beta) {
      double2 o = C[off];
      vr += o.x;
      vi += o.y;
    }
    C[off] = make_double2(vr, vi);
  }
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

template <bool LDS>
__global__ __launch_bounds__(1024) void eigh_jacobi_kernel(int n, int lda,
                                                           const double *const *in,
                                                           double *const *evals,
                                                           double *const *vecs, double2 *gws,
                                                           int max_sweeps) {
  extern __shared__ double2 smem[];
  __shared__ Rot rot[128];
  __shared__ int any_rot;
  __shared__ double diag_s[256];
  __shared__ double red_s[16];
  const int prob = blockIdx.x;
  const int tid = threadIdx.x, nt = blockDim.x;
  const int np = n + (n & 1);
  const int h = np / 2;
  double2 *A, *V;
  if (LDS) { A = smem; V = smem + (size_t)np * np; }
  else { A = gws + (size_t)prob * 2 * np * np; V = A + (size_t)np * np; }
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

// Jacobi for 64 < n <= 128: the Hermitian matrix is held packed (lower triangle) in LDS and
// the rotations of every round are logged to global memory; the eigenvector matrix is then
// rebuilt by replaying the log on blocks of 64 rows held in LDS (rows of V evolve independently
// under the right-multiplied rotations).
__device__ __forceinline__ size_t pk_idx(int i, int j) {   // i >= j
  return (size_t)i * (i + 1) / 2 + j;
}
__device__ __forceinline__ double2 pk_get(const double2 *P, int i, int j) {
  return i >= j ? P[pk_idx(i, j)] : cconj(P[pk_idx(j, i)]);
}
__device__ __forceinline__ void pk_set(double2 *P, int i, int j, double2 v) {
  if (i >= j) P[pk_idx(i, j)] = v;
  else P[pk_idx(j, i)] = cconj(v);
}

__global__ __launch_bounds__(1024) void eigh_jacobi_log_kernel(int n, int lda,
                                                               const double *const *in,
                                                               double *const *evals,
                                                               double *const *vecs,
                                                               double4_t *logbuf,
                                                               int max_sweeps,
                                                               double *meta_diag,
                                                               int *meta_rounds) {
  extern __shared__ double2 smem[];
  __shared__ Rot rot[64];
  __shared__ int any_rot, nrounds_s;
  __shared__ double diag_s[128];
  __shared__ double red_s[16];
  const int prob = blockIdx.x;
  const int tid = threadIdx.x, nt = blockDim.x;
  const int np = n + (n & 1);
  const int h = np / 2;
  double2 *P = smem;
  double4_t *lg = logbuf + (size_t)prob * max_sweeps * (np - 1) * h;
  const double2 *src = reinterpret_cast<const double2 *>(in[prob]);
  double fro2 = 0.0;
  for (int idx = tid; idx < np * (np + 1) / 2; idx += nt) {
    int i = (int)((sqrt(8.0 * idx + 1.0) - 1.0) * 0.5);
    while ((size_t)i * (i + 1) / 2 > (size_t)idx) --i;
    while ((size_t)(i + 1) * (i + 2) / 2 <= (size_t)idx) ++i;
    int j = idx - i * (i + 1) / 2;
    double2 v = make_double2(0.0, 0.0);
    if (i < n && j < n) {
      double2 a = src[(size_t)i * lda + j], b = src[(size_t)j * lda + i];
      v = make_double2(0.5 * (a.x + b.x), 0.5 * (a.y - b.y));
    }
    P[idx] = v;
    fro2 += (i == j ? 1.0 : 2.0) * (v.x * v.x + v.y * v.y);
  }
  if (tid == 0) nrounds_s = 0;
  __syncthreads();
  const double eps = 2.220446049250313e-16;
  const double thr_abs = 0.1 * eps * sqrt(block_allsum(fro2, red_s));
  // this thread's 2x2 blocks (I >= J) are the same in every round
  const int nblk = h * (h + 1) / 2;
  int bI[3], bJ[3];
  int nmine = 0;
  for (int blk = tid; blk < nblk && nmine < 3; blk += nt, ++nmine) {
    int I = (int)((sqrt(8.0 * blk + 1.0) - 1.0) * 0.5);
    while (I * (I + 1) / 2 > blk) --I;
    while ((I + 1) * (I + 2) / 2 <= blk) ++I;
    bI[nmine] = I;
    bJ[nmine] = blk - I * (I + 1) / 2;
  }
  int nrounds = 0;
  for (int sweep = 0; sweep < max_sweeps; ++sweep) {
    if (tid == 0) any_rot = 0;
    __syncthreads();
    for (int r = 0; r < np - 1; ++r) {
      if (tid < h) {
        int p, q;
        pair_of(r, tid, np, p, q);
        double a = P[pk_idx(p, p)].x, dd = P[pk_idx(q, q)].x;
        double2 b = pk_get(P, p, q);
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
        lg[(size_t)nrounds * h + tid] = (double4_t){R.c, R.s, R.wr, R.wi};
      }
      __syncthreads();
      // blocks (I, J) with I >= J cover every unordered element pair once
      for (int mb = 0; mb < nmine; ++mb) {
        const int I = bI[mb], J = bJ[mb];
        Rot ri = rot[I], rj = rot[J];
        if (ri.s == 0.0 && rj.s == 0.0) continue;
        double2 b00 = pk_get(P, ri.p, rj.p), b01 = pk_get(P, ri.p, rj.q);
        double2 b10 = pk_get(P, ri.q, rj.p), b11 = pk_get(P, ri.q, rj.q);
        // J = diag(1, w) R with R real: apply the phases, then the two real rotations
        const double2 wj = make_double2(rj.wr, rj.wi), wic = make_double2(ri.wr, -ri.wi);
        b01 = cmul(b01, wj);
        b10 = cmul(wic, b10);
        b11 = cmul(cmul(wic, b11), wj);
        double2 t00 = make_double2(rj.c * b00.x - rj.s * b01.x, rj.c * b00.y - rj.s * b01.y);
        double2 t01 = make_double2(rj.s * b00.x + rj.c * b01.x, rj.s * b00.y + rj.c * b01.y);
        double2 t10 = make_double2(rj.c * b10.x - rj.s * b11.x, rj.c * b10.y - rj.s * b11.y);
        double2 t11 = make_double2(rj.s * b10.x + rj.c * b11.x, rj.s * b10.y + rj.c * b11.y);
        double2 n00 = make_double2(ri.c * t00.x - ri.s * t10.x, ri.c * t00.y - ri.s * t10.y);
        double2 n01 = make_double2(ri.c * t01.x - ri.s * t11.x, ri.c * t01.y - ri.s * t11.y);
        double2 n10 = make_double2(ri.s * t00.x + ri.c * t10.x, ri.s * t00.y + ri.c * t10.y);
        double2 n11 = make_double2(ri.s * t01.x + ri.c * t11.x, ri.s * t01.y + ri.c * t11.y);
        if (I == J) {
          n00.y = 0.0; n11.y = 0.0;
          if (ri.s != 0.0) n10 = make_double2(0.0, 0.0);
          pk_set(P, ri.p, ri.p, n00);
          pk_set(P, ri.q, ri.q, n11);
          pk_set(P, ri.q, ri.p, n10);
        } else {
          pk_set(P, ri.p, rj.p, n00);
          pk_set(P, ri.p, rj.q, n01);
          pk_set(P, ri.q, rj.p, n10);
          pk_set(P, ri.q, rj.q, n11);
        }
      }
      ++nrounds;
      __syncthreads();
    }
    __syncthreads();
    int stop = (any_rot == 0);
    __syncthreads();
    if (stop) break;
  }
  for (int i = tid; i < np; i += nt) meta_diag[(size_t)prob * np + i] = P[pk_idx(i, i)].x;
  if (tid == 0) meta_rounds[prob] = nrounds;
}

// Rebuilds the eigenvectors from the rotation log: rows of V evolve independently under the
// right-multiplied rotations, so each workgroup replays the whole log on 16 rows held in LDS.
// grid: x = row blocks of 16, y = problem.  Also sorts into descending eigenvalue order.
__global__ __launch_bounds__(256) void eigh_replay_kernel(int n, const double4_t *logbuf,
                                                          int max_sweeps,
                                                          const double *meta_diag,
                                                          const int *meta_rounds,
                                                          double *const *evals,
                                                          double *const *vecs) {
  __shared__ double2 Vb[16 * 128];
  __shared__ double dg[128];
  const int prob = blockIdx.y, r0 = blockIdx.x * 16;
  const int tid = threadIdx.x, nt = blockDim.x;
  const int np = n + (n & 1), h = np / 2;
  const double4_t *lg = logbuf + (size_t)prob * max_sweeps * (np - 1) * h;
  const int nrounds = meta_rounds[prob];
  const int rows = min(16, np - r0);
  for (int i = tid; i < np; i += nt) dg[i] = meta_diag[(size_t)prob * np + i];
  for (int idx = tid; idx < rows * np; idx += nt) {
    int rr = idx / np, c = idx % np;
    Vb[idx] = make_double2((r0 + rr) == c ? 1.0 : 0.0, 0.0);
  }
  __syncthreads();
  for (int t = 0; t < nrounds; ++t) {
    const int rr0 = t % (np - 1);
    const double4_t *lr = lg + (size_t)t * h;
    for (int it = tid; it < rows * h; it += nt) {
      int rr = it / h, J = it % h;
      double4_t R = lr[J];
      if (R[1] == 0.0) continue;
      int p, q;
      pair_of(rr0, J, np, p, q);
      double2 vp = Vb[rr * np + p];
      double2 vq = cmul(make_double2(R[2], R[3]), Vb[rr * np + q]);
      Vb[rr * np + p] = make_double2(R[0] * vp.x - R[1] * vq.x, R[0] * vp.y - R[1] * vq.y);
      Vb[rr * np + q] = make_double2(R[1] * vp.x + R[0] * vq.x, R[1] * vp.y + R[0] * vq.y);
    }
    __syncthreads();
  }
  double *ev = evals[prob];
  double2 *vo = reinterpret_cast<double2 *>(vecs[prob]);
  for (int i = tid; i < n; i += nt) {
    double li = dg[i];
    int rank = 0;
    for (int j = 0; j < n; ++j) {
      double lj = dg[j];
      rank += (lj > li) || (lj == li && j < i);
    }
    for (int rr = 0; rr < rows; ++rr)
      if (r0 + rr < n) vo[(size_t)(r0 + rr) * n + rank] = Vb[rr * np + i];
    if (blockIdx.x == 0) ev[rank] = li;
  }
}

// ------------------------------------------------------------------------------------------
// Pivoted Cholesky factor of a Gram matrix (one workgroup per matrix, work arrays in an
// L2-resident global area).  Right-looking: pivot = largest remaining diagonal entry (wave
// reduction), column of L, rank-1 update of the trailing Schur complement; stops at the first
// pivot <= cut * max diag.  Then X = L1^{-1} by forward substitution (one thread per column).
__global__ __launch_bounds__(1024) void gram_chol_kernel(int n, const double *const *G,
                                                         double *const *R, double *const *Wsc,
                                                         double cut, double2 *ws) {
  __shared__ int perm[256];
  __shared__ double dg[256];
  __shared__ int piv_s, rank_s;
  __shared__ double gmax_s;
  const int prob = blockIdx.x, tid = threadIdx.x, nt = blockDim.x;
  const int lane = tid & 63, wave = tid >> 6;
  double2 *W = ws + (size_t)prob * 3 * n * n, *L = W + (size_t)n * n, *X = L + (size_t)n * n;
  const double2 *g = reinterpret_cast<const double2 *>(G[prob]);
  for (int idx = tid; idx < n * n; idx += nt) {
    int i = idx / n, j = idx % n;
    double2 a = g[(size_t)i * n + j], b = g[(size_t)j * n + i];
    W[idx] = make_double2(0.5 * (a.x + b.x), 0.5 * (a.y - b.y));
    L[idx] = make_double2(0.0, 0.0);
    X[idx] = make_double2(0.0, 0.0);
  }
  for (int i = tid; i < n; i += nt) {
    perm[i] = i;
    dg[i] = g[(size_t)i * n + i].x;
  }
  __syncthreads();
  if (wave == 0) {
    double m = 0;
    for (int i = lane; i < n; i += 64) m = fmax(m, dg[i]);
    for (int o = 32; o > 0; o >>= 1) m = fmax(m, __shfl_xor(m, o, 64));
    if (lane == 0) { gmax_s = m; rank_s = n; }
  }
  __syncthreads();
  const double gmax = gmax_s;
  for (int k = 0; k < n; ++k) {
    if (wave == 0) {
      double best = -1.0;
      int bj = k;
      for (int j = k + lane; j < n; j += 64) {
        double v = dg[perm[j]];
        if (v > best) { best = v; bj = j; }
      }
      for (int o = 32; o > 0; o >>= 1) {
        double ob = __shfl_xor(best, o, 64);
        int oj = __shfl_xor(bj, o, 64);
        if (ob > best || (ob == best && oj < bj)) { best = ob; bj = oj; }
      }
      if (lane == 0) {
        if (!(best > cut * gmax) || !(gmax > 0)) {
          rank_s = k;
          piv_s = -1;
        } else {
          int t = perm[k];
          perm[k] = perm[bj];
          perm[bj] = t;
          piv_s = bj;
        }
      }
    }
    __syncthreads();
    if (piv_s < 0) break;
    const int pk = perm[k];
    const double piv = sqrt(dg[pk]);
    for (int kk = k + 1 + tid; kk < n; kk += nt) {
      int i = perm[kk];
      double2 w = W[(size_t)i * n + pk];
      L[(size_t)i * n + k] = make_double2(w.x / piv, w.y / piv);
    }
    if (tid == 0) L[(size_t)pk * n + k] = make_double2(piv, 0.0);
    __syncthreads();
    const int m = n - k - 1;
    for (int idx = tid; idx < m * m; idx += nt) {
      int a = k + 1 + idx / m, b = k + 1 + idx % m;
      int i = perm[a], j = perm[b];
      double2 li = L[(size_t)i * n + k], lj = L[(size_t)j * n + k];
      double2 w = W[(size_t)i * n + j];
      // W[i][j] -= L[i][k] conj(L[j][k])
      w.x -= li.x * lj.x + li.y * lj.y;
      w.y -= li.y * lj.x - li.x * lj.y;
      W[(size_t)i * n + j] = w;
      if (a == b) dg[i] = w.x;
    }
    __syncthreads();
  }
  const int r = rank_s;
  // X = L1^{-1}: L1[i][m] = L[perm[i]][m] (i, m < r), lower triangular
  for (int j = tid; j < r; j += nt) {
    for (int i = j; i < r; ++i) {
      double sr = (i == j) ? 1.0 : 0.0, si = 0.0;
      const double2 *Li = L + (size_t)perm[i] * n;
      for (int mm = j; mm < i; ++mm) {
        double2 a = Li[mm], x = X[(size_t)mm * n + j];
        sr -= a.x * x.x - a.y * x.y;
        si -= a.x * x.y + a.y * x.x;
      }
      double2 dgl = Li[i];       // real positive pivot
      X[(size_t)i * n + j] = make_double2(sr / dgl.x, si / dgl.x);
    }
  }
  __syncthreads();
  double2 *Ro = reinterpret_cast<double2 *>(R[prob]);
  double2 *Wo = reinterpret_cast<double2 *>(Wsc[prob]);
  for (int idx = tid; idx < n * n; idx += nt) {
    int k = idx / n, c = idx % n;
    double2 l = L[(size_t)c * n + k];
    Ro[idx] = k < r ? make_double2(l.x, -l.y) : make_double2(0.0, 0.0);
    Wo[idx] = make_double2(0.0, 0.0);
  }
  __syncthreads();
  for (int idx = tid; idx < r * r; idx += nt) {
    int kk = idx / r, k = idx % r;     // Wsc[perm[kk]][k] = conj(X[k][kk])
    double2 x = X[(size_t)k * n + kk];
    Wo[(size_t)perm[kk] * n + k] = make_double2(x.x, -x.y);
  }
}

// ------------------------------------------------------------------------------------------
// small kernels

__global__ void rx_kernel(double *const *T, const int64_t *half, double c, double s) {
  double2 *t = reinterpret_cast<double2 *>(T[blockIdx.y]);
  int64_t h = half[blockIdx.y];
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < h;
       i += (int64_t)gridDim.x * blockDim.x) {
    double2 a = t[i], b = t[h + i];
    // [c, -is; -is, c]
    t[i] = make_double2(c * a.x + s * b.y, c * a.y - s * b.x);
    t[h + i] = make_double2(s * a.y + c * b.x, -s * a.x + c * b.y);
  }
}

__global__ void msg_sqrt_kernel(int n, const double *const *evals, const double *const *vecs,
                                double *const *X, double *const *Xp, double cut) {
  const double *l = evals[blockIdx.x];
  const double2 *W = reinterpret_cast<const double2 *>(vecs[blockIdx.x]);
  double2 *x = reinterpret_cast<double2 *>(X[blockIdx.x]);
  double2 *xp = reinterpret_cast<double2 *>(Xp[blockIdx.x]);
  double lmax = l[0] > 0 ? l[0] : 0.0;
  for (int idx = threadIdx.x; idx < n * n; idx += blockDim.x) {
    int i = idx / n, j = idx % n;
    double sr = 0, si = 0, pr = 0, pi = 0;
    for (int k = 0; k < n; ++k) {
      double lk = l[k];
      double f = lk > 0 ? sqrt(lk) : 0.0;
      double g = (lk > cut * lmax && lk > 0) ? 1.0 / sqrt(lk) : 0.0;
      double2 a = W[(size_t)i * n + k], b = W[(size_t)j * n + k];
      // a * conj(b)
      double re = a.x * b.x + a.y * b.y, im = a.y * b.x - a.x * b.y;
      sr += f * re; si += f * im;
      pr += g * re; pi += g * im;
    }
    x[idx] = make_double2(sr, si);
    xp[idx] = make_double2(pr, pi);
  }
}

__global__ void gram_factor_kernel(int n, int r, const double *const *evals,
                                   const double *const *vecs, double *const *R,
                                   double *const *Wsc, double cut) {
  const double *l = evals[blockIdx.x];
  const double2 *W = reinterpret_cast<const double2 *>(vecs[blockIdx.x]);
  double2 *Ro = reinterpret_cast<double2 *>(R[blockIdx.x]);
  double2 *Wo = reinterpret_cast<double2 *>(Wsc[blockIdx.x]);
  double l0 = l[0] > 0 ? l[0] : 0.0;
  for (int idx = threadIdx.x; idx < r * n; idx += blockDim.x) {
    int i = idx / n, c = idx % n;    // R[i][c]
    double li = l[i];
    bool keep = li > cut * l0 && li > 0;
    double sq = keep ? sqrt(li) : 0.0;
    double2 w = W[(size_t)c * n + i];
    Ro[idx] = make_double2(sq * w.x, -sq * w.y);
    double is = keep ? 1.0 / sq : 0.0;
    Wo[(size_t)c * r + i] = make_double2(is * w.x, is * w.y);
  }
}

__global__ void theta_kernel(int rB, int rS, int chi, const double *const *RB,
                             const double *const *RS, double *const *Th, double gsr, double gsi,
                             double gdr, double gdi) {
  const double2 *a = reinterpret_cast<const double2 *>(RB[blockIdx.y]);
  const double2 *b = reinterpret_cast<const double2 *>(RS[blockIdx.y]);
  double2 *t = reinterpret_cast<double2 *>(Th[blockIdx.y]);
  int rows = 2 * rB, cols = 2 * rS;
  for (int idx = blockIdx.x * blockDim.x + threadIdx.x; idx < rows * cols;
       idx += gridDim.x * blockDim.x) {
    int row = idx / cols, col = idx % cols;
    int rb = row >> 1, sbv = row & 1, rs = col >> 1, ss = col & 1;
    const double2 *pa = a + ((size_t)rb * 2 + sbv) * chi;
    const double2 *pb = b + ((size_t)rs * 2 + ss) * chi;
    double re = 0, im = 0;
    for (int k = 0; k < chi; ++k) {
      double2 x = pa[k], y = pb[k];
      re += x.x * y.x - x.y * y.y;
      im += x.x * y.y + x.y * y.x;
    }
    double gr = (sbv == ss) ? gsr : gdr, gi = (sbv == ss) ? gsi : gdi;
    t[idx] = make_double2(gr * re - gi * im, gr * im + gi * re);
  }
}

__global__ void svd_finish_kernel(int n, int chi, const double *const *evals,
                                  const double *const *vecs, double *const *Vs, double *const *S,
                                  int *kout, double *disc, double *const *mA, double *const *mB,
                                  double cutoff) {
  __shared__ double sig[512];
  __shared__ int ks;
  __shared__ double nrm, ssum;
  const int p = blockIdx.x;
  const double *l = evals[p];
  for (int i = threadIdx.x; i < n; i += blockDim.x) sig[i] = sqrt(fmax(l[i], 0.0));
  __syncthreads();
  if (threadIdx.x == 0) {
    double s0 = sig[0];
    int k = 0;
    for (int i = 0; i < n && k < chi; ++i)
      if (sig[i] > cutoff * s0) ++k;
    double tot = 0, kept = 0, sum = 0;
    for (int i = 0; i < n; ++i) tot += sig[i] * sig[i];
    for (int i = 0; i < k; ++i) kept += sig[i] * sig[i];
    double nr = sqrt(kept);
    for (int i = 0; i < k; ++i) sum += sig[i] / nr;
    ks = k;
    nrm = nr;
    ssum = sum;
    kout[p] = k;
    disc[p] = tot > 0 ? (tot - kept) / tot : 0.0;
  }
  __syncthreads();
  const int k = ks;
  double *Sp = S[p];
  for (int a = threadIdx.x; a < chi; a += blockDim.x) Sp[a] = a < k ? sig[a] / nrm : 0.0;
  const double2 *V = reinterpret_cast<const double2 *>(vecs[p]);
  double2 *vs = reinterpret_cast<double2 *>(Vs[p]);
  for (int idx = threadIdx.x; idx < n * chi; idx += blockDim.x) {
    int c = idx / chi, a = idx % chi;
    double2 v = make_double2(0.0, 0.0);
    if (a < k) { double2 w = V[(size_t)c * n + a]; v = make_double2(w.x / sig[a], w.y / sig[a]); }
    vs[idx] = v;
  }
  double2 *ma = reinterpret_cast<double2 *>(mA[p]);
  double2 *mb = reinterpret_cast<double2 *>(mB[p]);
  for (int idx = threadIdx.x; idx < chi * chi; idx += blockDim.x) {
    int i = idx / chi, j = idx % chi;
    double v = (i == j && i < k) ? (sig[i] / nrm) / ssum : 0.0;
    ma[idx] = make_double2(v, 0.0);
    mb[idx] = make_double2(v, 0.0);
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
      double q = sqrt(s[a]);
      double2 x = u[idx];
      rb[idx] = make_double2(q * x.x, q * x.y);
    } else {
      int j = idx - totB;
      int row = j / chi, a = j % chi;
      double2 o = make_double2(0.0, 0.0);
      if (a < n) {
        double q = sqrt(s[a]);
        double2 x = v[(size_t)row * n + a];
        o = make_double2(q * x.x, -q * x.y);
      }
      rs[j] = o;
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

__global__ __launch_bounds__(256) void normalize_residual_kernel(int chi, double *const *Mn,
                                                                 const double *const *Mo,
                                                                 double *res) {
  __shared__ double sh[8];
  __shared__ double trr, tri;
  const int p = blockIdx.x;
  double2 *m = reinterpret_cast<double2 *>(Mn[p]);
  const double2 *o = reinterpret_cast<const double2 *>(Mo[p]);
  double tr = 0, ti = 0;
  for (int i = threadIdx.x; i < chi; i += blockDim.x) {
    double2 v = m[(size_t)i * chi + i];
    tr += v.x;
    ti += v.y;
  }
  double a = block_sum<256>(tr, sh);
  double b = block_sum<256>(ti, sh);
  if (threadIdx.x == 0) { trr = a; tri = b; }
  __syncthreads();
  double den = trr * trr + tri * tri;
  double ir = trr / den, ii = -tri / den;   // 1/tr
  double acc = 0;
  for (int idx = threadIdx.x; idx < chi * chi; idx += blockDim.x) {
    double2 v = m[idx];
    double2 w = make_double2(v.x * ir - v.y * ii, v.x * ii + v.y * ir);
    m[idx] = w;
    double2 q = o[idx];
    double dx = w.x - q.x, dy = w.y - q.y;
    acc += dx * dx + dy * dy;
  }
  double s = block_sum<256>(acc, sh);
  if (threadIdx.x == 0) res[p] = (trr > 0 && isfinite(s)) ? sqrt(s) : INFINITY;
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

__global__ __launch_bounds__(256) void rho_dot_kernel(const double *const *Y,
                                                      const double *const *T, const int64_t *len,
                                                      double *rho) {
  __shared__ double sh[8];
  const int p = blockIdx.x;
  const double2 *y = reinterpret_cast<const double2 *>(Y[p]);
  const double2 *t = reinterpret_cast<const double2 *>(T[p]);
  int64_t L = len[p];
  double acc[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  for (int64_t i = threadIdx.x; i < L; i += blockDim.x) {
    double2 y0 = y[i], y1 = y[L + i], t0 = t[i], t1 = t[L + i];
    // y_s * conj(t_s')
    acc[0] += y0.x * t0.x + y0.y * t0.y; acc[1] += y0.y * t0.x - y0.x * t0.y;
    acc[2] += y0.x * t1.x + y0.y * t1.y; acc[3] += y0.y * t1.x - y0.x * t1.y;
    acc[4] += y1.x * t0.x + y1.y * t0.y; acc[5] += y1.y * t0.x - y1.x * t0.y;
    acc[6] += y1.x * t1.x + y1.y * t1.y; acc[7] += y1.y * t1.x - y1.x * t1.y;
  }
  for (int k = 0; k < 8; ++k) {
    double s = block_sum<256>(acc[k], sh);
    if (threadIdx.x == 0) rho[(size_t)p * 8 + k] = s;
  }
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
    HIPCHK(hipFuncSetAttribute((const void *)eigh_jacobi_kernel<true>,
                               hipFuncAttributeMaxDynamicSharedMemorySize, 140 * 1024));
    HIPCHK(hipFuncSetAttribute((const void *)eigh_jacobi_log_kernel,
                               hipFuncAttributeMaxDynamicSharedMemorySize, 140 * 1024));
  }
  ~HipBackend() override {
    for (auto &e : ev_)
      if (e) hipEventDestroy(e);
    if (gws_) HIPCHK(hipFree(gws_));
    if (skws_) HIPCHK(hipFree(skws_));
    if (cws_) HIPCHK(hipFree(cws_));
    if (lws_) HIPCHK(hipFree(lws_));
    if (own_) hipStreamDestroy(s_);
  }
  void *alloc(size_t bytes) override {
    void *p = nullptr;
    hipError_t e = hipMalloc(&p, bytes);
    if (e != hipSuccess) {
      if (err_ == 0) { err_ = -4; errmsg_ = "hipMalloc failed (out of device memory)"; }
      return nullptr;
    }
    HIPCHK(hipMemsetAsync(p, 0, bytes, s_));
    return p;
  }
  void release(void *p) override {
    if (p) {
      HIPCHK(hipStreamSynchronize(s_));
      HIPCHK(hipFree(p));
    }
  }
  void h2d(void *d, const void *h, size_t b) override {
    if (b) HIPCHK(hipMemcpyAsync(d, h, b, hipMemcpyHostToDevice, s_));
    HIPCHK(hipStreamSynchronize(s_));
  }
  void d2h(void *h, const void *d, size_t b) override {
    if (b) HIPCHK(hipMemcpyAsync(h, d, b, hipMemcpyDeviceToHost, s_));
    HIPCHK(hipStreamSynchronize(s_));
  }
  void d2d(void *d, const void *s, size_t b) override {
    if (b) HIPCHK(hipMemcpyAsync(d, s, b, hipMemcpyDeviceToDevice, s_));
  }
  void zero(void *d, size_t b) override { if (b) HIPCHK(hipMemsetAsync(d, 0, b, s_)); }
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
    if (prof_) {
      HIPCHK(hipEventCreate(&e0));
      HIPCHK(hipEventCreate(&e1));
      HIPCHK(hipEventRecord(e0, s_));
    }
    // split K when the output alone cannot fill the machine
    int blocks = tiles * d.batch * nprob;
    int ksplit = 1, kchunk = d.K;
    if (blocks < 512 && d.K >= 512) {
      int want = std::min((512 + blocks - 1) / blocks, d.K / 256);
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
      hipLaunchKernelGGL(gemm_kernel<float>, grid, dim3(256), 0, s_, d, A, B, C, ksplit, kchunk,
                         W);
      launch_check("gemm_kernel<float>");
    } else {
      stale_check("gemm_kernel<double>");
      hipLaunchKernelGGL(gemm_kernel<double>, grid, dim3(256), 0, s_, d, A, B, C, ksplit, kchunk,
                         W);
      launch_check("gemm_kernel<double>");
    }
    if (prof_) {
      HIPCHK(hipEventRecord(e1, s_));
      prof_ev_.push_back({e0, e1});
      prof_flops_ += 8.0 * d.M * d.N * (double)d.K * d.batch * nprob;
    }
    if (ksplit > 1) {
      int bx = std::min(64, (int)((d.M * (size_t)d.N + 255) / 256));
      stale_check("gemm_reduce_kernel");
      hipLaunchKernelGGL(gemm_reduce_kernel, dim3(bx, d.batch, nprob), dim3(256), 0, s_, d, C,
                         ksplit, (const double2 *)W);
      launch_check("gemm_reduce_kernel");
    }
  }
  void *splitk_ws(size_t need) {
    if (need > skws_bytes_) {
      HIPCHK(hipStreamSynchronize(s_));
      if (skws_) HIPCHK(hipFree(skws_));
      skws_ = nullptr;
      skws_bytes_ = 0;
      if (hipMalloc(&skws_, need) != hipSuccess) {
        err_ = -4;
        errmsg_ = "split-K workspace allocation failed";
        return nullptr;
      }
      skws_bytes_ = need;
    }
    return skws_;
  }
  void gemm_profile(bool enable) override {
    prof_ = enable;
    if (enable) {
      drain_profile();
      prof_launches_ = 0;
      prof_ms_ = 0;
      prof_flops_ = 0;
    }
  }
  void gemm_profile_read(long *launches, double *ms, double *flops) override {
    drain_profile();
    if (launches) *launches = prof_launches_;
    if (ms) *ms = prof_ms_;
    if (flops) *flops = prof_flops_;
  }
  void drain_profile() {
    for (auto &pr : prof_ev_) {
      HIPCHK(hipEventSynchronize(pr.second));
      float ms = 0;
      HIPCHK(hipEventElapsedTime(&ms, pr.first, pr.second));
      prof_ms_ += ms;
      prof_launches_ += 1;
      HIPCHK(hipEventDestroy(pr.first));
      HIPCHK(hipEventDestroy(pr.second));
    }
    prof_ev_.clear();
  }
  void eigh(int n, int lda, const double *const *in, double *const *evals, double *const *vecs,
            int nprob) override {
    if (nprob <= 0) return;
    int np = n + (n & 1);
    if (np <= 64) {
      size_t sm = (size_t)2 * np * np * sizeof(double2);
      stale_check("eigh_jacobi_kernel");
      hipLaunchKernelGGL(eigh_jacobi_kernel<true>, dim3(nprob), dim3(1024), sm, s_, n, lda, in,
                         evals, vecs, (double2 *)nullptr, 60);
    } else if (np <= 128) {
      const int sweeps = 24;
      size_t logb = (size_t)nprob * sweeps * (np - 1) * (np / 2) * sizeof(double4_t);
      size_t need = logb + (size_t)nprob * np * sizeof(double) + (size_t)nprob * sizeof(int);
      if (need > lws_bytes_) {
        HIPCHK(hipStreamSynchronize(s_));
        if (lws_) HIPCHK(hipFree(lws_));
        lws_ = nullptr;
        lws_bytes_ = 0;
        if (hipMalloc(&lws_, need) != hipSuccess) {
          err_ = -4;
          errmsg_ = "eigh rotation log allocation failed";
          return;
        }
        lws_bytes_ = need;
      }
      size_t sm = std::max((size_t)np * (np + 1) / 2, (size_t)64 * np) * sizeof(double2);
      stale_check("eigh_jacobi_log_kernel");
      double *mdiag = (double *)((char *)lws_ + logb);
      int *mrounds = (int *)(mdiag + (size_t)nprob * np);
      hipLaunchKernelGGL(eigh_jacobi_log_kernel, dim3(nprob), dim3(1024), sm, s_, n, lda, in,
                         evals, vecs, (double4_t *)lws_, sweeps, mdiag, mrounds);
      launch_check("eigh_jacobi_log_kernel");
      stale_check("eigh_replay_kernel");
      hipLaunchKernelGGL(eigh_replay_kernel, dim3((np + 15) / 16, nprob), dim3(256), 0, s_, n,
                         (const double4_t *)lws_, sweeps, (const double *)mdiag,
                         (const int *)mrounds, evals, vecs);
    } else {
      size_t need = (size_t)nprob * 2 * np * np * sizeof(double2);
      if (need > gws_bytes_) {
        HIPCHK(hipStreamSynchronize(s_));
        if (gws_) HIPCHK(hipFree(gws_));
        gws_ = nullptr;
        if (hipMalloc(&gws_, need) != hipSuccess) {
          err_ = -4;
          errmsg_ = "eigh workspace allocation failed";
          gws_bytes_ = 0;
          return;
        }
        gws_bytes_ = need;
      }
      stale_check("eigh_jacobi_kernel");
      hipLaunchKernelGGL(eigh_jacobi_kernel<false>, dim3(nprob), dim3(1024), 0, s_, n, lda, in,
                         evals, vecs, (double2 *)gws_, 60);
    }
    launch_check("eigh_jacobi_kernel");
  }
  void rx(double *const *t, const int64_t *half, int nprob, double c, double s) override {
    stale_check("rx_kernel");
    hipLaunchKernelGGL(rx_kernel, dim3(64, nprob), dim3(256), 0, s_, t, half, c, s);
    launch_check("rx_kernel");
  }
  void msg_sqrt(int n, const double *const *ev, const double *const *vec, double *const *X,
                double *const *Xp, double cut, int nprob) override {
    stale_check("msg_sqrt_kernel");
    hipLaunchKernelGGL(msg_sqrt_kernel, dim3(nprob), dim3(256), 0, s_, n, ev, vec, X, Xp, cut);
    launch_check("msg_sqrt_kernel");
  }
  void gram_factor(int n, int r, const double *const *ev, const double *const *vec,
                   double *const *R, double *const *W, double cut, int nprob) override {
    stale_check("gram_factor_kernel");
    hipLaunchKernelGGL(gram_factor_kernel, dim3(nprob), dim3(256), 0, s_, n, r, ev, vec, R, W,
                       cut);
    launch_check("gram_factor_kernel");
  }
  void gram_chol(int n, const double *const *G, double *const *R, double *const *Wsc, double cut,
                 int nprob) override {
    if (nprob <= 0) return;
    size_t need = (size_t)nprob * 3 * n * n * sizeof(double2);
    if (need > cws_bytes_) {
      HIPCHK(hipStreamSynchronize(s_));
      if (cws_) HIPCHK(hipFree(cws_));
      cws_ = nullptr;
      cws_bytes_ = 0;
      if (hipMalloc(&cws_, need) != hipSuccess) {
        err_ = -4;
        errmsg_ = "Cholesky workspace allocation failed";
        return;
      }
      cws_bytes_ = need;
    }
    stale_check("gram_chol_kernel");
    hipLaunchKernelGGL(gram_chol_kernel, dim3(nprob), dim3(1024), 0, s_, n, G, R, Wsc, cut,
                       (double2 *)cws_);
    launch_check("gram_chol_kernel");
  }
  void theta(int rB, int rS, int chi, const double *const *RB, const double *const *RS,
             double *const *Th, double a, double b, double c, double d, int nprob) override {
    int tot = 4 * rB * rS;
    int bx = std::min(1024, (tot + 255) / 256);
    stale_check("theta_kernel");
    hipLaunchKernelGGL(theta_kernel, dim3(bx, nprob), dim3(256), 0, s_, rB, rS, chi, RB, RS, Th,
                       a, b, c, d);
    launch_check("theta_kernel");
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
  void normalize_residual(int chi, double *const *Mn, const double *const *Mo, double *res,
                          int nprob) override {
    stale_check("normalize_residual_kernel");
    hipLaunchKernelGGL(normalize_residual_kernel, dim3(nprob), dim3(256), 0, s_, chi, Mn, Mo,
                       res);
    launch_check("normalize_residual_kernel");
  }
  void reduce_max(const double *x, int n, double *out) override {
    stale_check("reduce_max_kernel");
    hipLaunchKernelGGL(reduce_max_kernel, dim3(1), dim3(256), 0, s_, x, n, out);
    launch_check("reduce_max_kernel");
  }
  void rho_dot(const double *const *Y, const double *const *T, const int64_t *len, double *rho,
               int nprob) override {
    stale_check("rho_dot_kernel");
    hipLaunchKernelGGL(rho_dot_kernel, dim3(nprob), dim3(256), 0, s_, Y, T, len, rho);
    launch_check("rho_dot_kernel");
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
  void *gws_ = nullptr;
  size_t gws_bytes_ = 0;
  hipEvent_t ev_[8] = {};
  void *lws_ = nullptr;
  size_t lws_bytes_ = 0;
  void *cws_ = nullptr;
  size_t cws_bytes_ = 0;
  void *skws_ = nullptr;
  size_t skws_bytes_ = 0;
  bool prof_ = false;
  std::vector<std::pair<hipEvent_t, hipEvent_t>> prof_ev_;
  long prof_launches_ = 0;
  double prof_ms_ = 0, prof_flops_ = 0;
};

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
