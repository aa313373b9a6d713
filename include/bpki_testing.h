/*
 * Test hooks of libbpki: the device primitives every phase of the method is built from, exposed
 * so that each can be checked element by element against an independent host computation, and
 * the MFMA throughput probe that calibrates the roofline.  Not needed to run simulations (see
 * bpki.h).
 *
 * Buffers are host memory holding complex128 values as (re, im) pairs.  The library copies them
 * to the device, runs the primitive on the context's stream and copies the result back.
 * Errors: -1 invalid argument (including a descriptor that would address outside the buffers,
 * checked on the host before any launch), -4 out of memory, -5 device error.
 */
#ifndef BPKI_TESTING_H
#define BPKI_TESTING_H

#include <stddef.h>
#include <stdint.h>

#include "bpki.h"

#ifdef __cplusplus
extern "C" {
#endif

/* C[b][m][n] (=|+=) alpha * sum_k opA(A)[b][m][k] opB(B)[b][k][n] with composite indices:
 * i = i_outer * Xi + i_inner, offset = i_outer * s_o + i_inner * s_i (strides in complex
 * elements); opA/opB conjugate when conjA/conjB.  This is the contraction primitive of every
 * leg absorption, Gram matrix, BP message and environment in the library. */
typedef struct {
  int32_t M, N, K, Mi, Ni, Ki;
  int64_t a_mo, a_mi, a_ko, a_ki;
  int64_t b_ko, b_ki, b_no, b_ni;
  int64_t c_mo, c_mi, c_no, c_ni;
  int64_t a_b, b_b, c_b;
  int32_t batch, conjA, conjB, beta;
  double alpha_re, alpha_im;
  int32_t prec;      /* 0: FP64 MFMA; 1: operands rounded to FP32, FP32 MFMA, FP64 output */
  int32_t herm;      /* 1: the caller guarantees C = A B is Hermitian (M == N, Mi == M, Ni == N,
                        alpha_im == 0, beta == 0): the lower triangle is computed, the diagonal
                        stored real, the upper triangle written as its conjugate mirror
                        (exactly Hermitian output) */
  int32_t store32;   /* operands held on the device as complex FP32 (prec = 1 only): bit 0 A,
                        bit 1 B, bit 2 C; 5 (A, C) and 3 (A, B) are the supported sets.  Host
                        buffers stay complex128 (converted on upload and download). */
} bpki_test_gemm_desc;

/* Runs the FP64 MFMA GEMM on nprob problems; problem p uses A + 2*a_elems*p etc.  C is read
 * (for beta = 1) and overwritten. */
int bpki_test_gemm(bpki_ctx *ctx, const bpki_test_gemm_desc *d, int nprob, const double *A,
                   size_t a_elems, const double *B, size_t b_elems, double *C, size_t c_elems);

/* The fused BP message of a site (Methods, "Belief propagation on a tensor network state", Eq.
 * "MessageTensorSelfConsistency") at chi = 32 or 64, on nprob problems: with Y, T [nprob][y_elems]
 * site-sized tensors and M [nprob][chi][chi],
 *   out[p][b][b'] = sum_{s, x, a} W[b][a] conj(T[p][s ss + b' rs + a qs + x cs]),
 *   W[b][a] = sum_{a0} Y[p][s ss + b rs + a0 qs + x cs] M[p][a0][a],
 * s in {0, 1}, x in [0, xdim), b, b', a, a0 in [0, chi); strides in complex elements; xdim = chi (a
 * degree-3 site, Y holding the chunk leg's message already) or 1 (a degree-2 site, Y = T).  out
 * [nprob][chi][chi] is exactly Hermitian.  precision BPKI_FP64 or BPKI_FP32 (FP32 MFMA); store32 = 1
 * holds Y and T as complex FP32 on the device (BPKI_FP32 only).  pair = 1: no message is applied
 * (M is not read) and out[p][b][b'] = sum_{s, x, a} Y[p][s ss + b rs + a qs + x cs]
 * conj(T[p][s ss + b' rs + a qs + x cs]) for b >= b', its conjugate mirror above: the message when
 * Y and T are the site tensor with the messages of the two summed legs absorbed, one in each. */
int bpki_test_bp_close(bpki_ctx *ctx, int32_t chi, int precision, int store32, int32_t pair,
                       int64_t rs, int64_t qs, int64_t cs, int64_t ss, int32_t xdim, int nprob,
                       const double *Y, const double *T, size_t y_elems, const double *M,
                       double *out);

/* Batched Hermitian eigendecomposition (FP64; cyclic Jacobi for n < 32, Householder
 * tridiagonalisation + divide and conquer otherwise) of nprob n x n matrices (n <= 512):
 * evals [nprob][n] descending, vecs [nprob][n][n] (in/out) with column i the eigenvector of
 * evals[i] for i < ncols (1 <= ncols <= n); from n = 32 up, columns from ncols on keep the
 * values vecs held on entry. */
int bpki_test_eigh(bpki_ctx *ctx, int n, int nprob, int ncols, const double *A, double *evals,
                   double *vecs);

/* Pivoted Cholesky factor of nprob Hermitian PSD n x n Gram matrices G (n <= 512): R [n][n]
 * (R^H R = G, zero rows beyond the numerical rank) and Wsc [n][n] (A Wsc has orthonormal columns
 * when G = A^H A), with pivots stopping at cut * max(diag G). */
int bpki_test_gram_chol(bpki_ctx *ctx, int n, int nprob, const double *G, double cut, double *R,
                        double *Wsc);

/* Achievable MFMA rate on the context's stream: `blocks` workgroups of four waves each run `iters`
 * iterations of twelve independent 16x16x4 MFMA accumulation chains (precision BPKI_FP64:
 * v_mfma_f64_16x16x4f64; BPKI_FP32: v_mfma_f32_16x16x4f32), no memory traffic.  *tflops receives
 * 2048 * 12 * iters * 4 * blocks / elapsed time of the second of two launches. */
int bpki_test_mfma_rate(bpki_ctx *ctx, int precision, int blocks, int iters, double *tflops);

#ifdef __cplusplus
}
#endif
#endif /* BPKI_TESTING_H */
