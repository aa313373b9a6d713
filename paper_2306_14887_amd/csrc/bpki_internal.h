// Internal interfaces of the bpki library: device backend primitives and the engine.
//
// Data layout in device memory (complex numbers are (re, im) pairs, FP64 unless stated):
//   site tensor T_v : [s][a_0]..[a_{d-1}]  s in {0,1}, every virtual leg padded to chi
//                     (leg i points at the i-th neighbour in ascending id; zero beyond the bond)
//   message u->v    : [a_ket][a_bra], chi x chi, two buffers (BP double buffering)
#pragma once
#include <cstddef>
#include <cstdint>
#include <map>
#include <set>
#include <string>
#include <vector>

namespace bpki {

// C[b][m][n] (=|+=) alpha * sum_k opA(A)[b][m][k] * opB(B)[b][k][n]
// Every index may be composite, i = i_outer * Xi + i_inner, with independent strides for the
// outer and inner part (strides count complex elements).  A list of problems with equal shapes
// and strides is passed as device arrays of base pointers (one launch for all of them).
struct GemmDesc {
  int M = 0, N = 0, K = 0;
  int Mi = 1, Ni = 1, Ki = 1;            // inner extents (M % Mi == 0 ...)
  long a_mo = 0, a_mi = 0, a_ko = 0, a_ki = 0;
  long b_ko = 0, b_ki = 0, b_no = 0, b_ni = 0;
  long c_mo = 0, c_mi = 0, c_no = 0, c_ni = 0;
  long a_b = 0, b_b = 0, c_b = 0;        // batch strides
  int batch = 1;
  int conjA = 0, conjB = 0;
  int beta = 0;                          // 1: accumulate into C
  double alpha_re = 1.0, alpha_im = 0.0;
  int prec = 0;                          // 0: FP64 MFMA; 1: FP32 MFMA (FP64 storage)
  // 1: C = A B is Hermitian (M == N, single-stride M and N, real alpha, beta = 0): only the
  // lower triangle is computed, the diagonal is stored real and the upper triangle is written
  // as the conjugate mirror
  int herm = 0;
  // Storage of the operands (prec = 1 only): 1 = complex FP32 (float pairs) instead of FP64.
  // Supported: A and C FP32 with B FP64 (a leg absorption into an FP32 buffer), and A and B FP32
  // with C FP64 (a closing contraction into a message).
  int a32 = 0, b32 = 0, c32 = 0;
};

// The BP message of a site towards one leg, in one fused pass (chi = 32 or 64):
// out[b][b'] = sum_{s, x, a} W[b][a] conj(T[s; b', a, x]),  W[b][a] = sum_{a0} Y[s; b, a0, x] M[a0][a],
// with Y the site tensor T after the message of the chunk leg x was absorbed (degree 3), or T itself
// with no chunk leg (degree 2: xdim = 1), M the incoming message of the applied leg a and b the
// outgoing leg.  Strides (complex elements) of the
// outgoing, applied and chunk legs (one set per group of `group` consecutive problems, up to three
// sets: the three outgoing legs of a site in one launch) and of s, shared by Y and T.  The output is
// exactly Hermitian (lower triangle summed, upper triangle its mirror, real diagonal).
struct BpCloseDesc {
  int chi = 64;
  int nsets = 1, group = 1;              // problem p uses stride set min(p / group, nsets - 1)
  long rs[3] = {0, 0, 0}, qs[3] = {0, 0, 0}, cs[3] = {0, 0, 0};
  long ss = 0;
  int xdim = 64;                         // extent of the chunk leg (chi), or 1 without one
  int prec = 0;                          // 0: FP64 MFMA; 1: FP32 MFMA
  int s32 = 0;                           // Y and T stored as complex FP32 (prec = 1 only)
  // 1: out[b][b'] = sum over chunks of sum_a Y[b][a] conj(T[b'][a]) with T (the second tensor) a
  // second absorbed copy of the site tensor and no message applied (M unused)
  int pair = 0;
};
// The bond dimensions the fused closing is built for.
inline bool bp_close_chi(int chi) { return chi == 64 || chi == 32; }

// Simple composite-index helpers for descriptors.
inline void set_simple_m(GemmDesc &d, int M, long sa, long sc) { d.M = M; d.Mi = M; d.a_mi = sa; d.c_mi = sc; }

enum class Prec : int { F64 = 0, F32 = 1 };

// A caller's device allocator: memory for use on `stream`, and its return once that stream is idle.
typedef void *(*DevAlloc)(size_t bytes, void *stream, void *user);
typedef void (*DevFree)(void *ptr, void *stream, void *user);

// Small device kernels used by the engine (implemented in hip_backend.hip).
struct Backend {
  virtual ~Backend() {}
  // Route every device allocation of this backend through (a, f); -1 once it holds device memory.
  virtual int set_allocator(DevAlloc a, DevFree f, void *user) = 0;
  virtual void *alloc(size_t bytes) = 0;          // zero-initialised
  virtual void release(void *p) = 0;
  // Forget the cached workspaces without freeing them (their memory is an arena the caller
  // resets), and clear an allocation failure (a device error stays).
  virtual void forget_workspaces() = 0;
  virtual void clear_alloc_error() = 0;
  virtual void h2d(void *dst, const void *src, size_t bytes) = 0;
  virtual void d2h(void *dst, const void *src, size_t bytes) = 0;
  // One double read in stream order into slot 0 or 1 without waiting; wait_read(slot) returns it
  // once the stream has reached that read.
  virtual void read_async(const double *src, int slot) = 0;
  virtual double wait_read(int slot) = 0;
  virtual void d2d(void *dst, const void *src, size_t bytes) = 0;
  virtual void sync() = 0;
  virtual int check(std::string *msg) = 0;          // 0 or negative error code
  // HIP events on the backend's stream: mark slot i; elapsed milliseconds between two marks.
  virtual void timer_mark(int slot) = 0;
  virtual double timer_ms(int a, int b) = 0;
  // Per-launch GEMM timing (HIP events around every gemm launch while enabled).  read() returns
  // the number of launches, their summed duration (ms) and summed 8*M*N*K*batch*nprob flops.
  // GEMM timing: stride 0 = off, k >= 1 = bracket every k-th launch with HIP events (all
  // launches are counted).  read: bracketed launches, all launches, their ms and 8MNK flops.
  virtual void gemm_profile(int stride) = 0;
  virtual void gemm_profile_read(long *sampled, long *all, double *ms, double *flops) = 0;
  // the same for the bracketed launches of one arithmetic (0 FP64 MFMA, 1 FP32 MFMA)
  virtual void gemm_profile_read_prec(int prec, long *sampled, double *ms, double *flops) = 0;
  // kernel 0: gemm_kernel, 1: the fused BP closing (bp_close_kernel), 2: gemm_stream_kernel; prec
  // as above; bytes: the sampled launches' algorithmic HBM bytes (operands read once, outputs
  // written once); all: every launch of that kernel and arithmetic since enabling
  virtual void gemm_profile_read_kernel(int kernel, int prec, long *sampled, double *ms,
                                        double *flops, double *bytes, long *all) = 0;

  // complex FP64 grouped GEMM; A/B/C are device arrays of nprob pointers to double pairs
  virtual void gemm(const GemmDesc &d, const double *const *A, const double *const *B,
                    double *const *C, int nprob) = 0;
  // Fused BP closings of nprob messages (BpCloseDesc); out: FP64 chi x chi messages.
  virtual void bp_close(const BpCloseDesc &d, const double *const *Y, const double *const *T,
                        const double *const *M, double *const *out, int nprob) = 0;
  // Batched Hermitian eigendecomposition (FP64).  in[p]: n x n (lda), read only; its Hermitian
  // part is used.
  // evals[p]: n reals, descending; vecs[p]: n x n, column i = eigenvector i (ld = n), written
  // for the ncols largest eigenvalues (columns from ncols on are left as they were; n >= 32).
  virtual void eigh(int n, int lda, const double *const *in, double *const *evals,
                    double *const *vecs, int nprob, int ncols) = 0;

  // --- elementwise / small kernels -------------------------------------------------------
  // T_v <- RX(theta) on the physical leg for all sites; tensors[p] holds 2*half[p] complex.
  virtual void rx(double *const *tensors, const int64_t *half, int nprob, double c, double s) = 0;
  // X = W f(l) W^H with f = sqrt(max(l,0)) and Xp with f = 1/sqrt(l) for l > cut*l_max else 0.
  virtual void msg_sqrt(int n, const double *const *evals, const double *const *vecs,
                        double *const *X, double *const *Xp, double cut, int nprob) = 0;
  // Entropy -sum p log2 p of the Schmidt weights p = max(evals, 0) / sum (n per problem); out
  // [nprob] device, NaN for an all-zero spectrum.
  virtual void bond_entropy(int n, const double *const *evals, double *out, int nprob) = 0;
  // out[0..1] = trace of the n x n complex matrix R (device).
  virtual void trace(const double *R, int n, double *out) = 0;
  // Symmetric Vidal gauge factors of nprob edges from the eigenpairs of C^H C (C = X^T Y):
  // D1 = V diag(s^{1/2} / lambda), D2 = conj(V) diag(s^{1/2}) (s = lambda above cut * lambda_1,
  // unit 2-norm), both messages of the edge set to diag(s) / sum(s); lam [nprob][n] = s,
  // kept [nprob] (device).
  virtual void vidal_svd(int n, const double *const *evals, const double *const *vecs,
                         double *const *D1, double *const *D2, double *const *Mu,
                         double *const *Mv, double *lam, int *kept, double cut, int nprob) = 0;
  // Pivoted Cholesky factor of a Gram matrix G = A^H A (n x n, Hermitian PSD):
  // G[p][p] = L L^H for a pivot order p, stopping at the first pivot <= cut * max(diag G).
  // Writes R = L^H P^T (n x n, zero rows beyond the rank) and Wsc = P [L1^{-H}; 0] (n x n), so
  // that R^H R = G and Q = A Wsc has orthonormal columns.
  virtual void gram_chol(int n, const double *const *G, double *const *R, double *const *Wsc,
                         double cut, int nprob) = 0;
  // Theta[(rb,sb)][(rs,ss)] = g(sb,ss) sum_b RB[rb][sb][b] RS[rs][ss][b];  chi = bond extent
  virtual void theta(int rB, int rS, int chi, const double *const *RB, const double *const *RS,
                     double *const *Th, double g_same_re, double g_same_im, double g_diff_re,
                     double g_diff_im, int nprob) = 0;
  // Truncation from eigh(Theta^H Theta): k = min(chi, #{lambda_i > cutoff * lambda_1}), S,
  // new diagonal messages and the scaled right vectors Vs[c][a] = V[c][a]/sigma_a (a < k);
  // disc[2p] = discarded weight, disc[2p+1] = (sigma_k - sigma_{k+1}) / sigma_1 when chi (not the
  // cutoff) set k, else +inf.
  virtual void svd_finish(int n, int chi, const double *const *evals, const double *const *vecs,
                          double *const *Vs, double *const *S, int *kout, double *disc,
                          double *const *msg_a, double *const *msg_b, double cutoff,
                          int nprob) = 0;
  // RB'[(r,s)][a] = U[(r,s)][a] sqrt(S_a); RS'[(r,s)][a] = sqrt(S_a) conj(V[(r,s)][a]); a < chi
  virtual void split_sqrt(int rowsB, int rowsS, int n, int chi, const double *const *U,
                          const double *const *V, const double *const *S, double *const *RBn,
                          double *const *RSn, int nprob) = 0;
  // dst[i] = (float)src[i] for n complex elements (the FP32 copy of the site tensors).
  virtual void to_f32(const double *src, float *dst, size_t n) = 0;
  // BP: M_new <- M_new / tr(M_new); res[p] = ||M_new - M_old||_F.
  virtual void normalize_residual(int chi, double *const *Mnew, const double *const *Mold,
                                  double *res, int nprob) = 0;
  virtual void reduce_max(const double *x, int n, double *out) = 0;
  // Packed solves: out[j] = max of res[idx[k]] over k in [off[j], off[j+1]), and
  // act_next[j] = act[j] && !(out[j] < tol).
  virtual void member_residual(const double *res, const int *off, const int *idx, int nmem,
                               const int *act, int *act_next, double tol, double *out) = 0;
  // M[m] <- Mn[m] (elems complex each) for every message m whose member is active.
  virtual void commit_messages(double *M, const double *Mn, long elems, int nmsg,
                               const int *msg_member, const int *act) = 0;
  // Throughput of a loop of independent 16x16x4 MFMAs (no memory traffic) on this stream, in
  // TFLOP/s: prec 0 = FP64, 1 = FP32; `blocks` workgroups of four waves, `iters` iterations.
  virtual double mfma_rate(int prec, int blocks, int iters) = 0;
  // rho[p][s][s'] = sum_i Y[p][s][i] conj(T[p][s'][i]) over i < len[p]; out 4 complex per p.
  virtual void rho_dot(const double *const *Y, const double *const *T, const int64_t *len,
                       double *rho, int nprob) = 0;
  // T'[s] = sum_s' O[s][s'] T[s'] for a 2 x half tensor (one 2x2 complex op per problem)
  virtual void apply_op(const double *const *Tin, double *const *Tout, const int64_t *half,
                        const double *ops, int nprob) = 0;
};

Backend *make_hip_backend(int device, void *stream, std::string *err);

// The allocation-free solve's device memory: a static array of kScratchBytes per device; its
// address on `device`, which must be current (0, or -5 with *err set).
constexpr size_t kScratchBytes = size_t(64) << 20;
int scratch_region(int device, void **ptr, std::string *err);

// ------------------------------------------------------------------------------------------
struct Problem {
  int n_sites = 0;
  std::vector<int> edges;       // 2E
  std::vector<int> colour;      // E
  double theta = 0;
  int depth = 0, chi = 1;
  int precision = 0;            // 0 FP64; 1 FP32 contractions in BP sweeps and observables
  double bp_tol = 1e-12;
  int bp_max_iter = 1000;
  double svd_cutoff = 1e-12, eig_cutoff = 1e-12;
  std::vector<int> pauli_offsets, pauli_sites;
  std::vector<uint8_t> pauli_ops;
  int record_every_step = 1;
  int clifford_steps = 0;       // steps of U(pi/2)^dagger after the depth steps at theta
  // Packed solves (several requests on the disjoint union of their lattices): the X angle of
  // every site (empty: theta everywhere) and the first site of each member followed by n_sites
  // (empty: a single member).  Members are contiguous site ranges with contiguous edge ranges.
  std::vector<double> site_theta;
  std::vector<int> member_site0;
};

// Host-side graph plan (degrees, neighbours, layers) and device workspace sizes.
struct Plan;
struct EngineScratch;      // device buffers of one host-driven contraction

class Engine {
 public:
  Engine(Backend *be, const Problem &p);
  ~Engine();
  static size_t estimate_bytes(const Problem &p);

  void reset();                                   // |0...0>, messages [[1]]
  void apply_rx();
  void apply_rx_angle(double theta);              // the same X angle on every site
  // zz_sign = -1 applies exp(-i pi/4 ZZ), the gates of U(pi/2)^dagger; returns discarded weight
  double apply_layer(int colour, int zz_sign = 1);
  double bp_sweep();                              // returns residual
  int bp(int max_iter, double *residual);         // returns sweeps
  void observe_z(double *z);                      // host out [n_sites]
  void observe_pauli(double *out);                // host out [n_pauli]
  void observe_pauli_range(int k0, int k1, double *out);   // strings k0 .. k1-1
  void observe_entropy(double *out);              // host out [n_edges]: bond entropies (bits)
  void vidal_gauge(double *lambda);               // in place; host out [n_edges][chi] or NULL
  // BP error estimate on edge e (symmetric gauge first); spectrum [chi^2] or NULL.  Built for
  // bridges, networks whose 2-core is one loop and networks whose 2-core is two junction sites
  // joined by three paths; -1 for other networks.
  double bp_error(int e, double *spectrum);
  // Packed solves: sweeps until every member's residual is below bp_tol.  A member's messages
  // are frozen after the sweep that brought its own residual below the tolerance, so each member
  // follows its own BP schedule; per member: sweeps and final residual.
  void bp_members(int max_iter, int *sweeps, double *residual);
  int n_members() const;
  // Every edge of the last apply_layer: its kept bond dimension, discarded weight and cut gap
  // (sigma_k - sigma_{k+1}) / sigma_1 when chi limited the bond (+inf when the cutoff did).
  struct Cut {
    int e = -1, kept = 0;
    double discarded = 0, gap = 0;
  };
  const std::vector<Cut> &layer_cuts() const { return layer_cuts_; }
  // Current bond dimension of every edge (host copy).
  const std::vector<int> &bond_dims() const;
  int n_colours() const;
  const Problem &problem() const { return prob_; }

  size_t tensor_elems() const;
  size_t message_elems() const;
  void get_state(double *tensors, double *messages, int32_t *bond_dims);
  void set_state(const double *tensors, const double *messages, const int32_t *bond_dims);

 private:
  Backend *be_;
  Problem prob_;
  Plan *plan_;
  int bp_prec_ = 0;
  bool t32_stale_ = true;         // the FP32 copy of the site tensors needs refreshing
  std::vector<Cut> layer_cuts_;
  void sweep_classes();
  // The gate updates stay FP64 in every mode: the Gram-based bond isolation amplifies rounding
  // by the condition number of the isolated tensor, which FP32 cannot absorb.
  int su_prec() const { return 0; }
  void build();
  double pauli_value(int k, bool with_ops);
  // Pieces of the host-driven exact contractions (Pauli strings, BP error estimate).
  struct OpenLeg {                // chi^2 matrices X_x[a][a'] = base[x sx + a sk + a' sn]
    const double *base;
    long sx, sk, sn;
  };
  double *site_ket(int v, int opcode, EngineScratch &S);
  double *branch_env(int v, int parent, const std::set<int> &cs, const std::map<int, int> &op,
                     EngineScratch &S);
  void site_transfer(int v, int prev, int next, const std::set<int> &cs,
                     const std::map<int, int> &op, EngineScratch &S, double *dst,
                     const OpenLeg *open);
  std::vector<int> cycle_of(const std::set<int> &cs) const;
  double *chain(const std::vector<int> &walk, int before, int after, EngineScratch &S);
};

}  // namespace bpki
