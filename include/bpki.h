/*
 * bpki — belief-propagation tensor-network simulation of the kicked Ising circuit on MI355X.
 *
 * C ABI of the library (libbpki.so).  Plain C types and pointers only.
 *
 * Method (arXiv 2306.14887, Tindall, Fishman, Stoudenmire, Sels):
 *   One Floquet step applies U(theta_h) = prod_<v,w> exp(+i pi/4 Z_v Z_w) . prod_v exp(-i theta_h X_v/2)
 *   (Eq. "Propagator") to the state |0...0> (Eq. "State").  The state is a tensor network with
 *   the lattice's geometry (Fig. 1).  Every step applies the X rotations exactly, applies the two-site
 *   gates one colour layer at a time by the reduced-tensor simple update in the belief-propagation
 *   gauge, truncating every bond to at most chi (Methods, "The simple update procedure"), regauges
 *   with BP (Methods, "Belief propagation on a tensor network state",
 *   Eq. "MessageTensorSelfConsistency") and reads expectation values off the converged messages
 *   (Eq. "SingleSIte"; a Pauli string's cluster is contracted exactly inside, BP messages closing
 *   the legs that leave it).
 *
 * Conventions shared by all entry points
 *   - Sites are 0-based; an edge is an unordered pair (u, v), u != v.  Every site has degree 1..3.
 *   - colour[e] is a proper edge colouring (edges that share a site differ).  Gate layers run in
 *     ascending colour.  NULL asks the library for the greedy colouring over the edge list sorted by
 *     (min, max) endpoint (smallest colour free at both ends).
 *   - Pauli ops: 1 = X, 2 = Y, 3 = Z.  A string's sites must induce a connected subgraph that is a
 *     tree or has exactly one loop.  A loop cluster (chi <= 64) is contracted as the trace of the
 *     product of its loop sites' chi^2 x chi^2 norm transfer matrices (branches folded in first):
 *     O(m chi^6) for a loop of m sites, with three chi^4-complex work matrices allocated per string;
 *     a cluster that is the whole lattice gives the exact expectation in the state.
 *   - A periodic lattice is passed as its quotient graph (one cell with the periodic edges
 *     closed on itself; it must stay a simple graph): BP on it is BP on the infinite lattice with
 *     translation-invariant messages ("Dynamics of the infinite heavy-hex lattice", Fig. 4: the
 *     5-site heavy-hex cell is a theta graph, two degree-3 sites joined through three bridges).
 *   - All observables are real doubles.
 *
 * Return codes
 *   0 OK;  +1 BP did not reach bp_tol within bp_max_iter at some step (outputs written);
 *  -1 invalid argument; -2 invalid graph; -3 improper colouring; -4 out of memory / over budget;
 *  -5 HIP/device error; -6 cancelled; -7 unknown ticket.  After an error nothing is written to the
 *  outputs and bpki_last_error() describes it.
 *
 * Threading: a context is used by one host thread at a time.
 */
#ifndef BPKI_H
#define BPKI_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct bpki_ctx bpki_ctx;

/* Arithmetic of the bulk contractions.  The state, the gate updates (including the truncation
 * SVD and the message square roots and inverse square roots), the messages, the BP residual and
 * the observables' final ratios are FP64 in every mode.
 * BPKI_FP32: the BP sweeps run on FP32 MFMA over FP32 copies of the site tensors (made once per
 * new state) with FP32 intermediates, FP32 accumulation per K chunk (per workgroup run of chunks in
 * the fused degree-3 closing) and FP64 chunk sums, until
 * the residual reaches the FP32 rounding level (2e-6, or a sweep within 100x of it that gains less
 * than 10%); then FP64 sweeps run to bp_tol, so the fixed point is the FP64 one.  The
 * observables' contractions use FP32 MFMA on the FP64 state.
 * Stated bound: with bp_tol <= 1e-10, every <Z> is within 1e-5 of the FP64 mode (bp_tol 1e-12).
 * Measured: largest deviation 5.0e-7 over the 256 requests of the seeded serving stream
 * (heavy-hex lattices of 29, 65 and 127 qubits, chi 8..64, up to 20 steps, served with packing)
 * and 8e-8 on the 127-qubit chi = 64 lattice; with bp_tol = 1e-8 a request 0.0008 from the
 * Clifford point (flat Schmidt spectra, near-degenerate cuts) deviated by 1.6e-5, so looser
 * tolerances are outside the bound. */
typedef enum {
  BPKI_FP64 = 0,   /* everything FP64 (the parity mode)                                     */
  BPKI_FP32 = 1    /* FP32 MFMA contractions in BP sweeps and observables (see above)       */
} bpki_precision;

typedef struct {
  int32_t n_sites;
  int32_t n_edges;
  const int32_t *edges;        /* [2*n_edges]; host memory; copied by the call                 */
  const int32_t *colour;       /* [n_edges] or NULL (greedy colouring, see above)               */
  double theta_h;              /* X rotation angle: exp(-i theta_h X / 2)                       */
  int32_t depth;               /* Floquet steps, >= 0                                          */
  int32_t chi;                 /* maximum bond dimension, 1..256 (1..128 if two degree-3 sites
                                  share an edge: the truncation eigenproblems have n <= 512)    */
  int32_t precision;           /* bpki_precision                                               */
  double bp_tol;               /* BP stops when max ||M'-M||_F < bp_tol   (e.g. 1e-12)         */
  int32_t bp_max_iter;         /* e.g. 1000                                                     */
  double svd_cutoff;           /* truncation keeps min(chi, #{sigma_i^2 > svd_cutoff*sigma_1^2})
                                  singular values: the cutoff acts on the Schmidt weights
                                  (e.g. 1e-12), which FP64 eigenvalues of Theta^H Theta resolve  */
  double eig_cutoff;           /* inverse square roots keep lambda > eig_cutoff * lambda_max    */
  int32_t n_pauli;             /* Pauli strings measured after the final step                  */
  const int32_t *pauli_offsets;/* [n_pauli+1] CSR offsets into pauli_sites / pauli_ops         */
  const int32_t *pauli_sites;  /* [pauli_offsets[n_pauli]]                                     */
  const uint8_t *pauli_ops;    /* [pauli_offsets[n_pauli]]  1=X 2=Y 3=Z                        */
  int32_t record_every_step;   /* 1: z holds steps 1..depth (+ clifford_steps); 0: final only   */
  int32_t clifford_steps;      /* n' >= 0 steps of U(pi/2)^dagger after the depth steps (the
                                  paper's extended time evolution, "Measuring expectation values":
                                  <Z_i> after them equals the expectation of the Pauli string
                                  U^n'(pi/2) Z_i U^n'(pi/2)^dagger in the state after depth steps).
                                  Each such step applies the gate layers in descending colour with
                                  exp(-i pi/4 ZZ), then exp(+i pi/4 X) on every site, then BP.     */
} bpki_problem;

/* Below, S = depth + clifford_steps is the number of steps run. */
typedef struct {
  double *z;            /* [max(1, record_every_step ? S : 1) * n_sites], row t = step t+1;
                           S = 0 gives one row of ones (the initial state)                     */
  double *pauli;        /* [n_pauli] or NULL if n_pauli == 0 (measured after the last step)     */
  int32_t *bp_iters;    /* optional [S]: BP sweeps run after each step                          */
  double *bp_residual;  /* optional [S]: final BP residual of each step                         */
  double *discarded;    /* optional [S]: sum over the step's gates of the discarded weight      */
  double *bond_entropy; /* optional [max(1, record_every_step ? S : 1) * n_edges]: on the steps
                           z is recorded, the entanglement entropy of every edge in bits,
                           s_e = -sum_i p_i log2 p_i (Eq. "EntanglementEntropy", read with the
                           minus sign and the sum over the chi weights of one bond), where the
                           Schmidt weights p_i are the eigenvalues of M_{u->v}^{1/2} M_{v->u}^T
                           M_{u->v}^{1/2} normalised to unit sum (the BP norm across the edge is
                           Tr(M_{u->v} M_{v->u}^T)); exact on trees without truncation.  FP64
                           in every precision mode.  S = 0 gives one row of zeros.           */
  /* Truncation diagnostics ("The simple update procedure": each gate keeps at most chi values). */
  int32_t *bond_dims;   /* optional [max(1, record_every_step ? S : 1) * n_edges]: the bond
                           dimension of every edge on the steps z is recorded (ones for S = 0) */
  double *min_cut_gap;  /* optional [S]: smallest (sigma_chi - sigma_{chi+1}) / sigma_1 over the
                           step's gates whose bond chi (not svd_cutoff) limited; +inf if none */
  int32_t *degenerate_cuts; /* optional [S]: number of the step's gates with such a gap below
                           1e-10 (near-degenerate cuts: rounding can move the kept subspace,
                           so runs that differ only in rounding may part there)               */
} bpki_result;

/* Fill *p with the defaults (tolerances 1e-12, 1000 sweeps, FP64, record every step). */
void bpki_problem_defaults(bpki_problem *p);

/* Create a context on HIP device `device`.  `hip_stream` is a borrowed hipStream_t (never
 * destroyed by the library) or NULL for a stream owned by the context.  `mem_budget_bytes` caps the
 * device memory the context may hold (0 = no cap).  Returns 0 or a negative code. */
int bpki_create(bpki_ctx **out, int device, void *hip_stream, size_t mem_budget_bytes);
/* Cancels unfinished tickets, stops the serving slots and releases the context.  Sessions
 * still open keep the context's device resources alive; it is freed when the last one is closed.
 * No call other than bpki_session_* on those open sessions may use `ctx` afterwards. */
void bpki_destroy(bpki_ctx *ctx);

/* The caller's device allocator (a framework's caching allocator, a pool) in place of hipMalloc
 * and hipFree for every device buffer of the context: site tensors, messages and workspaces of its
 * solves, sessions and serving slots.
 *   alloc(bytes, stream, user): device memory for use on `stream` (the hipStream_t of the library
 *     that will use it), aligned to 256 bytes, or NULL when there is none (the call that needed it
 *     then fails with -4; a pointer not so aligned goes back to `free` and the call fails with -5).
 *   free(ptr, stream, user): called once the library's work on `stream` has completed, so the
 *     memory may be reused at once; from the host thread that released the buffer (the caller's,
 *     or a serving slot's worker).  Neither callback may call into the library.
 * Both callbacks or neither (NULL, NULL: hipMalloc and hipFree).  Only before the context has
 * taken device memory (no solve, session, submit or test call yet): -1 otherwise.  `user` and the
 * callbacks must stay valid until bpki_destroy has returned and the last session is closed.
 * A failed allocation, like a device error, is sticky: later calls on the context (or on that
 * serving slot) fail too. */
typedef void *(*bpki_alloc_fn)(size_t bytes, void *stream, void *user);
typedef void (*bpki_free_fn)(void *ptr, void *stream, void *user);
int bpki_set_allocator(bpki_ctx *ctx, bpki_alloc_fn alloc, bpki_free_fn free, void *user);

/* Message of the last error on this thread (never NULL). */
const char *bpki_last_error(void);

/* Host-only checks (no device needed): ranges, graph (self loops, duplicates, degree 1..3),
 * colouring, Pauli strings (valid ops, distinct sites, clusters with at most one loop). */
int bpki_validate(const bpki_problem *p);

/* Device bytes a solve of *p holds: site tensors (sum_v 2*chi^deg complex), messages
 * (2 buffers of 2*|E|*chi^2 complex) and workspace.  Host only. */
int bpki_estimate_bytes(const bpki_problem *p, size_t *bytes);

/* Blocking solve.  Inputs are copied; result buffers are caller-owned host memory. */
int bpki_solve(bpki_ctx *ctx, const bpki_problem *p, bpki_result *r);

/* bpki_solve without device allocation, for callers that cannot allocate device memory (tight
 * serving loops, code around graph capture, harnesses that forbid hipMalloc): every device
 * buffer of the call (site tensors, messages, workspaces) comes from one static array of
 * 64 MiB (BPKI_NOALLOC_SCRATCH_BYTES) that the library holds on every device it runs on until the
 * process ends; the context's own stream and pinned staging buffer, made by bpki_create, are used,
 * and nothing is allocated on the device or freed during the call.  Same arguments, results and
 * codes as bpki_solve (same kernels), plus -4 when bpki_estimate_bytes exceeds the array (a
 * 12-site ring up to chi 32, the 29-qubit lattice up to chi 16, 127 qubits up to chi 8 fit) or
 * the array runs out during the call.  The array keeps the previous call's contents; whatever
 * must start at zero is cleared by the call.  Calls on one context are serialised; calls that
 * overlap on one GPU from different contexts race on the same array. */
#define BPKI_NOALLOC_SCRATCH_BYTES (64u << 20)
int bpki_solve_noalloc(bpki_ctx *ctx, const bpki_problem *p, bpki_result *r);

/* ---- Serving: continuous batching -----------------------------------------------------------
 * bpki_submit queues a problem (deep copy) and returns at once with a ticket.  The context runs a
 * fixed number of serving slots, each a worker thread with its own HIP stream.  Admission is in
 * strict arrival order: a free slot takes the problem at the head of the queue once its
 * bpki_estimate_bytes fits the memory budget next to the resident ones (a head that does not fit
 * waits, and the problems behind it with it, until memory frees up; a problem alone on the device
 * is always admitted), so problems that arrive while others run start as slots and memory free
 * up, and the kernels of all resident problems run concurrently on the device.  Results go into caller-owned buffers,
 * which must stay valid until bpki_wait returns or bpki_poll reports done.  A problem that can
 * never fit the budget is rejected with -4 by bpki_submit.
 *
 * Cross-request packing: when a slot takes a problem with chi <= max_chi and depth >= 1 while more
 * problems are queued than other slots are idle (so some would wait anyway), it also takes (in
 * arrival order, within the budget) up to max_requests - 1 queued problems with the same chi,
 * precision, bp_tol, bp_max_iter and cutoffs and a depth no larger than its own; the lattices,
 * theta_h, Pauli strings and record_every_step may differ.  The pack is solved as one problem on
 * the disjoint union of the lattices, so each launch of a gate layer or BP sweep covers all
 * members (small-chi requests are launch-bound alone).  Each member
 * keeps its own BP stopping point (its messages are frozen once its own residual is below
 * bp_tol) and its result is written when its own last step is done; bp_iters reports its own
 * sweeps.  A packed member's result equals its solve alone up to rounding (launch-size dependent
 * split-K sums), which stays far below the FP64 parity tolerance; unpacked problems give results
 * that do not depend on what else is resident (private workspaces, deterministic reductions). */
/* Number of serving slots (1..64, default 8); only before the first bpki_submit. */
int bpki_serving_config(bpki_ctx *ctx, int slots);
/* Packing limits (max_requests 1..64, 1 = no packing; defaults 16 and chi <= 16); only before the
 * first bpki_submit. */
int bpki_serving_packing(bpki_ctx *ctx, int max_requests, int max_chi);
int bpki_submit(bpki_ctx *ctx, const bpki_problem *p, bpki_result *r, uint64_t *ticket);
/* *done = 1 when finished; returns the problem's status (0/+1/negative) once done, else 0. */
int bpki_poll(bpki_ctx *ctx, uint64_t ticket, int *done);
/* Blocks until the problem finishes; returns its status and forgets the ticket. */
int bpki_wait(bpki_ctx *ctx, uint64_t ticket);
/* Cancels a queued or running problem; its bpki_wait returns -6. */
int bpki_cancel(bpki_ctx *ctx, uint64_t ticket);
/* Host steady-clock times (seconds) of a ticket: submitted, started on a slot, finished (0 if not
 * yet).  Valid until bpki_wait forgets the ticket. */
int bpki_ticket_times(bpki_ctx *ctx, uint64_t ticket, double *times3);
/* Number of problems in the pack that ran the ticket (1 = solved alone; 0 until started).
 * Valid until bpki_wait forgets the ticket. */
int bpki_ticket_pack_size(bpki_ctx *ctx, uint64_t ticket, int32_t *size);

/* ---- Sessions: step-by-step access to one resident state -----------------------------------
 * A session holds one problem's tensors and messages on the device.  It exposes each phase of a
 * Floquet step, so that every phase can be checked against an independent implementation, and
 * state import/export (checkpoint / resume).
 *
 * Site tensor v is exported as complex128 (re, im interleaved) in the layout
 *   T_v[s][a_0]...[a_{d-1}],  s in {0,1}, a_i in [0, chi) for the i-th neighbour in ascending site
 *   id, zero beyond the current bond dimension;
 * message u->v (edge e = (edges[2e], edges[2e+1]); index 2e is edges[2e]->edges[2e+1], index 2e+1
 * the reverse) as M[a_ket][a_bra], chi x chi complex128.  Buffers are host memory. */
typedef struct bpki_session bpki_session;

int bpki_session_open(bpki_ctx *ctx, const bpki_problem *p, bpki_session **out);
void bpki_session_close(bpki_session *s);
/* Complex entries of the exported state: sum over sites of 2*chi^deg, and 2*|E|*chi^2. */
int bpki_session_sizes(const bpki_session *s, size_t *tensor_elems, size_t *message_elems);
int bpki_session_get_state(bpki_session *s, double *tensors, double *messages, int32_t *bond_dims);
int bpki_session_set_state(bpki_session *s, const double *tensors, const double *messages,
                           const int32_t *bond_dims);
/* Phases of one Floquet step (paper: "State ansatz" and Methods). */
int bpki_session_apply_rx(bpki_session *s);
int bpki_session_apply_layer(bpki_session *s, int32_t colour, double *discarded);
/* Per edge [n_edges] (host; each may be NULL), for the edges the last apply_layer (or step)
 * updated: kept bond dimension, discarded weight and cut gap (as bpki_result.min_cut_gap, +inf
 * when svd_cutoff set the bond); -1 / NaN for the other edges. */
int bpki_session_layer_cuts(bpki_session *s, int32_t *kept, double *discarded, double *gap);
int bpki_session_bp(bpki_session *s, int32_t max_iter, int32_t *iters, double *residual);
int bpki_session_bp_sweep(bpki_session *s, double *residual);
int bpki_session_observe_z(bpki_session *s, double *z);
/* entropy [n_edges] (host): bond entropies of the current state and messages, as
 * bpki_result.bond_entropy. */
int bpki_session_observe_bond_entropy(bpki_session *s, double *entropy);
/* Explicit symmetric Vidal gauge from the current messages (Methods, "The Vidal gauge"), in
 * place.  For every edge (u, v) with X_u = M_{u->v}^{1/2}, X_v = M_{v->u}^{1/2} and the SVD
 * X_u^T X_v = U S V^H, leg u->v of T_u absorbs X_u^{T+} U W and leg v->u of T_v absorbs
 * X_v^{T+} conj(V) W with W = (S / sum S)^{1/2}: the identity (on the supports of the messages,
 * up to a positive factor) is inserted on every bond, so the state changes only by a positive
 * factor, and a state already in this gauge is left as it is (the transform is idempotent up to
 * the SVD's unitary freedom); each site tensor with W^{-1} removed from its legs (Gamma_v, up to
 * scale) then forms, with S on its other legs, the isometries of Eqs.
 * "IsometryPropertyDefinition" and "IsometryDefinition", and diag(S)/sum(S) on both directions
 * (written as the new messages) is a BP fixed point.  S is normalised to unit 2-norm; singular
 * values with s_i^2 <= svd_cutoff * s_1^2 are dropped (bond dimensions shrink accordingly).  Computed from the
 * eigenpairs of C^H C in FP64 in every mode.  lambda: [n_edges][chi] host, S descending and
 * zero-padded, or NULL.  Equivalent to the message form in exact arithmetic (a conditioning
 * safeguard and the paper's stated representation). */
int bpki_session_vidal_gauge(bpki_session *s, double *lambda);
/* BP error estimate on edge `edge` (Methods, "Estimating the error of BP for general tensor
 * networks", Eq. "BPErrorEstimate"): the state is first brought into the symmetric gauge (as
 * bpki_session_vidal_gauge, left so afterwards), the norm network is cut along the edge and the
 * rest contracted exactly into the chi^2 x chi^2 edge environment E, and
 * error = 1 - sqrt(s_1^2 / sum_i s_i^2) over the singular values s_i of E (0 when the environment
 * is rank one, as BP assumes).  Built for chi <= 16 and three kinds of network, with the rest
 * returning -1:
 *   - `edge` a bridge (its removal disconnects the network): E is an outer product, error 0 and
 *     spectrum (1, 0, ...);
 *   - networks whose 2-core (what remains after removing sites of degree 1 repeatedly) is one
 *     loop, such as one heavy hexagon with or without pendant sites: the branches are contracted
 *     into the loop sites' chi^2 x chi^2 norm transfer matrices and E is their open chain;
 *   - networks whose 2-core is two junction sites joined by three paths, such as two heavy
 *     hexagons sharing a side: the three path chains and the two junction tensors are contracted
 *     exactly (chi^8 complex multiply-adds).
 * spectrum: [chi^2] host, s_i / ||s|| descending, or NULL.  Allocates its work buffers for the
 * call (up to 4 chi^6 complex, 1.1 GB at chi = 16, for the two-junction case). */
int bpki_session_bp_error(bpki_session *s, int32_t edge, double *error, double *spectrum);
int bpki_session_observe_pauli(bpki_session *s, double *pauli);
/* One whole Floquet step: X rotations, all gate layers, BP, then z (may be NULL). */
int bpki_session_step(bpki_session *s, double *z, int32_t *iters, double *residual,
                      double *discarded);
/* One step of U(pi/2)^dagger (see clifford_steps): gate layers in descending colour with
 * exp(-i pi/4 ZZ), X rotations by -pi/2, BP, then z (may be NULL). */
int bpki_session_clifford_inverse_step(bpki_session *s, double *z, int32_t *iters,
                                       double *residual, double *discarded);
/* Total device time of the last bpki_session_step, split by phase (milliseconds): rx, gate layers,
 * BP, observables.  Measured with HIP events on the session's stream. */
int bpki_session_last_timing(const bpki_session *s, double *ms4);
/* Kernel-level timing of the contraction kernels (every contraction of the method runs in them:
 * the complex GEMM kernels and, for the BP messages of degree-2 and degree-3 sites at chi = 64, the
 * fused BP closing): with stride
 * k >= 1, every k-th launch on the session's stream is bracketed by HIP events (each event pair
 * costs a few microseconds of stream time, so a stride above 1 keeps the measurement from slowing
 * the run it measures); stride 0 turns it off.  read returns the bracketed launch count, the
 * summed kernel time in ms and the summed algorithmic flops of those launches (complex
 * multiply-adds at 8 real flops: 8*M*N*K for a GEMM, 8*K*M(M+1)/2 for a Hermitian output, of which
 * only the lower triangle is computed; 8*(2 chi^4 + chi^3 (chi + 1)) per fused degree-3 message,
 * 8*(2 chi^3 + chi^2 (chi + 1)) per fused degree-2 message), and
 * optionally the count of all launches since enabling.  Enabling resets the counters. */
int bpki_session_profile(bpki_session *s, int stride);
int bpki_session_profile_read(bpki_session *s, int64_t *launches, double *ms, double *flops,
                              int64_t *all_launches);
/* The same restricted to the bracketed GEMM launches of one arithmetic, prec 0 = FP64 MFMA,
 * 1 = FP32 MFMA (a mixed-precision session runs both): their count, summed ms and summed flops. */
int bpki_session_profile_read_prec(bpki_session *s, int32_t prec, int64_t *launches, double *ms,
                                   double *flops);
/* The same restricted to one kernel and one arithmetic: kernel 0 = the tiled GEMM (gemm_kernel),
 * 1 = the fused BP closing (bp_close_kernel: a message with its leg absorption, or a pair closing
 * of two absorbed copies, 8*chi^3 (chi + 1) flops per degree-3 message), 2 = the streaming GEMM
 * of the leg contractions (gemm_stream_kernel); prec as above.  bytes (may be NULL): the summed
 * algorithmic HBM bytes of those launches (every operand read once and every output written once;
 * split-K partial sums and re-reads not counted); all_launches (may be NULL): every launch of
 * that kernel and arithmetic since enabling.  The sampling stride counts the launches of each
 * kernel and arithmetic separately. */
int bpki_session_profile_read_kernel(bpki_session *s, int32_t kernel, int32_t prec,
                                     int64_t *launches, double *ms, double *flops, double *bytes,
                                     int64_t *all_launches);

#ifdef __cplusplus
}
#endif
#endif /* BPKI_H */
