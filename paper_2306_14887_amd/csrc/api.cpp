// C ABI of libbpki: validation, memory estimate, blocking solves, sessions and serving.
#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <set>
#include <string>
#include <thread>
#include <vector>

#include "../../include/bpki.h"
#include "../../include/bpki_testing.h"
#include "bpki_internal.h"

using namespace bpki;

static_assert(kScratchBytes == BPKI_NOALLOC_SCRATCH_BYTES, "scratch size differs from the header");

static thread_local std::string g_err;

// A chi-limited cut whose gap (sigma_chi - sigma_{chi+1}) / sigma_1 is below this is reported as
// near-degenerate: there the kept subspace moves with rounding.
static constexpr double kDegenerateGap = 1e-10;

static int fail(int code, const std::string &msg) {
  g_err = msg;
  return code;
}

extern "C" const char *bpki_last_error(void) { return g_err.c_str(); }

extern "C" void bpki_problem_defaults(bpki_problem *p) {
  std::memset(p, 0, sizeof(*p));
  p->theta_h = 0.0;
  p->depth = 1;
  p->chi = 8;
  p->precision = BPKI_FP64;
  p->bp_tol = 1e-12;
  p->bp_max_iter = 1000;
  p->svd_cutoff = 1e-12;
  p->eig_cutoff = 1e-12;
  p->record_every_step = 1;
}

// Greedy proper edge colouring over the edges sorted by (min, max) endpoint.
static std::vector<int> greedy_colouring(int n, const int32_t *edges, int E) {
  std::vector<int> order(E);
  for (int i = 0; i < E; ++i) order[i] = i;
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
    int a0 = std::min(edges[2 * a], edges[2 * a + 1]), a1 = std::max(edges[2 * a], edges[2 * a + 1]);
    int b0 = std::min(edges[2 * b], edges[2 * b + 1]), b1 = std::max(edges[2 * b], edges[2 * b + 1]);
    return a0 != b0 ? a0 < b0 : a1 < b1;
  });
  std::vector<std::set<int>> used(n);
  std::vector<int> col(E, -1);
  for (int i : order) {
    int u = edges[2 * i], v = edges[2 * i + 1];
    int c = 0;
    while (used[u].count(c) || used[v].count(c)) ++c;
    col[i] = c;
    used[u].insert(c);
    used[v].insert(c);
  }
  return col;
}

extern "C" int bpki_validate(const bpki_problem *p) {
  if (!p) return fail(-1, "problem is NULL");
  if (p->n_sites < 1) return fail(-1, "n_sites must be >= 1");
  if (p->n_edges < 1) return fail(-2, "the lattice needs at least one edge");
  if (!p->edges) return fail(-1, "edges is NULL");
  if (!std::isfinite(p->theta_h)) return fail(-1, "theta_h must be finite");
  if (p->depth < 0) return fail(-1, "depth must be >= 0");
  if (p->chi < 1 || p->chi > 256) return fail(-1, "chi must be in 1..256");
  if (p->precision != BPKI_FP64 && p->precision != BPKI_FP32)
    return fail(-1, "precision must be BPKI_FP64 or BPKI_FP32");
  if (!std::isfinite(p->bp_tol) || p->bp_tol < 0) return fail(-1, "bp_tol must be finite, >= 0");
  if (p->bp_max_iter < 1) return fail(-1, "bp_max_iter must be >= 1");
  if (!std::isfinite(p->svd_cutoff) || p->svd_cutoff < 0 || !std::isfinite(p->eig_cutoff) ||
      p->eig_cutoff < 0)
    return fail(-1, "cutoffs must be finite and >= 0");
  if (p->record_every_step != 0 && p->record_every_step != 1)
    return fail(-1, "record_every_step must be 0 or 1");
  if (p->clifford_steps < 0) return fail(-1, "clifford_steps must be >= 0");
  const int n = p->n_sites, E = p->n_edges;
  std::vector<int> deg(n, 0);
  std::set<std::pair<int, int>> seen;
  for (int e = 0; e < E; ++e) {
    int u = p->edges[2 * e], v = p->edges[2 * e + 1];
    if (u < 0 || v < 0 || u >= n || v >= n) return fail(-2, "edge endpoint out of range");
    if (u == v) return fail(-2, "self loop");
    if (!seen.insert({std::min(u, v), std::max(u, v)}).second) return fail(-2, "duplicate edge");
    deg[u]++;
    deg[v]++;
  }
  for (int v = 0; v < n; ++v)
    if (deg[v] < 1 || deg[v] > 3) return fail(-2, "every site must have degree 1..3");
  // the truncated SVD of a gate block between two degree-3 sites is a 4chi x 4chi problem
  for (int e = 0; e < E; ++e)
    if (deg[p->edges[2 * e]] == 3 && deg[p->edges[2 * e + 1]] == 3 && p->chi > 128)
      return fail(-1, "chi must be <= 128 when two degree-3 sites share an edge");
  if (p->colour) {
    std::vector<std::set<int>> used(n);
    for (int e = 0; e < E; ++e) {
      int c = p->colour[e];
      if (c < 0) return fail(-3, "negative colour");
      int u = p->edges[2 * e], v = p->edges[2 * e + 1];
      if (used[u].count(c) || used[v].count(c)) return fail(-3, "improper edge colouring");
      used[u].insert(c);
      used[v].insert(c);
    }
  }
  if (p->n_pauli < 0) return fail(-1, "n_pauli must be >= 0");
  if (p->n_pauli > 0) {
    if (!p->pauli_offsets || !p->pauli_sites || !p->pauli_ops)
      return fail(-1, "Pauli arrays are NULL");
    if (p->pauli_offsets[0] != 0) return fail(-1, "pauli_offsets[0] must be 0");
    for (int k = 0; k < p->n_pauli; ++k) {
      int b = p->pauli_offsets[k], e = p->pauli_offsets[k + 1];
      if (e <= b) return fail(-1, "empty or decreasing Pauli string");
      std::set<int> s;
      for (int i = b; i < e; ++i) {
        int q = p->pauli_sites[i];
        if (q < 0 || q >= n) return fail(-1, "Pauli site out of range");
        if (!s.insert(q).second) return fail(-1, "repeated site in a Pauli string");
        if (p->pauli_ops[i] < 1 || p->pauli_ops[i] > 3) return fail(-1, "Pauli op must be 1..3");
      }
      // induced subgraph: connected with |S| - 1 edges (a tree) or |S| edges (one loop)
      int m = 0;
      std::map<int, std::vector<int>> adj;
      for (int ed = 0; ed < E; ++ed) {
        int u = p->edges[2 * ed], v = p->edges[2 * ed + 1];
        if (s.count(u) && s.count(v)) {
          ++m;
          adj[u].push_back(v);
          adj[v].push_back(u);
        }
      }
      if (m != (int)s.size() - 1 && m != (int)s.size())
        return fail(-1, "Pauli cluster must induce a tree or a graph with one loop");
      if (m == (int)s.size() && p->chi > 64)
        return fail(-1, "a Pauli cluster with a loop needs chi <= 64");
      std::set<int> vis;
      std::vector<int> st{*s.begin()};
      while (!st.empty()) {
        int x = st.back();
        st.pop_back();
        if (!vis.insert(x).second) continue;
        for (int y : adj[x]) st.push_back(y);
      }
      if (vis.size() != s.size()) return fail(-1, "Pauli cluster is not connected");
    }
  }
  return 0;
}

static Problem to_problem(const bpki_problem *p) {
  Problem q;
  q.n_sites = p->n_sites;
  q.edges.assign(p->edges, p->edges + 2 * p->n_edges);
  if (p->colour) q.colour.assign(p->colour, p->colour + p->n_edges);
  else q.colour = greedy_colouring(p->n_sites, p->edges, p->n_edges);
  q.theta = p->theta_h;
  q.depth = p->depth;
  q.chi = p->chi;
  q.precision = p->precision;
  q.bp_tol = p->bp_tol;
  q.bp_max_iter = p->bp_max_iter;
  q.svd_cutoff = p->svd_cutoff;
  q.eig_cutoff = p->eig_cutoff;
  q.record_every_step = p->record_every_step;
  q.clifford_steps = p->clifford_steps;
  if (p->n_pauli > 0) {
    q.pauli_offsets.assign(p->pauli_offsets, p->pauli_offsets + p->n_pauli + 1);
    int tot = p->pauli_offsets[p->n_pauli];
    q.pauli_sites.assign(p->pauli_sites, p->pauli_sites + tot);
    q.pauli_ops.assign(p->pauli_ops, p->pauli_ops + tot);
  } else {
    q.pauli_offsets.assign(1, 0);
  }
  return q;
}

extern "C" int bpki_estimate_bytes(const bpki_problem *p, size_t *bytes) {
  int rc = bpki_validate(p);
  if (rc) return rc;
  if (!bytes) return fail(-1, "bytes is NULL");
  *bytes = Engine::estimate_bytes(to_problem(p));
  return 0;
}

// ------------------------------------------------------------------------------------------
// Bump allocator over the static scratch array of bpki_solve_noalloc: reset at the start of every
// call, frees are no-ops (the whole region is reused by the next call).
struct ScratchArena {
  char *base = nullptr;
  size_t size = 0, top = 0;
};

static void *arena_alloc(size_t bytes, void *, void *user) {
  ScratchArena *a = static_cast<ScratchArena *>(user);
  const size_t n = (bytes + 255) & ~size_t(255);
  if (!a->base || n > a->size - a->top) return nullptr;
  void *p = a->base + a->top;
  a->top += n;
  return p;
}

static void arena_free(void *, void *, void *) {}

struct bpki_ctx {
  int device = 0;
  void *stream = nullptr;
  size_t budget = 0;
  std::unique_ptr<Backend> be;
  std::mutex mu;
  // serving
  struct Job;
  std::map<uint64_t, std::shared_ptr<Job>> jobs;
  std::deque<std::shared_ptr<Job>> queue;
  int n_slots = 8;
  int pack_max = 16, pack_max_chi = 16;     // cross-request packing (see bpki_serving_packing)
  std::vector<std::unique_ptr<Backend>> slot_be;
  std::vector<std::thread> slot_threads;
  std::condition_variable cv, done_cv;
  bool stop = false;
  size_t used = 0;
  int running = 0;                  // requests on the device (a pack counts each member)
  int busy = 0;                     // slots working
  uint64_t next_ticket = 1;
  // sessions run on `be`: the context is deleted when it has been destroyed and the last of its
  // sessions is closed, whichever comes second
  int open_sessions = 0;
  bool destroyed = false;
  // caller's device allocator (bpki_set_allocator), also given to the serving slots' backends
  bpki_alloc_fn ualloc = nullptr;
  bpki_free_fn ufree = nullptr;
  void *uuser = nullptr;
  // allocation-free solves: a backend whose every device buffer comes from the device's static
  // scratch array, set up with the context (no allocation at call time)
  std::unique_ptr<Backend> na_be;
  ScratchArena arena;
  std::string na_err;
  std::mutex na_mu;
};

extern "C" int bpki_create(bpki_ctx **out, int device, void *hip_stream, size_t budget) {
  if (!out) return fail(-1, "out is NULL");
  std::string err;
  Backend *be = make_hip_backend(device, hip_stream, &err);
  if (!be) return fail(-5, "bpki_create: " + err);
  bpki_ctx *c = new bpki_ctx;
  c->device = device;
  c->stream = hip_stream;
  c->budget = budget;
  c->be.reset(be);
  // the device's scratch array (looked up with the device current, as the backend left it) and
  // the backend that allocates from it; without them only bpki_solve_noalloc fails
  void *base = nullptr;
  if (scratch_region(device, &base, &err) == 0) {
    Backend *na = make_hip_backend(device, hip_stream, &err);
    if (na) {
      c->arena.base = static_cast<char *>(base);
      c->arena.size = kScratchBytes;
      na->set_allocator(arena_alloc, arena_free, &c->arena);
      c->na_be.reset(na);
    }
  }
  if (!c->na_be) c->na_err = err;
  *out = c;
  return 0;
}

extern "C" int bpki_set_allocator(bpki_ctx *c, bpki_alloc_fn alloc, bpki_free_fn free, void *user) {
  if (!c) return fail(-1, "ctx is NULL");
  if (!alloc != !free) return fail(-1, "give both alloc and free, or neither");
  std::lock_guard<std::mutex> lk(c->mu);
  if (!c->slot_threads.empty() || c->open_sessions || c->be->set_allocator(alloc, free, user))
    return fail(-1, "the context already holds device memory: set the allocator before the first "
                    "solve, session or submit");
  c->ualloc = alloc;
  c->ufree = free;
  c->uuser = user;
  return 0;
}

static void serving_shutdown(bpki_ctx *c);

extern "C" void bpki_destroy(bpki_ctx *c) {
  if (!c) return;
  serving_shutdown(c);
  bool last;
  {
    std::lock_guard<std::mutex> lk(c->mu);
    c->destroyed = true;
    last = c->open_sessions == 0;
  }
  if (last) delete c;
}

// One whole solve on an engine; outputs written only on success.
// Steps of U(pi/2)^dagger (the extended time evolution of "Measuring expectation values"):
// U = (ZZ gates)(X rotations) gives U^dagger = (X rotations by -theta)(gates exp(-i pi/4 ZZ)),
// so the gates come first (descending colour, mirroring the forward step), then the rotations.
static double clifford_inverse_step(Engine &eng, const std::vector<int> &cols) {
  double d = 0;
  for (auto it = cols.rbegin(); it != cols.rend(); ++it) d += eng.apply_layer(*it, -1);
  eng.apply_rx_angle(-M_PI / 2);
  return d;
}

static std::vector<int> sorted_colours(const Problem &q) {
  std::vector<int> cs(q.colour.begin(), q.colour.end());
  std::sort(cs.begin(), cs.end());
  cs.erase(std::unique(cs.begin(), cs.end()), cs.end());
  return cs;
}

// Cut diagnostics of one step: the smallest gap of a chi-limited cut and the number of cuts whose
// gap is below kDegenerateGap, accumulated over the step's layers for the edges [e0, e1).
struct StepCuts {
  double gap = INFINITY;
  int degenerate = 0;
  void add(const std::vector<Engine::Cut> &cuts, int e0 = 0, int e1 = 1 << 30) {
    for (const auto &c : cuts) {
      if (c.e < e0 || c.e >= e1) continue;
      gap = std::min(gap, c.gap);
      degenerate += c.gap < kDegenerateGap;
    }
  }
};

static int run_solve(Backend *be, Engine &eng, const Problem &q, bpki_result *r,
                     std::atomic<bool> *cancel) {
  const int n = q.n_sites;
  const int steps = q.depth + q.clifford_steps;
  const int rows = std::max(1, q.record_every_step ? steps : 1);
  std::vector<double> z((size_t)rows * n, 1.0);
  const int ne = (int)q.edges.size() / 2;
  std::vector<double> ent(r->bond_entropy ? (size_t)rows * ne : 0, 0.0);
  std::vector<int32_t> iters(steps, 0), ndeg(steps, 0), bdim((size_t)rows * ne, 1);
  std::vector<double> res(steps, 0.0), disc(steps, 0.0), gap(steps, INFINITY);
  const std::vector<int> cols = sorted_colours(q);
  int warn = 0;
  for (int t = 0; t < steps; ++t) {
    if (cancel && cancel->load()) return fail(-6, "cancelled");
    double d = 0;
    StepCuts sc;
    if (t < q.depth) {
      eng.apply_rx();
      for (int c : cols) {
        d += eng.apply_layer(c);
        sc.add(eng.layer_cuts());
      }
    } else {
      for (auto it = cols.rbegin(); it != cols.rend(); ++it) {
        d += eng.apply_layer(*it, -1);
        sc.add(eng.layer_cuts());
      }
      eng.apply_rx_angle(-M_PI / 2);
    }
    double rr = 0;
    iters[t] = eng.bp(q.bp_max_iter, &rr);
    res[t] = rr;
    disc[t] = d;
    gap[t] = sc.gap;
    ndeg[t] = sc.degenerate;
    if (!(rr < q.bp_tol)) warn = 1;
    if (q.record_every_step || t == steps - 1) {
      int row = q.record_every_step ? t : 0;
      eng.observe_z(&z[(size_t)row * n]);
      if (!ent.empty()) eng.observe_entropy(&ent[(size_t)row * ne]);
      std::copy(eng.bond_dims().begin(), eng.bond_dims().end(), bdim.begin() + (size_t)row * ne);
    }
    std::string msg;
    int e = be->check(&msg);
    if (e) return fail(e, "device error: " + msg);
  }
  std::vector<double> pv(q.pauli_offsets.size() - 1, 0.0);
  if (!pv.empty()) eng.observe_pauli(pv.data());
  std::string msg;
  int e = be->check(&msg);
  if (e) return fail(e, "device error: " + msg);
  for (double x : z)
    if (!std::isfinite(x)) return fail(-5, "non-finite observable (numerical breakdown)");
  for (double x : ent)
    if (!std::isfinite(x)) return fail(-5, "non-finite bond entropy (numerical breakdown)");
  if (r->z) std::memcpy(r->z, z.data(), (size_t)rows * n * sizeof(double));
  if (!ent.empty()) std::memcpy(r->bond_entropy, ent.data(), ent.size() * sizeof(double));
  if (r->pauli && !pv.empty()) std::memcpy(r->pauli, pv.data(), pv.size() * sizeof(double));
  if (steps > 0) {                  // the per-step arrays are empty for a zero-step solve
    if (r->bp_iters) std::memcpy(r->bp_iters, iters.data(), iters.size() * sizeof(int32_t));
    if (r->bp_residual) std::memcpy(r->bp_residual, res.data(), res.size() * sizeof(double));
    if (r->discarded) std::memcpy(r->discarded, disc.data(), disc.size() * sizeof(double));
    if (r->min_cut_gap) std::memcpy(r->min_cut_gap, gap.data(), gap.size() * sizeof(double));
    if (r->degenerate_cuts)
      std::memcpy(r->degenerate_cuts, ndeg.data(), ndeg.size() * sizeof(int32_t));
  }
  if (r->bond_dims) std::memcpy(r->bond_dims, bdim.data(), bdim.size() * sizeof(int32_t));
  return warn;
}

extern "C" int bpki_solve_noalloc(bpki_ctx *c, const bpki_problem *p, bpki_result *r) {
  if (!c || !r) return fail(-1, "NULL context or result");
  int rc = bpki_validate(p);
  if (rc) return rc;
  Problem q = to_problem(p);
  if (!c->na_be) return fail(-5, "bpki_solve_noalloc: no scratch on this device: " + c->na_err);
  const size_t need = Engine::estimate_bytes(q);
  if (need > kScratchBytes)
    return fail(-4, "bpki_solve_noalloc: the problem needs up to " + std::to_string(need) +
                        " bytes of device memory; the static scratch holds " +
                        std::to_string(kScratchBytes) + " (use bpki_solve)");
  std::lock_guard<std::mutex> lk(c->na_mu);
  Backend *be = c->na_be.get();
  be->forget_workspaces();       // their memory was the previous call's part of the scratch
  be->clear_alloc_error();
  c->arena.top = 0;
  std::string msg;
  if (int e = be->check(&msg)) return fail(e, "device error: " + msg);
  int status;
  {
    Engine eng(be, q);
    if (be->check(&msg) == -4)
      status = fail(-4, "bpki_solve_noalloc: the static scratch of " +
                            std::to_string(kScratchBytes) + " bytes is exhausted");
    else if (int e = be->check(&msg))
      status = fail(e, "device error: " + msg);
    else
      status = run_solve(be, eng, q, r, nullptr);
  }
  be->forget_workspaces();
  if (status == -4 && be->check(nullptr) == -4)
    fail(-4, "bpki_solve_noalloc: the static scratch of " + std::to_string(kScratchBytes) +
                 " bytes is exhausted");
  return status;
}

extern "C" int bpki_solve(bpki_ctx *c, const bpki_problem *p, bpki_result *r) {
  if (!c || !r) return fail(-1, "NULL context or result");
  int rc = bpki_validate(p);
  if (rc) return rc;
  Problem q = to_problem(p);
  size_t need = Engine::estimate_bytes(q);
  if (c->budget && need > c->budget) return fail(-4, "problem exceeds the memory budget");
  std::lock_guard<std::mutex> lk(c->mu);
  std::string msg;
  if (c->be->check(&msg)) return fail(-5, "device in error state: " + msg);
  std::unique_ptr<Engine> eng(new Engine(c->be.get(), q));
  if (int e = c->be->check(&msg)) return fail(e, "allocation: " + msg);
  return run_solve(c->be.get(), *eng, q, r, nullptr);
}

// ------------------------------------------------------------------------------------------
// sessions
struct bpki_session {
  bpki_ctx *ctx;
  std::unique_ptr<Engine> eng;
  std::vector<int> colours;
  double timing[4] = {0, 0, 0, 0};
};

extern "C" int bpki_session_open(bpki_ctx *c, const bpki_problem *p, bpki_session **out) {
  if (!c || !out) return fail(-1, "NULL argument");
  int rc = bpki_validate(p);
  if (rc) return rc;
  Problem q = to_problem(p);
  size_t need = Engine::estimate_bytes(q);
  if (c->budget && need > c->budget) return fail(-4, "problem exceeds the memory budget");
  auto *s = new bpki_session;
  s->ctx = c;
  s->eng.reset(new Engine(c->be.get(), q));
  std::string msg;
  if (int e = c->be->check(&msg)) {
    delete s;
    return fail(e, "session allocation: " + msg);
  }
  s->colours.assign(q.colour.begin(), q.colour.end());
  std::sort(s->colours.begin(), s->colours.end());
  s->colours.erase(std::unique(s->colours.begin(), s->colours.end()), s->colours.end());
  {
    std::lock_guard<std::mutex> lk(c->mu);
    ++c->open_sessions;
  }
  *out = s;
  return 0;
}

extern "C" void bpki_session_close(bpki_session *s) {
  if (!s) return;
  bpki_ctx *c = s->ctx;
  delete s;  // releases the session's device memory through c->be
  bool last;
  {
    std::lock_guard<std::mutex> lk(c->mu);
    last = --c->open_sessions == 0 && c->destroyed;
  }
  if (last) delete c;
}

static int sess_check(bpki_session *s) {
  std::string msg;
  int e = s->ctx->be->check(&msg);
  return e ? fail(e, "device error: " + msg) : 0;
}

extern "C" int bpki_session_sizes(const bpki_session *s, size_t *te, size_t *me) {
  if (!s) return fail(-1, "NULL session");
  if (te) *te = s->eng->tensor_elems();
  if (me) *me = s->eng->message_elems();
  return 0;
}

extern "C" int bpki_session_get_state(bpki_session *s, double *t, double *m, int32_t *b) {
  if (!s) return fail(-1, "NULL session");
  s->eng->get_state(t, m, b);
  return sess_check(s);
}

extern "C" int bpki_session_set_state(bpki_session *s, const double *t, const double *m,
                                      const int32_t *b) {
  if (!s) return fail(-1, "NULL session");
  s->eng->set_state(t, m, b);
  return sess_check(s);
}

extern "C" int bpki_session_apply_rx(bpki_session *s) {
  if (!s) return fail(-1, "NULL session");
  s->eng->apply_rx();
  return sess_check(s);
}

extern "C" int bpki_session_apply_layer(bpki_session *s, int32_t colour, double *disc) {
  if (!s) return fail(-1, "NULL session");
  double d = s->eng->apply_layer(colour);
  if (disc) *disc = d;
  return sess_check(s);
}

extern "C" int bpki_session_layer_cuts(bpki_session *s, int32_t *kept, double *discarded,
                                       double *gap) {
  if (!s) return fail(-1, "NULL session");
  const int ne = (int)s->eng->problem().edges.size() / 2;
  for (int e = 0; e < ne; ++e) {
    if (kept) kept[e] = -1;
    if (discarded) discarded[e] = NAN;
    if (gap) gap[e] = NAN;
  }
  for (const auto &c : s->eng->layer_cuts()) {
    if (kept) kept[c.e] = c.kept;
    if (discarded) discarded[c.e] = c.discarded;
    if (gap) gap[c.e] = c.gap;
  }
  return 0;
}

extern "C" int bpki_session_bp(bpki_session *s, int32_t max_iter, int32_t *iters, double *res) {
  if (!s || max_iter < 1) return fail(-1, "bad argument");
  double r = 0;
  int it = s->eng->bp(max_iter, &r);
  if (iters) *iters = it;
  if (res) *res = r;
  int e = sess_check(s);
  if (e) return e;
  return r < s->eng->problem().bp_tol ? 0 : 1;
}

extern "C" int bpki_session_bp_sweep(bpki_session *s, double *res) {
  if (!s) return fail(-1, "NULL session");
  double r = s->eng->bp_sweep();
  if (res) *res = r;
  return sess_check(s);
}

extern "C" int bpki_session_observe_z(bpki_session *s, double *z) {
  if (!s || !z) return fail(-1, "NULL argument");
  s->eng->observe_z(z);
  return sess_check(s);
}

extern "C" int bpki_session_vidal_gauge(bpki_session *s, double *lambda) {
  if (!s) return fail(-1, "NULL session");
  s->eng->vidal_gauge(lambda);
  return sess_check(s);
}

extern "C" int bpki_session_bp_error(bpki_session *s, int32_t edge, double *error,
                                     double *spectrum) {
  if (!s || !error) return fail(-1, "NULL argument");
  const Problem &q = s->eng->problem();
  if (edge < 0 || edge >= (int)q.edges.size() / 2) return fail(-1, "edge out of range");
  if (q.chi > 16) return fail(-1, "the BP error estimate needs chi <= 16 (chi^2 <= 256)");
  const double err = s->eng->bp_error(edge, spectrum);
  int rc = sess_check(s);
  if (rc < 0) return rc;
  if (err == -1.0)
    return fail(-1, "the BP error estimate is built for bridges and for networks whose 2-core is "
                    "one loop or two junctions joined by three paths");
  if (!std::isfinite(err)) return fail(-5, "BP error estimate: zero norm or allocation failure");
  *error = err;
  return 0;
}

extern "C" int bpki_session_observe_bond_entropy(bpki_session *s, double *entropy) {
  if (!s || !entropy) return fail(-1, "NULL argument");
  s->eng->observe_entropy(entropy);
  return sess_check(s);
}

extern "C" int bpki_session_observe_pauli(bpki_session *s, double *out) {
  if (!s) return fail(-1, "NULL session");
  if (s->eng->problem().pauli_offsets.size() <= 1) return 0;
  if (!out) return fail(-1, "NULL output");
  s->eng->observe_pauli(out);
  return sess_check(s);
}

extern "C" int bpki_session_step(bpki_session *s, double *z, int32_t *iters, double *res,
                                 double *disc) {
  if (!s) return fail(-1, "NULL session");
  Backend *be = s->ctx->be.get();
  be->timer_mark(0);
  s->eng->apply_rx();
  be->timer_mark(1);
  double d = 0;
  for (int c : s->colours) d += s->eng->apply_layer(c);
  be->timer_mark(2);
  double r = 0;
  int it = s->eng->bp(s->eng->problem().bp_max_iter, &r);
  be->timer_mark(3);
  if (z) s->eng->observe_z(z);
  be->timer_mark(4);
  s->timing[0] = be->timer_ms(0, 1);
  s->timing[1] = be->timer_ms(1, 2);
  s->timing[2] = be->timer_ms(2, 3);
  s->timing[3] = z ? be->timer_ms(3, 4) : 0.0;
  if (iters) *iters = it;
  if (res) *res = r;
  if (disc) *disc = d;
  int e = sess_check(s);
  if (e) return e;
  return r < s->eng->problem().bp_tol ? 0 : 1;
}

extern "C" int bpki_session_clifford_inverse_step(bpki_session *s, double *z, int32_t *iters,
                                                  double *res, double *disc) {
  if (!s) return fail(-1, "NULL session");
  Backend *be = s->ctx->be.get();
  be->timer_mark(0);
  be->timer_mark(1);
  const double d = clifford_inverse_step(*s->eng, s->colours);
  be->timer_mark(2);
  double r = 0;
  int it = s->eng->bp(s->eng->problem().bp_max_iter, &r);
  be->timer_mark(3);
  if (z) s->eng->observe_z(z);
  be->timer_mark(4);
  s->timing[0] = be->timer_ms(0, 1);
  s->timing[1] = be->timer_ms(1, 2);
  s->timing[2] = be->timer_ms(2, 3);
  s->timing[3] = z ? be->timer_ms(3, 4) : 0.0;
  if (iters) *iters = it;
  if (res) *res = r;
  if (disc) *disc = d;
  int e = sess_check(s);
  if (e) return e;
  return r < s->eng->problem().bp_tol ? 0 : 1;
}

extern "C" int bpki_session_profile(bpki_session *s, int stride) {
  if (!s) return fail(-1, "NULL session");
  if (stride < 0) return fail(-1, "stride must be >= 0");
  s->ctx->be->gemm_profile(stride);
  return sess_check(s);
}

extern "C" int bpki_session_profile_read(bpki_session *s, int64_t *launches, double *ms,
                                         double *flops, int64_t *all_launches) {
  if (!s) return fail(-1, "NULL session");
  long l = 0, a = 0;
  s->ctx->be->gemm_profile_read(&l, &a, ms, flops);
  if (launches) *launches = l;
  if (all_launches) *all_launches = a;
  return sess_check(s);
}

extern "C" int bpki_session_profile_read_prec(bpki_session *s, int32_t prec, int64_t *launches,
                                              double *ms, double *flops) {
  if (!s || (prec != 0 && prec != 1)) return fail(-1, "bad argument");
  long l = 0;
  s->ctx->be->gemm_profile_read_prec(prec, &l, ms, flops);
  if (launches) *launches = l;
  return sess_check(s);
}

extern "C" int bpki_session_profile_read_kernel(bpki_session *s, int32_t kernel, int32_t prec,
                                                int64_t *launches, double *ms, double *flops,
                                                double *bytes, int64_t *all_launches) {
  if (!s || kernel < 0 || kernel > 2 || (prec != 0 && prec != 1)) return fail(-1, "bad argument");
  long l = 0, a = 0;
  s->ctx->be->gemm_profile_read_kernel(kernel, prec, &l, ms, flops, bytes, &a);
  if (launches) *launches = l;
  if (all_launches) *all_launches = a;
  return sess_check(s);
}

extern "C" int bpki_session_last_timing(const bpki_session *s, double *ms4) {
  if (!s || !ms4) return fail(-1, "NULL argument");
  for (int i = 0; i < 4; ++i) ms4[i] = s->timing[i];
  return 0;
}

// ------------------------------------------------------------------------------------------
// serving: concurrent slots.  Each slot is a worker thread with its own HIP stream and backend;
// a slot takes the oldest queued request whose memory estimate fits the budget next to what is
// resident, runs it to completion on its stream and writes the result into the caller's buffers.
// Requests that arrive while others run are admitted as slots and memory free up, and the
// kernels of different slots run concurrently on the device.  A request's arithmetic does not
// depend on the other slots (same kernels, deterministic reductions, private workspaces).
struct bpki_ctx::Job {
  uint64_t ticket = 0;
  Problem q;
  bpki_result *r = nullptr;
  std::atomic<bool> cancel{false};
  bool done = false;
  int status = 0;
  size_t bytes = 0;
  int pack_size = 0;
  double t_submit = 0, t_start = 0, t_done = 0;
};

// Cross-request packing.  Requests on the same lattice (sites, edges and colours) with the same
// chi, precision, BP and truncation settings are solved together as one problem on the disjoint
// union of their lattices: every launch of a gate layer or BP sweep then covers all of them.  The
// members keep their own X angles, depths and Pauli strings; each member's messages are frozen
// once its own BP residual is below the tolerance (Engine::bp_members), so every member follows
// the schedule of a solve of its own, and its result is written as soon as its last step is done.
// Requests that share one launch set: the same chi (the layout is padded to one chi and the
// truncation keeps at most chi values), precision, BP tolerance and cutoffs; the lattices may
// differ (each member is a connected component of the union graph, so its gate layers and BP
// schedule are the ones it has alone).
static bool packable(const Problem &a, const Problem &b) {
  return a.chi == b.chi && a.precision == b.precision && a.bp_tol == b.bp_tol &&
         a.bp_max_iter == b.bp_max_iter && a.svd_cutoff == b.svd_cutoff &&
         a.eig_cutoff == b.eig_cutoff && b.depth >= 1 && a.clifford_steps == 0 &&
         b.clifford_steps == 0;
}

static Problem pack_problem(const std::vector<const Problem *> &qs, std::vector<int> *pauli0) {
  Problem u = *qs[0];
  u.n_sites = 0;
  u.depth = 0;
  u.record_every_step = 1;
  u.edges.clear();
  u.colour.clear();
  u.site_theta.clear();
  u.member_site0.clear();
  u.pauli_offsets.assign(1, 0);
  u.pauli_sites.clear();
  u.pauli_ops.clear();
  pauli0->clear();
  for (const Problem *q : qs) {
    const int s0 = u.n_sites;
    u.member_site0.push_back(s0);
    for (int x : q->edges) u.edges.push_back(x + s0);
    u.colour.insert(u.colour.end(), q->colour.begin(), q->colour.end());
    u.site_theta.insert(u.site_theta.end(), q->n_sites, q->theta);
    pauli0->push_back((int)u.pauli_offsets.size() - 1);
    for (size_t k = 0; k + 1 < q->pauli_offsets.size(); ++k) {
      for (int i = q->pauli_offsets[k]; i < q->pauli_offsets[k + 1]; ++i) {
        u.pauli_sites.push_back(q->pauli_sites[i] + s0);
        u.pauli_ops.push_back(q->pauli_ops[i]);
      }
      u.pauli_offsets.push_back((int)u.pauli_sites.size());
    }
    u.n_sites += q->n_sites;
    u.depth = std::max(u.depth, q->depth);
  }
  u.member_site0.push_back(u.n_sites);
  pauli0->push_back((int)u.pauli_offsets.size() - 1);
  return u;
}

static double now_s() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

static void serving_shutdown(bpki_ctx *c) {
  {
    std::lock_guard<std::mutex> lk(c->mu);
    c->stop = true;
    for (auto &kv : c->jobs) kv.second->cancel = true;
  }
  c->cv.notify_all();
  for (auto &t : c->slot_threads)
    if (t.joinable()) t.join();
  c->slot_threads.clear();
  c->slot_be.clear();
}

static void finish_job(bpki_ctx *c, const std::shared_ptr<bpki_ctx::Job> &job, int status) {
  {
    std::lock_guard<std::mutex> lk(c->mu);
    job->status = status;
    job->done = true;
    job->t_done = now_s();
  }
  c->done_cv.notify_all();
}

// Runs a pack to the largest member depth; finishes every member (result or error).
static void run_pack(bpki_ctx *c, Backend *be, Engine &eng, const Problem &U,
                     const std::vector<std::shared_ptr<bpki_ctx::Job>> &jobs,
                     const std::vector<int> &pauli0) {
  const int R = (int)jobs.size();
  struct Acc {
    std::vector<double> z, ent, res, disc, gap;
    std::vector<int32_t> iters, ndeg, bdim;
    int warn = 0;
    bool fin = false;
  };
  std::vector<Acc> acc(R);
  std::vector<int> edge_member(U.edges.size() / 2), edge0(R + 1, 0);
  bool any_ent = false;
  for (int j = 0, e0 = 0; j < R; ++j) {
    const Problem &q = jobs[j]->q;
    const int rows = std::max(1, q.record_every_step ? q.depth : 1);
    acc[j].z.assign((size_t)rows * q.n_sites, 1.0);
    if (jobs[j]->r->bond_entropy) {
      acc[j].ent.assign((size_t)rows * (q.edges.size() / 2), 0.0);
      any_ent = true;
    }
    acc[j].iters.assign(q.depth, 0);
    acc[j].res.assign(q.depth, 0.0);
    acc[j].disc.assign(q.depth, 0.0);
    acc[j].gap.assign(q.depth, INFINITY);
    acc[j].ndeg.assign(q.depth, 0);
    const int ne = (int)q.edges.size() / 2;
    acc[j].bdim.assign((size_t)rows * ne, 1);
    for (int e = 0; e < ne; ++e) edge_member[e0 + e] = j;
    e0 += ne;
    edge0[j + 1] = e0;
  }
  std::vector<int> cols(U.colour.begin(), U.colour.end());
  std::sort(cols.begin(), cols.end());
  cols.erase(std::unique(cols.begin(), cols.end()), cols.end());
  std::vector<int> sweeps(R);
  std::vector<double> rr(R), zall(U.n_sites), dj(R), eall(any_ent ? U.edges.size() / 2 : 0);
  auto fin = [&](int j, int status) {
    acc[j].fin = true;
    finish_job(c, jobs[j], status);
  };
  for (int t = 0; t < U.depth; ++t) {
    int open = 0;
    for (int j = 0; j < R; ++j) {
      if (acc[j].fin) continue;
      if (jobs[j]->cancel.load()) fin(j, -6);
      else ++open;
    }
    if (!open) return;
    eng.apply_rx();
    std::fill(dj.begin(), dj.end(), 0.0);
    std::vector<StepCuts> scj(R);
    for (int col : cols) {
      eng.apply_layer(col);
      for (auto &cut : eng.layer_cuts()) {
        const int j = edge_member[cut.e];
        dj[j] += cut.discarded;
        scj[j].add({cut});
      }
    }
    eng.bp_members(U.bp_max_iter, sweeps.data(), rr.data());
    bool need_z = false, need_e = false;
    for (int j = 0; j < R; ++j) {
      const Problem &q = jobs[j]->q;
      if (!acc[j].fin && t < q.depth && (q.record_every_step || t == q.depth - 1)) {
        need_z = true;
        need_e = need_e || !acc[j].ent.empty();
      }
    }
    if (need_z) eng.observe_z(zall.data());
    if (need_e) eng.observe_entropy(eall.data());
    std::string msg;
    if (int e = be->check(&msg)) {
      for (int j = 0; j < R; ++j)
        if (!acc[j].fin) fin(j, e);
      return;
    }
    for (int j = 0; j < R; ++j) {
      const Problem &q = jobs[j]->q;
      if (acc[j].fin || t >= q.depth) continue;
      Acc &a = acc[j];
      a.iters[t] = sweeps[j];
      a.res[t] = rr[j];
      a.disc[t] = dj[j];
      a.gap[t] = scj[j].gap;
      a.ndeg[t] = scj[j].degenerate;
      if (!(rr[j] < q.bp_tol)) a.warn = 1;
      const int s0 = U.member_site0[j];
      if (q.record_every_step || t == q.depth - 1) {
        const int row = q.record_every_step ? t : 0;
        std::copy(zall.begin() + s0, zall.begin() + s0 + q.n_sites,
                  a.z.begin() + (size_t)row * q.n_sites);
        const int ne = edge0[j + 1] - edge0[j];
        if (!a.ent.empty())
          std::copy(eall.begin() + edge0[j], eall.begin() + edge0[j + 1],
                    a.ent.begin() + (size_t)row * ne);
        std::copy(eng.bond_dims().begin() + edge0[j], eng.bond_dims().begin() + edge0[j + 1],
                  a.bdim.begin() + (size_t)row * ne);
      }
      if (t < q.depth - 1) continue;
      std::vector<double> pv(pauli0[j + 1] - pauli0[j], 0.0);
      if (!pv.empty()) eng.observe_pauli_range(pauli0[j], pauli0[j + 1], pv.data());
      if (int e = be->check(&msg)) {
        fin(j, e);
        continue;
      }
      bool finite = true;
      for (double x : a.z) finite = finite && std::isfinite(x);
      for (double x : a.ent) finite = finite && std::isfinite(x);
      if (!finite) {
        fin(j, -5);
        continue;
      }
      bpki_result *r = jobs[j]->r;
      if (r->z) std::memcpy(r->z, a.z.data(), a.z.size() * sizeof(double));
      if (!a.ent.empty()) std::memcpy(r->bond_entropy, a.ent.data(), a.ent.size() * sizeof(double));
      if (r->pauli && !pv.empty()) std::memcpy(r->pauli, pv.data(), pv.size() * sizeof(double));
      if (r->bp_iters) std::memcpy(r->bp_iters, a.iters.data(), a.iters.size() * sizeof(int32_t));
      if (r->bp_residual) std::memcpy(r->bp_residual, a.res.data(), a.res.size() * sizeof(double));
      if (r->discarded) std::memcpy(r->discarded, a.disc.data(), a.disc.size() * sizeof(double));
      if (r->bond_dims) std::memcpy(r->bond_dims, a.bdim.data(), a.bdim.size() * sizeof(int32_t));
      if (r->min_cut_gap) std::memcpy(r->min_cut_gap, a.gap.data(), a.gap.size() * sizeof(double));
      if (r->degenerate_cuts)
        std::memcpy(r->degenerate_cuts, a.ndeg.data(), a.ndeg.size() * sizeof(int32_t));
      fin(j, a.warn);
    }
  }
  for (int j = 0; j < R; ++j)
    if (!acc[j].fin) fin(j, -5);    // not reached: every member ends at its own depth
}

static void slot_loop(bpki_ctx *c, int slot) {
  Backend *be = c->slot_be[slot].get();
  for (;;) {
    // A backend's error state is sticky (a failed allocation leaves null buffers behind, a
    // device error poisons its stream): after the job that hit it has been failed with its
    // code, the slot takes a fresh backend before it takes another job.
    if (be->check(nullptr)) {
      std::string err;
      Backend *fresh = make_hip_backend(c->device, nullptr, &err);
      if (fresh) {
        fresh->set_allocator(c->ualloc, c->ufree, c->uuser);
        std::lock_guard<std::mutex> lk(c->mu);
        c->slot_be[slot].reset(fresh);
        be = fresh;
      }
    }
    std::shared_ptr<bpki_ctx::Job> job;
    std::vector<std::shared_ptr<bpki_ctx::Job>> pack;
    size_t pack_bytes = 0;
    {
      std::unique_lock<std::mutex> lk(c->mu);
      c->cv.wait(lk, [&] {
        if (c->stop) return true;
        if (c->queue.empty()) return false;
        auto &h = c->queue.front();
        return h->cancel.load() || c->budget == 0 || c->running == 0 ||
               c->used + h->bytes <= c->budget;
      });
      if (c->stop && c->queue.empty()) return;
      if (c->queue.empty()) continue;
      job = c->queue.front();
      c->queue.pop_front();
      if (job->cancel) {
        job->status = -6;
        job->done = true;
        job->t_done = now_s();
        c->done_cv.notify_all();
        continue;
      }
      pack.assign(1, job);
      size_t bytes = job->bytes;
      // pack only requests that would otherwise wait (more queued than idle slots, which would
      // run them concurrently), and only companions that end no later than the head
      const int idle = c->n_slots - c->busy - 1;
      if (c->pack_max > 1 && job->q.chi <= c->pack_max_chi && job->q.depth >= 1 &&
          job->q.clifford_steps == 0 && (int)c->queue.size() > idle) {
        for (auto it = c->queue.begin();
             it != c->queue.end() && (int)pack.size() < c->pack_max;) {
          const auto &h = *it;
          if (!h->cancel && packable(job->q, h->q) && h->q.depth <= job->q.depth &&
              (c->budget == 0 || c->used + bytes + h->bytes <= c->budget)) {
            bytes += h->bytes;
            pack.push_back(h);
            it = c->queue.erase(it);
          } else {
            ++it;
          }
        }
      }
      c->used += bytes;
      c->running += (int)pack.size();
      c->busy += 1;
      const double t0 = now_s();
      for (auto &m : pack) {
        m->t_start = t0;
        m->pack_size = (int)pack.size();
      }
      pack_bytes = bytes;
    }
    std::string msg;
    if (pack.size() == 1) {
      int status;
      if (be->check(&msg)) {
        status = -5;
      } else {
        std::unique_ptr<Engine> eng(new Engine(be, job->q));
        if (be->check(&msg)) status = -4;
        else status = run_solve(be, *eng, job->q, job->r, &job->cancel);
      }
      finish_job(c, job, status);
    } else {
      std::vector<const Problem *> qs;
      for (auto &m : pack) qs.push_back(&m->q);
      std::vector<int> pauli0;
      Problem U = pack_problem(qs, &pauli0);
      if (be->check(&msg)) {
        for (auto &m : pack) finish_job(c, m, -5);
      } else {
        std::unique_ptr<Engine> eng(new Engine(be, U));
        if (be->check(&msg)) {
          for (auto &m : pack) finish_job(c, m, -4);
        } else {
          run_pack(c, be, *eng, U, pack, pauli0);
        }
      }
    }
    {
      std::lock_guard<std::mutex> lk(c->mu);
      c->used -= pack_bytes;
      c->running -= (int)pack.size();
      c->busy -= 1;
    }
    c->cv.notify_all();
  }
}

static int start_slots(bpki_ctx *c) {
  if (!c->slot_threads.empty()) return 0;
  for (int i = 0; i < c->n_slots; ++i) {
    std::string err;
    Backend *be = make_hip_backend(c->device, nullptr, &err);
    if (!be) return fail(-5, "serving slot: " + err);
    be->set_allocator(c->ualloc, c->ufree, c->uuser);      // a fresh backend takes it
    c->slot_be.emplace_back(be);
  }
  for (int i = 0; i < c->n_slots; ++i) c->slot_threads.emplace_back(slot_loop, c, i);
  return 0;
}

extern "C" int bpki_serving_config(bpki_ctx *c, int slots) {
  if (!c || slots < 1 || slots > 64) return fail(-1, "slots must be in 1..64");
  std::lock_guard<std::mutex> lk(c->mu);
  if (!c->slot_threads.empty()) return fail(-1, "serving already started");
  c->n_slots = slots;
  return 0;
}

extern "C" int bpki_serving_packing(bpki_ctx *c, int max_requests, int max_chi) {
  if (!c || max_requests < 1 || max_requests > 64 || max_chi < 1)
    return fail(-1, "max_requests must be in 1..64 and max_chi >= 1");
  std::lock_guard<std::mutex> lk(c->mu);
  if (!c->slot_threads.empty()) return fail(-1, "serving already started");
  c->pack_max = max_requests;
  c->pack_max_chi = max_chi;
  return 0;
}

extern "C" int bpki_submit(bpki_ctx *c, const bpki_problem *p, bpki_result *r, uint64_t *ticket) {
  if (!c || !r || !ticket) return fail(-1, "NULL argument");
  int rc = bpki_validate(p);
  if (rc) return rc;
  auto job = std::make_shared<bpki_ctx::Job>();
  job->q = to_problem(p);
  job->r = r;
  job->bytes = Engine::estimate_bytes(job->q);
  if (c->budget && job->bytes > c->budget) return fail(-4, "problem can never fit the budget");
  std::lock_guard<std::mutex> lk(c->mu);
  if (int e = start_slots(c)) return e;
  job->ticket = c->next_ticket++;
  job->t_submit = now_s();
  c->jobs[job->ticket] = job;
  c->queue.push_back(job);
  c->cv.notify_all();
  *ticket = job->ticket;
  return 0;
}

extern "C" int bpki_poll(bpki_ctx *c, uint64_t t, int *done) {
  if (!c || !done) return fail(-1, "NULL argument");
  std::lock_guard<std::mutex> lk(c->mu);
  auto it = c->jobs.find(t);
  if (it == c->jobs.end()) return fail(-7, "unknown ticket");
  *done = it->second->done ? 1 : 0;
  return it->second->done ? it->second->status : 0;
}

extern "C" int bpki_ticket_times(bpki_ctx *c, uint64_t t, double *times3) {
  if (!c || !times3) return fail(-1, "NULL argument");
  std::lock_guard<std::mutex> lk(c->mu);
  auto it = c->jobs.find(t);
  if (it == c->jobs.end()) return fail(-7, "unknown ticket");
  times3[0] = it->second->t_submit;
  times3[1] = it->second->t_start;
  times3[2] = it->second->t_done;
  return 0;
}

extern "C" int bpki_ticket_pack_size(bpki_ctx *c, uint64_t t, int32_t *size) {
  if (!c || !size) return fail(-1, "NULL argument");
  std::lock_guard<std::mutex> lk(c->mu);
  auto it = c->jobs.find(t);
  if (it == c->jobs.end()) return fail(-7, "unknown ticket");
  *size = it->second->pack_size;
  return 0;
}

extern "C" int bpki_wait(bpki_ctx *c, uint64_t t) {
  if (!c) return fail(-1, "NULL context");
  std::unique_lock<std::mutex> lk(c->mu);
  auto it = c->jobs.find(t);
  if (it == c->jobs.end()) return fail(-7, "unknown ticket");
  auto job = it->second;
  c->done_cv.wait(lk, [&] { return job->done; });
  c->jobs.erase(t);
  if (job->status < 0) g_err = job->status == -6 ? "cancelled" : "request failed";
  return job->status;
}

extern "C" int bpki_cancel(bpki_ctx *c, uint64_t t) {
  if (!c) return fail(-1, "NULL context");
  std::lock_guard<std::mutex> lk(c->mu);
  auto it = c->jobs.find(t);
  if (it == c->jobs.end()) return fail(-7, "unknown ticket");
  it->second->cancel = true;
  c->cv.notify_all();
  return 0;
}

// ------------------------------------------------------------------------------------------
// test hooks (include/bpki_testing.h)
extern "C" int bpki_test_gemm(bpki_ctx *c, const bpki_test_gemm_desc *td, int nprob,
                              const double *A, size_t a_elems, const double *B, size_t b_elems,
                              double *C, size_t c_elems) {
  if (!c || !td || nprob < 1) return fail(-1, "bad argument");
  Backend *be = c->be.get();
  GemmDesc d;
  d.M = td->M; d.N = td->N; d.K = td->K; d.Mi = td->Mi; d.Ni = td->Ni; d.Ki = td->Ki;
  d.a_mo = td->a_mo; d.a_mi = td->a_mi; d.a_ko = td->a_ko; d.a_ki = td->a_ki;
  d.b_ko = td->b_ko; d.b_ki = td->b_ki; d.b_no = td->b_no; d.b_ni = td->b_ni;
  d.c_mo = td->c_mo; d.c_mi = td->c_mi; d.c_no = td->c_no; d.c_ni = td->c_ni;
  d.a_b = td->a_b; d.b_b = td->b_b; d.c_b = td->c_b; d.batch = td->batch;
  d.conjA = td->conjA; d.conjB = td->conjB; d.beta = td->beta;
  d.alpha_re = td->alpha_re; d.alpha_im = td->alpha_im;
  d.prec = td->prec;
  d.herm = td->herm;
  d.a32 = td->store32 & 1;
  d.b32 = (td->store32 >> 1) & 1;
  d.c32 = (td->store32 >> 2) & 1;
  if (d.prec != 0 && d.prec != 1) return fail(-1, "prec must be 0 (FP64) or 1 (FP32)");
  if (td->store32 && (d.prec != 1 || (td->store32 != 5 && td->store32 != 3)))
    return fail(-1, "store32 must be 0, 5 (A and C) or 3 (A and B), with prec = 1");
  if (d.herm && (d.M != d.N || d.Mi != d.M || d.Ni != d.N || d.alpha_im != 0 || d.beta))
    return fail(-1, "herm needs M == N, single-stride M and N, real alpha and beta = 0");
  if (d.M < 1 || d.N < 1 || d.K < 1 || d.Mi < 1 || d.Ni < 1 || d.Ki < 1 || d.batch < 1 ||
      d.M % d.Mi || d.N % d.Ni || d.K % d.Ki)
    return fail(-1, "inconsistent descriptor");
  // bounds: every addressed element must lie inside the buffers (host-side check)
  auto span = [](long o, long so, long si, int X, int Xi) {
    long a = (long)(X / Xi - 1) * so, b = (long)(Xi - 1) * si;
    return std::max(0L, a) + std::max(0L, b) + o;
  };
  long amax = span(0, d.a_mo, d.a_mi, d.M, d.Mi) + span(0, d.a_ko, d.a_ki, d.K, d.Ki) +
              (long)(d.batch - 1) * d.a_b;
  long bmax = span(0, d.b_ko, d.b_ki, d.K, d.Ki) + span(0, d.b_no, d.b_ni, d.N, d.Ni) +
              (long)(d.batch - 1) * d.b_b;
  long cmax = span(0, d.c_mo, d.c_mi, d.M, d.Mi) + span(0, d.c_no, d.c_ni, d.N, d.Ni) +
              (long)(d.batch - 1) * d.c_b;
  if (d.a_mo < 0 || d.a_mi < 0 || d.a_ko < 0 || d.a_ki < 0 || d.b_ko < 0 || d.b_ki < 0 ||
      d.b_no < 0 || d.b_ni < 0 || d.c_mo < 0 || d.c_mi < 0 || d.c_no < 0 || d.c_ni < 0 ||
      d.a_b < 0 || d.b_b < 0 || d.c_b < 0)
    return fail(-1, "negative stride");
  if ((size_t)amax >= a_elems || (size_t)bmax >= b_elems || (size_t)cmax >= c_elems)
    return fail(-1, "descriptor addresses outside the buffers");
  std::lock_guard<std::mutex> lk(c->mu);
  // device copy of an operand (complex FP64, or complex FP32 when flagged) and its base pointers
  auto upload = [&](const double *h, size_t elems, bool f32, char **dev) -> bool {
    const size_t esz = f32 ? 8 : 16;
    *dev = (char *)be->alloc(elems * esz * nprob);
    if (!*dev) return false;
    if (f32) {
      std::vector<float> t(2 * elems * nprob);
      for (size_t i = 0; i < t.size(); ++i) t[i] = (float)h[i];
      be->h2d(*dev, t.data(), t.size() * 4);
    } else {
      be->h2d(*dev, h, elems * 16 * nprob);
    }
    return true;
  };
  char *dA = nullptr, *dB = nullptr, *dC = nullptr;
  void **ptrs = (void **)be->alloc(3 * nprob * sizeof(void *));
  if (!ptrs || !upload(A, a_elems, d.a32, &dA) || !upload(B, b_elems, d.b32, &dB) ||
      !upload(C, c_elems, d.c32, &dC)) {
    for (void *q : {(void *)dA, (void *)dB, (void *)dC, (void *)ptrs}) be->release(q);
    return fail(-4, "allocation failed");
  }
  std::vector<void *> h(3 * nprob);
  for (int p = 0; p < nprob; ++p) {
    h[p] = dA + a_elems * (d.a32 ? 8 : 16) * p;
    h[nprob + p] = dB + b_elems * (d.b32 ? 8 : 16) * p;
    h[2 * nprob + p] = dC + c_elems * (d.c32 ? 8 : 16) * p;
  }
  be->h2d(ptrs, h.data(), h.size() * sizeof(void *));
  be->gemm(d, (const double *const *)ptrs, (const double *const *)(ptrs + nprob),
           (double *const *)(ptrs + 2 * nprob), nprob);
  if (d.c32) {
    std::vector<float> t(2 * c_elems * nprob);
    be->d2h(t.data(), dC, t.size() * 4);
    for (size_t i = 0; i < t.size(); ++i) C[i] = t[i];
  } else {
    be->d2h(C, dC, c_elems * 16 * nprob);
  }
  be->release(dA);
  be->release(dB);
  be->release(dC);
  be->release(ptrs);
  std::string msg;
  int e = be->check(&msg);
  return e ? fail(e, msg) : 0;
}

extern "C" int bpki_test_bp_close(bpki_ctx *c, int32_t chi, int precision, int store32,
                                  int32_t pair, int64_t rs, int64_t qs, int64_t cs, int64_t ss,
                                  int32_t xdim, int nprob, const double *Y, const double *T,
                                  size_t y_elems, const double *M, double *out) {
  if (!c || !Y || !T || !M || !out || nprob < 1 || !bp_close_chi(chi) ||
      (precision != BPKI_FP64 && precision != BPKI_FP32) || (store32 != 0 && store32 != 1) ||
      (store32 && precision != BPKI_FP32) || (xdim != 1 && xdim != chi) || (pair != 0 && pair != 1))
    return fail(-1, "bad argument");
  if (rs < 0 || qs < 0 || cs < 0 || ss < 0) return fail(-1, "negative stride");
  const long C = chi;
  if ((size_t)((C - 1) * (rs + qs) + (xdim - 1) * cs + ss) >= y_elems)
    return fail(-1, "strides address outside the tensors");
  Backend *be = c->be.get();
  std::lock_guard<std::mutex> lk(c->mu);
  const size_t esz = store32 ? 8 : 16, cc = (size_t)C * C;
  char *dY = (char *)be->alloc(y_elems * esz * nprob);
  char *dT = (char *)be->alloc(y_elems * esz * nprob);
  double *dM = (double *)be->alloc(cc * 16 * nprob);
  double *dO = (double *)be->alloc(cc * 16 * nprob);
  void **ptrs = (void **)be->alloc(4 * nprob * sizeof(void *));
  if (!dY || !dT || !dM || !dO || !ptrs) {
    for (void *q : {(void *)dY, (void *)dT, (void *)dM, (void *)dO, (void *)ptrs}) be->release(q);
    return fail(-4, "allocation failed");
  }
  auto up = [&](char *d, const double *h) {
    if (store32) {
      std::vector<float> t(2 * y_elems * nprob);
      for (size_t i = 0; i < t.size(); ++i) t[i] = (float)h[i];
      be->h2d(d, t.data(), t.size() * 4);
    } else {
      be->h2d(d, h, y_elems * 16 * nprob);
    }
  };
  up(dY, Y);
  up(dT, T);
  be->h2d(dM, M, cc * 16 * nprob);
  std::vector<void *> h(4 * nprob);
  for (int p = 0; p < nprob; ++p) {
    h[p] = dY + y_elems * esz * p;
    h[nprob + p] = dT + y_elems * esz * p;
    h[2 * nprob + p] = dM + 2 * cc * p;
    h[3 * nprob + p] = dO + 2 * cc * p;
  }
  be->h2d(ptrs, h.data(), h.size() * sizeof(void *));
  BpCloseDesc d;
  d.chi = chi;
  d.rs[0] = rs; d.qs[0] = qs; d.cs[0] = cs; d.ss = ss;
  d.xdim = xdim;
  d.group = nprob;
  d.prec = precision == BPKI_FP32 ? 1 : 0;
  d.s32 = store32;
  d.pair = pair;
  be->bp_close(d, (const double *const *)ptrs, (const double *const *)(ptrs + nprob),
               (const double *const *)(ptrs + 2 * nprob), (double *const *)(ptrs + 3 * nprob),
               nprob);
  be->d2h(out, dO, cc * 16 * nprob);
  for (void *q : {(void *)dY, (void *)dT, (void *)dM, (void *)dO, (void *)ptrs}) be->release(q);
  std::string msg;
  int e = be->check(&msg);
  return e ? fail(e, msg) : 0;
}

extern "C" int bpki_test_eigh(bpki_ctx *c, int n, int nprob, int ncols, const double *A,
                              double *evals, double *vecs) {
  if (!c || n < 1 || n > 512 || nprob < 1 || ncols < 1 || ncols > n)
    return fail(-1, "bad argument");
  Backend *be = c->be.get();
  std::lock_guard<std::mutex> lk(c->mu);
  size_t nn = (size_t)n * n;
  double *dA = (double *)be->alloc(nn * 16 * nprob);
  double *dE = (double *)be->alloc((size_t)n * 8 * nprob);
  double *dV = (double *)be->alloc(nn * 16 * nprob);
  void **ptrs = (void **)be->alloc(3 * nprob * sizeof(void *));
  if (!dA || !dE || !dV || !ptrs) return fail(-4, "allocation failed");
  be->h2d(dA, A, nn * 16 * nprob);
  be->h2d(dV, vecs, nn * 16 * nprob);      // columns from ncols on keep these values
  std::vector<void *> h(3 * nprob);
  for (int p = 0; p < nprob; ++p) {
    h[p] = dA + 2 * nn * p;
    h[nprob + p] = dE + (size_t)n * p;
    h[2 * nprob + p] = dV + 2 * nn * p;
  }
  be->h2d(ptrs, h.data(), h.size() * sizeof(void *));
  be->eigh(n, n, (const double *const *)ptrs, (double *const *)(ptrs + nprob),
           (double *const *)(ptrs + 2 * nprob), nprob, ncols);
  be->d2h(evals, dE, (size_t)n * 8 * nprob);
  be->d2h(vecs, dV, nn * 16 * nprob);
  be->release(dA);
  be->release(dE);
  be->release(dV);
  be->release(ptrs);
  std::string msg;
  int e = be->check(&msg);
  return e ? fail(e, msg) : 0;
}

extern "C" int bpki_test_mfma_rate(bpki_ctx *c, int precision, int blocks, int iters,
                                   double *tflops) {
  if (!c || !tflops || (precision != BPKI_FP64 && precision != BPKI_FP32) || blocks < 1 ||
      blocks > (1 << 20) || iters < 1 || iters > (1 << 20))
    return fail(-1, "bad argument");
  std::lock_guard<std::mutex> lk(c->mu);
  *tflops = c->be->mfma_rate(precision, blocks, iters);
  std::string msg;
  if (int e = c->be->check(&msg)) return fail(e, "device error: " + msg);
  return 0;
}

extern "C" int bpki_test_gram_chol(bpki_ctx *c, int n, int nprob, const double *G, double cut,
                                   double *R, double *Wsc) {
  if (!c || n < 1 || n > 512 || nprob < 1 || !(cut >= 0)) return fail(-1, "bad argument");
  Backend *be = c->be.get();
  std::lock_guard<std::mutex> lk(c->mu);
  size_t nn = (size_t)n * n;
  double *dG = (double *)be->alloc(nn * 16 * nprob);
  double *dR = (double *)be->alloc(nn * 16 * nprob);
  double *dW = (double *)be->alloc(nn * 16 * nprob);
  void **ptrs = (void **)be->alloc(3 * nprob * sizeof(void *));
  if (!dG || !dR || !dW || !ptrs) return fail(-4, "allocation failed");
  be->h2d(dG, G, nn * 16 * nprob);
  std::vector<void *> h(3 * nprob);
  for (int p = 0; p < nprob; ++p) {
    h[p] = dG + 2 * nn * p;
    h[nprob + p] = dR + 2 * nn * p;
    h[2 * nprob + p] = dW + 2 * nn * p;
  }
  be->h2d(ptrs, h.data(), h.size() * sizeof(void *));
  be->gram_chol(n, (const double *const *)ptrs, (double *const *)(ptrs + nprob),
                (double *const *)(ptrs + 2 * nprob), cut, nprob);
  be->d2h(R, dR, nn * 16 * nprob);
  be->d2h(Wsc, dW, nn * 16 * nprob);
  be->release(dG);
  be->release(dR);
  be->release(dW);
  be->release(ptrs);
  std::string msg;
  int e = be->check(&msg);
  return e ? fail(e, msg) : 0;
}
