// Drives the C ABI of libbpki on the host stand-in backend (stub_backend.cpp), for a build under
// AddressSanitizer and UBSan: argument validation, memory estimates, blocking and allocation-free
// solves, sessions (every phase, state export/import, a session outliving its context), serving
// (slots, packing across lattices, budget admission, cancellation, rejection) and the caller's
// allocator (including one that refuses a request).  Exits non-zero on the first unexpected code.
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <set>
#include <vector>

#include "../../include/bpki.h"

static int failures = 0;
#define EXPECT(cond)                                                           \
  do {                                                                         \
    if (!(cond)) {                                                             \
      std::fprintf(stderr, "FAILED %s:%d: %s (%s)\n", __FILE__, __LINE__, #cond, \
                   bpki_last_error());                                          \
      ++failures;                                                              \
    }                                                                          \
  } while (0)

// A heavy-hex style lattice: a ring of n sites with a pendant on every third site.
struct Lattice {
  int n = 0;
  std::vector<int32_t> edges;
};

static Lattice ring_with_pendants(int ring) {
  Lattice L;
  L.n = ring;
  for (int i = 0; i < ring; ++i) {
    L.edges.push_back(i);
    L.edges.push_back((i + 1) % ring);
  }
  for (int i = 0; i < ring; i += 3) {
    L.edges.push_back(i);
    L.edges.push_back(L.n++);
  }
  return L;
}

struct Run {
  bpki_problem p;
  std::vector<double> z, pauli, res, disc, ent, gap;
  std::vector<int32_t> iters, dims, degen;
  std::vector<int32_t> po, ps;
  std::vector<uint8_t> pops;
  bpki_result r;
  Run(const Lattice &L, int depth, int chi, int precision = BPKI_FP64, int strings = 0) {
    bpki_problem_defaults(&p);
    p.n_sites = L.n;
    p.n_edges = (int32_t)L.edges.size() / 2;
    p.edges = L.edges.data();
    p.theta_h = 0.7;
    p.depth = depth;
    p.chi = chi;
    p.precision = precision;
    if (strings) {
      po = {0, 2, 5};
      ps = {0, 1, 3, 4, 5};
      pops = {1, 3, 2, 3, 1};
      p.n_pauli = 2;
      p.pauli_offsets = po.data();
      p.pauli_sites = ps.data();
      p.pauli_ops = pops.data();
    }
    const int steps = depth, rows = steps > 0 ? steps : 1;
    z.assign((size_t)rows * L.n, 0.0);
    pauli.assign(2, 0.0);
    res.assign(rows, 0.0);
    disc.assign(rows, 0.0);
    gap.assign(rows, 0.0);
    ent.assign((size_t)rows * p.n_edges, 0.0);
    iters.assign(rows, 0);
    dims.assign((size_t)rows * p.n_edges, 0);
    degen.assign(rows, 0);
    std::memset(&r, 0, sizeof(r));
    r.z = z.data();
    r.pauli = pauli.data();
    r.bp_iters = iters.data();
    r.bp_residual = res.data();
    r.discarded = disc.data();
    r.bond_entropy = ent.data();
    r.bond_dims = dims.data();
    r.min_cut_gap = gap.data();
    r.degenerate_cuts = degen.data();
  }
};

// An aligned host allocator standing in for a framework's caching allocator, which refuses
// requests above `limit` bytes.
struct Pool {
  std::mutex mu;
  std::set<void *> live;
  size_t limit = (size_t)1 << 40;
};
static void *pool_alloc(size_t bytes, void *, void *user) {
  Pool *p = static_cast<Pool *>(user);
  if (bytes > p->limit) return nullptr;
  void *q = std::aligned_alloc(256, (bytes + 255) & ~(size_t)255);
  std::lock_guard<std::mutex> lk(p->mu);
  p->live.insert(q);
  return q;
}
static void pool_free(void *q, void *, void *user) {
  Pool *p = static_cast<Pool *>(user);
  {
    std::lock_guard<std::mutex> lk(p->mu);
    if (!p->live.erase(q)) std::abort();                     // freed twice or never given
  }
  std::free(q);
}

int main() {
  const Lattice L = ring_with_pendants(12), Lbig = ring_with_pendants(30);

  // validation
  {
    Run a(L, 3, 4);
    EXPECT(bpki_validate(&a.p) == 0);
    a.p.chi = 0;
    EXPECT(bpki_validate(&a.p) == -1);
    a.p.chi = 4;
    a.p.theta_h = NAN;
    EXPECT(bpki_validate(&a.p) == -1);
    a.p.theta_h = 0.7;
    std::vector<int32_t> bad = L.edges;
    bad[1] = bad[0];                                        // self loop
    a.p.edges = bad.data();
    EXPECT(bpki_validate(&a.p) == -2);
    a.p.edges = L.edges.data();
    std::vector<int32_t> col(a.p.n_edges, 0);               // improper colouring
    a.p.colour = col.data();
    EXPECT(bpki_validate(&a.p) == -3);
    a.p.colour = nullptr;
    size_t bytes = 0;
    EXPECT(bpki_estimate_bytes(&a.p, &bytes) == 0 && bytes > 0);
    EXPECT(bpki_validate(nullptr) == -1);
  }

  bpki_ctx *ctx = nullptr;
  EXPECT(bpki_create(&ctx, 1, nullptr, 0) == -5);           // the stub has device 0 only
  EXPECT(bpki_create(&ctx, 0, nullptr, 0) == 0);

  // blocking solves, FP64 and mixed, with Pauli strings
  for (int prec : {BPKI_FP64, BPKI_FP32}) {
    Run a(L, 4, 4, prec, 1);
    EXPECT(bpki_solve(ctx, &a.p, &a.r) == 0);
    EXPECT(a.z[0] == 1.0 && a.dims[0] == 1 && a.iters[0] == 1);
    Run b(L, 0, 4);
    EXPECT(bpki_solve(ctx, &b.p, &b.r) == 0);
  }
  {
    Run a(L, 2, 4);
    a.p.clifford_steps = 2;
    std::vector<double> z(4 * L.n);
    a.r.z = z.data();
    std::vector<int32_t> it(4), dm(4 * a.p.n_edges), dg(4);
    std::vector<double> rs(4), dc(4), gp(4), en(4 * a.p.n_edges);
    a.r.bp_iters = it.data();
    a.r.bp_residual = rs.data();
    a.r.discarded = dc.data();
    a.r.min_cut_gap = gp.data();
    a.r.bond_entropy = en.data();
    a.r.bond_dims = dm.data();
    a.r.degenerate_cuts = dg.data();
    EXPECT(bpki_solve(ctx, &a.p, &a.r) == 0);
  }

  // allocation-free solves: two in a row, then one above the scratch size
  {
    Run a(Lbig, 3, 8), b(L, 2, 4);
    EXPECT(bpki_solve_noalloc(ctx, &a.p, &a.r) == 0);
    EXPECT(bpki_solve_noalloc(ctx, &b.p, &b.r) == 0);
    Run c(Lbig, 2, 64);
    EXPECT(bpki_solve_noalloc(ctx, &c.p, &c.r) == -4);
    EXPECT(bpki_solve_noalloc(ctx, &b.p, &b.r) == 0);
  }

  // sessions: every phase, state round trip, a session that outlives its context
  bpki_session *s = nullptr;
  {
    Run a(L, 3, 4, BPKI_FP64, 1);
    EXPECT(bpki_session_open(ctx, &a.p, &s) == 0);
    size_t te = 0, me = 0;
    EXPECT(bpki_session_sizes(s, &te, &me) == 0);
    std::vector<double> t(2 * te), m(2 * me), z(L.n), ent(a.p.n_edges), lam(a.p.n_edges * 4);
    std::vector<int32_t> bd(a.p.n_edges), kept(a.p.n_edges);
    std::vector<double> dsc(a.p.n_edges), gp(a.p.n_edges), spec(16), ms4(4), pv(2);
    int32_t it = 0;
    double r = 0, d = 0, err = 0;
    EXPECT(bpki_session_apply_rx(s) == 0);
    EXPECT(bpki_session_apply_layer(s, 0, &d) == 0);
    EXPECT(bpki_session_layer_cuts(s, kept.data(), dsc.data(), gp.data()) == 0);
    EXPECT(bpki_session_bp(s, 50, &it, &r) == 0);
    EXPECT(bpki_session_bp_sweep(s, &r) == 0);
    EXPECT(bpki_session_observe_z(s, z.data()) == 0);
    EXPECT(bpki_session_observe_bond_entropy(s, ent.data()) == 0);
    EXPECT(bpki_session_step(s, z.data(), &it, &r, &d) == 0);
    EXPECT(bpki_session_clifford_inverse_step(s, z.data(), &it, &r, &d) == 0);
    EXPECT(bpki_session_get_state(s, t.data(), m.data(), bd.data()) == 0);
    EXPECT(bpki_session_set_state(s, t.data(), m.data(), bd.data()) == 0);
    EXPECT(bpki_session_observe_pauli(s, pv.data()) == 0);
    EXPECT(bpki_session_vidal_gauge(s, lam.data()) == 0);
    EXPECT(bpki_session_bp_error(s, 0, &err, spec.data()) == 0);    // an edge of the loop
    err = -1.0;
    EXPECT(bpki_session_bp_error(s, 12, &err, spec.data()) == 0);   // a pendant: a bridge
    EXPECT(err == 0.0 && spec[0] == 1.0 && spec[1] == 0.0);
    EXPECT(bpki_session_profile(s, 3) == 0);
    EXPECT(bpki_session_step(s, nullptr, &it, &r, &d) == 0);
    int64_t n1 = 0, n2 = 0;
    double ms = 0, fl = 0;
    EXPECT(bpki_session_profile_read(s, &n1, &ms, &fl, &n2) == 0);
    EXPECT(bpki_session_profile_read_prec(s, 1, &n1, &ms, &fl) == 0);
    double by = 0;
    EXPECT(bpki_session_profile_read_kernel(s, 1, 0, &n1, &ms, &fl, &by, &n2) == 0);
    EXPECT(bpki_session_profile_read_kernel(s, 2, 0, &n1, &ms, &fl, nullptr, nullptr) == 0);
    EXPECT(bpki_session_profile_read_kernel(s, 3, 0, &n1, &ms, &fl, &by, &n2) == -1);
    EXPECT(bpki_session_last_timing(s, ms4.data()) == 0);
  }
  {
    // BP error estimate on a network whose 2-core is two junctions (0, 3) joined by three paths,
    // then its refusal once a third loop is added
    Lattice T;
    T.n = 9;
    T.edges = {0, 1, 1, 2, 2, 3, 3, 4, 4, 5, 5, 0, 0, 6, 6, 7, 7, 8, 8, 3};
    bpki_session *st = nullptr;
    std::vector<double> sp(16);
    double e2 = 0.0;
    {
      Run a(T, 1, 4);
      EXPECT(bpki_session_open(ctx, &a.p, &st) == 0);
      for (int e = 0; e < a.p.n_edges; ++e)
        EXPECT(bpki_session_bp_error(st, e, &e2, sp.data()) == 0);
      bpki_session_close(st);
    }
    T.n = 10;
    for (int x : {1, 9, 9, 4}) T.edges.push_back(x);
    Run b(T, 1, 4);
    EXPECT(bpki_session_open(ctx, &b.p, &st) == 0);
    EXPECT(bpki_session_bp_error(st, 0, &e2, sp.data()) == -1);
    bpki_session_close(st);
  }
  bpki_destroy(ctx);                                          // the session keeps it alive
  {
    double r = 0;
    EXPECT(bpki_session_bp_sweep(s, &r) == 0);
    bpki_session_close(s);
  }

  // serving: slots, packing across lattices, cancellation, rejection, budget admission
  {
    Run probe(Lbig, 4, 8);
    size_t one = 0;
    bpki_estimate_bytes(&probe.p, &one);
    EXPECT(bpki_create(&ctx, 0, nullptr, 3 * one) == 0);
    EXPECT(bpki_serving_config(ctx, 3) == 0);
    EXPECT(bpki_serving_packing(ctx, 8, 16) == 0);
    std::vector<Run *> runs;
    std::vector<uint64_t> tickets;
    for (int i = 0; i < 24; ++i) {
      runs.push_back(new Run(i % 2 ? L : Lbig, 1 + i % 4, 8, i % 3 ? BPKI_FP64 : BPKI_FP32));
      uint64_t t = 0;
      EXPECT(bpki_submit(ctx, &runs.back()->p, &runs.back()->r, &t) == 0);
      tickets.push_back(t);
    }
    EXPECT(bpki_cancel(ctx, tickets[20]) == 0);
    Run huge(Lbig, 2, 64);
    uint64_t th = 0;
    EXPECT(bpki_submit(ctx, &huge.p, &huge.r, &th) == -4);     // can never fit the budget
    EXPECT(bpki_serving_config(ctx, 4) == -1);                  // serving already started
    for (size_t i = 0; i < tickets.size(); ++i) {
      int done = 0;
      EXPECT(bpki_poll(ctx, tickets[i], &done) >= -6);
      double times[3];
      EXPECT(bpki_ticket_times(ctx, tickets[i], times) == 0);
      int32_t ps = 0;
      EXPECT(bpki_ticket_pack_size(ctx, tickets[i], &ps) == 0);
      const int rc = bpki_wait(ctx, tickets[i]);
      EXPECT(rc == 0 || (i == 20 && rc == -6));
    }
    EXPECT(bpki_wait(ctx, tickets[0]) == -7);                   // forgotten
    // a few left queued when the context goes away
    for (int i = 0; i < 4; ++i) {
      uint64_t t = 0;
      EXPECT(bpki_submit(ctx, &runs[i]->p, &runs[i]->r, &t) == 0);
    }
    bpki_destroy(ctx);
    for (Run *r : runs) delete r;
  }

  // the caller's allocator, one request refused, later ones served
  {
    Pool pool;
    EXPECT(bpki_create(&ctx, 0, nullptr, 0) == 0);
    EXPECT(bpki_set_allocator(ctx, pool_alloc, pool_free, &pool) == 0);
    Run a(L, 2, 4);
    EXPECT(bpki_solve(ctx, &a.p, &a.r) == 0);
    EXPECT(bpki_set_allocator(ctx, nullptr, nullptr, nullptr) == -1);   // memory taken
    EXPECT(bpki_serving_config(ctx, 1) == 0);
    pool.limit = 1 << 16;
    Run big(Lbig, 3, 16);
    uint64_t t = 0;
    EXPECT(bpki_submit(ctx, &big.p, &big.r, &t) == 0);
    EXPECT(bpki_wait(ctx, t) == -4);
    pool.limit = (size_t)1 << 40;
    for (int i = 0; i < 3; ++i) {
      Run b(L, 2, 4);
      EXPECT(bpki_submit(ctx, &b.p, &b.r, &t) == 0);
      EXPECT(bpki_wait(ctx, t) == 0);
    }
    bpki_destroy(ctx);
    EXPECT(pool.live.empty());
  }
  if (failures) std::fprintf(stderr, "%d failures\n", failures);
  else std::printf("host ABI checks passed\n");
  return failures ? 1 : 0;
}
