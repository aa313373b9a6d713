// Engine: the Floquet-step schedule of the BP-gauged simple update (arXiv 2306.14887, Methods)
// expressed as batched device primitives.  All state lives in device memory; the host only
// builds launch descriptors and reads back scalars (BP residual, observables).
//
// Gate update on edge (x, y), both endpoints (Methods, "The simple update procedure", reduced-
// tensor variant):
//   1. X = M^{1/2}, X+ = M^{+1/2} of every message entering x from its other neighbours (eigh).
//   2. A_x = T_x with X absorbed on the environment legs, laid out [env][s][a_y].
//   3. Isolate the bond: degree <= 2: R_x = A_x (rows = environment), Q_x = I.
//      degree 3: A_x = Q_x R_x from the Gram matrix G = A^H A = W L W^H (eigh):
//      R_x = L^{1/2} W^H, Q_x = A_x W L^{-1/2} formed explicitly (orthonormal columns).
//   4. Theta = gate phases * (R_x contracted with R_y over the shared bond).
//   5. Truncated SVD of Theta from eigh(Theta^H Theta): keep min(chi, #sigma > cutoff*sigma_1)
//      values, normalise S; the edge's two messages become diag(S)/sum(S).
//   6. R_x' = U sqrt(S), R_y' = sqrt(S) V^H; T~_x' = Q_x R_x'; T_x' = T~_x' with X+ absorbed.
// BP sweep (Eq. "MessageTensorSelfConsistency"): every directed message from the site tensor, its
// conjugate and the other incoming messages; unit complex trace; residual = max Frobenius change.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <set>
#include <functional>
#include <stdexcept>
#include <tuple>

#include "bpki_internal.h"

namespace bpki {

namespace {

struct GemmOp {
  GemmDesc d;
  size_t a = 0, b = 0, c = 0;      // offsets into the pointer arena
  int n = 0;
  // fused: a fused degree-3 BP closing (BpCloseDesc f): Y at a, the message applied at b, the
  // output at c, the site tensor at t
  int fused = 0;
  BpCloseDesc f;
  size_t t = 0;
};

// Device arrays of pointers, built on the host and uploaded once.
struct PtrArena {
  std::vector<const void *> host;
  void **dev = nullptr;
  size_t add(const std::vector<const void *> &v) {
    size_t off = host.size();
    host.insert(host.end(), v.begin(), v.end());
    return off;
  }
  template <class T>
  T at(size_t off) const { return reinterpret_cast<T>(dev + off); }
};

inline long ipow(long b, int e) { long r = 1; while (e-- > 0) r *= b; return r; }

// Relative pivot threshold of the Gram-matrix Cholesky: directions of A whose squared weight is
// below this fraction of the largest are at the FP64 rounding level of the Gram matrix.
constexpr double kGramCut = 1e-15;

// Residual below which FP32 message contractions stop making progress (their rounding level).
// Within kFp32Near times that level, a sweep that reduces the residual by less than kFp32Stall
// also ends the FP32 phase (it has reached the noise of the FP32 products).
constexpr double kFp32BpFloor = 2e-6;
constexpr double kFp32Near = 100.0;
constexpr double kFp32Stall = 0.9;
// A sweep is launched ahead of the previous residual only if the residual extrapolated from the two
// before stays this many times above the point where the loop would stop or change arithmetic.
constexpr double kSpecMargin = 8.0;

inline bool fp32_done(double r, double prev) {
  return r < kFp32BpFloor || (r < kFp32Near * kFp32BpFloor && r > kFp32Stall * prev);
}

}  // namespace

// Strides of a site tensor's indices: s first, then one per leg.
struct Layout {
  long s = 0;
  long leg[3] = {0, 0, 0};
};

struct Endpoint {
  int x = -1, y = -1;     // this site, partner
  int j = -1;             // leg of x that points at y
  int deg = 0;
  int env[2] = {-1, -1};  // environment legs (ascending)
  int r = 0;              // rows of R_x
  bool big = false;       // rows side of Theta
  int edge_slot = -1;
};

struct EdgeWork {
  int e = -1;
  int ep[2] = {-1, -1};   // endpoint slots: [0] = big side, [1] = small side
};

struct LayerPlan {
  std::vector<Endpoint> eps;
  std::vector<EdgeWork> edges;
  // message eigh + sqrt
  size_t m_in = 0, m_ev = 0, m_vec = 0, m_X = 0, m_Xp = 0;
  int n_msg = 0;
  std::vector<GemmOp> absorb;       // (grouped)
  // deg-3 gram factor
  GemmOp gram;
  size_t g_in = 0, g_ev = 0, g_vec = 0, g_R = 0, g_Wsc = 0;
  int n_g = 0;
  GemmOp wr;                        // deg-3 endpoints: WR = Wsc R'
  // per (rB, rS) edge type
  struct Type {
    int rB = 0, rS = 0, n = 0;
    size_t RB = 0, RS = 0, Th = 0, ev = 0, vec = 0, Vs = 0, S = 0, mA = 0, mB = 0, RBn = 0, RSn = 0,
           U = 0;
    GemmOp hgemm, ugemm;
    int count = 0;
    int slot0 = 0;                  // first edge slot of this type (k / disc arrays)
  };
  std::vector<Type> types;
  // all Theta^H Theta of one size share one eigensolver launch (each matrix gets one workgroup,
  // so a launch costs the same for 3 or 50 matrices)
  struct EighGroup {
    int n = 0, count = 0;
    size_t in = 0, ev = 0, vec = 0;
  };
  std::vector<EighGroup> eig_groups;
  // deg-3 endpoints: Tt = A WR (= Q R' with Q = A Wsc), written in T-order; one per bond leg
  std::vector<GemmOp> rebuild;
  std::vector<GemmOp> remove;       // grouped
  std::vector<std::pair<size_t, size_t>> copies_in, copies_out;  // deg-1 (dst, src, bytes) as ptr
  std::vector<std::tuple<double *, const double *, size_t>> d2d_in, d2d_out;
};

struct Plan {
  int n = 0, chi = 1, E = 0;
  std::vector<int> deg;
  std::vector<std::vector<int>> nb;
  std::vector<long> toff;          // tensor offsets (complex elements)
  std::vector<long> tsize;
  std::vector<std::vector<int>> in_msg, out_msg;
  std::vector<int> layer_colours;
  std::vector<std::vector<int>> layer_edges;

  double *T = nullptr;             // all site tensors
  double *M = nullptr;             // current messages  [2E][chi][chi]
  double *Mn = nullptr;            // BP output buffer
  double *ws = nullptr;            // SU workspace (max over layers)
  double *bpws = nullptr;          // BP / observable workspace
  double *res = nullptr;           // per-message residual [2E]
  double *resmax = nullptr;        // [2]: the largest residual of a sweep (two in flight)
  double *rho = nullptr;           // [n][4] complex
  int *kbuf = nullptr;             // [max edges per layer]
  double *disc = nullptr;          // [max edges per layer]
  int *bond = nullptr;             // host copy of bond dims is kept in bond_h
  std::vector<int> bond_h;
  int64_t *rx_half = nullptr;
  int64_t *rho_len = nullptr;
  size_t rx_ptrs = 0;
  size_t ws_elems = 0, bpws_elems = 0;
  PtrArena arena;
  std::vector<LayerPlan> layers;
  // BP: one group of launches per vertex class of the sweep schedule
  struct BpClass {
    std::vector<GemmOp> ops;
    size_t norm_new = 0, norm_old = 0;
    int nmsg = 0, res_off = 0;
  };
  std::vector<BpClass> bp_classes;
  // mixed precision: the same sweep on FP32 copies of the site tensors and FP32 intermediates
  // (FP32 MFMA; messages, normalisation and residual stay FP64)
  std::vector<BpClass> bp_classes32;
  float *T32 = nullptr, *bpws32 = nullptr;
  // packed solves: member of every residual slot (CSR by member), member of every message,
  // active flags (ping-pong) and per-member residuals
  int nmem = 1;
  std::vector<int> site_member;
  int *mem_off = nullptr, *mem_idx = nullptr, *msg_member = nullptr, *act[2] = {nullptr, nullptr};
  double *res_m = nullptr;
  // observables
  std::vector<GemmOp> obs_ops;
  size_t obs_Y = 0, obs_T = 0;
  // bond entropies: X = sqrt(M_{u->v}), Y = X M_{v->u}^T, B = Y X, eigenvalues of B
  size_t ent_m = 0, ent_ev = 0, ent_vec = 0, ent_X = 0, ent_Y = 0, ent_B = 0;
  GemmOp ent_xm, ent_b;
  double *ent_out = nullptr;       // [E]
  // explicit Vidal gauge: square roots of all 2E messages, C = X_u^T X_v, eigh(C^H C), the gauge
  // factors P_u = X_u^{T+} C D1, P_v = X_v^{T+} D2, then every leg absorbs its factor
  size_t vg_m = 0, vg_ev = 0, vg_vec = 0, vg_X = 0, vg_Xp = 0, vg_ev3 = 0, vg_vec3 = 0,
         vg_D1 = 0, vg_D2 = 0, vg_Mu = 0, vg_Mv = 0;
  GemmOp vg_c, vg_h, vg_t1, vg_pu, vg_pv;
  std::vector<GemmOp> vg_ops;
  std::vector<std::pair<double *, const double *>> vg_copy;   // degree-1 sites: result -> T
  std::vector<size_t> vg_copy_len;
  double *vg_lam = nullptr;        // [E][chi]
  int *vg_kept = nullptr;          // [E]
  int max_layer_edges = 0;
  std::vector<void *> allocs;
};

// ------------------------------------------------------------------------------------------
// descriptor helpers

static Layout t_layout(int deg, int chi) {
  Layout L;
  L.s = ipow(chi, deg);
  for (int i = 0; i < deg; ++i) L.leg[i] = ipow(chi, deg - 1 - i);
  return L;
}

// Layout of A_x = [env_0][env_1][s][a_j] (environment legs in ascending leg order).
static Layout a_layout(const Endpoint &p, int chi) {
  Layout L;
  L.leg[p.j] = 1;
  L.s = chi;
  long st = 2L * chi;
  for (int t = p.deg - 2; t >= 0; --t) {
    L.leg[p.env[t]] = st;
    st *= chi;
  }
  return L;
}

// Contract leg `L` of a tensor (degree deg, layout in) with a chi x chi matrix X[a][b]; the new
// index b takes the place of the leg in layout out.  Batch over s, M over the other legs.
static GemmDesc leg_desc(int deg, int leg, const Layout &in, const Layout &out, int chi) {
  GemmDesc d;
  int others[2] = {-1, -1};
  int no = 0;
  for (int i = 0; i < deg; ++i)
    if (i != leg) others[no++] = i;
  d.batch = 2;
  d.a_b = in.s;
  d.b_b = 0;
  d.c_b = out.s;
  if (no == 0) {
    d.M = 1; d.Mi = 1;
  } else if (no == 1) {
    d.M = chi; d.Mi = chi;
    d.a_mi = in.leg[others[0]]; d.c_mi = out.leg[others[0]];
  } else {
    // M = (outer, inner) over the two other legs, in the order that lets both the loads (a unit
    // stride along K or the inner M index) and the stores (along the inner M index or N) run on
    // consecutive addresses when one order does; otherwise ascending leg order.  The order only
    // decides which rows a workgroup owns, not how an element is summed.
    auto coalesced = [&](int inner) {
      return (in.leg[inner] == 1 || in.leg[leg] == 1) && (out.leg[inner] == 1 || out.leg[leg] == 1);
    };
    const bool swap = !coalesced(others[1]) && coalesced(others[0]);
    const int mo = swap ? others[1] : others[0], mi = swap ? others[0] : others[1];
    d.M = chi * chi; d.Mi = chi;
    d.a_mo = in.leg[mo]; d.a_mi = in.leg[mi];
    d.c_mo = out.leg[mo]; d.c_mi = out.leg[mi];
  }
  d.K = chi; d.Ki = chi; d.a_ki = in.leg[leg];
  d.b_ki = chi;
  d.N = chi; d.Ni = chi; d.b_ni = 1; d.c_ni = out.leg[leg];
  return d;
}

// out[a][a'] = sum over s and all legs but `leg` of Y[..a..] conj(T[..a'..]) (both in layout L).
static GemmDesc close_desc(int deg, int leg, const Layout &L, int chi) {
  GemmDesc d;
  d.M = chi; d.Mi = chi; d.a_mi = L.leg[leg];
  d.N = chi; d.Ni = chi; d.b_ni = L.leg[leg]; d.c_ni = 1;
  d.c_mi = chi;
  d.conjB = 1;
  // K = (s, other legs).  T-order layouts have s outermost and the other legs in order, so the
  // summed indices split into at most two uniformly strided runs.
  int others[2] = {-1, -1};
  int no = 0;
  for (int i = 0; i < deg; ++i)
    if (i != leg) others[no++] = i;
  if (no == 0) {                    // K = s
    d.K = 2; d.Ki = 2; d.a_ki = L.s; d.b_ki = L.s;
  } else if (no == 1) {             // K = (s, o)
    d.K = 2 * chi; d.Ki = chi;
    d.a_ko = L.s; d.a_ki = L.leg[others[0]];
    d.b_ko = L.s; d.b_ki = L.leg[others[0]];
  } else {
    // (s, o0, o1): s and the outer other leg fuse when the summed leg is not between them
    if (leg == 0) {                 // (s) x (o0 o1 contiguous)
      d.K = 2 * chi * chi; d.Ki = chi * chi;
      d.a_ko = L.s; d.a_ki = L.leg[2];
      d.b_ko = L.s; d.b_ki = L.leg[2];
    } else if (leg == 1) {          // (s o0) x (o1)
      d.K = 2 * chi * chi; d.Ki = chi;
      d.a_ko = L.leg[0]; d.a_ki = L.leg[2];
      d.b_ko = L.leg[0]; d.b_ki = L.leg[2];
    } else {                        // (s o0 o1) uniform stride
      d.K = 2 * chi * chi; d.Ki = 2 * chi * chi;
      d.a_ki = L.leg[1];
      d.b_ki = L.leg[1];
    }
  }
  return d;
}

// ------------------------------------------------------------------------------------------

Engine::Engine(Backend *be, const Problem &p)
    : be_(be), prob_(p), plan_(new Plan), bp_prec_(p.precision ? 1 : 0) {
  build();
}

Engine::~Engine() {
  for (void *a : plan_->allocs) be_->release(a);
  if (plan_->arena.dev) be_->release(plan_->arena.dev);
  delete plan_;
}

int Engine::n_colours() const { return (int)plan_->layer_colours.size(); }
size_t Engine::tensor_elems() const {
  size_t s = 0;
  for (long t : plan_->tsize) s += (size_t)t;
  return s;
}
size_t Engine::message_elems() const { return (size_t)2 * plan_->E * plan_->chi * plan_->chi; }

size_t Engine::estimate_bytes(const Problem &p) {
  // tensors + 2 message buffers + SU workspace bound + BP workspace bound
  int n = p.n_sites;
  std::vector<int> deg(n, 0);
  for (size_t i = 0; i < p.edges.size(); ++i) deg[p.edges[i]]++;
  long chi = p.chi;
  size_t t = 0, bp = 0, su = 0;
  for (int v = 0; v < n; ++v) {
    long sz = 2 * ipow(chi, deg[v]);
    t += sz;
    bp += (deg[v] == 3 ? 5 : deg[v] == 2 ? 2 : 0) * sz;
    su += (deg[v] == 3 ? 4 : 3) * sz + 16 * chi * chi;
  }
  size_t m = (size_t)2 * p.edges.size() / 2 * chi * chi;
  size_t elems = t + 2 * m + su + bp + (size_t)p.edges.size() * 64 * chi * chi;
  // mixed precision: FP32 copies of the site tensors and of the BP intermediates
  if (p.precision == 1) elems += (t + bp + 64 * (size_t)n) / 2;
  return elems * 16 + (8u << 20);
}

void Engine::build() {
  Plan &P = *plan_;
  const Problem &p = prob_;
  P.n = p.n_sites;
  P.chi = p.chi;
  P.E = (int)p.edges.size() / 2;
  const int chi = P.chi;
  const long c2 = (long)chi * chi;
  P.nb.assign(P.n, {});
  for (int e = 0; e < P.E; ++e) {
    P.nb[p.edges[2 * e]].push_back(p.edges[2 * e + 1]);
    P.nb[p.edges[2 * e + 1]].push_back(p.edges[2 * e]);
  }
  P.deg.resize(P.n);
  for (int v = 0; v < P.n; ++v) {
    std::sort(P.nb[v].begin(), P.nb[v].end());
    P.deg[v] = (int)P.nb[v].size();
  }
  P.site_member.assign(P.n, 0);
  if (p.member_site0.size() > 2) {
    P.nmem = (int)p.member_site0.size() - 1;
    for (int j = 0; j < P.nmem; ++j)
      for (int v = p.member_site0[j]; v < p.member_site0[j + 1]; ++v) P.site_member[v] = j;
  }
  // messages: 2e = edges[2e] -> edges[2e+1], 2e+1 reverse
  std::map<std::pair<int, int>, int> midx;
  for (int e = 0; e < P.E; ++e) {
    midx[{p.edges[2 * e], p.edges[2 * e + 1]}] = 2 * e;
    midx[{p.edges[2 * e + 1], p.edges[2 * e]}] = 2 * e + 1;
  }
  P.in_msg.assign(P.n, {});
  P.out_msg.assign(P.n, {});
  for (int v = 0; v < P.n; ++v)
    for (int u : P.nb[v]) {
      P.in_msg[v].push_back(midx[{u, v}]);
      P.out_msg[v].push_back(midx[{v, u}]);
    }
  long off = 0;
  P.toff.resize(P.n);
  P.tsize.resize(P.n);
  for (int v = 0; v < P.n; ++v) {
    P.toff[v] = off;
    P.tsize[v] = 2 * ipow(chi, P.deg[v]);
    off += P.tsize[v];
  }
  // layers
  std::vector<int> cols(p.colour.begin(), p.colour.end());
  std::vector<int> uniq = cols;
  std::sort(uniq.begin(), uniq.end());
  uniq.erase(std::unique(uniq.begin(), uniq.end()), uniq.end());
  P.layer_colours = uniq;
  P.layer_edges.assign(uniq.size(), {});
  for (int e = 0; e < P.E; ++e) {
    int li = (int)(std::lower_bound(uniq.begin(), uniq.end(), cols[e]) - uniq.begin());
    P.layer_edges[li].push_back(e);
  }
  for (auto &le : P.layer_edges) P.max_layer_edges = std::max(P.max_layer_edges, (int)le.size());

  // ---- device allocations ----
  auto A = [&](size_t bytes) {
    void *q = be_->alloc(bytes ? bytes : 16);
    P.allocs.push_back(q);
    return q;
  };
  P.T = (double *)A((size_t)off * 16);
  P.M = (double *)A(message_elems() * 16);
  P.Mn = (double *)A(message_elems() * 16);
  P.res = (double *)A((size_t)std::max(1, 2 * P.E) * 8);
  P.resmax = (double *)A(16);
  P.rho = (double *)A((size_t)P.n * 8 * 8);
  P.kbuf = (int *)A((size_t)std::max(1, P.max_layer_edges) * 4);
  P.disc = (double *)A((size_t)std::max(1, P.max_layer_edges) * 16);   // (discarded, gap) pairs
  P.bond_h.assign(P.E, 1);

  auto Tp = [&](int v) { return (const void *)(P.T + 2 * P.toff[v]); };
  auto Mp = [&](int m) { return (const void *)(P.M + 2 * (size_t)m * c2); };
  auto Mnp = [&](int m) { return (const void *)(P.Mn + 2 * (size_t)m * c2); };

  // ---- SU layer plans (workspace offsets computed first, pointers after allocation) ----
  struct Slot { size_t off, elems; };
  size_t ws_max = 0;
  std::vector<std::vector<size_t>> dummy;
  // First pass: compute per-layer workspace need.
  auto ep_need = [&](int deg) -> size_t {
    long env = ipow(chi, deg - 1);
    size_t need = 0;
    need += 2 * (2 * c2) + 2 * c2 + 2 * chi;       // X, Xp (2 legs), W, evals (per leg reuse)
    need += 2 * c2 * 2;                            // more eigh room
    need += (size_t)env * 2 * chi * 3;             // Y1/A, Q, Tt
    need += 4 * c2 * 4 + 2 * chi;                  // G, W, R, Wsc
    need += (size_t)(deg == 3 ? 2 * chi : env) * 2 * chi; // R'
    return need;
  };
  (void)ep_need;

  P.layers.resize(P.layer_edges.size());
  std::vector<size_t> layer_ws(P.layers.size(), 0);
  // Sizes of the per-layer arena are determined while building; we build with a bump allocator
  // over a virtual base and allocate once with the maximum.
  for (size_t li = 0; li < P.layers.size(); ++li) {
    LayerPlan &LP = P.layers[li];
    const auto &le = P.layer_edges[li];
    for (size_t q = 0; q < le.size(); ++q) {
      int e = le[q];
      int u = p.edges[2 * e], v = p.edges[2 * e + 1];
      Endpoint a, b;
      a.x = u; a.y = v; b.x = v; b.y = u;
      for (Endpoint *ep : {&a, &b}) {
        ep->deg = P.deg[ep->x];
        ep->j = (int)(std::find(P.nb[ep->x].begin(), P.nb[ep->x].end(), ep->y) -
                      P.nb[ep->x].begin());
        int t = 0;
        for (int i = 0; i < ep->deg; ++i)
          if (i != ep->j) ep->env[t++] = i;
        ep->r = ep->deg == 3 ? 2 * chi : (int)ipow(chi, ep->deg - 1);
        ep->edge_slot = (int)q;
      }
      // big side = more rows (ties: first endpoint)
      Endpoint *B = &a, *S = &b;
      if (b.r > a.r) std::swap(B, S);
      B->big = true;
      S->big = false;
      EdgeWork w;
      w.e = e;
      w.ep[0] = (int)LP.eps.size();
      LP.eps.push_back(*B);
      w.ep[1] = (int)LP.eps.size();
      LP.eps.push_back(*S);
      LP.edges.push_back(w);
    }
  }

  // workspace per layer: bump allocator (offsets in complex elements)
  struct Bump {
    size_t top = 0;
    size_t take(size_t n) { size_t o = top; top += (n + 31) & ~size_t(31); return o; }
  };
  // we need to know the base pointer before building pointer arrays; compute sizes in a dry run
  auto layer_build = [&](LayerPlan &LP, double *base, Bump &bump, bool real) {
    auto W = [&](size_t off) { return (const void *)(base + 2 * off); };
    auto Wr = [&](size_t off) { return (const void *)((double *)base + 2 * off); };
    (void)Wr;
    // 1. message eigh for env legs
    std::vector<const void *> min, mev, mvec, mX, mXp;
    std::vector<size_t> xoff(LP.eps.size() * 2, 0), xpoff(LP.eps.size() * 2, 0);
    for (size_t q = 0; q < LP.eps.size(); ++q) {
      const Endpoint &ep = LP.eps[q];
      for (int t = 0; t < ep.deg - 1; ++t) {
        int m = P.in_msg[ep.x][ep.env[t]];
        size_t o_ev = bump.take(chi), o_vec = bump.take(c2), o_X = bump.take(c2),
               o_Xp = bump.take(c2);
        xoff[2 * q + t] = o_X;
        xpoff[2 * q + t] = o_Xp;
        min.push_back(Mp(m));
        mev.push_back(W(o_ev));
        mvec.push_back(W(o_vec));
        mX.push_back(W(o_X));
        mXp.push_back(W(o_Xp));
      }
    }
    LP.n_msg = (int)min.size();
    if (real) {
      LP.m_in = P.arena.add(min); LP.m_ev = P.arena.add(mev); LP.m_vec = P.arena.add(mvec);
      LP.m_X = P.arena.add(mX); LP.m_Xp = P.arena.add(mXp);
    }
    // 2. absorb into A-layout; allocate A, WR, Tt, Y1 per endpoint
    std::vector<size_t> aoff(LP.eps.size()), wroff(LP.eps.size()), ttoff(LP.eps.size()),
        y1off(LP.eps.size()), roff(LP.eps.size()), rnoff(LP.eps.size());
    for (size_t q = 0; q < LP.eps.size(); ++q) {
      const Endpoint &ep = LP.eps[q];
      size_t sz = (size_t)P.tsize[ep.x];
      aoff[q] = bump.take(sz);
      ttoff[q] = bump.take(sz);
      y1off[q] = ep.deg == 3 ? bump.take(sz) : 0;
      wroff[q] = ep.deg == 3 ? bump.take((size_t)4 * c2) : 0;        // WR (2chi x 2chi)
      roff[q] = ep.deg == 3 ? bump.take((size_t)4 * c2) : aoff[q];   // R (r x 2chi)
      rnoff[q] = bump.take((size_t)ep.r * 2 * chi);                  // R' (r x 2 x chi)
    }
    // group absorb ops by (deg, j): descriptor depends on the leg pattern
    std::map<std::pair<int, int>, std::vector<size_t>> groups;
    for (size_t q = 0; q < LP.eps.size(); ++q)
      groups[{LP.eps[q].deg, LP.eps[q].j}].push_back(q);
    LP.absorb.clear();
    LP.remove.clear();
    LP.d2d_in.clear();
    LP.d2d_out.clear();
    for (auto &g : groups) {
      int deg = g.first.first;
      const Endpoint &ep0 = LP.eps[g.second[0]];
      Layout Lt = t_layout(deg, chi), La = a_layout(ep0, chi);
      if (deg == 1) {
        for (size_t q : g.second) {
          const Endpoint &ep = LP.eps[q];
          if (real) {
            LP.d2d_in.emplace_back((double *)W(aoff[q]), (const double *)Tp(ep.x),
                                   (size_t)P.tsize[ep.x] * 16);
            LP.d2d_out.emplace_back((double *)Tp(ep.x), (const double *)W(rnoff[q]),
                                    (size_t)P.tsize[ep.x] * 16);
          }
        }
        continue;
      }
      if (deg == 2) {
        GemmOp op, rm;
        op.d = leg_desc(2, ep0.env[0], Lt, La, chi);
        rm.d = leg_desc(2, ep0.env[0], La, Lt, chi);
        std::vector<const void *> a, b, c, ra, rb, rc;
        for (size_t q : g.second) {
          const Endpoint &ep = LP.eps[q];
          a.push_back(Tp(ep.x)); b.push_back(W(xoff[2 * q])); c.push_back(W(aoff[q]));
          ra.push_back(W(rnoff[q])); rb.push_back(W(xpoff[2 * q])); rc.push_back(Tp(ep.x));
        }
        op.n = rm.n = (int)a.size();
        if (real) {
          op.a = P.arena.add(a); op.b = P.arena.add(b); op.c = P.arena.add(c);
          rm.a = P.arena.add(ra); rm.b = P.arena.add(rb); rm.c = P.arena.add(rc);
        }
        LP.absorb.push_back(op);
        LP.remove.push_back(rm);
        continue;
      }
      // deg 3: T --(env0)--> Y1 (T-order) --(env1)--> A (A-layout); remove mirrors it.
      GemmOp s1, s2, r1, r2;
      s1.d = leg_desc(3, ep0.env[0], Lt, Lt, chi);
      s2.d = leg_desc(3, ep0.env[1], Lt, La, chi);
      r1.d = leg_desc(3, ep0.env[0], Lt, Lt, chi);   // Tt is in T-order
      r2.d = leg_desc(3, ep0.env[1], Lt, Lt, chi);
      std::vector<const void *> a1, b1, c1, a2, b2, c2v, ra1, rb1, rc1, ra2, rb2, rc2;
      for (size_t q : g.second) {
        const Endpoint &ep = LP.eps[q];
        a1.push_back(Tp(ep.x)); b1.push_back(W(xoff[2 * q])); c1.push_back(W(y1off[q]));
        a2.push_back(W(y1off[q])); b2.push_back(W(xoff[2 * q + 1])); c2v.push_back(W(aoff[q]));
        ra1.push_back(W(ttoff[q])); rb1.push_back(W(xpoff[2 * q])); rc1.push_back(W(y1off[q]));
        ra2.push_back(W(y1off[q])); rb2.push_back(W(xpoff[2 * q + 1])); rc2.push_back(Tp(ep.x));
      }
      s1.n = s2.n = r1.n = r2.n = (int)a1.size();
      if (real) {
        s1.a = P.arena.add(a1); s1.b = P.arena.add(b1); s1.c = P.arena.add(c1);
        s2.a = P.arena.add(a2); s2.b = P.arena.add(b2); s2.c = P.arena.add(c2v);
        r1.a = P.arena.add(ra1); r1.b = P.arena.add(rb1); r1.c = P.arena.add(rc1);
        r2.a = P.arena.add(ra2); r2.b = P.arena.add(rb2); r2.c = P.arena.add(rc2);
      }
      LP.absorb.push_back(s1);
      LP.absorb.push_back(s2);
      LP.remove.push_back(r1);
      LP.remove.push_back(r2);
    }
    // 3. Gram factor for degree-3 endpoints
    {
      std::vector<const void *> ga, gc, gev, gvec, gR, gW, wa, wb, wc;
      std::map<int, std::vector<const void *>> ra, rb, rc;          // by bond leg
      for (size_t q = 0; q < LP.eps.size(); ++q) {
        const Endpoint &ep = LP.eps[q];
        if (ep.deg != 3) continue;
        size_t o_G = bump.take(4 * c2), o_ev = bump.take(2 * chi), o_vec = bump.take(4 * c2),
               o_W = bump.take(4 * c2);
        ga.push_back(W(aoff[q])); gc.push_back(W(o_G));
        gev.push_back(W(o_ev)); gvec.push_back(W(o_vec));
        gR.push_back(W(roff[q])); gW.push_back(W(o_W));
        wa.push_back(W(o_W)); wb.push_back(W(rnoff[q])); wc.push_back(W(wroff[q]));
        ra[ep.j].push_back(W(aoff[q])); rb[ep.j].push_back(W(wroff[q]));
        rc[ep.j].push_back(W(ttoff[q]));
      }
      LP.n_g = (int)ga.size();
      GemmDesc g;                       // G = A^H A, A: [env][2chi]
      g.M = 2 * chi; g.Mi = 2 * chi; g.a_mi = 1; g.conjA = 1;
      g.K = (int)c2; g.Ki = (int)c2; g.a_ki = 2 * chi; g.b_ki = 2 * chi;
      g.N = 2 * chi; g.Ni = 2 * chi; g.b_ni = 1;
      g.c_mi = 2 * chi; g.c_ni = 1;
      g.herm = 1;                       // Hermitian: lower triangle, conjugate mirror
      LP.gram.d = g;
      // The isometry Q = A Wsc is never formed: the rebuilt tensor Q R' is taken as A (Wsc R'),
      // a small product first (2chi x 2chi x 2chi) and one environment-sized one instead of two.
      GemmDesc wd;                      // WR = Wsc R' : [2chi][2chi] x [2chi][2chi]
      wd.M = 2 * chi; wd.Mi = 2 * chi; wd.a_mi = 2 * chi; wd.c_mi = 2 * chi;
      wd.K = 2 * chi; wd.Ki = 2 * chi; wd.a_ki = 1; wd.b_ki = 2 * chi;
      wd.N = 2 * chi; wd.Ni = 2 * chi; wd.b_ni = 1; wd.c_ni = 1;
      LP.wr.d = wd;
      // Tt = A WR : [env][2chi] x [2chi][2chi], written straight into T-order (rows (env0, env1),
      // columns (s, a_j)), so that the environment is removed with the loads and stores of the
      // leg contractions running along unit-stride legs
      const Layout Lt3 = t_layout(3, chi);
      LP.rebuild.clear();
      for (auto &jr : ra) {
        const int j = jr.first;
        int env[2], ne = 0;
        for (int i = 0; i < 3; ++i)
          if (i != j) env[ne++] = i;
        GemmOp op;
        GemmDesc rd = wd;
        rd.M = (int)c2; rd.Mi = chi; rd.a_mo = 2L * chi * chi; rd.a_mi = 2 * chi;
        rd.c_mo = Lt3.leg[env[0]]; rd.c_mi = Lt3.leg[env[1]];
        rd.Ni = chi; rd.b_no = chi; rd.b_ni = 1; rd.c_no = Lt3.s; rd.c_ni = Lt3.leg[j];
        op.d = rd;
        op.n = (int)jr.second.size();
        if (real) {
          op.a = P.arena.add(jr.second); op.b = P.arena.add(rb[j]); op.c = P.arena.add(rc[j]);
        }
        LP.rebuild.push_back(op);
      }
      LP.gram.n = LP.wr.n = LP.n_g;
      if (real) {
        LP.gram.a = P.arena.add(ga); LP.gram.b = LP.gram.a; LP.gram.c = P.arena.add(gc);
        LP.g_in = LP.gram.c; LP.g_ev = P.arena.add(gev); LP.g_vec = P.arena.add(gvec);
        LP.g_R = P.arena.add(gR); LP.g_Wsc = P.arena.add(gW);
        LP.wr.a = P.arena.add(wa); LP.wr.b = P.arena.add(wb); LP.wr.c = P.arena.add(wc);
      }
    }
    // 4-6. per edge type
    std::map<std::pair<int, int>, std::vector<size_t>> types;
    for (size_t q = 0; q < LP.edges.size(); ++q) {
      const EdgeWork &w = LP.edges[q];
      types[{LP.eps[w.ep[0]].r, LP.eps[w.ep[1]].r}].push_back(q);
    }
    LP.types.clear();
    LP.eig_groups.clear();
    std::map<int, std::vector<const void *>> g_in, g_ev, g_vec;
    for (auto &t : types) {
      LayerPlan::Type T;
      T.rB = t.first.first;
      T.rS = t.first.second;
      T.n = 2 * T.rS;
      T.count = (int)t.second.size();
      std::vector<const void *> RB, RS, Th, H, ev, vec, Vs, S, mA, mB, RBn, RSn, U;
      std::vector<int> slots;
      for (size_t q : t.second) {
        const EdgeWork &w = LP.edges[q];
        const Endpoint &eb = LP.eps[w.ep[0]], &es = LP.eps[w.ep[1]];
        size_t o_Th = bump.take((size_t)2 * T.rB * T.n), o_H = bump.take((size_t)T.n * T.n),
               o_ev = bump.take(T.n), o_vec = bump.take((size_t)T.n * T.n),
               o_Vs = bump.take((size_t)T.n * chi), o_S = bump.take(chi),
               o_U = bump.take((size_t)2 * T.rB * chi);
        (void)o_H;
        RB.push_back(W(eb.deg == 3 ? roff[w.ep[0]] : aoff[w.ep[0]]));
        RS.push_back(W(es.deg == 3 ? roff[w.ep[1]] : aoff[w.ep[1]]));
        Th.push_back(W(o_Th));
        H.push_back(W(o_H));
        ev.push_back(W(o_ev)); vec.push_back(W(o_vec));
        Vs.push_back(W(o_Vs)); S.push_back(W(o_S)); U.push_back(W(o_U));
        mA.push_back(Mp(2 * w.e)); mB.push_back(Mp(2 * w.e + 1));
        RBn.push_back(W(rnoff[w.ep[0]])); RSn.push_back(W(rnoff[w.ep[1]]));
        slots.push_back((int)q);
        T.hgemm.n = T.ugemm.n = T.count;
        // H buffer pointer list built below (stash in Th list order)
        (void)o_H;
      }
      GemmDesc hd;
      hd.M = T.n; hd.Mi = T.n; hd.a_mi = 1; hd.conjA = 1;
      hd.K = 2 * T.rB; hd.Ki = 2 * T.rB; hd.a_ki = T.n; hd.b_ki = T.n;
      hd.N = T.n; hd.Ni = T.n; hd.b_ni = 1; hd.c_mi = T.n; hd.c_ni = 1;
      hd.herm = 1;                      // Theta^H Theta is Hermitian
      T.hgemm.d = hd;
      GemmDesc ud;                      // U = Theta Vs : [2rB][n] x [n][chi]
      ud.M = 2 * T.rB; ud.Mi = 2 * T.rB; ud.a_mi = T.n; ud.c_mi = chi;
      ud.K = T.n; ud.Ki = T.n; ud.a_ki = 1; ud.b_ki = chi;
      ud.N = chi; ud.Ni = chi; ud.b_ni = 1; ud.c_ni = 1;
      T.ugemm.d = ud;
      // edges of a type are contiguous in `slots` order; k/disc indexed by edge slot, so we
      // require slots to be a contiguous range -> reorder edges by type beforehand (see below)
      T.slot0 = slots.empty() ? 0 : slots[0];
      for (size_t i = 1; i < slots.size(); ++i)
        if (slots[i] != slots[0] + (int)i) throw std::logic_error("edge slots not contiguous");
      if (real) {
        T.RB = P.arena.add(RB); T.RS = P.arena.add(RS); T.Th = P.arena.add(Th);
        T.ev = P.arena.add(ev); T.vec = P.arena.add(vec); T.Vs = P.arena.add(Vs);
        T.S = P.arena.add(S); T.mA = P.arena.add(mA); T.mB = P.arena.add(mB);
        T.RBn = P.arena.add(RBn); T.RSn = P.arena.add(RSn); T.U = P.arena.add(U);
        size_t hoff = P.arena.add(H);
        T.hgemm.a = T.Th; T.hgemm.b = T.Th; T.hgemm.c = hoff;
        T.ugemm.a = T.Th; T.ugemm.b = T.Vs; T.ugemm.c = T.U;
      }
      g_in[T.n].insert(g_in[T.n].end(), H.begin(), H.end());
      g_ev[T.n].insert(g_ev[T.n].end(), ev.begin(), ev.end());
      g_vec[T.n].insert(g_vec[T.n].end(), vec.begin(), vec.end());
      LP.types.push_back(T);
    }
    for (auto &g : g_in) {
      LayerPlan::EighGroup G;
      G.n = g.first;
      G.count = (int)g.second.size();
      if (real) {
        G.in = P.arena.add(g.second);
        G.ev = P.arena.add(g_ev[g.first]);
        G.vec = P.arena.add(g_vec[g.first]);
      }
      LP.eig_groups.push_back(G);
    }
  };

  // order each layer's edges by type so that type groups are contiguous edge slots
  for (auto &LP : P.layers) {
    std::stable_sort(LP.edges.begin(), LP.edges.end(), [&](const EdgeWork &a, const EdgeWork &b) {
      auto ka = std::make_pair(LP.eps[a.ep[0]].r, LP.eps[a.ep[1]].r);
      auto kb = std::make_pair(LP.eps[b.ep[0]].r, LP.eps[b.ep[1]].r);
      return ka < kb;
    });
    for (size_t q = 0; q < LP.edges.size(); ++q) {
      LP.eps[LP.edges[q].ep[0]].edge_slot = (int)q;
      LP.eps[LP.edges[q].ep[1]].edge_slot = (int)q;
    }
  }
  for (auto &LP : P.layers) {
    Bump b;
    layer_build(LP, nullptr, b, false);
    ws_max = std::max(ws_max, b.top);
  }
  // the bond-entropy observable borrows the SU workspace (idle while observing)
  Bump eb;
  std::vector<size_t> e_ev(P.E), e_vec(P.E), e_X(P.E), e_Y(P.E), e_B(P.E);
  for (int e = 0; e < P.E; ++e) {
    e_ev[e] = eb.take(chi);
    e_vec[e] = eb.take(c2);
    e_X[e] = eb.take(c2);
    e_Y[e] = eb.take(c2);
    e_B[e] = eb.take(c2);
  }
  ws_max = std::max(ws_max, eb.top);
  // the Vidal gauge transform also borrows it (from offset 0: never live with the above)
  Bump vb;
  std::vector<size_t> v_ev(2 * P.E), v_vec(2 * P.E), v_X(2 * P.E), v_Xp(2 * P.E), v_C(P.E),
      v_H(P.E), v_ev3(P.E), v_vec3(P.E), v_D1(P.E), v_D2(P.E);
  for (int m = 0; m < 2 * P.E; ++m) {
    v_ev[m] = vb.take(chi);
    v_vec[m] = vb.take(c2);
    v_X[m] = vb.take(c2);
    v_Xp[m] = vb.take(c2);
  }
  for (int e = 0; e < P.E; ++e) {
    v_C[e] = vb.take(c2);
    v_H[e] = vb.take(c2);
    v_ev3[e] = vb.take(chi);
    v_vec3[e] = vb.take(c2);
    v_D1[e] = vb.take(c2);
    v_D2[e] = vb.take(c2);
  }
  ws_max = std::max(ws_max, vb.top);
  P.ws_elems = ws_max;
  P.ws = (double *)A(ws_max * 16);
  for (auto &LP : P.layers) {
    Bump b;
    layer_build(LP, P.ws, b, true);
  }
  if (P.E) {
    auto W = [&](size_t off) { return (const void *)(P.ws + 2 * off); };
    std::vector<const void *> m, mt, ev, vec, X, Y, B;
    for (int e = 0; e < P.E; ++e) {
      m.push_back(Mp(2 * e));
      mt.push_back(Mp(2 * e + 1));
      ev.push_back(W(e_ev[e]));
      vec.push_back(W(e_vec[e]));
      X.push_back(W(e_X[e]));
      Y.push_back(W(e_Y[e]));
      B.push_back(W(e_B[e]));
    }
    P.ent_m = P.arena.add(m); P.ent_ev = P.arena.add(ev); P.ent_vec = P.arena.add(vec);
    P.ent_X = P.arena.add(X); P.ent_Y = P.arena.add(Y); P.ent_B = P.arena.add(B);
    GemmDesc d;
    d.M = d.N = d.K = d.Mi = d.Ni = d.Ki = chi;
    d.a_mi = chi; d.a_ki = 1;
    d.b_ki = 1; d.b_ni = chi;          // B[k][n] = M_{v->u}[n][k]
    d.c_mi = chi; d.c_ni = 1;
    P.ent_xm.d = d;
    P.ent_xm.n = P.E;
    P.ent_xm.a = P.ent_X; P.ent_xm.b = P.arena.add(mt); P.ent_xm.c = P.ent_Y;
    d.b_ki = chi; d.b_ni = 1;
    d.herm = 1;                        // X M^T X with Hermitian X and M
    P.ent_b.d = d;
    P.ent_b.n = P.E;
    P.ent_b.a = P.ent_Y; P.ent_b.b = P.ent_X; P.ent_b.c = P.ent_B;
    P.ent_out = (double *)A((size_t)P.E * 8);

    // Vidal gauge: square roots of every message (index m = 2e: u -> v, 2e + 1: v -> u)
    std::vector<const void *> am, aev, avec, aX, aXp;
    for (int m2 = 0; m2 < 2 * P.E; ++m2) {
      am.push_back(Mp(m2));
      aev.push_back(W(v_ev[m2]));
      avec.push_back(W(v_vec[m2]));
      aX.push_back(W(v_X[m2]));
      aXp.push_back(W(v_Xp[m2]));
    }
    P.vg_m = P.arena.add(am); P.vg_ev = P.arena.add(aev); P.vg_vec = P.arena.add(avec);
    P.vg_X = P.arena.add(aX); P.vg_Xp = P.arena.add(aXp);
    std::vector<const void *> xu, xv, xpu, xpv, cc, hh, ev3, vec3, d1, d2, mu, mv, pu, pv;
    for (int e = 0; e < P.E; ++e) {
      xu.push_back(W(v_X[2 * e]));
      xv.push_back(W(v_X[2 * e + 1]));
      xpu.push_back(W(v_Xp[2 * e]));
      xpv.push_back(W(v_Xp[2 * e + 1]));
      cc.push_back(W(v_C[e]));
      hh.push_back(W(v_H[e]));
      ev3.push_back(W(v_ev3[e]));
      vec3.push_back(W(v_vec3[e]));
      d1.push_back(W(v_D1[e]));
      d2.push_back(W(v_D2[e]));
      mu.push_back(Mp(2 * e));
      mv.push_back(Mp(2 * e + 1));
      pu.push_back(W(v_vec[2 * e]));        // the message eigenvectors are spent by then
      pv.push_back(W(v_vec[2 * e + 1]));
    }
    GemmDesc tn;                            // C[m][n] = sum_k A[k][m] B[k][n]
    tn.M = tn.N = tn.K = tn.Mi = tn.Ni = tn.Ki = chi;
    tn.a_mi = 1; tn.a_ki = chi;
    tn.b_ki = chi; tn.b_ni = 1;
    tn.c_mi = chi; tn.c_ni = 1;
    GemmDesc nn = tn;                       // C = A B
    nn.a_mi = chi; nn.a_ki = 1;
    auto op = [&](const GemmDesc &d, const std::vector<const void *> &a,
                  const std::vector<const void *> &b, const std::vector<const void *> &c) {
      GemmOp o;
      o.d = d;
      o.n = P.E;
      o.a = P.arena.add(a); o.b = P.arena.add(b); o.c = P.arena.add(c);
      return o;
    };
    P.vg_c = op(tn, xu, xv, cc);            // C = X_u^T X_v
    GemmDesc hd = tn;
    hd.conjA = 1;
    hd.herm = 1;
    P.vg_h = op(hd, cc, cc, hh);            // C^H C
    P.vg_ev3 = P.arena.add(ev3); P.vg_vec3 = P.arena.add(vec3);
    P.vg_D1 = P.arena.add(d1); P.vg_D2 = P.arena.add(d2);
    P.vg_Mu = P.arena.add(mu); P.vg_Mv = P.arena.add(mv);
    P.vg_t1 = op(nn, cc, d1, hh);           // C D1 = U S^{1/2} (into the spent C^H C)
    P.vg_pu = op(tn, xpu, hh, pu);          // P_u = X_u^{T+} U S^{1/2}
    P.vg_pv = op(tn, xpv, d2, pv);          // P_v = X_v^{T+} conj(V) S^{1/2}
    P.vg_lam = (double *)A((size_t)P.E * chi * 8);
    P.vg_kept = (int *)A((size_t)P.E * 4);
  }

  // ---- BP plan ----
  {
    size_t top = 0;
    auto take = [&](size_t n) { size_t o = top; top += (n + 31) & ~size_t(31); return o; };
    struct SiteWs { size_t y[5]; };
    std::vector<SiteWs> sws(P.n);
    for (int v = 0; v < P.n; ++v) {
      int nbuf = P.deg[v] == 3 ? 5 : P.deg[v] == 2 ? 2 : 0;
      for (int i = 0; i < nbuf; ++i) sws[v].y[i] = take((size_t)P.tsize[v]);
    }
    // observables need 3 buffers per site (reuse BP slots: deg3 has 5, deg2 has 2, deg1 needs 1)
    std::vector<size_t> obs1(P.n);
    for (int v = 0; v < P.n; ++v)
      if (P.deg[v] == 1) obs1[v] = take((size_t)P.tsize[v]);
    P.bpws_elems = top;
    P.bpws = (double *)A(top * 16);
    auto B = [&](size_t o) { return (const void *)(P.bpws + 2 * o); };
    const bool mixed = prob_.precision == 1;
    if (mixed) {
      P.T32 = (float *)A(tensor_elems() * 8);
      P.bpws32 = (float *)A(top * 8);
    }
    // the FP32 copy of an address in the site tensors or the BP workspace (complex element i is
    // at double offset 2 i there and float offset 2 i here); messages keep their FP64 address
    auto to32 = [&](const void *q) -> const void * {
      const double *x = (const double *)q;
      if (x >= P.T && x < P.T + 2 * tensor_elems()) return (const void *)(P.T32 + (x - P.T));
      if (x >= P.bpws && x < P.bpws + 2 * top) return (const void *)(P.bpws32 + (x - P.bpws));
      return q;
    };
    auto map32 = [&](const std::vector<const void *> &v) {
      std::vector<const void *> r;
      for (const void *q : v) r.push_back(to32(q));
      return r;
    };

    auto add_op1 = [&](std::vector<GemmOp> &ops, const GemmDesc &d,
                       const std::vector<const void *> &a, const std::vector<const void *> &b,
                       const std::vector<const void *> &c) {
      if (a.empty()) return;
      GemmOp op;
      op.d = d;
      op.n = (int)a.size();
      op.a = P.arena.add(a); op.b = P.arena.add(b); op.c = P.arena.add(c);
      ops.push_back(op);
    };
    // A BP contraction in both plans: FP64 storage, and (mixed precision) FP32 storage of the
    // site tensors and intermediates: a leg absorption reads A and writes C in FP32 (B is a
    // message), a closing reads A and B in FP32 and writes the FP64 message
    std::vector<GemmOp> *ops32 = nullptr;
    auto add_op = [&](std::vector<GemmOp> &ops, const GemmDesc &d,
                      const std::vector<const void *> &a, const std::vector<const void *> &b,
                      const std::vector<const void *> &c) {
      add_op1(ops, d, a, b, c);
      if (!ops32 || a.empty()) return;
      GemmDesc d32 = d;
      d32.prec = 1;
      d32.a32 = 1;
      if (d.herm) d32.b32 = 1;
      else d32.c32 = 1;
      add_op1(*ops32, d32, map32(a), map32(b), map32(c));
    };
    // A fused degree-3 closing in both plans (FP32 plan: Y and T from their FP32 copies)
    auto add_fused = [&](std::vector<GemmOp> &ops, const BpCloseDesc &f,
                         const std::vector<const void *> &y, const std::vector<const void *> &t,
                         const std::vector<const void *> &m, const std::vector<const void *> &o) {
      if (y.empty()) return;
      GemmOp op;
      op.fused = 1;
      op.f = f;
      op.n = (int)y.size();
      op.a = P.arena.add(y); op.t = P.arena.add(t); op.b = P.arena.add(m); op.c = P.arena.add(o);
      ops.push_back(op);
      if (!ops32) return;
      GemmOp o32 = op;
      o32.f.prec = 1;
      o32.f.s32 = 1;
      o32.a = P.arena.add(map32(y));
      o32.t = P.arena.add(map32(t));
      ops32->push_back(o32);
    };
    // Sweep schedule: vertex classes (the two sides of a bipartite graph, else a greedy proper
    // vertex colouring).  The messages sent by one class are recomputed together and normalised
    // before the next class; a site reads the message of a neighbour whose class has already
    // been updated in this sweep from the new buffer, otherwise from the current one.
    std::vector<int> cls(P.n, -1);
    bool bip = true;
    for (int s0 = 0; s0 < P.n; ++s0) {
      if (cls[s0] >= 0) continue;
      cls[s0] = 0;
      std::vector<int> queue{s0};
      for (size_t qi = 0; qi < queue.size(); ++qi) {
        int x = queue[qi];
        for (int y : P.nb[x]) {
          if (cls[y] < 0) { cls[y] = 1 - cls[x]; queue.push_back(y); }
          else if (cls[y] == cls[x]) bip = false;
        }
      }
    }
    if (!bip) {
      std::fill(cls.begin(), cls.end(), -1);
      for (int v = 0; v < P.n; ++v) {
        std::set<int> used;
        for (int u : P.nb[v]) if (cls[u] >= 0) used.insert(cls[u]);
        int c = 0;
        while (used.count(c)) ++c;
        cls[v] = c;
      }
    }
    const int ncls = P.n ? *std::max_element(cls.begin(), cls.end()) + 1 : 0;
    std::vector<int> res_src;             // source site of every residual slot
    Layout L3 = t_layout(3, chi), L2 = t_layout(2, chi), L1 = t_layout(1, chi);
    // a closing contraction sum T (prod M) conj(T) with Hermitian messages is Hermitian: only its
    // lower triangle is computed (messages stay exactly Hermitian)
    auto hclose = [&](int deg, int leg, const Layout &L) {
      GemmDesc d = close_desc(deg, leg, L, chi);
      d.herm = 1;
      return d;
    };
    int res_off = 0;
    for (int c = 0; c < ncls; ++c) {
      Plan::BpClass C, C32;
      ops32 = mixed ? &C32.ops : nullptr;
      auto in = [&](int v, int i) { return cls[P.nb[v][i]] < c ? Mnp(P.in_msg[v][i]) : Mp(P.in_msg[v][i]); };
      // A degree-3 message is the closing of two copies of the site tensor, each holding the
      // message of one of its two summed legs (for Hermitian M, sum_{a'} M[x][a'] conj(T[.. a' ..])
      // = conj((T x M)[.. x ..])): three leg absorptions Y_l = T x_l M_l and three Hermitian
      // pair closings per site, 9 chi^4 complex multiply-adds instead of the 13 of absorbing two
      // messages into one copy for every outgoing leg.  At chi = 32 and 64 the closings run in
      // the fused kernel, otherwise on the GEMM.
      if (bp_close_chi(chi)) {
        // Y1 = T x1 M1, Y0 = T x0 M0, Y2 = T x2 M2 (three leg absorptions), then every message is
        // a pair closing of the two copies that hold its summed legs' messages:
        //   out0 = pair(Y1, Y2), out1 = pair(Y0, Y2), out2 = pair(Y0, Y1)
        // with the in-chunk sum along leg 2 (out0, out1) or leg 0 (out2) and the chunks over the
        // remaining leg, so that every chunk's slices run along a unit-stride leg where they can
        std::vector<const void *> a[3], b[3], cc[3], fy[3], ft[3], fm[3], fo[3];
        for (int v = 0; v < P.n; ++v) {
          if (P.deg[v] != 3 || cls[v] != c) continue;
          const auto &y = sws[v].y;
          a[0].push_back(Tp(v)); b[0].push_back(in(v, 1)); cc[0].push_back(B(y[0]));
          a[1].push_back(Tp(v)); b[1].push_back(in(v, 0)); cc[1].push_back(B(y[1]));
          a[2].push_back(Tp(v)); b[2].push_back(in(v, 2)); cc[2].push_back(B(y[2]));
          const void *ys[3] = {B(y[0]), B(y[1]), B(y[1])};
          const void *ts[3] = {B(y[2]), B(y[2]), B(y[0])};
          for (int o = 0; o < 3; ++o) {
            fy[o].push_back(ys[o]);
            ft[o].push_back(ts[o]);
            fm[o].push_back(in(v, o));                 // (not read by a pair)
            fo[o].push_back(Mnp(P.out_msg[v][o]));
          }
        }
        add_op(C.ops, leg_desc(3, 1, L3, L3, chi), a[0], b[0], cc[0]);
        add_op(C.ops, leg_desc(3, 0, L3, L3, chi), a[1], b[1], cc[1]);
        add_op(C.ops, leg_desc(3, 2, L3, L3, chi), a[2], b[2], cc[2]);
        // the three pairs in one launch: problems [36 o, 36 o + 36) take stride set o
        const int qleg[3] = {2, 2, 0}, cleg[3] = {1, 0, 1};
        BpCloseDesc f;
        f.chi = chi;
        f.xdim = chi;
        f.pair = 1;
        f.nsets = 3;
        f.group = (int)fy[0].size();
        f.ss = L3.s;
        std::vector<const void *> ay, at, am, ao;
        for (int o = 0; o < 3; ++o) {
          f.rs[o] = L3.leg[o];
          f.qs[o] = L3.leg[qleg[o]];
          f.cs[o] = L3.leg[cleg[o]];
          ay.insert(ay.end(), fy[o].begin(), fy[o].end());
          at.insert(at.end(), ft[o].begin(), ft[o].end());
          am.insert(am.end(), fm[o].begin(), fm[o].end());
          ao.insert(ao.end(), fo[o].begin(), fo[o].end());
        }
        add_fused(C.ops, f, ay, at, am, ao);
      } else {
        // the same pairs on the GEMM: Y0, Y1, Y2 (three absorptions), then the Hermitian
        // closings out0 = Y1 conj(Y2), out1 = Y0 conj(Y2), out2 = Y0 conj(Y1) over s and the two
        // summed legs (lower triangles)
        std::vector<const void *> a[6], b[6], cc[6];
        for (int v = 0; v < P.n; ++v) {
          if (P.deg[v] != 3 || cls[v] != c) continue;
          const auto &y = sws[v].y;
          auto push = [&](int k, const void *aa, const void *bb, const void *c3) {
            a[k].push_back(aa); b[k].push_back(bb); cc[k].push_back(c3);
          };
          push(0, Tp(v), in(v, 0), B(y[0]));
          push(1, Tp(v), in(v, 1), B(y[1]));
          push(2, Tp(v), in(v, 2), B(y[2]));
          push(3, B(y[1]), B(y[2]), Mnp(P.out_msg[v][0]));
          push(4, B(y[0]), B(y[2]), Mnp(P.out_msg[v][1]));
          push(5, B(y[0]), B(y[1]), Mnp(P.out_msg[v][2]));
        }
        add_op(C.ops, leg_desc(3, 0, L3, L3, chi), a[0], b[0], cc[0]);
        add_op(C.ops, leg_desc(3, 1, L3, L3, chi), a[1], b[1], cc[1]);
        add_op(C.ops, leg_desc(3, 2, L3, L3, chi), a[2], b[2], cc[2]);
        add_op(C.ops, hclose(3, 0, L3), a[3], b[3], cc[3]);
        add_op(C.ops, hclose(3, 1, L3), a[4], b[4], cc[4]);
        add_op(C.ops, hclose(3, 2, L3), a[5], b[5], cc[5]);
      }
      if (bp_close_chi(chi)) {
        // degree 2 at chi = 32 or 64, fused: out_o = close(T, apply the other leg's message), the chunks
        // being the two values of s (no chunk leg); both legs of every site in one launch
        std::vector<const void *> ft, fm, fo;
        BpCloseDesc f;
        f.chi = chi;
        f.nsets = 2;
        f.xdim = 1;
        f.ss = L2.s;
        for (int o = 0; o < 2; ++o) {
          f.rs[o] = L2.leg[o];
          f.qs[o] = L2.leg[1 - o];
          f.cs[o] = 0;
          for (int v = 0; v < P.n; ++v) {
            if (P.deg[v] != 2 || cls[v] != c) continue;
            ft.push_back(Tp(v));
            fm.push_back(in(v, 1 - o));
            fo.push_back(Mnp(P.out_msg[v][o]));
          }
        }
        f.group = (int)ft.size() / 2;
        add_fused(C.ops, f, ft, ft, fm, fo);
      } else {
        std::vector<const void *> a[4], b[4], cc[4];
        for (int v = 0; v < P.n; ++v) {
          if (P.deg[v] != 2 || cls[v] != c) continue;
          const auto &y = sws[v].y;
          a[0].push_back(Tp(v)); b[0].push_back(in(v, 1)); cc[0].push_back(B(y[0]));
          a[1].push_back(Tp(v)); b[1].push_back(in(v, 0)); cc[1].push_back(B(y[1]));
          a[2].push_back(B(y[0])); b[2].push_back(Tp(v)); cc[2].push_back(Mnp(P.out_msg[v][0]));
          a[3].push_back(B(y[1])); b[3].push_back(Tp(v)); cc[3].push_back(Mnp(P.out_msg[v][1]));
        }
        add_op(C.ops, leg_desc(2, 1, L2, L2, chi), a[0], b[0], cc[0]);
        add_op(C.ops, leg_desc(2, 0, L2, L2, chi), a[1], b[1], cc[1]);
        add_op(C.ops, hclose(2, 0, L2), a[2], b[2], cc[2]);
        add_op(C.ops, hclose(2, 1, L2), a[3], b[3], cc[3]);
      }
      {
        std::vector<const void *> a, b, cc;
        for (int v = 0; v < P.n; ++v) {
          if (P.deg[v] != 1 || cls[v] != c) continue;
          a.push_back(Tp(v)); b.push_back(Tp(v)); cc.push_back(Mnp(P.out_msg[v][0]));
        }
        add_op(C.ops, hclose(1, 0, L1), a, b, cc);
      }
      std::vector<const void *> nn, no;
      for (int v = 0; v < P.n; ++v) {
        if (cls[v] != c) continue;
        for (int i = 0; i < P.deg[v]; ++i) {
          nn.push_back(Mnp(P.out_msg[v][i]));
          no.push_back(Mp(P.out_msg[v][i]));
          res_src.push_back(v);
        }
      }
      C.nmsg = (int)nn.size();
      C.res_off = res_off;
      res_off += C.nmsg;
      if (C.nmsg) {
        C.norm_new = P.arena.add(nn);
        C.norm_old = P.arena.add(no);
      }
      P.bp_classes.push_back(C);
      if (mixed) {
        C32.nmsg = C.nmsg;
        C32.res_off = C.res_off;
        C32.norm_new = C.norm_new;
        C32.norm_old = C.norm_old;
        P.bp_classes32.push_back(C32);
      }
    }
    ops32 = nullptr;
    if (P.nmem > 1) {
      std::vector<std::vector<int>> by(P.nmem);
      for (size_t r = 0; r < res_src.size(); ++r) by[P.site_member[res_src[r]]].push_back((int)r);
      std::vector<int> off(1, 0), idx;
      for (auto &b : by) {
        idx.insert(idx.end(), b.begin(), b.end());
        off.push_back((int)idx.size());
      }
      std::vector<int> mm(2 * P.E, 0);
      for (int v = 0; v < P.n; ++v)
        for (int m : P.out_msg[v]) mm[m] = P.site_member[v];
      P.mem_off = (int *)A(off.size() * 4);
      P.mem_idx = (int *)A(std::max<size_t>(1, idx.size()) * 4);
      P.msg_member = (int *)A(std::max<size_t>(1, mm.size()) * 4);
      P.act[0] = (int *)A((size_t)P.nmem * 4);
      P.act[1] = (int *)A((size_t)P.nmem * 4);
      P.res_m = (double *)A((size_t)P.nmem * 8);
      be_->h2d(P.mem_off, off.data(), off.size() * 4);
      if (!idx.empty()) be_->h2d(P.mem_idx, idx.data(), idx.size() * 4);
      if (!mm.empty()) be_->h2d(P.msg_member, mm.data(), mm.size() * 4);
    }
    // observables: Y = T x0 M0 x1 M1 x2 M2 (T-order), rho = sum Y conj(T)
    {
      std::vector<const void *> a[3][3], b[3][3], c[3][3];   // [deg-1][step]
      std::vector<const void *> ry, rt;
      std::vector<int64_t> lens;
      for (int v = 0; v < P.n; ++v) {
        int d = P.deg[v];
        const void *cur = Tp(v);
        for (int l = 0; l < d; ++l) {
          const void *dst = d == 1 ? B(obs1[v]) : B(sws[v].y[l]);
          a[d - 1][l].push_back(cur); b[d - 1][l].push_back(Mp(P.in_msg[v][l]));
          c[d - 1][l].push_back(dst);
          cur = dst;
        }
        ry.push_back(cur);
        rt.push_back(Tp(v));
        lens.push_back(P.tsize[v] / 2);
      }
      for (int d = 1; d <= 3; ++d) {
        Layout L = t_layout(d, chi);
        for (int l = 0; l < d; ++l) add_op(P.obs_ops, leg_desc(d, l, L, L, chi), a[d - 1][l],
                                           b[d - 1][l], c[d - 1][l]);
      }
      P.obs_Y = P.arena.add(ry);
      P.obs_T = P.arena.add(rt);
      // Vidal gauge factors on every leg: T x0 P0 x1 P1 x2 P2, the last product written back
      // into T (degree 1: through a buffer and a copy)
      if (P.E) {
        auto Wv = [&](size_t off) { return (const void *)(P.ws + 2 * off); };
        std::vector<const void *> va[3][3], vb2[3][3], vc[3][3];
        for (int v = 0; v < P.n; ++v) {
          const int d = P.deg[v];
          const void *cur = Tp(v);
          for (int l = 0; l < d; ++l) {
            const int m = P.in_msg[v][l], e = m / 2;
            // m odd: the message comes from edges[2e+1], so v = edges[2e] holds P_u
            const void *f = Wv(v_vec[(m & 1) ? 2 * e : 2 * e + 1]);
            const void *dst = l == d - 1 && d > 1 ? Tp(v) : d == 1 ? B(obs1[v]) : B(sws[v].y[l]);
            va[d - 1][l].push_back(cur); vb2[d - 1][l].push_back(f); vc[d - 1][l].push_back(dst);
            cur = dst;
          }
          if (d == 1) {
            P.vg_copy.push_back({P.T + 2 * P.toff[v], (const double *)B(obs1[v])});
            P.vg_copy_len.push_back((size_t)P.tsize[v] * 16);   // complex entries
          }
        }
        for (int d = 1; d <= 3; ++d) {
          Layout L = t_layout(d, chi);
          for (int l = 0; l < d; ++l) add_op(P.vg_ops, leg_desc(d, l, L, L, chi), va[d - 1][l],
                                             vb2[d - 1][l], vc[d - 1][l]);
        }
      }
      P.rho_len = (int64_t *)A(lens.size() * 8);
      be_->h2d(P.rho_len, lens.data(), lens.size() * 8);
    }
    // RX
    {
      std::vector<const void *> t;
      std::vector<int64_t> half;
      for (int v = 0; v < P.n; ++v) { t.push_back(Tp(v)); half.push_back(P.tsize[v] / 2); }
      P.rx_ptrs = P.arena.add(t);
      P.rx_half = (int64_t *)A(half.size() * 8);
      be_->h2d(P.rx_half, half.data(), half.size() * 8);
    }
  }
  // upload pointer arena
  P.arena.dev = (void **)be_->alloc(std::max<size_t>(1, P.arena.host.size()) * sizeof(void *));
  be_->h2d(P.arena.dev, P.arena.host.data(), P.arena.host.size() * sizeof(void *));
  reset();
}

void Engine::reset() {
  t32_stale_ = true;
  Plan &P = *plan_;
  const long c2 = (long)P.chi * P.chi;
  std::vector<double> t(2 * tensor_elems(), 0.0);
  for (int v = 0; v < P.n; ++v) t[2 * P.toff[v]] = 1.0;
  be_->h2d(P.T, t.data(), t.size() * 8);
  std::vector<double> m(2 * message_elems(), 0.0);
  for (int k = 0; k < 2 * P.E; ++k) m[2 * (size_t)k * c2] = 1.0;
  be_->h2d(P.M, m.data(), m.size() * 8);
  std::fill(P.bond_h.begin(), P.bond_h.end(), 1);
}

static void run(Backend *be, const PtrArena &ar, const GemmOp &op, int prec) {
  if (op.n == 0) return;
  if (op.fused) {
    BpCloseDesc f = op.f;
    f.prec = prec;
    be->bp_close(f, ar.at<const double *const *>(op.a), ar.at<const double *const *>(op.t),
                 ar.at<const double *const *>(op.b), ar.at<double *const *>(op.c), op.n);
    return;
  }
  GemmDesc d = op.d;
  d.prec = prec;
  be->gemm(d, ar.at<const double *const *>(op.a), ar.at<const double *const *>(op.b),
           ar.at<double *const *>(op.c), op.n);
}

void Engine::apply_rx() {
  t32_stale_ = true;
  Plan &P = *plan_;
  if (prob_.site_theta.empty()) {
    double c = std::cos(prob_.theta / 2), s = std::sin(prob_.theta / 2);
    be_->rx(P.arena.at<double *const *>(P.rx_ptrs), P.rx_half, P.n, c, s);
    return;
  }
  // one launch per run of sites with the same angle
  for (int v0 = 0; v0 < P.n;) {
    int v1 = v0 + 1;
    const double th = prob_.site_theta[v0];
    while (v1 < P.n && prob_.site_theta[v1] == th) ++v1;
    be_->rx(P.arena.at<double *const *>(P.rx_ptrs) + v0, P.rx_half + v0, v1 - v0,
            std::cos(th / 2), std::sin(th / 2));
    v0 = v1;
  }
}

void Engine::apply_rx_angle(double theta) {
  t32_stale_ = true;
  Plan &P = *plan_;
  be_->rx(P.arena.at<double *const *>(P.rx_ptrs), P.rx_half, P.n, std::cos(theta / 2),
          std::sin(theta / 2));
}

double Engine::apply_layer(int colour, int zz_sign) {
  t32_stale_ = true;
  Plan &P = *plan_;
  auto it = std::find(P.layer_colours.begin(), P.layer_colours.end(), colour);
  if (it == P.layer_colours.end()) return 0.0;
  LayerPlan &LP = P.layers[it - P.layer_colours.begin()];
  const PtrArena &ar = P.arena;
  const int chi = P.chi;
  // 1. X, X+ of the environment messages
  if (LP.n_msg) {
    be_->eigh(chi, chi, ar.at<const double *const *>(LP.m_in), ar.at<double *const *>(LP.m_ev),
              ar.at<double *const *>(LP.m_vec), LP.n_msg, chi);
    be_->msg_sqrt(chi, ar.at<const double *const *>(LP.m_ev),
                  ar.at<const double *const *>(LP.m_vec), ar.at<double *const *>(LP.m_X),
                  ar.at<double *const *>(LP.m_Xp), prob_.eig_cutoff, LP.n_msg);
  }
  // 2. absorb
  for (auto &t : LP.d2d_in) be_->d2d(std::get<0>(t), std::get<1>(t), std::get<2>(t));
  for (auto &op : LP.absorb) run(be_, ar, op, su_prec());
  // 3. isolate degree-3 endpoints
  if (LP.n_g) {
    run(be_, ar, LP.gram, su_prec());
    be_->gram_chol(2 * chi, ar.at<const double *const *>(LP.g_in), ar.at<double *const *>(LP.g_R),
                   ar.at<double *const *>(LP.g_Wsc), kGramCut, LP.n_g);
  }
  // 4-6. Theta, truncated SVD, new factors
  const double q = M_PI / 4;
  for (auto &T : LP.types) {
    be_->theta(T.rB, T.rS, chi, ar.at<const double *const *>(T.RB),
               ar.at<const double *const *>(T.RS), ar.at<double *const *>(T.Th), std::cos(q),
               zz_sign * std::sin(q), std::cos(q), -zz_sign * std::sin(q), T.count);
    run(be_, ar, T.hgemm, 0);        // the truncation SVD is FP64 in every mode
  }
  for (auto &G : LP.eig_groups)
    be_->eigh(G.n, G.n, ar.at<const double *const *>(G.in), ar.at<double *const *>(G.ev),
              ar.at<double *const *>(G.vec), G.count, std::min(G.n, chi));   // kept columns only
  for (auto &T : LP.types) {
    be_->svd_finish(T.n, chi, ar.at<const double *const *>(T.ev),
                    ar.at<const double *const *>(T.vec), ar.at<double *const *>(T.Vs),
                    ar.at<double *const *>(T.S), P.kbuf + T.slot0, P.disc + 2 * T.slot0,
                    ar.at<double *const *>(T.mA), ar.at<double *const *>(T.mB), prob_.svd_cutoff,
                    T.count);
    run(be_, ar, T.ugemm, 0);
    be_->split_sqrt(2 * T.rB, 2 * T.rS, T.n, chi, ar.at<const double *const *>(T.U),
                    ar.at<const double *const *>(T.vec), ar.at<const double *const *>(T.S),
                    ar.at<double *const *>(T.RBn), ar.at<double *const *>(T.RSn), T.count);
  }
  // 7. rebuild and remove the environment
  if (LP.n_g) {
    run(be_, ar, LP.wr, su_prec());
    for (auto &op : LP.rebuild) run(be_, ar, op, su_prec());
  }
  // degree <= 2: T~' = R' (already in A-layout); point remove ops at R' directly
  for (auto &op : LP.remove) run(be_, ar, op, su_prec());
  for (auto &t : LP.d2d_out) be_->d2d(std::get<0>(t), std::get<1>(t), std::get<2>(t));
  // bookkeeping: discarded weight, cut gap and bond dimension of every edge of the layer
  int ne = (int)LP.edges.size();
  std::vector<double> disc(2 * (size_t)ne);
  std::vector<int> k(ne);
  be_->d2h(disc.data(), P.disc, (size_t)ne * 16);
  be_->d2h(k.data(), P.kbuf, ne * 4);
  double dsum = 0;
  layer_cuts_.resize(ne);
  for (int i = 0; i < ne; ++i) {
    dsum += disc[2 * i];
    P.bond_h[LP.edges[i].e] = k[i];
    layer_cuts_[i] = {LP.edges[i].e, k[i], disc[2 * i], disc[2 * i + 1]};
  }
  return dsum;
}

void Engine::sweep_classes() {
  Plan &P = *plan_;
  const bool f32 = bp_prec_ == 1 && !P.bp_classes32.empty();
  if (f32 && t32_stale_) {          // the FP32 copy of the site tensors, once per new state
    be_->to_f32(P.T, P.T32, tensor_elems());
    t32_stale_ = false;
  }
  for (auto &C : f32 ? P.bp_classes32 : P.bp_classes) {
    for (auto &op : C.ops) run(be_, P.arena, op, f32 ? 1 : bp_prec_);
    if (C.nmsg)
      be_->normalize_residual(P.chi, P.arena.at<double *const *>(C.norm_new),
                              P.arena.at<const double *const *>(C.norm_old), P.res + C.res_off,
                              C.nmsg);
  }
}

double Engine::bp_sweep() {
  Plan &P = *plan_;
  sweep_classes();
  be_->reduce_max(P.res, 2 * P.E, P.resmax);
  be_->d2d(P.M, P.Mn, message_elems() * 16);
  double r = 0;
  be_->d2h(&r, P.resmax, 8);
  return r;
}

int Engine::bp(int max_iter, double *residual) {
  // Mixed modes sweep with FP32 contractions while the residual is above the FP32 floor, then
  // (if the tolerance asks for more) finish with FP64 sweeps: the fixed point is the FP64 one.
  // While the residual is predicted to stay well above the tolerance, the next sweep's launches
  // are enqueued before this sweep's residual has come back to the host; its message copy (the
  // commit) is enqueued only once that residual says it is needed, so a sweep that is not needed
  // is never committed and the messages are those of one sweep at a time.
  Plan &P = *plan_;
  const size_t mbytes = message_elems() * 16;
  auto launch = [&](int slot) {
    sweep_classes();
    be_->reduce_max(P.res, 2 * P.E, P.resmax + slot);
    be_->read_async(P.resmax + slot, slot);
  };
  auto commit = [&]() { be_->d2d(P.M, P.Mn, mbytes); };
  double r = INFINITY, prev = INFINITY, prev2 = INFINITY;
  bp_prec_ = prob_.precision ? 1 : 0;
  int it = 0, slot = 0;
  if (max_iter > 0) {
    launch(slot);
    commit();
  }
  while (it < max_iter) {
    ++it;                                // sweep `it` is committed; its residual is in `slot`
    // speculate only with two residuals to extrapolate from, predicted well above the point
    // where the loop stops or changes arithmetic
    bool spec = false;
    if (it < max_iter && std::isfinite(prev2) && prev2 > 0.0) {
      const double pred = prev * std::min(1.0, prev / prev2);
      const double stop = bp_prec_ == 1 ? kFp32Near * kFp32BpFloor : prob_.bp_tol;
      spec = pred > kSpecMargin * stop;
    }
    const int pprec = bp_prec_;
    if (spec) launch(slot ^ 1);
    r = be_->wait_read(slot);
    if (r < prob_.bp_tol || it >= max_iter) break;    // a speculated sweep stays uncommitted
    if (bp_prec_ == 1 && fp32_done(r, prev)) bp_prec_ = 0;
    prev2 = prev;
    prev = r;
    slot ^= 1;
    if (!spec || bp_prec_ != pprec) launch(slot);     // (re)launch in the current arithmetic
    commit();
  }
  bp_prec_ = prob_.precision ? 1 : 0;
  if (residual) *residual = r;
  return it;
}

int Engine::n_members() const { return plan_->nmem; }

void Engine::bp_members(int max_iter, int *sweeps, double *residual) {
  Plan &P = *plan_;
  const int R = P.nmem;
  std::vector<int> act(R, 1);
  std::vector<double> r(R, INFINITY);
  for (int j = 0; j < R; ++j) {
    sweeps[j] = 0;
    residual[j] = INFINITY;
  }
  be_->h2d(P.act[0], act.data(), (size_t)R * 4);
  int cur = 0;
  double prev = INFINITY;
  bp_prec_ = prob_.precision ? 1 : 0;
  for (int it = 1; it <= max_iter; ++it) {
    sweep_classes();
    be_->member_residual(P.res, P.mem_off, P.mem_idx, R, P.act[cur], P.act[cur ^ 1],
                         prob_.bp_tol, P.res_m);
    be_->commit_messages(P.M, P.Mn, (long)P.chi * P.chi, 2 * P.E, P.msg_member, P.act[cur]);
    be_->d2h(r.data(), P.res_m, (size_t)R * 8);
    cur ^= 1;
    bool any = false;
    double rmax = 0.0;
    for (int j = 0; j < R; ++j) {
      if (!act[j]) continue;
      sweeps[j] = it;
      residual[j] = r[j];
      if (r[j] < prob_.bp_tol) act[j] = 0;
      else any = true;
      rmax = std::max(rmax, r[j]);
    }
    if (!any) break;
    if (bp_prec_ == 1 && fp32_done(rmax, prev)) bp_prec_ = 0;
    prev = rmax;
  }
  bp_prec_ = prob_.precision ? 1 : 0;
}

void Engine::observe_pauli_range(int k0, int k1, double *out) {
  for (int k = k0; k < k1; ++k) {
    double a = pauli_value(k, true);
    double b = pauli_value(k, false);
    out[k - k0] = a / b;
  }
}

void Engine::observe_z(double *z) {
  Plan &P = *plan_;
  for (auto &op : P.obs_ops) run(be_, P.arena, op, prob_.precision ? 1 : 0);
  be_->rho_dot(P.arena.at<const double *const *>(P.obs_Y),
               P.arena.at<const double *const *>(P.obs_T), P.rho_len, P.rho, P.n);
  std::vector<double> rho((size_t)P.n * 8);
  be_->d2h(rho.data(), P.rho, rho.size() * 8);
  for (int v = 0; v < P.n; ++v) {
    const double *r = &rho[(size_t)v * 8];   // rho00, rho01, rho10, rho11 (complex)
    double nr = r[0] - r[6], ni = r[1] - r[7];
    double dr = r[0] + r[6], di = r[1] + r[7];
    double den = dr * dr + di * di;
    z[v] = (nr * dr + ni * di) / den;
  }
}

// Bond entanglement entropy of every edge (Eq. "EntanglementEntropy"): with the BP norm across
// the edge equal to Tr(M_{u->v} M_{v->u}^T), the Schmidt weights are the eigenvalues of the
// Hermitian X M_{v->u}^T X, X = M_{u->v}^{1/2}, normalised to unit sum.  FP64 in every mode.
void Engine::observe_entropy(double *out) {
  Plan &P = *plan_;
  if (!P.E) return;
  const PtrArena &ar = P.arena;
  const int chi = P.chi;
  be_->eigh(chi, chi, ar.at<const double *const *>(P.ent_m), ar.at<double *const *>(P.ent_ev),
            ar.at<double *const *>(P.ent_vec), P.E, chi);
  // the pseudo-inverse root lands in the Y buffer and is overwritten by the product below
  be_->msg_sqrt(chi, ar.at<const double *const *>(P.ent_ev), ar.at<const double *const *>(P.ent_vec),
                ar.at<double *const *>(P.ent_X), ar.at<double *const *>(P.ent_Y),
                prob_.eig_cutoff, P.E);
  run(be_, ar, P.ent_xm, 0);
  run(be_, ar, P.ent_b, 0);
  be_->eigh(chi, chi, ar.at<const double *const *>(P.ent_B), ar.at<double *const *>(P.ent_ev),
            ar.at<double *const *>(P.ent_vec), P.E, 1);   // eigenvalues only
  be_->bond_entropy(chi, ar.at<const double *const *>(P.ent_ev), P.ent_out, P.E);
  be_->d2h(out, P.ent_out, (size_t)P.E * 8);
}

// Explicit symmetric Vidal gauge from the BP messages (Methods, "The Vidal gauge"): for every
// edge (u, v), X_u = M_{u->v}^{1/2}, X_v = M_{v->u}^{1/2}, C = X_u^T X_v = U S V^H; leg u->v of T_u
// absorbs P_u = X_u^{T+} U S^{1/2} and leg v->u of T_v absorbs P_v = X_v^{T+} conj(V) S^{1/2},
// which inserts the identity (on the supports) on the bond and makes every grouping of a site
// tensor with the bond weights of its other legs an isometry.  S is normalised to unit 2-norm,
// values <= svd_cutoff * s_1 are dropped, and the messages become the fixed point diag(S)/sum S.
void Engine::vidal_gauge(double *lambda) {
  t32_stale_ = true;
  Plan &P = *plan_;
  if (!P.E) return;
  const PtrArena &ar = P.arena;
  const int chi = P.chi;
  be_->eigh(chi, chi, ar.at<const double *const *>(P.vg_m), ar.at<double *const *>(P.vg_ev),
            ar.at<double *const *>(P.vg_vec), 2 * P.E, chi);
  be_->msg_sqrt(chi, ar.at<const double *const *>(P.vg_ev), ar.at<const double *const *>(P.vg_vec),
                ar.at<double *const *>(P.vg_X), ar.at<double *const *>(P.vg_Xp),
                prob_.eig_cutoff, 2 * P.E);
  run(be_, ar, P.vg_c, 0);
  run(be_, ar, P.vg_h, 0);
  be_->eigh(chi, chi, ar.at<const double *const *>(P.vg_h.c), ar.at<double *const *>(P.vg_ev3),
            ar.at<double *const *>(P.vg_vec3), P.E, chi);
  be_->vidal_svd(chi, ar.at<const double *const *>(P.vg_ev3),
                 ar.at<const double *const *>(P.vg_vec3), ar.at<double *const *>(P.vg_D1),
                 ar.at<double *const *>(P.vg_D2), ar.at<double *const *>(P.vg_Mu),
                 ar.at<double *const *>(P.vg_Mv), P.vg_lam, P.vg_kept, prob_.svd_cutoff, P.E);
  run(be_, ar, P.vg_t1, 0);
  run(be_, ar, P.vg_pu, 0);
  run(be_, ar, P.vg_pv, 0);
  for (auto &o : P.vg_ops) run(be_, ar, o, 0);
  for (size_t i = 0; i < P.vg_copy.size(); ++i)
    be_->d2d(P.vg_copy[i].first, P.vg_copy[i].second, P.vg_copy_len[i]);
  std::vector<int> k(P.E);
  be_->d2h(k.data(), P.vg_kept, (size_t)P.E * 4);
  for (int e = 0; e < P.E; ++e) P.bond_h[e] = std::min(P.bond_h[e], k[e]);
  if (lambda) be_->d2h(lambda, P.vg_lam, (size_t)P.E * chi * 8);
}

// C = A B for chi^2 x chi^2 matrices (row-major).
static GemmDesc square_desc(long n) {
  GemmDesc c;
  c.M = c.N = c.K = c.Mi = c.Ni = c.Ki = (int)n;
  c.a_mi = n; c.a_ki = 1;
  c.b_ki = n; c.b_ni = 1;
  c.c_mi = n; c.c_ni = 1;
  return c;
}

// Device buffers of one host-driven contraction (a Pauli string, a BP error estimate): allocated
// for the call, released (after the stream drains) at its end.  Single-problem launches take
// their pointer triple through one small device array, rewritten in stream order.
struct EngineScratch {
  Backend *be;
  int prec;                       // GemmDesc::prec of every contraction
  std::vector<void *> bufs;
  void **parr = nullptr;
  EngineScratch(Backend *b, int precision) : be(b), prec(precision) {
    parr = (void **)be->alloc(3 * sizeof(void *));
    bufs.push_back(parr);
  }
  ~EngineScratch() {
    be->sync();
    for (void *q : bufs) be->release(q);
  }
  double *alloc(size_t elems) {
    void *q = be->alloc(elems * 16);
    bufs.push_back(q);
    return (double *)q;
  }
  // a device array holding the given pointers
  void **ptrs(const std::vector<const void *> &v) {
    void **q = (void **)be->alloc(std::max<size_t>(1, v.size()) * sizeof(void *));
    bufs.push_back(q);
    be->h2d(q, v.data(), v.size() * sizeof(void *));
    return q;
  }
  void gemm(GemmDesc d, const std::vector<const void *> &a, const std::vector<const void *> &b,
            const std::vector<const void *> &c) {
    d.prec = prec;
    void **pa = ptrs(a), **pb = ptrs(b), **pc = ptrs(c);
    be->gemm(d, (const double *const *)pa, (const double *const *)pb, (double *const *)pc,
             (int)a.size());
  }
  void gemm1(GemmDesc d, const double *a, const double *b, double *c) {
    d.prec = prec;
    const void *h[3] = {a, b, c};
    be->h2d(parr, h, sizeof(h));
    be->gemm(d, (const double *const *)parr, (const double *const *)(parr + 1),
             (double *const *)(parr + 2), 1);
  }
};

// BP error estimate (Eq. "BPErrorEstimate") on edge e = (u, v), in the symmetric gauge
// (vidal_gauge first): the norm network with the edge cut and every other bond contracted exactly
// is the chi^2 x chi^2 edge environment E; with s_i its singular values the estimate is
// 1 - sqrt(s_1^2 / sum s_i^2).  The singular values come from eigh(E^H E).
// * e a bridge: E is an outer product, the estimate 0 and the spectrum (1, 0, ...).
// * The 2-core of the network (what is left after removing sites of degree 1 repeatedly) one
//   loop: the branches fold into the transfer matrices of the loop sites, and E is the open chain
//   F_v ... F_u walking from v around the loop to u.
// * The 2-core two junction sites a, b joined by three paths (two heavy hexagons sharing a side),
//   the cut on one of them: Q_u is the chain from a to u on that path, Q_v the chain from v to b,
//   M_1 and M_2 the chains along the other two paths from a to b.  G_a(x) is a's transfer matrix
//   between its legs to M_1 and M_2 with its third leg closed with column x of Q_u, G_b(y) the same
//   at b with row y of Q_v, and E[x][y] = sum_jk (M_1^T G_a(x) M_2)[j][k] G_b(y)[j][k].
// Other networks return -1.  Each transfer matrix is divided by ||T||^2 (positive factors leave
// the estimate unchanged).
double Engine::bp_error(int e, double *spectrum) {
  Plan &P = *plan_;
  vidal_gauge(nullptr);
  const int chi = P.chi, n = P.n;
  const long c2 = (long)chi * chi;
  const long c4 = c2 * c2;
  const int u = prob_.edges[2 * e], v = prob_.edges[2 * e + 1];
  auto unit = [&]() {
    if (spectrum)
      for (long i = 0; i < c2; ++i) spectrum[i] = i == 0 ? 1.0 : 0.0;
    return 0.0;
  };
  // a bridge: v is not reached from u without the edge
  {
    std::vector<char> seen(n, 0);
    std::vector<int> st{u};
    seen[u] = 1;
    while (!st.empty()) {
      const int w = st.back();
      st.pop_back();
      for (int x : P.nb[w])
        if (!seen[x] && !((w == u && x == v) || (w == v && x == u))) {
          seen[x] = 1;
          st.push_back(x);
        }
    }
    if (!seen[v]) return unit();
  }
  // the 2-core and its junctions
  std::vector<int> cdeg(n);
  for (int w = 0; w < n; ++w) cdeg[w] = P.deg[w];
  std::vector<char> core(n, 1);
  {
    std::vector<int> leaves;
    for (int w = 0; w < n; ++w)
      if (cdeg[w] <= 1) leaves.push_back(w);
    while (!leaves.empty()) {
      const int w = leaves.back();
      leaves.pop_back();
      if (!core[w]) continue;
      core[w] = 0;
      for (int x : P.nb[w])
        if (core[x] && --cdeg[x] == 1) leaves.push_back(x);
    }
  }
  std::vector<int> junctions;
  int ncore = 0;
  for (int w = 0; w < n; ++w) {
    if (!core[w]) continue;
    ++ncore;
    if (cdeg[w] == 3) junctions.push_back(w);
    else if (cdeg[w] != 2) return -1.0;
  }
  // walk along core sites of core degree 2 from `from` through `first` to the next junction (or
  // back to `from`): the interior sites and the end
  auto walk_path = [&](int from, int first, std::vector<int> *inner) {
    int prev = from, w = first;
    while (cdeg[w] == 2 && w != from) {
      inner->push_back(w);
      int nx = -1;
      for (int x : P.nb[w])
        if (core[x] && x != prev) nx = x;
      prev = w;
      w = nx;
    }
    return w;
  };
  EngineScratch S(be_, 0);
  double *E = nullptr;
  if (junctions.empty()) {
    // one loop (the 2-core is connected: the network is, or the edge would have been a bridge
    // inside a tree component)
    std::vector<int> loop;
    const int end = walk_path(u, v, &loop);
    if (end != u || (int)loop.size() + 1 != ncore) return -1.0;
    loop.push_back(u);
    E = chain(loop, u, v, S);                   // F_v ... F_u
  } else if (junctions.size() == 2) {
    const int a = junctions[0], b = junctions[1];
    std::vector<std::vector<int>> paths;
    int covered = 2;
    for (int x : P.nb[a]) {
      if (!core[x]) continue;
      std::vector<int> inner;
      if (walk_path(a, x, &inner) != b) return -1.0;
      covered += (int)inner.size();
      paths.push_back(inner);
    }
    if (paths.size() != 3 || covered != ncore) return -1.0;
    // the path of the cut, as a = s_0, s_1, ..., s_L = b, cut between s_t and s_{t+1}
    int pc = -1, t = -1;
    for (int k = 0; k < 3 && pc < 0; ++k) {
      std::vector<int> s{a};
      s.insert(s.end(), paths[k].begin(), paths[k].end());
      s.push_back(b);
      for (int i = 0; i + 1 < (int)s.size(); ++i)
        if ((s[i] == u && s[i + 1] == v) || (s[i] == v && s[i + 1] == u)) {
          pc = k;
          t = i;
        }
    }
    if (pc < 0) return -1.0;
    std::vector<int> sp{a};
    sp.insert(sp.end(), paths[pc].begin(), paths[pc].end());
    sp.push_back(b);
    const int L = (int)sp.size() - 1;
    std::vector<int> wu(sp.begin() + 1, sp.begin() + t + 1);        // s_1 .. s_t
    std::vector<int> wv(sp.begin() + t + 1, sp.begin() + L);        // s_{t+1} .. s_{L-1}
    double *Qu = chain(wu, a, sp[t + 1], S);     // rows: a's cut-path leg, cols: cut (s_t side)
    double *Qv = chain(wv, sp[t], b, S);         // rows: cut (s_{t+1} side), cols: b's leg
    const std::vector<int> &p1 = paths[(pc + 1) % 3], &p2 = paths[(pc + 2) % 3];
    double *M1 = chain(p1, a, b, S), *M2 = chain(p2, a, b, S);
    const int a1 = p1.empty() ? b : p1.front(), a2 = p2.empty() ? b : p2.front();
    const int b1 = p1.empty() ? a : p1.back(), b2 = p2.empty() ? a : p2.back();
    std::set<int> all;
    for (int w = 0; w < n; ++w) all.insert(w);
    const std::map<int, int> none;
    double *Ga = S.alloc((size_t)c2 * c4), *Gb = S.alloc((size_t)c2 * c4);
    const OpenLeg xu{Qu, 1, c2 * chi, c2};       // X_x[a][a'] = Qu[(a a')][x]
    const OpenLeg yv{Qv, c2, chi, 1};            // X_y[b][b'] = Qv[y][(b b')]
    site_transfer(a, a1, a2, all, none, S, Ga, &xu);
    site_transfer(b, b1, b2, all, none, S, Gb, &yv);
    // H(x) = M_1^T G_a(x) M_2, batched over x
    double *H1 = S.alloc((size_t)c2 * c4), *H = S.alloc((size_t)c2 * c4);
    std::vector<const void *> pa, pb, pc1, qa, qb, qc;
    for (long x = 0; x < c2; ++x) {
      pa.push_back(M1);
      pb.push_back(Ga + 2 * (size_t)x * c4);
      pc1.push_back(H1 + 2 * (size_t)x * c4);
      qa.push_back(pc1.back());
      qb.push_back(M2);
      qc.push_back(H + 2 * (size_t)x * c4);
    }
    GemmDesc tA = square_desc(c2);
    tA.a_mi = 1;
    tA.a_ki = c2;
    S.gemm(tA, pa, pb, pc1);
    S.gemm(square_desc(c2), qa, qb, qc);
    // E[x][y] = sum_{(j k)} H[x][(j k)] G_b[y][(j k)]
    GemmDesc f;
    f.M = f.Mi = (int)c2;
    f.N = f.Ni = (int)c2;
    f.K = f.Ki = (int)c4;
    f.a_mi = c4; f.a_ki = 1;
    f.b_ki = 1; f.b_ni = c4;
    f.c_mi = c2; f.c_ni = 1;
    E = S.alloc(c4);
    S.gemm1(f, H, Gb, E);
  } else {
    return -1.0;
  }
  // E^H E, then its eigenvalues s_i^2 (descending)
  GemmDesc h = square_desc(c2);
  h.a_mi = 1;
  h.a_ki = c2;
  h.conjA = 1;
  h.herm = 1;
  double *G = S.alloc(c4), *V = S.alloc(c4), *ev = S.alloc(c2);
  S.gemm1(h, E, E, G);
  const void *ep[3] = {G, ev, V};
  S.be->h2d(S.parr, ep, sizeof(ep));
  S.be->eigh((int)c2, (int)c2, (const double *const *)S.parr, (double *const *)(S.parr + 1),
             (double *const *)(S.parr + 2), 1, 1);   // eigenvalues only
  std::vector<double> l(c2);
  S.be->d2h(l.data(), ev, (size_t)c2 * 8);
  double tot = 0.0;
  for (double x : l) tot += std::max(x, 0.0);
  const double l1 = std::max(l[0], 0.0);
  if (spectrum)
    for (long i = 0; i < c2; ++i)
      spectrum[i] = tot > 0 ? std::sqrt(std::max(l[i], 0.0) / tot) : 0.0;
  return tot > 0 ? 1.0 - std::sqrt(l1 / tot) : NAN;
}

void Engine::observe_pauli(double *out) {
  int np = (int)prob_.pauli_offsets.size() - 1;
  for (int k = 0; k < np; ++k) {
    double a = pauli_value(k, true);
    double b = pauli_value(k, false);
    out[k] = a / b;
  }
}

// Exact contraction of a tree cluster with BP messages on the cut legs; Re(value).
namespace {
// 2x2 complex Pauli matrices (row-major re, im): I, X, Y, Z
const double kPauli[4][8] = {
    {1, 0, 0, 0, 0, 0, 1, 0},
    {0, 0, 1, 0, 1, 0, 0, 0},
    {0, 0, 0, -1, 0, 1, 0, 0},
    {1, 0, 0, 0, 0, 0, -1, 0}};
}  // namespace

// The ket of site v with its operator (0 = identity) applied on the physical leg.
double *Engine::site_ket(int v, int opcode, EngineScratch &S) {
  Plan &P = *plan_;
  double *cur = S.alloc((size_t)P.tsize[v]);
  double *opbuf = S.alloc(4);
  int64_t *hbuf = (int64_t *)S.alloc(1);
  const int64_t half = P.tsize[v] / 2;
  S.be->h2d(opbuf, kPauli[opcode], sizeof(kPauli[opcode]));
  S.be->h2d(hbuf, &half, 8);
  const void *pp[2] = {P.T + 2 * P.toff[v], cur};
  S.be->h2d(S.parr, pp, sizeof(pp));
  S.be->apply_op((const double *const *)S.parr, (double *const *)(S.parr + 1), hbuf, opbuf, 1);
  return cur;
}

// Environment of the subtree at v seen from `parent` (a chi x chi matrix on v's leg to parent):
// the ket with the site's operator, the bra, every leg to another cluster site closed with that
// site's own subtree environment, every leg leaving the cluster with its incoming BP message.
double *Engine::branch_env(int v, int parent, const std::set<int> &cs, const std::map<int, int> &op,
                           EngineScratch &S) {
  Plan &P = *plan_;
  const int chi = P.chi, d = P.deg[v];
  const long c2 = (long)chi * chi;
  Layout L = t_layout(d, chi);
  auto o = op.find(v);
  double *cur = site_ket(v, o == op.end() ? 0 : o->second, S);
  int pleg = -1;
  for (int i = 0; i < d; ++i) {
    const int u = P.nb[v][i];
    if (u == parent) {
      pleg = i;
      continue;
    }
    const double *E = cs.count(u) ? branch_env(u, v, cs, op, S)
                                  : P.M + 2 * (size_t)P.in_msg[v][i] * c2;
    double *nxt = S.alloc((size_t)P.tsize[v]);
    S.gemm1(leg_desc(d, i, L, L, chi), cur, E, nxt);
    cur = nxt;
  }
  double *out = S.alloc(c2);
  S.gemm1(close_desc(d, pleg, L, chi), cur, P.T + 2 * P.toff[v], out);
  return out;
}

// Norm transfer matrix of site v between its legs to `prev` and `next`:
// F[(a a'), (b b')] = sum T'[s][a][b][x] conj(T[s][a'][b'][x]) / ||T_v||^2, a the leg to prev, b to
// next, x the remaining leg (if any) closed with its cluster environment or message; T' the ket
// with the site's operator.  `open`: instead, chi^2 transfer matrices, the x-th with the remaining
// leg closed with the chi x chi matrix X_x of `open`, written at dst + x chi^4.
void Engine::site_transfer(int v, int prev, int next, const std::set<int> &cs,
                           const std::map<int, int> &op, EngineScratch &S, double *dst,
                           const OpenLeg *open) {
  Plan &P = *plan_;
  const int chi = P.chi, d = P.deg[v];
  const long c2 = (long)chi * chi;
  const size_t c4 = (size_t)c2 * c2;
  Layout L = t_layout(d, chi);
  const double *Tv = P.T + 2 * P.toff[v];
  auto o = op.find(v);
  double *cur = site_ket(v, o == op.end() ? 0 : o->second, S);
  int lp = -1, ln = -1, lx = -1;
  for (int i = 0; i < d; ++i) {
    const int u = P.nb[v][i];
    if (u == prev) lp = i;
    else if (u == next) ln = i;
    else lx = i;
  }
  std::vector<double> th((size_t)2 * P.tsize[v]);
  S.be->d2h(th.data(), Tv, (size_t)P.tsize[v] * 16);
  double nrm2 = 0.0;
  for (double x : th) nrm2 += x * x;
  GemmDesc g;
  g.M = (int)c2; g.Mi = chi; g.a_mo = L.leg[lp]; g.a_mi = L.leg[ln];
  g.N = (int)c2; g.Ni = chi; g.b_no = L.leg[lp]; g.b_ni = L.leg[ln];
  g.c_mo = c2 * chi; g.c_mi = chi; g.c_no = c2; g.c_ni = 1;
  g.conjB = 1;
  if (lx < 0) {                      // K = s
    g.K = 2; g.Ki = 2; g.a_ki = L.s; g.b_ki = L.s;
  } else {                           // K = (s, x)
    g.K = 2 * chi; g.Ki = chi;
    g.a_ko = L.s; g.a_ki = L.leg[lx];
    g.b_ko = L.s; g.b_ki = L.leg[lx];
  }
  g.alpha_re = nrm2 > 0.0 ? 1.0 / nrm2 : 1.0;
  if (!open) {
    if (lx >= 0) {
      const int u = P.nb[v][lx];
      const double *E = cs.count(u) ? branch_env(u, v, cs, op, S)
                                    : P.M + 2 * (size_t)P.in_msg[v][lx] * c2;
      double *nxt = S.alloc((size_t)P.tsize[v]);
      S.gemm1(leg_desc(d, lx, L, L, chi), cur, E, nxt);
      cur = nxt;
    }
    S.gemm1(g, cur, Tv, dst);
    return;
  }
  // batched over the chi^2 matrices X_x: the ket's leg x closed with X_x, then the transfer
  double *curs = S.alloc((size_t)c2 * P.tsize[v]);
  std::vector<const void *> a, b, c, a2, b2, c2v;
  for (long x = 0; x < c2; ++x) {
    a.push_back(cur);
    b.push_back(open->base + 2 * (size_t)(x * open->sx));
    c.push_back(curs + 2 * (size_t)x * P.tsize[v]);
    a2.push_back(c.back());
    b2.push_back(Tv);
    c2v.push_back(dst + 2 * (size_t)x * c4);
  }
  GemmDesc ab = leg_desc(d, lx, L, L, chi);
  ab.b_ki = open->sk;
  ab.b_ni = open->sn;
  S.gemm(ab, a, b, c);
  S.gemm(g, a2, b2, c2v);
}

// Product of the transfer matrices of the sites of `walk`, each between its legs to the site
// before it (`before` for the first) and after it (`after` for the last); the identity for an
// empty walk.  A chi^2 x chi^2 matrix, rows the first site's leg to `before`.
double *Engine::chain(const std::vector<int> &walk, int before, int after, EngineScratch &S) {
  const int chi = plan_->chi;
  const long c2 = (long)chi * chi;
  const size_t c4 = (size_t)c2 * c2;
  std::set<int> all;
  for (int w = 0; w < plan_->n; ++w) all.insert(w);
  const std::map<int, int> none;
  double *acc = S.alloc(c4);
  if (walk.empty()) {
    std::vector<double> id(2 * c4, 0.0);
    for (long i = 0; i < c2; ++i) id[2 * (i * c2 + i)] = 1.0;
    S.be->h2d(acc, id.data(), c4 * 16);
    return acc;
  }
  const int m = (int)walk.size();
  double *F = m > 1 ? S.alloc(c4) : nullptr, *other = m > 1 ? S.alloc(c4) : nullptr;
  for (int k = 0; k < m; ++k) {
    const int pv = k ? walk[k - 1] : before, nx = k + 1 < m ? walk[k + 1] : after;
    site_transfer(walk[k], pv, nx, all, none, S, k ? F : acc, nullptr);
    if (k) {
      S.gemm1(square_desc(c2), acc, F, other);
      std::swap(acc, other);
    }
  }
  return acc;
}

double Engine::pauli_value(int k, bool with_ops) {
  Plan &P = *plan_;
  const int chi = P.chi;
  const long c2 = (long)chi * chi;
  int b0 = prob_.pauli_offsets[k], b1 = prob_.pauli_offsets[k + 1];
  std::vector<int> sites(prob_.pauli_sites.begin() + b0, prob_.pauli_sites.begin() + b1);
  std::map<int, int> op;
  if (with_ops)
    for (int i = b0; i < b1; ++i) op[prob_.pauli_sites[i]] = prob_.pauli_ops[i];
  EngineScratch S(be_, prob_.precision);
  std::set<int> cs(sites.begin(), sites.end());
  int inner = 0;
  for (int v : sites)
    for (int u : P.nb[v]) inner += cs.count(u) ? 1 : 0;
  inner /= 2;
  if (inner == (int)sites.size() - 1) {
    // a tree cluster: every neighbour of the root closed with its subtree, then rho at the root
    const int v = sites[0], d = P.deg[v];
    Layout L = t_layout(d, chi);
    double *cur = site_ket(v, with_ops ? op[v] : 0, S);
    for (int i = 0; i < d; ++i) {
      const int u = P.nb[v][i];
      const double *E = cs.count(u) ? branch_env(u, v, cs, op, S)
                                    : P.M + 2 * (size_t)P.in_msg[v][i] * c2;
      double *nxt = S.alloc((size_t)P.tsize[v]);
      S.gemm1(leg_desc(d, i, L, L, chi), cur, E, nxt);
      cur = nxt;
    }
    double *rho = S.alloc(4);
    int64_t *hbuf = (int64_t *)S.alloc(1);
    const int64_t half = P.tsize[v] / 2;
    S.be->h2d(hbuf, &half, 8);
    const void *rp[2] = {cur, P.T + 2 * P.toff[v]};
    S.be->h2d(S.parr, rp, sizeof(rp));
    S.be->rho_dot((const double *const *)S.parr, (const double *const *)(S.parr + 1), hbuf, rho,
                  1);
    double r[8];
    S.be->d2h(r, rho, sizeof(r));
    return r[0] + r[6];        // Re(rho00 + rho11); imaginary part ~ 0 for Hermitian ops
  }
  // a cluster with one loop: the branches hanging off the loop are contracted into
  // environments; every loop site becomes its norm transfer matrix (scaled by 1 / ||T||^2) and
  // the value is Tr(F_0 F_1 ... F_{m-1}).
  std::vector<int> loop = cycle_of(cs);
  if (loop.empty()) return NAN;             // not a single loop (rejected on input)
  const int m = (int)loop.size();
  const size_t c4 = (size_t)c2 * c2;
  double *F = S.alloc(c4), *Ra = S.alloc(c4), *Rb = S.alloc(c4), *acc = nullptr;
  for (int i = 0; i < m; ++i) {
    double *dst = i == 0 ? Ra : F;
    site_transfer(loop[i], loop[(i + m - 1) % m], loop[(i + 1) % m], cs, op, S, dst, nullptr);
    if (i > 0) {
      double *out = acc == Ra ? Rb : Ra;
      S.gemm1(square_desc(c2), acc, F, out);
      acc = out;
    } else {
      acc = Ra;
    }
  }
  double *tr = S.alloc(1);
  S.be->trace(acc, (int)c2, tr);
  double t2[2];
  S.be->d2h(t2, tr, sizeof(t2));
  return t2[0];
}

// The cycle of a set of sites whose induced subgraph has exactly one loop (the branches peeled
// off), in walk order from its smallest site; empty if there is not exactly one loop.
std::vector<int> Engine::cycle_of(const std::set<int> &cs) const {
  const Plan &P = *plan_;
  std::map<int, int> cdeg;
  for (int v : cs)
    for (int u : P.nb[v]) cdeg[v] += cs.count(u) ? 1 : 0;
  std::set<int> cyc = cs;
  std::vector<int> leaves;
  for (int v : cs)
    if (cdeg[v] <= 1) leaves.push_back(v);
  while (!leaves.empty()) {
    const int v = leaves.back();
    leaves.pop_back();
    if (!cyc.erase(v)) continue;
    for (int u : P.nb[v])
      if (cyc.count(u) && --cdeg[u] == 1) leaves.push_back(u);
  }
  if (cyc.size() < 3) return {};
  std::vector<int> loop{*cyc.begin()};
  for (int prev = -1;;) {
    const int w = loop.back();
    int nx = -1;
    for (int u : P.nb[w])
      if (cyc.count(u) && u != prev && (nx < 0 || u < nx)) nx = u;
    if (nx < 0 || loop.size() > cyc.size()) return {};
    if (nx == loop.front() && loop.size() > 2) break;
    prev = w;
    loop.push_back(nx);
  }
  return loop.size() == cyc.size() ? loop : std::vector<int>{};
}

const std::vector<int> &Engine::bond_dims() const { return plan_->bond_h; }

void Engine::get_state(double *tensors, double *messages, int32_t *bond_dims) {
  Plan &P = *plan_;
  if (tensors) be_->d2h(tensors, P.T, tensor_elems() * 16);
  if (messages) be_->d2h(messages, P.M, message_elems() * 16);
  if (bond_dims)
    for (int e = 0; e < P.E; ++e) bond_dims[e] = P.bond_h[e];
}

void Engine::set_state(const double *tensors, const double *messages, const int32_t *bond_dims) {
  t32_stale_ = true;
  Plan &P = *plan_;
  if (tensors) be_->h2d(P.T, tensors, tensor_elems() * 16);
  if (messages) be_->h2d(P.M, messages, message_elems() * 16);
  if (bond_dims)
    for (int e = 0; e < P.E; ++e) P.bond_h[e] = bond_dims[e];
}

}  // namespace bpki
