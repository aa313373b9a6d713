// Host stand-in for the device backend of libbpki, for checking the host code (engine schedule,
// C ABI, serving threads, sessions, allocators) under AddressSanitizer and UBSan without a GPU.
// "Device" memory is host memory; every copy is a memcpy, so the sanitizers see each copy's
// bounds against its allocation.  The compute kernels only write the scalars the host reads back,
// with values that let a solve run its whole schedule (BP converges in one sweep, bonds stay at
// one, <Z> = 1); their numbers mean nothing.
#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <string>

#include "../../paper_2306_14887_amd/csrc/bpki_internal.h"

namespace bpki {

namespace {

class StubBackend : public Backend {
  double rd_[2] = {0, 0};

 public:
  int set_allocator(DevAlloc a, DevFree f, void *user) override {
    if (touched_ || !a != !f) return -1;
    ua_ = a;
    uf_ = f;
    uu_ = user;
    return 0;
  }
  void *alloc(size_t bytes) override {
    touched_ = true;
    if (err_) return nullptr;
    void *p = ua_ ? ua_(bytes ? bytes : 16, this, uu_) : std::calloc(1, bytes ? bytes : 16);
    if (!p) {
      err_ = -4;
      msg_ = "stub allocation failed";
      return nullptr;
    }
    if (ua_ && (reinterpret_cast<uintptr_t>(p) & 255)) {
      uf_(p, this, uu_);
      err_ = -5;
      msg_ = "allocator returned memory not aligned to 256 bytes";
      return nullptr;
    }
    if (ua_) std::memset(p, 0, bytes ? bytes : 16);
    return p;
  }
  void release(void *p) override {
    if (!p) return;
    if (uf_) uf_(p, this, uu_);
    else std::free(p);
  }
  void forget_workspaces() override {}
  void clear_alloc_error() override {
    if (err_ == -4) {
      err_ = 0;
      msg_.clear();
    }
  }
  void h2d(void *d, const void *h, size_t b) override {
    if (!err_ && b) std::memcpy(d, h, b);
  }
  void d2h(void *h, const void *d, size_t b) override {
    if (!err_ && b) std::memcpy(h, d, b);
  }
  void read_async(const double *src, int slot) override {
    if (!err_) std::memcpy(&rd_[slot & 1], src, 8);
  }
  double wait_read(int slot) override { return rd_[slot & 1]; }
  void d2d(void *d, const void *s, size_t b) override {
    if (!err_ && b) std::memmove(d, s, b);
  }
  void sync() override {}
  int check(std::string *m) override {
    if (m) *m = msg_;
    return err_;
  }
  void timer_mark(int) override {}
  double timer_ms(int, int) override { return 0.0; }
  void gemm_profile(int) override {}
  void gemm_profile_read(long *s, long *a, double *ms, double *f) override {
    if (s) *s = 0;
    if (a) *a = 0;
    if (ms) *ms = 0;
    if (f) *f = 0;
  }
  void gemm_profile_read_prec(int, long *s, double *ms, double *f) override {
    if (s) *s = 0;
    if (ms) *ms = 0;
    if (f) *f = 0;
  }
  void gemm_profile_read_kernel(int, int, long *s, double *ms, double *f, double *b,
                                long *a) override {
    gemm_profile_read_prec(0, s, ms, f);
    if (b) *b = 0;
    if (a) *a = 0;
  }
  void bp_close(const BpCloseDesc &, const double *const *, const double *const *,
                const double *const *, double *const *, int) override {}
  void gemm(const GemmDesc &, const double *const *, const double *const *, double *const *,
            int) override {}
  void eigh(int n, int, const double *const *, double *const *evals, double *const *,
            int nprob, int) override {
    for (int p = 0; p < nprob; ++p)
      for (int i = 0; i < n; ++i) evals[p][i] = i == 0 ? 1.0 : 0.0;
  }
  void rx(double *const *, const int64_t *, int, double, double) override {}
  void msg_sqrt(int, const double *const *, const double *const *, double *const *,
                double *const *, double, int) override {}
  void bond_entropy(int, const double *const *, double *out, int nprob) override {
    for (int p = 0; p < nprob; ++p) out[p] = 0.0;
  }
  void trace(const double *, int, double *out) override {
    out[0] = 1.0;
    out[1] = 0.0;
  }
  void vidal_svd(int n, const double *const *, const double *const *, double *const *,
                 double *const *, double *const *, double *const *, double *lam, int *kept,
                 double, int nprob) override {
    for (int p = 0; p < nprob; ++p) {
      kept[p] = 1;
      for (int i = 0; i < n; ++i) lam[(size_t)p * n + i] = i == 0 ? 1.0 : 0.0;
    }
  }
  void gram_chol(int, const double *const *, double *const *, double *const *, double,
                 int) override {}
  void theta(int, int, int, const double *const *, const double *const *, double *const *,
             double, double, double, double, int) override {}
  void svd_finish(int, int, const double *const *, const double *const *, double *const *,
                  double *const *, int *kout, double *disc, double *const *, double *const *,
                  double, int nprob) override {
    for (int p = 0; p < nprob; ++p) {
      kout[p] = 1;
      disc[2 * p] = 0.0;
      disc[2 * p + 1] = INFINITY;
    }
  }
  void split_sqrt(int, int, int, int, const double *const *, const double *const *,
                  const double *const *, double *const *, double *const *, int) override {}
  void to_f32(const double *src, float *dst, size_t n) override {
    for (size_t i = 0; i < 2 * n; ++i) dst[i] = (float)src[i];
  }
  void normalize_residual(int, double *const *, const double *const *, double *res,
                          int nprob) override {
    for (int p = 0; p < nprob; ++p) res[p] = 0.0;
  }
  void reduce_max(const double *x, int n, double *out) override {
    double m = 0.0;
    for (int i = 0; i < n; ++i) m = std::max(m, x[i]);
    *out = m;
  }
  void member_residual(const double *res, const int *off, const int *idx, int nmem,
                       const int *act, int *act_next, double tol, double *out) override {
    for (int j = 0; j < nmem; ++j) {
      double m = 0.0;
      for (int k = off[j]; k < off[j + 1]; ++k) m = std::max(m, res[idx[k]]);
      out[j] = m;
      act_next[j] = act[j] && !(m < tol);
    }
  }
  void commit_messages(double *M, const double *Mn, long elems, int nmsg, const int *member,
                       const int *act) override {
    for (int m = 0; m < nmsg; ++m)
      if (act[member[m]])
        std::memcpy(M + 2 * (size_t)m * elems, Mn + 2 * (size_t)m * elems, 16 * (size_t)elems);
  }
  double mfma_rate(int, int, int) override { return 0.0; }
  void rho_dot(const double *const *, const double *const *, const int64_t *, double *rho,
               int nprob) override {
    for (int p = 0; p < nprob; ++p) {
      std::fill(rho + 8 * (size_t)p, rho + 8 * (size_t)p + 8, 0.0);
      rho[8 * (size_t)p] = 1.0;                     // rho = |0><0|
    }
  }
  void apply_op(const double *const *, double *const *, const int64_t *, const double *,
                int) override {}

 private:
  int err_ = 0;
  std::string msg_;
  DevAlloc ua_ = nullptr;
  DevFree uf_ = nullptr;
  void *uu_ = nullptr;
  bool touched_ = false;
};

}  // namespace

Backend *make_hip_backend(int device, void *, std::string *err) {
  if (device != 0) {
    if (err) *err = "stub: only device 0";
    return nullptr;
  }
  return new StubBackend;
}

// The stand-in for the per-device static array: one host block per device, held until the process
// ends (a plain static array, so the block stays referenced through exit).
int scratch_region(int device, void **ptr, std::string *err) {
  static std::mutex mu;
  static void *addr[8] = {};
  if (device < 0 || device >= 8) {
    if (err) *err = "stub scratch: device";
    return -5;
  }
  std::lock_guard<std::mutex> lk(mu);
  if (!addr[device]) addr[device] = std::aligned_alloc(256, kScratchBytes);
  if (!addr[device]) {
    if (err) *err = "stub scratch";
    return -5;
  }
  *ptr = addr[device];
  return 0;
}

}  // namespace bpki
