// Krylov drivers (sections IV and V): right-preconditioned GMRES(m) for the
// inner solves Z^-1 v, and the implicitly restarted Arnoldi iteration (exact
// shifts) on OP = Z^-1 R, whose largest-magnitude eigenvalues mu give the
// characteristic values of smallest magnitude, lambda = i (1 - 1/mu)
// (eqs. (23)-(24)).  Krylov vectors live on the device in FP64 and are
// orthogonalised there (classical Gram-Schmidt with one DGKS correction);
// the small Hessenberg matrices (<= a few hundred) are factorised on the host.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <complex>
#include <cstdio>
#include <memory>
#include <numeric>
#include <vector>

#include "cm_device.h"

namespace cm {

int blas_multidot_blocks(int64_t N);
void blas_multidot_wide(const double2* V, int64_t ldv, const double2* w, int64_t N, int nk, double2* part,
                        double2* h, const int* flag, hipStream_t s);
void blas_gemv_sub(const double2* V, int64_t ldv, const double2* h, int nk, double2* w, int64_t N, hipStream_t s,
                   const int* flag = nullptr);
void blas_gmres_step(int j, int m, const double2* hc, double2* col, double2* H, double2* g, double2* cs, double2* sn,
                     GmState* st, int pass, hipStream_t s);
void blas_scale_by_state(double2* y, const GmState* st, int64_t N, hipStream_t s);
void blas_axpby(const double2* x, double2 alpha, double2* y, int64_t N, int accumulate, hipStream_t s);
void blas_scale(double2* y, double2 alpha, int64_t N, hipStream_t s);
void blas_basis_update(const double2* V, int64_t ldv, const double2* Q, int ldq, int nk, int nc, double2* Vout,
                       int64_t N, hipStream_t s);
void blas_to_c64(const double2* x, float2* y, int64_t N, hipStream_t s);
void blas_to_c128(const float2* x, double2* y, int64_t N, hipStream_t s);

static void chk_d(hipError_t e, const char* what) {
  if (e != hipSuccess) {
    if (e == hipErrorOutOfMemory) throw Error(-3, std::string(what) + ": out of device memory");
    throw Error(-4, std::string(what) + ": " + hipGetErrorString(e));
  }
}

struct DevBuf {
  void* p = nullptr;
  // bytes == 0: empty until alloc()
  explicit DevBuf(size_t bytes) {
    if (bytes) alloc(bytes);
  }
  void alloc(size_t bytes) { chk_d(hipMalloc(&p, std::max<size_t>(bytes, 16)), "driver workspace"); }
  ~DevBuf() {
    if (p) (void)hipFree(p);
  }
  DevBuf(const DevBuf&) = delete;
  DevBuf& operator=(const DevBuf&) = delete;
  double2* d() const { return (double2*)p; }
};

// Shared machinery: the operator applications on FP64 vectors, and the
// orthogonalisation of w against V[0..j).
class KrylovCtx {
 public:
  // sai_part: the SAI slot that precond() applies (0: of Z_near, 1: of the
  // shifted operator's near field); tau: the shift of op 5, y = tau R x + i X x
  KrylovCtx(Dev& d, const Plan& P, bool far64, hipStream_t s, int sai_part = 0, double tau = 1.0)
      : d_(d), P_(P), far64_(far64), s_(s), N_(d.N), sai_part_(sai_part), tau_(tau), t32a_(d.N * sizeof(float2)),
        t32b_(d.N * sizeof(float2)), hdev_(1025 * sizeof(double2)),
        part_((size_t)1025 * blas_multidot_blocks(d.N) * sizeof(double2)) {
    chk_d(hipHostMalloc((void**)&pin_, kRing * sizeof(double), hipHostMallocDefault), "pinned residuals");
    for (auto& e : ev_) {
      if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) {
        release();
        throw Error(-4, "hipEventCreateWithFlags");
      }
    }
  }
  ~KrylovCtx() { release(); }
  KrylovCtx(const KrylovCtx&) = delete;
  KrylovCtx& operator=(const KrylovCtx&) = delete;

  // residual estimate of device GMRES iteration j: copied to pinned host
  // memory behind the iteration's work (post_residual) and read once its
  // event has completed (residual); a ring of kRing slots
  void post_residual(int j, const double* dres) {
    chk_d(hipMemcpyAsync(pin_ + j % kRing, dres, sizeof(double), hipMemcpyDeviceToHost, s_), "residual copy");
    chk_d(hipEventRecord(ev_[j % kRing], s_), "residual event");
  }
  double residual(int j) {
    chk_d(hipEventSynchronize(ev_[j % kRing]), "residual event");
    return pin_[j % kRing];
  }

  int64_t N() const { return N_; }
  hipStream_t stream() const { return s_; }
  bool verbose() const { return (P_.opt.flags & CM_FLAG_VERBOSE) != 0; }

  // the Calderon preconditioner that ops 6 and 7 use (cm_cmp_build)
  void set_cmp(const CmpD* c) { cmp_ = c; }

  // y = op(x), op 0 = Z, 1 = R, 2 = X, 5 = tau R + i X (an R and an X
  // apply), 6 = Z~ G^-1 Z (the Calderon-preconditioned operator of eq. (25)),
  // 7 = G (the mixed Gram matrix); far field in FP64 or FP32
  void apply(int op, const double2* x, double2* y) {
    if (op == 6) {
      if (!c6_.p) c6_.alloc((size_t)N_ * sizeof(double2));
      apply(0, x, c6_.d());
      cmp_left(c6_.d(), y);
      return;
    }
    if (op == 7) {
      blas_csr_real(cmp_->G, x, y, s_);
      return;
    }
    if (op == 5) {
      if (!tsh_.p) tsh_.alloc((size_t)N_ * sizeof(double2));
      apply(1, x, tsh_.d());
      apply(2, x, y);
      blas_scale(y, make_double2(0.0, 1.0), N_, s_);
      blas_axpby(tsh_.d(), make_double2(tau_, 0.0), y, N_, 1, s_);
      return;
    }
    ++n_apply;
    if (far64_) {
      dev_apply(d_, P_, op, x, y, 1, 1, true, s_);
    } else {
      blas_to_c64(x, (float2*)t32a_.p, N_, s_);
      dev_apply(d_, P_, op, t32a_.p, t32b_.p, 1, 1, false, s_);
      blas_to_c128((const float2*)t32b_.p, y, N_, s_);
    }
  }
  void precond(const double2* x, double2* y) { dev_sai_apply(d_, P_, x, y, 1, 1, true, sai_part_, s_); }

  // y = Z~ G^-1 u: the Gram solve by GMRES on G to a relative residual of
  // 1e-12 (a context of its own), then B Z_ref B^T on the refined mesh
  void cmp_left(const double2* u, double2* y);
  // y = Z~ x (B Z_ref B^T x)
  void cmp_ztilde(const double2* x, double2* y);
  int64_t n_ref_apply = 0, n_gram_iters = 0, n_gram_fail = 0;
  double gram_tol = 1e-12;   // relative residual of the Gram solves

  // h[k] = V[k]^H w, k < nk <= 1025 (device output), over all CUs
  void multidot(const double2* V, int nk, const double2* w, double2* h) {
    if (nk > 1025) throw Error(-1, "multidot: more than 1025 vectors");
    blas_multidot_wide(V, N_, w, N_, nk, part_.d(), h, nullptr, s_);
  }

  double norm(const double2* w) {
    multidot(w, 1, w, hdev_.d());
    double2 h;
    chk_d(hipMemcpyAsync(&h, hdev_.p, sizeof h, hipMemcpyDeviceToHost, s_), "norm");
    chk_d(hipStreamSynchronize(s_), "norm");
    return std::sqrt(std::max(h.x, 0.0));
  }

  // Orthogonalise w against V[0..j) (columns of length N, stride N); h[0..j)
  // receives the coefficients, the return value is ||w|| afterwards.
  double orth(const double2* V, int j, double2* w, std::vector<cplx>& h) {
    h.assign(j, cplx(0));
    double before = norm(w);
    if (j == 0) return before;
    std::vector<double2> hh(j);
    for (int pass = 0; pass < 2; ++pass) {
      multidot(V, j, w, hdev_.d());
      blas_gemv_sub(V, N_, hdev_.d(), j, w, N_, s_);
      chk_d(hipMemcpyAsync(hh.data(), hdev_.p, j * sizeof(double2), hipMemcpyDeviceToHost, s_), "orth");
      chk_d(hipStreamSynchronize(s_), "orth");
      for (int k = 0; k < j; ++k) h[k] += cplx(hh[k].x, hh[k].y);
      double after = norm(w);
      if (after > 0.717 * before) return after;   // DGKS: one correction when cancellation occurred
      before = after;
    }
    return norm(w);
  }

  // The new Krylov vector w = V[:, j] orthogonalised in place against
  // V[0..j): classical Gram-Schmidt with w^H w taken in the same reduction,
  // so one host round trip per pass; ||w|| afterwards from Pythagoras unless
  // cancellation occurred, when a second pass follows (DGKS, as in orth).
  double orth_next(double2* V, int j, std::vector<cplx>& h) {
    double2* w = V + (size_t)j * N_;
    h.assign(j, cplx(0));
    std::vector<double2> hh(j + 1);
    for (int pass = 0; pass < 2; ++pass) {
      multidot(V, j + 1, w, hdev_.d());   // V[0..j]^H w; the last entry is w^H w
      if (j > 0) blas_gemv_sub(V, N_, hdev_.d(), j, w, N_, s_);
      chk_d(hipMemcpyAsync(hh.data(), hdev_.p, (j + 1) * sizeof(double2), hipMemcpyDeviceToHost, s_), "orth");
      chk_d(hipStreamSynchronize(s_), "orth");
      const double ww = hh[j].x;
      double hs = 0;
      for (int k = 0; k < j; ++k) {
        h[k] += cplx(hh[k].x, hh[k].y);
        hs += hh[k].x * hh[k].x + hh[k].y * hh[k].y;
      }
      const double r2 = ww - hs;
      if (j == 0 || r2 > 0.514 * ww) return std::sqrt(std::max(r2, 0.0));   // 0.514 = 0.717^2
    }
    return norm(w);
  }

  void scale_copy(const double2* x, cplx a, double2* y) {
    blas_axpby(x, make_double2(a.real(), a.imag()), y, N_, 0, s_);
  }
  void axpy(const double2* x, cplx a, double2* y) { blas_axpby(x, make_double2(a.real(), a.imag()), y, N_, 1, s_); }

  // Vout[:, c] = sum_k V[:, k] Q(k, c), c < nc, Q column-major host matrix (ldq rows)
  void combine(const double2* V, int nk, const std::vector<cplx>& Q, int ldq, int nc, double2* Vout) {
    std::vector<double2> q(Q.size());
    for (size_t i = 0; i < Q.size(); ++i) q[i] = make_double2(Q[i].real(), Q[i].imag());
    DevBuf qd(q.size() * sizeof(double2));
    chk_d(hipMemcpyAsync(qd.p, q.data(), q.size() * sizeof(double2), hipMemcpyHostToDevice, s_), "combine");
    blas_basis_update(V, N_, qd.d(), ldq, nk, nc, Vout, N_, s_);
    chk_d(hipStreamSynchronize(s_), "combine");
  }

  int64_t n_apply = 0;

 private:
  Dev& d_;
  const Plan& P_;
  bool far64_;
  hipStream_t s_;
  int64_t N_;
  int sai_part_;
  double tau_;
  DevBuf t32a_, t32b_, hdev_, part_, tsh_{0};
  const CmpD* cmp_ = nullptr;
  std::unique_ptr<KrylovCtx> gk_;            // the Gram solves' context
  DevBuf c6_{0}, cg_{0}, r1_{0}, r2_{0}, r32a_{0}, r32b_{0};
  static constexpr int kRing = 8;
  double* pin_ = nullptr;
  hipEvent_t ev_[kRing] = {};
  void release() {
    for (auto& e : ev_)
      if (e) {
        (void)hipEventDestroy(e);
        e = nullptr;
      }
    if (pin_) (void)hipHostFree(pin_);
    pin_ = nullptr;
  }
};

// ---------------------------------------------------------------- GMRES
struct GmresResult {
  int iters = 0;
  double relres = 0;
  bool converged = false;
};

// Solve A x = b, right-preconditioned by the SAI P (x = P u) when precond;
// A = Z (aop 0), X (aop 2, the route of eq. (14)) or tau R + i X (aop 5), P
// the SAI that the context's precond() applies (of the matching near field).
//
// Each iteration is enqueued without a host round trip: the Gram-Schmidt
// coefficients come from an all-CU multidot, the Hessenberg column, its
// Givens rotation and the residual estimate from k_gmres_step, and the
// conditional second (DGKS) pass runs or skips on a device flag.  The host
// reads the residual estimate of the iteration two behind the one it has just
// enqueued (pinned memory, one event per iteration), so the GPU always has
// work queued; a cycle that converges may therefore take up to two more
// columns, which only lowers the residual.  The small triangular solve at the
// end of a cycle runs on the host.
static GmresResult gmres(KrylovCtx& K, const double2* b, double2* x, int m, int maxit, double tol, bool precond,
                         int aop = 0) {
  const int64_t N = K.N();
  hipStream_t s = K.stream();
  const int nblk = blas_multidot_blocks(N);
  DevBuf Vb((size_t)(m + 1) * N * sizeof(double2)), w(N * sizeof(double2)), z(N * sizeof(double2)),
      u(N * sizeof(double2)), part((size_t)(m + 2) * nblk * sizeof(double2)),
      small((size_t)((m + 1) * m + (m + 1) + 2 * m + 2 * (m + 2)) * sizeof(double2) + sizeof(GmState));
  double2* V = Vb.d();
  double2* Hd = small.d();
  double2* gd = Hd + (size_t)(m + 1) * m;
  double2* csd = gd + (m + 1);
  double2* snd = csd + m;
  double2* hc = snd + m;
  double2* col = hc + (m + 2);
  GmState* st = reinterpret_cast<GmState*>(col + (m + 2));
  constexpr int kLag = 2;
  GmresResult res;
  chk_d(hipMemsetAsync(x, 0, N * sizeof(double2), s), "gmres");
  const double bn = K.norm(b);
  if (bn == 0) {
    res.converged = true;
    return res;
  }
  K.scale_copy(b, 1.0, w.d());   // r = b (x0 = 0)
  double beta = bn;
  std::vector<cplx> H((size_t)(m + 1) * m), g(m + 1);
  std::vector<double2> Hh((size_t)(m + 1) * m), gh(m + 1);
  while (res.iters < maxit) {
    K.scale_copy(w.d(), 1.0 / beta, V);
    GmState s0{};
    std::vector<double2> g0(m + 1, make_double2(0.0, 0.0));
    g0[0] = make_double2(beta, 0.0);
    chk_d(hipMemcpyAsync(gd, g0.data(), (m + 1) * sizeof(double2), hipMemcpyHostToDevice, s), "gmres");
    chk_d(hipMemcpyAsync(st, &s0, sizeof s0, hipMemcpyHostToDevice, s), "gmres");
    const int jmax = std::min(m, maxit - res.iters);
    int j = 0;
    for (; j < jmax; ++j) {
      const double2* vj = V + (size_t)j * N;
      double2* vn = V + (size_t)(j + 1) * N;   // the new vector is built in its slot
      if (precond) {
        K.precond(vj, z.d());
        K.apply(aop, z.d(), vn);
      } else {
        K.apply(aop, vj, vn);
      }
      blas_multidot_wide(V, N, vn, N, j + 2, part.d(), hc, nullptr, s);   // V[0..j]^H w and w^H w
      blas_gemv_sub(V, N, hc, j + 1, vn, N, s);
      blas_gmres_step(j, m, hc, col, Hd, gd, csd, snd, st, 0, s);
      blas_multidot_wide(V, N, vn, N, j + 2, part.d(), hc, &st->need2, s);   // second pass, if requested
      blas_gemv_sub(V, N, hc, j + 1, vn, N, s, &st->need2);
      blas_gmres_step(j, m, hc, col, Hd, gd, csd, snd, st, 1, s);
      blas_scale_by_state(vn, st, N, s);
      K.post_residual(j, &st->res);
      if (j >= kLag && K.residual(j - kLag) <= tol * bn) {
        ++j;
        break;
      }
    }
    chk_d(hipStreamSynchronize(s), "gmres cycle");
    GmState sh;
    chk_d(hipMemcpy(&sh, st, sizeof sh, hipMemcpyDeviceToHost), "gmres state");
    const int n = sh.nvalid;
    res.iters += n;
    if (n == 0) break;
    chk_d(hipMemcpy(Hh.data(), Hd, (size_t)(m + 1) * n * sizeof(double2), hipMemcpyDeviceToHost), "gmres H");
    chk_d(hipMemcpy(gh.data(), gd, (size_t)(n + 1) * sizeof(double2), hipMemcpyDeviceToHost), "gmres g");
    // y = R^-1 g (upper triangular), u = V y, x += P u
    std::vector<cplx> y(n);
    for (int k = n - 1; k >= 0; --k) {
      cplx sacc(gh[k].x, gh[k].y);
      for (int c = k + 1; c < n; ++c) {
        const double2 hv = Hh[(size_t)c * (m + 1) + k];
        sacc -= cplx(hv.x, hv.y) * y[c];
      }
      const double2 d = Hh[(size_t)k * (m + 1) + k];
      y[k] = sacc / cplx(d.x, d.y);
    }
    K.combine(V, n, y, n, 1, u.d());
    if (precond) {
      K.precond(u.d(), z.d());
      K.axpy(z.d(), 1.0, x);
    } else {
      K.axpy(u.d(), 1.0, x);
    }
    // explicit residual
    K.apply(aop, x, z.d());
    K.scale_copy(b, 1.0, w.d());
    K.axpy(z.d(), -1.0, w.d());
    beta = K.norm(w.d());
    res.relres = beta / bn;
    if (res.relres <= tol) {
      res.converged = true;
      break;
    }
    if (sh.stop) break;   // invariant Krylov space: x is as good as this operator allows
  }
  return res;
}

// ---------------------------------------------------------------- small dense helpers
using Mat = std::vector<cplx>;   // column-major
static inline cplx& at(Mat& A, int ld, int r, int c) { return A[(size_t)c * ld + r]; }

static void rotation(cplx x, cplx y, double& c, cplx& s) {
  double ax = std::abs(x), r = std::hypot(ax, std::abs(y));
  if (r == 0) {
    c = 1;
    s = 0;
  } else if (ax == 0) {
    c = 0;
    s = std::conj(y) / std::abs(y);
  } else {
    c = ax / r;
    s = (x / ax) * std::conj(y) / r;
  }
}

// One implicit single-shift QR step on the active window [lo, hi] of the
// upper Hessenberg A (n x n): A <- G^H A G, Z <- Z G.
static void qr_sweep(Mat& A, int n, int lo, int hi, cplx mu, Mat* Z, int nz, bool full) {
  cplx x = at(A, n, lo, lo) - mu, y = at(A, n, lo + 1, lo);
  for (int i = lo; i < hi; ++i) {
    if (i > lo) {
      x = at(A, n, i, i - 1);
      y = at(A, n, i + 1, i - 1);
    }
    double c;
    cplx s;
    rotation(x, y, c, s);
    int c0 = full ? std::max(0, i - 1) : std::max(lo, i - 1);
    int r1 = std::min(hi + 1, i + 3);
    if (full) r1 = std::min(n, i + 3);
    // left rotation on rows i, i+1 over columns c0..n-1 (or ..hi in a window)
    for (int k = c0; k < (full ? n : hi + 1); ++k) {
      cplx a = at(A, n, i, k), b = at(A, n, i + 1, k);
      at(A, n, i, k) = c * a + s * b;
      at(A, n, i + 1, k) = -std::conj(s) * a + c * b;
    }
    for (int r = (full ? 0 : lo); r < r1; ++r) {
      cplx a = at(A, n, r, i), b = at(A, n, r, i + 1);
      at(A, n, r, i) = c * a + std::conj(s) * b;
      at(A, n, r, i + 1) = -s * a + c * b;
    }
    if (i > lo) at(A, n, i + 1, i - 1) = 0;
    if (Z)
      for (int r = 0; r < nz; ++r) {
        cplx a = at(*Z, nz, r, i), b = at(*Z, nz, r, i + 1);
        at(*Z, nz, r, i) = c * a + std::conj(s) * b;
        at(*Z, nz, r, i + 1) = -s * a + c * b;
      }
  }
}

// Complex Schur form of an upper Hessenberg matrix: A = Z T Z^H (T overwrites A).
static bool schur(Mat& A, int n, Mat& Z) {
  Z.assign((size_t)n * n, cplx(0));
  for (int i = 0; i < n; ++i) at(Z, n, i, i) = 1;
  int hi = n - 1, iter = 0, total = 0;
  while (hi > 0) {
    int l = hi;
    while (l > 0) {
      double sd = std::abs(at(A, n, l, l - 1));
      double dd = std::abs(at(A, n, l - 1, l - 1)) + std::abs(at(A, n, l, l));
      if (sd <= 1e-15 * (dd > 0 ? dd : 1.0)) {
        at(A, n, l, l - 1) = 0;
        break;
      }
      --l;
    }
    if (l == hi) {
      --hi;
      iter = 0;
      continue;
    }
    cplx a = at(A, n, hi - 1, hi - 1), b = at(A, n, hi - 1, hi), c = at(A, n, hi, hi - 1), d = at(A, n, hi, hi);
    cplx tr = a + d, det = a * d - b * c;
    cplx disc = std::sqrt(tr * tr / 4.0 - det);
    cplx m1 = tr / 2.0 + disc, m2 = tr / 2.0 - disc;
    cplx mu = (std::abs(m1 - d) < std::abs(m2 - d)) ? m1 : m2;
    if (iter > 0 && iter % 12 == 0) mu = d + cplx(std::abs(at(A, n, hi, hi - 1)), 0.0);   // exceptional shift
    qr_sweep(A, n, l, hi, mu, &Z, n, true);
    ++iter;
    if (++total > 200 * n) return false;
  }
  return true;
}

// Eigenvectors of the Hessenberg matrix H from its Schur form: columns of Y.
static void schur_vectors(const Mat& T, const Mat& Z, int n, Mat& Y) {
  Y.assign((size_t)n * n, cplx(0));
  double tn = 0;
  for (auto& v : T) tn = std::max(tn, std::abs(v));
  std::vector<cplx> y(n);
  for (int i = 0; i < n; ++i) {
    std::fill(y.begin(), y.end(), cplx(0));
    y[i] = 1;
    cplx li = T[(size_t)i * n + i];
    for (int r = i - 1; r >= 0; --r) {
      cplx s = 0;
      for (int c = r + 1; c <= i; ++c) s += T[(size_t)c * n + r] * y[c];
      cplx den = T[(size_t)r * n + r] - li;
      if (std::abs(den) < 1e-14 * tn) den = 1e-14 * tn;
      y[r] = -s / den;
    }
    double nr = 0;
    for (int r = 0; r < n; ++r) {
      cplx s = 0;
      for (int c = 0; c <= i; ++c) s += Z[(size_t)c * n + r] * y[c];
      Y[(size_t)i * n + r] = s;
      nr += std::norm(s);
    }
    nr = std::sqrt(nr);
    for (int r = 0; r < n; ++r) Y[(size_t)i * n + r] /= nr;
  }
}

// Reduction of a general n x n complex matrix to upper Hessenberg form by
// Householder reflections: A <- Qh^H A Qh (A becomes Hessenberg), Qh unitary.
static void hess_reduce(Mat& A, int n, Mat& Qh) {
  Qh.assign((size_t)n * n, cplx(0));
  for (int i = 0; i < n; ++i) at(Qh, n, i, i) = 1;
  std::vector<cplx> v(n);
  for (int k = 0; k + 2 < n; ++k) {
    double nx = 0;
    for (int i = k + 1; i < n; ++i) nx += std::norm(at(A, n, i, k));
    nx = std::sqrt(nx);
    if (nx == 0) continue;
    const cplx x0 = at(A, n, k + 1, k);
    const cplx ph = std::abs(x0) > 0 ? x0 / std::abs(x0) : cplx(1);
    std::fill(v.begin(), v.end(), cplx(0));
    for (int i = k + 1; i < n; ++i) v[i] = at(A, n, i, k);
    v[k + 1] += ph * nx;
    double nv = 0;
    for (int i = k + 1; i < n; ++i) nv += std::norm(v[i]);
    nv = std::sqrt(nv);
    if (nv == 0) continue;
    for (int i = k + 1; i < n; ++i) v[i] /= nv;
    // A <- (I - 2 v v^H) A (I - 2 v v^H), Qh <- Qh (I - 2 v v^H)
    for (int c = 0; c < n; ++c) {
      cplx sacc = 0;
      for (int i = k + 1; i < n; ++i) sacc += std::conj(v[i]) * at(A, n, i, c);
      for (int i = k + 1; i < n; ++i) at(A, n, i, c) -= 2.0 * v[i] * sacc;
    }
    for (int r = 0; r < n; ++r) {
      cplx sacc = 0, sq = 0;
      for (int i = k + 1; i < n; ++i) {
        sacc += at(A, n, r, i) * v[i];
        sq += at(Qh, n, r, i) * v[i];
      }
      for (int i = k + 1; i < n; ++i) {
        at(A, n, r, i) -= 2.0 * sacc * std::conj(v[i]);
        at(Qh, n, r, i) -= 2.0 * sq * std::conj(v[i]);
      }
    }
    for (int i = k + 2; i < n; ++i) at(A, n, i, k) = 0;
  }
}

// Eigenvalues ev and unit eigenvectors (columns of Y) of a general complex
// n x n matrix: Hessenberg reduction, complex Schur form, back substitution.
static bool gen_eig(Mat A, int n, std::vector<cplx>& ev, Mat& Y) {
  Mat Qh, Z;
  hess_reduce(A, n, Qh);
  if (!schur(A, n, Z)) return false;
  Mat QZ((size_t)n * n, cplx(0));
  for (int c = 0; c < n; ++c)
    for (int r = 0; r < n; ++r) {
      cplx sacc = 0;
      for (int k = 0; k < n; ++k) sacc += at(Qh, n, r, k) * at(Z, n, k, c);
      at(QZ, n, r, c) = sacc;
    }
  schur_vectors(A, QZ, n, Y);
  ev.resize(n);
  for (int i = 0; i < n; ++i) ev[i] = at(A, n, i, i);
  return true;
}

// Orthonormal columns (standard inner product, two modified Gram-Schmidt
// passes) spanning the first nc columns of S (m rows); columns that vanish
// are dropped.  Returns the number kept.
static int orthonormal_columns(const Mat& S, int m, int nc, Mat& Qo) {
  Qo.assign((size_t)m * nc, cplx(0));
  int kept = 0;
  for (int c = 0; c < nc; ++c) {
    std::vector<cplx> v(S.begin() + (size_t)c * m, S.begin() + (size_t)(c + 1) * m);
    const double n0 = std::sqrt(std::accumulate(v.begin(), v.end(), 0.0, [](double a, cplx z) { return a + std::norm(z); }));
    for (int pass = 0; pass < 2; ++pass)
      for (int q = 0; q < kept; ++q) {
        cplx d = 0;
        for (int r = 0; r < m; ++r) d += std::conj(Qo[(size_t)q * m + r]) * v[r];
        for (int r = 0; r < m; ++r) v[r] -= d * Qo[(size_t)q * m + r];
      }
    const double nv = std::sqrt(std::accumulate(v.begin(), v.end(), 0.0, [](double a, cplx z) { return a + std::norm(z); }));
    if (!(nv > 1e-10 * n0) || nv == 0) continue;
    for (int r = 0; r < m; ++r) Qo[(size_t)kept * m + r] = v[r] / nv;
    ++kept;
  }
  return kept;
}

void KrylovCtx::cmp_ztilde(const double2* x, double2* y) {
  if (!cmp_) throw Error(CM_E_NOT_BUILT, "Calderon preconditioner not built");
  const int64_t Nr = cmp_->Nr;
  if (!r1_.p) {
    r1_.alloc((size_t)Nr * sizeof(double2));
    r2_.alloc((size_t)Nr * sizeof(double2));
  }
  blas_csr_real(cmp_->Bt, x, r1_.d(), s_);
  cm_handle* rh = cmp_->ref;
  if (far64_) {
    dev_apply(rh->dev, rh->plan, 0, r1_.p, r2_.p, 1, 1, true, s_);
  } else {
    if (!r32a_.p) {
      r32a_.alloc((size_t)Nr * sizeof(float2));
      r32b_.alloc((size_t)Nr * sizeof(float2));
    }
    blas_to_c64(r1_.d(), (float2*)r32a_.p, Nr, s_);
    dev_apply(rh->dev, rh->plan, 0, r32a_.p, r32b_.p, 1, 1, false, s_);
    blas_to_c128((const float2*)r32b_.p, r2_.d(), Nr, s_);
  }
  ++n_ref_apply;
  blas_csr_real(cmp_->B, r2_.d(), y, s_);
}

void KrylovCtx::cmp_left(const double2* u, double2* y) {
  if (!cmp_) throw Error(CM_E_NOT_BUILT, "Calderon preconditioner not built");
  if (!gk_) {
    gk_.reset(new KrylovCtx(d_, P_, true, s_));
    gk_->set_cmp(cmp_);
  }
  if (!cg_.p) cg_.alloc((size_t)N_ * sizeof(double2));
  GmresResult g = gmres(*gk_, u, cg_.d(), 60, 600, gram_tol, false, 7);
  n_gram_iters += g.iters;
  if (!g.converged) ++n_gram_fail;
  cmp_ztilde(cg_.d(), y);
}

// Solve Z x = b (aop 0) or A x = b for the other operators of gmres():
// precond 0 none, 1 the SAI (right), 2 the Calderon preconditioner (left:
// Z~ G^-1 Z x = Z~ G^-1 b, eq. (25), aop 0 only; the residual is that of
// the preconditioned system)
static GmresResult solve(KrylovCtx& K, const double2* b, double2* x, int m, int maxit, double tol, int precond,
                         int aop, DevBuf& tmp) {
  if (precond == 2) {
    if (aop != 0) throw Error(CM_E_BADARG, "the Calderon preconditioner applies to Z only");
    if (!tmp.p) tmp.alloc((size_t)K.N() * sizeof(double2));
    // Gram solves well below the outer tolerance keep the operator fixed to
    // within 1e-2 of what GMRES resolves
    K.gram_tol = std::min(1e-6, std::max(1e-13, 1e-2 * tol));
    K.cmp_left(b, tmp.d());
    return gmres(K, tmp.d(), x, m, maxit, tol, false, 6);
  }
  return gmres(K, b, x, m, maxit, tol, precond != 0, aop);
}

// ---------------------------------------------------------------- implicitly restarted Arnoldi
struct EigsResult {
  int nconv = 0, restarts = 0;
  int64_t n_op = 0, gmres_iters = 0, n_matvec = 0;
  int64_t inner_retries = 0;   // preconditioned solves that missed gm_tol, redone without P
  int64_t inner_failures = 0;  // solves that missed gm_tol either way
  std::vector<cplx> mu;       // Ritz values of OP, largest magnitude first
  std::vector<double> resid;  // Ritz residual estimates |beta e_m^T y| / |mu|
};

// aop: the matrix inverted by the inner solves, Z (0: OP = Z^-1 R, eq. (24)),
// X (2: OP = X^-1 R, eq. (14)) or tau R + i X (5: OP = (tau R + i X)^-1 R,
// whose eigenvalues mu = 1/(tau + i lambda) spread the modes with |lambda|
// near or below tau around a circle of diameter 1/tau)
static EigsResult eigs(KrylovCtx& K, int nev, int ncv, int maxrestart, double tol, const double2* v0, int gm_m,
                       int gm_maxit, double gm_tol, int precond, double2* Xout, int aop = 0) {
  const int64_t N = K.N();
  DevBuf Vb((size_t)ncv * N * sizeof(double2)), Vt((size_t)ncv * N * sizeof(double2)), f(N * sizeof(double2)),
      ru(N * sizeof(double2)), pre(0);
  double2* V = Vb.d();
  double2* Vw = Vt.d();
  EigsResult out;
  Mat H((size_t)ncv * ncv, cplx(0));
  std::vector<cplx> h;
  double nv0 = K.norm(v0);
  if (!(nv0 > 0)) throw Error(-1, "start vector is zero");
  K.scale_copy(v0, 1.0 / nv0, V);
  int j0 = 0;
  double beta = 0;
  const int kkeep = std::min(ncv - 1, nev + std::max(1, (ncv - nev) / 3));
  Mat T, Z, Y;
  std::vector<int> order;
  for (int rs = 0;; ++rs) {
    for (int j = j0; j < ncv; ++j) {
      // w = Z^-1 R v_j
      K.apply(1, V + (size_t)j * N, ru.d());
      GmresResult g = solve(K, ru.d(), f.d(), gm_m, gm_maxit, gm_tol, precond, aop, pre);
      out.gmres_iters += g.iters;
      if (!g.converged && precond == 1) {
        // the SAI can be nearly singular (e.g. the plate at low frequency,
        // where the column-wise least squares leave Z P with condition
        // number ~1e5): solve this product again without it
        ++out.inner_retries;
        g = gmres(K, ru.d(), f.d(), gm_m, gm_maxit, gm_tol, false, aop);
        out.gmres_iters += g.iters;
      }
      // an inexact OP product makes the Ritz residual estimates meaningless
      if (!g.converged) ++out.inner_failures;
      ++out.n_op;
      if (K.verbose()) {
        std::fprintf(stderr, "cm_eigs: OP product %lld: %d GMRES iterations (%lld in all)%s\n", (long long)out.n_op,
                     g.iters, (long long)out.gmres_iters, g.converged ? "" : ", missed the tolerance");
        std::fflush(stderr);
      }
      double hn = K.orth(V, j + 1, f.d(), h);
      for (int k = 0; k <= j; ++k) at(H, ncv, k, j) = h[k];
      if (j + 1 < ncv) {
        at(H, ncv, j + 1, j) = hn;
        K.scale_copy(f.d(), 1.0 / hn, V + (size_t)(j + 1) * N);
      } else {
        beta = hn;
      }
    }
    // Ritz pairs of H
    T = H;
    if (!schur(T, ncv, Z)) throw Error(-6, "Hessenberg QR did not converge");
    schur_vectors(T, Z, ncv, Y);
    order.resize(ncv);
    std::iota(order.begin(), order.end(), 0);
    std::sort(order.begin(), order.end(), [&](int a, int b) {
      return std::abs(T[(size_t)a * ncv + a]) > std::abs(T[(size_t)b * ncv + b]);
    });
    out.mu.assign(nev, 0);
    out.resid.assign(nev, 0);
    int nconv = 0;
    for (int i = 0; i < nev; ++i) {
      int c = order[i];
      cplx mu = T[(size_t)c * ncv + c];
      double r = beta * std::abs(Y[(size_t)c * ncv + ncv - 1]) / std::max(std::abs(mu), 1e-300);
      out.mu[i] = mu;
      out.resid[i] = r;
      if (r <= tol) ++nconv;
    }
    out.nconv = nconv;
    out.restarts = rs;
    if (K.verbose()) {
      std::fprintf(stderr, "cm_eigs: restart %d: %d of %d converged, %lld OP products, %lld GMRES iterations\n", rs,
                   nconv, nev, (long long)out.n_op, (long long)out.gmres_iters);
      std::fflush(stderr);
    }
    if (nconv >= nev || rs >= maxrestart) break;
    // implicit restart: the ncv - kkeep unwanted Ritz values are the shifts
    Mat Q((size_t)ncv * ncv, cplx(0));
    for (int i = 0; i < ncv; ++i) at(Q, ncv, i, i) = 1;
    for (int i = kkeep; i < ncv; ++i) {
      int c = order[i];
      qr_sweep(H, ncv, 0, ncv - 1, T[(size_t)c * ncv + c], &Q, ncv, true);
    }
    // new factorisation of length kkeep
    cplx hk = at(H, ncv, kkeep, kkeep - 1);
    cplx sig = at(Q, ncv, ncv - 1, kkeep - 1);
    K.combine(V, ncv, Q, ncv, kkeep + 1, Vw);
    // f+ = V Q e_{k} h_{k,k-1} + f sigma  (f holds the last residual, norm beta)
    DevBuf fn(N * sizeof(double2));
    K.scale_copy(Vw + (size_t)kkeep * N, hk, fn.d());
    K.axpy(f.d(), sig, fn.d());
    std::swap(V, Vw);
    double b2 = K.norm(fn.d());
    for (int c = 0; c < ncv; ++c)
      for (int r = 0; r < ncv; ++r)
        if (c >= kkeep || r >= kkeep) at(H, ncv, r, c) = 0;
    if (b2 == 0) throw Error(-6, "Arnoldi restart produced a zero residual");
    at(H, ncv, kkeep, kkeep - 1) = b2;
    K.scale_copy(fn.d(), 1.0 / b2, V + (size_t)kkeep * N);
    j0 = kkeep;
  }
  // Ritz vectors of the wanted values: X = V Y_wanted
  if (Xout) {
    Mat Yw((size_t)ncv * nev);
    for (int i = 0; i < nev; ++i)
      for (int r = 0; r < ncv; ++r) Yw[(size_t)i * ncv + r] = Y[(size_t)order[i] * ncv + r];
    K.combine(V, ncv, Yw, ncv, nev, Xout);
  }
  out.n_matvec = K.n_apply;
  return out;
}

// ---------------------------------------------------------------- Jacobi-Davidson on the pencil (X, R)
// Eigenpairs X J = lambda R J of the characteristic-mode pencil (eq. (6))
// without inverting Z or X (eqs. (28)-(29)): an R-orthonormal search space V,
// Ritz pairs of the Hermitian projection V^H X V (V^H R V = I), the Ritz value
// closest to the target selected, and the space expanded by an approximate
// solution t (a fixed number of unpreconditioned GMRES steps) of the
// projected correction equation
//   (I - R Qu Qu^H)(X - theta R)(I - Qu Qu^H R) t = -(X u - theta R u),
// with Qu = [locked eigenvectors, u], t R-orthogonal to Qu.  Converged pairs
// are locked (deflation); the space restarts from the mmin Ritz vectors
// nearest the target when it reaches mmax.  With precond the correction is
// solved right-preconditioned by i P, P the SAI of Z: for targets near 0,
// X - theta R is close to X = -i (Z - R), and the SAI approximates the
// inverse of Z's near field (t = i P y; the R-orthogonalisation of the next
// step removes its components along the locked vectors and u).  Where the
// SAI is nearly singular (the plate at low frequency) that preconditioner
// stalls the iteration: after max(50, maxit / 8) outer iterations without a
// new converged pair it is dropped for the rest of the solve.

// Eigenvalues (ascending) and eigenvectors (columns of S) of a small
// Hermitian matrix by cyclic complex Jacobi rotations.
void herm_eig(Mat A, int n, std::vector<double>& w, Mat& S) {
  S.assign((size_t)n * n, cplx(0));
  for (int i = 0; i < n; ++i) at(S, n, i, i) = 1;
  for (int sweep = 0; sweep < 100; ++sweep) {
    double off = 0, tot = 0;
    for (int c = 0; c < n; ++c)
      for (int r = 0; r < n; ++r) {
        double a2 = std::norm(at(A, n, r, c));
        tot += a2;
        if (r != c) off += a2;
      }
    if (off <= 1e-30 * std::max(tot, 1e-300)) break;
    for (int p = 0; p < n - 1; ++p)
      for (int q = p + 1; q < n; ++q) {
        cplx apq = at(A, n, p, q);
        double ab = std::abs(apq);
        if (ab == 0) continue;
        double app = at(A, n, p, p).real(), aqq = at(A, n, q, q).real();
        // rotate so that the (p, q) entry vanishes: with apq = |apq| e^{i phi},
        // G = [[c, -s e^{i phi}], [s e^{-i phi}, c]] applied as A <- G^H A G
        cplx ph = apq / ab;
        double tau = (aqq - app) / (2 * ab);
        double t = (tau >= 0 ? 1.0 : -1.0) / (std::abs(tau) + std::sqrt(1 + tau * tau));
        double c = 1 / std::sqrt(1 + t * t), sn = t * c;
        for (int k = 0; k < n; ++k) {   // columns p, q of A and S
          cplx akp = at(A, n, k, p), akq = at(A, n, k, q);
          at(A, n, k, p) = c * akp - sn * std::conj(ph) * akq;
          at(A, n, k, q) = sn * ph * akp + c * akq;
          cplx skp = at(S, n, k, p), skq = at(S, n, k, q);
          at(S, n, k, p) = c * skp - sn * std::conj(ph) * skq;
          at(S, n, k, q) = sn * ph * skp + c * skq;
        }
        for (int k = 0; k < n; ++k) {   // rows p, q of A
          cplx apk = at(A, n, p, k), aqk = at(A, n, q, k);
          at(A, n, p, k) = c * apk - sn * ph * aqk;
          at(A, n, q, k) = sn * std::conj(ph) * apk + c * aqk;
        }
        at(A, n, p, q) = at(A, n, q, p) = 0;
      }
  }
  std::vector<int> ord(n);
  std::iota(ord.begin(), ord.end(), 0);
  std::sort(ord.begin(), ord.end(), [&](int a, int b) { return at(A, n, a, a).real() < at(A, n, b, b).real(); });
  Mat S2((size_t)n * n);
  w.resize(n);
  for (int c = 0; c < n; ++c) {
    w[c] = at(A, n, ord[c], ord[c]).real();
    for (int r = 0; r < n; ++r) at(S2, n, r, c) = at(S, n, r, ord[c]);
  }
  S.swap(S2);
}

struct JdResult {
  std::vector<double> lam, resid;
  int nconv = 0, outer = 0, precond_dropped = 0;
  int64_t inner_steps = 0, n_apply = 0;
};

// precond: 0 none, 1 i P with P the SAI of Z_near, 2 P the SAI of X_near
// (the context's SAI slot).  harmonic: select harmonic Ritz pairs for the
// target instead of Ritz pairs (interior eigenvalues, see below).
static JdResult jd(KrylovCtx& K, int nev, double target, int mmin, int mmax, int maxit, double tol, int inner,
                   const double2* v0, double2* Jout, int precond, bool harmonic) {
  const int64_t N = K.N();
  hipStream_t s = K.stream();
  DevBuf Vb((size_t)mmax * N * sizeof(double2)), XVb((size_t)mmax * N * sizeof(double2)),
      RVb((size_t)mmax * N * sizeof(double2)), Tmp((size_t)mmax * N * sizeof(double2)),
      Qb((size_t)(nev + 1) * N * sizeof(double2)), RQb((size_t)(nev + 1) * N * sizeof(double2)),
      t(N * sizeof(double2)), Rt(N * sizeof(double2)), Xt(N * sizeof(double2)), r(N * sizeof(double2)),
      Xu(N * sizeof(double2)), y(N * sizeof(double2)), Ry(N * sizeof(double2)), py(N * sizeof(double2)),
      Gb((size_t)(inner + 1) * N * sizeof(double2)), hd(1024 * sizeof(double2));
  double2 *V = Vb.d(), *XV = XVb.d(), *RV = RVb.d(), *Q = Qb.d(), *RQ = RQb.d();
  JdResult out;
  std::vector<double2> hh(1024);
  auto dots = [&](const double2* A, int nk, const double2* w) {   // A^H w, nk <= 1024, on the host
    K.multidot(A, nk, w, hd.d());
    chk_d(hipMemcpyAsync(hh.data(), hd.p, nk * sizeof(double2), hipMemcpyDeviceToHost, s), "jd dots");
    chk_d(hipStreamSynchronize(s), "jd dots");
  };
  // w -= B (A^H w) for the nk columns of A, B
  auto project = [&](const double2* A, const double2* B, int nk, double2* w) {
    if (nk == 0) return;
    K.multidot(A, nk, w, hd.d());
    blas_gemv_sub(B, N, hd.d(), nk, w, N, s);
  };
  auto copy = [&](const double2* x, double2* z, size_t n) {
    chk_d(hipMemcpyAsync(z, x, n * sizeof(double2), hipMemcpyDeviceToDevice, s), "jd copy");
  };
  // basis restart / deflation: M <- M S[:, c0 .. c0 + nc)
  auto recombine = [&](double2* M, int m, const Mat& S, int c0, int nc) {
    Mat Sc((size_t)m * nc);
    for (int c = 0; c < nc; ++c)
      for (int r2 = 0; r2 < m; ++r2) Sc[(size_t)c * m + r2] = S[(size_t)(c0 + c) * m + r2];
    K.combine(M, m, Sc, m, nc, Tmp.d());
    copy(Tmp.d(), M, (size_t)nc * N);
  };
  // basis change V <- V Qm (nc orthonormal columns of m rows: the new basis
  // stays R-orthonormal), with X V, R V and H = V^H X V following
  auto change_basis = [&](const Mat& Qm, int nc, Mat& Hm, int m) {
    recombine(V, m, Qm, 0, nc);
    recombine(XV, m, Qm, 0, nc);
    recombine(RV, m, Qm, 0, nc);
    Mat HQ((size_t)m * nc, cplx(0)), Hn((size_t)nc * nc, cplx(0));
    for (int c = 0; c < nc; ++c)
      for (int r2 = 0; r2 < m; ++r2) {
        cplx acc = 0;
        for (int q = 0; q < m; ++q) acc += at(Hm, m, r2, q) * Qm[(size_t)c * m + q];
        HQ[(size_t)c * m + r2] = acc;
      }
    for (int c = 0; c < nc; ++c)
      for (int r2 = 0; r2 < nc; ++r2) {
        cplx acc = 0;
        for (int q = 0; q < m; ++q) acc += std::conj(Qm[(size_t)r2 * m + q]) * HQ[(size_t)c * m + q];
        at(Hn, nc, r2, c) = acc;
      }
    for (int c = 0; c < nc; ++c) {   // Hermitian up to rounding
      at(Hn, nc, c, c) = at(Hn, nc, c, c).real();
      for (int r2 = c + 1; r2 < nc; ++r2) at(Hn, nc, r2, c) = std::conj(at(Hn, nc, c, r2));
    }
    Hm.swap(Hn);
  };
  // Harmonic Ritz pairs for the target tau: W = X V - tau R V, W^H (X - theta
  // R) V s = 0, i.e. (W^H W) s = nu (W^H R V) s with theta = tau + nu; the
  // pairs of smallest |nu| are the harmonic approximations closest to tau
  // (extreme eigenvalues of (W^H W)^-1 W^H R V), which unlike Ritz values do
  // not wander where the target lies inside a dense part of the spectrum.
  // S receives the vectors (unit norm, ordered by |nu|), w their Rayleigh
  // quotients s^H H s (the eigenvalue estimates and correction shifts).
  auto harmonic_pairs = [&](int m, const Mat& Hm, Mat& Sout, std::vector<double>& wout) {
    for (int c = 0; c < m; ++c) {
      copy(XV + (size_t)c * N, Tmp.d() + (size_t)c * N, N);
      K.axpy(RV + (size_t)c * N, -target, Tmp.d() + (size_t)c * N);
    }
    Mat A((size_t)m * m), B((size_t)m * m);
    for (int c = 0; c < m; ++c) {
      dots(Tmp.d(), m, Tmp.d() + (size_t)c * N);
      for (int r2 = 0; r2 < m; ++r2) at(A, m, r2, c) = cplx(hh[r2].x, hh[r2].y);
      dots(Tmp.d(), m, RV + (size_t)c * N);
      for (int r2 = 0; r2 < m; ++r2) at(B, m, r2, c) = cplx(hh[r2].x, hh[r2].y);
    }
    // A = L L^H (a tiny diagonal shift keeps it definite when W loses rank)
    double tr = 0;
    for (int c = 0; c < m; ++c) tr += at(A, m, c, c).real();
    Mat L((size_t)m * m, cplx(0));
    for (int c = 0; c < m; ++c) {
      cplx d = at(A, m, c, c) + 1e-14 * tr / m;
      for (int q = 0; q < c; ++q) d -= at(L, m, c, q) * std::conj(at(L, m, c, q));
      const double ld = std::sqrt(std::max(d.real(), 1e-300));
      at(L, m, c, c) = ld;
      for (int r2 = c + 1; r2 < m; ++r2) {
        cplx acc = at(A, m, r2, c);
        for (int q = 0; q < c; ++q) acc -= at(L, m, r2, q) * std::conj(at(L, m, c, q));
        at(L, m, r2, c) = acc / ld;
      }
    }
    // C = L^-1 B L^-H
    auto lsolve = [&](std::vector<cplx>& x) {   // x <- L^-1 x
      for (int r2 = 0; r2 < m; ++r2) {
        cplx acc = x[r2];
        for (int q = 0; q < r2; ++q) acc -= at(L, m, r2, q) * x[q];
        x[r2] = acc / at(L, m, r2, r2);
      }
    };
    auto lhsolve = [&](std::vector<cplx>& x) {   // x <- L^-H x
      for (int r2 = m - 1; r2 >= 0; --r2) {
        cplx acc = x[r2];
        for (int q = r2 + 1; q < m; ++q) acc -= std::conj(at(L, m, q, r2)) * x[q];
        x[r2] = acc / at(L, m, r2, r2);
      }
    };
    Mat Cm((size_t)m * m);
    {
      Mat T1((size_t)m * m);   // L^-1 B
      std::vector<cplx> col(m);
      for (int c = 0; c < m; ++c) {
        for (int r2 = 0; r2 < m; ++r2) col[r2] = at(B, m, r2, c);
        lsolve(col);
        for (int r2 = 0; r2 < m; ++r2) at(T1, m, r2, c) = col[r2];
      }
      // (L^-1 B) L^-H = (L^-1 (L^-1 B)^H)^H
      for (int r2 = 0; r2 < m; ++r2) {
        for (int c = 0; c < m; ++c) col[c] = std::conj(at(T1, m, r2, c));
        lsolve(col);
        for (int c = 0; c < m; ++c) at(Cm, m, r2, c) = std::conj(col[c]);
      }
    }
    std::vector<cplx> ev;
    Mat Y;
    if (!gen_eig(Cm, m, ev, Y)) throw Error(-6, "Jacobi-Davidson: harmonic eigenproblem did not converge");
    std::vector<int> ord(m);
    std::iota(ord.begin(), ord.end(), 0);
    std::stable_sort(ord.begin(), ord.end(), [&](int a, int b) { return std::abs(ev[a]) > std::abs(ev[b]); });
    Sout.assign((size_t)m * m, cplx(0));
    wout.assign(m, 0.0);
    std::vector<cplx> sv(m);
    for (int c = 0; c < m; ++c) {
      for (int r2 = 0; r2 < m; ++r2) sv[r2] = at(Y, m, r2, ord[c]);
      lhsolve(sv);
      double nrm = 0;
      for (auto& z : sv) nrm += std::norm(z);
      nrm = std::sqrt(std::max(nrm, 1e-300));
      cplx rq = 0;
      for (int r2 = 0; r2 < m; ++r2) {
        sv[r2] /= nrm;
        Sout[(size_t)c * m + r2] = sv[r2];
      }
      for (int r2 = 0; r2 < m; ++r2)
        for (int q = 0; q < m; ++q) rq += std::conj(sv[r2]) * Hm[(size_t)q * m + r2] * sv[q];
      wout[c] = rq.real();
    }
  };
  copy(v0, t.d(), N);
  int k = 0, m = 0, since_lock = 0;
  const int stall = std::max(50, maxit / 8);
  Mat H;   // m x m, V^H X V
  std::vector<double> w;
  Mat S;
  while (out.outer < maxit) {
    ++out.outer;
    // R-orthonormalise t against the locked vectors and V (two passes)
    for (int pass = 0; pass < 2; ++pass) {
      project(RQ, Q, k, t.d());
      project(RV, V, m, t.d());
    }
    K.apply(1, t.d(), Rt.d());
    dots(t.d(), 1, Rt.d());
    double nr = std::sqrt(std::max(hh[0].x, 0.0));
    if (!(nr > 1e-300)) throw Error(-6, "Jacobi-Davidson: expansion vector has no R-norm");
    K.scale_copy(t.d(), 1.0 / nr, V + (size_t)m * N);
    K.scale_copy(Rt.d(), 1.0 / nr, RV + (size_t)m * N);
    K.apply(2, V + (size_t)m * N, XV + (size_t)m * N);
    dots(V, m + 1, XV + (size_t)m * N);
    Mat Hn((size_t)(m + 1) * (m + 1), cplx(0));
    for (int c = 0; c < m; ++c)
      for (int r2 = 0; r2 < m; ++r2) at(Hn, m + 1, r2, c) = at(H, m, r2, c);
    for (int r2 = 0; r2 <= m; ++r2) {
      cplx v(hh[r2].x, hh[r2].y);
      at(Hn, m + 1, r2, m) = v;
      at(Hn, m + 1, m, r2) = std::conj(v);
    }
    at(Hn, m + 1, m, m) = at(Hn, m + 1, m, m).real();
    H.swap(Hn);
    ++m;
    double theta = 0;
    bool expand = false;
    while (m > 0) {
      if (harmonic) {
        harmonic_pairs(m, H, S, w);
      } else {
        herm_eig(H, m, w, S);
        // order by distance to the target
        std::vector<int> ord(m);
        std::iota(ord.begin(), ord.end(), 0);
        std::stable_sort(ord.begin(), ord.end(),
                         [&](int a, int b) { return std::abs(w[a] - target) < std::abs(w[b] - target); });
        Mat So((size_t)m * m);
        std::vector<double> wo(m);
        for (int c = 0; c < m; ++c) {
          wo[c] = w[ord[c]];
          for (int r2 = 0; r2 < m; ++r2) So[(size_t)c * m + r2] = S[(size_t)ord[c] * m + r2];
        }
        S.swap(So);
        w.swap(wo);
      }
      theta = w[0];
      // u (into the locked block's next column), R u, X u, r = X u - theta R u
      Mat s0(S.begin(), S.begin() + m);
      K.combine(V, m, s0, m, 1, Q + (size_t)k * N);
      K.combine(RV, m, s0, m, 1, RQ + (size_t)k * N);
      K.combine(XV, m, s0, m, 1, Xu.d());
      copy(Xu.d(), r.d(), N);
      K.axpy(RQ + (size_t)k * N, -theta, r.d());
      double rn = K.norm(r.d()) / std::max(K.norm(RQ + (size_t)k * N), 1e-300);
      if (rn <= tol * std::max(1.0, std::abs(theta))) {
        out.lam.push_back(theta);
        out.resid.push_back(rn);
        ++k;
        if (K.verbose()) {
          std::fprintf(stderr, "cm_jd: %d of %d converged (lambda %.9g) after %d outer iterations\n", k, nev, theta,
                       out.outer);
          std::fflush(stderr);
        }
        since_lock = 0;
        if (k == nev) break;
        // deflate: the rest of the (harmonic) Ritz vectors stay, as an
        // orthonormal basis of the complement of the locked one
        if (harmonic) {
          Mat Qo;
          const int kept = orthonormal_columns(S, m, m, Qo);   // S[:, 0] first: drop it after
          Mat Qr(Qo.begin() + (size_t)m, Qo.begin() + (size_t)kept * m);
          change_basis(Qr, kept - 1, H, m);
          m = kept - 1;
        } else {
          recombine(V, m, S, 1, m - 1);
          recombine(XV, m, S, 1, m - 1);
          recombine(RV, m, S, 1, m - 1);
          --m;
          H.assign((size_t)m * m, cplx(0));
          for (int c = 0; c < m; ++c) at(H, m, c, c) = w[c + 1];
        }
        continue;
      }
      expand = true;
      break;
    }
    if (k == nev) break;
    if (precond && ++since_lock > stall) {
      precond = 0;
      out.precond_dropped = 1;
    }
    if (!expand) {   // every Ritz vector locked: expand from the start vector again
      copy(v0, t.d(), N);
      continue;
    }
    if (m >= mmax) {
      const int keep = std::min(mmin, m);
      if (harmonic) {
        Mat Qo;
        const int kept = orthonormal_columns(S, m, keep, Qo);
        change_basis(Qo, kept, H, m);
        m = kept;
      } else {
        recombine(V, m, S, 0, keep);
        recombine(XV, m, S, 0, keep);
        recombine(RV, m, S, 0, keep);
        m = keep;
        H.assign((size_t)m * m, cplx(0));
        for (int c = 0; c < m; ++c) at(H, m, c, c) = w[c];
      }
    }
    // correction equation, fixed number of GMRES steps from t = 0, rhs -r
    const int kq = k + 1;   // Qu = Q[:, 0..k], R Qu = RQ[:, 0..k]
    auto op = [&](const double2* x, double2* z) {
      if (precond == 1) {
        K.precond(x, py.d());
        K.scale_copy(py.d(), cplx(0, 1), y.d());   // y = i P x
      } else if (precond == 2) {
        K.precond(x, y.d());                       // y = P x, P the SAI of X_near
      } else {
        copy(x, y.d(), N);
      }
      project(RQ, Q, kq, y.d());          // y = (I - Qu Qu^H R) y
      K.apply(1, y.d(), Ry.d());
      K.apply(2, y.d(), z);
      K.axpy(Ry.d(), -theta, z);           // z = (X - theta R) y
      project(Q, RQ, kq, z);              // z = (I - R Qu Qu^H) z
    };
    double2* G = Gb.d();
    const double bn = K.norm(r.d());
    K.scale_copy(r.d(), -1.0 / bn, G);
    std::vector<cplx> Hg((size_t)(inner + 1) * inner, cplx(0)), g(inner + 1, cplx(0)), cs(inner), sn(inner), h;
    g[0] = bn;
    int nst = 0;
    for (int j = 0; j < inner; ++j) {
      double2* gn = G + (size_t)(j + 1) * N;   // the new vector is built in its slot
      op(G + (size_t)j * N, gn);
      double hn = K.orth_next(G, j + 1, h);
      cplx* col = &Hg[(size_t)j * (inner + 1)];
      for (int q = 0; q <= j; ++q) col[q] = h[q];
      col[j + 1] = hn;
      if (hn > 0) blas_scale(gn, make_double2(1.0 / hn, 0.0), N, s);
      for (int q = 0; q < j; ++q) {
        cplx a = col[q], b = col[q + 1];
        col[q] = std::conj(cs[q]) * a + std::conj(sn[q]) * b;
        col[q + 1] = -sn[q] * a + cs[q] * b;
      }
      double rr = std::hypot(std::abs(col[j]), std::abs(col[j + 1]));
      cs[j] = rr == 0 ? cplx(1) : col[j] / rr;
      sn[j] = rr == 0 ? cplx(0) : col[j + 1] / rr;
      col[j] = rr;
      col[j + 1] = 0;
      g[j + 1] = -sn[j] * g[j];
      g[j] = std::conj(cs[j]) * g[j];
      nst = j + 1;
      if (hn == 0) break;
    }
    out.inner_steps += nst;
    std::vector<cplx> yv(nst);
    for (int q = nst - 1; q >= 0; --q) {
      cplx acc = g[q];
      for (int c = q + 1; c < nst; ++c) acc -= Hg[(size_t)c * (inner + 1) + q] * yv[c];
      yv[q] = acc / Hg[(size_t)q * (inner + 1) + q];
    }
    K.combine(G, nst, yv, nst, 1, t.d());
    if (precond == 1) {
      K.precond(t.d(), py.d());
      K.scale_copy(py.d(), cplx(0, 1), t.d());
    } else if (precond == 2) {
      K.precond(t.d(), py.d());
      copy(py.d(), t.d(), N);
    }
  }
  out.nconv = k;
  if (Jout && k > 0) copy(Q, Jout, (size_t)k * N);
  out.n_apply = K.n_apply;
  chk_d(hipStreamSynchronize(s), "jd");
  return out;
}

}  // namespace cm

// ---------------------------------------------------------------- C ABI entry points
namespace cm {
cm_status driver_fail(int code, const std::string& msg);
}

extern "C" cm_status cm_gmres(cm_handle* h, const void* b, void* x, int32_t restart, int32_t maxit, double tol,
                              int32_t precond, cm_dtype far_dtype, int32_t* iters, double* relres,
                              void* hip_stream) {
  if (!h || !b || !x) return cm::driver_fail(CM_E_BADARG, "null argument");
  if (!h->has_dev) return cm::driver_fail(CM_E_NOT_BUILT, "handle was built host-only");
  if (restart < 1 || restart > 1000 || maxit < 1 || !(tol > 0)) return cm::driver_fail(CM_E_BADARG, "bad GMRES parameters");
  if (precond < 0 || precond > 2) return cm::driver_fail(CM_E_BADARG, "precond must be 0, 1 or 2");
  if (precond == 1 && !h->dev.sai[0].val) return cm::driver_fail(CM_E_NOT_BUILT, "SAI preconditioner not built");
  if (precond == 2 && !h->cmp) return cm::driver_fail(CM_E_NOT_BUILT, "Calderon preconditioner not built");
  if (b == x) return cm::driver_fail(CM_E_BADARG, "b and x must not alias");
  try {
    cm::KrylovCtx K(h->dev, h->plan, far_dtype == CM_C128, (hipStream_t)hip_stream);
    K.set_cmp(h->cmp);
    cm::DevBuf tmp(0);
    cm::GmresResult r = cm::solve(K, (const double2*)b, (double2*)x, restart, maxit, tol, precond, 0, tmp);
    if (iters) *iters = r.iters;
    if (relres) *relres = r.relres;
    return r.converged ? CM_OK : CM_E_NOT_CONVERGED;
  } catch (const cm::Error& e) {
    return cm::driver_fail(e.code, e.what());
  } catch (const std::exception& e) {
    return cm::driver_fail(CM_E_OOM, e.what());
  }
}

extern "C" cm_status cm_jd(cm_handle* h, int32_t nev, double target, int32_t mmin, int32_t mmax, int32_t maxit,
                           double tol, int32_t inner_steps, int32_t precond, int32_t harmonic, const void* v0,
                           cm_dtype far_dtype, double* lambda,
                           double* resid, void* J, int32_t* nconv, int64_t* counters, void* hip_stream) {
  if (!h || !v0 || !lambda) return cm::driver_fail(CM_E_BADARG, "null argument");
  if (!h->has_dev) return cm::driver_fail(CM_E_NOT_BUILT, "handle was built host-only");
  if (nev < 1 || nev > 512 || mmin < 1 || mmax < mmin + 1 || mmax > 512 || mmax > h->dev.N || maxit < 1 ||
      !(tol > 0) || inner_steps < 1 || inner_steps > 512 || !std::isfinite(target))
    return cm::driver_fail(CM_E_BADARG,
                           "bad Jacobi-Davidson parameters (need 1 <= nev <= 512, 1 <= mmin < mmax <= min(N, 512), "
                           "maxit >= 1, tol > 0, 1 <= inner_steps <= 512)");
  if (precond < 0 || precond > 2) return cm::driver_fail(CM_E_BADARG, "precond must be 0, 1 or 2");
  if (precond == 1 && !h->dev.sai[0].val) return cm::driver_fail(CM_E_NOT_BUILT, "SAI of Z_near not built");
  if (precond == 2 && (!h->dev.sai[1].val || h->dev.sai_tau1 != 0.0))
    return cm::driver_fail(CM_E_NOT_BUILT, "SAI of X_near (tau 0) not built");
  try {
    cm::KrylovCtx K(h->dev, h->plan, far_dtype == CM_C128, (hipStream_t)hip_stream, precond == 2 ? 1 : 0);
    cm::JdResult r = cm::jd(K, nev, target, mmin, mmax, maxit, tol, inner_steps, (const double2*)v0, (double2*)J,
                            precond, harmonic != 0);
    for (int i = 0; i < nev; ++i) {
      lambda[i] = i < r.nconv ? r.lam[i] : 0.0;
      if (resid) resid[i] = i < r.nconv ? r.resid[i] : 0.0;
    }
    if (nconv) *nconv = r.nconv;
    if (counters) {
      counters[0] = r.outer;
      counters[1] = r.inner_steps;
      counters[2] = r.n_apply;
      counters[3] = r.precond_dropped;
    }
    return r.nconv >= nev ? CM_OK : CM_E_NOT_CONVERGED;
  } catch (const cm::Error& e) {
    return cm::driver_fail(e.code, e.what());
  } catch (const std::exception& e) {
    return cm::driver_fail(CM_E_OOM, e.what());
  }
}

extern "C" cm_status cm_eigs(cm_handle* h, int32_t nev, int32_t ncv, int32_t maxrestart, double tol, const void* v0,
                             int32_t gmres_restart, int32_t gmres_maxit, double gmres_tol, int32_t precond,
                             double tau, cm_dtype far_dtype, double* lambda, double* ritz_resid, void* J,
                             int32_t* nconv, int64_t* counters, void* hip_stream) {
  if (!h || !v0 || !lambda) return cm::driver_fail(CM_E_BADARG, "null argument");
  if (!h->has_dev) return cm::driver_fail(CM_E_NOT_BUILT, "handle was built host-only");
  if (nev < 1 || ncv <= nev || ncv > 1000 || ncv > h->dev.N || maxrestart < 0 || !(tol > 0))
    return cm::driver_fail(CM_E_BADARG, "bad eigensolver parameters (need 1 <= nev < ncv <= min(N, 1000))");
  if (gmres_restart < 1 || gmres_restart > 1000 || gmres_maxit < 1 || !(gmres_tol > 0))
    return cm::driver_fail(CM_E_BADARG, "bad GMRES parameters (need 1 <= gmres_restart <= 1000)");
  if (!(tau > 0) || !(tau <= 1e6)) return cm::driver_fail(CM_E_BADARG, "tau must be in (0, 1e6]");
  if (precond < 0 || precond > 2) return cm::driver_fail(CM_E_BADARG, "precond must be 0, 1 or 2");
  const int slot = cm::sai_slot(tau);
  if (precond == 1 && (!h->dev.sai[slot].val || (slot == 1 && h->dev.sai_tau1 != tau)))
    return cm::driver_fail(CM_E_NOT_BUILT, "SAI preconditioner not built for this tau");
  if (precond == 2 && (!h->cmp || tau != 1.0))
    return cm::driver_fail(h->cmp ? CM_E_BADARG : CM_E_NOT_BUILT,
                           "the Calderon preconditioner needs cm_cmp_build and tau = 1");
  try {
    cm::KrylovCtx K(h->dev, h->plan, far_dtype == CM_C128, (hipStream_t)hip_stream, slot, tau);
    K.set_cmp(h->cmp);
    cm::EigsResult r = cm::eigs(K, nev, ncv, maxrestart, tol, (const double2*)v0, gmres_restart, gmres_maxit,
                                gmres_tol, precond, (double2*)J, tau == 1.0 ? 0 : 5);
    for (int i = 0; i < nev; ++i) {
      // (tau R + i X) J = (tau + i lambda) R J:  lambda = i (tau - 1/mu)
      cm::cplx lam = cm::cplx(0, 1) * (tau - 1.0 / r.mu[i]);
      lambda[2 * i] = lam.real();
      lambda[2 * i + 1] = lam.imag();
      if (ritz_resid) ritz_resid[i] = r.resid[i];
    }
    if (nconv) *nconv = r.nconv;
    if (counters) {
      counters[0] = r.n_op;
      counters[1] = r.gmres_iters;
      counters[2] = r.n_matvec;
      counters[3] = r.restarts;
      counters[4] = r.inner_retries;
      counters[5] = r.inner_failures;
    }
    return (r.nconv >= nev && r.inner_failures == 0) ? CM_OK : CM_E_NOT_CONVERGED;
  } catch (const cm::Error& e) {
    return cm::driver_fail(e.code, e.what());
  } catch (const std::exception& e) {
    return cm::driver_fail(CM_E_OOM, e.what());
  }
}

extern "C" cm_status cm_eigs_xinv(cm_handle* h, int32_t nev, int32_t ncv, int32_t maxrestart, double tol,
                                  const void* v0, int32_t gmres_restart, int32_t gmres_maxit, double gmres_tol,
                                  int32_t precond, cm_dtype far_dtype, double* lambda, double* ritz_resid, void* J,
                                  int32_t* nconv, int64_t* counters, void* hip_stream) {
  if (!h || !v0 || !lambda) return cm::driver_fail(CM_E_BADARG, "null argument");
  if (!h->has_dev) return cm::driver_fail(CM_E_NOT_BUILT, "handle was built host-only");
  if (nev < 1 || ncv <= nev || ncv > 1000 || ncv > h->dev.N || maxrestart < 0 || !(tol > 0))
    return cm::driver_fail(CM_E_BADARG, "bad eigensolver parameters (need 1 <= nev < ncv <= min(N, 1000))");
  if (gmres_restart < 1 || gmres_restart > 1000 || gmres_maxit < 1 || !(gmres_tol > 0))
    return cm::driver_fail(CM_E_BADARG, "bad GMRES parameters (need 1 <= gmres_restart <= 1000)");
  if (precond && (!h->dev.sai[1].val || h->dev.sai_tau1 != 0.0))
    return cm::driver_fail(CM_E_NOT_BUILT, "SAI of X_near (tau 0) not built");
  try {
    cm::KrylovCtx K(h->dev, h->plan, far_dtype == CM_C128, (hipStream_t)hip_stream, 1);
    cm::EigsResult r = cm::eigs(K, nev, ncv, maxrestart, tol, (const double2*)v0, gmres_restart, gmres_maxit,
                                gmres_tol, precond != 0 ? 1 : 0, (double2*)J, 2);
    for (int i = 0; i < nev; ++i) {
      // X^-1 R J = mu J  <=>  X J = (1 / mu) R J
      cm::cplx lam = 1.0 / r.mu[i];
      lambda[2 * i] = lam.real();
      lambda[2 * i + 1] = lam.imag();
      if (ritz_resid) ritz_resid[i] = r.resid[i];
    }
    if (nconv) *nconv = r.nconv;
    if (counters) {
      counters[0] = r.n_op;
      counters[1] = r.gmres_iters;
      counters[2] = r.n_matvec;
      counters[3] = r.restarts;
      counters[4] = r.inner_retries;
      counters[5] = r.inner_failures;
    }
    return (r.nconv >= nev && r.inner_failures == 0) ? CM_OK : CM_E_NOT_CONVERGED;
  } catch (const cm::Error& e) {
    return cm::driver_fail(e.code, e.what());
  } catch (const std::exception& e) {
    return cm::driver_fail(CM_E_OOM, e.what());
  }
}

extern "C" cm_status cm_cmp_apply(cm_handle* h, int32_t which, const void* x, void* y, cm_dtype far_dtype,
                                  void* hip_stream) {
  if (!h || !x || !y) return cm::driver_fail(CM_E_BADARG, "null argument");
  if (!h->has_dev) return cm::driver_fail(CM_E_NOT_BUILT, "handle was built host-only");
  if (!h->cmp) return cm::driver_fail(CM_E_NOT_BUILT, "Calderon preconditioner not built");
  if (which < 0 || which > 2) return cm::driver_fail(CM_E_BADARG, "which must be 0 (Z~), 1 (G) or 2 (Z~ G^-1 Z)");
  if (far_dtype != CM_C128 && far_dtype != CM_C64) return cm::driver_fail(CM_E_BADARG, "bad far-field dtype");
  if (x == y) return cm::driver_fail(CM_E_BADARG, "x and y must not alias");
  try {
    cm::KrylovCtx K(h->dev, h->plan, far_dtype == CM_C128, (hipStream_t)hip_stream);
    K.set_cmp(h->cmp);
    if (which == 0) K.cmp_ztilde((const double2*)x, (double2*)y);
    if (which == 1) K.apply(7, (const double2*)x, (double2*)y);
    if (which == 2) K.apply(6, (const double2*)x, (double2*)y);
    if (hipStreamSynchronize((hipStream_t)hip_stream) != hipSuccess)
      return cm::driver_fail(CM_E_HIP, "cm_cmp_apply: stream synchronisation");
    if (K.n_gram_fail) return cm::driver_fail(CM_E_NOT_CONVERGED, "the Gram solve missed its tolerance");
    return CM_OK;
  } catch (const cm::Error& e) {
    return cm::driver_fail(e.code, e.what());
  } catch (const std::exception& e) {
    return cm::driver_fail(CM_E_OOM, e.what());
  }
}
