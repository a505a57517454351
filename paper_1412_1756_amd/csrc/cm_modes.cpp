// Characteristic-mode post-processing on the device (section V): real
// R-normalised currents, the modal correlation used to follow modes over a
// frequency sweep, and d lambda/dk of a mode or a degenerate cluster from the
// dZ/dk pass.  Every N-vector operation is a device kernel; only the small
// (cluster-size) projected matrices are diagonalised on the host.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <complex>
#include <string>
#include <vector>

#include "cm_device.h"

namespace cm {

cm_status driver_fail(int code, const std::string& msg);
void herm_eig(std::vector<cplx> A, int n, std::vector<double>& w, std::vector<cplx>& S);
int blas_gram_blocks(int64_t N);
void blas_gram(const double2* A, int64_t lda, int na, const double2* B, int64_t ldb, int nb, int64_t N, bool conjA,
               double2* part, double2* out, hipStream_t s);
void blas_phase_real(const double2* J, int64_t ldj, int m, const double2* ph, double2* W, int64_t ldw, int64_t N,
                     hipStream_t s);
void blas_split_reim(const double2* J, int64_t ldj, int m, double2* W, int64_t ldw, int64_t N, hipStream_t s);
void blas_rowmix(const double2* A, int64_t lda, int na, const double2* M, int nb, double2* Out, int64_t ldo,
                 int64_t N, hipStream_t s);
void blas_scale_cols(double2* A, int64_t lda, int m, const double* sc, int64_t N, hipStream_t s);

namespace {

void ck(hipError_t e, const char* what) {
  if (e != hipSuccess) {
    if (e == hipErrorOutOfMemory) throw Error(CM_E_OOM, std::string(what) + ": out of device memory");
    throw Error(CM_E_HIP, std::string(what) + ": " + hipGetErrorString(e));
  }
}

struct Buf {
  void* p = nullptr;
  explicit Buf(size_t bytes) { ck(hipMalloc(&p, std::max<size_t>(bytes, 16)), "mode post-processing workspace"); }
  ~Buf() {
    if (p) (void)hipFree(p);
  }
  Buf(const Buf&) = delete;
  Buf& operator=(const Buf&) = delete;
  double2* d() const { return (double2*)p; }
};

// y = op(x) for m complex128 columns (row stride ld), in batches of at most
// the handle's max_cols columns
void apply_cols(cm_handle* h, int op, const double2* x, double2* y, int64_t ld, int m, hipStream_t s) {
  const int mc = h->dev.max_cols;
  for (int c0 = 0; c0 < m; c0 += mc) dev_apply(h->dev, h->plan, op, x + c0, y + c0, ld, std::min(mc, m - c0), true, s);
}

// host copy of the Gram product A^H B (conjA) or A^T B of row-major blocks
std::vector<cplx> gram_host(const double2* A, int64_t lda, int na, const double2* B, int64_t ldb, int nb, int64_t N,
                            bool conjA, hipStream_t s) {
  Buf part((size_t)blas_gram_blocks(N) * na * nb * sizeof(double2)), out((size_t)na * nb * sizeof(double2));
  blas_gram(A, lda, na, B, ldb, nb, N, conjA, part.d(), out.d(), s);
  std::vector<double2> h((size_t)na * nb);
  ck(hipMemcpyAsync(h.data(), out.p, h.size() * sizeof(double2), hipMemcpyDeviceToHost, s), "gram copy");
  ck(hipStreamSynchronize(s), "gram");
  std::vector<cplx> r(h.size());
  for (size_t i = 0; i < h.size(); ++i) r[i] = cplx(h[i].x, h[i].y);
  return r;
}

// per-column sums sum_i op(A[i, c]) B[i, c], c < m
std::vector<cplx> coldots(const double2* A, int64_t lda, const double2* B, int64_t ldb, int m, int64_t N, bool conjA,
                          hipStream_t s) {
  Buf part((size_t)blas_gram_blocks(N) * sizeof(double2)), out((size_t)m * sizeof(double2));
  for (int c = 0; c < m; ++c) blas_gram(A + c, lda, 1, B + c, ldb, 1, N, conjA, part.d(), out.d() + c, s);
  std::vector<double2> h(m);
  ck(hipMemcpyAsync(h.data(), out.p, m * sizeof(double2), hipMemcpyDeviceToHost, s), "column dots copy");
  ck(hipStreamSynchronize(s), "column dots");
  std::vector<cplx> r(m);
  for (int c = 0; c < m; ++c) r[c] = cplx(h[c].x, h[c].y);
  return r;
}

cm_status check_handle(const cm_handle* h) {
  if (!h) return driver_fail(CM_E_BADARG, "null handle");
  if (!h->has_dev) return driver_fail(CM_E_NOT_BUILT, "handle was built host-only");
  return CM_OK;
}

}  // namespace
}  // namespace cm

extern "C" cm_status cm_real_currents(cm_handle* h, const void* J, int64_t ldj, int32_t m, void* Jr, void* RJr,
                                      int64_t ldo, void* hip_stream) {
  cm_status st = cm::check_handle(h);
  if (st != CM_OK) return st;
  if (!J || !Jr || !RJr) return cm::driver_fail(CM_E_BADARG, "null argument");
  if (m < 1 || m > 512 || ldj < m || ldo < m) return cm::driver_fail(CM_E_BADARG, "need 1 <= m <= 512, ldj >= m, ldo >= m");
  if (J == Jr || J == RJr || Jr == RJr) return cm::driver_fail(CM_E_BADARG, "J, Jr and RJr must not alias");
  try {
    hipStream_t s = (hipStream_t)hip_stream;
    const int64_t N = h->dev.N;
    const double2* Jd = (const double2*)J;
    double2* W = (double2*)Jr;
    double2* RW = (double2*)RJr;
    // the phase that makes sum_i J_i^2 real and positive
    std::vector<cm::cplx> sq = cm::coldots(Jd, ldj, Jd, ldj, m, N, false, s);
    std::vector<double2> ph(m);
    for (int c = 0; c < m; ++c) {
      const double a = -0.5 * std::arg(sq[c]);
      ph[c] = make_double2(std::cos(a), std::sin(a));
    }
    cm::Buf phd(m * sizeof(double2)), scd(m * sizeof(double));
    cm::ck(hipMemcpyAsync(phd.p, ph.data(), m * sizeof(double2), hipMemcpyHostToDevice, s), "phase upload");
    cm::blas_phase_real(Jd, ldj, m, phd.d(), W, ldo, N, s);
    cm::apply_cols(h, 1, W, RW, ldo, m, s);
    std::vector<cm::cplx> nr = cm::coldots(W, ldo, RW, ldo, m, N, true, s);
    std::vector<double> sc(m);
    for (int c = 0; c < m; ++c) {
      if (!(nr[c].real() > 0)) return cm::driver_fail(CM_E_NUMERIC, "a current has no positive R-norm");
      sc[c] = 1.0 / std::sqrt(nr[c].real());
    }
    cm::ck(hipMemcpyAsync(scd.p, sc.data(), m * sizeof(double), hipMemcpyHostToDevice, s), "scale upload");
    cm::blas_scale_cols(W, ldo, m, (const double*)scd.p, N, s);
    cm::blas_scale_cols(RW, ldo, m, (const double*)scd.p, N, s);
    cm::ck(hipGetLastError(), "real currents launch");
    cm::ck(hipStreamSynchronize(s), "real currents");
    return CM_OK;
  } catch (const cm::Error& e) {
    return cm::driver_fail(e.code, e.what());
  } catch (const std::exception& e) {
    return cm::driver_fail(CM_E_OOM, e.what());
  }
}

extern "C" cm_status cm_modal_correlation(cm_handle* h, const void* Ja, int64_t lda, int32_t ma, const void* Jb,
                                          int64_t ldb, int32_t mb, double* C, void* hip_stream) {
  cm_status st = cm::check_handle(h);
  if (st != CM_OK) return st;
  if (!Ja || !Jb || !C) return cm::driver_fail(CM_E_BADARG, "null argument");
  if (ma < 1 || mb < 1 || ma > 512 || mb > 512 || lda < ma || ldb < mb)
    return cm::driver_fail(CM_E_BADARG, "need 1 <= ma, mb <= 512, lda >= ma, ldb >= mb");
  try {
    hipStream_t s = (hipStream_t)hip_stream;
    const int64_t N = h->dev.N;
    const double2* A = (const double2*)Ja;
    const double2* B = (const double2*)Jb;
    // R Ja and R Jb with the inputs' row strides (the apply reads and writes
    // with one stride)
    cm::Buf RA((size_t)N * lda * sizeof(double2)), RB((size_t)N * ldb * sizeof(double2));
    cm::apply_cols(h, 1, A, RA.d(), lda, ma, s);
    cm::apply_cols(h, 1, B, RB.d(), ldb, mb, s);
    std::vector<cm::cplx> G = cm::gram_host(A, lda, ma, RB.d(), ldb, mb, N, false, s);
    std::vector<cm::cplx> na = cm::coldots(A, lda, RA.d(), lda, ma, N, false, s);
    std::vector<cm::cplx> nb = cm::coldots(B, ldb, RB.d(), ldb, mb, N, false, s);
    for (int a = 0; a < ma; ++a)
      for (int b = 0; b < mb; ++b) {
        const double den = std::sqrt(std::abs(na[a]) * std::abs(nb[b]));
        C[(size_t)a * mb + b] = den > 0 ? std::abs(G[(size_t)a * mb + b]) / den : 0.0;
      }
    return CM_OK;
  } catch (const cm::Error& e) {
    return cm::driver_fail(e.code, e.what());
  } catch (const std::exception& e) {
    return cm::driver_fail(CM_E_OOM, e.what());
  }
}

extern "C" cm_status cm_dlambda_dk(cm_handle* h, double lambda, const void* J, int64_t ldj, int32_t m, double* dldk,
                                   void* hip_stream) {
  cm_status st = cm::check_handle(h);
  if (st != CM_OK) return st;
  if (!J || !dldk) return cm::driver_fail(CM_E_BADARG, "null argument");
  if (m < 1 || m > 256 || ldj < m) return cm::driver_fail(CM_E_BADARG, "need 1 <= m <= 256 and ldj >= m");
  if (!std::isfinite(lambda)) return cm::driver_fail(CM_E_BADARG, "lambda must be finite");
  if (!(h->plan.opt.flags & CM_FLAG_DERIV)) return cm::driver_fail(CM_E_NOT_BUILT, "dZ/dk needs CM_FLAG_DERIV at create");
  try {
    hipStream_t s = (hipStream_t)hip_stream;
    const int64_t N = h->dev.N;
    const int m2 = 2 * m;
    cm::Buf W((size_t)N * m2 * sizeof(double2)), RW((size_t)N * m2 * sizeof(double2)),
        Q((size_t)N * m * sizeof(double2)), D((size_t)N * m * sizeof(double2)),
        Md((size_t)m2 * m * sizeof(double2));
    // real span of the cluster: real and imaginary parts of the vectors
    cm::blas_split_reim((const double2*)J, ldj, m, W.d(), m2, N, s);
    cm::apply_cols(h, 1, W.d(), RW.d(), m2, m2, s);
    std::vector<cm::cplx> G = cm::gram_host(W.d(), m2, m2, RW.d(), m2, m2, N, true, s);
    // R-orthonormal basis Q of the span from the m largest eigenpairs of W^T R W
    std::vector<cm::cplx> Gs((size_t)m2 * m2);
    for (int a = 0; a < m2; ++a)
      for (int b = 0; b < m2; ++b)
        Gs[(size_t)b * m2 + a] = 0.5 * (G[(size_t)a * m2 + b].real() + G[(size_t)b * m2 + a].real());
    std::vector<double> w;
    std::vector<cm::cplx> S;
    cm::herm_eig(Gs, m2, w, S);
    std::vector<double2> M((size_t)m2 * m);
    for (int c = 0; c < m; ++c) {
      const int e = m2 - 1 - c;                   // descending
      if (!(w[e] > 0)) return cm::driver_fail(CM_E_NUMERIC, "the cluster's span has no positive R-norm");
      const double sc = 1.0 / std::sqrt(w[e]);
      for (int k = 0; k < m2; ++k) M[(size_t)c * m2 + k] = make_double2(S[(size_t)e * m2 + k].real() * sc, 0.0);
    }
    cm::ck(hipMemcpyAsync(Md.p, M.data(), M.size() * sizeof(double2), hipMemcpyHostToDevice, s), "basis upload");
    cm::blas_rowmix(W.d(), m2, m2, Md.d(), m, Q.d(), m, N, s);
    cm::apply_cols(h, 4, Q.d(), D.d(), m, m, s);
    std::vector<cm::cplx> P = cm::gram_host(Q.d(), m, m, D.d(), m, m, N, true, s);
    // Q^T (X' - lambda R') Q with X' = Im dZ/dk, R' = Re dZ/dk (Q real)
    std::vector<cm::cplx> Mx((size_t)m * m);
    for (int a = 0; a < m; ++a)
      for (int b = 0; b < m; ++b) {
        const cm::cplx pab = P[(size_t)a * m + b], pba = P[(size_t)b * m + a];
        Mx[(size_t)b * m + a] = 0.5 * ((pab.imag() - lambda * pab.real()) + (pba.imag() - lambda * pba.real()));
      }
    cm::herm_eig(Mx, m, w, S);
    for (int c = 0; c < m; ++c) dldk[c] = w[c];
    return CM_OK;
  } catch (const cm::Error& e) {
    return cm::driver_fail(e.code, e.what());
  } catch (const std::exception& e) {
    return cm::driver_fail(CM_E_OOM, e.what());
  }
}
