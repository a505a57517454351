// SAI preconditioner build (section IV): P minimises ||I - Z_near P||_F column
// by column over a prescribed pattern.  Thresholds (the paper does not define
// them): Z~ drops entries |z_ij| < eps1 |z_jj| of column j; column j of P lives
// on J_j = {i : |z_ij| >= eps2 |z_jj|}; the rows taking part are the nonzero
// rows of Z~(:, J_j); entries |p_ij| < eps3 max_i |p_ij| are dropped after the
// solve.  The same construction serves the near field of the shifted
// operator tau R + i X of the Arnoldi inner solves (tau Re Z_near + i Im
// Z_near; tau = 0: the real X_near).  Set-up work on the host: the near
// field is copied down once, every
// column's small least-squares problem is solved by Householder QR in FP64,
// and P is uploaded in CSR by rows for the device apply.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <complex>
#include <exception>
#include <thread>
#include <vector>

#include "cm_device.h"

namespace cm {

static void chk_s(hipError_t e, const char* what) {
  if (e != hipSuccess) throw Error(-4, std::string(what) + ": " + hipGetErrorString(e));
}

// Least squares min ||b - A p|| for a dense column-major m x n complex A (m >= n)
// by Householder QR; columns with a vanishing pivot get p = 0.
static void lsq_householder(int m, int n, std::vector<cplx>& A, std::vector<cplx>& b, std::vector<cplx>& p) {
  std::vector<cplx> v(m);
  for (int k = 0; k < n && k < m; ++k) {
    double nx = 0;
    for (int i = k; i < m; ++i) nx += std::norm(A[(size_t)k * m + i]);
    nx = std::sqrt(nx);
    if (nx == 0) continue;
    cplx x0 = A[(size_t)k * m + k];
    cplx ph = (std::abs(x0) > 0) ? x0 / std::abs(x0) : cplx(1, 0);
    cplx alpha = -ph * nx;
    for (int i = k; i < m; ++i) v[i] = A[(size_t)k * m + i];
    v[k] -= alpha;
    double nv = 0;
    for (int i = k; i < m; ++i) nv += std::norm(v[i]);
    nv = std::sqrt(nv);
    if (nv == 0) continue;
    for (int i = k; i < m; ++i) v[i] /= nv;
    for (int c = k; c < n; ++c) {
      cplx s = 0;
      for (int i = k; i < m; ++i) s += std::conj(v[i]) * A[(size_t)c * m + i];
      for (int i = k; i < m; ++i) A[(size_t)c * m + i] -= 2.0 * v[i] * s;
    }
    cplx s = 0;
    for (int i = k; i < m; ++i) s += std::conj(v[i]) * b[i];
    for (int i = k; i < m; ++i) b[i] -= 2.0 * v[i] * s;
  }
  p.assign(n, cplx(0));
  double rmax = 0;
  for (int k = 0; k < std::min(m, n); ++k) rmax = std::max(rmax, std::abs(A[(size_t)k * m + k]));
  for (int k = std::min(m, n) - 1; k >= 0; --k) {
    cplx s = b[k];
    for (int c = k + 1; c < n; ++c) s -= A[(size_t)c * m + k] * p[c];
    cplx r = A[(size_t)k * m + k];
    p[k] = (std::abs(r) > 1e-14 * rmax) ? s / r : cplx(0);
  }
}

void dev_sai_build(Dev& d, const Plan& P, double e1, double e2, double e3, double tau, hipStream_t s) {
  const int part = sai_slot(tau);
  const int64_t N = d.N;
  std::vector<double2> zn(P.nnz);
  chk_s(hipMemcpyAsync(zn.data(), d.Zn, P.nnz * sizeof(double2), hipMemcpyDeviceToHost, s), "SAI: copy near field");
  chk_s(hipStreamSynchronize(s), "SAI: copy near field");
  // the near field of tau R + i X: tau Re z + i Im z; tau = 0 selects the
  // real matrix X_near = Im Z_near itself (the solves with X)
  if (tau == 0.0)
    for (auto& z : zn) z = make_double2(z.y, 0.0);
  else if (tau != 1.0)
    for (auto& z : zn) z = make_double2(tau * z.x, z.y);
  // row i of Z_near (internal order) = column i (Z_near is symmetric)
  auto row_cols = [&](int64_t i, const int32_t*& cols, const double2*& vals, int& n) {
    int b = P.box_of[i];
    cols = &P.bcol[P.bcol_ptr[b]];
    n = P.bcol_ptr[b + 1] - P.bcol_ptr[b];
    vals = &zn[P.row_ptr[i]];
  };
  std::vector<double> diag(N);
  for (int64_t i = 0; i < N; ++i) {
    const int32_t* c;
    const double2* v;
    int n;
    row_cols(i, c, v, n);
    const int32_t* at = std::lower_bound(c, c + n, (int32_t)i);
    diag[i] = std::hypot(v[at - c].x, v[at - c].y);
  }
  // per column: list of (row, value) of P
  std::vector<std::vector<std::pair<int32_t, cplx>>> colP(N);
  unsigned nth = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
  std::vector<std::thread> th;
  // an exception in a worker (e.g. std::bad_alloc) is kept and rethrown after
  // the join, so that the C ABI returns a status instead of terminating
  std::vector<std::exception_ptr> err(nth);
  for (unsigned t = 0; t < nth; ++t)
    th.emplace_back([&, t]() {
     try {
      std::vector<int32_t> J, I;
      std::vector<cplx> A, b, p;
      for (int64_t j = t; j < N; j += nth) {
        const int32_t* cj;
        const double2* vj;
        int nj;
        row_cols(j, cj, vj, nj);
        J.clear();
        for (int q = 0; q < nj; ++q)
          if (std::hypot(vj[q].x, vj[q].y) >= e2 * diag[j] && (vj[q].x != 0 || vj[q].y != 0)) J.push_back(cj[q]);
        // rows: union of the kept entries of Z~(:, a), a in J
        I.clear();
        for (int32_t a : J) {
          const int32_t* ca;
          const double2* va;
          int na;
          row_cols(a, ca, va, na);
          for (int q = 0; q < na; ++q)
            if (std::hypot(va[q].x, va[q].y) >= e1 * diag[a] && (va[q].x != 0 || va[q].y != 0)) I.push_back(ca[q]);
        }
        std::sort(I.begin(), I.end());
        I.erase(std::unique(I.begin(), I.end()), I.end());
        const int m = (int)I.size(), n = (int)J.size();
        if (n == 0 || m == 0) continue;
        A.assign((size_t)m * n, cplx(0));
        for (int c = 0; c < n; ++c) {
          const int32_t* ca;
          const double2* va;
          int na;
          row_cols(J[c], ca, va, na);
          for (int q = 0; q < na; ++q)
            if (std::hypot(va[q].x, va[q].y) >= e1 * diag[J[c]] && (va[q].x != 0 || va[q].y != 0)) {
              int r = (int)(std::lower_bound(I.begin(), I.end(), ca[q]) - I.begin());
              A[(size_t)c * m + r] = cplx(va[q].x, va[q].y);
            }
        }
        b.assign(m, cplx(0));
        int rj = (int)(std::lower_bound(I.begin(), I.end(), (int32_t)j) - I.begin());
        if (rj < m && I[rj] == j) b[rj] = 1.0;
        lsq_householder(m, n, A, b, p);
        double pm = 0;
        for (auto& z : p) pm = std::max(pm, std::abs(z));
        for (int c = 0; c < n; ++c)
          if (std::abs(p[c]) >= e3 * pm && std::abs(p[c]) > 0) colP[j].push_back({J[c], p[c]});
      }
     } catch (...) {
      err[t] = std::current_exception();
     }
    });
  for (auto& x : th) x.join();
  for (auto& e : err)
    if (e) std::rethrow_exception(e);
  // transpose to CSR by rows (internal indices)
  std::vector<int64_t> ptr(N + 1, 0);
  for (int64_t j = 0; j < N; ++j)
    for (auto& e : colP[j]) ptr[e.first + 1]++;
  for (int64_t i = 0; i < N; ++i) ptr[i + 1] += ptr[i];
  const int64_t nnz = ptr[N];
  std::vector<int32_t> col(nnz);
  std::vector<double2> val(nnz);
  std::vector<int64_t> fill(ptr.begin(), ptr.end() - 1);
  for (int64_t j = 0; j < N; ++j)
    for (auto& e : colP[j]) {
      int64_t at = fill[e.first]++;
      col[at] = (int32_t)j;
      val[at] = make_double2(e.second.real(), e.second.imag());
    }
  SaiD& q = d.sai[part];
  if (q.ptr) {
    (void)hipFree(q.ptr);
    (void)hipFree(q.col);
    (void)hipFree(q.val);
    q = SaiD();
  }
  chk_s(hipMalloc(&q.ptr, (N + 1) * sizeof(int64_t)), "SAI alloc");
  chk_s(hipMalloc(&q.col, std::max<int64_t>(1, nnz) * sizeof(int32_t)), "SAI alloc");
  chk_s(hipMalloc(&q.val, std::max<int64_t>(1, nnz) * sizeof(double2)), "SAI alloc");
  chk_s(hipMemcpy(q.ptr, ptr.data(), (N + 1) * sizeof(int64_t), hipMemcpyHostToDevice), "SAI upload");
  if (nnz) {
    chk_s(hipMemcpy(q.col, col.data(), nnz * sizeof(int32_t), hipMemcpyHostToDevice), "SAI upload");
    chk_s(hipMemcpy(q.val, val.data(), nnz * sizeof(double2), hipMemcpyHostToDevice), "SAI upload");
  }
  q.nnz = nnz;
  if (part == 1) d.sai_tau1 = tau;
}

}  // namespace cm
