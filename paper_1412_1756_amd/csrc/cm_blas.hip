// FP64 vector kernels for the Krylov drivers (GMRES inner solves and the
// Arnoldi outer iteration): block dot products V^H w, w -= V h, norms,
// scaling, precision conversion, and the basis update V Q of an implicit
// restart.  Vectors are complex double, one column of N contiguous entries.
#include <hip/hip_runtime.h>

#include "cm_device.h"

namespace cm {

// h[k] = sum_i conj(V[k][i]) w[i], k < nk: one block per k, 256 threads.
__global__ void __launch_bounds__(256) k_multidot(const double2* __restrict__ V, int64_t ldv,
                                                  const double2* __restrict__ w, int64_t N,
                                                  double2* __restrict__ h) {
  __shared__ double sx[256], sy[256];
  const double2* v = V + (int64_t)blockIdx.x * ldv;
  double ax = 0, ay = 0;
  for (int64_t i = threadIdx.x; i < N; i += blockDim.x) {
    double2 a = v[i], b = w[i];
    ax = fma(a.x, b.x, ax);
    ax = fma(a.y, b.y, ax);
    ay = fma(a.x, b.y, ay);
    ay = fma(-a.y, b.x, ay);
  }
  sx[threadIdx.x] = ax;
  sy[threadIdx.x] = ay;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) {
      sx[threadIdx.x] += sx[threadIdx.x + s];
      sy[threadIdx.x] += sy[threadIdx.x + s];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) h[blockIdx.x] = make_double2(sx[0], sy[0]);
}

// w[i] -= sum_k V[k][i] h[k]
__global__ void __launch_bounds__(256) k_gemv_sub(const double2* __restrict__ V, int64_t ldv,
                                                  const double2* __restrict__ h, int nk, double2* __restrict__ w,
                                                  int64_t N) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N) return;
  double2 r = w[i];
  for (int k = 0; k < nk; ++k) {
    double2 a = V[(int64_t)k * ldv + i], b = h[k];
    r.x -= a.x * b.x - a.y * b.y;
    r.y -= a.x * b.y + a.y * b.x;
  }
  w[i] = r;
}

// y = alpha x (+ y if accumulate)
__global__ void __launch_bounds__(256) k_axpby(const double2* __restrict__ x, double2 alpha, double2* __restrict__ y,
                                               int64_t N, int accumulate) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N) return;
  double2 a = x[i];
  double2 r = make_double2(alpha.x * a.x - alpha.y * a.y, alpha.x * a.y + alpha.y * a.x);
  if (accumulate) {
    r.x += y[i].x;
    r.y += y[i].y;
  }
  y[i] = r;
}

// Vout[c][i] = sum_k V[k][i] Q[k + c*ldq], c < nc  (Q column-major, on the device)
__global__ void __launch_bounds__(256) k_basis_update(const double2* __restrict__ V, int64_t ldv,
                                                      const double2* __restrict__ Q, int ldq, int nk, int nc,
                                                      double2* __restrict__ Vout, int64_t N) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N) return;
  for (int c = 0; c < nc; ++c) {
    double ax = 0, ay = 0;
    for (int k = 0; k < nk; ++k) {
      double2 a = V[(int64_t)k * ldv + i], b = Q[k + (int64_t)c * ldq];
      ax += a.x * b.x - a.y * b.y;
      ay += a.x * b.y + a.y * b.x;
    }
    Vout[(int64_t)c * ldv + i] = make_double2(ax, ay);
  }
}

__global__ void __launch_bounds__(256) k_to_c64(const double2* __restrict__ x, float2* __restrict__ y, int64_t N) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < N) y[i] = make_float2((float)x[i].x, (float)x[i].y);
}

__global__ void __launch_bounds__(256) k_to_c128(const float2* __restrict__ x, double2* __restrict__ y, int64_t N) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < N) y[i] = make_double2((double)x[i].x, (double)x[i].y);
}

// xs[i][j] = x[i][cols[j]] (xs dense, ld = cols.n); ys -> y the other way
template <typename C>
__global__ void __launch_bounds__(256) k_gather_cols(const C* __restrict__ x, int64_t ld, ColList cols, int ws,
                                                     C* __restrict__ xs, int64_t N) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= N * ws) return;
  const int64_t i = e / ws;
  const int j = (int)(e - i * ws);
  C v;
  v.x = 0;
  v.y = 0;
  xs[e] = (j < cols.n) ? x[i * ld + cols.c[j]] : v;   // columns past the list: zero padding
}
template <typename C>
__global__ void __launch_bounds__(256) k_scatter_cols(const C* __restrict__ ys, int ws, ColList cols,
                                                      C* __restrict__ y, int64_t ld, int64_t N) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= N * cols.n) return;
  const int64_t i = e / cols.n;
  const int j = (int)(e - i * cols.n);
  y[i * ld + cols.c[j]] = ys[i * ws + j];
}

static inline dim3 g1(int64_t N) { return dim3((unsigned)((N + 255) / 256)); }

void blas_gather_cols(const void* x, int64_t ld, ColList cols, int ws, void* xs, int64_t N, bool fp64,
                      hipStream_t s) {
  if (fp64)
    hipLaunchKernelGGL(k_gather_cols<double2>, g1(N * ws), dim3(256), 0, s, (const double2*)x, ld, cols, ws,
                       (double2*)xs, N);
  else
    hipLaunchKernelGGL(k_gather_cols<float2>, g1(N * ws), dim3(256), 0, s, (const float2*)x, ld, cols, ws,
                       (float2*)xs, N);
}
void blas_scatter_cols(const void* ys, int ws, ColList cols, void* y, int64_t ld, int64_t N, bool fp64,
                       hipStream_t s) {
  if (fp64)
    hipLaunchKernelGGL(k_scatter_cols<double2>, g1(N * cols.n), dim3(256), 0, s, (const double2*)ys, ws, cols,
                       (double2*)y, ld, N);
  else
    hipLaunchKernelGGL(k_scatter_cols<float2>, g1(N * cols.n), dim3(256), 0, s, (const float2*)ys, ws, cols,
                       (float2*)y, ld, N);
}

void blas_multidot(const double2* V, int64_t ldv, const double2* w, int64_t N, int nk, double2* h, hipStream_t s) {
  if (nk > 0) hipLaunchKernelGGL(k_multidot, dim3(nk), dim3(256), 0, s, V, ldv, w, N, h);
}
void blas_gemv_sub(const double2* V, int64_t ldv, const double2* h, int nk, double2* w, int64_t N, hipStream_t s) {
  if (nk > 0) hipLaunchKernelGGL(k_gemv_sub, g1(N), dim3(256), 0, s, V, ldv, h, nk, w, N);
}
// y <- alpha y in place
__global__ void __launch_bounds__(256) k_scale(double2* y, double2 alpha, int64_t N) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N) return;
  double2 a = y[i];
  y[i] = make_double2(alpha.x * a.x - alpha.y * a.y, alpha.x * a.y + alpha.y * a.x);
}

void blas_scale(double2* y, double2 alpha, int64_t N, hipStream_t s) {
  hipLaunchKernelGGL(k_scale, g1(N), dim3(256), 0, s, y, alpha, N);
}
void blas_axpby(const double2* x, double2 alpha, double2* y, int64_t N, int accumulate, hipStream_t s) {
  hipLaunchKernelGGL(k_axpby, g1(N), dim3(256), 0, s, x, alpha, y, N, accumulate);
}
void blas_basis_update(const double2* V, int64_t ldv, const double2* Q, int ldq, int nk, int nc, double2* Vout,
                       int64_t N, hipStream_t s) {
  hipLaunchKernelGGL(k_basis_update, g1(N), dim3(256), 0, s, V, ldv, Q, ldq, nk, nc, Vout, N);
}
void blas_to_c64(const double2* x, float2* y, int64_t N, hipStream_t s) {
  hipLaunchKernelGGL(k_to_c64, g1(N), dim3(256), 0, s, x, y, N);
}
void blas_to_c128(const float2* x, double2* y, int64_t N, hipStream_t s) {
  hipLaunchKernelGGL(k_to_c128, g1(N), dim3(256), 0, s, x, y, N);
}

}  // namespace cm
