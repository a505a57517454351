// FP64 vector kernels for the Krylov drivers (GMRES inner solves and the
// Arnoldi outer iteration): block dot products V^H w, w -= V h, norms,
// scaling, precision conversion, and the basis update V Q of an implicit
// restart.  Vectors are complex double, one column of N contiguous entries.
#include <hip/hip_runtime.h>

#include <algorithm>

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

// The same over all CUs: block b sums rows [b rpb, (b + 1) rpb) for KG basis
// vectors at a time (w read once per group), wave sums by lane shuffles,
// part[k * nblk + b]; k_multidot_final adds the blocks in order.  flag (may
// be null): the launch does nothing unless *flag != 0 (the conditional
// second Gram-Schmidt pass of the device GMRES).
template <int KG>
__global__ void __launch_bounds__(256) k_multidot_part(const double2* __restrict__ V, int64_t ldv,
                                                       const double2* __restrict__ w, int64_t N, int nk, int64_t rpb,
                                                       double2* __restrict__ part, const int* __restrict__ flag) {
  if (flag && *flag == 0) return;
  __shared__ double rx[4][KG], ry[4][KG];
  const int64_t i0 = (int64_t)blockIdx.x * rpb, i1 = min(N, i0 + rpb);
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  for (int k0 = 0; k0 < nk; k0 += KG) {
    double ax[KG], ay[KG];
#pragma unroll
    for (int u = 0; u < KG; ++u) ax[u] = ay[u] = 0.0;
    const int ku = min(KG, nk - k0);
    for (int64_t i = i0 + threadIdx.x; i < i1; i += 256) {
      const double2 b = w[i];
#pragma unroll
      for (int u = 0; u < KG; ++u)
        if (u < ku) {
          const double2 a = V[(int64_t)(k0 + u) * ldv + i];
          ax[u] = fma(a.x, b.x, ax[u]);
          ax[u] = fma(a.y, b.y, ax[u]);
          ay[u] = fma(a.x, b.y, ay[u]);
          ay[u] = fma(-a.y, b.x, ay[u]);
        }
    }
#pragma unroll
    for (int u = 0; u < KG; ++u)
      for (int off = 32; off > 0; off >>= 1) {
        ax[u] += __shfl_xor(ax[u], off);
        ay[u] += __shfl_xor(ay[u], off);
      }
    if (lane == 0)
#pragma unroll
      for (int u = 0; u < KG; ++u) {
        rx[wv][u] = ax[u];
        ry[wv][u] = ay[u];
      }
    __syncthreads();
    if ((int)threadIdx.x < ku) {
      const int u = threadIdx.x;
      part[(int64_t)(k0 + u) * gridDim.x + blockIdx.x] =
          make_double2(rx[0][u] + rx[1][u] + rx[2][u] + rx[3][u], ry[0][u] + ry[1][u] + ry[2][u] + ry[3][u]);
    }
    __syncthreads();
  }
}

__global__ void __launch_bounds__(256) k_multidot_final(const double2* __restrict__ part, int nblk, int nk,
                                                        double2* __restrict__ h, const int* __restrict__ flag) {
  if (flag && *flag == 0) return;
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= nk) return;
  double ax = 0, ay = 0;
  for (int b = 0; b < nblk; ++b) {
    ax += part[(int64_t)k * nblk + b].x;
    ay += part[(int64_t)k * nblk + b].y;
  }
  h[k] = make_double2(ax, ay);
}

// w[i] -= sum_k V[k][i] h[k] (nothing when flag is given and *flag == 0)
__global__ void __launch_bounds__(256) k_gemv_sub(const double2* __restrict__ V, int64_t ldv,
                                                  const double2* __restrict__ h, int nk, double2* __restrict__ w,
                                                  int64_t N, const int* __restrict__ flag) {
  if (flag && *flag == 0) return;
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
  xs[e] = (j < cols.n && cols.c[j] >= 0) ? x[i * ld + cols.c[j]] : v;   // past the list or -1: zero padding
}
template <typename C>
__global__ void __launch_bounds__(256) k_scatter_cols(const C* __restrict__ ys, int ws, ColList cols,
                                                      C* __restrict__ y, int64_t ld, int64_t N) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= N * cols.n) return;
  const int64_t i = e / cols.n;
  const int j = (int)(e - i * cols.n);
  if (cols.c[j] >= 0) y[i * ld + cols.c[j]] = ys[i * ws + j];   // -1: a padding column
}

// ---------------------------------------------------------------- small dense projections
// Partial Gram products of row-major N x na and N x nb complex128 blocks:
// part[blk][a * nb + b] = sum over the block's rows of op(A[i, a]) B[i, b],
// op = conj when conjA.  Block = 256 threads = PB pairs x (256 / PB) row
// lanes; the row lanes are summed in LDS in a fixed order, and the blocks by
// k_gram_final, so the result does not depend on the launch timing.
__global__ void __launch_bounds__(256) k_gram_partial(const double2* __restrict__ A, int64_t lda, int na,
                                                      const double2* __restrict__ B, int64_t ldb, int nb, int64_t N,
                                                      int conjA, int PB, int64_t rows_per_blk,
                                                      double2* __restrict__ part) {
  __shared__ double sx[256], sy[256];
  const int npair = na * nb;
  const int pl = threadIdx.x % PB, lane = threadIdx.x / PB, tpr = 256 / PB;
  const int pair = blockIdx.y * PB + pl;
  double ax = 0, ay = 0;
  if (pair < npair) {
    const int a = pair / nb, b = pair % nb;
    const int64_t i0 = (int64_t)blockIdx.x * rows_per_blk, i1 = min(N, i0 + rows_per_blk);
    for (int64_t i = i0 + lane; i < i1; i += tpr) {
      double2 u = A[i * lda + a], v = B[i * ldb + b];
      if (conjA) u.y = -u.y;
      ax = fma(u.x, v.x, ax);
      ax = fma(-u.y, v.y, ax);
      ay = fma(u.x, v.y, ay);
      ay = fma(u.y, v.x, ay);
    }
  }
  sx[threadIdx.x] = ax;
  sy[threadIdx.x] = ay;
  __syncthreads();
  for (int s = tpr / 2; s > 0; s >>= 1) {
    if (lane < s) {
      sx[threadIdx.x] += sx[threadIdx.x + s * PB];
      sy[threadIdx.x] += sy[threadIdx.x + s * PB];
    }
    __syncthreads();
  }
  if (lane == 0 && pair < npair) part[(int64_t)blockIdx.x * npair + pair] = make_double2(sx[threadIdx.x], sy[threadIdx.x]);
}

__global__ void __launch_bounds__(256) k_gram_final(const double2* __restrict__ part, int nblk, int npair,
                                                    double2* __restrict__ out) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= npair) return;
  double ax = 0, ay = 0;
  for (int b = 0; b < nblk; ++b) {
    ax += part[(int64_t)b * npair + p].x;
    ay += part[(int64_t)b * npair + p].y;
  }
  out[p] = make_double2(ax, ay);
}

// number of row blocks of a Gram product (also the size of its partial buffer
// in units of npair complex values)
int blas_gram_blocks(int64_t N) { return (int)std::max<int64_t>(1, std::min<int64_t>(512, (N + 2047) / 2048)); }

// out[a * nb + b] = sum_i op(A[i, a]) B[i, b] (device, na * nb complex128);
// part: device scratch of blas_gram_blocks(N) * na * nb complex128
void blas_gram(const double2* A, int64_t lda, int na, const double2* B, int64_t ldb, int nb, int64_t N, bool conjA,
               double2* part, double2* out, hipStream_t s) {
  const int npair = na * nb;
  if (npair <= 0) return;
  int PB = 1;
  while (PB < npair && PB < 256) PB *= 2;
  const int nblk = blas_gram_blocks(N);
  const int64_t rpb = (N + nblk - 1) / nblk;
  hipLaunchKernelGGL(k_gram_partial, dim3(nblk, (npair + PB - 1) / PB), dim3(256), 0, s, A, lda, na, B, ldb, nb, N,
                     conjA ? 1 : 0, PB, rpb, part);
  hipLaunchKernelGGL(k_gram_final, dim3((npair + 255) / 256), dim3(256), 0, s, part, nblk, npair, out);
}

// sum over i < N, c < nc of conj(x[i, c]) y[i, c] for complex float or double
// x, y (row stride ld), accumulated in FP64: partial sums per block, then the
// blocks in a fixed order into out (device, one complex128)
template <typename C>
__global__ void __launch_bounds__(256) k_vdot_partial(const C* __restrict__ x, const C* __restrict__ y, int64_t ld,
                                                      int nc, int64_t N, double2* __restrict__ part) {
  __shared__ double sx[256], sy[256];
  const int64_t tot = N * nc;
  double ax = 0, ay = 0;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < tot; e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = e / nc;
    const int c = (int)(e - i * nc);
    const C u = x[i * ld + c], v = y[i * ld + c];
    ax = fma((double)u.x, (double)v.x, ax);
    ax = fma((double)u.y, (double)v.y, ax);
    ay = fma((double)u.x, (double)v.y, ay);
    ay = fma(-(double)u.y, (double)v.x, ay);
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
  if (threadIdx.x == 0) part[blockIdx.x] = make_double2(sx[0], sy[0]);
}

constexpr int kVdotBlocks = 512;
int blas_vdot_blocks() { return kVdotBlocks; }
// part: device scratch of blas_vdot_blocks() complex128
void blas_vdot(const void* x, const void* y, int64_t ld, int nc, int64_t N, bool fp64, double2* part, double2* out,
               hipStream_t s) {
  if (fp64)
    hipLaunchKernelGGL(k_vdot_partial<double2>, dim3(kVdotBlocks), dim3(256), 0, s, (const double2*)x,
                       (const double2*)y, ld, nc, N, part);
  else
    hipLaunchKernelGGL(k_vdot_partial<float2>, dim3(kVdotBlocks), dim3(256), 0, s, (const float2*)x,
                       (const float2*)y, ld, nc, N, part);
  hipLaunchKernelGGL(k_gram_final, dim3(1), dim3(256), 0, s, part, kVdotBlocks, 1, out);
}

// W[i, c] = Re(J[i, c] ph[c]) (as complex128 with zero imaginary part), c < m
__global__ void __launch_bounds__(256) k_phase_real(const double2* __restrict__ J, int64_t ldj, int m,
                                                    const double2* __restrict__ ph, double2* __restrict__ W,
                                                    int64_t ldw, int64_t N) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= N * m) return;
  const int64_t i = e / m;
  const int c = (int)(e - i * m);
  const double2 a = J[i * ldj + c], p = ph[c];
  W[i * ldw + c] = make_double2(a.x * p.x - a.y * p.y, 0.0);
}

// W[i, c] = (Re J[i, c], 0), W[i, m + c] = (Im J[i, c], 0), c < m
__global__ void __launch_bounds__(256) k_split_reim(const double2* __restrict__ J, int64_t ldj, int m,
                                                    double2* __restrict__ W, int64_t ldw, int64_t N) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= N * m) return;
  const int64_t i = e / m;
  const int c = (int)(e - i * m);
  const double2 a = J[i * ldj + c];
  W[i * ldw + c] = make_double2(a.x, 0.0);
  W[i * ldw + m + c] = make_double2(a.y, 0.0);
}

// Out[i, c] = sum_k A[i, k] M[k + c * na], c < nb (M column-major on the device)
__global__ void __launch_bounds__(256) k_rowmix(const double2* __restrict__ A, int64_t lda, int na,
                                                const double2* __restrict__ M, int nb, double2* __restrict__ Out,
                                                int64_t ldo, int64_t N) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= N * nb) return;
  const int64_t i = e / nb;
  const int c = (int)(e - i * nb);
  double ax = 0, ay = 0;
  for (int k = 0; k < na; ++k) {
    const double2 a = A[i * lda + k], b = M[k + (int64_t)c * na];
    ax = fma(a.x, b.x, ax);
    ax = fma(-a.y, b.y, ax);
    ay = fma(a.x, b.y, ay);
    ay = fma(a.y, b.x, ay);
  }
  Out[i * ldo + c] = make_double2(ax, ay);
}

// A[i, c] *= sc[c]
__global__ void __launch_bounds__(256) k_scale_cols(double2* __restrict__ A, int64_t lda, int m,
                                                    const double* __restrict__ sc, int64_t N) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= N * m) return;
  const int64_t i = e / m;
  const int c = (int)(e - i * m);
  A[i * lda + c].x *= sc[c];
  A[i * lda + c].y *= sc[c];
}

// ---------------------------------------------------------------- device-resident GMRES step
// One Hessenberg column of GMRES(m) formed on the device, so that an
// iteration needs no host round trip.  hc = V[0..j+1]^H w from this pass's
// multidot (the last entry is w^H w before this pass's projection); col
// accumulates the raw column over the Gram-Schmidt passes.  Pass 0: if the
// projection cancelled more than half of w (squared norm ratio 0.514), the
// second pass is requested (st->need2) and the column waits for it; else
// (and after pass 1) ||w|| follows by Pythagoras, the earlier Givens
// rotations are applied to the column, a new rotation zeroes its subdiagonal
// and updates g; st receives 1/||w|| (for the scaling of the new vector), the
// residual estimate |g[j+1]|, the number of valid columns, and stop = 1 on a
// breakdown (||w|| = 0: the Krylov space is invariant and x is exact).
__global__ void __launch_bounds__(64) k_gmres_step(int j, int m, const double2* __restrict__ hc,
                                                   double2* __restrict__ col, double2* __restrict__ H,
                                                   double2* __restrict__ g, double2* __restrict__ cs,
                                                   double2* __restrict__ sn, GmState* __restrict__ st, int pass) {
  extern __shared__ double2 sm[];   // col[j+2], cs[j], sn[j]
  if (st->stop) return;
  if (pass == 1 && st->need2 == 0) return;
  const int lane = threadIdx.x;
  double hs = 0;
  for (int k = lane; k <= j; k += 64) {
    const double2 v = hc[k];
    hs += v.x * v.x + v.y * v.y;
    const double2 a = pass == 0 ? make_double2(0.0, 0.0) : col[k];
    col[k] = make_double2(a.x + v.x, a.y + v.y);
  }
  for (int off = 32; off > 0; off >>= 1) hs += __shfl_xor(hs, off);
  const double ww = hc[j + 1].x;
  const double r2 = ww - hs;
  if (pass == 0 && !(r2 > 0.514 * ww)) {
    if (lane == 0) st->need2 = 1;
    return;
  }
  __syncthreads();
  double2* c = sm;
  double2* scs = sm + (j + 2);
  double2* ssn = scs + j;
  for (int k = lane; k <= j; k += 64) c[k] = col[k];
  for (int k = lane; k < j; k += 64) {
    scs[k] = cs[k];
    ssn[k] = sn[k];
  }
  __syncthreads();
  if (lane != 0) return;
  const double hn = sqrt(fmax(r2, 0.0));
  c[j + 1] = make_double2(hn, 0.0);
  for (int k = 0; k < j; ++k) {
    const double2 a = c[k], b = c[k + 1], ck = scs[k], sk = ssn[k];
    // c[k] = conj(cs) a + conj(sn) b ; c[k+1] = -sn a + cs b
    c[k] = make_double2(ck.x * a.x + ck.y * a.y + sk.x * b.x + sk.y * b.y,
                        ck.x * a.y - ck.y * a.x + sk.x * b.y - sk.y * b.x);
    c[k + 1] = make_double2(-(sk.x * a.x - sk.y * a.y) + (ck.x * b.x - ck.y * b.y),
                            -(sk.x * a.y + sk.y * a.x) + (ck.x * b.y + ck.y * b.x));
  }
  const double r = hypot(hypot(c[j].x, c[j].y), hypot(c[j + 1].x, c[j + 1].y));
  double2 cj = make_double2(1.0, 0.0), sj = make_double2(0.0, 0.0);
  if (r > 0) {
    cj = make_double2(c[j].x / r, c[j].y / r);
    sj = make_double2(c[j + 1].x / r, c[j + 1].y / r);
  }
  cs[j] = cj;
  sn[j] = sj;
  c[j] = make_double2(r, 0.0);
  c[j + 1] = make_double2(0.0, 0.0);
  const double2 gj = g[j];
  g[j + 1] = make_double2(-(sj.x * gj.x - sj.y * gj.y), -(sj.x * gj.y + sj.y * gj.x));
  g[j] = make_double2(cj.x * gj.x + cj.y * gj.y, cj.x * gj.y - cj.y * gj.x);
  for (int k = 0; k <= j + 1; ++k) H[(int64_t)j * (m + 1) + k] = c[k];
  st->need2 = 0;
  st->inv_hn = hn > 0 ? 1.0 / hn : 0.0;
  st->res = hypot(g[j + 1].x, g[j + 1].y);
  st->nvalid = j + 1;
  if (!(hn > 0)) st->stop = 1;
}

// y *= st->inv_hn
__global__ void __launch_bounds__(256) k_scale_by_state(double2* __restrict__ y, const GmState* __restrict__ st,
                                                        int64_t N) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N) return;
  const double a = st->inv_hn;
  y[i].x *= a;
  y[i].y *= a;
}

static inline dim3 g1(int64_t N) { return dim3((unsigned)((N + 255) / 256)); }

void blas_gmres_step(int j, int m, const double2* hc, double2* col, double2* H, double2* g, double2* cs, double2* sn,
                     GmState* st, int pass, hipStream_t s) {
  hipLaunchKernelGGL(k_gmres_step, dim3(1), dim3(64), (size_t)(3 * j + 2) * sizeof(double2), s, j, m, hc, col, H, g,
                     cs, sn, st, pass);
}
void blas_scale_by_state(double2* y, const GmState* st, int64_t N, hipStream_t s) {
  hipLaunchKernelGGL(k_scale_by_state, g1(N), dim3(256), 0, s, y, st, N);
}

void blas_phase_real(const double2* J, int64_t ldj, int m, const double2* ph, double2* W, int64_t ldw, int64_t N,
                     hipStream_t s) {
  hipLaunchKernelGGL(k_phase_real, g1(N * m), dim3(256), 0, s, J, ldj, m, ph, W, ldw, N);
}
void blas_split_reim(const double2* J, int64_t ldj, int m, double2* W, int64_t ldw, int64_t N, hipStream_t s) {
  hipLaunchKernelGGL(k_split_reim, g1(N * m), dim3(256), 0, s, J, ldj, m, W, ldw, N);
}
void blas_rowmix(const double2* A, int64_t lda, int na, const double2* M, int nb, double2* Out, int64_t ldo,
                 int64_t N, hipStream_t s) {
  hipLaunchKernelGGL(k_rowmix, g1(N * nb), dim3(256), 0, s, A, lda, na, M, nb, Out, ldo, N);
}
void blas_scale_cols(double2* A, int64_t lda, int m, const double* sc, int64_t N, hipStream_t s) {
  hipLaunchKernelGGL(k_scale_cols, g1(N * m), dim3(256), 0, s, A, lda, m, sc, N);
}

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
// blocks of the all-CU multidot, and the size of its partial buffer in units
// of nk complex values
int blas_multidot_blocks(int64_t N) { return (int)std::max<int64_t>(1, std::min<int64_t>(256, (N + 511) / 512)); }
void blas_multidot_wide(const double2* V, int64_t ldv, const double2* w, int64_t N, int nk, double2* part,
                        double2* h, const int* flag, hipStream_t s) {
  if (nk <= 0) return;
  const int nblk = blas_multidot_blocks(N);
  const int64_t rpb = (N + nblk - 1) / nblk;
  hipLaunchKernelGGL(k_multidot_part<8>, dim3(nblk), dim3(256), 0, s, V, ldv, w, N, nk, rpb, part, flag);
  hipLaunchKernelGGL(k_multidot_final, dim3((nk + 255) / 256), dim3(256), 0, s, part, nblk, nk, h, flag);
}
void blas_gemv_sub(const double2* V, int64_t ldv, const double2* h, int nk, double2* w, int64_t N, hipStream_t s,
                   const int* flag) {
  if (nk > 0) hipLaunchKernelGGL(k_gemv_sub, g1(N), dim3(256), 0, s, V, ldv, h, nk, w, N, flag);
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

// y = M x, M real CSR, x and y complex double; one row per thread (the
// Calderon matrices hold a few tens of entries per row)
__global__ void __launch_bounds__(256) k_csr_real(int64_t rows, const int64_t* __restrict__ ptr,
                                                  const int32_t* __restrict__ col, const double* __restrict__ val,
                                                  const double2* __restrict__ x, double2* __restrict__ y) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= rows) return;
  double ax = 0.0, ay = 0.0;
  for (int64_t p = ptr[i]; p < ptr[i + 1]; ++p) {
    const double v = val[p];
    const double2 xv = x[col[p]];
    ax = fma(v, xv.x, ax);
    ay = fma(v, xv.y, ay);
  }
  y[i] = make_double2(ax, ay);
}

void blas_csr_real(const CsrD& M, const double2* x, double2* y, hipStream_t s) {
  if (M.rows > 0) hipLaunchKernelGGL(k_csr_real, g1(M.rows), dim3(256), 0, s, M.rows, M.ptr, M.col, M.val, x, y);
}

}  // namespace cm
