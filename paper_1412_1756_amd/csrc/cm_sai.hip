// SAI preconditioner build on the device (section IV): P minimises
// ||I - Z_near P||_F column by column over a prescribed pattern.  Thresholds
// (the paper does not define them): Z~ drops entries |z_ij| < eps1 |z_jj| of
// column j; column j of P lives on J_j = {i : |z_ij| >= eps2 |z_jj|}; the
// rows taking part are I_j, the nonzero rows of Z~(:, J_j); entries
// |p_ij| < eps3 max_i |p_ij| are dropped after the solve.  The same
// construction serves the near field of the shifted operator tau R + i X of
// the Arnoldi inner solves (tau Re Z_near + i Im Z_near; tau = 0: the real
// X_near).
//
// Z_near is symmetric, so column j is row j of the stored near field (the
// leaf box's column list, ascending internal indices).  One wave per column:
//   pass 1 (k_sai_count): |J_j| and |I_j|;
//   pass 2 (k_sai_solve): J_j, the row set I_j as a bitmap in LDS over the
//     leaf boxes within twice the near radius of j's box (a local grid of
//     (4 nr + 1)^3 box slots of max_box unknowns each; ranks by a prefix
//     count of the bitmap words, so I_j is ordered by box slot and unknown),
//     the m x n least-squares matrix Z~(I_j, J_j) in a per-wave scratch slab,
//     Householder QR with the reflector's phase chosen against cancellation,
//     back substitution (pivots below 1e-14 of the largest give 0), the eps3
//     drop, and the kept entries of column j;
//   then the columns are transposed to CSR by rows (ascending columns per
//   row) for the apply.  Nothing of the near field goes to the host.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <numeric>
#include <vector>

#include "cm_device.h"

namespace cm {

static void chk_s(hipError_t e, const char* what) {
  if (e != hipSuccess) throw Error(-4, std::string(what) + ": " + hipGetErrorString(e));
}

// device buffers of the build, freed on every exit path
struct SaiTmp {
  std::vector<void*> p;
  template <typename T>
  T* alloc(size_t n) {
    void* q = nullptr;
    chk_s(hipMalloc(&q, std::max<size_t>(1, n) * sizeof(T)), "SAI build: hipMalloc");
    p.push_back(q);
    return (T*)q;
  }
  ~SaiTmp() {
    for (void* q : p) (void)hipFree(q);
  }
};

struct SaiArgs {
  const int64_t* row_ptr;
  const int32_t* box_of;
  const int32_t* box_start;
  const int32_t* bcol_ptr;
  const int32_t* bcol;
  const int32_t* ijk;       // 3 x nleaf leaf box coordinates
  const double2* Zn;
  const double* diag;       // |z_jj| of the transformed near field
  double e1, e2, e3, tau;
  int64_t N;
  int R2, G, max_box, nwords;   // local grid radius (2 nr), side, unknowns per slot, bitmap words
};

__device__ __forceinline__ double2 sai_val(double2 z, double tau) {
  return tau == 1.0 ? z : (tau == 0.0 ? make_double2(z.y, 0.0) : make_double2(tau * z.x, z.y));
}
__device__ __forceinline__ bool nz(double2 v) { return v.x != 0.0 || v.y != 0.0; }
__device__ __forceinline__ double wsum(double v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}
__device__ __forceinline__ double wmax(double v) {
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
  return v;
}
__device__ __forceinline__ int wsumi(int v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}
// memory written by some lanes of the wave is read by others next
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
}

__global__ void k_sai_diag(SaiArgs a, double* diag) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= a.N) return;
  const int b = a.box_of[i];
  const int32_t* c = a.bcol + a.bcol_ptr[b];
  int lo = 0, hi = a.bcol_ptr[b + 1] - a.bcol_ptr[b];
  while (lo < hi) {   // position of i in its row
    const int mid = (lo + hi) >> 1;
    if (c[mid] < i) lo = mid + 1; else hi = mid;
  }
  const double2 v = sai_val(a.Zn[a.row_ptr[i] + lo], a.tau);
  diag[i] = hypot(v.x, v.y);
}

// local bitmap index of unknown c relative to the box bj (-1: outside the grid)
__device__ __forceinline__ int sai_local(const SaiArgs& a, int32_t c, int bj) {
  const int b = a.box_of[c];
  const int dx = a.ijk[3 * b] - a.ijk[3 * bj] + a.R2, dy = a.ijk[3 * b + 1] - a.ijk[3 * bj + 1] + a.R2,
            dz = a.ijk[3 * b + 2] - a.ijk[3 * bj + 2] + a.R2;
  if (dx < 0 || dy < 0 || dz < 0 || dx >= a.G || dy >= a.G || dz >= a.G) return -1;
  return ((dx * a.G + dy) * a.G + dz) * a.max_box + (c - a.box_start[b]);
}

// J_j into Jg (if non-null) and its size; the I_j bitmap into bm (cleared
// first), returns m = |I_j| through *m_out; *bad set when an entry falls
// outside the local grid (cannot happen for the near lists built here)
__device__ int sai_pattern(const SaiArgs& a, int64_t j, int32_t* Jg, int nmax, unsigned* bm, int* m_out,
                           int* bad) {
  const int lane = threadIdx.x & 63;
  const int bj = a.box_of[j];
  const int32_t* cj = a.bcol + a.bcol_ptr[bj];
  const int nj = a.bcol_ptr[bj + 1] - a.bcol_ptr[bj];
  const double2* vj = a.Zn + a.row_ptr[j];
  const double tj = a.e2 * a.diag[j];
  int n = 0;
  for (int e0 = 0; e0 < nj; e0 += 64) {
    const int e = e0 + lane;
    bool keep = false;
    if (e < nj) {
      const double2 v = sai_val(vj[e], a.tau);
      keep = hypot(v.x, v.y) >= tj && nz(v);
    }
    const unsigned long long bal = __ballot(keep);
    if (keep && Jg) {
      const int pos = n + __popcll(bal & ((1ull << lane) - 1ull));
      if (pos < nmax) Jg[pos] = cj[e];
    }
    n += __popcll(bal);
  }
  for (int w = lane; w < a.nwords; w += 64) bm[w] = 0u;
  wave_sync();
  // rows of Z~(:, J_j): walk the rows a in J_j again from the row of j
  int nbad = 0;
  for (int e0 = 0; e0 < nj; e0 += 64) {
    const int e = e0 + lane;
    bool keep = false;
    if (e < nj) {
      const double2 v = sai_val(vj[e], a.tau);
      keep = hypot(v.x, v.y) >= tj && nz(v);
    }
    unsigned long long bal = __ballot(keep);
    while (bal) {   // uniform: one member a of J_j at a time, its row over the lanes
      const int l = __ffsll((long long)bal) - 1;
      bal &= bal - 1ull;
      const int32_t ra = cj[e0 + l];
      const int ba = a.box_of[ra];
      const int32_t* ca = a.bcol + a.bcol_ptr[ba];
      const int na = a.bcol_ptr[ba + 1] - a.bcol_ptr[ba];
      const double2* va = a.Zn + a.row_ptr[ra];
      const double ta = a.e1 * a.diag[ra];
      for (int f = lane; f < na; f += 64) {
        const double2 v = sai_val(va[f], a.tau);
        if (hypot(v.x, v.y) >= ta && nz(v)) {
          const int loc = sai_local(a, ca[f], bj);
          if (loc < 0)
            ++nbad;
          else
            atomicOr(&bm[loc >> 5], 1u << (loc & 31));
        }
      }
    }
  }
  wave_sync();
  int m = 0;
  for (int w = lane; w < a.nwords; w += 64) m += __popc(bm[w]);
  *m_out = wsumi(m);
  *bad = wsumi(nbad);
  return n;
}

// pass 1: n_j = |J_j|, m_j = |I_j| (one wave per column)
__global__ void __launch_bounds__(256) k_sai_count(SaiArgs a, int32_t* nj_out, int32_t* mj_out, int* bad) {
  extern __shared__ unsigned sh_bm[];
  const int w = threadIdx.x >> 6;
  const int64_t j = (int64_t)blockIdx.x * (blockDim.x >> 6) + w;
  if (j >= a.N) return;
  int m, nb;
  const int n = sai_pattern(a, j, nullptr, 0, sh_bm + (size_t)w * a.nwords, &m, &nb);
  if ((threadIdx.x & 63) == 0) {
    nj_out[j] = n;
    mj_out[j] = m;
    if (nb) atomicAdd(bad, nb);
  }
}

// pass 2: the least-squares solve of every column; kept entries of column j
// go to (prow, pval)[cptr[j] ..], their count to pcnt[j].  Scratch per wave:
// nmax ints (J_j) + mn_max complex (A) + 2 mmax complex (v, b) + nmax complex (p).
__global__ void __launch_bounds__(256) k_sai_solve(SaiArgs a, const int64_t* __restrict__ cptr, int nmax, int mmax,
                                                   int64_t mn_max, char* scratch, int64_t slab, int32_t* prow,
                                                   double2* pval, int32_t* pcnt) {
  extern __shared__ unsigned sh[];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, wpb = blockDim.x >> 6;
  unsigned* bm = sh + (size_t)w * 2 * a.nwords;
  unsigned* pre = bm + a.nwords;   // exclusive prefix counts of the bitmap words
  char* base = scratch + ((int64_t)blockIdx.x * wpb + w) * slab;
  int32_t* J = reinterpret_cast<int32_t*>(base);
  double2* A = reinterpret_cast<double2*>(base + (((int64_t)nmax * 4 + 15) / 16) * 16);
  double2* V = A + mn_max;
  double2* B = V + mmax;
  double2* Pv = B + mmax;
  const int64_t stride = (int64_t)gridDim.x * wpb;
  for (int64_t j = (int64_t)blockIdx.x * wpb + w; j < a.N; j += stride) {
    int m, nb;
    const int n = min(sai_pattern(a, j, J, nmax, bm, &m, &nb), nmax);
    if (n == 0 || m == 0 || m > mmax) {
      if (lane == 0) pcnt[j] = 0;
      continue;
    }
    // ranks of the bitmap
    {
      unsigned run = 0;
      for (int w0 = 0; w0 < a.nwords; w0 += 64) {
        const int ww = w0 + lane;
        const unsigned c = ww < a.nwords ? (unsigned)__popc(bm[ww]) : 0u;
        unsigned x = c;   // inclusive scan over the wave
        for (int o = 1; o < 64; o <<= 1) {
          const unsigned y = __shfl_up(x, o, 64);
          if (lane >= o) x += y;
        }
        if (ww < a.nwords) pre[ww] = run + x - c;
        run += __shfl(x, 63, 64);
      }
    }
    const int bj = a.box_of[j];
    auto rank = [&](int loc) -> int {
      const unsigned wv = bm[loc >> 5], bit = 1u << (loc & 31);
      return (wv & bit) ? (int)(pre[loc >> 5] + __popc(wv & (bit - 1u))) : -1;
    };
    // A = Z~(I_j, J_j), column-major m x n; b = e_j on I_j
    for (int64_t t = lane; t < (int64_t)m * n; t += 64) A[t] = make_double2(0.0, 0.0);
    for (int t = lane; t < m; t += 64) B[t] = make_double2(0.0, 0.0);
    wave_sync();
    for (int p = 0; p < n; ++p) {
      const int32_t ra = J[p];
      const int ba = a.box_of[ra];
      const int32_t* ca = a.bcol + a.bcol_ptr[ba];
      const int na = a.bcol_ptr[ba + 1] - a.bcol_ptr[ba];
      const double2* va = a.Zn + a.row_ptr[ra];
      const double ta = a.e1 * a.diag[ra];
      for (int f = lane; f < na; f += 64) {
        const double2 v = sai_val(va[f], a.tau);
        if (hypot(v.x, v.y) >= ta && nz(v)) {
          const int loc = sai_local(a, ca[f], bj);
          if (loc >= 0) A[(int64_t)p * m + rank(loc)] = v;
        }
      }
    }
    if (lane == 0) {
      const int rj = rank(sai_local(a, (int32_t)j, bj));
      if (rj >= 0) B[rj] = make_double2(1.0, 0.0);
    }
    wave_sync();
    // Householder QR, the reflectors applied to the columns and to b
    const int kmax = min(m, n);
    for (int k = 0; k < kmax; ++k) {
      double s2 = 0.0;
      for (int i = k + lane; i < m; i += 64) {
        const double2 z = A[(int64_t)k * m + i];
        s2 += z.x * z.x + z.y * z.y;
      }
      const double nx = sqrt(wsum(s2));
      if (nx == 0.0) continue;
      const double2 x0 = A[(int64_t)k * m + k];
      const double ax0 = hypot(x0.x, x0.y);
      const double2 ph = ax0 > 0.0 ? make_double2(x0.x / ax0, x0.y / ax0) : make_double2(1.0, 0.0);
      const double2 alpha = make_double2(-ph.x * nx, -ph.y * nx);
      double v2 = 0.0;
      for (int i = k + lane; i < m; i += 64) {
        double2 z = A[(int64_t)k * m + i];
        if (i == k) z = make_double2(z.x - alpha.x, z.y - alpha.y);
        V[i] = z;
        v2 += z.x * z.x + z.y * z.y;
      }
      const double nv = sqrt(wsum(v2));
      if (nv == 0.0) continue;
      for (int i = k + lane; i < m; i += 64) V[i] = make_double2(V[i].x / nv, V[i].y / nv);
      wave_sync();
      for (int c = k; c <= n; ++c) {   // c == n: the right-hand side
        double2* col = (c < n) ? A + (int64_t)c * m : B;
        double sx = 0.0, sy = 0.0;   // s = v^H col
        for (int i = k + lane; i < m; i += 64) {
          const double2 v = V[i], z = col[i];
          sx += v.x * z.x + v.y * z.y;
          sy += v.x * z.y - v.y * z.x;
        }
        sx = wsum(sx);
        sy = wsum(sy);
        for (int i = k + lane; i < m; i += 64) {
          const double2 v = V[i];
          double2 z = col[i];
          z.x -= 2.0 * (v.x * sx - v.y * sy);
          z.y -= 2.0 * (v.x * sy + v.y * sx);
          col[i] = z;
        }
      }
      wave_sync();
    }
    // back substitution (lane 0), pivots below 1e-14 of the largest give 0
    if (lane == 0) {
      double rmax = 0.0;
      for (int k = 0; k < kmax; ++k) {
        const double2 r = A[(int64_t)k * m + k];
        rmax = fmax(rmax, hypot(r.x, r.y));
      }
      for (int c = kmax; c < n; ++c) Pv[c] = make_double2(0.0, 0.0);
      for (int k = kmax - 1; k >= 0; --k) {
        double2 s = B[k];
        for (int c = k + 1; c < n; ++c) {
          const double2 r = A[(int64_t)c * m + k], p = Pv[c];
          s.x -= r.x * p.x - r.y * p.y;
          s.y -= r.x * p.y + r.y * p.x;
        }
        const double2 r = A[(int64_t)k * m + k];
        const double ar = hypot(r.x, r.y);
        if (ar > 1e-14 * rmax) {
          const double d = r.x * r.x + r.y * r.y;
          Pv[k] = make_double2((s.x * r.x + s.y * r.y) / d, (s.y * r.x - s.x * r.y) / d);
        } else {
          Pv[k] = make_double2(0.0, 0.0);
        }
      }
    }
    wave_sync();
    double pm = 0.0;
    for (int c = lane; c < n; c += 64) pm = fmax(pm, hypot(Pv[c].x, Pv[c].y));
    pm = wmax(pm);
    int cnt = 0;
    for (int c0 = 0; c0 < n; c0 += 64) {
      const int c = c0 + lane;
      bool keep = false;
      double2 p = make_double2(0.0, 0.0);
      if (c < n) {
        p = Pv[c];
        const double ap = hypot(p.x, p.y);
        keep = ap >= a.e3 * pm && ap > 0.0;
      }
      const unsigned long long bal = __ballot(keep);
      if (keep) {
        const int64_t at = cptr[j] + cnt + __popcll(bal & ((1ull << lane) - 1ull));
        prow[at] = J[c];
        pval[at] = p;
      }
      cnt += __popcll(bal);
    }
    if (lane == 0) pcnt[j] = cnt;
    wave_sync();
  }
}

__global__ void k_sai_rowcount(const int64_t* cptr, const int32_t* pcnt, const int32_t* prow, int64_t N,
                               int32_t* rc) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= N) return;
  for (int t = 0; t < pcnt[j]; ++t) atomicAdd(&rc[prow[cptr[j] + t]], 1);
}

__global__ void k_sai_scatter(const int64_t* cptr, const int32_t* pcnt, const int32_t* prow, const double2* pval,
                              int64_t N, const int64_t* rptr, int32_t* fill, int32_t* col, double2* val) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= N) return;
  for (int t = 0; t < pcnt[j]; ++t) {
    const int32_t i = prow[cptr[j] + t];
    const int64_t at = rptr[i] + atomicAdd(&fill[i], 1);
    col[at] = (int32_t)j;
    val[at] = pval[cptr[j] + t];
  }
}

// ascending columns in every row (insertion sort: rows hold tens of entries)
__global__ void k_sai_rowsort(const int64_t* rptr, int64_t N, int32_t* col, double2* val) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N) return;
  for (int64_t t = rptr[i] + 1; t < rptr[i + 1]; ++t) {
    const int32_t c = col[t];
    const double2 v = val[t];
    int64_t u = t - 1;
    while (u >= rptr[i] && col[u] > c) {
      col[u + 1] = col[u];
      val[u + 1] = val[u];
      --u;
    }
    col[u + 1] = c;
    val[u + 1] = v;
  }
}

void dev_sai_build(Dev& d, const Plan& P, double e1, double e2, double e3, double tau, hipStream_t s) {
  const int part = sai_slot(tau);
  const int64_t N = d.N;
  const Level& Lf = P.lev[P.lf];
  // near radius of the stored near field (Chebyshev, in leaf boxes)
  int nr = 0;
  for (int b = 0; b < Lf.nbox; ++b)
    for (int e = P.near_ptr[b]; e < P.near_ptr[b + 1]; ++e) {
      const int q = P.near_box[e];
      for (int c = 0; c < 3; ++c) nr = std::max(nr, std::abs(Lf.ijk[3 * q + c] - Lf.ijk[3 * b + c]));
    }
  SaiTmp tmp;
  SaiArgs a;
  a.row_ptr = d.row_ptr;
  a.box_of = d.box_of;
  a.box_start = d.box_start;
  a.bcol_ptr = d.bcol_ptr;
  a.bcol = d.bcol;
  int32_t* ijk = tmp.alloc<int32_t>(Lf.ijk.size());
  chk_s(hipMemcpyAsync(ijk, Lf.ijk.data(), Lf.ijk.size() * sizeof(int32_t), hipMemcpyHostToDevice, s), "SAI: ijk");
  a.ijk = ijk;
  a.Zn = d.Zn;
  double* diag = tmp.alloc<double>(N);
  a.diag = diag;
  a.e1 = e1;
  a.e2 = e2;
  a.e3 = e3;
  a.tau = tau;
  a.N = N;
  a.R2 = 2 * nr;
  a.G = 4 * nr + 1;
  a.max_box = std::max(1, d.max_box);
  const int64_t nbits = (int64_t)a.G * a.G * a.G * a.max_box;
  a.nwords = (int)((nbits + 31) / 32);
  const size_t wbytes = (size_t)a.nwords * sizeof(unsigned);
  if (2 * wbytes > 160 * 1024) throw Error(-7, "SAI build: leaf boxes too populated for the row bitmap");
  hipLaunchKernelGGL(k_sai_diag, dim3((unsigned)((N + 255) / 256)), dim3(256), 0, s, a, diag);
  chk_s(hipGetLastError(), "SAI: diag");
  // pass 1: pattern sizes
  const int wpb1 = (int)std::max<size_t>(1, std::min<size_t>(4, (64 * 1024) / wbytes));
  int32_t* nj = tmp.alloc<int32_t>(N);
  int32_t* mj = tmp.alloc<int32_t>(N);
  int* bad = tmp.alloc<int>(1);
  chk_s(hipMemsetAsync(bad, 0, sizeof(int), s), "SAI: memset");
  const size_t sh1 = wpb1 * wbytes;
  if (sh1 > 64 * 1024)
    chk_s(hipFuncSetAttribute((const void*)k_sai_count, hipFuncAttributeMaxDynamicSharedMemorySize, (int)sh1),
          "SAI: LDS limit");
  hipLaunchKernelGGL(k_sai_count, dim3((unsigned)((N + wpb1 - 1) / wpb1)), dim3(64 * wpb1), sh1, s, a, nj, mj, bad);
  chk_s(hipGetLastError(), "SAI: count");
  std::vector<int32_t> hn(N), hm(N);
  int hbad = 0;
  chk_s(hipMemcpyAsync(hn.data(), nj, N * sizeof(int32_t), hipMemcpyDeviceToHost, s), "SAI: sizes");
  chk_s(hipMemcpyAsync(hm.data(), mj, N * sizeof(int32_t), hipMemcpyDeviceToHost, s), "SAI: sizes");
  chk_s(hipMemcpyAsync(&hbad, bad, sizeof(int), hipMemcpyDeviceToHost, s), "SAI: sizes");
  chk_s(hipStreamSynchronize(s), "SAI: sizes");
  if (hbad) throw Error(-6, "SAI build: a near-field entry lies outside the local box grid");
  int nmax = 1, mmax = 1;
  int64_t mn_max = 1;
  std::vector<int64_t> cptr(N + 1, 0);
  for (int64_t j = 0; j < N; ++j) {
    nmax = std::max(nmax, hn[j]);
    mmax = std::max(mmax, hm[j]);
    mn_max = std::max(mn_max, (int64_t)hn[j] * hm[j]);
    cptr[j + 1] = cptr[j] + hn[j];
  }
  // pass 2: the solves, in a grid sized so that the scratch slabs stay below
  // about 2 GB
  const int64_t slab = (((int64_t)nmax * 4 + 15) / 16) * 16 + (mn_max + 2 * (int64_t)mmax + nmax) * 16;
  const int wpb2 = (int)std::max<size_t>(1, std::min<size_t>(4, (64 * 1024) / (2 * wbytes)));
  int64_t nw = std::min<int64_t>(N, std::max<int64_t>(wpb2, ((int64_t)2048 << 20) / slab));
  nw = std::min<int64_t>(nw, 16384);
  const int64_t nblk = (nw + wpb2 - 1) / wpb2;
  char* scratch = tmp.alloc<char>((size_t)(nblk * wpb2 * slab));
  int64_t* dcptr = tmp.alloc<int64_t>(N + 1);
  chk_s(hipMemcpyAsync(dcptr, cptr.data(), (N + 1) * sizeof(int64_t), hipMemcpyHostToDevice, s), "SAI: cptr");
  int32_t* prow = tmp.alloc<int32_t>(cptr[N]);
  double2* pval = tmp.alloc<double2>(cptr[N]);
  int32_t* pcnt = tmp.alloc<int32_t>(N);
  const size_t sh2 = (size_t)wpb2 * 2 * wbytes;
  if (sh2 > 64 * 1024)
    chk_s(hipFuncSetAttribute((const void*)k_sai_solve, hipFuncAttributeMaxDynamicSharedMemorySize, (int)sh2),
          "SAI: LDS limit");
  hipLaunchKernelGGL(k_sai_solve, dim3((unsigned)nblk), dim3(64 * wpb2), sh2, s, a, (const int64_t*)dcptr, nmax,
                     mmax, mn_max, scratch, slab, prow, pval, pcnt);
  chk_s(hipGetLastError(), "SAI: solve");
  // transpose to CSR by rows
  int32_t* rc = tmp.alloc<int32_t>(N);
  chk_s(hipMemsetAsync(rc, 0, N * sizeof(int32_t), s), "SAI: memset");
  const dim3 g1((unsigned)((N + 255) / 256));
  hipLaunchKernelGGL(k_sai_rowcount, g1, dim3(256), 0, s, (const int64_t*)dcptr, (const int32_t*)pcnt,
                     (const int32_t*)prow, N, rc);
  chk_s(hipGetLastError(), "SAI: row counts");
  std::vector<int32_t> hrc(N);
  chk_s(hipMemcpyAsync(hrc.data(), rc, N * sizeof(int32_t), hipMemcpyDeviceToHost, s), "SAI: row counts");
  chk_s(hipStreamSynchronize(s), "SAI: row counts");
  std::vector<int64_t> ptr(N + 1, 0);
  for (int64_t i = 0; i < N; ++i) ptr[i + 1] = ptr[i] + hrc[i];
  const int64_t nnz = ptr[N];
  SaiD& q = d.sai[part];
  if (q.ptr) {
    (void)hipFree(q.ptr);
    (void)hipFree(q.col);
    (void)hipFree(q.val);
    q = SaiD();
  }
  SaiD nq;
  chk_s(hipMalloc(&nq.ptr, (N + 1) * sizeof(int64_t)), "SAI alloc");
  chk_s(hipMalloc(&nq.col, std::max<int64_t>(1, nnz) * sizeof(int32_t)), "SAI alloc");
  chk_s(hipMalloc(&nq.val, std::max<int64_t>(1, nnz) * sizeof(double2)), "SAI alloc");
  q = nq;
  chk_s(hipMemcpyAsync(q.ptr, ptr.data(), (N + 1) * sizeof(int64_t), hipMemcpyHostToDevice, s), "SAI upload");
  chk_s(hipMemsetAsync(rc, 0, N * sizeof(int32_t), s), "SAI: memset");
  hipLaunchKernelGGL(k_sai_scatter, g1, dim3(256), 0, s, (const int64_t*)dcptr, (const int32_t*)pcnt,
                     (const int32_t*)prow, (const double2*)pval, N, (const int64_t*)q.ptr, rc, q.col, q.val);
  chk_s(hipGetLastError(), "SAI: scatter");
  hipLaunchKernelGGL(k_sai_rowsort, g1, dim3(256), 0, s, (const int64_t*)q.ptr, N, q.col, q.val);
  chk_s(hipGetLastError(), "SAI: row sort");
  chk_s(hipStreamSynchronize(s), "SAI: build");
  q.nnz = nnz;
  if (part == 1) d.sai_tau1 = tau;
}

}  // namespace cm
