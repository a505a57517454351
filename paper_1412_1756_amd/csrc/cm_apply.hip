// Matrix-vector kernels of the MLFMA (section III, eqs. (11), (18), (22)):
// near-field sparse product, leaf aggregation, interpolation + centre shift up
// the tree, diagonal translation, shift + anterpolation down the tree,
// disaggregation/testing.  Templated on the far-field real type R (float for
// the FP32 batched path, double for the FP64 path); the near field is always
// stored and accumulated in FP64.
//
// Pattern layout at level l: [box][component (theta, phi)][direction q][column c],
// q = t * np + p (theta-major), columns innermost so that a batch of right-hand
// sides shares every translator, interpolation weight and leaf pattern load.
#include <hip/hip_runtime.h>

#include "cm_device.h"

namespace cm {

template <typename R>
struct C2 {
  R x, y;
};
template <typename R>
__device__ __forceinline__ C2<R> mk(R a, R b) {
  return C2<R>{a, b};
}
template <typename R>
__device__ __forceinline__ C2<R> cmul(C2<R> a, C2<R> b) {
  return C2<R>{a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
template <typename R>
__device__ __forceinline__ C2<R> cfma(C2<R> acc, C2<R> a, C2<R> b) {
  acc.x = fma(a.x, b.x, acc.x);
  acc.x = fma(-a.y, b.y, acc.x);
  acc.y = fma(a.x, b.y, acc.y);
  acc.y = fma(a.y, b.x, acc.y);
  return acc;
}
// acc += conj(a) * b
template <typename R>
__device__ __forceinline__ C2<R> cfma_conj(C2<R> acc, C2<R> a, C2<R> b) {
  acc.x = fma(a.x, b.x, acc.x);
  acc.x = fma(a.y, b.y, acc.x);
  acc.y = fma(a.x, b.y, acc.y);
  acc.y = fma(-a.y, b.x, acc.y);
  return acc;
}
template <typename R>
__device__ __forceinline__ C2<R> cscale(R s, C2<R> a) {
  return C2<R>{s * a.x, s * a.y};
}

__device__ __forceinline__ int pow2ceil(int n) {
  int p = 1;
  while (p < n) p <<= 1;
  return p;
}

// ---------------------------------------------------------------- permutation
// x (public order, row stride ld) -> xi (internal order, nc contiguous)
template <typename R>
__global__ void __launch_bounds__(256) k_permute_in(const C2<R>* __restrict__ x, int64_t ld, int nc,
                                                    const int32_t* __restrict__ perm, C2<R>* __restrict__ xi,
                                                    int64_t N, int conj_in) {
  int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= N * nc) return;
  int64_t i = g / nc;
  int c = (int)(g % nc);
  C2<R> v = x[(int64_t)perm[i] * ld + c];
  if (conj_in) v.y = -v.y;
  xi[g] = v;
}

// ---------------------------------------------------------------- near field
// One 64-lane wavefront per row.  Lane (s, c): c = column of the batch,
// s = slice of the row's nonzeros (stride S = 64/NC); slices are summed with
// cross-lane shuffles.  mode 0: Z_near, 1: Re Z_near restricted to the own
// leaf box (R), 2: Im Z_near (X).  FP64 products and sums.
template <typename R>
__global__ void __launch_bounds__(256) k_near(const int64_t* __restrict__ row_ptr, const int32_t* __restrict__ box_of,
                                              const int32_t* __restrict__ bcol_ptr, const int32_t* __restrict__ bcol,
                                              const int32_t* __restrict__ self_off,
                                              const int32_t* __restrict__ box_start, const double2* __restrict__ Zn,
                                              const C2<R>* __restrict__ xi, C2<R>* __restrict__ yi, int64_t N, int nc,
                                              int mode) {
  const int lane = threadIdx.x & 63;
  const int64_t i = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
  if (i >= N) return;
  const int NC = pow2ceil(nc);
  const int S = 64 / NC;
  const int c = lane % NC, s = lane / NC;
  const int b = box_of[i];
  const int32_t* cols = bcol + bcol_ptr[b];
  int t0 = 0, t1 = bcol_ptr[b + 1] - bcol_ptr[b];
  if (mode == 1) {
    t0 = self_off[b];
    t1 = t0 + (box_start[b + 1] - box_start[b]);
  }
  const double2* z = Zn + row_ptr[i];
  double ax = 0.0, ay = 0.0;
  if (c < nc) {
    for (int t = t0 + s; t < t1; t += S) {
      double2 v = z[t];
      if (mode == 1) v.y = 0.0;
      if (mode == 2) {
        v.x = v.y;
        v.y = 0.0;
      }
      C2<R> xv = xi[(int64_t)cols[t] * nc + c];
      double xr = (double)xv.x, xim = (double)xv.y;
      ax = fma(v.x, xr, ax);
      ax = fma(-v.y, xim, ax);
      ay = fma(v.x, xim, ay);
      ay = fma(v.y, xr, ay);
    }
  }
  for (int o = NC; o < 64; o <<= 1) {
    ax += __shfl_xor(ax, o, 64);
    ay += __shfl_xor(ay, o, 64);
  }
  if (s == 0 && c < nc) yi[i * nc + c] = mk<R>((R)ax, (R)ay);
}

// ---------------------------------------------------------------- aggregation
// S_b(q) = sum_{j in box b} V_j(q) x_j  (eq. (13) summed over the box), 2 components
template <typename R>
__global__ void __launch_bounds__(256) k_aggregate(const C2<R>* __restrict__ V, const C2<R>* __restrict__ xi,
                                                   C2<R>* __restrict__ S, const int32_t* __restrict__ box_start,
                                                   int K, int nc) {
  const int b = blockIdx.x;
  const int j0 = box_start[b], j1 = box_start[b + 1];
  const int tot = 2 * K * nc;
  for (int o = blockIdx.y * blockDim.x + threadIdx.x; o < tot; o += gridDim.y * blockDim.x) {
    const int c = o % nc, cq = o / nc;
    C2<R> acc = mk<R>(0, 0);
    for (int j = j0; j < j1; ++j) acc = cfma(acc, V[(int64_t)j * 2 * K + cq], xi[(int64_t)j * nc + c]);
    S[(int64_t)b * tot + o] = acc;
  }
}

// ---------------------------------------------------------------- interpolation up
// S_parent(q) = sum_children exp(ik khat_q.(r_c - r_p)) [I_phi I_theta S_child](q)
// theta first (child theta -> parent theta, with pole reflections), then phi.
template <typename R>
__global__ void __launch_bounds__(256) k_interp_up(const C2<R>* __restrict__ Sc, C2<R>* __restrict__ Sp,
                                                   const int32_t* __restrict__ child_ptr,
                                                   const int8_t* __restrict__ octant, LevelD<R> P, int Kc, int nc) {
  extern __shared__ unsigned char smem_raw[];
  C2<R>* tmp = reinterpret_cast<C2<R>*>(smem_raw);   // [2][ntp][npc]
  const int m = blockIdx.x, c = blockIdx.y;
  const int ntp = P.nt, npp = P.np, ntc = P.ntc, npc = P.npc, p = P.p, Kp = P.K;
  const int half = npc / 2;
  const C2<R>* shift = reinterpret_cast<const C2<R>*>(P.shift);
  C2<R>* out = Sp + (int64_t)m * 2 * Kp * nc;
  for (int e = threadIdx.x; e < 2 * Kp; e += blockDim.x) out[(int64_t)e * nc + c] = mk<R>(0, 0);
  for (int ch = child_ptr[m]; ch < child_ptr[m + 1]; ++ch) {
    const C2<R>* src = Sc + (int64_t)ch * 2 * Kc * nc;
    const int oc = octant[ch];
    __syncthreads();
    for (int e = threadIdx.x; e < 2 * ntp * npc; e += blockDim.x) {
      const int uc = e % npc, tp = (e / npc) % ntp, comp = e / (npc * ntp);
      C2<R> acc = mk<R>(0, 0);
      for (int j = 0; j < p; ++j) {
        const int tc = P.th_idx[tp * p + j];
        const int rf = P.th_ref[tp * p + j];
        const R w = rf ? -P.th_w[tp * p + j] : P.th_w[tp * p + j];
        const int u = rf ? (uc + half) % npc : uc;
        const C2<R> v = src[((int64_t)comp * Kc + tc * npc + u) * nc + c];
        acc.x = fma(w, v.x, acc.x);
        acc.y = fma(w, v.y, acc.y);
      }
      tmp[e] = acc;
    }
    __syncthreads();
    for (int e = threadIdx.x; e < 2 * Kp; e += blockDim.x) {
      const int up = e % npp, tp = (e / npp) % ntp, comp = e / (npp * ntp);
      const C2<R>* row = tmp + (comp * ntp + tp) * npc;
      C2<R> acc = mk<R>(0, 0);
      for (int j = 0; j < p; ++j) {
        const R w = P.ph_w[up * p + j];
        const C2<R> v = row[P.ph_idx[up * p + j]];
        acc.x = fma(w, v.x, acc.x);
        acc.y = fma(w, v.y, acc.y);
      }
      const C2<R> sh = shift[oc * Kp + tp * npp + up];
      C2<R>& o = out[(int64_t)e * nc + c];
      o = cfma(o, acc, sh);
    }
  }
}

// ---------------------------------------------------------------- translation
// G_m(q) (+)= sum_{m' in list(m)} T_off(m,m')(q) S_m'(q)  (eq. (10)/(16)/(20), diagonal)
template <typename R>
__global__ void __launch_bounds__(256) k_m2l(const int32_t* __restrict__ ptr, const int32_t* __restrict__ src,
                                             const int32_t* __restrict__ off, const C2<R>* __restrict__ T,
                                             const C2<R>* __restrict__ S, C2<R>* __restrict__ G, int K, int nc) {
  const int m = blockIdx.x;
  const int tot = 2 * K * nc;
  const int o = blockIdx.y * blockDim.x + threadIdx.x;
  if (o >= tot) return;
  const int q = (o / nc) % K;
  C2<R> acc = mk<R>(0, 0);
  for (int e = ptr[m]; e < ptr[m + 1]; ++e)
    acc = cfma(acc, T[(int64_t)off[e] * K + q], S[(int64_t)src[e] * tot + o]);
  G[(int64_t)m * tot + o] = acc;
}

// ---------------------------------------------------------------- anterpolation down
// G_child += A [exp(-ik khat.(r_c - r_p)) G_parent],  A = W_c^-1 I^T W_p (gather form)
template <typename R>
__global__ void __launch_bounds__(256) k_anterp_down(const C2<R>* __restrict__ Gp, C2<R>* __restrict__ Gc,
                                                     const int32_t* __restrict__ parent,
                                                     const int8_t* __restrict__ octant, LevelD<R> P, int Kc, int nc) {
  extern __shared__ unsigned char smem_raw[];
  C2<R>* tmp = reinterpret_cast<C2<R>*>(smem_raw);   // [2][ntp][npc]
  const int ch = blockIdx.x, c = blockIdx.y;
  const int ntp = P.nt, npp = P.np, ntc = P.ntc, npc = P.npc, Kp = P.K;
  const int half = npc / 2;
  const int m = parent[ch], oc = octant[ch];
  const C2<R>* shift = reinterpret_cast<const C2<R>*>(P.shift);
  const C2<R>* g = Gp + (int64_t)m * 2 * Kp * nc;
  for (int e = threadIdx.x; e < 2 * ntp * npc; e += blockDim.x) {
    const int uc = e % npc, tp = (e / npc) % ntp, comp = e / (npc * ntp);
    C2<R> acc = mk<R>(0, 0);
    for (int j = P.pht_ptr[uc]; j < P.pht_ptr[uc + 1]; ++j) {
      const int up = P.pht_idx[j];
      const R w = P.pht_w[j];
      const C2<R> v = g[((int64_t)comp * Kp + tp * npp + up) * nc + c];
      const C2<R> sh = shift[oc * Kp + tp * npp + up];
      C2<R> t = mk<R>(0, 0);
      t = cfma_conj(t, sh, v);
      acc.x = fma(w, t.x, acc.x);
      acc.y = fma(w, t.y, acc.y);
    }
    tmp[e] = acc;
  }
  __syncthreads();
  C2<R>* out = Gc + (int64_t)ch * 2 * Kc * nc;
  for (int e = threadIdx.x; e < 2 * Kc; e += blockDim.x) {
    const int uc = e % npc, tc = (e / npc) % ntc, comp = e / (npc * ntc);
    C2<R> acc = mk<R>(0, 0);
    for (int j = P.tht_ptr[tc]; j < P.tht_ptr[tc + 1]; ++j) {
      const int tp = P.tht_idx[j];
      const int rf = P.tht_ref[j];
      const R w = rf ? -P.tht_w[j] : P.tht_w[j];
      const C2<R> v = tmp[(comp * ntp + tp) * npc + (rf ? (uc + half) % npc : uc)];
      acc.x = fma(w, v.x, acc.x);
      acc.y = fma(w, v.y, acc.y);
    }
    C2<R>& o = out[(int64_t)e * nc + c];
    o.x += acc.x;
    o.y += acc.y;
  }
}

// ---------------------------------------------------------------- disaggregation
// y_i = y_near_i + sum_q (k^2 eta/4pi) w_q conj(V_i(q)) . G_box(i)(q), written to
// the public position perm[i] (conjugated for Z^H).  One wavefront per unknown.
template <typename R>
__global__ void __launch_bounds__(256) k_disagg(const C2<R>* __restrict__ V, const C2<R>* __restrict__ G,
                                                const R* __restrict__ qwc, const C2<R>* __restrict__ yi,
                                                const int32_t* __restrict__ box_of, const int32_t* __restrict__ perm,
                                                int K, int nc, int64_t N, C2<R>* __restrict__ y, int64_t ld,
                                                int conj_out) {
  const int lane = threadIdx.x & 63;
  const int64_t i = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
  if (i >= N) return;
  const int NC = pow2ceil(nc);
  const int S = 64 / NC;
  const int c = lane % NC, s = lane / NC;
  const int b = box_of[i];
  const C2<R>* v = V + i * 2 * K;
  const C2<R>* g = G + (int64_t)b * 2 * K * nc;
  R ax = 0, ay = 0;
  if (c < nc) {
    for (int cq = s; cq < 2 * K; cq += S) {
      const R w = qwc[cq % K];
      const C2<R> a = v[cq];
      const C2<R> gg = g[(int64_t)cq * nc + c];
      // w conj(a) gg
      ax = fma(w * a.x, gg.x, ax);
      ax = fma(w * a.y, gg.y, ax);
      ay = fma(w * a.x, gg.y, ay);
      ay = fma(-w * a.y, gg.x, ay);
    }
  }
  for (int o = NC; o < 64; o <<= 1) {
    ax += __shfl_xor(ax, o, 64);
    ay += __shfl_xor(ay, o, 64);
  }
  if (s == 0 && c < nc) {
    C2<R> r = yi[i * nc + c];
    r.x += ax;
    r.y += ay;
    if (conj_out) r.y = -r.y;
    y[(int64_t)perm[i] * ld + c] = r;
  }
}

// ---------------------------------------------------------------- SAI apply
// y_pub[perm[i]] = sum_t P[i, t] x_int[col[t]]  (FP64 products), one wavefront per row
template <typename R>
__global__ void __launch_bounds__(256) k_sai_apply(const int64_t* __restrict__ ptr, const int32_t* __restrict__ col,
                                                   const double2* __restrict__ val, const C2<R>* __restrict__ xi,
                                                   const int32_t* __restrict__ perm, C2<R>* __restrict__ y, int64_t ld,
                                                   int64_t N, int nc) {
  const int lane = threadIdx.x & 63;
  const int64_t i = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
  if (i >= N) return;
  const int NC = pow2ceil(nc);
  const int S = 64 / NC;
  const int c = lane % NC, s = lane / NC;
  double ax = 0.0, ay = 0.0;
  if (c < nc) {
    for (int64_t t = ptr[i] + s; t < ptr[i + 1]; t += S) {
      double2 v = val[t];
      C2<R> xv = xi[(int64_t)col[t] * nc + c];
      double xr = (double)xv.x, xim = (double)xv.y;
      ax = fma(v.x, xr, ax);
      ax = fma(-v.y, xim, ax);
      ay = fma(v.x, xim, ay);
      ay = fma(v.y, xr, ay);
    }
  }
  for (int o = NC; o < 64; o <<= 1) {
    ax += __shfl_xor(ax, o, 64);
    ay += __shfl_xor(ay, o, 64);
  }
  if (s == 0 && c < nc) y[(int64_t)perm[i] * ld + c] = mk<R>((R)ax, (R)ay);
}

// ---------------------------------------------------------------- launchers
static inline void chk(hipError_t e, const char* what) {
  if (e != hipSuccess) throw Error(-4, std::string(what) + ": " + hipGetErrorString(e));
}

static void check_lds(size_t bytes) {
  if (bytes > 65536) throw Error(-7, "angular grid too large for the one-tile interpolation kernel (LDS > 64 KiB)");
}

template <typename R>
static void apply_impl(Dev& d, const Plan& P, PrecD<R>& pd, int op, const void* x, void* y, int64_t ld, int nc,
                       hipStream_t s) {
  using CR = C2<R>;
  const int lf = d.lf;
  const int64_t N = d.N;
  CR* xi = (CR*)d.xi;
  CR* yi = (CR*)d.yi;
  const int conj = (op == 3);
  const int kind = (op == 1) ? 1 : (op == 2) ? 2 : 0;   // 0 Z, 1 R, 2 X
  {
    int64_t tot = N * nc;
    hipLaunchKernelGGL(k_permute_in<R>, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, (const CR*)x, ld, nc,
                       d.perm, xi, N, conj);
  }
  const dim3 rows_grid((unsigned)((N + 3) / 4));
  hipLaunchKernelGGL(k_near<R>, rows_grid, dim3(256), 0, s, d.row_ptr, d.box_of, d.bcol_ptr, d.bcol, d.self_off,
                     d.box_start, (const double2*)d.Zn, (const CR*)xi, yi, N, nc, kind);
  // upward pass
  {
    const int K = P.lev[lf].K;
    int gy = std::max(1, std::min(8, (2 * K * nc + 255) / 256));
    hipLaunchKernelGGL(k_aggregate<R>, dim3(d.nleaf, gy), dim3(256), 0, s, (const CR*)pd.V, (const CR*)xi,
                       (CR*)d.S[lf], d.box_start, K, nc);
  }
  for (int l = lf - 1; l >= 2; --l) {
    LevelD<R>& Lp = pd.lev[l];
    size_t sh = (size_t)2 * Lp.nt * Lp.npc * sizeof(CR);
    check_lds(sh);
    hipLaunchKernelGGL(k_interp_up<R>, dim3(Lp.nbox, nc), dim3(256), sh, s, (const CR*)d.S[l + 1], (CR*)d.S[l],
                       Lp.child_ptr, pd.lev[l + 1].octant, Lp, P.lev[l + 1].K, nc);
  }
  // translations
  for (int l = 2; l <= lf; ++l) {
    LevelD<R>& Lv = pd.lev[l];
    const void* T = (kind == 1) ? Lv.TR : (kind == 2) ? Lv.TX : Lv.TZ;
    const int32_t* ptr = (kind == 1) ? Lv.farR_ptr : Lv.far_ptr;
    const int32_t* src = (kind == 1) ? Lv.farR_src : Lv.far_src;
    const int32_t* off = (kind == 1) ? Lv.farR_off : Lv.far_off;
    int gy = (2 * Lv.K * nc + 255) / 256;
    hipLaunchKernelGGL(k_m2l<R>, dim3(Lv.nbox, gy), dim3(256), 0, s, ptr, src, off, (const CR*)T,
                       (const CR*)d.S[l], (CR*)d.G[l], Lv.K, nc);
  }
  // downward pass
  for (int l = 2; l < lf; ++l) {
    LevelD<R>& Lp = pd.lev[l];
    size_t sh = (size_t)2 * Lp.nt * Lp.npc * sizeof(CR);
    check_lds(sh);
    hipLaunchKernelGGL(k_anterp_down<R>, dim3(pd.lev[l + 1].nbox, nc), dim3(256), sh, s, (const CR*)d.G[l],
                       (CR*)d.G[l + 1], pd.lev[l + 1].parent, pd.lev[l + 1].octant, Lp, P.lev[l + 1].K, nc);
  }
  hipLaunchKernelGGL(k_disagg<R>, rows_grid, dim3(256), 0, s, (const CR*)pd.V, (const CR*)d.G[lf],
                     (const R*)pd.qwc, (const CR*)yi, d.box_of, d.perm, P.lev[lf].K, nc, N, (CR*)y, ld, conj);
  chk(hipGetLastError(), "apply launch");
}

void dev_apply(Dev& d, const Plan& P, int op, const void* x, void* y, int64_t ld, int nc, bool fp64,
               hipStream_t s) {
  if (op == 4) throw Error(-7, "dZ/dk apply is not available in this build");
  if (fp64)
    apply_impl<double>(d, P, d.f64, op, x, y, ld, nc, s);
  else
    apply_impl<float>(d, P, d.f32, op, x, y, ld, nc, s);
}

template <typename R>
static void sai_apply_impl(Dev& d, const void* x, void* y, int64_t ld, int nc, hipStream_t s) {
  using CR = C2<R>;
  const int64_t N = d.N;
  int64_t tot = N * nc;
  hipLaunchKernelGGL(k_permute_in<R>, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, (const CR*)x, ld, nc,
                     d.perm, (CR*)d.xi, N, 0);
  hipLaunchKernelGGL(k_sai_apply<R>, dim3((unsigned)((N + 3) / 4)), dim3(256), 0, s, d.sai_ptr, d.sai_col,
                     (const double2*)d.sai_val, (const CR*)d.xi, d.perm, (CR*)y, ld, N, nc);
  chk(hipGetLastError(), "sai apply launch");
}

void dev_sai_apply(Dev& d, const Plan& P, const void* x, void* y, int64_t ld, int nc, bool fp64, hipStream_t s) {
  (void)P;
  if (!d.sai_val) throw Error(-5, "SAI preconditioner not built");
  if (fp64)
    sai_apply_impl<double>(d, x, y, ld, nc, s);
  else
    sai_apply_impl<float>(d, x, y, ld, nc, s);
}

}  // namespace cm
