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

#include <cstdio>
#include <string>
#include <vector>

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
// x (public order, row stride ld) -> xi (internal order, row stride ldo >=
// nc; columns nc .. ldo-1 are set to zero)
template <typename R>
__global__ void __launch_bounds__(256) k_permute_in(const C2<R>* __restrict__ x, int64_t ld, int nc,
                                                    const int32_t* __restrict__ perm, C2<R>* __restrict__ xi,
                                                    int64_t N, int conj_in, int ldo) {
  int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= N * ldo) return;
  int64_t i = g / ldo;
  int c = (int)(g % ldo);
  C2<R> v = mk<R>(0, 0);
  if (c < nc) {
    v = x[(int64_t)perm[i] * ld + c];
    if (conj_in) v.y = -v.y;
  }
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
#pragma unroll 4
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


// Batched near field: one block per leaf box computes the dense block product
// (rows of the box) x (near columns) x (nc columns).  x rows of a chunk of
// near columns are staged in LDS; each thread owns (row, 4 columns) outputs
// and reads its row's FP64 values once per chunk (shared by the threads of
// the row).  FP64 products and sums.
template <typename R>
__global__ void __launch_bounds__(256) k_near_box(const int64_t* __restrict__ row_ptr,
                                                  const int32_t* __restrict__ box_start,
                                                  const int32_t* __restrict__ bcol_ptr, const int32_t* __restrict__ bcol,
                                                  const int32_t* __restrict__ self_off, const double2* __restrict__ Zn,
                                                  const C2<R>* __restrict__ xi, C2<R>* __restrict__ yi, int nc,
                                                  int mode) {
  constexpr int TC = 32, OPT = 2;
  __shared__ C2<R> xs[TC * 64];
  const int b = blockIdx.x;
  const int r0 = box_start[b], nb = box_start[b + 1] - r0;
  const int32_t* cols = bcol + bcol_ptr[b];
  int t0 = 0, t1 = bcol_ptr[b + 1] - bcol_ptr[b];
  if (mode == 1) {
    t0 = self_off[b];
    t1 = t0 + nb;
  }
  const int ncg = nc / 4;
  const int nout = nb * ncg;
  for (int base = 0; base < nout; base += (int)blockDim.x * OPT) {
    double2 acc[OPT][4];
#pragma unroll
    for (int u = 0; u < OPT; ++u)
#pragma unroll
      for (int q = 0; q < 4; ++q) acc[u][q] = make_double2(0.0, 0.0);
    for (int tc0 = t0; tc0 < t1; tc0 += TC) {
      const int tn = min(TC, t1 - tc0);
      __syncthreads();
#pragma unroll 4
      for (int e = threadIdx.x; e < tn * nc; e += blockDim.x) {
        const int tt = e / nc, c = e % nc;
        xs[tt * nc + c] = xi[(int64_t)cols[tc0 + tt] * nc + c];
      }
      __syncthreads();
#pragma unroll
      for (int u = 0; u < OPT; ++u) {
        const int o = base + u * blockDim.x + threadIdx.x;
        if (o >= nout) continue;
        const int ii = o / ncg, cg = o % ncg;
        const double2* z = Zn + row_ptr[r0 + ii] + tc0;
#pragma unroll 8
        for (int tt = 0; tt < tn; ++tt) {
          double2 v = z[tt];
          if (mode == 1) v.y = 0.0;
          if (mode == 2) {
            v.x = v.y;
            v.y = 0.0;
          }
          const C2<R>* xr = xs + tt * nc + cg * 4;
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            const double xr_ = (double)xr[q].x, xim = (double)xr[q].y;
            acc[u][q].x = fma(v.x, xr_, acc[u][q].x);
            acc[u][q].x = fma(-v.y, xim, acc[u][q].x);
            acc[u][q].y = fma(v.x, xim, acc[u][q].y);
            acc[u][q].y = fma(v.y, xr_, acc[u][q].y);
          }
        }
      }
    }
#pragma unroll
    for (int u = 0; u < OPT; ++u) {
      const int o = base + u * blockDim.x + threadIdx.x;
      if (o >= nout) continue;
      const int ii = o / ncg, cg = o % ncg;
      C2<R>* out = yi + (int64_t)(r0 + ii) * nc + cg * 4;
#pragma unroll
      for (int q = 0; q < 4; ++q) out[q] = mk<R>((R)acc[u][q].x, (R)acc[u][q].y);
    }
  }
}

// ---------------------------------------------------------------- aggregation
// S_b(q) = sum_{j in box b} V_j(q) x_j  (eq. (13) summed over the box), 2 components.
// CG columns per thread (1, or 4 when nc % 4 == 0): one leaf-pattern load feeds
// CG complex multiply-adds.
template <typename R, int CG>
__global__ void __launch_bounds__(256) k_aggregate(const C2<R>* __restrict__ V, const C2<R>* __restrict__ xi,
                                                   int ldx, C2<R>* __restrict__ S, int ldS,
                                                   const int32_t* __restrict__ box_start, int K, int nc) {
  const int b = blockIdx.x;
  const int j0 = box_start[b], j1 = box_start[b + 1];
  const int ncg = nc / CG;
  const int tot = 2 * K * ncg;
  for (int o = blockIdx.y * blockDim.x + threadIdx.x; o < tot; o += gridDim.y * blockDim.x) {
    const int cg = o % ncg, cq = o / ncg;
    C2<R> acc[CG];
#pragma unroll
    for (int u = 0; u < CG; ++u) acc[u] = mk<R>(0, 0);
#pragma unroll 8
    for (int j = j0; j < j1; ++j) {
      const C2<R> v = V[(int64_t)j * 2 * K + cq];
      const C2<R>* xr = xi + (int64_t)j * ldx + cg * CG;
#pragma unroll
      for (int u = 0; u < CG; ++u) acc[u] = cfma(acc[u], v, xr[u]);
    }
    C2<R>* out = S + ((int64_t)b * 2 * K + cq) * ldS + cg * CG;
#pragma unroll
    for (int u = 0; u < CG; ++u) out[u] = acc[u];
  }
}

// ---------------------------------------------------------------- interpolation up
// S_parent(q) = sum_children exp(ik khat_q.(r_c - r_p)) [I_theta I_phi S_child](q).
// The local Lagrange operators in theta and phi commute (the phi stencil is
// invariant under the half-turn phi -> phi + pi that the pole reflection uses),
// so phi is interpolated first, within each child theta row (row-local global
// reads), into an LDS grid [ntc][npp][cs]; the theta stencil then reads LDS.
// Block = (parent box, column slice of width cs, component); every thread
// owns up to JMAX parent samples, accumulated in registers over the children.
template <typename R, int JMAX>
__global__ void __launch_bounds__(256) k_interp_up_direct(const C2<R>* __restrict__ Sc, C2<R>* __restrict__ Sp,
                                                   const int32_t* __restrict__ child_ptr,
                                                   const int8_t* __restrict__ octant, LevelD<R> P, int Kc, int nc,
                                                   int cs, int tpc, int span, int ldp, int accum) {
  extern __shared__ unsigned char smem_raw[];
  C2<R>* tmp = reinterpret_cast<C2<R>*>(smem_raw);   // [span][npp][cs]: child rows tlo ..
  const int ntp = P.nt, npp = P.np, ntc = P.ntc, npc = P.npc, p = P.p, Kp = P.K;
  const int nchunk = (ntp + tpc - 1) / tpc;
  const int m = blockIdx.x / nchunk, tp0 = (blockIdx.x % nchunk) * tpc;
  const int c0 = blockIdx.y * cs, comp = blockIdx.z;
  const int cw = min(cs, nc - c0);
  const int hp = npp / 2;
  const C2<R>* shift = reinterpret_cast<const C2<R>*>(P.shift);
  const int nout = min(tpc, ntp - tp0) * npp * cs;   // this block's parent rows tp0 .. tp0+tpc-1
  // the child rows those parent rows read: tlo .. tlo + span - 1 (the host
  // sized span for the widest chunk)
  int tlo = ntc;
  for (int t = tp0; t < min(ntp, tp0 + tpc); ++t)
    for (int j = 0; j < p; ++j) tlo = min(tlo, P.th_idx[t * p + j]);
  const int nmid = min(span, ntc - tlo) * npp * cs;
  C2<R> acc[JMAX];
#pragma unroll
  for (int j = 0; j < JMAX; ++j) acc[j] = mk<R>(0, 0);
  for (int ch = child_ptr[m]; ch < child_ptr[m + 1]; ++ch) {
    const C2<R>* src = Sc + ((int64_t)ch * 2 + comp) * Kc * ldp + c0;
    const int oc = octant[ch];
    __syncthreads();
    for (int e = threadIdx.x; e < nmid; e += blockDim.x) {
      const int c = e % cs, up = (e / cs) % npp, tc = tlo + e / (cs * npp);
      C2<R> a = mk<R>(0, 0);
      if (c < cw) {
        const C2<R>* row = src + (int64_t)tc * npc * ldp + c;
        for (int j = 0; j < p; ++j) {
          const R w = P.ph_w[up * p + j];
          const C2<R> v = row[(int64_t)P.ph_idx[up * p + j] * ldp];
          a.x = fma(w, v.x, a.x);
          a.y = fma(w, v.y, a.y);
        }
      }
      tmp[e] = a;
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < JMAX; ++j) {
      const int o = threadIdx.x + j * blockDim.x;
      if (o < nout) {
        const int c = o % cs, up = (o / cs) % npp, tp = tp0 + o / (cs * npp);
        C2<R> a = mk<R>(0, 0);
        for (int t = 0; t < p; ++t) {
          const int tc = P.th_idx[tp * p + t];
          const int rf = P.th_ref[tp * p + t];
          const R w = rf ? -P.th_w[tp * p + t] : P.th_w[tp * p + t];
          const C2<R> v = tmp[((tc - tlo) * npp + (rf ? (up + hp) % npp : up)) * cs + c];
          a.x = fma(w, v.x, a.x);
          a.y = fma(w, v.y, a.y);
        }
        acc[j] = cfma(acc[j], a, shift[oc * Kp + tp * npp + up]);
      }
    }
  }
  C2<R>* out = Sp + ((int64_t)m * 2 + comp) * Kp * ldp + c0;
#pragma unroll
  for (int j = 0; j < JMAX; ++j) {
    const int o = threadIdx.x + j * blockDim.x;
    if (o < nout) {
      const int c = o % cs, q = tp0 * npp + o / cs;
      if (c < cw) {
        C2<R>& o = out[(int64_t)q * ldp + c];
        if (accum) {
          o.x += acc[j].x;
          o.y += acc[j].y;
        } else {
          o = acc[j];
        }
      }
    }
  }
}

// ---------------------------------------------------------------- translation
// G_m(q) = sum_{m' in list(m)} T_off(m,m')(q) S_m'(q)  (diagonal translation,
// eqs. (10)/(16)/(20)).  Block = (tile of kTile consecutive receivers,
// direction chunk, column chunk).  The tile's sources are the union of its
// receivers' lists; each source pattern element is loaded once and applied to
// every receiver of the tile that lists it (register accumulators).  With
// STAGE the block's translator rows are staged in LDS first.
template <typename R, bool STAGE, int QPT, int RT, int PD>
__global__ void __launch_bounds__(256) k_m2l(const int32_t* __restrict__ tptr, const int32_t* __restrict__ tsrc,
                                             const int32_t* __restrict__ toff, const C2<R>* __restrict__ T,
                                             int n_off, const C2<R>* __restrict__ S, C2<R>* __restrict__ G,
                                             int nbox, int ntile, int K, int nc, int cw, int ldp, int accum) {
  extern __shared__ unsigned char smem_raw[];
  const int qb = blockDim.x / cw;                     // direction rows per block pass
  const int qspan = qb * QPT;                         // directions per block
  C2<R>* Ts = reinterpret_cast<C2<R>*>(smem_raw);    // [n_off][qb][QPT]: a thread's QPT translators adjacent
  // XCD-aware order: consecutive tiles (which share most sources) go to the
  // same XCD, i.e. the same L2
  const int per_xcd = gridDim.x / 8;
  const int tile = (blockIdx.x % 8) * per_xcd + blockIdx.x / 8;
  if (tile >= ntile) return;
  // grid z: column chunks x groups of RT receivers of the tile (RT < kTile
  // splits the tile's receivers over blocks, for narrow batches whose grid
  // would otherwise leave SIMDs idle)
  constexpr int NRG = kTile / RT;
  const int zc = (int)blockIdx.z / NRG, zr = (int)blockIdx.z % NRG;
  const int c = zc * cw + (int)(threadIdx.x % cw);
  const int ql = threadIdx.x / cw;
  const int qlr = min(ql, qb - 1);
  int q[QPT];
  bool act[QPT];
#pragma unroll
  for (int u = 0; u < QPT; ++u) {
    q[u] = blockIdx.y * qspan + u * qb + ql;
    act[u] = (ql < qb) && (q[u] < K) && (c < nc);
  }
  if (STAGE) {
    for (int e = threadIdx.x; e < n_off * qspan; e += blockDim.x) {
      const int f = e / qspan, r = e % qspan;
      const int qq = blockIdx.y * qspan + (r % QPT) * qb + r / QPT;
      Ts[e] = (qq < K) ? T[(int64_t)f * K + qq] : mk<R>(0, 0);
    }
    __syncthreads();
  }
  const int e0 = tptr[tile], e1 = tptr[tile + 1];
  // the tile's kTile receivers, RT at a time in registers (each pass walks the
  // tile's source list once)
  for (int h = zr * RT; h < zr * RT + RT; h += RT) {
    C2<R> a0[QPT][RT], a1[QPT][RT];
#pragma unroll
    for (int u = 0; u < QPT; ++u)
#pragma unroll
      for (int r = 0; r < RT; ++r) a0[u][r] = a1[u][r] = mk<R>(0, 0);
    // software pipelining: the loads of the next PD - 1 sources are in flight
    // while the current one is applied to the tile's receivers (a ring of PD
    // register sets, rotated by unrolling, so no copies and no wait on loads
    // issued in the same step).  Source patterns: a uniform per-box base plus a
    // loop-invariant 32-bit lane offset in bytes (inactive lanes read
    // direction 0, which is always in range).
    const int64_t bstride = (int64_t)2 * K * ldp, cstride = (int64_t)K * ldp;
    const uint32_t cbytes = (uint32_t)K * (uint32_t)ldp * (uint32_t)sizeof(C2<R>);
    int lo[QPT];
    uint32_t lob[QPT];
#pragma unroll
    for (int u = 0; u < QPT; ++u) {
      lo[u] = (act[u] ? q[u] * ldp : 0) + (c < nc ? c : 0);
      lob[u] = (uint32_t)lo[u] * (uint32_t)sizeof(C2<R>);
    }
    auto load_src = [&](int sb, C2<R>(&n0)[QPT], C2<R>(&n1)[QPT]) {
      const char* sp = reinterpret_cast<const char*>(S + sb * bstride);
#pragma unroll
      for (int u = 0; u < QPT; ++u) {
        n0[u] = *reinterpret_cast<const C2<R>*>(sp + lob[u]);
        n1[u] = *reinterpret_cast<const C2<R>*>(sp + (lob[u] + cbytes));
      }
      // keep the slots' loads in issue order (the waits for a slot then leave
      // the younger slots in flight)
      __builtin_amdgcn_sched_barrier(0);
    };
    // the translator ids of this pass's receivers for source e: uniform, one
    // batch of scalar loads (issued for a whole ring step at once, so that
    // the step waits on the scalar cache once)
    auto load_ids = [&](int e, int(&f)[RT]) {
      if constexpr (RT % 4 == 0) {
        const int4* of4 = reinterpret_cast<const int4*>(toff + (int64_t)e * kTile + h);
#pragma unroll
        for (int r4 = 0; r4 < RT / 4; ++r4) {
          const int4 v = of4[r4];
          f[4 * r4 + 0] = v.x;
          f[4 * r4 + 1] = v.y;
          f[4 * r4 + 2] = v.z;
          f[4 * r4 + 3] = v.w;
        }
      } else {
#pragma unroll
        for (int r = 0; r < RT; ++r) f[r] = toff[(int64_t)e * kTile + h + r];
      }
    };
    auto apply_src = [&](const int(&f)[RT], const C2<R>(&s0)[QPT], const C2<R>(&s1)[QPT]) {
#pragma unroll
      for (int r = 0; r < RT; ++r) {
        if (f[r] >= 0) {
          C2<R> t[QPT];
          if constexpr (STAGE) {
            // staged rows: in range for every thread (ql clamped), zero beyond K
            const C2<R>* tp = Ts + f[r] * qspan + qlr * QPT;
            if constexpr (QPT == 2 && sizeof(R) == 4) {
              const float4 t4 = *reinterpret_cast<const float4*>(tp);
              t[0] = mk<R>(t4.x, t4.y);
              t[1] = mk<R>(t4.z, t4.w);
            } else {
#pragma unroll
              for (int u = 0; u < QPT; ++u) t[u] = tp[u];
            }
          } else {
#pragma unroll
            for (int u = 0; u < QPT; ++u) t[u] = act[u] ? T[(int64_t)f[r] * K + q[u]] : mk<R>(0, 0);
          }
#pragma unroll
          for (int u = 0; u < QPT; ++u) {
            a0[u][r] = cfma(a0[u][r], t[u], s0[u]);
            a1[u][r] = cfma(a1[u][r], t[u], s1[u]);
          }
        }
      }
    };
    if (e0 < e1) {
      C2<R> b0[PD][QPT], b1[PD][QPT];
#pragma unroll
      for (int d = 0; d < PD; ++d) load_src(tsrc[min(e0 + d, e1 - 1)], b0[d], b1[d]);
      int e = e0;
      for (; e + PD <= e1; e += PD) {
        // the step's scalar loads together: translator ids of its sources and
        // the box indices of the sources PD ahead (past the end: the last
        // source again, loaded but never applied)
        int f[PD][RT], sb[PD];
#pragma unroll
        for (int d = 0; d < PD; ++d) {
          load_ids(e + d, f[d]);
          sb[d] = tsrc[min(e + d + PD, e1 - 1)];
        }
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int d = 0; d < PD; ++d) {
          apply_src(f[d], b0[d], b1[d]);
          load_src(sb[d], b0[d], b1[d]);   // refill the slot
        }
      }
#pragma unroll
      for (int d = 0; d < PD; ++d)
        if (e + d < e1) {
          int f[RT];
          load_ids(e + d, f);
          apply_src(f, b0[d], b1[d]);
        }
    }
#pragma unroll
    for (int u = 0; u < QPT; ++u) {
      if (!act[u]) continue;
#pragma unroll
      for (int r = 0; r < RT; ++r) {
        const int m = tile * kTile + h + r;
        if (m < nbox) {
          C2<R>* gp = G + m * bstride + lo[u];
          C2<R>& g0 = gp[0];
          C2<R>& g1 = gp[cstride];
          if (accum) {
            g0.x += a0[u][r].x;
            g0.y += a0[u][r].y;
            g1.x += a1[u][r].x;
            g1.y += a1[u][r].y;
          } else {
            g0 = a0[u][r];
            g1 = a1[u][r];
          }
        }
      }
    }
  }
}

// Translation of a single column, receiver-major: one wave per (receiver
// box, 64 directions), walking the receiver's far list (sorted by source, so
// each receiver sums its sources in the order of the tile kernel and gives
// the same bits) in groups of kGP = 8 entries whose source-pattern and
// translator loads (24 per lane) are all issued before the group is applied
// (4 entries: 0.305 ms at level 5 of the FP64 vector on the 122,880-unknown
// sphere, 8: 0.283 ms, 12 or 16: no faster).  Without the tile's
// register reuse each pair reads its source rows again, but a single
// column's patterns of a level (tens of MB) stay in L2 and the MALL, and
// every wave has independent work: the tile kernel has few blocks per level
// for one column and loads each source of a tile once per block of its
// receiver split.  Block = 4 waves; consecutive receivers go to the same XCD.
template <typename R>
__global__ void __launch_bounds__(256) k_m2l_pairs(const int32_t* __restrict__ fptr,
                                                   const int32_t* __restrict__ fsrc,
                                                   const int32_t* __restrict__ foff, const C2<R>* __restrict__ T,
                                                   const C2<R>* __restrict__ S, C2<R>* __restrict__ G, int nbox,
                                                   int K, int nqc, int ldp, int accum) {
  constexpr int kGP = 8;
  const int per_xcd = gridDim.x / 8;
  const int lb = (blockIdx.x % 8) * per_xcd + blockIdx.x / 8;
  const int wid = lb * 4 + (int)(threadIdx.x >> 6);
  const int m = wid / nqc, qc = wid - m * nqc;
  if (m >= nbox) return;
  const int q = qc * 64 + (int)(threadIdx.x & 63);
  const bool act = q < K;
  const int qq = act ? q : 0;
  const int64_t bstride = (int64_t)2 * K * ldp;
  const uint32_t lob = (uint32_t)qq * (uint32_t)ldp * (uint32_t)sizeof(C2<R>);
  const uint32_t cbytes = (uint32_t)K * (uint32_t)ldp * (uint32_t)sizeof(C2<R>);
  const uint32_t tob = (uint32_t)qq * (uint32_t)sizeof(C2<R>);
  C2<R> a0 = mk<R>(0, 0), a1 = mk<R>(0, 0);
  const int e0 = fptr[m], e1 = fptr[m + 1];
  auto group = [&](int e, int n) {
    C2<R> s0[kGP], s1[kGP], t[kGP];
#pragma unroll
    for (int i = 0; i < kGP; ++i)
      if (i < n) {
        const char* sp = reinterpret_cast<const char*>(S + fsrc[e + i] * bstride);
        const char* tp = reinterpret_cast<const char*>(T + (int64_t)foff[e + i] * K);
        s0[i] = *reinterpret_cast<const C2<R>*>(sp + lob);
        s1[i] = *reinterpret_cast<const C2<R>*>(sp + (lob + cbytes));
        t[i] = *reinterpret_cast<const C2<R>*>(tp + tob);
      }
#pragma unroll
    for (int i = 0; i < kGP; ++i)
      if (i < n) {
        a0 = cfma(a0, t[i], s0[i]);
        a1 = cfma(a1, t[i], s1[i]);
      }
  };
  int e = e0;
  for (; e + kGP <= e1; e += kGP) group(e, kGP);
  if (e < e1) group(e, e1 - e);
  if (!act) return;
  C2<R>* gp = G + m * bstride + (int64_t)qq * ldp;
  C2<R>& g0 = gp[0];
  C2<R>& g1 = gp[(int64_t)K * ldp];
  if (accum) {
    g0.x += a0.x;
    g0.y += a0.y;
    g1.x += a1.x;
    g1.y += a1.y;
  } else {
    g0 = a0;
    g1 = a1;
  }
}

// Translation of a wavenumber-sweep batch (FP32): the columns come in slots
// of four, slot j at wavenumber sw.k[j], and the translators of all nk
// wavenumbers are interleaved, T[(f K + q) nk + k].  Thread = (direction,
// slot): the slot's four columns of both components in registers, so one
// translator load (L1/L2) serves eight complex products.  Block = (tile of
// kTile receivers, chunk of 256 / sw.n directions, group of RT of the tile's
// receivers).  The tile's source list is walked as in k_m2l: source loads in
// a ring of PD register sets, translator ids by scalar loads, and the
// translators of a ring step's listed pairs issued together before the step
// is applied; each receiver sums its sources in increasing source order.
__device__ __forceinline__ float4 cfma2(float4 a, float2 t, float4 v) {
  a.x = fmaf(t.x, v.x, a.x);
  a.x = fmaf(-t.y, v.y, a.x);
  a.y = fmaf(t.x, v.y, a.y);
  a.y = fmaf(t.y, v.x, a.y);
  a.z = fmaf(t.x, v.z, a.z);
  a.z = fmaf(-t.y, v.w, a.z);
  a.w = fmaf(t.x, v.w, a.w);
  a.w = fmaf(t.y, v.z, a.w);
  return a;
}

template <int RT, int PD>
__global__ void __launch_bounds__(256) k_m2l_slots(const int32_t* __restrict__ tptr, const int32_t* __restrict__ tsrc,
                                                   const int32_t* __restrict__ toff, const float2* __restrict__ T,
                                                   int nk, SweepSlots sw, const float2* __restrict__ S,
                                                   float2* __restrict__ G, int nbox, int ntile, int K, int ldp,
                                                   int accum) {
  // grid x = tiles x receiver groups, XCD-aware: the kTile / RT blocks of a
  // tile are consecutive on one XCD, so the later ones find the tile's
  // sources in that XCD's L2
  constexpr int NRG = kTile / RT;
  const int per_xcd = gridDim.x / 8;
  const int pos = (blockIdx.x % 8) * per_xcd + blockIdx.x / 8;
  const int tile = pos / NRG;
  if (tile >= ntile) return;
  const int ns = sw.n;
  const int qb = (int)blockDim.x / ns;
  const int slot = (int)threadIdx.x % ns, ql = (int)threadIdx.x / ns;
  const int q = (int)blockIdx.y * qb + ql;
  const bool act = ql < qb && q < K;
  const int qq = act ? q : 0;   // inactive lanes read direction 0 (always in range)
  const int h = (pos % NRG) * RT;
  const float2* Tq = T + (int64_t)qq * nk + sw.k[slot];
  const int64_t fstride = (int64_t)K * nk;
  const int64_t bstride = (int64_t)2 * K * ldp;
  const uint32_t lob = ((uint32_t)qq * (uint32_t)ldp + 4u * (uint32_t)slot) * 8u;   // bytes into a box
  const uint32_t cbytes = (uint32_t)K * (uint32_t)ldp * 8u;                          // component plane
  float4 acc[RT][2][2];   // [receiver][component][column pair]
#pragma unroll
  for (int r = 0; r < RT; ++r)
#pragma unroll
    for (int c = 0; c < 2; ++c) acc[r][c][0] = acc[r][c][1] = float4{0.f, 0.f, 0.f, 0.f};
  auto load_src = [&](int sb, float4(&v)[2][2]) {
    const char* sp = reinterpret_cast<const char*>(S + sb * bstride);
    v[0][0] = *reinterpret_cast<const float4*>(sp + lob);
    v[0][1] = *reinterpret_cast<const float4*>(sp + (lob + 16u));
    v[1][0] = *reinterpret_cast<const float4*>(sp + (lob + cbytes));
    v[1][1] = *reinterpret_cast<const float4*>(sp + (lob + cbytes + 16u));
    __builtin_amdgcn_sched_barrier(0);
  };
  auto load_ids = [&](int e, int(&f)[RT]) {
    const int4* of4 = reinterpret_cast<const int4*>(toff + (int64_t)e * kTile + h);
#pragma unroll
    for (int r4 = 0; r4 < RT / 4; ++r4) {
      const int4 v = of4[r4];
      f[4 * r4 + 0] = v.x;
      f[4 * r4 + 1] = v.y;
      f[4 * r4 + 2] = v.z;
      f[4 * r4 + 3] = v.w;
    }
  };
  auto apply_src = [&](const int(&f)[RT], const float2(&t)[RT], const float4(&v)[2][2]) {
#pragma unroll
    for (int r = 0; r < RT; ++r)
      if (f[r] >= 0) {
#pragma unroll
        for (int c = 0; c < 2; ++c) {
          acc[r][c][0] = cfma2(acc[r][c][0], t[r], v[c][0]);
          acc[r][c][1] = cfma2(acc[r][c][1], t[r], v[c][1]);
        }
      }
  };
  auto load_t = [&](const int(&f)[RT], float2(&t)[RT]) {
#pragma unroll
    for (int r = 0; r < RT; ++r)
      if (f[r] >= 0) t[r] = Tq[(int64_t)f[r] * fstride];
  };
  const int e0 = tptr[tile], e1 = tptr[tile + 1];
  if (e0 < e1) {
    float4 b[PD][2][2];
#pragma unroll
    for (int d = 0; d < PD; ++d) load_src(tsrc[min(e0 + d, e1 - 1)], b[d]);
    int e = e0;
    for (; e + PD <= e1; e += PD) {
      int f[PD][RT], sb[PD];
#pragma unroll
      for (int d = 0; d < PD; ++d) {
        load_ids(e + d, f[d]);
        sb[d] = tsrc[min(e + d + PD, e1 - 1)];
      }
      float2 t[PD][RT];
#pragma unroll
      for (int d = 0; d < PD; ++d) load_t(f[d], t[d]);
#pragma unroll
      for (int d = 0; d < PD; ++d) {
        apply_src(f[d], t[d], b[d]);
        load_src(sb[d], b[d]);   // refill the slot
      }
    }
#pragma unroll
    for (int d = 0; d < PD; ++d)
      if (e + d < e1) {
        int f[RT];
        float2 t[RT];
        load_ids(e + d, f);
        load_t(f, t);
        apply_src(f, t, b[d]);
      }
  }
  if (!act) return;
#pragma unroll
  for (int r = 0; r < RT; ++r) {
    const int m = tile * kTile + h + r;
    if (m >= nbox) continue;
    char* gp = reinterpret_cast<char*>(G + m * bstride);
#pragma unroll
    for (int c = 0; c < 2; ++c)
#pragma unroll
      for (int p2 = 0; p2 < 2; ++p2) {
        float4* o = reinterpret_cast<float4*>(gp + (lob + (c ? cbytes : 0u) + 16u * p2));
        if (accum) {
          float4 v = *o;
          v.x += acc[r][c][p2].x;
          v.y += acc[r][c][p2].y;
          v.z += acc[r][c][p2].z;
          v.w += acc[r][c][p2].w;
          *o = v;
        } else {
          *o = acc[r][c][p2];
        }
      }
  }
}

// Translation for FP32 batches with receiver tiles of kTile64 boxes: the
// four waves of a block own 16 receivers each and share the tile's sources,
// which the block stages through LDS in chunks of kCH64 sources (one global
// load per element per block, double-buffered: the next chunk's loads are in
// flight while the current chunk is applied).  Each wave walks the staged
// sources in order and applies each to those of its receivers that list it
// (register accumulators), so every receiver sums its sources in increasing
// source order, as the 16-box tiles of k_m2l do: the two kernels give the
// same bits.  Thread = (direction row, column) of the block's slab of
// qspan = QPT * 64 / cw directions and cw columns.  kCH64 sources per
// staged chunk; MINW: the waves per SIMD the register allocation aims at
// (3 spills a few registers, 2 does not: the autotuner picks per level).
template <int QPT, int kCH64, int MINW>
__global__ void __launch_bounds__(256, MINW) k_m2l64(const int32_t* __restrict__ tptr, const int32_t* __restrict__ tsrc,
                                               const int32_t* __restrict__ toff, const C2<float>* __restrict__ T,
                                               int n_off, const C2<float>* __restrict__ S, C2<float>* __restrict__ G,
                                               int nbox, int ntile, int K, int nc, int cw, int ldp, int accum) {
  extern __shared__ unsigned char smem_raw[];
  constexpr int SLAB = 2 * QPT * 64;                 // complex values of one staged source
  constexpr int PER = kCH64 * SLAB / 256;            // staged values per thread and chunk
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int qw = 64 / cw, qspan = qw * QPT;
  C2<float>* Ts = reinterpret_cast<C2<float>*>(smem_raw);   // [n_off][qspan]
  C2<float>* Sb = Ts + n_off * qspan;                    // [2][kCH64][2 comps][qspan][cw]
  const int per_xcd = gridDim.x / 8;
  const int tile = (blockIdx.x % 8) * per_xcd + blockIdx.x / 8;
  if (tile >= ntile) return;
  const int q0 = blockIdx.y * qspan, c0 = blockIdx.z * cw;
  for (int e = threadIdx.x; e < n_off * qspan; e += blockDim.x) {
    const int f = e / qspan, qq = q0 + e % qspan;
    Ts[e] = (qq < K) ? T[(int64_t)f * K + qq] : mk<float>(0.f, 0.f);
  }
  const int cl = lane % cw, ql = lane / cw;
  const int c = c0 + cl;
  const int64_t bstride = (int64_t)2 * K * ldp, cstride = (int64_t)K * ldp;
  const int e0 = tptr[tile], e1 = tptr[tile + 1];
  // staging: thread t stages value t % SLAB of sources t / SLAB, t / SLAB +
  // 256 / SLAB, ... of a chunk (pre[i]); its (component, direction, column)
  // is fixed for the whole block
  static_assert(256 % SLAB == 0 && (kCH64 * SLAB) % 256 == 0, "whole sources per pass of the block");
  constexpr int SPP = 256 / SLAB;                    // sources per pass of the block
  const int sub = threadIdx.x / SLAB;
  int64_t my_off;
  bool my_ok;
  {
    const int v = threadIdx.x % SLAB;
    const int comp = v / (QPT * 64), r2 = v % (QPT * 64);
    const int qq = q0 + r2 / cw, cc = c0 + r2 % cw;
    my_ok = qq < K && cc < nc;
    my_off = comp * cstride + (int64_t)qq * ldp + cc;
  }
  C2<float> pre[PER];
  auto fetch = [&](int cs) {
#pragma unroll
    for (int i = 0; i < PER; ++i) {
      const int src = cs + SPP * i + sub;
      pre[i] = (src < e1 && my_ok) ? S[tsrc[src] * bstride + my_off] : mk<float>(0.f, 0.f);
    }
  };
  auto commit = [&](int buf) {
#pragma unroll
    for (int i = 0; i < PER; ++i) Sb[buf * kCH64 * SLAB + threadIdx.x + 256 * i] = pre[i];
  };
  C2<float> a0[QPT][16], a1[QPT][16];
#pragma unroll
  for (int u = 0; u < QPT; ++u)
#pragma unroll
    for (int r = 0; r < 16; ++r) a0[u][r] = a1[u][r] = mk<float>(0.f, 0.f);
  if (e0 < e1) {
    fetch(e0);
    commit(0);
  }
  __syncthreads();
  int buf = 0;
  for (int cs = e0; cs < e1; cs += kCH64) {
    const bool more = cs + kCH64 < e1;
    if (more) fetch(cs + kCH64);
    const int n = min(kCH64, e1 - cs);
    const C2<float>* sb = Sb + buf * kCH64 * SLAB;
    for (int s = 0; s < n; ++s) {
      // this wave's 16 translator ids for the source (uniform scalar loads)
      const int4* of4 = reinterpret_cast<const int4*>(toff + (int64_t)(cs + s) * kTile64 + 16 * w);
      int f[16];
#pragma unroll
      for (int r4 = 0; r4 < 4; ++r4) {
        const int4 v = of4[r4];
        f[4 * r4 + 0] = v.x;
        f[4 * r4 + 1] = v.y;
        f[4 * r4 + 2] = v.z;
        f[4 * r4 + 3] = v.w;
      }
      int all = f[0];
#pragma unroll
      for (int r = 1; r < 16; ++r) all &= f[r];
      if (all < 0) continue;   // none of this wave's receivers lists the source
      C2<float> s0[QPT], s1[QPT];
#pragma unroll
      for (int u = 0; u < QPT; ++u) {   // (u qw + ql) cw + cl = 64 u + lane
        s0[u] = sb[s * SLAB + 64 * u + lane];
        s1[u] = sb[s * SLAB + QPT * 64 + 64 * u + lane];
      }
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        if (f[r] >= 0) {
#pragma unroll
          for (int u = 0; u < QPT; ++u) {
            const C2<float> t = Ts[f[r] * qspan + u * qw + ql];
            a0[u][r] = cfma(a0[u][r], t, s0[u]);
            a1[u][r] = cfma(a1[u][r], t, s1[u]);
          }
        }
      }
    }
    if (more) commit(buf ^ 1);
    __syncthreads();
    buf ^= 1;
  }
#pragma unroll
  for (int u = 0; u < QPT; ++u) {
    const int q = q0 + u * qw + ql;
    if (q >= K || c >= nc) continue;
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const int m = tile * kTile64 + 16 * w + r;
      if (m < nbox) {
        C2<float>* gp = G + m * bstride + (int64_t)q * ldp + c;
        if (accum) {
          gp[0].x += a0[u][r].x;
          gp[0].y += a0[u][r].y;
          gp[cstride].x += a1[u][r].x;
          gp[cstride].y += a1[u][r].y;
        } else {
          gp[0] = a0[u][r];
          gp[cstride] = a1[u][r];
        }
      }
    }
  }
}

// ---------------------------------------------------------------- anterpolation down
// G_child += W_c^-1 I^T W_p [exp(-ik khat.(r_c - r_p)) G_parent]: the weighted
// transposes of the two stencils, phi first (row-local reads of the parent
// into an LDS grid [ntp][npc][cs]), then theta from LDS.  Block = (child box,
// column slice, component).
template <typename R>
__global__ void __launch_bounds__(256) k_anterp_down_direct(const C2<R>* __restrict__ Gp, C2<R>* __restrict__ Gc,
                                                     const int32_t* __restrict__ parent,
                                                     const int8_t* __restrict__ octant, LevelD<R> P, int Kc, int nc,
                                                     int cs, int tcc, int span, int ldp) {
  extern __shared__ unsigned char smem_raw[];
  C2<R>* tmp = reinterpret_cast<C2<R>*>(smem_raw);   // [span][npc][cs]: parent rows plo ..
  const int ntp = P.nt, npp = P.np, ntc = P.ntc, npc = P.npc, Kp = P.K;
  const int nchunk = (ntc + tcc - 1) / tcc;
  const int ch = blockIdx.x / nchunk, tc0 = (blockIdx.x % nchunk) * tcc, tc1 = min(ntc, tc0 + tcc);
  const int c0 = blockIdx.y * cs, comp = blockIdx.z;
  const int cw = min(cs, nc - c0);
  const int hc = npc / 2;
  const int m = parent[ch], oc = octant[ch];
  const C2<R>* shift = reinterpret_cast<const C2<R>*>(P.shift) + oc * Kp;
  const C2<R>* g = Gp + ((int64_t)m * 2 + comp) * Kp * ldp + c0;
  // the parent rows this block's child rows tc0 .. tc1-1 read: plo .. plo +
  // span - 1 (the host sized span for the widest chunk)
  int plo = ntp;
  for (int j = P.tht_ptr[tc0]; j < P.tht_ptr[tc1]; ++j) plo = min(plo, P.tht_idx[j]);
  if (plo >= ntp) plo = 0;
  const int nrow = min(span, ntp - plo);
  for (int e = threadIdx.x; e < nrow * npc * cs; e += blockDim.x) {
    const int c = e % cs, uc = (e / cs) % npc, tp = plo + e / (cs * npc);
    C2<R> a = mk<R>(0, 0);
    if (c < cw) {
      for (int j = P.pht_ptr[uc]; j < P.pht_ptr[uc + 1]; ++j) {
        const int up = P.pht_idx[j];
        const R w = P.pht_w[j];
        const C2<R> v = g[(int64_t)(tp * npp + up) * ldp + c];
        C2<R> t = mk<R>(0, 0);
        t = cfma_conj(t, shift[tp * npp + up], v);
        a.x = fma(w, t.x, a.x);
        a.y = fma(w, t.y, a.y);
      }
    }
    tmp[e] = a;
  }
  __syncthreads();
  C2<R>* out = Gc + ((int64_t)ch * 2 + comp) * Kc * ldp + c0;
  for (int e = threadIdx.x; e < (tc1 - tc0) * npc * cs; e += blockDim.x) {
    const int c = e % cs, uc = (e / cs) % npc, tc = tc0 + e / (cs * npc);
    if (c >= cw) continue;
    C2<R> a = mk<R>(0, 0);
    for (int j = P.tht_ptr[tc]; j < P.tht_ptr[tc + 1]; ++j) {
      const int tp = P.tht_idx[j];
      const int rf = P.tht_ref[j];
      const R w = rf ? -P.tht_w[j] : P.tht_w[j];
      const C2<R> v = tmp[((tp - plo) * npc + (rf ? (uc + hc) % npc : uc)) * cs + c];
      a.x = fma(w, v.x, a.x);
      a.y = fma(w, v.y, a.y);
    }
    C2<R>& o = out[(int64_t)(tc * npc + uc) * ldp + c];
    o.x += a.x;
    o.y += a.y;
  }
}


// Staged variants (used whenever both LDS grids fit): the input grid of the
// block is copied to LDS once (coalesced), the phi stencil runs LDS -> LDS, the
// theta stencil reads LDS.  Interpolation: A = child [ntc][npc][cs],
// B = [ntc][npp][cs].  Anterpolation: A = conj-shifted parent [ntp][npp][cs],
// B = [ntp][npc][cs].
template <typename R, int JMAX>
__global__ void __launch_bounds__(256) k_interp_up(const C2<R>* __restrict__ Sc, C2<R>* __restrict__ Sp,
                                                   const int32_t* __restrict__ child_ptr,
                                                   const int8_t* __restrict__ octant, LevelD<R> P, int Kc, int nc,
                                                   int cs, int tpc, int ldp, int accum) {
  extern __shared__ unsigned char smem_raw[];
  const int ntp = P.nt, npp = P.np, ntc = P.ntc, npc = P.npc, p = P.p, Kp = P.K;
  C2<R>* A = reinterpret_cast<C2<R>*>(smem_raw);            // [ntc][npc][cs]
  C2<R>* B = A + ntc * npc * cs;                             // [ntc][npp][cs]
  // stencil tables: phi (index, weight) per parent phi, theta (index | reflect<<30, weight) per parent theta
  R* phW = reinterpret_cast<R*>(B + ntc * npp * cs);       // weights first (alignment)
  R* thW = phW + npp * p;
  int32_t* phI = reinterpret_cast<int32_t*>(thW + ntp * p);
  int32_t* thI = phI + npp * p;
  for (int e = threadIdx.x; e < npp * p; e += blockDim.x) {
    phI[e] = P.ph_idx[e] * cs;
    phW[e] = P.ph_w[e];
  }
  for (int e = threadIdx.x; e < ntp * p; e += blockDim.x) {
    thI[e] = P.th_idx[e] | (P.th_ref[e] << 30);
    thW[e] = P.th_ref[e] ? -P.th_w[e] : P.th_w[e];
  }
  const int nchunk = (ntp + tpc - 1) / tpc;
  const int m = blockIdx.x / nchunk, tp0 = (blockIdx.x % nchunk) * tpc;
  const int c0 = blockIdx.y * cs, comp = blockIdx.z;
  const int cw = min(cs, nc - c0);
  const int hp = npp / 2;
  const C2<R>* shift = reinterpret_cast<const C2<R>*>(P.shift);
  const int nout = min(tpc, ntp - tp0) * npp * cs;
  C2<R> acc[JMAX];
#pragma unroll
  for (int j = 0; j < JMAX; ++j) acc[j] = mk<R>(0, 0);
  for (int ch = child_ptr[m]; ch < child_ptr[m + 1]; ++ch) {
    const C2<R>* src = Sc + ((int64_t)ch * 2 + comp) * Kc * ldp + c0;
    const int oc = octant[ch];
    __syncthreads();
#pragma unroll 4
    for (int e = threadIdx.x; e < Kc * cs; e += blockDim.x) {
      const int c = e % cs, q = e / cs;
      A[e] = (c < cw) ? src[(int64_t)q * ldp + c] : mk<R>(0, 0);
    }
    __syncthreads();
    for (int e = threadIdx.x; e < ntc * npp * cs; e += blockDim.x) {
      const int c = e % cs, up = (e / cs) % npp, tc = e / (cs * npp);
      const C2<R>* row = A + tc * npc * cs + c;
      const int32_t* ii = phI + up * p;
      const R* ww = phW + up * p;
      C2<R> a = mk<R>(0, 0);
      for (int j = 0; j < p; ++j) {
        const R w = ww[j];
        const C2<R> v = row[ii[j]];
        a.x = fma(w, v.x, a.x);
        a.y = fma(w, v.y, a.y);
      }
      B[e] = a;
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < JMAX; ++j) {
      const int o = threadIdx.x + j * blockDim.x;
      if (o < nout) {
        const int c = o % cs, up = (o / cs) % npp, tp = tp0 + o / (cs * npp);
        const int upr = (up + hp) % npp;
        C2<R> a = mk<R>(0, 0);
        for (int t = 0; t < p; ++t) {
          const int code = thI[tp * p + t];
          const int tc = code & 0x3fffffff;
          const R w = thW[tp * p + t];
          const C2<R> v = B[(tc * npp + ((code >> 30) ? upr : up)) * cs + c];
          a.x = fma(w, v.x, a.x);
          a.y = fma(w, v.y, a.y);
        }
        acc[j] = cfma(acc[j], a, shift[oc * Kp + tp * npp + up]);
      }
    }
  }
  C2<R>* out = Sp + ((int64_t)m * 2 + comp) * Kp * ldp + c0;
#pragma unroll
  for (int j = 0; j < JMAX; ++j) {
    const int o = threadIdx.x + j * blockDim.x;
    if (o < nout) {
      const int c = o % cs, q = tp0 * npp + o / cs;
      if (c < cw) {
        C2<R>& o = out[(int64_t)q * ldp + c];
        if (accum) {
          o.x += acc[j].x;
          o.y += acc[j].y;
        } else {
          o = acc[j];
        }
      }
    }
  }
}

// Anterpolation, one block per child box: the block stages its parent's
// pattern, applies the child's conjugated shift (LDS -> LDS), the
// phi-transpose stencil (LDS -> LDS) and the theta-transpose stencil (LDS ->
// child, RMW).  (One block per parent looping over its children gives the
// same sums but a quarter of the blocks: 112 blocks for the 56 level-2 boxes
// of the 122,880-unknown sphere.)
// LDS: P0 [Kp][cs], A [Kp][cs], B [ntp][npc][cs], stencil tables.
template <typename R>
__global__ void __launch_bounds__(256) k_anterp_down(const C2<R>* __restrict__ Gp, C2<R>* __restrict__ Gc,
                                                     const int32_t* __restrict__ parent,
                                                     const int8_t* __restrict__ octant, LevelD<R> P, int Kc, int nc,
                                                     int cs, int ldp) {
  extern __shared__ unsigned char smem_raw[];
  const int ntp = P.nt, npp = P.np, ntc = P.ntc, npc = P.npc, Kp = P.K;
  C2<R>* P0 = reinterpret_cast<C2<R>*>(smem_raw);           // [ntp][npp][cs]
  C2<R>* A = P0 + Kp * cs;                                   // shifted copy
  C2<R>* B = A + Kp * cs;                                    // [ntp][npc][cs]
  const int nph = P.pht_ptr[npc], nth = P.tht_ptr[ntc];
  R* phW = reinterpret_cast<R*>(B + ntp * npc * cs);
  R* thW = phW + nph;
  int32_t* phP = reinterpret_cast<int32_t*>(thW + nth);
  int32_t* thP = phP + npc + 1;
  int32_t* phI = thP + ntc + 1;
  int32_t* thI = phI + nph;
  for (int e = threadIdx.x; e <= npc; e += blockDim.x) phP[e] = P.pht_ptr[e];
  for (int e = threadIdx.x; e <= ntc; e += blockDim.x) thP[e] = P.tht_ptr[e];
  for (int e = threadIdx.x; e < nph; e += blockDim.x) {
    phI[e] = P.pht_idx[e] * cs;
    phW[e] = P.pht_w[e];
  }
  for (int e = threadIdx.x; e < nth; e += blockDim.x) {
    thI[e] = P.tht_idx[e] | (P.tht_ref[e] << 30);
    thW[e] = P.tht_ref[e] ? -P.tht_w[e] : P.tht_w[e];
  }
  const int ch = blockIdx.x, m = parent[ch], c0 = blockIdx.y * cs, comp = blockIdx.z;
  const int cw = min(cs, nc - c0);
  const int hc = npc / 2;
  const C2<R>* g = Gp + ((int64_t)m * 2 + comp) * Kp * ldp + c0;
#pragma unroll 4
  for (int e = threadIdx.x; e < Kp * cs; e += blockDim.x) {
    const int c = e % cs, q = e / cs;
    P0[e] = (c < cw) ? g[(int64_t)q * ldp + c] : mk<R>(0, 0);
  }
  {
    const C2<R>* shift = reinterpret_cast<const C2<R>*>(P.shift) + octant[ch] * Kp;
    __syncthreads();
    for (int e = threadIdx.x; e < Kp * cs; e += blockDim.x) {
      C2<R> t = mk<R>(0, 0);
      A[e] = cfma_conj(t, shift[e / cs], P0[e]);
    }
    __syncthreads();
    for (int e = threadIdx.x; e < ntp * npc * cs; e += blockDim.x) {
      const int c = e % cs, uc = (e / cs) % npc, tp = e / (cs * npc);
      const C2<R>* row = A + tp * npp * cs + c;
      C2<R> a = mk<R>(0, 0);
      for (int j = phP[uc]; j < phP[uc + 1]; ++j) {
        const R w = phW[j];
        const C2<R> v = row[phI[j]];
        a.x = fma(w, v.x, a.x);
        a.y = fma(w, v.y, a.y);
      }
      B[e] = a;
    }
    __syncthreads();
    C2<R>* out = Gc + ((int64_t)ch * 2 + comp) * Kc * ldp + c0;
    for (int e = threadIdx.x; e < ntc * npc * cs; e += blockDim.x) {
      const int c = e % cs, uc = (e / cs) % npc, tc = e / (cs * npc);
      if (c >= cw) continue;
      const int ucr = (uc + hc) % npc;
      C2<R> a = mk<R>(0, 0);
      for (int j = thP[tc]; j < thP[tc + 1]; ++j) {
        const int code = thI[j];
        const int tp = code & 0x3fffffff;
        const R w = thW[j];
        const C2<R> v = B[(tp * npc + ((code >> 30) ? ucr : uc)) * cs + c];
        a.x = fma(w, v.x, a.x);
        a.y = fma(w, v.y, a.y);
      }
      C2<R>& o = out[(int64_t)(tc * npc + uc) * ldp + c];
      o.x += a.x;
      o.y += a.y;
    }
  }
}

// ---------------------------------------------------------------- disaggregation
// y_i = y_near_i + sum_q (k^2 eta/4pi) w_q conj(V_i(q)) . G_box(i)(q), written to
// the public position perm[i] (conjugated for Z^H).  nc == 1: one wavefront
// per unknown, lanes over directions.
template <typename R>
__global__ void __launch_bounds__(256) k_disagg1(const C2<R>* __restrict__ V, const C2<R>* __restrict__ G,
                                                 const R* __restrict__ qwc, const C2<R>* __restrict__ yi,
                                                 const int32_t* __restrict__ box_of, const int32_t* __restrict__ perm,
                                                 int K, int64_t N, int ldp, C2<R>* __restrict__ y, int64_t ld,
                                                 int conj_out) {
  const int lane = threadIdx.x & 63;
  const int64_t i = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
  if (i >= N) return;
  const int b = box_of[i];
  const C2<R>* v = V + i * 2 * K;
  const C2<R>* g = G + (int64_t)b * 2 * K * ldp;
  R ax = 0, ay = 0;
#pragma unroll 4
  for (int cq = lane; cq < 2 * K; cq += 64) {
    const R w = qwc[cq < K ? cq : cq - K];
    const C2<R> a = v[cq];
    const C2<R> gg = g[(int64_t)cq * ldp];
    ax = fma(w * a.x, gg.x, ax);
    ax = fma(w * a.y, gg.y, ax);
    ay = fma(w * a.x, gg.y, ay);
    ay = fma(-w * a.y, gg.x, ay);
  }
  for (int o = 1; o < 64; o <<= 1) {
    ax += __shfl_xor(ax, o, 64);
    ay += __shfl_xor(ay, o, 64);
  }
  if (lane == 0) {
    C2<R> r = yi[i];
    r.x += ax;
    r.y += ay;
    if (conj_out) r.y = -r.y;
    y[(int64_t)(perm ? perm[i] : i) * ld] = r;
  }
}

// Batched: one block per leaf box, thread = (unknown of the box, CG columns).
template <typename R, int CG>
__global__ void __launch_bounds__(256) k_disagg(const C2<R>* __restrict__ V, const C2<R>* __restrict__ G,
                                                const R* __restrict__ qwc, const C2<R>* __restrict__ yi,
                                                const int32_t* __restrict__ box_start,
                                                const int32_t* __restrict__ perm, int K, int nc, int ldp,
                                                C2<R>* __restrict__ y, int64_t ld, int conj_out) {
  const int b = blockIdx.x;
  const int j0 = box_start[b], nb = box_start[b + 1] - j0;
  const int ncg = nc / CG;
  const C2<R>* g = G + (int64_t)b * 2 * K * ldp;
  for (int o = threadIdx.x; o < nb * ncg; o += blockDim.x) {
    const int cg = o % ncg, ii = o / ncg;
    const int64_t i = j0 + ii;
    const C2<R>* v = V + i * 2 * K;
    C2<R> acc[CG];
#pragma unroll
    for (int u = 0; u < CG; ++u) acc[u] = mk<R>(0, 0);
    for (int cq = 0; cq < 2 * K; ++cq) {
      const R w = qwc[cq < K ? cq : cq - K];
      C2<R> a = v[cq];
      a.x *= w;
      a.y *= w;
      const C2<R>* gr = g + (int64_t)cq * ldp + cg * CG;
#pragma unroll
      for (int u = 0; u < CG; ++u) acc[u] = cfma_conj(acc[u], a, gr[u]);
    }
#pragma unroll
    for (int u = 0; u < CG; ++u) {
      C2<R> r = yi[i * nc + cg * CG + u];
      r.x += acc[u].x;
      r.y += acc[u].y;
      if (conj_out) r.y = -r.y;
      y[(int64_t)(perm ? perm[i] : i) * ld + cg * CG + u] = r;
    }
  }
}

// y[:, 0:nc] += alpha x[:, 0:nc] over rows of a pattern buffer with column stride ld
template <typename R>
__global__ void __launch_bounds__(256) k_pattern_axpy(const C2<R>* __restrict__ x, C2<R>* __restrict__ y, int64_t rows,
                                                      int nc, int ld, R alpha) {
  int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= rows * nc) return;
  int64_t r = g / nc;
  int c = (int)(g % nc);
  C2<R> a = x[r * ld + c];
  C2<R>& o = y[r * ld + c];
  o.x += alpha * a.x;
  o.y += alpha * a.y;
}


// Batched aggregation, one block per leaf box: the box's x rows are staged in
// LDS; thread = (4 columns, direction-component cq), looping over the box's
// unknowns with one leaf-pattern load per 4 complex multiply-adds.
template <typename R>
__global__ void __launch_bounds__(256) k_aggregate_box(const C2<R>* __restrict__ V, const C2<R>* __restrict__ xi,
                                                       int ldx, C2<R>* __restrict__ S, int ldS,
                                                       const int32_t* __restrict__ box_start, int K, int nc) {
  extern __shared__ unsigned char smem_raw[];
  C2<R>* xs = reinterpret_cast<C2<R>*>(smem_raw);          // [nb][nc]
  const int b = blockIdx.x;
  const int j0 = box_start[b], nb = box_start[b + 1] - j0;
  for (int e = threadIdx.x; e < nb * nc; e += blockDim.x) xs[e] = xi[(int64_t)(j0 + e / nc) * ldx + e % nc];
  __syncthreads();
  const int ncg = nc / 4;
  const int tot = 2 * K * ncg;
  for (int o = blockIdx.y * blockDim.x + threadIdx.x; o < tot; o += gridDim.y * blockDim.x) {
    const int cg = o % ncg, cq = o / ncg;
    C2<R> a0 = mk<R>(0, 0), a1 = a0, a2 = a0, a3 = a0;
    const C2<R>* v = V + (int64_t)j0 * 2 * K + cq;
    const C2<R>* xr = xs + cg * 4;
#pragma unroll 8
    for (int j = 0; j < nb; ++j) {
      const C2<R> w = v[(int64_t)j * 2 * K];
      a0 = cfma(a0, w, xr[0]);
      a1 = cfma(a1, w, xr[1]);
      a2 = cfma(a2, w, xr[2]);
      a3 = cfma(a3, w, xr[3]);
      xr += nc;
    }
    C2<R>* out = S + ((int64_t)b * 2 * K + cq) * ldS + cg * 4;
    out[0] = a0;
    out[1] = a1;
    out[2] = a2;
    out[3] = a3;
  }
}

// Batched disaggregation, one block per leaf box: chunks of 64 direction-
// components of the box's incoming pattern G and of the box's leaf patterns
// (weighted and conjugated) are staged in LDS; thread = (unknown, 4 columns).
template <typename R>
__global__ void __launch_bounds__(256) k_disagg_box(const C2<R>* __restrict__ V, const C2<R>* __restrict__ G,
                                                    const R* __restrict__ qwc, const C2<R>* __restrict__ yi,
                                                    const int32_t* __restrict__ box_start,
                                                    const int32_t* __restrict__ perm, int K, int nc, int ldp,
                                                    C2<R>* __restrict__ y, int64_t ld, int conj_out) {
  constexpr int CH = 64;
  extern __shared__ unsigned char smem_raw[];
  const int b = blockIdx.x;
  const int j0 = box_start[b], nb = box_start[b + 1] - j0;
  C2<R>* gs = reinterpret_cast<C2<R>*>(smem_raw);          // [CH][nc]
  C2<R>* vs = gs + CH * nc;                                // [nb][CH]
  const int ncg = nc / 4;
  const int nout = nb * ncg;
  const C2<R>* g = G + (int64_t)b * 2 * K * ldp;
  for (int base = 0; base < nout; base += blockDim.x) {
    const int o = base + threadIdx.x;
    const int cg = o % ncg, ii = o / ncg;
    C2<R> a0 = mk<R>(0, 0), a1 = a0, a2 = a0, a3 = a0;
    for (int q0 = 0; q0 < 2 * K; q0 += CH) {
      const int qn = min(CH, 2 * K - q0);
      __syncthreads();
#pragma unroll 4
      for (int e = threadIdx.x; e < qn * nc; e += blockDim.x) gs[e] = g[(int64_t)(q0 + e / nc) * ldp + e % nc];
#pragma unroll 4
      for (int e = threadIdx.x; e < nb * qn; e += blockDim.x) {
        const int jj = e / qn, qq = e % qn;
        const int cq = q0 + qq;
        C2<R> v = V[(int64_t)(j0 + jj) * 2 * K + cq];
        const R w = qwc[cq < K ? cq : cq - K];
        vs[jj * CH + qq] = mk<R>(w * v.x, -w * v.y);       // w conj(V)
      }
      __syncthreads();
      if (o < nout) {
        const C2<R>* vr = vs + ii * CH;
        const C2<R>* gr = gs + cg * 4;
        for (int qq = 0; qq < qn; ++qq) {
          const C2<R> w = vr[qq];
          a0 = cfma(a0, w, gr[0]);
          a1 = cfma(a1, w, gr[1]);
          a2 = cfma(a2, w, gr[2]);
          a3 = cfma(a3, w, gr[3]);
          gr += nc;
        }
      }
    }
    if (o < nout) {
      const int64_t i = j0 + ii;
      C2<R> acc[4] = {a0, a1, a2, a3};
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        C2<R> r = yi[i * nc + cg * 4 + u];
        r.x += acc[u].x;
        r.y += acc[u].y;
        if (conj_out) r.y = -r.y;
        y[(int64_t)(perm ? perm[i] : i) * ld + cg * 4 + u] = r;
      }
    }
  }
}

// ---------------------------------------------------------------- SAI apply
// y_pub[perm[i]] = sum_t P[i, t] x_int[col[t]]  (FP64 products)
template <typename R>
__global__ void __launch_bounds__(256) k_sai_apply(const int64_t* __restrict__ ptr, const int32_t* __restrict__ col,
                                                   const double2* __restrict__ val, const C2<R>* __restrict__ xi,
                                                   const int32_t* __restrict__ perm, C2<R>* __restrict__ y, int64_t ld,
                                                   int64_t N, int nc) {
  // a group of G = max(8, NC) lanes per row: NC column lanes times G / NC
  // entry strides (P has about ten entries per row), 64 / G rows per wave
  const int lane = threadIdx.x & 63;
  const int NC = pow2ceil(nc);
  const int G = NC < 8 ? 8 : NC;
  const int l = lane % G;
  const int c = l % NC, s = l / NC, S = G / NC;
  const int64_t i = ((int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6)) * (64 / G) + lane / G;
  double ax = 0.0, ay = 0.0;
  if (i < N && c < nc) {
#pragma unroll 4
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
  for (int o = NC; o < G; o <<= 1) {
    ax += __shfl_xor(ax, o, 64);
    ay += __shfl_xor(ay, o, 64);
  }
  if (i < N && s == 0 && c < nc) y[(int64_t)perm[i] * ld + c] = mk<R>((R)ax, (R)ay);
}

// ---------------------------------------------------------------- launchers
static inline void chk(hipError_t e, const char* what) {
  if (e != hipSuccess) throw Error(-4, std::string(what) + ": " + hipGetErrorString(e));
}

static hipEvent_t take_event(Dev& d) {
  if (!d.event_pool.empty()) {
    hipEvent_t e = d.event_pool.back();
    d.event_pool.pop_back();
    return e;
  }
  hipEvent_t e;
  chk(hipEventCreate(&e), "hipEventCreate");
  return e;
}

void stage_begin(Dev& d, hipStream_t s, int stage) {
  if (!d.timing) return;
  if (d.marks.size() > 65536) collect_stage_times(d);
  Dev::Mark m{stage, take_event(d), take_event(d)};
  chk(hipEventRecord(m.a, s), "hipEventRecord");
  d.marks.push_back(m);
}

void stage_end(Dev& d, hipStream_t s) {
  if (!d.timing) return;
  chk(hipEventRecord(d.marks.back().b, s), "hipEventRecord");
}

void collect_stage_times(Dev& d) {
  if (d.stage_ms.size() < 256) {
    d.stage_ms.assign(256, 0.0);
    d.stage_calls.assign(256, 0);
  }
  for (auto& m : d.marks) {
    chk(hipEventSynchronize(m.b), "hipEventSynchronize");
    float ms = 0.f;
    chk(hipEventElapsedTime(&ms, m.a, m.b), "hipEventElapsedTime");
    d.stage_ms[m.stage] += ms;
    d.stage_calls[m.stage] += 1;
    d.event_pool.push_back(m.a);
    d.event_pool.push_back(m.b);
  }
  d.marks.clear();
}

// column slice width for the interpolation kernels: the LDS grid and the
// per-thread register outputs must fit
template <typename R>
static int interp_cs(int nc, int rows_lds, int cols_lds, int nout_per_col, int jmax, int threads) {
  const size_t lds_cap = 64 * 1024;
  int cs = nc;
  while (cs > 1 && ((size_t)rows_lds * cols_lds * cs * sizeof(C2<R>) > lds_cap || nout_per_col * cs > jmax * threads))
    --cs;
  return cs;
}

static void set_lds_limit(const void* f, size_t bytes) {
  if (bytes > 64 * 1024) chk(hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes),
                             "hipFuncSetAttribute");
}

template <typename R>
struct Stages {
  using CR = C2<R>;
  Dev& d;
  const Plan& P;
  PrecD<R>& pd;
  hipStream_t s;

  void aggregate(const void* V, const CR* xi, int ldx, CR* S, int ldS, int nc) {
    const int K = P.lev[d.lf].K;
    if constexpr (sizeof(R) == 4) {
      if (!(P.opt.flags & CM_FLAG_NO_MATRIX_CORES) &&
          mf_aggregate(V, (const float2*)xi, ldx, (float2*)S, ldS, d.box_start, d.nleaf, K, nc, s))
        return;
    }
    if (nc % 4 == 0 && (size_t)d.max_box * nc * sizeof(CR) <= 48 * 1024) {
      int tot = 2 * K * nc / 4;
      int gy = std::max(1, std::min(4, (tot + 1023) / 1024));
      hipLaunchKernelGGL(k_aggregate_box<R>, dim3(d.nleaf, gy), dim3(256), (size_t)d.max_box * nc * sizeof(CR), s,
                         (const CR*)V, xi, ldx, S, ldS, d.box_start, K, nc);
    } else if (nc % 4 == 0) {
      int tot = 2 * K * nc / 4;
      int gy = std::max(1, std::min(16, (tot + 255) / 256));
      hipLaunchKernelGGL((k_aggregate<R, 4>), dim3(d.nleaf, gy), dim3(256), 0, s, (const CR*)V, xi, ldx, S, ldS,
                         d.box_start, K, nc);
    } else {
      int tot = 2 * K * nc;
      int gy = std::max(1, std::min(16, (tot + 255) / 256));
      hipLaunchKernelGGL((k_aggregate<R, 1>), dim3(d.nleaf, gy), dim3(256), 0, s, (const CR*)V, xi, ldx, S, ldS,
                         d.box_start, K, nc);
    }
  }

  // child level l+1 -> level l; shift = per-octant phase table (or its k-derivative)
  void interp(int l, const CR* Sc, CR* Sp, int nc, int ldp, int accum, const void* shift) {
    if constexpr (sizeof(R) == 4) {
      const void* sT = (shift == pd.lev[l].dshift) ? pd.lev[l].dshiftT : pd.lev[l].shiftT;
      if (!(P.opt.flags & CM_FLAG_NO_MATRIX_CORES) &&
          mf_interp(pd.lev[l], pd.lev[l + 1], (const float2*)Sc, (float2*)Sp, nc, ldp, accum, sT, s))
        return;
    }
    constexpr int kJ = sizeof(R) == 4 ? 16 : 8;
    LevelD<R> Lp = pd.lev[l];
    Lp.shift = const_cast<void*>(shift);
    const int Kc = P.lev[l + 1].K;
    const int per_col = (Lp.ntc * Lp.npc + Lp.ntc * Lp.np) * (int)sizeof(CR);
    const int tables = (Lp.np + Lp.nt) * Lp.p * (4 + (int)sizeof(R));
    const dim3 blk(256);
    if (per_col + tables <= 96 * 1024 && Lp.np <= kJ * 256) {
      int cs = std::max(1, std::min(nc, (64 * 1024 - tables) / per_col));
      while (cs > 1 && std::min(Lp.nt * Lp.np, kJ * 256) * cs > kJ * 256) --cs;
      const int tpc = std::max(1, std::min(Lp.nt, kJ * 256 / (Lp.np * cs)));
      const int nchunk = (Lp.nt + tpc - 1) / tpc;
      const size_t sh = (size_t)per_col * cs + tables;
      set_lds_limit((const void*)k_interp_up<R, kJ>, sh);
      hipLaunchKernelGGL((k_interp_up<R, kJ>), dim3(Lp.nbox * nchunk, (nc + cs - 1) / cs, 2), blk, sh, s, Sc, Sp,
                         Lp.child_ptr, pd.lev[l + 1].octant, Lp, Kc, nc, cs, tpc, ldp, accum);
    } else {
      // each block stages only the child rows its chunk of parent rows reads
      // (a contiguous range: the stencil windows, reflections included, of
      // consecutive parent rows); the chunk shrinks until the range fits
      const Interp& I = P.ip[l];
      const int cs = interp_cs<R>(nc, Lp.ntc, Lp.np, std::min(Lp.nt * Lp.np, kJ * 256), kJ, 256);
      int tpc = std::max(1, std::min(Lp.nt, kJ * 256 / (Lp.np * cs)));
      auto span_of = [&](int tc) {
        int span = 1;
        for (int t0 = 0; t0 < Lp.nt; t0 += tc) {
          int lo = Lp.ntc, hi = -1;
          for (int t = t0; t < std::min(Lp.nt, t0 + tc); ++t)
            for (int j = 0; j < Lp.p; ++j) {
              lo = std::min(lo, I.th_idx[t * Lp.p + j]);
              hi = std::max(hi, I.th_idx[t * Lp.p + j]);
            }
          span = std::max(span, hi - lo + 1);
        }
        return span;
      };
      int span = span_of(tpc);
      while (tpc > 1 && (size_t)span * Lp.np * cs * sizeof(CR) > 160 * 1024) span = span_of(--tpc);
      const int nchunk = (Lp.nt + tpc - 1) / tpc;
      const size_t sh = (size_t)span * Lp.np * cs * sizeof(CR);
      if (sh > 160 * 1024 || tpc * Lp.np * cs > kJ * 256)
        throw Error(-7, "angular grid too large for the interpolation kernel");
      set_lds_limit((const void*)k_interp_up_direct<R, kJ>, sh);
      hipLaunchKernelGGL((k_interp_up_direct<R, kJ>), dim3(Lp.nbox * nchunk, (nc + cs - 1) / cs, 2), blk, sh, s, Sc,
                         Sp, Lp.child_ptr, pd.lev[l + 1].octant, Lp, Kc, nc, cs, tpc, span, ldp, accum);
    }
  }

  void m2l(int l, int kind, const void* T, const CR* S, CR* G, int nc, int ldp, int accum) {
    LevelD<R>& Lv = pd.lev[l];
    const int32_t* tptr = (kind == 1) ? Lv.tileR_ptr : Lv.tile_ptr;
    const int32_t* tsrc = (kind == 1) ? Lv.tileR_src : Lv.tile_src;
    const int32_t* toff = (kind == 1) ? Lv.tileR_off : Lv.tile_off;
    const int cw = std::min(nc, 32);
    const int threads = (nc == 1) ? 64 : 256;           // single vector: more, smaller blocks
    const int qb = threads / cw;
    const int gx = (Lv.ntile + 7) / 8 * 8;              // multiple of 8 for the XCD-aware tile order
    const size_t sh2 = (size_t)Lv.n_off * qb * 2 * sizeof(CR);
    if constexpr (sizeof(R) == 4)
      if (cw >= 8 && (cw & (cw - 1)) == 0 && !(P.opt.flags & CM_FLAG_M2L_TILE16) && Lv.tile64_ptr &&
          Lv.m2l_variant >= 2) {
        // FP32 batched: 64-box tiles sharing their sources through LDS
        // (variant 2: two directions per thread, chunks of 8 sources; 3: the
        // same with chunks of 4 at three waves per SIMD; 4: one direction
        // per thread, chunks of 8, four waves per SIMD)
        const int v = Lv.m2l_variant;
        const int qpt = v == 4 ? 1 : 2, ch = v == 3 ? 4 : 8;
        const int qspan = qpt * 64 / cw;
        const size_t sh = (size_t)Lv.n_off * qspan * sizeof(CR) + (size_t)2 * ch * 2 * qpt * 64 * sizeof(CR);
        if (sh <= 64 * 1024) {
          const int32_t* p64 = (kind == 1) ? Lv.tileR64_ptr : Lv.tile64_ptr;
          const int32_t* s64 = (kind == 1) ? Lv.tileR64_src : Lv.tile64_src;
          const int32_t* o64 = (kind == 1) ? Lv.tileR64_off : Lv.tile64_off;
          dim3 grid((Lv.ntile64 + 7) / 8 * 8, (Lv.K + qspan - 1) / qspan, (nc + cw - 1) / cw);
#define CM_M2L64(Q, CH, W)                                                                                     \
  hipLaunchKernelGGL((k_m2l64<Q, CH, W>), grid, dim3(256), sh, s, p64, s64, o64, (const C2<float>*)T, Lv.n_off, \
                     (const C2<float>*)S, (C2<float>*)G, Lv.nbox, Lv.ntile64, Lv.K, nc, cw, ldp, accum)
          if (v == 3)
            CM_M2L64(2, 4, 3);
          else if (v == 4)
            CM_M2L64(1, 8, 4);
          else
            CM_M2L64(2, 8, 2);
#undef CM_M2L64
          return;
        }
      }
    if constexpr (sizeof(R) == 4)
      if (cw >= 8 && sh2 <= 64 * 1024) {
        // FP32 batched: two directions per thread share the translator ids
        dim3 grid(gx, (Lv.K + 2 * qb - 1) / (2 * qb), (nc + cw - 1) / cw);
        hipLaunchKernelGGL((k_m2l<R, true, 2, kTile, 3>), grid, dim3(threads), sh2, s, tptr, tsrc, toff, (const CR*)T,
                           Lv.n_off, S, G, Lv.nbox, Lv.ntile, Lv.K, nc, cw, ldp, accum);
        return;
      }
    const size_t sh = (size_t)Lv.n_off * qb * sizeof(CR);
    const bool stage = (cw >= 8) && sh <= 64 * 1024;
    dim3 grid(gx, (Lv.K + qb - 1) / qb, (nc + cw - 1) / cw);
    if (nc == 1 && !(P.opt.flags & CM_FLAG_M2L_SINGLE_TILES)) {
      const int32_t* fptr = (kind == 1) ? Lv.farR_ptr : Lv.far_ptr;
      const int32_t* fsrc = (kind == 1) ? Lv.farR_src : Lv.far_src;
      const int32_t* foff = (kind == 1) ? Lv.farR_off : Lv.far_off;
      const int nqc = (Lv.K + 63) / 64;
      const int64_t nw = (int64_t)Lv.nbox * nqc;
      const unsigned gb = (unsigned)((nw + 31) / 32 * 8);   // 4 waves per block, a multiple of 8 blocks
      hipLaunchKernelGGL(k_m2l_pairs<R>, dim3(gb), dim3(256), 0, s, fptr, fsrc, foff, (const CR*)T, S, G, Lv.nbox,
                         Lv.K, nqc, ldp, accum);
      return;
    }
    if (nc == 1) {
      // single vector: one wave per block and few blocks per level, so the
      // tile's 16 receivers go to 4 blocks of grid z (8 where the level has
      // fewer than 32 tiles): 2.30 -> 1.81 ms for the FP64 vector at
      // N = 122,880 (same sums in the same order)
      if (Lv.ntile < 32) {
        grid.z *= kTile / 2;
        hipLaunchKernelGGL((k_m2l<R, false, 1, 2, 4>), grid, dim3(threads), 0, s, tptr, tsrc, toff, (const CR*)T,
                           Lv.n_off, S, G, Lv.nbox, Lv.ntile, Lv.K, nc, cw, ldp, accum);
      } else {
        grid.z *= kTile / 4;
        hipLaunchKernelGGL((k_m2l<R, false, 1, 4, 4>), grid, dim3(threads), 0, s, tptr, tsrc, toff, (const CR*)T,
                           Lv.n_off, S, G, Lv.nbox, Lv.ntile, Lv.K, nc, cw, ldp, accum);
      }
      return;
    }
    if (stage)
      hipLaunchKernelGGL((k_m2l<R, true, 1, kTile, 2>), grid, dim3(threads), sh, s, tptr, tsrc, toff, (const CR*)T, Lv.n_off, S,
                         G, Lv.nbox, Lv.ntile, Lv.K, nc, cw, ldp, accum);
    else
      hipLaunchKernelGGL((k_m2l<R, false, 1, kTile, 2>), grid, dim3(threads), 0, s, tptr, tsrc, toff, (const CR*)T, Lv.n_off, S,
                         G, Lv.nbox, Lv.ntile, Lv.K, nc, cw, ldp, accum);
  }

  // level l -> child level l+1 (accumulates into the child patterns)
  // matrix-core anterpolation: stores into the child patterns (add: adds onto them)
  void anterp_mf(int l, const CR* Gp, CR* Gc, int nc, int ldp, const void* shift, int add) {
    if constexpr (sizeof(R) == 4) {
      const void* zg = (shift == pd.lev[l].dshift) ? pd.lev[l].dzg : pd.lev[l].zg;
      if (mf_anterp(pd.lev[l], pd.lev[l + 1], (const float2*)Gp, (float2*)Gc, nc, ldp, add, zg, s)) return;
    }
    throw Error(-7, "matrix-core anterpolation does not cover this level");
  }

  // vector-ALU anterpolation: adds onto the child patterns
  void anterp(int l, const CR* Gp, CR* Gc, int nc, int ldp, const void* shift) {
    LevelD<R> Lp = pd.lev[l];
    Lp.shift = const_cast<void*>(shift);
    const int Kc = P.lev[l + 1].K;
    const int per_col = (2 * Lp.nt * Lp.np + Lp.nt * Lp.npc) * (int)sizeof(CR);
    const Interp& Ip = P.ip[l];
    const int tables = (Lp.npc + 1 + Lp.ntc + 1) * 4 +
                       (int)(Ip.pht_idx.size() + Ip.tht_idx.size()) * (4 + (int)sizeof(R)) + 16;
    if (per_col + tables <= 144 * 1024) {
      const int cs = std::max(1, std::min(nc, (48 * 1024 - tables) / per_col));   // >= 3 blocks per CU
      const size_t sh = (size_t)per_col * cs + tables;
      set_lds_limit((const void*)k_anterp_down<R>, sh);
      hipLaunchKernelGGL(k_anterp_down<R>, dim3(pd.lev[l + 1].nbox, (nc + cs - 1) / cs, 2), dim3(256), sh, s, Gp,
                         Gc, pd.lev[l + 1].parent, pd.lev[l + 1].octant, Lp, Kc, nc, cs, ldp);
    } else {
      // each block takes a chunk of child rows and stages the transposed phi
      // step of only the parent rows they read (a contiguous range); the
      // chunk shrinks until that range fits
      const int cs = interp_cs<R>(nc, Lp.nt, Lp.npc, 0, 1, 1);
      auto span_of = [&](int tc) {
        int span = 1;
        for (int t0 = 0; t0 < Lp.ntc; t0 += tc) {
          int lo = Lp.nt, hi = -1;
          for (int q = Ip.tht_ptr[t0]; q < Ip.tht_ptr[std::min(Lp.ntc, t0 + tc)]; ++q) {
            lo = std::min(lo, Ip.tht_idx[q]);
            hi = std::max(hi, Ip.tht_idx[q]);
          }
          span = std::max(span, hi - lo + 1);
        }
        return span;
      };
      int tcc = Lp.ntc, span = span_of(tcc);
      while (tcc > 1 && (size_t)span * Lp.npc * cs * sizeof(CR) > 160 * 1024) span = span_of(--tcc);
      const size_t sh = (size_t)span * Lp.npc * cs * sizeof(CR);
      if (sh > 160 * 1024) throw Error(-7, "anterpolation LDS grid exceeds 160 KiB");
      const int nchunk = (Lp.ntc + tcc - 1) / tcc;
      set_lds_limit((const void*)k_anterp_down_direct<R>, sh);
      hipLaunchKernelGGL(k_anterp_down_direct<R>, dim3(pd.lev[l + 1].nbox * nchunk, (nc + cs - 1) / cs, 2),
                         dim3(256), sh, s, Gp, Gc, pd.lev[l + 1].parent, pd.lev[l + 1].octant, Lp, Kc, nc, cs, tcc,
                         span, ldp);
    }
  }

  // y = yi + (k^2 eta/4pi) sum_q w_q conj(V) . G; perm == nullptr writes internal order
  void disagg(const void* V, const CR* G, int ldp, const CR* yi, CR* y, int64_t ld, const int32_t* perm, int nc,
              int conj) {
    const int K = P.lev[d.lf].K;
    if constexpr (sizeof(R) == 4) {
      if (!(P.opt.flags & CM_FLAG_NO_MATRIX_CORES) &&
          mf_disagg(V, (const float2*)G, ldp, (const float*)pd.qwc, (const float2*)yi, d.box_start, d.nleaf,
                    d.max_box, perm, K, nc, (float2*)y, ld, conj, s))
        return;
    }
    if (nc == 1)
      hipLaunchKernelGGL(k_disagg1<R>, dim3((unsigned)((d.N + 3) / 4)), dim3(256), 0, s, (const CR*)V, G,
                         (const R*)pd.qwc, yi, d.box_of, perm, K, d.N, ldp, y, ld, conj);
    else if (nc % 4 == 0 && (size_t)(64 * nc + 64 * d.max_box) * sizeof(CR) <= 64 * 1024)
      hipLaunchKernelGGL(k_disagg_box<R>, dim3(d.nleaf), dim3(256), (size_t)(64 * nc + 64 * d.max_box) * sizeof(CR), s,
                         (const CR*)V, G, (const R*)pd.qwc, yi, d.box_start, perm, K, nc, ldp, y, ld, conj);
    else if (nc % 4 == 0)
      hipLaunchKernelGGL((k_disagg<R, 4>), dim3(d.nleaf), dim3(256), 0, s, (const CR*)V, G, (const R*)pd.qwc, yi,
                         d.box_start, perm, K, nc, ldp, y, ld, conj);
    else
      hipLaunchKernelGGL((k_disagg<R, 1>), dim3(d.nleaf), dim3(256), 0, s, (const CR*)V, G, (const R*)pd.qwc, yi,
                         d.box_start, perm, K, nc, ldp, y, ld, conj);
  }
};

// yi = Z_near xi (kind 0; 1 Re Z of the own box, 2 Im Z; dual: dZ_near/dk),
// internal order, nc contiguous columns
template <typename R>
static void near_product(Dev& d, const Plan& P, const C2<R>* xi, C2<R>* yi, int nc, int kind, bool dual,
                         hipStream_t s) {
  bool done = false;
  if (!(P.opt.flags & CM_FLAG_NO_MATRIX_CORES)) {
    if (sizeof(R) == 4 && (P.opt.flags & CM_FLAG_NEAR_FP32))
      done = mf_near32(d.row_ptr, d.box_start, d.bcol_ptr, d.bcol, d.self_off, dual ? d.dZn32 : d.Zn32,
                       (const float2*)xi, (float2*)yi, d.nleaf, d.max_near_cols, nc, kind, s);
    else
      done = mf_near<R>(d.row_ptr, d.box_start, d.bcol_ptr, d.bcol, d.self_off, (const double2*)(dual ? d.dZn : d.Zn),
                        xi, yi, d.nleaf, d.max_box, d.max_near_cols, nc, kind, s);
  }
  if (done) return;
  if (nc % 4 == 0 && nc <= 64)
    hipLaunchKernelGGL(k_near_box<R>, dim3(d.nleaf), dim3(256), 0, s, d.row_ptr, d.box_start, d.bcol_ptr, d.bcol,
                       d.self_off, (const double2*)(dual ? d.dZn : d.Zn), xi, yi, nc, kind);
  else
    hipLaunchKernelGGL(k_near<R>, dim3((unsigned)((d.N + 3) / 4)), dim3(256), 0, s, d.row_ptr, d.box_of, d.bcol_ptr,
                       d.bcol, d.self_off, d.box_start, (const double2*)(dual ? d.dZn : d.Zn), xi, yi, d.N, nc, kind);
}

template <typename R>
static void apply_impl(Dev& d, const Plan& P, PrecD<R>& pd, int op, const void* x, void* y, int64_t ld, int nc,
                       const Work& w, hipStream_t s) {
  using CR = C2<R>;
  const int lf = d.lf;
  const int64_t N = d.N;
  CR* xi = (CR*)w.xi;
  CR* yi = (CR*)w.yi;
  const bool dual = (op == 4);                          // dZ/dk: values and k-derivatives side by side
  const int conj = (op == 3);
  const int kind = (op == 1) ? 1 : (op == 2) ? 2 : 0;   // 0 Z, 1 R, 2 X
  const int ldp = dual ? 2 * nc : nc;                   // pattern column stride
  // Concurrent schedule (not with stage timing or the dual pass): the near
  // field runs on aux[0] and the translations of levels lf .. 3 on aux[1],
  // each level's as soon as its patterns exist, while the main stream runs
  // the critical path aggregate -> interpolation -> M2L at level 2 ->
  // anterpolation -> disaggregation; both auxiliary streams join the main
  // stream before the first kernel that reads their results.
  const bool fork = !d.timing && !dual && d.aux[0] && d.aux[1] && d.fork_ev.size() >= (size_t)(4 + lf);
  hipStream_t sA = fork ? d.aux[0] : s, sB = fork ? d.aux[1] : s;
  auto fork_to = [&](hipStream_t from, hipStream_t to, int e) {
    if (!fork) return;
    chk(hipEventRecord(d.fork_ev[e], from), "hipEventRecord");
    chk(hipStreamWaitEvent(to, d.fork_ev[e], 0), "hipStreamWaitEvent");
  };
  Stages<R> st{d, P, pd, s};
  Stages<R> stB{d, P, pd, sB};
  {
    int64_t tot = N * nc;
    stage_begin(d, s, 0);
    hipLaunchKernelGGL(k_permute_in<R>, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, (const CR*)x, ld, nc,
                       d.perm, xi, N, conj, nc);
    stage_end(d, s);
  }
  fork_to(s, sA, 0);
  stage_begin(d, sA, 1);
  near_product<R>(d, P, xi, yi, nc, kind, dual, sA);
  stage_end(d, sA);
  if (fork) chk(hipEventRecord(d.fork_ev[1], sA), "hipEventRecord");   // near field done
  // translations and downward pass: the translations of a level are stored,
  // then the parent's anterpolated pattern is added onto them (the
  // matrix-core kernel adds with one atomic per element, so the sum is still
  // formed in a fixed order).
  auto m2l_level = [&](Stages<R>& sx, hipStream_t ss, int l, int accum) {
    LevelD<R>& Lv = pd.lev[l];
    const void* T = (kind == 1) ? Lv.TR : (kind == 2) ? Lv.TX : Lv.TZ;
    stage_begin(d, ss, 4 + 10 * l);
    sx.m2l(l, kind, T, (const CR*)w.S[l], (CR*)w.G[l], dual ? 2 * nc : nc, ldp, accum);
    if (dual) sx.m2l(l, 0, Lv.dTZ, (const CR*)w.S[l], (CR*)w.G[l] + nc, nc, ldp, 1);
    stage_end(d, ss);
  };
  // upward pass; each level's translations start once its patterns exist
  stage_begin(d, s, 2);
  st.aggregate(pd.V, xi, nc, (CR*)w.S[lf], ldp, nc);
  if (dual) st.aggregate(pd.dV, xi, nc, (CR*)w.S[lf] + nc, ldp, nc);
  stage_end(d, s);
  fork_to(s, sB, 2);
  m2l_level(stB, sB, lf, 0);
  for (int l = lf - 1; l >= 2; --l) {
    stage_begin(d, s, 3 + 10 * l);
    st.interp(l, (const CR*)w.S[l + 1], (CR*)w.S[l], dual ? 2 * nc : nc, ldp, 0, pd.lev[l].shift);
    if (dual) st.interp(l, (const CR*)w.S[l + 1], (CR*)w.S[l] + nc, nc, ldp, 1, pd.lev[l].dshift);
    stage_end(d, s);
    if (l >= 3) {
      fork_to(s, sB, 3 + l);
      m2l_level(stB, sB, l, 0);
    } else {
      m2l_level(st, s, l, 0);
    }
  }
  fork_to(sB, s, 3);   // the translations of levels 3 .. lf are stored
  // matrix-core anterpolation where it covers the level (both kernels add
  // onto the child level's stored translations)
  auto mf_down = [&](int l) {
    if constexpr (sizeof(R) == 4)
      return !(P.opt.flags & CM_FLAG_NO_MATRIX_CORES) && nc % 8 == 0 && mf_covers(pd.lev[l], nc);
    return false;
  };
  for (int l = 2; l < lf; ++l) {
    stage_begin(d, s, 5 + 10 * (l + 1));
    if (mf_down(l)) {
      st.anterp_mf(l, (const CR*)w.G[l], (CR*)w.G[l + 1], dual ? 2 * nc : nc, ldp, pd.lev[l].shift, 1);
      if (dual) st.anterp_mf(l, (const CR*)w.G[l], (CR*)w.G[l + 1] + nc, nc, ldp, pd.lev[l].dshift, 1);
    } else {
      st.anterp(l, (const CR*)w.G[l], (CR*)w.G[l + 1], dual ? 2 * nc : nc, ldp, pd.lev[l].shift);
      if (dual) st.anterp(l, (const CR*)w.G[l], (CR*)w.G[l + 1] + nc, nc, ldp, pd.lev[l].dshift);
    }
    stage_end(d, s);
  }
  if (fork) chk(hipStreamWaitEvent(s, d.fork_ev[1], 0), "hipStreamWaitEvent");   // near field
  stage_begin(d, s, 6);
  if (dual) {
    // d/dk of (k^2 eta/4pi) sum w conj(V).G = (2/k)(...) + conj(dV).G + conj(V).dG
    const int64_t rows = (int64_t)d.nleaf * 2 * P.lev[lf].K;
    hipLaunchKernelGGL(k_pattern_axpy<R>, dim3((unsigned)((rows * nc + 255) / 256)), dim3(256), 0, s,
                       (const CR*)w.G[lf], (CR*)w.G[lf] + nc, rows, nc, ldp, (R)(2.0 / P.k));
    st.disagg(pd.dV, (const CR*)w.G[lf], ldp, yi, yi, nc, nullptr, nc, 0);
    st.disagg(pd.V, (const CR*)w.G[lf] + nc, ldp, yi, (CR*)y, ld, d.perm, nc, 0);
  } else {
    st.disagg(pd.V, (const CR*)w.G[lf], ldp, yi, (CR*)y, ld, d.perm, nc, conj);
  }
  stage_end(d, s);
  chk(hipGetLastError(), "apply launch");
}

// One pass over a wavenumber-sweep batch (FP32 far field and vectors, op Z
// or Z^H).  x (public order, row stride ld) holds 4 sw.n columns, slot j being
// columns 4j .. 4j+3 at the wavenumber with index sw.k[j], whose device data
// and plan are dk[sw.k[j]], Pk[sw.k[j]].  Per slot, with its wavenumber's
// tables: the permutation into the slot's block of the permuted input (slot
// blocks N x 8, one after another: the four columns and four zero columns,
// one column tile of the matrix-core kernels), the near field on that block
// (on aux[0] when the handle has its auxiliary streams), the aggregation of
// the slot's four columns into the leaf patterns, and at the end the
// disaggregation.  The interpolation, the translations (levels lf .. 3 on
// aux[1]) and the anterpolation run once over all columns with d0's sweep
// tables: all the wavenumbers share tree, lists and angular sampling.
void dev_apply_sweep(Dev& d0, const Plan& P0, Dev* const* dk, const Plan* const* Pk, const SweepSlots& sw, int op,
                     const void* x, void* y, int64_t ld, hipStream_t s) {
  using CR = C2<float>;
  const int lf = d0.lf;
  const int64_t N = d0.N;
  const int nc = 4 * sw.n;
  const int conj = (op == 3);
  if (!sw.on || sw.n < 1 || !sweep_covers(d0, P0, nc))
    throw Error(-7, "sweep batch not covered by the handle's sweep tables and matrix-core kernels");
  CR* xi = (CR*)d0.xi;
  CR* yi = (CR*)d0.yi;
  const bool fork = !d0.timing && d0.aux[0] && d0.aux[1] && d0.fork_ev.size() >= (size_t)(4 + lf);
  hipStream_t sA = fork ? d0.aux[0] : s, sB = fork ? d0.aux[1] : s;
  auto fork_to = [&](hipStream_t from, hipStream_t to, int e) {
    if (!fork) return;
    chk(hipEventRecord(d0.fork_ev[e], from), "hipEventRecord");
    chk(hipStreamWaitEvent(to, d0.fork_ev[e], 0), "hipStreamWaitEvent");
  };
  constexpr int kSB = 8;   // columns of a slot block (4 of the slot, 4 zero)
  auto xs = [&](int j) { return xi + (int64_t)j * N * kSB; };
  auto ys = [&](int j) { return yi + (int64_t)j * N * kSB; };
  stage_begin(d0, s, 0);
  for (int j = 0; j < sw.n; ++j)
    hipLaunchKernelGGL(k_permute_in<float>, dim3((unsigned)((N * kSB + 255) / 256)), dim3(256), 0, s,
                       (const CR*)x + 4 * j, ld, 4, d0.perm, xs(j), N, conj, kSB);
  stage_end(d0, s);
  fork_to(s, sA, 0);
  // the leaf stages of all slots in one launch each (grid z = slot; the
  // wavenumbers share tree and near-field structure, only the values differ)
  Dev& dz = *dk[sw.k[0]];
  SlotTabs tn;
  for (int j = 0; j < sw.n; ++j) tn.t0[j] = dk[sw.k[j]]->Zn;
  tn.in_off = tn.out_off = 2 * N * kSB;   // floats per slot block
  stage_begin(d0, sA, 1);
  if (!mf_near<float>(dz.row_ptr, dz.box_start, dz.bcol_ptr, dz.bcol, dz.self_off, dz.Zn, xs(0), ys(0), dz.nleaf,
                      dz.max_box, dz.max_near_cols, kSB, 0, sA, &tn, sw.n))
    throw Error(-7, "sweep batch: near-field kernel does not cover the leaf boxes");
  stage_end(d0, sA);
  if (fork) chk(hipEventRecord(d0.fork_ev[1], sA), "hipEventRecord");
  auto m2l = [&](hipStream_t ss, int l) {
    LevelD<float>& Lv = d0.f32.lev[l];
    constexpr int RT = 8, PD = 3;
    const int qb = 256 / sw.n;
    const dim3 grid((Lv.ntile * (kTile / RT) + 7) / 8 * 8, (Lv.K + qb - 1) / qb);
    stage_begin(d0, ss, 4 + 10 * l);
    hipLaunchKernelGGL((k_m2l_slots<RT, PD>), grid, dim3(256), 0, ss, Lv.tile_ptr, Lv.tile_src, Lv.tile_off,
                       (const float2*)Lv.sw_T, d0.sw_nk, sw, (const float2*)d0.S[l], (float2*)d0.G[l], Lv.nbox,
                       Lv.ntile, Lv.K, nc, 0);
    stage_end(d0, ss);
  };
  stage_begin(d0, s, 2);
  SlotTabs ta;
  for (int j = 0; j < sw.n; ++j) ta.t0[j] = dk[sw.k[j]]->f32.V;
  ta.in_off = 2 * N * kSB;   // xi floats per slot block
  ta.out_off = 8;            // S floats per slot (four complex columns)
  mf_aggregate(dz.f32.V, (const float2*)xs(0), kSB, (float2*)d0.S[lf], nc, dz.box_start, dz.nleaf, P0.lev[lf].K, kSB,
               s, 4, &ta, sw.n);
  stage_end(d0, s);
  fork_to(s, sB, 2);
  m2l(sB, lf);
  for (int l = lf - 1; l >= 2; --l) {
    SweepSlots si = sw;
    si.stride = d0.f32.lev[l].sw_shift_stride;
    stage_begin(d0, s, 3 + 10 * l);
    if (!mf_interp(d0.f32.lev[l], d0.f32.lev[l + 1], (const float2*)d0.S[l + 1], (float2*)d0.S[l], nc, nc, 0,
                   d0.f32.lev[l].sw_shiftT, s, &si))
      throw Error(-7, "sweep batch: matrix-core interpolation does not cover this level");
    stage_end(d0, s);
    if (l >= 3) {
      fork_to(s, sB, 3 + l);
      m2l(sB, l);
    } else {
      m2l(s, l);
    }
  }
  fork_to(sB, s, 3);
  for (int l = 2; l < lf; ++l) {
    SweepSlots sz = sw;
    sz.stride = d0.f32.lev[l].sw_zg_stride;
    stage_begin(d0, s, 5 + 10 * (l + 1));
    if (!mf_anterp(d0.f32.lev[l], d0.f32.lev[l + 1], (const float2*)d0.G[l], (float2*)d0.G[l + 1], nc, nc, 1,
                   d0.f32.lev[l].sw_zg, s, &sz))
      throw Error(-7, "sweep batch: matrix-core anterpolation does not cover this level");
    stage_end(d0, s);
  }
  if (fork) chk(hipStreamWaitEvent(s, d0.fork_ev[1], 0), "hipStreamWaitEvent");
  stage_begin(d0, s, 6);
  SlotTabs td;
  for (int j = 0; j < sw.n; ++j) {
    td.t0[j] = dk[sw.k[j]]->f32.V;
    td.t1[j] = dk[sw.k[j]]->f32.qwc;
  }
  td.in_off = 8;               // G floats per slot
  td.aux_off = 2 * N * kSB;    // near-field result floats per slot block
  td.out_off = 8;              // y floats per slot
  if (!mf_disagg(dz.f32.V, (const float2*)d0.G[lf], nc, (const float*)dz.f32.qwc, (const float2*)ys(0),
                 dz.box_start, dz.nleaf, dz.max_box, d0.perm, P0.lev[lf].K, kSB, (float2*)y, ld, conj, s, 4, kSB,
                 &td, sw.n))
    throw Error(-7, "sweep batch: leaf boxes too large for the matrix-core disaggregation");
  stage_end(d0, s);
  chk(hipGetLastError(), "sweep apply launch");
  ++d0.sw_calls;
}

bool sweep_covers(const Dev& d0, const Plan& P0, int nc) {
  if (d0.sw_nk <= 0 || nc % 4 != 0 || nc / 4 > kMaxSlots || nc > d0.max_cols) return false;
  if ((P0.opt.flags & CM_FLAG_NO_MATRIX_CORES) || d0.max_box > 64 || d0.max_near_cols > 4096) return false;
  for (int l = 2; l < d0.lf; ++l)
    if (!mf_interp_covers(d0.f32.lev[l], d0.f32.lev[l + 1], nc, true) || !mf_covers(d0.f32.lev[l], nc, true) ||
        !d0.f32.lev[l].sw_shiftT || !d0.f32.lev[l].sw_zg)
      return false;
  return true;
}

// Autotuning of the FP32 batched translation at nc columns: for every level
// the 16-box-tile kernel and the two 64-box shared-source variants are timed
// on the workspace (one untimed and three timed launches, HIP events on the
// stream) and the fastest is kept.  All variants sum every receiver's
// sources in the same order, so the choice does not change the result.
// Returns the choices as JSON array entries (without brackets).
std::string m2l_autotune(Dev& d, const Plan& P, const std::vector<void*>& S, const std::vector<void*>& G, int nc,
                         hipStream_t s) {
  struct Events {
    hipEvent_t a = nullptr, b = nullptr;
    ~Events() {
      if (a) (void)hipEventDestroy(a);
      if (b) (void)hipEventDestroy(b);
    }
  } ev;
  chk(hipEventCreate(&ev.a), "hipEventCreate (autotune)");
  chk(hipEventCreate(&ev.b), "hipEventCreate (autotune)");
  Stages<float> st{d, P, d.f32, s};
  std::string js;
  for (int l = 2; l <= d.lf; ++l) {
    LevelD<float>& Lv = d.f32.lev[l];
    float best = 1e30f, base = -1.f, vms[5] = {0.f, 0.f, 0.f, 0.f, 0.f};
    int best_v = 0;
    for (int v : {1, 2, 3, 4}) {
      Lv.m2l_variant = v;
      auto launch = [&] { st.m2l(l, 0, Lv.TZ, (const C2<float>*)S[l], (C2<float>*)G[l], nc, nc, 0); };
      launch();
      chk(hipEventRecord(ev.a, s), "hipEventRecord (autotune)");
      for (int i = 0; i < 3; ++i) launch();
      chk(hipEventRecord(ev.b, s), "hipEventRecord (autotune)");
      chk(hipEventSynchronize(ev.b), "autotune timing");
      float ms = 0.f;
      chk(hipEventElapsedTime(&ms, ev.a, ev.b), "hipEventElapsedTime (autotune)");
      ms /= 3.f;
      vms[v] = ms;
      if (v == 1) base = ms;
      if (ms < best) {
        best = ms;
        best_v = v;
      }
    }
    Lv.m2l_variant = best_v;
    char item[256];
    std::snprintf(item, sizeof item,
                  "%s{\"stage\": \"m2l_l%d\", \"tile\": %d, \"chunk\": %d, \"ms\": %.6g, \"tile16_ms\": %.6g, "
                  "\"tile64_chunk8_ms\": %.6g, \"tile64_chunk4_ms\": %.6g, \"tile64_one_direction_ms\": %.6g}",
                  js.empty() ? "" : ", ", l, best_v == 1 ? 16 : 64, best_v == 3 ? 4 : (best_v == 1 ? 0 : 8), best,
                  base, vms[2], vms[3], vms[4]);
    js += item;
  }
  chk(hipGetLastError(), "autotune launches");
  return js;
}

void dev_apply(Dev& d, const Plan& P, int op, const void* x, void* y, int64_t ld, int nc, bool fp64,
               hipStream_t s) {
  if (op == 4 && (!d.dZn || !d.f64.dV)) throw Error(-5, "dZ/dk needs CM_FLAG_DERIV at create");
  Work w;
  for (int l = 2; l <= d.lf; ++l) {
    w.S[l] = d.S[l];
    w.G[l] = d.G[l];
  }
  w.xi = d.xi;
  w.yi = d.yi;
  if (fp64)
    apply_impl<double>(d, P, d.f64, op, x, y, ld, nc, w, s);
  else
    apply_impl<float>(d, P, d.f32, op, x, y, ld, nc, w, s);
}

size_t work_bytes(const Plan& P, int op, int nc, bool fp64, size_t sizes[kMaxLevels]) {
  const size_t cb = fp64 ? 16 : 8;
  const size_t ldp = (op == 4) ? 2 * (size_t)nc : (size_t)nc;
  auto up = [](size_t b) { return (b + 255) / 256 * 256; };
  size_t tot = 0;
  for (int l = 0; l < kMaxLevels; ++l) sizes[l] = 0;
  sizes[0] = up((size_t)P.rwg.N * nc * cb);
  tot += 2 * sizes[0];
  for (int l = 2; l <= P.lf; ++l) {
    sizes[l] = up((size_t)P.lev[l].nbox * 2 * P.lev[l].K * ldp * cb);
    tot += 2 * sizes[l];
  }
  return tot;
}

void dev_apply_ws(Dev& d, const Plan& P, int op, const void* x, void* y, int64_t ld, int nc, bool fp64,
                  const Work& w, hipStream_t s) {
  if (op == 4 && (!d.dZn || !d.f64.dV)) throw Error(-5, "dZ/dk needs CM_FLAG_DERIV at create");
  // stage timing records events from a pool that may grow: off for this call
  const bool timing = d.timing;
  d.timing = false;
  try {
    if (fp64)
      apply_impl<double>(d, P, d.f64, op, x, y, ld, nc, w, s);
    else
      apply_impl<float>(d, P, d.f32, op, x, y, ld, nc, w, s);
  } catch (...) {
    d.timing = timing;
    throw;
  }
  d.timing = timing;
}

template <typename R>
static void sai_apply_impl(Dev& d, const SaiD& q, const void* x, void* y, int64_t ld, int nc, hipStream_t s) {
  using CR = C2<R>;
  const int64_t N = d.N;
  int64_t tot = N * nc;
  hipLaunchKernelGGL(k_permute_in<R>, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, (const CR*)x, ld, nc,
                     d.perm, (CR*)d.xi, N, 0, nc);
  stage_begin(d, s, 7);
  const int NC = nc <= 1 ? 1 : 1 << (32 - __builtin_clz((unsigned)(nc - 1)));
  const int64_t waves = (N + 64 / std::max(8, NC) - 1) / (64 / std::max(8, NC));
  hipLaunchKernelGGL(k_sai_apply<R>, dim3((unsigned)((waves + 3) / 4)), dim3(256), 0, s, q.ptr, q.col,
                     (const double2*)q.val, (const CR*)d.xi, d.perm, (CR*)y, ld, N, nc);
  stage_end(d, s);
  chk(hipGetLastError(), "sai apply launch");
}

void dev_sai_apply(Dev& d, const Plan& P, const void* x, void* y, int64_t ld, int nc, bool fp64, int part,
                   hipStream_t s) {
  (void)P;
  const SaiD& q = d.sai[part];
  if (!q.val) throw Error(-5, "SAI preconditioner not built");
  if (fp64)
    sai_apply_impl<double>(d, q, x, y, ld, nc, s);
  else
    sai_apply_impl<float>(d, q, x, y, ld, nc, s);
}

}  // namespace cm
