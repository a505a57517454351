// Set-up kernels (FP64): near-field Galerkin fill with singularity extraction
// (eq. (5), first term of eq. (11)) and leaf radiation patterns (eq. (13)).
#include <hip/hip_runtime.h>

#include "cm_device.h"

namespace cm {

// 7-point degree-5 triangle rule (barycentric points, weights summing to 1)
__constant__ double c_bary[7][3];
__constant__ double c_w7[7];

struct cd {
  double x, y;
};
__device__ __forceinline__ cd cmk(double a, double b) { return cd{a, b}; }
__device__ __forceinline__ cd operator+(cd a, cd b) { return cd{a.x + b.x, a.y + b.y}; }
__device__ __forceinline__ cd operator-(cd a, cd b) { return cd{a.x - b.x, a.y - b.y}; }
__device__ __forceinline__ cd operator*(cd a, cd b) { return cd{a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x}; }
__device__ __forceinline__ cd operator*(double s, cd a) { return cd{s * a.x, s * a.y}; }

__device__ __forceinline__ void qpoint(const TriD& T, int p, double* r) {
  for (int d = 0; d < 3; ++d)
    r[d] = c_bary[p][0] * T.v[d] + c_bary[p][1] * T.v[3 + d] + c_bary[p][2] * T.v[6 + d];
}

// ln(R + l) without cancellation: for l < 0, R + l = R0^2/(R - l)
__device__ __forceinline__ double log_rl(double R, double l, double R0sq) {
  return (l >= 0.0) ? log(R + l) : log(R0sq) - log(R - l);
}

// Closed-form int_T 1/|r-r'| dS' and int_T (rho'-rho)/|r-r'| dS' over a flat
// triangle (Wilton et al. 1984, Graglia 1993): edge-by-edge sums of
// logarithms and arctangents in the triangle's own plane.
__device__ void potint(const double* r, const TriD& T, double& I1, double* Iv) {
  const double* n = T.n;
  double d = (r[0] - T.v[0]) * n[0] + (r[1] - T.v[1]) * n[1] + (r[2] - T.v[2]) * n[2];
  double rho[3] = {r[0] - d * n[0], r[1] - d * n[1], r[2] - d * n[2]};
  double ad = fabs(d);
  I1 = 0.0;
  Iv[0] = Iv[1] = Iv[2] = 0.0;
  double e0[3] = {T.v[3] - T.v[0], T.v[4] - T.v[1], T.v[5] - T.v[2]};
  double scale2 = e0[0] * e0[0] + e0[1] * e0[1] + e0[2] * e0[2];
  for (int i = 0; i < 3; ++i) {
    const double* a = &T.v[3 * i];
    const double* b = &T.v[3 * ((i + 1) % 3)];
    double s[3] = {b[0] - a[0], b[1] - a[1], b[2] - a[2]};
    double sl = sqrt(s[0] * s[0] + s[1] * s[1] + s[2] * s[2]);
    s[0] /= sl; s[1] /= sl; s[2] /= sl;
    double u[3] = {s[1] * n[2] - s[2] * n[1], s[2] * n[0] - s[0] * n[2], s[0] * n[1] - s[1] * n[0]};
    double lp = (b[0] - rho[0]) * s[0] + (b[1] - rho[1]) * s[1] + (b[2] - rho[2]) * s[2];
    double lm = (a[0] - rho[0]) * s[0] + (a[1] - rho[1]) * s[1] + (a[2] - rho[2]) * s[2];
    double P0 = (a[0] - rho[0]) * u[0] + (a[1] - rho[1]) * u[1] + (a[2] - rho[2]) * u[2];
    double Rp = sqrt((r[0] - b[0]) * (r[0] - b[0]) + (r[1] - b[1]) * (r[1] - b[1]) + (r[2] - b[2]) * (r[2] - b[2]));
    double Rm = sqrt((r[0] - a[0]) * (r[0] - a[0]) + (r[1] - a[1]) * (r[1] - a[1]) + (r[2] - a[2]) * (r[2] - a[2]));
    double R0sq = P0 * P0 + d * d;
    double Lg = 0.0, At = 0.0;
    if (R0sq > 1e-28 * scale2) {
      Lg = log_rl(Rp, lp, R0sq) - log_rl(Rm, lm, R0sq);
      At = atan(P0 * lp / (R0sq + ad * Rp)) - atan(P0 * lm / (R0sq + ad * Rm));
    }
    I1 += P0 * Lg - ad * At;
    double g = 0.5 * (R0sq * Lg + lp * Rp - lm * Rm);
    Iv[0] += g * u[0];
    Iv[1] += g * u[1];
    Iv[2] += g * u[2];
  }
}

// Integrals over a triangle pair, outer 7-point rule on To, inner on Ts:
//   S0 = int int G,  Sv = int int (r - v_a).(r' - v'_b) G,  G = exp(-ikR)/R,
// with the 1/R part of the inner integral in closed form when sing is set;
// with deriv, E0/Ev are the same integrals of exp(-ikR).
__device__ void pair_int(double k, const TriD& To, int a, const TriD& Ts, int b, bool sing, bool deriv, cd& S0,
                         cd& Sv, cd& E0, cd& Ev) {
  S0 = Sv = E0 = Ev = cmk(0, 0);
  const double* va = &To.v[3 * a];
  const double* vb = &Ts.v[3 * b];
  double rs[7][3];
  for (int q = 0; q < 7; ++q) qpoint(Ts, q, rs[q]);
  for (int p = 0; p < 7; ++p) {
    double r[3];
    qpoint(To, p, r);
    double ua[3] = {r[0] - va[0], r[1] - va[1], r[2] - va[2]};
    double wo = c_w7[p] * To.area;
    cd s0 = cmk(0, 0), sv = cmk(0, 0), e0 = cmk(0, 0), ev = cmk(0, 0);
    for (int q = 0; q < 7; ++q) {
      double dx = r[0] - rs[q][0], dy = r[1] - rs[q][1], dz = r[2] - rs[q][2];
      double R = sqrt(dx * dx + dy * dy + dz * dz);
      double dot = ua[0] * (rs[q][0] - vb[0]) + ua[1] * (rs[q][1] - vb[1]) + ua[2] * (rs[q][2] - vb[2]);
      double ws = c_w7[q] * Ts.area;
      double sn, cs;
      sincos(k * R, &sn, &cs);
      cd g;
      if (sing) {
        if (R > 0.0) {
          double sh = sin(0.5 * k * R);
          g = cmk(-2.0 * sh * sh / R, -sn / R);   // (exp(-ikR) - 1)/R
        } else {
          g = cmk(0.0, -k);
        }
      } else {
        g = cmk(cs / R, -sn / R);
      }
      s0 = s0 + (ws)*g;
      sv = sv + (ws * dot) * g;
      if (deriv) {
        cd e = cmk(cs, -sn);
        e0 = e0 + ws * e;
        ev = ev + (ws * dot) * e;
      }
    }
    if (sing) {
      double I1, Iv[3];
      potint(r, Ts, I1, Iv);
      double d = (r[0] - Ts.v[0]) * Ts.n[0] + (r[1] - Ts.v[1]) * Ts.n[1] + (r[2] - Ts.v[2]) * Ts.n[2];
      // int (r' - v'_b)/R = [int (rho'-rho)/R - d n int 1/R] + (r - v'_b) int 1/R
      double in[3];
      for (int c = 0; c < 3; ++c) in[c] = Iv[c] - d * Ts.n[c] * I1 + (r[c] - vb[c]) * I1;
      s0 = s0 + cmk(I1, 0.0);
      sv = sv + cmk(ua[0] * in[0] + ua[1] * in[1] + ua[2] * in[2], 0.0);
    }
    S0 = S0 + wo * s0;
    Sv = Sv + wo * sv;
    if (deriv) {
      E0 = E0 + wo * e0;
      Ev = Ev + wo * ev;
    }
  }
}

// Galerkin block of one half-function pair: Z part and dZ/dk part (without
// the sign and edge-length factors).
__device__ void half_block(double k, double eta, const TriD& To, int a, const TriD& Ts, int b, bool deriv, cd& z,
                           cd& dz) {
  double dx = To.c[0] - Ts.c[0], dy = To.c[1] - Ts.c[1], dzz = To.c[2] - Ts.c[2];
  double h = 1.5 * fmax(To.hmax, Ts.hmax);
  bool sing = (dx * dx + dy * dy + dzz * dzz) < h * h;
  double AA = To.area * Ts.area;
  cd S0, Sv, E0, Ev;
  pair_int(k, To, a, Ts, b, sing, deriv, S0, Sv, E0, Ev);
  cd inner = (1.0 / (4.0 * AA)) * Sv - (1.0 / (k * k * AA)) * S0;
  z = cmk(0.0, k * eta) * inner;
  if (deriv) {
    cd t1 = cmk(0.0, eta) * ((1.0 / (4.0 * AA)) * Sv + (1.0 / (k * k * AA)) * S0);
    cd t2 = eta * ((k / (4.0 * AA)) * Ev - (1.0 / (k * AA)) * E0);
    dz = t1 + t2;
  }
  if (sing) {
    // average with the evaluation that has the roles of the triangles exchanged
    cd S0b, Svb, E0b, Evb;
    pair_int(k, Ts, b, To, a, true, deriv, S0b, Svb, E0b, Evb);
    cd innerb = (1.0 / (4.0 * AA)) * Svb - (1.0 / (k * k * AA)) * S0b;
    z = 0.5 * (z + cmk(0.0, k * eta) * innerb);
    if (deriv) {
      cd t1 = cmk(0.0, eta) * ((1.0 / (4.0 * AA)) * Svb + (1.0 / (k * k * AA)) * S0b);
      cd t2 = eta * ((k / (4.0 * AA)) * Evb - (1.0 / (k * AA)) * E0b);
      dz = 0.5 * (dz + t1 + t2);
    }
  }
}

// One workgroup per leaf box: the dense block (rows of the box) x (columns of
// its near boxes), stored row by row at row_ptr.
__global__ void __launch_bounds__(256) k_near_fill(double k, double eta, const TriD* __restrict__ tri,
                                                   const RwgD* __restrict__ rwg, const int32_t* __restrict__ box_start,
                                                   const int32_t* __restrict__ bcol_ptr,
                                                   const int32_t* __restrict__ bcol, const int64_t* __restrict__ row_ptr,
                                                   double2* __restrict__ Zn, double2* __restrict__ dZn, int nbox) {
  int b = blockIdx.x;
  if (b >= nbox) return;
  int r0 = box_start[b], nr = box_start[b + 1] - r0;
  int c0 = bcol_ptr[b], ncl = bcol_ptr[b + 1] - c0;
  int64_t tot = (int64_t)nr * ncl;
  bool deriv = (dZn != nullptr);
  for (int64_t e = threadIdx.x; e < tot; e += blockDim.x) {
    int ir = (int)(e / ncl), t = (int)(e % ncl);
    int i = r0 + ir, j = bcol[c0 + t];
    RwgD m = rwg[i], n = rwg[j];
    cd z = cmk(0, 0), dz = cmk(0, 0);
    for (int sm = 0; sm < 2; ++sm) {
      TriD To = tri[m.t[sm]];
      for (int sn = 0; sn < 2; ++sn) {
        const TriD& Ts = tri[n.t[sn]];
        cd zb, dzb;
        half_block(k, eta, To, m.a[sm], Ts, n.a[sn], deriv, zb, dzb);
        double sg = ((sm == sn) ? 1.0 : -1.0) * m.len * n.len;
        z = z + sg * zb;
        if (deriv) dz = dz + sg * dzb;
      }
    }
    int64_t at = row_ptr[i] + t;
    Zn[at] = make_double2(z.x, z.y);
    if (deriv) dZn[at] = make_double2(dz.x, dz.y);
  }
}

// Leaf radiation patterns (eq. (13), exp(-ikR) convention):
//   V_j(khat) = (theta-hat, phi-hat) . sum_{T in j} sum_p w_p A f_j(r_p) exp(ik khat.(r_p - c_box))
// and their k-derivative (factor i khat.(r_p - c_box)).
__global__ void __launch_bounds__(256) k_leaf_patterns(double k, const TriD* __restrict__ tri,
                                                       const RwgD* __restrict__ rwg,
                                                       const int32_t* __restrict__ box_of,
                                                       const double* __restrict__ center,
                                                       const double* __restrict__ dirs, int K, int64_t N,
                                                       double2* __restrict__ V64, float2* __restrict__ V32,
                                                       double2* __restrict__ dV64, float2* __restrict__ dV32) {
  int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (gid >= N * K) return;
  int64_t i = gid / K;
  int q = (int)(gid % K);
  const double* D = &dirs[9 * q];
  const double* cb = &center[3 * box_of[i]];
  RwgD m = rwg[i];
  cd F[3] = {cmk(0, 0), cmk(0, 0), cmk(0, 0)};
  cd dF[3] = {cmk(0, 0), cmk(0, 0), cmk(0, 0)};
  for (int s = 0; s < 2; ++s) {
    const TriD& T = tri[m.t[s]];
    const double* pv = &T.v[3 * m.a[s]];
    double coef = (s == 0 ? 1.0 : -1.0) * m.len / (2.0 * T.area);
    for (int p = 0; p < 7; ++p) {
      double r[3];
      qpoint(T, p, r);
      double ph = D[0] * (r[0] - cb[0]) + D[1] * (r[1] - cb[1]) + D[2] * (r[2] - cb[2]);
      double sn, cs;
      sincos(k * ph, &sn, &cs);
      double w = c_w7[p] * T.area * coef;
      for (int d = 0; d < 3; ++d) {
        double f = w * (r[d] - pv[d]);
        F[d] = F[d] + cmk(f * cs, f * sn);
        dF[d] = dF[d] + cmk(-f * ph * sn, f * ph * cs);   // i ph exp(i k ph)
      }
    }
  }
  cd vt = D[3] * F[0] + D[4] * F[1] + D[5] * F[2];
  cd vp = D[6] * F[0] + D[7] * F[1] + D[8] * F[2];
  int64_t o0 = (i * 2 + 0) * K + q, o1 = (i * 2 + 1) * K + q;
  V64[o0] = make_double2(vt.x, vt.y);
  V64[o1] = make_double2(vp.x, vp.y);
  V32[o0] = make_float2((float)vt.x, (float)vt.y);
  V32[o1] = make_float2((float)vp.x, (float)vp.y);
  if (dV64) {
    cd dvt = D[3] * dF[0] + D[4] * dF[1] + D[5] * dF[2];
    cd dvp = D[6] * dF[0] + D[7] * dF[1] + D[8] * dF[2];
    dV64[o0] = make_double2(dvt.x, dvt.y);
    dV64[o1] = make_double2(dvp.x, dvp.y);
    dV32[o0] = make_float2((float)dvt.x, (float)dvt.y);
    dV32[o1] = make_float2((float)dvp.x, (float)dvp.y);
  }
}

void set_quadrature_constants() {
  const double s15 = sqrt(15.0);
  const double A = (6.0 - s15) / 21.0, B = (6.0 + s15) / 21.0;
  const double WA = (155.0 - s15) / 1200.0, WB = (155.0 + s15) / 1200.0;
  double bary[7][3] = {{1.0 / 3, 1.0 / 3, 1.0 / 3}, {A, A, 1 - 2 * A}, {A, 1 - 2 * A, A}, {1 - 2 * A, A, A},
                       {B, B, 1 - 2 * B}, {B, 1 - 2 * B, B}, {1 - 2 * B, B, B}};
  double w[7] = {9.0 / 40.0, WA, WA, WA, WB, WB, WB};
  if (hipMemcpyToSymbol(HIP_SYMBOL(c_bary), bary, sizeof bary) != hipSuccess ||
      hipMemcpyToSymbol(HIP_SYMBOL(c_w7), w, sizeof w) != hipSuccess)
    throw Error(-4, "hipMemcpyToSymbol failed for the quadrature rule");
}

void launch_near_fill(double k, double eta, const Dev& d, int nbox, hipStream_t s) {
  hipLaunchKernelGGL(k_near_fill, dim3(nbox), dim3(256), 0, s, k, eta, d.tri, d.rwg, d.box_start, d.bcol_ptr, d.bcol,
                     d.row_ptr, d.Zn, d.dZn, nbox);
}

void launch_leaf_patterns(double k, const Dev& d, hipStream_t s) {
  int64_t tot = d.N * d.Kleaf;
  int nb = (int)((tot + 255) / 256);
  hipLaunchKernelGGL(k_leaf_patterns, dim3(nb), dim3(256), 0, s, k, d.tri, d.rwg, d.box_of, d.leaf_center,
                     d.leaf_dirs, d.Kleaf, d.N, (double2*)d.f64.V, (float2*)d.f32.V, (double2*)d.f64.dV,
                     (float2*)d.f32.dV);
}

}  // namespace cm
