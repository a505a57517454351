// Calderon multiplicative preconditioner (section IV, eqs. (25)-(27)): host
// set-up.  The preconditioned system is Z~ G^-1 Z x = Z~ G^-1 u with Z~ the
// EFIE between Buffa-Christiansen (BC) functions and G_ij = <n x f_i, f~_j>.
//
// The BC functions live on the barycentric refinement (six small triangles
// per triangle: corner a of triangle t gives small triangles 6t + 2a =
// (v_a, m(a, a+1), c_t) and 6t + 2a + 1 = (v_a, c_t, m(a-1, a)), with m the
// edge midpoints and c_t the centroid, in t's orientation).  Z~ is applied as
// B Z_ref B^T with Z_ref the MLFMA of the refined mesh's RWG functions and B
// the BC functions' coefficients on them.  The BC function of the primal edge
// e = (v_s, v_t) (v_s -> v_t along n x f_e, n the normal of T+) carries the
// flux l_e out of the dual cell of v_s (its 2N_s small triangles) into that
// of v_t, half through each half of the dual edge (the refined edges from the
// midpoint of e to the centroids of T+ and T-), with equal charge on every
// small triangle of a cell and no flux through the refined edges from v_s and
// v_t to the midpoint of e: walking the cell of v from that refined edge, the
// flux through the j-th radiating refined edge is (j - N) l_e / (2N) for the
// source cell and its negative for the sink cell.  Closed surfaces only.
#include <algorithm>
#include <array>
#include <cmath>
#include <unordered_map>
#include <vector>

#include "cm_device.h"

namespace cm {

static inline uint64_t pair_key(int32_t a, int32_t b) {
  if (a > b) std::swap(a, b);
  return ((uint64_t)(uint32_t)a << 32) | (uint32_t)b;
}

static std::unordered_map<uint64_t, int32_t> edge_index(const Rwg& r) {
  std::unordered_map<uint64_t, int32_t> m;
  m.reserve((size_t)r.N * 2);
  for (int64_t e = 0; e < r.N; ++e) m[pair_key(r.edge[2 * e], r.edge[2 * e + 1])] = (int32_t)e;
  return m;
}

void cmp_refine(const Plan& P, std::vector<double>& Vr, std::vector<int32_t>& Fr) {
  const int64_t nv = P.nv, nt = P.nt, N = P.rwg.N;
  if (3 * nt != 2 * N)
    throw Error(CM_E_MESH, "the Calderon preconditioner needs a closed surface (every edge shared by two triangles)");
  // vertices: primal, then the midpoint of RWG e (nv + e), then the centroid of t (nv + N + t)
  Vr.assign((size_t)3 * (nv + N + nt), 0.0);
  std::copy(P.V.begin(), P.V.end(), Vr.begin());
  for (int64_t e = 0; e < N; ++e)
    for (int d = 0; d < 3; ++d)
      Vr[3 * (nv + e) + d] = 0.5 * (P.V[3 * P.rwg.edge[2 * e] + d] + P.V[3 * P.rwg.edge[2 * e + 1] + d]);
  for (int64_t t = 0; t < nt; ++t)
    for (int d = 0; d < 3; ++d)
      Vr[3 * (nv + N + t) + d] =
          (P.V[3 * P.F[3 * t] + d] + P.V[3 * P.F[3 * t + 1] + d] + P.V[3 * P.F[3 * t + 2] + d]) / 3.0;
  const auto eid = edge_index(P.rwg);
  Fr.assign((size_t)18 * nt, 0);
  for (int64_t t = 0; t < nt; ++t) {
    const int32_t* v = &P.F[3 * t];
    const int32_t c = (int32_t)(nv + N + t);
    for (int a = 0; a < 3; ++a) {
      const int32_t mn = (int32_t)nv + eid.at(pair_key(v[a], v[(a + 1) % 3]));
      const int32_t mp = (int32_t)nv + eid.at(pair_key(v[(a + 2) % 3], v[a]));
      int32_t* s0 = &Fr[18 * t + 6 * a];
      s0[0] = v[a], s0[1] = mn, s0[2] = c;
      s0[3] = v[a], s0[4] = c, s0[5] = mp;
    }
  }
}

static void to_csr(int64_t rows, std::vector<std::pair<int64_t, std::pair<int32_t, double>>>& coo, CsrHost& M) {
  std::sort(coo.begin(), coo.end(), [](const auto& x, const auto& y) {
    return x.first != y.first ? x.first < y.first : x.second.first < y.second.first;
  });
  M.rows = rows;
  M.ptr.assign(rows + 1, 0);
  M.col.clear();
  M.val.clear();
  for (size_t i = 0; i < coo.size();) {
    size_t k = i;
    double s = 0;
    while (k < coo.size() && coo[k].first == coo[i].first && coo[k].second.first == coo[i].second.first)
      s += coo[k++].second.second;
    if (s != 0.0) {
      M.col.push_back(coo[i].second.first);
      M.val.push_back(s);
      M.ptr[coo[i].first + 1]++;
    }
    i = k;
  }
  for (int64_t r = 0; r < rows; ++r) M.ptr[r + 1] += M.ptr[r];
}

void cmp_tables(const Plan& P, const Plan& Pr, const std::vector<double>& Vr, const std::vector<int32_t>& Fr,
                CsrHost& B, CsrHost& Bt, CsrHost& G) {
  const int64_t N = P.rwg.N, Nr = Pr.rwg.N;
  const auto eid = edge_index(P.rwg);
  const auto rid = edge_index(Pr.rwg);
  auto corner = [&](int64_t T, int32_t v) {
    for (int a = 0; a < 3; ++a)
      if (P.F[3 * T + a] == v) return a;
    throw Error(CM_E_MESH, "Calderon set-up: inconsistent vertex fan");
  };
  auto sub = [](const double* a, const double* b, double* o) {
    for (int d = 0; d < 3; ++d) o[d] = a[d] - b[d];
  };
  auto cross = [](const double* a, const double* b, double* o) {
    o[0] = a[1] * b[2] - a[2] * b[1];
    o[1] = a[2] * b[0] - a[0] * b[2];
    o[2] = a[0] * b[1] - a[1] * b[0];
  };
  auto dot = [](const double* a, const double* b) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; };
  std::vector<std::pair<int64_t, std::pair<int32_t, double>>> cb, cg;
  cb.reserve((size_t)N * 26);
  cg.reserve((size_t)N * 40);
  std::vector<int64_t> seq;
  std::vector<std::pair<int64_t, std::array<double, 3>>> out;   // small triangle -> outward fluxes
  for (int64_t j = 0; j < N; ++j) {
    const int32_t a = P.rwg.edge[2 * j], b = P.rwg.edge[2 * j + 1];
    const double le = P.rwg.len[j];
    const int64_t Tp = P.rwg.tri[2 * j];
    const double* pp = &P.V[3 * P.F[3 * Tp + P.rwg.loc[2 * j]]];
    double mid[3], d[3], nd[3], ab[3];
    for (int q = 0; q < 3; ++q) mid[q] = 0.5 * (P.V[3 * a + q] + P.V[3 * b + q]);
    sub(mid, pp, d);
    cross(&P.normal[3 * Tp], d, nd);
    sub(&P.V[3 * b], &P.V[3 * a], ab);
    const int32_t vs = dot(ab, nd) > 0 ? a : b, vt = vs == a ? b : a;
    out.clear();
    auto outflux = [&](int64_t t, int32_t u, int32_t w, double f) {
      // add f to the outward flux of small triangle t through its edge (u, w)
      int loc = -1;
      for (int q = 0; q < 3; ++q)
        if (Fr[3 * t + q] != u && Fr[3 * t + q] != w) loc = q;
      for (auto& o : out)
        if (o.first == t) {
          o.second[loc] += f;
          return;
        }
      std::array<double, 3> z{0.0, 0.0, 0.0};
      z[loc] = f;
      out.push_back({t, z});
    };
    auto flux = [&](int64_t t_from, int32_t u, int32_t w, double f) {
      // flux f from small triangle t_from through refined edge (u, w) into its neighbour
      const auto it = rid.find(pair_key(u, w));
      if (it == rid.end()) throw Error(CM_E_MESH, "Calderon set-up: refined edge without an RWG");
      const int32_t r = it->second;
      const int64_t tp = Pr.rwg.tri[2 * r], tm = Pr.rwg.tri[2 * r + 1];
      if (t_from != tp && t_from != tm) throw Error(CM_E_MESH, "Calderon set-up: inconsistent refined edge");
      cb.push_back({j, {r, (t_from == tp ? f : -f) / Pr.rwg.len[r]}});
      outflux(t_from, u, w, f);
      outflux(t_from == tp ? tm : tp, u, w, -f);
    };
    for (int side = 0; side < 2; ++side) {
      const int32_t v = side == 0 ? vs : vt;
      const double sign = side == 0 ? 1.0 : -1.0;
      // the fan of v from edge j: two small triangles per primal triangle
      seq.clear();
      int64_t T = Tp;
      int32_t e_in = (int32_t)j;
      for (;;) {
        const int ac = corner(T, v);
        const int32_t e_next = eid.at(pair_key(v, P.F[3 * T + (ac + 1) % 3]));
        const int32_t e_prev = eid.at(pair_key(P.F[3 * T + (ac + 2) % 3], v));
        int32_t e_out;
        if (e_in == e_next) {
          seq.push_back(6 * T + 2 * ac);
          seq.push_back(6 * T + 2 * ac + 1);
          e_out = e_prev;
        } else if (e_in == e_prev) {
          seq.push_back(6 * T + 2 * ac + 1);
          seq.push_back(6 * T + 2 * ac);
          e_out = e_next;
        } else {
          throw Error(CM_E_MESH, "Calderon set-up: inconsistent vertex fan");
        }
        if (e_out == (int32_t)j) break;
        T = P.rwg.tri[2 * e_out] == T ? P.rwg.tri[2 * e_out + 1] : P.rwg.tri[2 * e_out];
        e_in = e_out;
        if (seq.size() > 2 * (size_t)P.nt) throw Error(CM_E_MESH, "Calderon set-up: open vertex fan");
      }
      const int64_t n2 = (int64_t)seq.size(), nh = n2 / 2;
      for (int64_t q = 1; q < n2; ++q) {
        // the radiating refined edge (v, w) shared by seq[q-1] and seq[q]
        int32_t w = -1;
        for (int x = 0; x < 3; ++x) {
          const int32_t cand = Fr[3 * seq[q - 1] + x];
          if (cand == v) continue;
          for (int y = 0; y < 3; ++y)
            if (Fr[3 * seq[q] + y] == cand) w = cand;
        }
        if (w < 0) throw Error(CM_E_MESH, "Calderon set-up: inconsistent vertex fan");
        flux(seq[q - 1], v, w, sign * le * (double)(q - nh) / (double)n2);
      }
      if (side == 0) {
        // half of the flux out through each half of the dual edge (the rim
        // edges of the first and last small triangles, opposite v)
        for (int64_t t : {seq.front(), seq.back()}) {
          int32_t rim[2], k = 0;
          for (int x = 0; x < 3; ++x)
            if (Fr[3 * t + x] != v) rim[k++] = Fr[3 * t + x];
          flux(t, rim[0], rim[1], 0.5 * le);
        }
      }
    }
    // column j of G: <n x f_i, f~_j> on every small triangle of the support,
    // the three edge-midpoint rule being exact for the quadratic integrand
    for (const auto& o : out) {
      const int64_t t = o.first, T = t / 6;
      const double* w0 = &Vr[3 * Fr[3 * t]];
      const double* w1 = &Vr[3 * Fr[3 * t + 1]];
      const double* w2 = &Vr[3 * Fr[3 * t + 2]];
      const double* wv[3] = {w0, w1, w2};
      double e1[3], e2[3], cr[3];
      sub(w1, w0, e1);
      sub(w2, w0, e2);
      cross(e1, e2, cr);
      const double At = 0.5 * std::sqrt(dot(cr, cr));
      double qp[3][3];
      for (int q = 0; q < 3; ++q)
        for (int x = 0; x < 3; ++x) qp[q][x] = 0.5 * (wv[(q + 1) % 3][x] + wv[(q + 2) % 3][x]);
      const double* nT = &P.normal[3 * T];
      const double AT = P.area[T];
      for (int c = 0; c < 3; ++c) {
        const int32_t i = eid.at(pair_key(P.F[3 * T + c], P.F[3 * T + (c + 1) % 3]));
        const double sg = P.rwg.tri[2 * i] == T ? 1.0 : -1.0;
        const double* pi = &P.V[3 * P.F[3 * T + (c + 2) % 3]];
        double val = 0;
        for (int q = 0; q < 3; ++q) {
          double fi[3], nf[3], bc[3] = {0, 0, 0};
          sub(qp[q], pi, fi);
          for (int x = 0; x < 3; ++x) fi[x] *= sg * P.rwg.len[i] / (2 * AT);
          cross(nT, fi, nf);
          for (int loc = 0; loc < 3; ++loc) {
            double rw[3];
            sub(qp[q], wv[loc], rw);
            for (int x = 0; x < 3; ++x) bc[x] += o.second[loc] * rw[x] / (2 * At);
          }
          val += dot(nf, bc);
        }
        cg.push_back({i, {(int32_t)j, val * At / 3.0}});
      }
    }
  }
  std::vector<std::pair<int64_t, std::pair<int32_t, double>>> cbt;
  cbt.reserve(cb.size());
  for (const auto& x : cb) cbt.push_back({x.second.first, {(int32_t)x.first, x.second.second}});
  to_csr(N, cb, B);
  to_csr(Nr, cbt, Bt);
  to_csr(N, cg, G);
}

}  // namespace cm
