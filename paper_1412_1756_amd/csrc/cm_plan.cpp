// Host-side MLFMA plan (section III): RWG table (eq. (4)), octree with
// Morton-sorted occupied boxes, near lists B_m and far (translation) lists,
// Gauss-Legendre x uniform angular sampling, truncation rule (eq. (30)),
// translators of eqs. (10), (16), (20) in the library's exp(-ikR) convention,
// local Lagrange interpolation / anterpolation tables and centre-shift phases.
#include "cm_plan.h"

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <numeric>
#include <sstream>
#include <thread>
#include <unordered_map>

namespace cm {

static const double kPi = 3.14159265358979323846;

// ---------------------------------------------------------------- special functions
void gauss_legendre(int n, std::vector<double>& x, std::vector<double>& w) {
  x.assign(n, 0.0);
  w.assign(n, 0.0);
  for (int i = 0; i < n; ++i) {
    double z = std::cos(kPi * (i + 0.75) / (n + 0.5));
    double dp = 1.0;
    for (int it = 0; it < 100; ++it) {
      double p0 = 1.0, p1 = z;
      for (int l = 2; l <= n; ++l) {
        double p2 = ((2.0 * l - 1.0) * z * p1 - (l - 1.0) * p0) / l;
        p0 = p1;
        p1 = p2;
      }
      if (n == 0) p1 = 1.0;
      dp = n * (z * p1 - p0) / (z * z - 1.0);
      double dz = p1 / dp;
      z -= dz;
      if (std::fabs(dz) < 1e-16) break;
    }
    double p0 = 1.0, p1 = z;
    for (int l = 2; l <= n; ++l) {
      double p2 = ((2.0 * l - 1.0) * z * p1 - (l - 1.0) * p0) / l;
      p0 = p1;
      p1 = p2;
    }
    dp = n * (z * p1 - p0) / (z * z - 1.0);
    x[i] = z;  // descending in i, so theta = acos(x) ascends
    w[i] = 2.0 / ((1.0 - z * z) * dp * dp);
  }
}

// j_l by Miller's downward recurrence normalised on j_0 or j_1 (whichever is
// larger), y_l by the (stable) upward recurrence.
void sph_jy(int L, double x, std::vector<double>& j, std::vector<double>& y) {
  j.assign(L + 1, 0.0);
  y.assign(L + 1, 0.0);
  const double s = std::sin(x), c = std::cos(x);
  y[0] = -c / x;
  if (L >= 1) y[1] = -c / (x * x) - s / x;
  for (int l = 1; l < L; ++l) y[l + 1] = (2.0 * l + 1.0) / x * y[l] - y[l - 1];
  const double j0 = s / x, j1 = s / (x * x) - c / x;
  int Ns = std::max(L, (int)x) + 40 + (int)std::sqrt(40.0 * std::max(x, 1.0));
  std::vector<double> f(Ns + 2, 0.0);
  f[Ns + 1] = 0.0;
  f[Ns] = 1e-300;
  for (int l = Ns; l >= 1; --l) {
    f[l - 1] = (2.0 * l + 1.0) / x * f[l] - f[l + 1];
    if (std::fabs(f[l - 1]) > 1e250) {
      for (int m = l - 1; m <= Ns + 1; ++m) f[m] *= 1e-250;
    }
  }
  double scale = (std::fabs(j0) >= std::fabs(j1)) ? j0 / f[0] : j1 / f[1];
  for (int l = 0; l <= L; ++l) j[l] = f[l] * scale;
}

// ---------------------------------------------------------------- helpers
static inline uint64_t spread3(uint64_t v) {
  v &= 0x1fffff;
  v = (v | v << 32) & 0x1f00000000ffffULL;
  v = (v | v << 16) & 0x1f0000ff0000ffULL;
  v = (v | v << 8) & 0x100f00f00f00f00fULL;
  v = (v | v << 4) & 0x10c30c30c30c30c3ULL;
  v = (v | v << 2) & 0x1249249249249249ULL;
  return v;
}
static inline uint64_t morton(int x, int y, int z) {
  return spread3((uint64_t)x) | (spread3((uint64_t)y) << 1) | (spread3((uint64_t)z) << 2);
}
static inline int compact3(uint64_t v) {
  v &= 0x1249249249249249ULL;
  v = (v ^ (v >> 2)) & 0x10c30c30c30c30c3ULL;
  v = (v ^ (v >> 4)) & 0x100f00f00f00f00fULL;
  v = (v ^ (v >> 8)) & 0x1f0000ff0000ffULL;
  v = (v ^ (v >> 16)) & 0x1f00000000ffffULL;
  v = (v ^ (v >> 32)) & 0x1fffff;
  return (int)v;
}
static inline int find_code(const std::vector<uint64_t>& codes, uint64_t c) {
  auto it = std::lower_bound(codes.begin(), codes.end(), c);
  if (it == codes.end() || *it != c) return -1;
  return (int)(it - codes.begin());
}
static inline int cheb(const int32_t* a, const int32_t* b) {
  return std::max(std::abs(a[0] - b[0]), std::max(std::abs(a[1] - b[1]), std::abs(a[2] - b[2])));
}
static void lagrange_weights(const double* nodes, int p, double x, double* w) {
  for (int j = 0; j < p; ++j) {
    double v = 1.0;
    for (int m = 0; m < p; ++m)
      if (m != j) v *= (x - nodes[m]) / (nodes[j] - nodes[m]);
    w[j] = v;
  }
}
template <typename F>
static void parallel_for(int64_t n, F fn) {
  unsigned nth = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
  if (n < 64 || nth == 1) {
    for (int64_t i = 0; i < n; ++i) fn(i);
    return;
  }
  std::vector<std::thread> th;
  for (unsigned t = 0; t < nth; ++t)
    th.emplace_back([&, t]() {
      for (int64_t i = t; i < n; i += nth) fn(i);
    });
  for (auto& x : th) x.join();
}

// ---------------------------------------------------------------- build

// ---- operand tables of the matrix-core interpolation kernels
namespace {
using RowList = std::vector<std::vector<std::pair<int32_t, double>>>;   // 16 output rows: (input key, weight)

// Union of the inputs of 16 output rows, four per K step (by2: the step count
// rounded up to an even number); A[k][16 g + r] is the weight of input
// key[4k + g] in row r (unused lanes point at a valid input with weight 0).
int gather_steps(const RowList& rows, std::vector<int32_t>& key, std::vector<double>& A, bool by2) {
  std::vector<int32_t> u;
  for (auto& r : rows)
    for (auto& e : r) u.push_back(e.first);
  std::sort(u.begin(), u.end());
  u.erase(std::unique(u.begin(), u.end()), u.end());
  const int nk = by2 ? (int)(u.size() + 7) / 8 * 2 : (int)(u.size() + 3) / 4;
  key.assign((size_t)nk * 4, u.empty() ? 0 : u[0]);
  for (size_t i = 0; i < u.size(); ++i) key[i] = u[i];
  A.assign((size_t)nk * 64, 0.0);
  for (int r = 0; r < (int)rows.size(); ++r)
    for (auto& e : rows[r]) {
      const int i = (int)(std::lower_bound(u.begin(), u.end(), e.first) - u.begin());
      A[(size_t)(i / 4) * 64 + (i % 4) * 16 + r] += e.second;
    }
  return nk;
}

// phi_rows(idx) lists the phi-step inputs of slotted index idx; theta_rows(t)
// the theta-step inputs of theta row t.
// lds_rows: theta rows each wave keeps in LDS (32 S2 + 16 floats per row);
// the half slot count drops to 4 where S2 = 8 would take more than 80 KiB
// for a block of four waves (two blocks per CU), or more than 128
// accumulator registers.  alt: the other width instead (8 <-> 4); the table
// is left not ok where that is 8 and would need more than 128 accumulators.
template <typename PhiRows, typename ThetaRows>
void build_tab(MfTab& T, int nth, int nph, int lds_rows, PhiRows phi_rows, ThetaRows theta_rows, bool alt = false) {
  T.NT = (nth + 15) / 16;
  T.S2 = (T.NT <= 2 && (size_t)lds_rows * (16 * 16 + 16) * 4 * 4 <= 80 * 1024) ? 8 : 4;
  if (alt) {
    T.S2 = 12 - T.S2;
    if (T.S2 == 8 && T.NT > 2) {
      T.ok = false;
      return;
    }
  }
  T.half = nph / 2;
  T.nchunk = (T.half + T.S2 - 1) / T.S2;
  std::vector<std::vector<int32_t>> keys(T.nchunk);
  std::vector<std::vector<double>> As(T.nchunk);
  T.chunk.assign(2 * (size_t)T.nchunk, 0);
  T.nk.assign(T.nchunk, 0);
  int u0 = 0;
  for (int c = 0; c < T.nchunk; ++c) {
    const int h = T.half / T.nchunk + (c < T.half % T.nchunk ? 1 : 0);
    T.chunk[2 * c] = u0;
    T.chunk[2 * c + 1] = h;
    RowList rows(16);
    for (int s = 0; s < 2 * T.S2; ++s) {
      const int i = s % T.S2, hf = s / T.S2;
      if (i < h) rows[s] = phi_rows(u0 + i + hf * T.half);
    }
    T.nk[c] = gather_steps(rows, keys[c], As[c], true);
    T.kmax = std::max(T.kmax, T.nk[c]);
    u0 += h;
  }
  std::vector<std::vector<int32_t>> tkeys(T.NT);
  std::vector<std::vector<double>> tAs(T.NT);
  T.nkt.assign(T.NT, 0);
  for (int t = 0; t < T.NT; ++t) {
    RowList rows(16);
    for (int r = 0; r < 16 && 16 * t + r < nth; ++r) rows[r] = theta_rows(16 * t + r);
    T.nkt[t] = gather_steps(rows, tkeys[t], tAs[t], false);
    T.ktmax = std::max(T.ktmax, T.nkt[t]);
  }
  const int km = std::max(1, T.kmax), ktm = std::max(1, T.ktmax);
  T.kidx.assign((size_t)T.nchunk * km * 4, 0);
  T.kA.assign((size_t)T.nchunk * km * 64, 0.0);
  for (int c = 0; c < T.nchunk; ++c) {
    std::copy(keys[c].begin(), keys[c].end(), T.kidx.begin() + (size_t)c * km * 4);
    std::copy(As[c].begin(), As[c].end(), T.kA.begin() + (size_t)c * km * 64);
  }
  T.tidx.assign((size_t)T.NT * ktm * 4, 0);
  T.tA.assign((size_t)T.NT * ktm * 64, 0.0);
  for (int t = 0; t < T.NT; ++t) {
    std::copy(tkeys[t].begin(), tkeys[t].end(), T.tidx.begin() + (size_t)t * ktm * 4);
    std::copy(tAs[t].begin(), tAs[t].end(), T.tA.begin() + (size_t)t * ktm * 64);
  }
  T.kmax = km;
  T.ktmax = ktm;
  T.ok = T.kmax <= 16;   // more than four theta tiles are split over blocks
}
}  // namespace

static void build_mf_tables(Plan& P, bool alt) {
  std::vector<MfTab>& ip = alt ? P.mf_ip_alt : P.mf_ip;
  std::vector<MfTab>& at = alt ? P.mf_at_alt : P.mf_at;
  ip.assign(P.lf + 1, MfTab());
  at.assign(P.lf + 1, MfTab());
  for (int l = 2; l < P.lf; ++l) {
    const Interp& I = P.ip[l];
    const int p = I.p;
    // interpolation child l+1 -> l: phi first (child phi -> parent phi), then
    // theta over child rows, reflected entries read the partner phi column
    build_tab(
        ip[l], I.ntp, I.npp, I.ntc,
        [&](int up) {
          std::vector<std::pair<int32_t, double>> e;
          for (int j = 0; j < p; ++j) e.push_back({I.ph_idx[up * p + j], I.ph_w[up * p + j]});
          return e;
        },
        [&](int tp) {
          std::vector<std::pair<int32_t, double>> e;
          for (int j = 0; j < p; ++j) {
            const int ref = I.th_ref[tp * p + j];
            e.push_back({I.th_idx[tp * p + j] | (ref << 16), ref ? -I.th_w[tp * p + j] : I.th_w[tp * p + j]});
          }
          return e;
        },
        alt);
    // anterpolation l -> l+1: weighted transposes, phi first (parent phi ->
    // child phi), then theta over parent rows with reflection in child phi
    build_tab(
        at[l], I.ntc, I.npc, I.ntp,
        [&](int uc) {
          std::vector<std::pair<int32_t, double>> e;
          for (int q = I.pht_ptr[uc]; q < I.pht_ptr[uc + 1]; ++q) e.push_back({I.pht_idx[q], I.pht_w[q]});
          return e;
        },
        [&](int tc) {
          std::vector<std::pair<int32_t, double>> e;
          for (int q = I.tht_ptr[tc]; q < I.tht_ptr[tc + 1]; ++q) {
            const int ref = I.tht_ref[q];
            e.push_back({I.tht_idx[q] | (ref << 16), ref ? -I.tht_w[q] : I.tht_w[q]});
          }
          return e;
        },
        alt);
  }
}

void Plan::build(const double* xyz, int64_t n_vert, const int32_t* tri, int64_t n_tri, double kk,
                 const Opts& o) {
  opt = o;
  k = kk;
  if (!(k > 0) || !std::isfinite(k)) throw Error(-1, "wavenumber must be positive and finite");
  if (o.nlv < 3 || o.nlv > 20) throw Error(-1, "nlv must be in [3, 20]");
  if (o.p < 2 || o.p > 12 || (o.p & 1)) throw Error(-1, "interp_p must be even in [2, 12]");
  if (!(o.d0 > 0) || o.d0 > 20) throw Error(-1, "d0 must be in (0, 20]");
  if (!(o.k_sampling <= 0 || (std::isfinite(o.k_sampling) && o.k_sampling < 1e6)))
    throw Error(-1, "k_sampling must be finite");
  if (o.max_cols < 1 || o.max_cols > 64) throw Error(-1, "max_cols must be in [1, 64]");
  nv = n_vert;
  nt = n_tri;
  if (nv < 3 || nt < 2) throw Error(-1, "mesh too small");
  V.assign(xyz, xyz + 3 * nv);
  F.assign(tri, tri + 3 * nt);
  for (double v : V)
    if (!std::isfinite(v)) throw Error(-2, "non-finite vertex coordinate");
  for (int32_t v : F)
    if (v < 0 || v >= nv) throw Error(-1, "triangle vertex index out of range");
  area.resize(nt);
  hmax.resize(nt);
  cent.resize(3 * nt);
  normal.resize(3 * nt);
  for (int64_t t = 0; t < nt; ++t) {
    const double* a = &V[3 * F[3 * t]];
    const double* b = &V[3 * F[3 * t + 1]];
    const double* c = &V[3 * F[3 * t + 2]];
    double e1[3], e2[3], cr[3];
    for (int d = 0; d < 3; ++d) {
      e1[d] = b[d] - a[d];
      e2[d] = c[d] - a[d];
    }
    cr[0] = e1[1] * e2[2] - e1[2] * e2[1];
    cr[1] = e1[2] * e2[0] - e1[0] * e2[2];
    cr[2] = e1[0] * e2[1] - e1[1] * e2[0];
    double n2 = std::sqrt(cr[0] * cr[0] + cr[1] * cr[1] + cr[2] * cr[2]);
    double h2 = 0.0;
    for (int e = 0; e < 3; ++e) {
      const double* p = &V[3 * F[3 * t + e]];
      const double* q = &V[3 * F[3 * t + (e + 1) % 3]];
      double s = 0;
      for (int d = 0; d < 3; ++d) s += (q[d] - p[d]) * (q[d] - p[d]);
      h2 = std::max(h2, s);
    }
    if (!(n2 > 1e-14 * h2)) throw Error(-2, "degenerate (zero-area) triangle");
    area[t] = 0.5 * n2;
    hmax[t] = std::sqrt(h2);
    for (int d = 0; d < 3; ++d) {
      normal[3 * t + d] = cr[d] / n2;
      cent[3 * t + d] = (a[d] + b[d] + c[d]) / 3.0;
    }
  }

  // ---- RWG: interior edges sorted by (lo, hi); the lower triangle is T+
  {
    struct E { int32_t lo, hi, t, a; };
    std::vector<E> es(3 * nt);
    for (int64_t t = 0; t < nt; ++t)
      for (int a = 0; a < 3; ++a) {
        int32_t u = F[3 * t + (a + 1) % 3], v = F[3 * t + (a + 2) % 3];
        es[3 * t + a] = {std::min(u, v), std::max(u, v), (int32_t)t, a};
      }
    std::sort(es.begin(), es.end(), [](const E& x, const E& y) {
      if (x.lo != y.lo) return x.lo < y.lo;
      if (x.hi != y.hi) return x.hi < y.hi;
      return x.t < y.t;
    });
    size_t i = 0;
    while (i < es.size()) {
      size_t j = i;
      while (j < es.size() && es[j].lo == es[i].lo && es[j].hi == es[i].hi) ++j;
      if (j - i > 2) throw Error(-2, "non-manifold edge shared by more than two triangles");
      if (j - i == 2) {
        rwg.edge.push_back(es[i].lo);
        rwg.edge.push_back(es[i].hi);
        rwg.tri.push_back(es[i].t);
        rwg.tri.push_back(es[i + 1].t);
        rwg.loc.push_back(es[i].a);
        rwg.loc.push_back(es[i + 1].a);
        double s = 0;
        for (int d = 0; d < 3; ++d) {
          double q = V[3 * es[i].hi + d] - V[3 * es[i].lo + d];
          s += q * q;
        }
        rwg.len.push_back(std::sqrt(s));
      }
      i = j;
    }
    rwg.N = (int64_t)rwg.len.size();
    if (rwg.N < 1) throw Error(-2, "mesh has no interior edge");
  }
  const int64_t N = rwg.N;

  // ---- octree: root = bounding cube (x (1 + 1e-9)) about the bounding-box centre
  nlv = o.nlv;
  lf = nlv - 1;
  {
    double lo[3] = {1e300, 1e300, 1e300}, hi[3] = {-1e300, -1e300, -1e300};
    for (int64_t v = 0; v < nv; ++v)
      for (int d = 0; d < 3; ++d) {
        lo[d] = std::min(lo[d], V[3 * v + d]);
        hi[d] = std::max(hi[d], V[3 * v + d]);
      }
    side = 0;
    for (int d = 0; d < 3; ++d) side = std::max(side, hi[d] - lo[d]);
    side *= (1.0 + 1e-9);
    for (int d = 0; d < 3; ++d) origin[d] = 0.5 * (lo[d] + hi[d]) - 0.5 * side;
  }
  lev.assign(lf + 1, Level());
  for (int l = 0; l <= lf; ++l) {
    lev[l].l = l;
    lev[l].a = side / std::ldexp(1.0, l);
  }
  const double aleaf = lev[lf].a;
  const int nside = 1 << lf;
  std::vector<uint64_t> ucode(N);
  for (int64_t n = 0; n < N; ++n) {
    int c[3];
    for (int d = 0; d < 3; ++d) {
      double m = 0.5 * (V[3 * rwg.edge[2 * n] + d] + V[3 * rwg.edge[2 * n + 1] + d]);
      int ix = (int)std::floor((m - origin[d]) / aleaf);
      c[d] = std::min(std::max(ix, 0), nside - 1);
    }
    ucode[n] = morton(c[0], c[1], c[2]);
  }
  perm.resize(N);
  std::iota(perm.begin(), perm.end(), 0);
  std::stable_sort(perm.begin(), perm.end(), [&](int32_t x, int32_t y) { return ucode[x] < ucode[y]; });
  iperm.resize(N);
  for (int64_t i = 0; i < N; ++i) iperm[perm[i]] = (int32_t)i;
  {
    Level& L5 = lev[lf];
    box_of.resize(N);
    for (int64_t i = 0; i < N; ++i) {
      uint64_t c = ucode[perm[i]];
      if (L5.code.empty() || L5.code.back() != c) {
        L5.code.push_back(c);
        box_start.push_back((int32_t)i);
      }
      box_of[i] = (int32_t)L5.code.size() - 1;
    }
    box_start.push_back((int32_t)N);
    L5.nbox = (int)L5.code.size();
  }
  for (int l = lf - 1; l >= 0; --l) {
    for (uint64_t c : lev[l + 1].code) {
      uint64_t pc = c >> 3;
      if (lev[l].code.empty() || lev[l].code.back() != pc) lev[l].code.push_back(pc);
    }
    lev[l].nbox = (int)lev[l].code.size();
  }
  for (int l = 0; l <= lf; ++l) {
    Level& Lv = lev[l];
    Lv.ijk.resize(3 * Lv.nbox);
    for (int b = 0; b < Lv.nbox; ++b) {
      Lv.ijk[3 * b] = compact3(Lv.code[b]);
      Lv.ijk[3 * b + 1] = compact3(Lv.code[b] >> 1);
      Lv.ijk[3 * b + 2] = compact3(Lv.code[b] >> 2);
    }
    Lv.parent.assign(Lv.nbox, -1);
    if (l > 0)
      for (int b = 0; b < Lv.nbox; ++b) Lv.parent[b] = find_code(lev[l - 1].code, Lv.code[b] >> 3);
    Lv.child_ptr.assign(Lv.nbox + 1, 0);
    if (l < lf) {
      const auto& cc = lev[l + 1].code;
      for (int b = 0; b < Lv.nbox; ++b)
        Lv.child_ptr[b] = (int)(std::lower_bound(cc.begin(), cc.end(), Lv.code[b] << 3) - cc.begin());
      Lv.child_ptr[Lv.nbox] = lev[l + 1].nbox;
    }
  }
  // Near radius (Chebyshev distance, in boxes) per level: 1, or 2 at the two
  // finest levels with the wide-near option (flag 32).
  const bool wide = (o.flags & 32u) != 0;
  auto near_radius = [&](int l) { return (wide && l >= lf - 1) ? 2 : 1; };
  auto box_lookup = [&](int l, int x, int y, int z) -> int {
    int ns = 1 << l;
    if (x < 0 || y < 0 || z < 0 || x >= ns || y >= ns || z >= ns) return -1;
    return find_code(lev[l].code, morton(x, y, z));
  };

  // ---- near lists and near-field CSR (leaf)
  {
    const Level& Lf = lev[lf];
    near_ptr.assign(Lf.nbox + 1, 0);
    const int nr = near_radius(lf);
    for (int b = 0; b < Lf.nbox; ++b) {
      std::vector<int> nb;
      for (int dx = -nr; dx <= nr; ++dx)
        for (int dy = -nr; dy <= nr; ++dy)
          for (int dz = -nr; dz <= nr; ++dz) {
            int q = box_lookup(lf, Lf.ijk[3 * b] + dx, Lf.ijk[3 * b + 1] + dy, Lf.ijk[3 * b + 2] + dz);
            if (q >= 0) nb.push_back(q);
          }
      std::sort(nb.begin(), nb.end());
      near_box.insert(near_box.end(), nb.begin(), nb.end());
      near_ptr[b + 1] = (int32_t)near_box.size();
    }
    bcol_ptr.assign(Lf.nbox + 1, 0);
    self_off.assign(Lf.nbox, 0);
    for (int b = 0; b < Lf.nbox; ++b) {
      for (int e = near_ptr[b]; e < near_ptr[b + 1]; ++e) {
        int q = near_box[e];
        if (q == b) self_off[b] = (int32_t)(bcol.size() - bcol_ptr[b]);
        for (int j = box_start[q]; j < box_start[q + 1]; ++j) bcol.push_back(j);
      }
      bcol_ptr[b + 1] = (int32_t)bcol.size();
    }
    row_ptr.assign(N + 1, 0);
    for (int64_t i = 0; i < N; ++i) {
      int b = box_of[i];
      row_ptr[i + 1] = row_ptr[i] + (bcol_ptr[b + 1] - bcol_ptr[b]);
    }
    nnz = row_ptr[N];
  }

  // ---- every near-singular triangle pair must lie inside the near field
  {
    double hg = 0;
    for (double h : hmax) hg = std::max(hg, h);
    const double thr = 1.5 * hg;
    const double cell = std::max(thr, 1e-300);
    std::unordered_map<uint64_t, std::vector<int32_t>> grid;
    auto cell_of = [&](int64_t t, int* c) {
      for (int d = 0; d < 3; ++d) c[d] = (int)std::floor((cent[3 * t + d] - origin[d]) / cell) + 1;
    };
    for (int64_t t = 0; t < nt; ++t) {
      int c[3];
      cell_of(t, c);
      grid[morton(c[0], c[1], c[2])].push_back((int32_t)t);
    }
    // RWGs carried by each triangle (internal index -> leaf box)
    std::vector<int32_t> tri_box(3 * nt, -1);
    for (int64_t n = 0; n < N; ++n)
      for (int s = 0; s < 2; ++s) tri_box[3 * rwg.tri[2 * n + s] + rwg.loc[2 * n + s]] = box_of[iperm[n]];
    const Level& Lf = lev[lf];
    for (int64_t t = 0; t < nt; ++t) {
      int c[3];
      cell_of(t, c);
      for (int dx = -1; dx <= 1; ++dx)
        for (int dy = -1; dy <= 1; ++dy)
          for (int dz = -1; dz <= 1; ++dz) {
            auto it = grid.find(morton(c[0] + dx, c[1] + dy, c[2] + dz));
            if (it == grid.end()) continue;
            for (int32_t u : it->second) {
              double d2 = 0;
              for (int d = 0; d < 3; ++d) {
                double q = cent[3 * t + d] - cent[3 * u + d];
                d2 += q * q;
              }
              double h = 1.5 * std::max(hmax[t], hmax[u]);
              if (d2 >= h * h) continue;
              for (int a = 0; a < 3; ++a)
                for (int b = 0; b < 3; ++b) {
                  int ba = tri_box[3 * t + a], bb = tri_box[3 * u + b];
                  if (ba < 0 || bb < 0) continue;
                  if (cheb(&Lf.ijk[3 * ba], &Lf.ijk[3 * bb]) > 1)
                    throw Error(-2, "mesh too coarse for the leaf boxes: a near-singular triangle pair "
                                    "falls outside the near field (use fewer levels)");
                }
            }
          }
    }
  }

  // ---- far (translation) lists, levels 2..lf
  // R (sin kernel, eq. (22)): its addition theorem holds at any separation, so
  // a box needs no near field beyond itself.  Default bookkeeping (the one
  // the paper recommends for R): at levels 3..lf a box translates from the
  // other children of its parent only, and at the coarsest level (2 here,
  // where the paper goes on to level 1) from every other box; each pair of
  // distinct leaf boxes is then covered at the coarsest level where their
  // ancestors differ.  Flag 128 selects the standard MLFMA lists instead
  // (Z's far lists, plus the neighbouring boxes at the leaf level).
  const bool r_std = (o.flags & 128u) != 0;
  for (int l = 2; l <= lf; ++l) {
    Level& Lv = lev[l];
    const Level& Pl = lev[l - 1];
    Lv.far_ptr.assign(Lv.nbox + 1, 0);
    Lv.farR_ptr.assign(Lv.nbox + 1, 0);
    for (int m = 0; m < Lv.nbox; ++m) {
      std::vector<std::pair<int, int>> lst, lstR;
      int P = Lv.parent[m];
      if (!r_std) {
        const int c0 = (l == 2) ? 0 : Pl.child_ptr[P], c1 = (l == 2) ? Lv.nbox : Pl.child_ptr[P + 1];
        for (int c = c0; c < c1; ++c)
          if (c != m)
            lstR.push_back({c, off_id(Lv.ijk[3 * m] - Lv.ijk[3 * c], Lv.ijk[3 * m + 1] - Lv.ijk[3 * c + 1],
                                      Lv.ijk[3 * m + 2] - Lv.ijk[3 * c + 2])});
      }
      // parents within the near radius of the level above; children beyond
      // this level's near radius are translated here
      const int pr = near_radius(l - 1), dfar = near_radius(l) + 1;
      for (int dx = -pr; dx <= pr; ++dx)
        for (int dy = -pr; dy <= pr; ++dy)
          for (int dz = -pr; dz <= pr; ++dz) {
            int Q = box_lookup(l - 1, Pl.ijk[3 * P] + dx, Pl.ijk[3 * P + 1] + dy, Pl.ijk[3 * P + 2] + dz);
            if (Q < 0) continue;
            for (int c = Pl.child_ptr[Q]; c < Pl.child_ptr[Q + 1]; ++c) {
              int dd = cheb(&Lv.ijk[3 * m], &Lv.ijk[3 * c]);
              int off = off_id(Lv.ijk[3 * m] - Lv.ijk[3 * c], Lv.ijk[3 * m + 1] - Lv.ijk[3 * c + 1],
                               Lv.ijk[3 * m + 2] - Lv.ijk[3 * c + 2]);
              if (dd >= dfar) {
                lst.push_back({c, off});
                if (r_std) lstR.push_back({c, off});
              } else if (r_std && l == lf && dd >= 1) {
                lstR.push_back({c, off});   // R translates neighbouring leaf boxes too
              }
            }
          }
      std::sort(lst.begin(), lst.end());
      std::sort(lstR.begin(), lstR.end());
      for (auto& e : lst) {
        Lv.far_src.push_back(e.first);
        Lv.far_off.push_back(e.second);
      }
      for (auto& e : lstR) {
        Lv.farR_src.push_back(e.first);
        Lv.farR_off.push_back(e.second);
      }
      Lv.far_ptr[m + 1] = (int32_t)Lv.far_src.size();
      Lv.farR_ptr[m + 1] = (int32_t)Lv.farR_src.size();
    }
  }

  // ---- sampling (levels 2..lf): L from eq. (30), nt = L+1 GL nodes, np = 2(L+1)
  dirs.assign(lf + 1, {});
  qw.assign(lf + 1, {});
  for (int l = 2; l <= lf; ++l) {
    Level& Lv = lev[l];
    const double kd = (o.k_sampling > 0 ? o.k_sampling : k) * std::sqrt(3.0) * Lv.a;
    Lv.L = (int)std::ceil(kd + 1.8 * std::pow(o.d0, 2.0 / 3.0) * std::cbrt(kd));
    // translator truncation: eq. (30) at the sampling wavenumber, or for a
    // sweep sharing its sampling (CM_FLAG_SWEEP_SHARED) at this plan's own
    // k (the grid of the largest k integrates the smaller degree exactly,
    // and a translator truncated beyond its own rule loses accuracy through
    // the growth of the high-order Hankel terms)
    Lv.Lt = Lv.L;
    if ((o.flags & 2048u) && o.k_sampling > 0 && k < o.k_sampling) {
      const double kdo = k * std::sqrt(3.0) * Lv.a;
      Lv.Lt = std::min(Lv.L, (int)std::ceil(kdo + 1.8 * std::pow(o.d0, 2.0 / 3.0) * std::cbrt(kdo)));
    }
    Lv.nt = Lv.L + 1;
    Lv.np = 2 * (Lv.L + 1);
    Lv.K = Lv.nt * Lv.np;
    std::vector<double> x, w;
    gauss_legendre(Lv.nt, x, w);
    Lv.theta.resize(Lv.nt);
    Lv.wtheta = w;
    for (int t = 0; t < Lv.nt; ++t) Lv.theta[t] = std::acos(x[t]);
    dirs[l].resize(9 * (size_t)Lv.K);
    qw[l].resize(Lv.K);
    for (int t = 0; t < Lv.nt; ++t)
      for (int p = 0; p < Lv.np; ++p) {
        int q = t * Lv.np + p;
        double th = Lv.theta[t], ph = 2.0 * kPi * p / Lv.np;
        double st = std::sin(th), ct = x[t], sp = std::sin(ph), cp = std::cos(ph);
        double* D = &dirs[l][9 * (size_t)q];
        D[0] = st * cp; D[1] = st * sp; D[2] = ct;
        D[3] = ct * cp; D[4] = ct * sp; D[5] = -st;
        D[6] = -sp;     D[7] = cp;      D[8] = 0.0;
        qw[l][q] = w[t] * 2.0 * kPi / Lv.np;
      }
  }

  // ---- translators (levels 2..lf), exp(-ikR) convention:
  //   TZ = sum (-i)^l (2l+1) h2_l(k r) P_l,  TR = sum (-i)^l (2l+1) j_l P_l,
  //   TX = -sum (-i)^l (2l+1) y_l P_l,       dTZ = d TZ / dk
  TZ.assign(lf + 1, {});
  TR.assign(lf + 1, {});
  TX.assign(lf + 1, {});
  dTZ.assign(lf + 1, {});
  off_used.assign(lf + 1, std::vector<uint8_t>(kNoff, 0));
  const bool want_d = (o.flags & 2u) != 0;
  for (int l = 2; l <= lf; ++l) {
    Level& Lv = lev[l];
    for (int32_t f : Lv.farR_off) off_used[l][f] = 1;
    for (int32_t f : Lv.far_off) off_used[l][f] = 1;
    const int K = Lv.K, Lt = Lv.Lt;
    std::vector<int> offs;
    Lv.off_compact.assign(kNoff, -1);
    for (int f = 0; f < kNoff; ++f)
      if (off_used[l][f]) {
        Lv.off_compact[f] = (int32_t)offs.size();
        offs.push_back(f);
      }
    Lv.n_off_used = (int)offs.size();
    const size_t nu = std::max<size_t>(1, offs.size());
    TZ[l].assign(nu * K, cplx(0));
    TR[l].assign(nu * K, cplx(0));
    TX[l].assign(nu * K, cplx(0));
    if (want_d) dTZ[l].assign(nu * K, cplx(0));
    parallel_for((int64_t)offs.size(), [&](int64_t oi) {
      int f = offs[oi];
      int dx = f / (kOffW * kOffW) - kOffH, dy = (f / kOffW) % kOffW - kOffH, dz = f % kOffW - kOffH;
      double X[3] = {dx * Lv.a, dy * Lv.a, dz * Lv.a};
      double r = std::sqrt(X[0] * X[0] + X[1] * X[1] + X[2] * X[2]);
      std::vector<double> jl, yl;
      sph_jy(Lt + 1, k * r, jl, yl);
      std::vector<cplx> cz(Lt + 1), cr(Lt + 1), cx(Lt + 1), cd(Lt + 1);
      cplx ip(1, 0);
      const cplx mi(0, -1);
      for (int n = 0; n <= Lt; ++n) {
        double c2 = 2.0 * n + 1.0;
        cz[n] = ip * c2 * cplx(jl[n], -yl[n]);
        cr[n] = ip * c2 * jl[n];
        cx[n] = -ip * c2 * yl[n];
        // d/dx z_n = z_{n-1} - (n+1)/x z_n  (z_0' = -z_1), z = h2 = j - i y
        double x = k * r;
        cplx z = cplx(jl[n], -yl[n]);
        cplx zm = (n == 0) ? -cplx(jl[1], -yl[1]) : cplx(jl[n - 1], -yl[n - 1]);
        cplx dz = (n == 0) ? zm : zm - (n + 1.0) / x * z;
        cd[n] = ip * c2 * r * dz;
        ip *= mi;
      }
      for (int q = 0; q < K; ++q) {
        const double* D = &dirs[l][9 * (size_t)q];
        double c = (D[0] * X[0] + D[1] * X[1] + D[2] * X[2]) / r;
        double p0 = 1.0, p1 = c;
        cplx sz = cz[0], sr = cr[0], sx = cx[0], sd = cd[0];
        for (int n = 1; n <= Lt; ++n) {
          double P = (n == 1) ? p1 : 0.0;
          if (n >= 2) {
            P = ((2.0 * n - 1.0) * c * p1 - (n - 1.0) * p0) / n;
            p0 = p1;
            p1 = P;
          }
          sz += cz[n] * P;
          sr += cr[n] * P;
          sx += cx[n] * P;
          sd += cd[n] * P;
        }
        size_t idx = (size_t)oi * K + q;
        TZ[l][idx] = sz;
        TR[l][idx] = sr;
        TX[l][idx] = sx;
        if (want_d) dTZ[l][idx] = sd;
      }
    });
    for (size_t i = 0; i < TZ[l].size(); ++i)
      if (!std::isfinite(TZ[l][i].real()) || !std::isfinite(TZ[l][i].imag()))
        throw Error(-6, "non-finite translator entry");
  }

  // ---- receiver tiles for the translation kernel
  for (int l = 2; l <= lf; ++l) {
    Level& Lv = lev[l];
    auto make = [&](const std::vector<int32_t>& ptr, const std::vector<int32_t>& src,
                    const std::vector<int32_t>& off, std::vector<int32_t>& tptr, std::vector<int32_t>& tsrc,
                    std::vector<int32_t>& toff, int TS) {
      const int ntile = (Lv.nbox + TS - 1) / TS;
      tptr.assign(ntile + 1, 0);
      for (int t = 0; t < ntile; ++t) {
        std::vector<std::pair<int, std::pair<int, int>>> ent;   // (source, (receiver slot, compact off))
        for (int r = 0; r < TS; ++r) {
          int m = t * TS + r;
          if (m >= Lv.nbox) break;
          for (int e = ptr[m]; e < ptr[m + 1]; ++e) ent.push_back({src[e], {r, Lv.off_compact[off[e]]}});
        }
        std::sort(ent.begin(), ent.end());
        size_t i = 0;
        while (i < ent.size()) {
          int sbox = ent[i].first;
          tsrc.push_back(sbox);
          size_t base = toff.size();
          toff.resize(base + TS, -1);
          while (i < ent.size() && ent[i].first == sbox) {
            toff[base + ent[i].second.first] = ent[i].second.second;
            ++i;
          }
        }
        tptr[t + 1] = (int32_t)tsrc.size();
      }
    };
    make(Lv.far_ptr, Lv.far_src, Lv.far_off, Lv.tile_ptr, Lv.tile_src, Lv.tile_off, kTile);
    make(Lv.farR_ptr, Lv.farR_src, Lv.farR_off, Lv.tileR_ptr, Lv.tileR_src, Lv.tileR_off, kTile);
    make(Lv.far_ptr, Lv.far_src, Lv.far_off, Lv.tile64_ptr, Lv.tile64_src, Lv.tile64_off, kTile64);
    make(Lv.farR_ptr, Lv.farR_src, Lv.farR_off, Lv.tileR64_ptr, Lv.tileR64_src, Lv.tileR64_off, kTile64);
  }

  // ---- interpolation (child l+1 -> parent l, l = 2..lf-1) and shift phases
  ip.assign(lf + 1, Interp());
  shift.assign(lf + 1, {});
  dshift.assign(lf + 1, {});
  const int p = o.p;
  for (int l = 2; l < lf; ++l) {
    const Level& C = lev[l + 1];
    const Level& P = lev[l];
    if (p > C.nt || p > C.np) throw Error(-1, "interp_p exceeds the child sampling");
    Interp& I = ip[l];
    I.p = p;
    I.ntc = C.nt; I.npc = C.np; I.ntp = P.nt; I.npp = P.np;
    // theta: extended child nodes with reflections over both poles
    std::vector<double> ext(3 * C.nt);
    std::vector<int> eidx(3 * C.nt), eref(3 * C.nt);
    for (int e = 0; e < C.nt; ++e) {
      ext[e] = -C.theta[C.nt - 1 - e];
      eidx[e] = C.nt - 1 - e;
      eref[e] = 1;
      ext[C.nt + e] = C.theta[e];
      eidx[C.nt + e] = e;
      eref[C.nt + e] = 0;
      ext[2 * C.nt + e] = 2.0 * kPi - C.theta[C.nt - 1 - e];
      eidx[2 * C.nt + e] = C.nt - 1 - e;
      eref[2 * C.nt + e] = 1;
    }
    I.th_idx.resize(P.nt * p);
    I.th_ref.resize(P.nt * p);
    I.th_w.resize(P.nt * p);
    for (int t = 0; t < P.nt; ++t) {
      double th = P.theta[t];
      int e0 = (int)(std::upper_bound(ext.begin(), ext.end(), th) - ext.begin()) - 1;
      int s = std::min(std::max(e0 - p / 2 + 1, 0), 3 * C.nt - p);
      lagrange_weights(&ext[s], p, th, &I.th_w[t * p]);
      for (int j = 0; j < p; ++j) {
        I.th_idx[t * p + j] = eidx[s + j];
        I.th_ref[t * p + j] = eref[s + j];
      }
    }
    // phi: periodic uniform
    const double dc = 2.0 * kPi / C.np;
    I.ph_idx.resize(P.np * p);
    I.ph_w.resize(P.np * p);
    for (int u = 0; u < P.np; ++u) {
      double ph = 2.0 * kPi * u / P.np;
      int j0 = (int)std::floor(ph / dc + 1e-9);
      int s = j0 - p / 2 + 1;
      std::vector<double> nodes(p);
      for (int j = 0; j < p; ++j) nodes[j] = (s + j) * dc;
      lagrange_weights(nodes.data(), p, ph, &I.ph_w[u * p]);
      for (int j = 0; j < p; ++j) I.ph_idx[u * p + j] = ((s + j) % C.np + C.np) % C.np;
    }
    // weighted transposes A = Wc^-1 I^T Wp in gather form
    {
      std::vector<std::vector<std::tuple<int, int, double>>> th(C.nt);
      for (int t = 0; t < P.nt; ++t)
        for (int j = 0; j < p; ++j) {
          int tc = I.th_idx[t * p + j];
          th[tc].push_back({t, I.th_ref[t * p + j], I.th_w[t * p + j] * P.wtheta[t] / C.wtheta[tc]});
        }
      I.tht_ptr.assign(C.nt + 1, 0);
      for (int tc = 0; tc < C.nt; ++tc) {
        for (auto& e : th[tc]) {
          I.tht_idx.push_back(std::get<0>(e));
          I.tht_ref.push_back(std::get<1>(e));
          I.tht_w.push_back(std::get<2>(e));
        }
        I.tht_ptr[tc + 1] = (int32_t)I.tht_idx.size();
      }
      std::vector<std::vector<std::pair<int, double>>> ph(C.np);
      for (int u = 0; u < P.np; ++u)
        for (int j = 0; j < p; ++j)
          ph[I.ph_idx[u * p + j]].push_back({u, I.ph_w[u * p + j] * (double)C.np / (double)P.np});
      I.pht_ptr.assign(C.np + 1, 0);
      for (int uc = 0; uc < C.np; ++uc) {
        for (auto& e : ph[uc]) {
          I.pht_idx.push_back(e.first);
          I.pht_w.push_back(e.second);
        }
        I.pht_ptr[uc + 1] = (int32_t)I.pht_idx.size();
      }
    }
    // shift phases exp(ik khat . (r_child - r_parent)) for the 8 octants
    shift[l].resize(8 * (size_t)P.K);
    dshift[l].resize(8 * (size_t)P.K);
    for (int oc = 0; oc < 8; ++oc) {
      double dv[3] = {((oc & 1) ? 0.5 : -0.5) * C.a, ((oc & 2) ? 0.5 : -0.5) * C.a,
                      ((oc & 4) ? 0.5 : -0.5) * C.a};
      for (int q = 0; q < P.K; ++q) {
        const double* D = &dirs[l][9 * (size_t)q];
        double kd = D[0] * dv[0] + D[1] * dv[1] + D[2] * dv[2];
        double ph = k * kd;
        shift[l][(size_t)oc * P.K + q] = cplx(std::cos(ph), std::sin(ph));
        dshift[l][(size_t)oc * P.K + q] = cplx(0.0, kd) * cplx(std::cos(ph), std::sin(ph));
      }
    }
  }
  build_mf_tables(*this, false);
  if (o.flags & 64u) build_mf_tables(*this, true);   // candidates for the autotuner
  if (o.flags & 4u) check_coverage();
}

// Every pair of leaf boxes must be covered exactly once: by the near list at
// the leaf, or by the far list of exactly one level (for the ancestors).
void Plan::check_coverage() const {
  const Level& Lf = lev[lf];
  const int nb = Lf.nbox;
  std::vector<std::vector<int>> anc(lf + 1, std::vector<int>(nb));
  for (int b = 0; b < nb; ++b) {
    int x = b;
    for (int l = lf; l >= 0; --l) {
      anc[l][b] = x;
      if (l > 0) x = lev[l].parent[x];
    }
  }
  auto in_list = [](const std::vector<int32_t>& ptr, const std::vector<int32_t>& src, int m, int s) {
    for (int e = ptr[m]; e < ptr[m + 1]; ++e)
      if (src[e] == s) return true;
    return false;
  };
  for (int b1 = 0; b1 < nb; ++b1)
    for (int b2 = 0; b2 < nb; ++b2) {
      int cz = 0, cr = 0;
      bool nearb = in_list(near_ptr, near_box, b1, b2);
      cz += nearb;
      cr += (b1 == b2);
      for (int l = 2; l <= lf; ++l) {
        cz += in_list(lev[l].far_ptr, lev[l].far_src, anc[l][b1], anc[l][b2]);
        cr += in_list(lev[l].farR_ptr, lev[l].farR_src, anc[l][b1], anc[l][b2]);
      }
      if (cz != 1 || cr != 1) {
        char msg[160];
        std::snprintf(msg, sizeof msg, "coverage check failed for leaf boxes %d, %d (Z %d, R %d)", b1, b2, cz, cr);
        throw Error(-6, msg);
      }
    }
}

std::string Plan::stats_json() const {
  std::ostringstream s;
  s.precision(17);
  s << "{\"N\": " << rwg.N << ", \"n_tri\": " << nt << ", \"k\": " << k << ", \"nlv\": " << nlv
    << ", \"d0\": " << opt.d0 << ", \"k_sampling\": " << (opt.k_sampling > 0 ? opt.k_sampling : k) << ", \"interp_p\": " << opt.p << ", \"wide_near\": " << ((opt.flags & 32u) ? 1 : 0) << ", \"r_lists\": \"" << ((opt.flags & 128u) ? "standard" : "siblings") << "\"" << ", \"root_side\": " << side
    << ", \"nnz_near\": " << nnz << ", \"near_cols_total\": " << bcol.size()
    << ", \"n_leaf\": " << lev[lf].nbox << ", \"levels\": [";
  for (int l = 0; l <= lf; ++l) {
    const Level& Lv = lev[l];
    if (l) s << ", ";
    s << "{\"l\": " << l << ", \"a\": " << Lv.a << ", \"nbox\": " << Lv.nbox << ", \"L\": " << Lv.L << ", \"L_translator\": " << Lv.Lt
      << ", \"nt\": " << Lv.nt << ", \"np\": " << Lv.np << ", \"K\": " << Lv.K
      << ", \"far_pairs\": " << (Lv.far_src.size()) << ", \"farR_pairs\": " << (Lv.farR_src.size())
      << ", \"tile_sources\": " << Lv.tile_src.size() << ", \"tile64_sources\": " << Lv.tile64_src.size()
      << ", \"n_off_used\": " << Lv.n_off_used;
    // matrix-core interpolation tables (into level l, and anterpolation from it)
    auto mf = [&](const char* key, const std::vector<MfTab>& v) {
      if (l >= (int)v.size() || !v[l].nchunk) return;
      const MfTab& T = v[l];
      s << ", \"" << key << "\": {\"ok\": " << (T.ok ? 1 : 0) << ", \"NT\": " << T.NT << ", \"S2\": " << T.S2
        << ", \"nchunk\": " << T.nchunk << ", \"kmax\": " << T.kmax << ", \"ktmax\": " << T.ktmax << "}";
    };
    mf("mf_interp", mf_ip);
    mf("mf_anterp", mf_at);
    s << "}";
  }
  s << "]}";
  return s.str();
}

}  // namespace cm
