// C ABI (include/cmmlfma.h): handle life cycle, device set-up, argument checks.
#include <hip/hip_runtime.h>

#include <cmath>
#include <algorithm>
#include <cstdio>
#include <cstring>
#include <memory>
#include <new>
#include <string>

#include "cm_device.h"

namespace cm {
void set_quadrature_constants();
void launch_near_fill(double k, double eta, const Dev& d, int nbox, hipStream_t s);
void launch_leaf_patterns(double k, const Dev& d, hipStream_t s);
int blas_vdot_blocks();
void blas_vdot(const void* x, const void* y, int64_t ld, int nc, int64_t N, bool fp64, double2* part, double2* out,
               hipStream_t s);

static void chk(hipError_t e, const char* what) {
  if (e != hipSuccess) {
    if (e == hipErrorOutOfMemory || e == hipErrorMemoryAllocation)
      throw Error(-3, std::string(what) + ": out of device memory");
    throw Error(-4, std::string(what) + ": " + hipGetErrorString(e));
  }
}

static void* dmalloc(Dev& d, size_t bytes) {
  if (bytes == 0) bytes = 16;
  void* p = nullptr;
  chk(hipMalloc(&p, bytes), "hipMalloc");
  d.allocs.push_back(p);
  return p;
}

template <typename T>
static T* upload(Dev& d, const std::vector<T>& v, hipStream_t s) {
  T* p = (T*)dmalloc(d, v.size() * sizeof(T));
  if (!v.empty()) chk(hipMemcpyAsync(p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice, s), "upload");
  return p;
}

template <typename R>
static void* upload_complex(Dev& d, const std::vector<cplx>& v, hipStream_t s) {
  std::vector<R> h(2 * v.size());
  for (size_t i = 0; i < v.size(); ++i) {
    h[2 * i] = (R)v[i].real();
    h[2 * i + 1] = (R)v[i].imag();
  }
  return upload(d, h, s);
}

template <typename R>
static std::vector<R> cast(const std::vector<double>& v) {
  return std::vector<R>(v.begin(), v.end());
}

static MfD upload_mf(Dev& d, const MfTab& T, hipStream_t s) {
  MfD m;
  if (!T.ok) return m;
  m.ok = 1;
  m.NT = T.NT;
  m.S2 = T.S2;
  m.half = T.half;
  m.nchunk = T.nchunk;
  m.kmax = T.kmax;
  m.ktmax = T.ktmax;
  m.chunk = upload(d, T.chunk, s);
  m.nk = upload(d, T.nk, s);
  m.kidx = upload(d, T.kidx, s);
  m.kA = upload(d, cast<float>(T.kA), s);
  m.nkt = upload(d, T.nkt, s);
  m.tidx = upload(d, T.tidx, s);
  m.tA = upload(d, cast<float>(T.tA), s);
  return m;
}

// phase table [8][K] (q = t*np + u) re-laid as [8][np][16 NT] with theta fastest
static std::vector<cplx> shiftT_table(const std::vector<cplx>& sh, int nt, int np, int NT) {
  const int tp = 16 * NT;
  std::vector<cplx> v((size_t)8 * np * tp, cplx(0, 0));
  for (int oc = 0; oc < 8; ++oc)
    for (int t = 0; t < nt; ++t)
      for (int u = 0; u < np; ++u) v[((size_t)oc * np + u) * tp + t] = sh[(size_t)oc * nt * np + (size_t)t * np + u];
  return v;
}
static void* upload_shiftT(Dev& d, const std::vector<cplx>& sh, int nt, int np, int NT, hipStream_t s) {
  return upload_complex<float>(d, shiftT_table(sh, nt, np, NT), s);
}

// phase values of the anterpolation K steps: [chunk][octant][t][4 kmax]
static std::vector<cplx> zg_table(const std::vector<cplx>& sh, const MfTab& T, int nt, int np) {
  const int kz = 4 * T.kmax;
  std::vector<cplx> v((size_t)T.nchunk * 8 * nt * kz, cplx(0, 0));
  for (int c = 0; c < T.nchunk; ++c)
    for (int oc = 0; oc < 8; ++oc)
      for (int t = 0; t < nt; ++t)
        for (int k = 0; k < 4 * T.nk[c]; ++k)
          v[(((size_t)c * 8 + oc) * nt + t) * kz + k] =
              sh[(size_t)oc * nt * np + (size_t)t * np + T.kidx[((size_t)c * T.kmax) * 4 + k]];
  return v;
}
static void* upload_zg(Dev& d, const std::vector<cplx>& sh, const MfTab& T, int nt, int np, hipStream_t s) {
  return upload_complex<float>(d, zg_table(sh, T, nt, np), s);
}

// The one-pass sweep tables of d (the first wavenumber's device data): per
// level Z's FP32 translators of all wavenumbers interleaved [n_off][K][n_k],
// and the interpolation / anterpolation phase tables of every wavenumber one
// after another, laid out for the matrix-core tables d uses (after its
// autotuning).  Every plan must have the same tree, lists and sampling.
void build_sweep_tables(Dev& d, const Plan& P, const std::vector<const Plan*>& Pk, hipStream_t s) {
  const int nk = (int)Pk.size();
  for (const Plan* q : Pk) {
    if (q->lf != P.lf || q->rwg.N != P.rwg.N) throw Error(CM_E_UNSUPPORTED, "sweep plans differ in their tree");
    for (int l = 2; l <= P.lf; ++l)
      if (q->lev[l].K != P.lev[l].K || q->lev[l].nt != P.lev[l].nt || q->lev[l].np != P.lev[l].np ||
          q->lev[l].n_off_used != P.lev[l].n_off_used || q->lev[l].nbox != P.lev[l].nbox)
        throw Error(CM_E_UNSUPPORTED, "sweep plans differ in their sampling or lists");
  }
  for (int l = 2; l <= P.lf; ++l) {
    const Level& Lv = P.lev[l];
    LevelD<float>& D = d.f32.lev[l];
    const size_t nT = P.TZ[l].size();   // n_off_used x K (one row of zeros at a level without translations)
    for (const Plan* q : Pk)
      if (q->TZ[l].size() != nT) throw Error(CM_E_UNSUPPORTED, "sweep plans differ in their translator tables");
    std::vector<float> T(2 * nT * nk);
    for (int kk = 0; kk < nk; ++kk)
      for (size_t e = 0; e < nT; ++e) {
        T[2 * (e * nk + kk)] = (float)Pk[kk]->TZ[l][e].real();
        T[2 * (e * nk + kk) + 1] = (float)Pk[kk]->TZ[l][e].imag();
      }
    D.sw_T = upload(d, T, s);
    if (l == P.lf) continue;
    if (D.mip.ok) {
      std::vector<cplx> all;
      for (int kk = 0; kk < nk; ++kk) {
        const std::vector<cplx> v = shiftT_table(Pk[kk]->shift[l], Lv.nt, Lv.np, D.mip.NT);
        D.sw_shift_stride = (int64_t)v.size();
        all.insert(all.end(), v.begin(), v.end());
      }
      D.sw_shiftT = upload_complex<float>(d, all, s);
    }
    if (D.mat.ok) {
      // the anterpolation table in use: the plan's, or the other width the autotuner swapped in
      // (the other width exists only on an autotuned handle)
      const MfTab* A = nullptr;
      for (const std::vector<MfTab>* v : {&P.mf_at, &P.mf_at_alt})
        if (l < (int)v->size()) {
          const MfTab& c = (*v)[l];
          if (c.ok && c.S2 == D.mat.S2 && c.nchunk == D.mat.nchunk && c.kmax == D.mat.kmax) A = &c;
        }
      if (!A) throw Error(CM_E_UNSUPPORTED, "sweep tables: anterpolation table not found");
      std::vector<cplx> all;
      for (int kk = 0; kk < nk; ++kk) {
        const std::vector<cplx> v = zg_table(Pk[kk]->shift[l], *A, Lv.nt, Lv.np);
        D.sw_zg_stride = (int64_t)v.size();
        all.insert(all.end(), v.begin(), v.end());
      }
      D.sw_zg = upload_complex<float>(d, all, s);
    }
  }
  chk(hipStreamSynchronize(s), "sweep tables");
  d.sw_nk = nk;
}

template <typename R>
static void build_prec(Dev& d, const Plan& P, PrecD<R>& pd, const std::vector<int32_t>& octant_dummy,
                       std::vector<int32_t*>& lists, hipStream_t s) {
  (void)octant_dummy;
  const int lf = P.lf;
  pd.lev.assign(lf + 1, LevelD<R>());
  for (int l = 2; l <= lf; ++l) {
    const Level& Lv = P.lev[l];
    LevelD<R>& D = pd.lev[l];
    D.nbox = Lv.nbox;
    D.K = Lv.K;
    D.nt = Lv.nt;
    D.np = Lv.np;
    // index arrays are shared between the precisions (uploaded once in `lists`)
    D.far_ptr = lists[8 * l + 0];
    D.far_src = lists[8 * l + 1];
    D.far_off = lists[8 * l + 2];
    D.farR_ptr = lists[8 * l + 3];
    D.farR_src = lists[8 * l + 4];
    D.farR_off = lists[8 * l + 5];
    D.child_ptr = lists[8 * l + 6];
    D.parent = lists[8 * l + 7];
    D.n_off = Lv.n_off_used;
    D.ntile = (Lv.nbox + kTile - 1) / kTile;
    D.tile_ptr = lists[8 * (lf + 1) + (lf + 1) + 6 * l + 0];
    D.tile_src = lists[8 * (lf + 1) + (lf + 1) + 6 * l + 1];
    D.tile_off = lists[8 * (lf + 1) + (lf + 1) + 6 * l + 2];
    D.tileR_ptr = lists[8 * (lf + 1) + (lf + 1) + 6 * l + 3];
    D.tileR_src = lists[8 * (lf + 1) + (lf + 1) + 6 * l + 4];
    D.tileR_off = lists[8 * (lf + 1) + (lf + 1) + 6 * l + 5];
    if constexpr (sizeof(R) == 4) {
      D.ntile64 = (Lv.nbox + kTile64 - 1) / kTile64;
      D.tile64_ptr = upload(d, Lv.tile64_ptr, s);
      D.tile64_src = upload(d, Lv.tile64_src, s);
      D.tile64_off = upload(d, Lv.tile64_off, s);
      D.tileR64_ptr = upload(d, Lv.tileR64_ptr, s);
      D.tileR64_src = upload(d, Lv.tileR64_src, s);
      D.tileR64_off = upload(d, Lv.tileR64_off, s);
    }
    D.TZ = upload_complex<R>(d, P.TZ[l], s);
    D.TR = upload_complex<R>(d, P.TR[l], s);
    D.TX = upload_complex<R>(d, P.TX[l], s);
    if (!P.dTZ[l].empty()) D.dTZ = upload_complex<R>(d, P.dTZ[l], s);
    if (l < lf) {
      const Interp& I = P.ip[l];
      D.p = I.p;
      D.ntc = I.ntc;
      D.npc = I.npc;
      D.th_idx = upload(d, I.th_idx, s);
      D.th_ref = upload(d, I.th_ref, s);
      D.th_w = upload(d, cast<R>(I.th_w), s);
      D.ph_idx = upload(d, I.ph_idx, s);
      D.ph_w = upload(d, cast<R>(I.ph_w), s);
      D.tht_ptr = upload(d, I.tht_ptr, s);
      D.tht_idx = upload(d, I.tht_idx, s);
      D.tht_ref = upload(d, I.tht_ref, s);
      D.tht_w = upload(d, cast<R>(I.tht_w), s);
      D.pht_ptr = upload(d, I.pht_ptr, s);
      D.pht_idx = upload(d, I.pht_idx, s);
      D.pht_w = upload(d, cast<R>(I.pht_w), s);
      D.shift = upload_complex<R>(d, P.shift[l], s);
      if (P.opt.flags & CM_FLAG_DERIV) D.dshift = upload_complex<R>(d, P.dshift[l], s);
      if constexpr (sizeof(R) == 4) {
        D.mip = upload_mf(d, P.mf_ip[l], s);
        D.mat = upload_mf(d, P.mf_at[l], s);
        if (D.mip.ok) {
          D.shiftT = upload_shiftT(d, P.shift[l], Lv.nt, Lv.np, D.mip.NT, s);
          if (P.opt.flags & CM_FLAG_DERIV) D.dshiftT = upload_shiftT(d, P.dshift[l], Lv.nt, Lv.np, D.mip.NT, s);
        }
        if (D.mat.ok) {
          D.zg = upload_zg(d, P.shift[l], P.mf_at[l], Lv.nt, Lv.np, s);
          if (P.opt.flags & CM_FLAG_DERIV) D.dzg = upload_zg(d, P.dshift[l], P.mf_at[l], Lv.nt, Lv.np, s);
        }
        if (P.opt.flags & CM_FLAG_AUTOTUNE) {   // the autotuner's other slot-chunk width
          D.mip_alt = upload_mf(d, P.mf_ip_alt[l], s);
          D.mat_alt = upload_mf(d, P.mf_at_alt[l], s);
          if (D.mat_alt.ok) {
            D.zg_alt = upload_zg(d, P.shift[l], P.mf_at_alt[l], Lv.nt, Lv.np, s);
            if (P.opt.flags & CM_FLAG_DERIV)
              D.dzg_alt = upload_zg(d, P.dshift[l], P.mf_at_alt[l], Lv.nt, Lv.np, s);
          }
        }
      }
    }
  }
  for (int l = 2; l <= lf; ++l) pd.lev[l].octant = reinterpret_cast<int8_t*>(lists[8 * (lf + 1) + l]);
  const int K = P.lev[lf].K;
  std::vector<R> qwc(K);
  const double c0 = P.k * P.k * P.opt.eta / (4.0 * M_PI);
  for (int q = 0; q < K; ++q) qwc[q] = (R)(c0 * P.qw[lf][q]);
  pd.qwc = upload(d, qwc, s);
  const size_t vb = (size_t)d.N * 2 * K * 2 * sizeof(R);
  pd.V = dmalloc(d, vb);
  if (P.opt.flags & CM_FLAG_DERIV) pd.dV = dmalloc(d, vb);
}

void dev_build(Dev& d, const Plan& P, hipStream_t s) {
  chk(hipGetDevice(&d.device), "hipGetDevice");
  set_quadrature_constants();
  d.N = P.rwg.N;
  d.nnz = P.nnz;
  d.lf = P.lf;
  d.nleaf = P.lev[P.lf].nbox;
  d.Kleaf = P.lev[P.lf].K;
  d.max_cols = P.opt.max_cols;
  for (int b = 0; b < P.lev[P.lf].nbox; ++b) {
    d.max_box = std::max(d.max_box, P.box_start[b + 1] - P.box_start[b]);
    d.max_near_cols = std::max(d.max_near_cols, P.bcol_ptr[b + 1] - P.bcol_ptr[b]);
  }
  const int lf = P.lf;
  // triangles
  std::vector<TriD> tri(P.nt);
  for (int64_t t = 0; t < P.nt; ++t) {
    for (int v = 0; v < 3; ++v)
      for (int c = 0; c < 3; ++c) tri[t].v[3 * v + c] = P.V[3 * P.F[3 * t + v] + c];
    for (int c = 0; c < 3; ++c) {
      tri[t].n[c] = P.normal[3 * t + c];
      tri[t].c[c] = P.cent[3 * t + c];
    }
    tri[t].area = P.area[t];
    tri[t].hmax = P.hmax[t];
  }
  d.tri = upload(d, tri, s);
  std::vector<RwgD> rw(d.N);
  for (int64_t i = 0; i < d.N; ++i) {
    int64_t n = P.perm[i];
    rw[i].t[0] = P.rwg.tri[2 * n];
    rw[i].t[1] = P.rwg.tri[2 * n + 1];
    rw[i].a[0] = P.rwg.loc[2 * n];
    rw[i].a[1] = P.rwg.loc[2 * n + 1];
    rw[i].len = P.rwg.len[n];
  }
  d.rwg = upload(d, rw, s);
  d.perm = upload(d, P.perm, s);
  d.box_of = upload(d, P.box_of, s);
  d.box_start = upload(d, P.box_start, s);
  d.bcol_ptr = upload(d, P.bcol_ptr, s);
  d.bcol = upload(d, P.bcol, s);
  d.self_off = upload(d, P.self_off, s);
  d.row_ptr = upload(d, P.row_ptr, s);
  {
    const Level& Lf = P.lev[lf];
    std::vector<double> cen(3 * (size_t)Lf.nbox);
    for (int b = 0; b < Lf.nbox; ++b)
      for (int c = 0; c < 3; ++c) cen[3 * b + c] = P.origin[c] + (Lf.ijk[3 * b + c] + 0.5) * Lf.a;
    d.leaf_center = upload(d, cen, s);
    d.leaf_dirs = upload(d, P.dirs[lf], s);
  }
  // index lists shared by both precisions
  std::vector<int32_t*> lists(8 * (lf + 1) + (lf + 1) + 6 * (lf + 1), nullptr);
  for (int l = 2; l <= lf; ++l) {
    const Level& Lv = P.lev[l];
    // receiver-major lists for the single-column translation: each
    // receiver's sources in increasing order with compact translator ids
    auto sorted_lists = [&](const std::vector<int32_t>& ptr, const std::vector<int32_t>& src,
                            const std::vector<int32_t>& off, int slot) {
      std::vector<int32_t> ss(src.size()), so(off.size());
      std::vector<std::pair<int32_t, int32_t>> ent;
      for (int m = 0; m < Lv.nbox; ++m) {
        ent.clear();
        for (int e = ptr[m]; e < ptr[m + 1]; ++e) ent.push_back({src[e], Lv.off_compact[off[e]]});
        std::sort(ent.begin(), ent.end());
        for (size_t i = 0; i < ent.size(); ++i) {
          ss[ptr[m] + i] = ent[i].first;
          so[ptr[m] + i] = ent[i].second;
        }
      }
      lists[8 * l + slot] = upload(d, ptr, s);
      lists[8 * l + slot + 1] = upload(d, ss, s);
      lists[8 * l + slot + 2] = upload(d, so, s);
      chk(hipStreamSynchronize(s), "hipStreamSynchronize");   // ss, so are about to go
    };
    sorted_lists(Lv.far_ptr, Lv.far_src, Lv.far_off, 0);
    sorted_lists(Lv.farR_ptr, Lv.farR_src, Lv.farR_off, 3);
    lists[8 * l + 6] = upload(d, Lv.child_ptr, s);
    lists[8 * l + 7] = upload(d, Lv.parent, s);
    std::vector<int8_t> oc(Lv.nbox);
    for (int b = 0; b < Lv.nbox; ++b) oc[b] = (int8_t)(Lv.code[b] & 7);
    lists[8 * (lf + 1) + l] = reinterpret_cast<int32_t*>(upload(d, oc, s));
    const int tb = 8 * (lf + 1) + (lf + 1) + 6 * l;
    lists[tb + 0] = upload(d, Lv.tile_ptr, s);
    lists[tb + 1] = upload(d, Lv.tile_src, s);
    lists[tb + 2] = upload(d, Lv.tile_off, s);
    lists[tb + 3] = upload(d, Lv.tileR_ptr, s);
    lists[tb + 4] = upload(d, Lv.tileR_src, s);
    lists[tb + 5] = upload(d, Lv.tileR_off, s);
  }
  std::vector<int32_t> dummy;
  build_prec<float>(d, P, d.f32, dummy, lists, s);
  build_prec<double>(d, P, d.f64, dummy, lists, s);
  // near field and leaf patterns (FP64 on the device)
  const bool deriv = (P.opt.flags & CM_FLAG_DERIV) != 0;
  d.Zn = (double2*)dmalloc(d, (size_t)d.nnz * sizeof(double2));
  if (deriv) d.dZn = (double2*)dmalloc(d, (size_t)d.nnz * sizeof(double2));
  launch_leaf_patterns(P.k, d, s);
  chk(hipGetLastError(), "leaf pattern launch");
  launch_near_fill(P.k, P.opt.eta, d, d.nleaf, s);
  chk(hipGetLastError(), "near fill launch");
  // FP32 copies for the FP32 near-field product (CM_FLAG_NEAR_FP32)
  if (P.opt.flags & CM_FLAG_NEAR_FP32) {
    d.Zn32 = (float2*)dmalloc(d, (size_t)std::max<int64_t>(1, d.nnz) * sizeof(float2));
    blas_to_c64(d.Zn, d.Zn32, d.nnz, s);
  }
  if (deriv && (P.opt.flags & CM_FLAG_NEAR_FP32)) {
    d.dZn32 = (float2*)dmalloc(d, (size_t)std::max<int64_t>(1, d.nnz) * sizeof(float2));
    blas_to_c64(d.dZn, d.dZn32, d.nnz, s);
  }
  // workspace
  d.S.assign(lf + 1, nullptr);
  d.G.assign(lf + 1, nullptr);
  const int colmul = deriv ? 2 : 1;   // the dZ/dk pass keeps values and derivatives side by side
  for (int l = 2; l <= lf; ++l) {
    size_t b = (size_t)P.lev[l].nbox * 2 * P.lev[l].K * d.max_cols * colmul * sizeof(double2);
    d.S[l] = dmalloc(d, b);
    d.G[l] = dmalloc(d, b);
  }
  d.xi = dmalloc(d, (size_t)d.N * d.max_cols * sizeof(double2));
  d.yi = dmalloc(d, (size_t)d.N * d.max_cols * sizeof(double2));
  d.red = (double2*)dmalloc(d, (size_t)blas_vdot_blocks() * sizeof(double2));
  // streams and events of the concurrent apply
  for (auto& a : d.aux) chk(hipStreamCreateWithFlags(&a, hipStreamNonBlocking), "hipStreamCreateWithFlags");
  d.fork_ev.assign(4 + lf, nullptr);
  for (auto& e : d.fork_ev) chk(hipEventCreateWithFlags(&e, hipEventDisableTiming), "hipEventCreateWithFlags");
  // autotuning of the matrix-core interpolation shapes at the batch width
  // (the largest multiple of 8 up to max_cols, at most 64) on zeroed workspace
  if ((P.opt.flags & CM_FLAG_AUTOTUNE) && !(P.opt.flags & CM_FLAG_NO_MATRIX_CORES) && d.max_cols >= 8) {
    for (int l = 2; l <= lf; ++l) {
      const size_t b = (size_t)P.lev[l].nbox * 2 * P.lev[l].K * d.max_cols * colmul * sizeof(double2);
      chk(hipMemsetAsync(d.S[l], 0, b, s), "hipMemsetAsync");
      chk(hipMemsetAsync(d.G[l], 0, b, s), "hipMemsetAsync");
    }
    const int tnc = std::min(64, d.max_cols / 8 * 8);
    d.tune_json = mf_autotune(d.f32, lf, d.S, d.G, tnc, s);
    chk(hipGetLastError(), "autotune launches");
    if (!(P.opt.flags & CM_FLAG_M2L_TILE16)) {
      const std::string m = m2l_autotune(d, P, d.S, d.G, tnc, s);
      if (!m.empty()) d.tune_json = d.tune_json.substr(0, d.tune_json.size() - 1) +
                                    (d.tune_json.size() > 2 ? ", " : "") + m + "]";
    }
  }
  chk(hipStreamSynchronize(s), "device set-up");
}

void dev_free(Dev& d) {
  for (void* p : d.allocs) (void)hipFree(p);
  d.allocs.clear();
  for (SaiD& q : d.sai) {
    if (q.ptr) (void)hipFree(q.ptr);
    if (q.col) (void)hipFree(q.col);
    if (q.val) (void)hipFree(q.val);
    q = SaiD();
  }
  for (auto& m : d.marks) {
    (void)hipEventDestroy(m.a);
    (void)hipEventDestroy(m.b);
  }
  d.marks.clear();
  for (auto e : d.event_pool) (void)hipEventDestroy(e);
  for (auto e : d.fork_ev) (void)hipEventDestroy(e);
  d.fork_ev.clear();
  for (auto& a : d.aux)
    if (a) {
      (void)hipStreamDestroy(a);
      a = nullptr;
    }
  d.event_pool.clear();
}


}  // namespace cm

static thread_local std::string g_err;

static cm_status fail(int code, const std::string& msg) {
  g_err = msg;
  return (cm_status)code;
}

namespace cm {
cm_status driver_fail(int code, const std::string& msg) { return fail(code, msg); }
}

#define CM_TRY(...)                                                    \
  try {                                                                \
    __VA_ARGS__                                                        \
  } catch (const cm::Error& e) {                                       \
    return fail(e.code, e.what());                                     \
  } catch (const std::bad_alloc&) {                                    \
    return fail(CM_E_OOM, "host allocation failed");                   \
  } catch (const std::exception& e) {                                  \
    return fail(CM_E_BADARG, e.what());                                \
  }

extern "C" {

void cm_default_opts(cm_opts* o) {
  if (!o) return;
  o->nlv = 0;
  o->d0 = 3.0;
  o->interp_p = 6;
  o->eta = 376.730313668;
  o->flags = 0;
  o->max_cols = 32;
  o->k_sampling = 0;
}

static void free_csr(cm::CsrD& m) {
  if (m.ptr) (void)hipFree(m.ptr);
  if (m.col) (void)hipFree(m.col);
  if (m.val) (void)hipFree(m.val);
  m = cm::CsrD();
}

static void destroy_handle(cm_handle* h);

static void free_cmp(cm::CmpD* c) {
  if (!c) return;
  destroy_handle(c->ref);
  free_csr(c->B);
  free_csr(c->Bt);
  free_csr(c->G);
  delete c;
}

static void destroy_handle(cm_handle* h) {
  if (!h) return;
  free_cmp(h->cmp);
  h->cmp = nullptr;
  for (cm_handle* t : h->sub) destroy_handle(t);
  h->sub.clear();
  if (h->xs) (void)hipFree(h->xs);
  if (h->ys) (void)hipFree(h->ys);
  if (h->ks_in) (void)hipEventDestroy(h->ks_in);
  if (h->ks_out) (void)hipEventDestroy(h->ks_out);
  if (h->ks) (void)hipStreamDestroy(h->ks);
  cm::dev_free(h->dev);
  delete h;
}

static cm_handle* build_handle(const double* xyz, int64_t n_vert, const int32_t* tri, int64_t n_tri, double k,
                               const cm::Opts& op, uint32_t flags, hipStream_t s) {
  std::unique_ptr<cm_handle> h(new cm_handle());
  h->plan.build(xyz, n_vert, tri, n_tri, k, op);
  if (!(flags & CM_FLAG_HOST_ONLY)) {
    try {
      cm::dev_build(h->dev, h->plan, s);
    } catch (...) {
      cm::dev_free(h->dev);
      throw;
    }
    h->has_dev = true;
  }
  return h.release();
}

cm_status cm_create(const double* xyz, int64_t n_vert, const int32_t* tri, int64_t n_tri, const double* k,
                    int32_t n_k, const cm_opts* o, void* hip_stream, cm_handle** out) {
  g_err.clear();
  if (out) *out = nullptr;
  if (!xyz || !tri || !k || !o || !out) return fail(CM_E_BADARG, "null argument");
  if (n_k < 1 || n_k > 64) return fail(CM_E_BADARG, "n_k out of range [1, 64]");
  if (n_vert < 3 || n_tri < 2 || n_vert > (1LL << 31) - 1 || n_tri > (1LL << 31) - 1)
    return fail(CM_E_BADARG, "mesh size out of range");
  CM_TRY({
    cm::Opts op;
    op.nlv = o->nlv;
    op.d0 = o->d0;
    op.p = o->interp_p;
    op.eta = (o->eta > 0) ? o->eta : 376.730313668;
    op.flags = o->flags;
    op.max_cols = o->max_cols;
    op.k_sampling = o->k_sampling;
    const bool shared = n_k > 1 && (o->flags & CM_FLAG_SWEEP_SHARED);
    if (shared && !(o->k_sampling > 0)) {
      op.k_sampling = k[0];
      for (int i = 1; i < n_k; ++i) op.k_sampling = std::max(op.k_sampling, k[i]);
    }
    cm_handle* h = build_handle(xyz, n_vert, tri, n_tri, k[0], op, o->flags, (hipStream_t)hip_stream);
    try {
      for (int i = 1; i < n_k; ++i)
        h->sub.push_back(build_handle(xyz, n_vert, tri, n_tri, k[i], op, o->flags, (hipStream_t)hip_stream));
      if (shared && h->has_dev) {
        std::vector<const cm::Plan*> pk{&h->plan};
        for (cm_handle* t : h->sub) pk.push_back(&t->plan);
        cm::build_sweep_tables(h->dev, h->plan, pk, (hipStream_t)hip_stream);
      }
      if (n_k > 1 && h->has_dev) {
        const size_t b = (size_t)h->dev.N * h->dev.max_cols * 16;
        for (int i = 0; i < n_k; ++i) {
          cm_handle* t = i == 0 ? h : h->sub[i - 1];
          if (hipMalloc(&t->xs, b) != hipSuccess || hipMalloc(&t->ys, b) != hipSuccess)
            throw cm::Error(CM_E_OOM, "sweep staging buffers");
          if (hipStreamCreateWithFlags(&t->ks, hipStreamNonBlocking) != hipSuccess ||
              hipEventCreateWithFlags(&t->ks_in, hipEventDisableTiming) != hipSuccess ||
              hipEventCreateWithFlags(&t->ks_out, hipEventDisableTiming) != hipSuccess)
            throw cm::Error(CM_E_HIP, "sweep stream and events");
        }
      }
    } catch (...) {
      destroy_handle(h);
      throw;
    }
    *out = h;
    return CM_OK;
  })
}

void cm_destroy(cm_handle* h) { destroy_handle(h); }

static void upload_csr(const cm::CsrHost& m, cm::CsrD& d) {
  d.rows = m.rows;
  d.nnz = (int64_t)m.col.size();
  auto chk = [](hipError_t e) {
    if (e != hipSuccess) throw cm::Error(e == hipErrorOutOfMemory ? CM_E_OOM : CM_E_HIP, "Calderon tables upload");
  };
  chk(hipMalloc(&d.ptr, (m.rows + 1) * sizeof(int64_t)));
  chk(hipMalloc(&d.col, std::max<int64_t>(1, d.nnz) * sizeof(int32_t)));
  chk(hipMalloc(&d.val, std::max<int64_t>(1, d.nnz) * sizeof(double)));
  chk(hipMemcpy(d.ptr, m.ptr.data(), (m.rows + 1) * sizeof(int64_t), hipMemcpyHostToDevice));
  if (d.nnz) {
    chk(hipMemcpy(d.col, m.col.data(), d.nnz * sizeof(int32_t), hipMemcpyHostToDevice));
    chk(hipMemcpy(d.val, m.val.data(), d.nnz * sizeof(double), hipMemcpyHostToDevice));
  }
}

cm_status cm_cmp_build(cm_handle* h, int32_t nlv_refined, int32_t interp_p_refined, double d0_refined,
                       int64_t* info, void* hip_stream) {
  g_err.clear();
  if (!h) return fail(CM_E_BADARG, "null argument");
  if (nlv_refined != 0 && (nlv_refined < 3 || nlv_refined > 20))
    return fail(CM_E_BADARG, "nlv_refined must be 0 or in [3, 20]");
  if (interp_p_refined < 0 || interp_p_refined > 32 || !(d0_refined >= 0) || d0_refined > 20)
    return fail(CM_E_BADARG, "interp_p_refined must be in [0, 32] and d0_refined in [0, 20]");
  CM_TRY({
    std::vector<double> Vr;
    std::vector<int32_t> Fr;
    cm::cmp_refine(h->plan, Vr, Fr);
    cm::Opts op = h->plan.opt;
    op.nlv = nlv_refined > 0 ? nlv_refined : h->plan.nlv + 1;
    if (interp_p_refined > 0) op.p = interp_p_refined;
    if (d0_refined > 0) op.d0 = d0_refined;
    op.max_cols = 1;
    op.flags &= ~(uint32_t)(CM_FLAG_DERIV | CM_FLAG_AUTOTUNE | CM_FLAG_VERBOSE | CM_FLAG_HOST_ONLY);
    op.flags |= CM_FLAG_NEAR_FP32;   // FP32 products of Z~ read FP32 near-field values
    if (!h->has_dev) op.flags |= CM_FLAG_HOST_ONLY;
    std::unique_ptr<cm::CmpD, void (*)(cm::CmpD*)> c(new cm::CmpD(), free_cmp);
    c->ref = build_handle(Vr.data(), (int64_t)Vr.size() / 3, Fr.data(), (int64_t)Fr.size() / 3, h->plan.k, op,
                          op.flags, (hipStream_t)hip_stream);
    c->Nr = c->ref->plan.rwg.N;
    cm::CsrHost Bt;
    cm::cmp_tables(h->plan, c->ref->plan, Vr, Fr, c->hB, Bt, c->hG);
    if (h->has_dev) {
      upload_csr(c->hB, c->B);
      upload_csr(Bt, c->Bt);
      upload_csr(c->hG, c->G);
    }
    if (info) {
      info[0] = c->Nr;
      info[1] = (int64_t)c->hB.col.size();
      info[2] = (int64_t)c->hG.col.size();
      info[3] = c->ref->plan.nnz;
      info[4] = c->ref->plan.nlv;
    }
    free_cmp(h->cmp);
    h->cmp = c.release();
    return CM_OK;
  })
}

cm_status cm_cmp_export(const cm_handle* h, int32_t which, int64_t* rows, int64_t* nnz, int64_t* ptr, int32_t* col,
                        double* val) {
  g_err.clear();
  if (!h || !rows || !nnz) return fail(CM_E_BADARG, "null argument");
  if (!h->cmp) return fail(CM_E_NOT_BUILT, "Calderon preconditioner not built");
  if (which != 0 && which != 1) return fail(CM_E_BADARG, "which must be 0 (B) or 1 (G)");
  const cm::CsrHost& m = which == 0 ? h->cmp->hB : h->cmp->hG;
  *rows = m.rows;
  *nnz = (int64_t)m.col.size();
  if (ptr && col && val) {
    std::memcpy(ptr, m.ptr.data(), (m.rows + 1) * sizeof(int64_t));
    std::memcpy(col, m.col.data(), m.col.size() * sizeof(int32_t));
    std::memcpy(val, m.val.data(), m.val.size() * sizeof(double));
  }
  return CM_OK;
}

cm_status cm_num_unknowns(const cm_handle* h, int64_t* n) {
  if (!h || !n) return fail(CM_E_BADARG, "null argument");
  *n = h->plan.rwg.N;
  return CM_OK;
}

cm_status cm_rwg_table(const cm_handle* h, int32_t* edge_v, int32_t* tri_pm) {
  if (!h || !edge_v || !tri_pm) return fail(CM_E_BADARG, "null argument");
  const auto& r = h->plan.rwg;
  std::memcpy(edge_v, r.edge.data(), r.edge.size() * sizeof(int32_t));
  std::memcpy(tri_pm, r.tri.data(), r.tri.size() * sizeof(int32_t));
  return CM_OK;
}

static cm_status check_vec_args(const cm_handle* h, const void* x, const void* y, int64_t ld, int32_t ncols,
                                cm_dtype dt) {
  if (!h || !x || !y) return fail(CM_E_BADARG, "null argument");
  if (!h->has_dev) return fail(CM_E_NOT_BUILT, "handle was built host-only");
  if (ncols < 1 || ncols > h->dev.max_cols) return fail(CM_E_BADARG, "ncols out of range [1, max_cols]");
  if (ld < ncols) return fail(CM_E_BADARG, "ld < ncols");
  if (dt != CM_C64 && dt != CM_C128) return fail(CM_E_BADARG, "bad dtype");
  if (x == y) return fail(CM_E_BADARG, "x and y must not alias");
  return CM_OK;
}

}  // extern "C"

// Run per_k(t, x, y, ld, ncols, stream) for the columns of each wavenumber:
// in place when every column has the same wavenumber, otherwise the columns
// of each wavenumber are gathered into that wavenumber's staging block
// (padded with zero columns to a multiple of 8 where the buffers allow it, so
// that the batch takes the matrix-core kernels), processed on that
// wavenumber's stream (forked from and joined to the caller's stream by
// events) and scattered back.
template <typename F>
static void by_wavenumber(cm_handle* h, const void* x, void* y, int64_t ld, int32_t ncols, const int32_t* k_index,
                          bool fp64, hipStream_t s, F per_k) {
  auto at = [&](int kk) { return kk == 0 ? h : h->sub[kk - 1]; };
  const int nk = 1 + (int)h->sub.size();
  bool one = true;
  for (int j = 1; k_index && j < ncols; ++j) one = one && k_index[j] == k_index[0];
  if (one) {
    per_k(at(k_index ? k_index[0] : 0), x, y, ld, ncols, s);
    return;
  }
  auto ok = [](hipError_t e) {
    if (e != hipSuccess) throw cm::Error(CM_E_HIP, std::string("sweep: ") + hipGetErrorString(e));
  };
  ok(hipEventRecord(h->ks_in, s));
  for (int kk = 0; kk < nk; ++kk) {
    cm::ColList cl;
    cl.n = 0;
    for (int j = 0; j < ncols; ++j)
      if (k_index[j] == kk) cl.c[cl.n++] = j;
    if (cl.n == 0) continue;
    cm_handle* t = at(kk);
    const int w8 = (cl.n + 7) / 8 * 8;
    const int ws = (w8 <= h->dev.max_cols) ? w8 : cl.n;
    ok(hipStreamWaitEvent(t->ks, h->ks_in, 0));
    cm::blas_gather_cols(x, ld, cl, ws, t->xs, h->dev.N, fp64, t->ks);
    per_k(t, t->xs, t->ys, ws, ws, t->ks);
    cm::blas_scatter_cols(t->ys, ws, cl, y, ld, h->dev.N, fp64, t->ks);
    ok(hipEventRecord(t->ks_out, t->ks));
    ok(hipStreamWaitEvent(s, t->ks_out, 0));
  }
  if (hipGetLastError() != hipSuccess) throw cm::Error(CM_E_HIP, "sweep gather/scatter launch");
}

// The one-pass route of a wavenumber sweep (CM_FLAG_SWEEP_SHARED, FP32, op Z
// or Z^H, columns at more than one wavenumber): the columns of each
// wavenumber in slots of four (the last one padded with zero columns).  When
// slot j is exactly columns 4j .. 4j+3 of x the pass reads x and writes y in
// place, otherwise it gathers the slots into the staging block and scatters
// the result back.  False (nothing launched) when the batch does not fit:
// more than 16 slots, more than max_cols slot columns, or a level the
// matrix-core kernels do not cover.
static bool sweep_one_pass(cm_handle* h, int op, const void* x, void* y, int64_t ld, int ncols,
                           const int32_t* k_index, hipStream_t s) {
  if (h->dev.sw_nk <= 0 || !k_index) return false;
  bool one = true;
  for (int j = 1; j < ncols; ++j) one = one && k_index[j] == k_index[0];
  if (one) return false;
  const int nk = 1 + (int)h->sub.size();
  cm::SweepSlots sw;
  sw.on = 1;
  cm::ColList cl;
  cl.n = 0;
  for (int kk = 0; kk < nk; ++kk) {
    int cnt = 0;
    for (int j = 0; j < ncols; ++j)
      if (k_index[j] == kk) {
        if (cnt % 4 == 0) {
          if (sw.n == cm::kMaxSlots) return false;
          sw.k[sw.n++] = kk;
        }
        if (cl.n == 64) return false;
        cl.c[cl.n++] = j;
        ++cnt;
      }
    while (cnt % 4 != 0) {
      if (cl.n == 64) return false;
      cl.c[cl.n++] = -1;
      ++cnt;
    }
  }
  const int nc = 4 * sw.n;
  if (!cm::sweep_covers(h->dev, h->plan, nc)) return false;
  std::vector<cm::Dev*> dk{&h->dev};
  std::vector<const cm::Plan*> pk{&h->plan};
  for (cm_handle* t : h->sub) {
    dk.push_back(&t->dev);
    pk.push_back(&t->plan);
  }
  bool inplace = true;
  for (int j = 0; j < cl.n; ++j) inplace = inplace && cl.c[j] == j;
  if (inplace) {
    cm::dev_apply_sweep(h->dev, h->plan, dk.data(), pk.data(), sw, op, x, y, ld, s);
  } else {
    cm::blas_gather_cols(x, ld, cl, nc, h->xs, h->dev.N, false, s);
    cm::dev_apply_sweep(h->dev, h->plan, dk.data(), pk.data(), sw, op, h->xs, h->ys, nc, s);
    cm::blas_scatter_cols(h->ys, nc, cl, y, ld, h->dev.N, false, s);
  }
  return true;
}

extern "C" {

static cm_status check_k_index(const cm_handle* h, const int32_t* k_index, int32_t ncols) {
  const int nk = 1 + (int)h->sub.size();
  if (k_index)
    for (int j = 0; j < ncols; ++j)
      if (k_index[j] < 0 || k_index[j] >= nk) return fail(CM_E_BADARG, "k_index out of range [0, n_k)");
  return CM_OK;
}

cm_status cm_apply(cm_handle* h, cm_op op, const void* x, void* y, int64_t ld, int32_t ncols,
                   const int32_t* k_index, cm_dtype dt, void* hip_stream) {
  g_err.clear();
  cm_status st = check_vec_args(h, x, y, ld, ncols, dt);
  if (st != CM_OK) return st;
  if ((int)op < 0 || (int)op > 4) return fail(CM_E_BADARG, "bad op");
  if (op == CM_OP_DZDK && !(h->plan.opt.flags & CM_FLAG_DERIV))
    return fail(CM_E_NOT_BUILT, "dZ/dk needs CM_FLAG_DERIV at create");
  if ((st = check_k_index(h, k_index, ncols)) != CM_OK) return st;
  const bool fp64 = dt == CM_C128;
  CM_TRY({
    if (!fp64 && (op == CM_OP_Z || op == CM_OP_ZH) && sweep_one_pass(h, (int)op, x, y, ld, ncols, k_index,
                                                                    (hipStream_t)hip_stream))
      return CM_OK;
    by_wavenumber(h, x, y, ld, ncols, k_index, fp64, (hipStream_t)hip_stream,
                  [&](cm_handle* t, const void* xx, void* yy, int64_t l, int n, hipStream_t ss) {
                    cm::dev_apply(t->dev, t->plan, (int)op, xx, yy, l, n, fp64, ss);
                  });
    return CM_OK;
  })
}

static cm_status check_tau(double tau) {
  if (!(tau >= 0) || !(tau <= 1e6)) return fail(CM_E_BADARG, "tau must be in [0, 1e6]");
  return CM_OK;
}

cm_status cm_sai_build(cm_handle* h, double eps1, double eps2, double eps3, int32_t k_index, double tau) {
  g_err.clear();
  if (!h) return fail(CM_E_BADARG, "null argument");
  if (!h->has_dev) return fail(CM_E_NOT_BUILT, "handle was built host-only");
  if (!(eps1 >= 0) || !(eps2 >= 0) || !(eps3 >= 0) || eps1 > 1 || eps2 > 1 || eps3 > 1)
    return fail(CM_E_BADARG, "thresholds must be in [0, 1]");
  if (k_index < 0 || k_index > (int)h->sub.size()) return fail(CM_E_BADARG, "k_index out of range [0, n_k)");
  cm_status st = check_tau(tau);
  if (st != CM_OK) return st;
  cm_handle* t = k_index == 0 ? h : h->sub[k_index - 1];
  CM_TRY({
    cm::dev_sai_build(t->dev, t->plan, eps1, eps2, eps3, tau, nullptr);
    return CM_OK;
  })
}

cm_status cm_sai_apply(cm_handle* h, const void* x, void* y, int64_t ld, int32_t ncols, const int32_t* k_index,
                       double tau, cm_dtype dt, void* hip_stream) {
  g_err.clear();
  cm_status st = check_vec_args(h, x, y, ld, ncols, dt);
  if (st != CM_OK) return st;
  if ((st = check_k_index(h, k_index, ncols)) != CM_OK) return st;
  if ((st = check_tau(tau)) != CM_OK) return st;
  const int slot = cm::sai_slot(tau);
  for (int j = 0; j < (k_index ? ncols : 1); ++j) {
    const cm_handle* t = (!k_index || k_index[j] == 0) ? h : h->sub[k_index[j] - 1];
    if (!t->dev.sai[slot].val || (slot == 1 && t->dev.sai_tau1 != tau))
      return fail(CM_E_NOT_BUILT, "SAI not built for this wavenumber and tau");
  }
  const bool fp64 = dt == CM_C128;
  CM_TRY({
    by_wavenumber(h, x, y, ld, ncols, k_index, fp64, (hipStream_t)hip_stream,
                  [&](cm_handle* t, const void* xx, void* yy, int64_t l, int n, hipStream_t ss) {
                    cm::dev_sai_apply(t->dev, t->plan, xx, yy, l, n, fp64, slot, ss);
                  });
    return CM_OK;
  })
}

cm_status cm_vdot(cm_handle* h, const void* x, const void* y, int64_t ld, int32_t ncols, cm_dtype dt, void* out,
                  void* hip_stream) {
  g_err.clear();
  if (!h || !x || !y || !out) return fail(CM_E_BADARG, "null argument");
  if (!h->has_dev) return fail(CM_E_NOT_BUILT, "handle was built host-only");
  if (ncols < 1 || ld < ncols) return fail(CM_E_BADARG, "need ncols >= 1 and ld >= ncols");
  if (dt != CM_C64 && dt != CM_C128) return fail(CM_E_BADARG, "bad dtype");
  CM_TRY({
    cm::blas_vdot(x, y, ld, ncols, h->dev.N, dt == CM_C128, h->dev.red, (double2*)out, (hipStream_t)hip_stream);
    if (hipGetLastError() != hipSuccess) throw cm::Error(CM_E_HIP, "vdot launch");
    return CM_OK;
  })
}

cm_status cm_export_near(const cm_handle* h, int32_t which, int64_t* nnz, int64_t* row_ptr, int32_t* col,
                         double* val) {
  g_err.clear();
  if (!h || !nnz) return fail(CM_E_BADARG, "null argument");
  if (!h->has_dev) return fail(CM_E_NOT_BUILT, "handle was built host-only");
  const cm::Plan& P = h->plan;
  const cm::Dev& d = h->dev;
  if (which == 0 || which == 1) {
    if (which == 1 && !d.dZn) return fail(CM_E_NOT_BUILT, "dZ/dk near field needs CM_FLAG_DERIV");
    *nnz = P.nnz;
    if (!row_ptr && !col && !val) return CM_OK;
    if (!row_ptr || !col || !val) return fail(CM_E_BADARG, "null output array");
    CM_TRY({
      std::vector<double2> v(P.nnz);
      cm::chk(hipMemcpy(v.data(), which ? d.dZn : d.Zn, P.nnz * sizeof(double2), hipMemcpyDeviceToHost),
              "export copy");
      const int64_t N = P.rwg.N;
      row_ptr[0] = 0;
      for (int64_t m = 0; m < N; ++m) {
        int64_t i = P.iperm[m];
        row_ptr[m + 1] = row_ptr[m] + (P.row_ptr[i + 1] - P.row_ptr[i]);
      }
      for (int64_t m = 0; m < N; ++m) {
        int64_t i = P.iperm[m];
        int b = P.box_of[i];
        int64_t src = P.row_ptr[i], dst = row_ptr[m];
        int ncl = P.bcol_ptr[b + 1] - P.bcol_ptr[b];
        for (int t = 0; t < ncl; ++t) {
          col[dst + t] = P.perm[P.bcol[P.bcol_ptr[b] + t]];
          val[2 * (dst + t)] = v[src + t].x;
          val[2 * (dst + t) + 1] = v[src + t].y;
        }
      }
      return CM_OK;
    })
  }
  if (which == 2 || which == 3) {
    const cm::SaiD& q = d.sai[which - 2];
    if (!q.val) return fail(CM_E_NOT_BUILT, "SAI not built");
    *nnz = q.nnz;
    if (!row_ptr && !col && !val) return CM_OK;
    if (!row_ptr || !col || !val) return fail(CM_E_BADARG, "null output array");
    CM_TRY({
      const int64_t N = P.rwg.N;
      std::vector<int64_t> ptr(N + 1);
      std::vector<int32_t> c(q.nnz);
      std::vector<double2> v(q.nnz);
      cm::chk(hipMemcpy(ptr.data(), q.ptr, (N + 1) * sizeof(int64_t), hipMemcpyDeviceToHost), "export");
      cm::chk(hipMemcpy(c.data(), q.col, q.nnz * sizeof(int32_t), hipMemcpyDeviceToHost), "export");
      cm::chk(hipMemcpy(v.data(), q.val, q.nnz * sizeof(double2), hipMemcpyDeviceToHost), "export");
      row_ptr[0] = 0;
      for (int64_t m = 0; m < N; ++m) {
        int64_t i = P.iperm[m];
        row_ptr[m + 1] = row_ptr[m] + (ptr[i + 1] - ptr[i]);
      }
      for (int64_t m = 0; m < N; ++m) {
        int64_t i = P.iperm[m];
        int64_t dst = row_ptr[m];
        for (int64_t t = ptr[i]; t < ptr[i + 1]; ++t, ++dst) {
          col[dst] = P.perm[c[t]];
          val[2 * dst] = v[t].x;
          val[2 * dst + 1] = v[t].y;
        }
      }
      return CM_OK;
    })
  }
  return fail(CM_E_BADARG, "which must be 0, 1, 2 or 3");
}

cm_status cm_stats(const cm_handle* h, char* buf, int64_t buf_len, int64_t* needed) {
  if (!h) return fail(CM_E_BADARG, "null argument");
  std::string s = h->plan.stats_json();
  if (h->has_dev && !h->dev.tune_json.empty() && !s.empty() && s.back() == '}')
    s = s.substr(0, s.size() - 1) + ", \"autotune\": " + h->dev.tune_json + "}";
  if (h->has_dev && h->dev.sw_nk > 0 && !s.empty() && s.back() == '}')
    s = s.substr(0, s.size() - 1) + ", \"sweep_tables\": " + std::to_string(h->dev.sw_nk) +
        ", \"sweep_one_pass_calls\": " + std::to_string(h->dev.sw_calls) + "}";
  if (needed) *needed = (int64_t)s.size() + 1;
  if (!buf || buf_len < (int64_t)s.size() + 1) return fail(CM_E_BADARG, "buffer too small");
  std::memcpy(buf, s.c_str(), s.size() + 1);
  return CM_OK;
}

cm_status cm_set_translation_kernel(cm_handle* h, int32_t variant) {
  g_err.clear();
  if (!h) return fail(CM_E_BADARG, "null argument");
  if (!h->has_dev) return fail(CM_E_NOT_BUILT, "handle was built host-only");
  if (variant < 1 || variant > 4) return fail(CM_E_BADARG, "variant must be in 1..4");
  auto pin = [&](cm_handle* t) {
    for (auto& L : t->dev.f32.lev) L.m2l_variant = variant;
  };
  pin(h);
  for (cm_handle* u : h->sub) pin(u);
  return CM_OK;
}

cm_status cm_stage_timing(cm_handle* h, int32_t enable) {
  g_err.clear();
  if (!h) return fail(CM_E_BADARG, "null argument");
  if (!h->has_dev) return fail(CM_E_NOT_BUILT, "handle was built host-only");
  CM_TRY({
    cm::collect_stage_times(h->dev);
    h->dev.timing = (enable != 0);
    std::fill(h->dev.stage_ms.begin(), h->dev.stage_ms.end(), 0.0);
    std::fill(h->dev.stage_calls.begin(), h->dev.stage_calls.end(), 0);
    return CM_OK;
  })
}

cm_status cm_stage_times(cm_handle* h, char* buf, int64_t buf_len, int64_t* needed) {
  g_err.clear();
  if (!h) return fail(CM_E_BADARG, "null argument");
  if (!h->has_dev) return fail(CM_E_NOT_BUILT, "handle was built host-only");
  CM_TRY({
    cm::collect_stage_times(h->dev);
    static const char* names[8] = {"permute", "near", "aggregate", "interp", "m2l", "anterp", "disagg", "sai"};
    std::string s = "{";
    bool first = true;
    for (int id = 0; id < (int)h->dev.stage_ms.size(); ++id) {
      if (!h->dev.stage_calls[id]) continue;
      char item[128];
      int base = id % 10, lvl = id / 10;
      std::string nm = names[base];
      if (base >= 3 && base <= 5) nm += "_l" + std::to_string(lvl);
      std::snprintf(item, sizeof item, "%s\"%s\": {\"ms\": %.9g, \"calls\": %lld}", first ? "" : ", ", nm.c_str(),
                    h->dev.stage_ms[id], (long long)h->dev.stage_calls[id]);
      s += item;
      first = false;
    }
    s += "}";
    if (needed) *needed = (int64_t)s.size() + 1;
    if (!buf || buf_len < (int64_t)s.size() + 1) return fail(CM_E_BADARG, "buffer too small");
    std::memcpy(buf, s.c_str(), s.size() + 1);
    return CM_OK;
  })
}

const char* cm_last_error(void) { return g_err.c_str(); }

}  // extern "C"
