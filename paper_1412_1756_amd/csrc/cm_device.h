// Device-side data of a handle and the kernel launchers (gfx950).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/cmmlfma.h"
#include "cm_plan.h"

namespace cm {

// Triangle record used by the fill kernels (17 doubles).
struct TriD {
  double v[9];      // vertices
  double n[3];      // unit normal
  double c[3];      // centroid
  double area, hmax;
};
// RWG record in internal (box-sorted) order.
struct RwgD {
  int32_t t[2];     // T+, T-
  int32_t a[2];     // local vertex opposite the edge in T+, T-
  double len;
};

// Columns of a one-pass wavenumber-sweep batch: slots of four columns, slot
// j at the handle's wavenumber k[j]; the kernels index per-wavenumber tables
// (translators, shift phases) `stride` complex values apart.  on == 0: an
// ordinary batch (one wavenumber, columns in tiles of eight).
constexpr int kMaxSlots = 16;
struct SweepSlots {
  int on = 0;
  int n = 0;
  int32_t k[kMaxSlots] = {};
  int64_t stride = 0;
  int zg_global = 0;   // anterpolation: read the slot's phase values from global memory (set by the launcher)
};

// Leaf stages of a one-pass sweep launched for all slots at once: slot z > 0
// takes the tables t0[z], t1[z] and the kernel's arrays moved by z times the
// given element offsets (slot 0: the launch arguments).  The near field puts
// the slot on grid z; aggregation and disaggregation make it the fastest
// block index (n slots), so that the slots' 32-byte pieces of a box's
// pattern rows are written (read) back to back while the lines are in L2.
struct SlotTabs {
  const void* t0[kMaxSlots] = {};
  const void* t1[kMaxSlots] = {};
  int64_t in_off = 0, out_off = 0, aux_off = 0;
  int n = 1;
};

// Matrix-core interpolation tables of one level pair (FP32 path), see MfTab.
struct MfD {
  int ok = 0, NT = 0, S2 = 0, half = 0, nchunk = 0, kmax = 0, ktmax = 0;
  int32_t *chunk = nullptr, *nk = nullptr, *kidx = nullptr, *nkt = nullptr, *tidx = nullptr;
  float *kA = nullptr, *tA = nullptr;
};

template <typename R>
struct LevelD {
  int nbox = 0, K = 0, nt = 0, np = 0;
  int32_t *far_ptr = nullptr, *far_src = nullptr, *far_off = nullptr;
  int32_t *farR_ptr = nullptr, *farR_src = nullptr, *farR_off = nullptr;
  int32_t *child_ptr = nullptr, *parent = nullptr;
  int8_t* octant = nullptr;                 // child position in its parent (code & 7)
  int n_off = 0;                            // translators stored for the used offsets only
  void *TZ = nullptr, *TR = nullptr, *TX = nullptr, *dTZ = nullptr;  // n_off x K complex<R>
  int ntile = 0;
  int32_t *tile_ptr = nullptr, *tile_src = nullptr, *tileR_ptr = nullptr, *tileR_src = nullptr;
  int32_t *tile_off = nullptr, *tileR_off = nullptr;
  int ntile64 = 0;                          // tiles of kTile64 receivers (FP32 shared-source translation)
  int m2l_variant = 0;                      // FP32 batched translation kernel (0, 1: 16-box tiles, 2-4:
                                            // 64-box shared-source tiles, only where the autotuner picks them)
  int32_t *tile64_ptr = nullptr, *tile64_src = nullptr, *tile64_off = nullptr;
  int32_t *tileR64_ptr = nullptr, *tileR64_src = nullptr, *tileR64_off = nullptr;
  // interpolation from level l+1 into this level (l = 2..lf-1)
  int p = 0, ntc = 0, npc = 0;
  int32_t *th_idx = nullptr, *th_ref = nullptr, *ph_idx = nullptr;
  R *th_w = nullptr, *ph_w = nullptr;
  int32_t *tht_ptr = nullptr, *tht_idx = nullptr, *tht_ref = nullptr, *pht_ptr = nullptr, *pht_idx = nullptr;
  R *tht_w = nullptr, *pht_w = nullptr;
  void* shift = nullptr;                    // 8 x K complex<R>: exp(ik khat.(r_child - r_parent))
  void* dshift = nullptr;                   // its k-derivative (CM_FLAG_DERIV)
  // FP32 matrix-core path: tables and the phase tables as [8][np][16 NT] (theta fastest, zero padded)
  MfD mip, mat;
  void *shiftT = nullptr, *dshiftT = nullptr;
  // anterpolation: phase values per slot chunk and octant in K-step key order,
  // [nchunk][8][nt][4 kmax] complex (and the k-derivative)
  void *zg = nullptr, *dzg = nullptr;
  // autotuning: the tables with the other slot-chunk width (swapped in when
  // faster) and the rows per load group of each kernel (0: default)
  MfD mip_alt, mat_alt;
  void *zg_alt = nullptr, *dzg_alt = nullptr;
  int rg_ip = 0, rg_at = 0;
  // one-pass wavenumber sweeps (CM_FLAG_SWEEP_SHARED, on the first
  // wavenumber's handle): Z's translators of all wavenumbers interleaved,
  // [n_off][K][n_k], and the shift tables of the interpolation into this
  // level (shiftT layout) and of the anterpolation from it (zg layout of the
  // table in use), one wavenumber after the other
  void* sw_T = nullptr;
  void *sw_shiftT = nullptr, *sw_zg = nullptr;
  int64_t sw_shift_stride = 0, sw_zg_stride = 0;
};

template <typename R>
struct PrecD {
  void* V = nullptr;                        // N x 2 x K_leaf complex<R>, leaf radiation patterns
  void* dV = nullptr;                       // d/dk of V (CM_FLAG_DERIV)
  R* qwc = nullptr;                         // K_leaf: (k^2 eta / 4 pi) w_q
  std::vector<LevelD<R>> lev;
};

// A sparse approximate inverse in CSR by internal rows (internal column indices).
struct SaiD {
  int64_t nnz = 0;
  int64_t* ptr = nullptr;                   // N + 1
  int32_t* col = nullptr;
  double2* val = nullptr;
};

struct Dev {
  int device = 0;
  int64_t N = 0, nnz = 0;
  int lf = 0, nleaf = 0, Kleaf = 0, max_cols = 0, max_box = 0;   // max_box: most unknowns in a leaf box
  int max_near_cols = 0;                    // most near-field columns of a leaf box
  TriD* tri = nullptr;
  RwgD* rwg = nullptr;
  int32_t *perm = nullptr, *box_of = nullptr, *box_start = nullptr;
  int32_t *bcol_ptr = nullptr, *bcol = nullptr, *self_off = nullptr;
  int64_t* row_ptr = nullptr;
  double* leaf_center = nullptr;            // 3 x nleaf
  double* leaf_dirs = nullptr;              // 9 x K_leaf
  double2* Zn = nullptr;                    // near-field values (nnz)
  double2* dZn = nullptr;                   // dZ_near/dk values (nnz)
  float2 *Zn32 = nullptr, *dZn32 = nullptr; // their FP32 copies (FP32 matrix-core near field)
  PrecD<float> f32;
  PrecD<double> f64;
  // workspace (sized for max_cols, complex double; reused as complex float)
  std::vector<void*> S, G, dS, dG;          // per level
  void *xi = nullptr, *yi = nullptr, *dxi = nullptr;
  // SAI preconditioners: sai[0] of Z_near; sai[1] of the near field of the
  // shifted operator tau R + i X for sai_tau1 (tau 0: the real X_near)
  SaiD sai[2];
  double sai_tau1 = -1;
  double2* red = nullptr;                   // partial sums of cm_vdot (blas_vdot_blocks() entries)
  std::vector<void*> allocs;
  // optional per-stage timing (HIP events on the apply stream)
  bool timing = false;
  struct Mark {
    int stage;
    hipEvent_t a, b;
  };
  std::vector<Mark> marks;
  std::vector<hipEvent_t> event_pool;
  // concurrent apply: two auxiliary streams (default priority, non-blocking)
  // for the near field and the translations off the critical path, and the
  // fork/join events (timing disabled); null when not created
  hipStream_t aux[2] = {nullptr, nullptr};
  std::vector<hipEvent_t> fork_ev;
  std::vector<double> stage_ms;
  std::vector<int64_t> stage_calls;
  std::string tune_json;                    // autotuner's choices (empty when not tuned)
  int sw_nk = 0;                            // wavenumbers of the one-pass sweep tables (0: none)
  int64_t sw_calls = 0;                     // one-pass sweep applies so far
};

// stage ids for timing: 0 permute, 1 near, 2 aggregate, 3 interp, 4 m2l,
// 5 anterp, 6 disagg, 7 sai; the level is added as 10*l for per-level stages.
void stage_begin(Dev& d, hipStream_t s, int stage);
void stage_end(Dev& d, hipStream_t s);
void collect_stage_times(Dev& d);

// Matrix-core interpolation (level l+1 -> l) and anterpolation (l -> l+1) for
// complex-float patterns with nc % 8 == 0; false when the level is not covered.
// Lp: the parent level, Lc: the child level.  shiftT: Lp.shiftT or
// Lp.dshiftT; zg: Lp.zg or Lp.dzg.
// sw: a sweep batch (nc = 4 sw.n; shiftT / zg then hold the tables of all
// wavenumbers, sw.stride apart), or nullptr.
bool mf_interp(const LevelD<float>& Lp, const LevelD<float>& Lc, const float2* Sc, float2* Sp, int nc, int ldp,
               int accum, const void* shiftT, hipStream_t s, const SweepSlots* sw = nullptr);
bool mf_anterp(const LevelD<float>& Lp, const LevelD<float>& Lc, const float2* Gp, float2* Gc, int nc, int ldp,
               int add, const void* zg, hipStream_t s, const SweepSlots* sw = nullptr);
// Matrix-core leaf aggregation / disaggregation (complex float, nc % 8 == 0);
// false when not covered (disaggregation: boxes of more than 64 unknowns).
// ncv (< 0: nc): only the first ncv columns are read from x / G and written
// to S / y (the rest of the column tiles count as zero); ldyi (< 0: nc): the
// row stride of the near-field result yi.
// st, nslot: a sweep's slots in one launch (aggregation: t0 = V, offsets
// in = xi, out = S; disaggregation: t0 = V, t1 = qwc, in = G, aux = yi,
// out = y; element offsets in floats).
bool mf_aggregate(const void* V, const float2* xi, int ldx, float2* S, int ldS, const int32_t* box_start, int nbox,
                  int K, int nc, hipStream_t s, int ncv = -1, const SlotTabs* st = nullptr, int nslot = 1);
bool mf_disagg(const void* V, const float2* G, int ldp, const float* qwc, const float2* yi, const int32_t* box_start,
               int nbox, int max_box, const int32_t* perm, int K, int nc, float2* y, int64_t ld, int conj,
               hipStream_t s, int ncv = -1, int ldyi = -1, const SlotTabs* st = nullptr, int nslot = 1);
// Near-field product on the FP64 matrix cores (x, y complex R; nc % 8 == 0,
// nc <= 64, leaf boxes of at most 64 unknowns); mode 0 Z, 1 Re Z self box, 2 Im Z.
// (st, nslot: a sweep's slots in one launch, t0 = near-field values, in /
// out = xi / yi in elements of R)
template <typename R>
bool mf_near(const int64_t* row_ptr, const int32_t* box_start, const int32_t* bcol_ptr, const int32_t* bcol,
             const int32_t* self_off, const double2* Zn, const void* xi, void* yi, int nleaf, int max_box,
             int max_cols_box, int nc, int mode, hipStream_t s, const SlotTabs* st = nullptr, int nslot = 1);
// the same on FP32 near-field values and FP32 matrix cores (complex float x, y)
bool mf_near32(const int64_t* row_ptr, const int32_t* box_start, const int32_t* bcol_ptr, const int32_t* bcol,
               const int32_t* self_off, const float2* Zn, const float2* xi, float2* yi, int nleaf,
               int max_cols_box, int nc, int mode, hipStream_t s);
// Time the matrix-core interpolation/anterpolation variants of every level on
// the workspace at nc columns and keep the fastest; returns the choices (JSON).
std::string mf_autotune(PrecD<float>& pd, int lf, const std::vector<void*>& S, const std::vector<void*>& G, int nc,
                        hipStream_t s);
// Time the FP32 batched translation kernels of every level at nc columns on
// the workspace and keep the fastest; returns JSON array entries.
std::string m2l_autotune(Dev& d, const Plan& P, const std::vector<void*>& S, const std::vector<void*>& G, int nc,
                         hipStream_t s);
// whether mf_anterp takes the anterpolation from level Lp for nc columns
bool mf_covers(const LevelD<float>& Lp, int nc, bool sweep = false);
// whether mf_interp takes the interpolation into level Lp (sweep batch: nc = 4 slots)
bool mf_interp_covers(const LevelD<float>& Lp, const LevelD<float>& Lc, int nc, bool sweep);

void blas_to_c64(const double2* x, float2* y, int64_t N, hipStream_t s);   // complex double -> float
void dev_build(Dev& d, const Plan& P, hipStream_t s);
void dev_free(Dev& d);

// Workspace of one apply: the radiation (S) and incoming (G) patterns of
// levels 2..lf, [box][component][direction][column] with column stride ldp
// (nc, or 2 nc for the dZ/dk pass), and the permuted input / near-field
// output, N x nc.  Levels are at most 20 (the plan's limit).
constexpr int kMaxLevels = 20;
struct Work {
  void* S[kMaxLevels] = {};
  void* G[kMaxLevels] = {};
  void* xi = nullptr;
  void* yi = nullptr;
};
// bytes of each part of the workspace for nc columns (fp64: complex double
// patterns; op 4 doubles the patterns); sizes[l] for S[l] (= G[l]),
// sizes[0] for xi (= yi).  Returns the total of all parts, each rounded up to
// 256 bytes.
size_t work_bytes(const Plan& P, int op, int nc, bool fp64, size_t sizes[kMaxLevels]);
// op: 0 Z, 1 R, 2 X, 3 Z^H, 4 dZ/dk
void dev_apply(Dev& d, const Plan& P, int op, const void* x, void* y, int64_t ld, int nc, bool fp64,
               hipStream_t s);
// the same on a caller-provided workspace (no allocation, no stage timing)
void dev_apply_ws(Dev& d, const Plan& P, int op, const void* x, void* y, int64_t ld, int nc, bool fp64,
                  const Work& w, hipStream_t s);
// one pass over a wavenumber-sweep batch (FP32, op 0 Z or 3 Z^H; dk, Pk
// indexed by wavenumber), see cm_apply.hip; sweep_covers: whether the
// handle's sweep tables and the matrix-core kernels cover nc columns
void dev_apply_sweep(Dev& d0, const Plan& P0, Dev* const* dk, const Plan* const* Pk, const SweepSlots& sw, int op,
                     const void* x, void* y, int64_t ld, hipStream_t s);
bool sweep_covers(const Dev& d0, const Plan& P0, int nc);
// SAI of the near field of tau R + i X: tau = 1 is Z_near (slot 0); any
// other tau goes to slot 1, tau = 0 meaning the real matrix X_near
void dev_sai_build(Dev& d, const Plan& P, double e1, double e2, double e3, double tau, hipStream_t s);
inline int sai_slot(double tau) { return tau == 1.0 ? 0 : 1; }
void dev_sai_apply(Dev& d, const Plan& P, const void* x, void* y, int64_t ld, int nc, bool fp64, int slot,
                   hipStream_t s);

}  // namespace cm

// Device state of a device-resident GMRES cycle (k_gmres_step).
struct GmState {
  int need2;       // the current column needs the second Gram-Schmidt pass
  int stop;        // breakdown: the Krylov space is invariant
  int nvalid;      // columns formed in this cycle
  int pad;
  double inv_hn;   // 1 / ||w|| of the last column (0 on breakdown)
  double res;      // |g[j+1]|: the residual norm estimate after the last column
};

// gather / scatter of up to 64 columns (by index) of an N x ld complex array
namespace cm {
// Real sparse matrices of the Calderon preconditioner, CSR by rows (public
// unknown indices): on the host while built, on the device for the products.
struct CsrHost {
  int64_t rows = 0;
  std::vector<int64_t> ptr;
  std::vector<int32_t> col;
  std::vector<double> val;
};
struct CsrD {
  int64_t rows = 0, nnz = 0;
  int64_t* ptr = nullptr;
  int32_t* col = nullptr;
  double* val = nullptr;
};
// y = M x for complex double x, y (one column)
void blas_csr_real(const CsrD& M, const double2* x, double2* y, hipStream_t s);

// Calderon multiplicative preconditioner of a handle (eqs. (25)-(27)): the
// MLFMA handle of the barycentric refinement, the BC functions' coefficients
// B (N x Nr) on its RWG functions and their transpose, and the mixed Gram
// matrix G (N x N).
struct CmpD {
  cm_handle* ref = nullptr;
  int64_t Nr = 0;
  CsrD B, Bt, G;          // device copies (empty on a host-only handle)
  CsrHost hB, hG;         // host copies (cm_cmp_export)
};
// the barycentric refinement of a closed mesh (vertices 3 x (nv + N + nt),
// triangles 3 x 6 nt); CM_E_MESH for an open surface
void cmp_refine(const Plan& P, std::vector<double>& Vr, std::vector<int32_t>& Fr);
// B, B^T and G from the primal plan and the refined mesh's plan
void cmp_tables(const Plan& P, const Plan& Pr, const std::vector<double>& Vr, const std::vector<int32_t>& Fr,
                CsrHost& B, CsrHost& Bt, CsrHost& G);

struct ColList {
  int n;
  int c[64];
};
// gather the listed columns of x into the staging block xs (N x ws, ws >=
// cols.n; columns past the list and entries -1 are zero) / scatter the first
// cols.n columns of ys (N x ws) back to the listed columns of y (entries -1
// skipped)
void blas_gather_cols(const void* x, int64_t ld, ColList cols, int ws, void* xs, int64_t N, bool fp64,
                      hipStream_t s);
void blas_scatter_cols(const void* ys, int ws, ColList cols, void* y, int64_t ld, int64_t N, bool fp64,
                       hipStream_t s);
}  // namespace cm

// the opaque handle of the C ABI; a wavenumber sweep keeps one handle per
// further wavenumber in `sub` (sub[i] at k[i + 1]) and column staging buffers
struct cm_handle {
  cm::Plan plan;
  cm::Dev dev;
  bool has_dev = false;
  std::vector<cm_handle*> sub;
  // sweeps (n_k > 1), on every wavenumber's handle: staging blocks N x
  // max_cols complex128 each, and a stream (default priority) with two
  // events so that the wavenumbers' batched applies run concurrently
  void *xs = nullptr, *ys = nullptr;
  hipStream_t ks = nullptr;
  hipEvent_t ks_in = nullptr, ks_out = nullptr;
  cm::CmpD* cmp = nullptr;   // Calderon preconditioner (cm_cmp_build), null when not built
};
