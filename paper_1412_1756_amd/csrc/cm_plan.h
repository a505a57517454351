// Host-side plan of the MLFMA: RWG table, octree, interaction lists, angular
// sampling, translators, interpolation and shift tables.  Pure C++ (no HIP).
#pragma once

#include <complex>
#include <cstdint>
#include <stdexcept>
#include <string>
#include <vector>

namespace cm {

using cplx = std::complex<double>;

struct Error : std::runtime_error {
  int code;
  Error(int c, const std::string& m) : std::runtime_error(m), code(c) {}
};

// RWG basis functions (eq. (4)), public order: interior edges sorted by
// (smaller vertex, larger vertex); T+ = lower-numbered triangle.
struct Rwg {
  int64_t N = 0;
  std::vector<int32_t> edge;   // 2N
  std::vector<int32_t> tri;    // 2N: T+, T-
  std::vector<int32_t> loc;    // 2N: local vertex (0..2) of T+/T- opposite the edge
  std::vector<double> len;     // N
};

// One octree level.  Boxes are the occupied cubes of side a, Morton-sorted.
struct Level {
  int l = 0;
  double a = 0;
  int L = 0, nt = 0, np = 0, K = 0;          // truncation and sampling (nt x np)
  int Lt = 0;                                 // translator truncation (L, or less in a shared-sampling sweep)
  std::vector<double> theta, wtheta;          // nt Gauss-Legendre nodes (theta ascending)
  int nbox = 0;
  std::vector<uint64_t> code;
  std::vector<int32_t> ijk;                   // 3 nbox integer box coordinates
  std::vector<int32_t> parent;                // index at level l-1
  std::vector<int32_t> child_ptr;             // nbox+1, range of children at level l+1
  // translation lists (receiver-major CSR): source box and offset id
  std::vector<int32_t> far_ptr, far_src, far_off;     // Z and X
  std::vector<int32_t> farR_ptr, farR_src, farR_off;  // R (leaf level adds neighbours)
  // receiver tiles of kTile consecutive boxes: union of their sources and, per
  // (tile, source), the compact translator index for each receiver (-1: none)
  std::vector<int32_t> tile_ptr, tile_src;
  std::vector<int32_t> tile_off;            // int32: read with scalar loads in the kernel
  std::vector<int32_t> tileR_ptr, tileR_src;
  std::vector<int32_t> tileR_off;
  // the same for tiles of kTile64 boxes (the shared-source translation of
  // batched FP32 applies; on a surface mesh a 64-box tile loads each source
  // for about 12 receivers, a 16-box tile for about 6)
  std::vector<int32_t> tile64_ptr, tile64_src, tile64_off;
  std::vector<int32_t> tileR64_ptr, tileR64_src, tileR64_off;
  std::vector<int32_t> off_compact;                   // kNoff -> compact id (-1 unused)
  int n_off_used = 0;
};

constexpr int kTile = 16;
constexpr int kTile64 = 64;

// Local Lagrange interpolation from level c = l+1 (child) to level l (parent),
// separable: theta first (with reflection over the poles), then phi.
struct Interp {
  int p = 0;
  int ntc = 0, npc = 0, ntp = 0, npp = 0;
  std::vector<int32_t> th_idx;  std::vector<int32_t> th_ref; std::vector<double> th_w;   // ntp*p
  std::vector<int32_t> ph_idx;  std::vector<double> ph_w;                                // npp*p
  // gather form of the weighted transposes (anterpolation), CSR over child index
  std::vector<int32_t> tht_ptr, tht_idx, tht_ref; std::vector<double> tht_w;
  std::vector<int32_t> pht_ptr, pht_idx; std::vector<double> pht_w;
};

// Operand tables of the matrix-core (16x16x4 MFMA) interpolation kernels for
// one level pair.  A block of S = 2*S2 "slots" holds a set U of phi indices
// and U + np/2 (its pole-reflection partners); the slots are the M rows of
// the phi step.  K steps gather the inputs a row block actually needs, four
// per step (lane group g = lane/16 holds input key[k*4+g]); the A operand of
// step k for lane l = 16 g + r is the weight of input key[k*4+g] in output row r.
struct MfTab {
  bool ok = false;
  int NT = 0, S2 = 0;           // theta row tiles of 16; half slot count
  int half = 0;                 // np/2 of the slotted grid
  int nchunk = 0, kmax = 0, ktmax = 0;
  std::vector<int32_t> chunk;   // nchunk x 2: first phi index, slots used per half
  std::vector<int32_t> nk;      // nchunk: phi K steps
  std::vector<int32_t> kidx;    // nchunk x kmax x 4: phi input index
  std::vector<double> kA;       // nchunk x kmax x 64
  std::vector<int32_t> nkt;     // NT: theta K steps per row tile
  std::vector<int32_t> tidx;    // NT x ktmax x 4: theta input row | reflected << 16
  std::vector<double> tA;       // NT x ktmax x 64
};

struct Opts {
  int nlv = 0;
  double d0 = 3.0;
  int p = 6;
  double eta = 376.730313668;
  uint32_t flags = 0;
  int max_cols = 32;
  double k_sampling = 0;   // wavenumber of the truncation rule and sampling (<= 0: k)
};

// Offsets between boxes at one level (each component in -5..5, enough for
// parents within two boxes of each other) are coded as
// (dx+5)*121 + (dy+5)*11 + (dz+5).
constexpr int kOffH = 5, kOffW = 2 * kOffH + 1, kNoff = kOffW * kOffW * kOffW;
inline int off_id(int dx, int dy, int dz) { return ((dx + kOffH) * kOffW + (dy + kOffH)) * kOffW + (dz + kOffH); }

struct Plan {
  Opts opt;
  double k = 0;
  // mesh
  int64_t nv = 0, nt = 0;
  std::vector<double> V;        // 3 nv
  std::vector<int32_t> F;       // 3 nt
  std::vector<double> area, hmax, cent, normal;  // per triangle
  Rwg rwg;
  // tree
  double origin[3] = {0, 0, 0};
  double side = 0;
  int nlv = 0, lf = 0;          // leaf level = nlv - 1
  std::vector<Level> lev;       // 0..lf
  std::vector<Interp> ip;       // ip[l] maps level l+1 -> l, for l = 2..lf-1
  std::vector<MfTab> mf_ip, mf_at;  // matrix-core tables: interpolation into l, anterpolation from l
  // the same with the other slot-chunk width (built for autotuning only; ok = false where none)
  std::vector<MfTab> mf_ip_alt, mf_at_alt;
  std::vector<int32_t> perm;    // internal index -> public RWG index
  std::vector<int32_t> iperm;   // public -> internal
  std::vector<int32_t> box_start;  // leaf box -> first internal unknown (nleaf+1)
  std::vector<int32_t> box_of;     // internal unknown -> leaf box
  // near field (leaf): per box, near boxes sorted; unified column list per box
  std::vector<int32_t> near_ptr, near_box;     // CSR over leaf boxes
  std::vector<int32_t> bcol_ptr, bcol;         // per box: concatenated internal columns
  std::vector<int32_t> self_off;               // per box: offset of own columns in its row
  std::vector<int64_t> row_ptr;                // internal rows -> value offset (N+1)
  int64_t nnz = 0;
  // tables (FP64)
  std::vector<std::vector<cplx>> TZ, TR, TX, dTZ;   // [level][n_off_used*K] (compact offset index)
  std::vector<std::vector<uint8_t>> off_used;        // [level][kNoff]
  std::vector<std::vector<cplx>> shift;             // [level l][8*K_l]: child l+1 -> l
  std::vector<std::vector<cplx>> dshift;            // d shift / dk
  std::vector<std::vector<double>> qw;              // [level][K] quadrature weights
  std::vector<std::vector<double>> dirs;            // [level][9*K]: khat, theta-hat, phi-hat

  void build(const double* xyz, int64_t n_vert, const int32_t* tri, int64_t n_tri, double k,
             const Opts& o);
  void check_coverage() const;
  std::string stats_json() const;
};

// spherical Bessel j_l and Neumann y_l, l = 0..L
void sph_jy(int L, double x, std::vector<double>& j, std::vector<double>& y);
void gauss_legendre(int n, std::vector<double>& x, std::vector<double>& w);

}  // namespace cm
