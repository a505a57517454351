// Matrix-core interpolation and anterpolation between adjacent MLFMA levels
// (section III: local Lagrange interpolation of the radiation patterns in
// theta and phi, with the shift to the parent centre; the anterpolation is the
// weighted transpose).  FP32 patterns, columns in multiples of 8.
//
// Layout of the work: one wave owns 16 real columns (8 complex columns of one
// polarisation component) of one parent box and one slot chunk.  The separable
// stencils become small dense products on v_mfma_f32_16x16x4_f32:
//   phi step   M = 16 slots (a set U of phi indices and its pole partners
//              U + np/2), K = the inputs those slots need, N = 16 columns;
//   theta step M = 16 theta rows, K = the (row, reflected) inputs of the tile,
//              N = 16 columns, once per slot; a reflected input reads the
//              partner slot of the same LDS row (sign folded into the weight).
// The phi-step result of every theta row of the box goes through LDS (one
// region per wave, rows padded by 16 floats so the four lane groups of a
// K step fall into different banks).  The K-step tables hold the weights as
// the per-lane A operand (lane 16 g + r: output row r, input key 4 k + g).
#include <hip/hip_runtime.h>

#include <sstream>
#include <string>
#include <utility>

#include "cm_device.h"

namespace cm {

typedef float f4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ f4 mma(float a, float b, f4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}
// value held by lane ^ 1 (the other half of the complex column)
__device__ __forceinline__ float pair_swap(float v) {
  return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0xB1, 0xF, 0xF, true));
}
// LDS written by some lanes of a wave and then read by others
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// kRG rows of phi-step inputs for K steps [0, nk): rows r0 .. r0+kRG-1 of
// base (clamped to nrows-1), each row at off[k] from its start.
template <int kRG, int kMK>
__device__ __forceinline__ void load_rows(float (&v)[kRG][kMK], const float* base, int r0, int nrows,
                                          int64_t rstride, const unsigned (&off)[kMK], int nk) {
#pragma unroll
  for (int r = 0; r < kRG; ++r) {
    const float* row = base + (int64_t)min(r0 + r, nrows - 1) * rstride;
#pragma unroll
    for (int k2 = 0; k2 < kMK; k2 += 2)
      if (k2 < nk) {
#pragma unroll
        for (int i = 0; i < 2; ++i) v[r][k2 + i] = row[off[k2 + i]];
      }
  }
}

// theta-step tables of the block's row tiles t0 .. t0+NT-1 into LDS (ktmax
// steps each: 4 keys, 64 A values; tiles past the last are zero)
__device__ __forceinline__ void stage_theta_tables(const MfD& T, int t0, int NT, int* tcode, float* tA) {
  const int nv = (T.NT - t0) * T.ktmax;   // valid steps of the group
  for (int e = threadIdx.x; e < NT * T.ktmax * 4; e += blockDim.x)
    tcode[e] = (e / 4 < nv) ? T.tidx[t0 * T.ktmax * 4 + e] : 0;
  for (int e = threadIdx.x; e < NT * T.ktmax * 64; e += blockDim.x)
    tA[e] = (e / 64 < nv) ? T.tA[t0 * T.ktmax * 64 + e] : 0.f;
}

// Interpolation child level -> parent level, summed over the children of a
// parent with the shift phase of each child's octant; parent rows are written
// (or accumulated onto, accum != 0).  Grid: x = parent boxes x slot chunks
// (padded to a multiple of 8, XCD-major order), y = groups of column tiles,
// one per wave (four waves per block, fewer where their LDS rows do not fit),
// z = groups of NT theta row tiles (more than four tiles are split over
// blocks, each redoing the phi step).  The phi-step loads of a child are
// double-buffered in groups of kRG rows and the first group of the next
// child is loaded during the theta step, which touches only LDS.  A column
// tile is eight columns of one component, or in a wavenumber-sweep batch (sw)
// the four columns of one slot in both components (the Lagrange weights and
// the shift phase are the same for both), with the slot's shift table.
template <int NT, int S2, int kMK, int kRG, int kW>
__global__ void __launch_bounds__(256, kW) k_interp_mf(const float* __restrict__ Sc, float* __restrict__ Sp,
                                                   const int32_t* __restrict__ child_ptr,
                                                   const int8_t* __restrict__ octant, MfD T,
                                                   const float2* __restrict__ shiftT, int ntc, int npc, int ntp,
                                                   int npp, int nbox, int nc, int ldp, int accum, SweepSlots sw) {
  constexpr int S = 2 * S2, RS = 16 * S + 16, SB = S < 8 ? S : 8, SH = S * 16 * NT;   // SH: shift entries
  extern __shared__ float lds[];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int b = (blockIdx.x & 7) * (gridDim.x >> 3) + (blockIdx.x >> 3);
  if (b >= nbox * T.nchunk) return;   // whole block
  const int t0 = blockIdx.z * NT;   // first theta row tile of this block
  int* tcode = reinterpret_cast<int*>(lds);
  float* tAl = lds + NT * T.ktmax * 4;
  stage_theta_tables(T, t0, NT, tcode, tAl);
  __syncthreads();
  const int cpt = nc >> 3;
  const int tile = blockIdx.y * (int)(blockDim.x >> 6) + w;
  if (tile >= (sw.on ? sw.n : 2 * cpt)) return;
  float* O = tAl + NT * T.ktmax * 64 + w * (ntc * RS + 2 * SH);
  float2* ShL = reinterpret_cast<float2*>(O + ntc * RS);   // [slot][16 NT] shift of the current child
  const int m = b / T.nchunk, c = b - m * T.nchunk;
  const int g = lane >> 4, n = lane & 15;
  // this lane's component and float offset within a row of that component
  int comp, lcol;
  const float2* shk = shiftT;
  if (sw.on) {
    comp = n >> 3;
    lcol = 8 * tile + (n & 7);
    shk += (int64_t)sw.k[tile] * sw.stride;
  } else {
    comp = tile / cpt;
    lcol = 16 * (tile - comp * cpt) + n;
  }
  const int ld2 = 2 * ldp;
  const int64_t Kc = (int64_t)ntc * npc, Kp = (int64_t)ntp * npp;
  const unsigned coff = (unsigned)comp * (unsigned)(Kc * ld2) + (unsigned)lcol;
  const int u0 = T.chunk[2 * c], h = T.chunk[2 * c + 1];
  const int nk = T.nk[c];
  unsigned uoff[kMK];
  float pa[kMK];
#pragma unroll
  for (int kk = 0; kk < kMK; ++kk) {
    uoff[kk] = 0;
    pa[kk] = 0.f;
    if (kk < nk) {
      uoff[kk] = (unsigned)T.kidx[(c * T.kmax + kk) * 4 + g] * (unsigned)ld2 + coff;
      pa[kk] = T.kA[(c * T.kmax + kk) * 64 + lane];
    }
  }
  f4 acc[NT][S];
#pragma unroll
  for (int t = 0; t < NT; ++t)
#pragma unroll
    for (int s = 0; s < S; ++s) acc[t][s] = f4{0.f, 0.f, 0.f, 0.f};
  const float sg = (n & 1) ? 1.f : -1.f;   // (sx + i sy)(re + i im): re lane -sy*im, im lane +sy*re
  const int64_t rstride = (int64_t)npc * ld2;
  auto child_src = [&](int ch) { return Sc + (int64_t)ch * 2 * Kc * ld2; };
  // phi step of kRG rows from v into LDS rows r0 ..
  auto phi_rows = [&](const float (&v)[kRG][kMK], int r0) {
    f4 d[kRG];
#pragma unroll
    for (int r = 0; r < kRG; ++r) d[r] = f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int k2 = 0; k2 < kMK; k2 += 2)
      if (k2 < nk) {
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
          for (int r = 0; r < kRG; ++r) d[r] = mma(pa[k2 + i], v[r][k2 + i], d[r]);
      }
#pragma unroll
    for (int r = 0; r < kRG; ++r)
      if (r0 + r < ntc) {
#pragma unroll
        for (int j = 0; j < 4; ++j)
          if (4 * g + j < S) O[(r0 + r) * RS + (4 * g + j) * 16 + n] = d[r][j];
      }
  };
  const int ch0 = child_ptr[m], ch1 = child_ptr[m + 1];
  float va[kRG][kMK], vb[kRG][kMK];
  if (ch0 < ch1) load_rows(va, child_src(ch0), 0, ntc, rstride, uoff, nk);
  for (int ch = ch0; ch < ch1; ++ch) {
    const float* src = child_src(ch);
    // this child's shift rows of the chunk's slots (written to LDS after the phi step)
    // table rows hold 16 T.NT values per phi slot; this block's tiles start at 16 t0
    const float4* shg = reinterpret_cast<const float4*>(shk + (size_t)octant[ch] * npp * (16 * T.NT));
    float4 shv[(SH / 2 + 63) / 64];
#pragma unroll
    for (int i = 0; i < (SH / 2 + 63) / 64; ++i) {
      const int e = lane + 64 * i;                  // float4 index: slot e / (8 NT), pair e % (8 NT)
      const int sl = e / (8 * NT), q = e - sl * (8 * NT);
      const int up = (sl % S2) < h ? u0 + (sl % S2) + (sl / S2) * T.half : u0;
      if (e < SH / 2) shv[i] = (t0 + q / 8 < T.NT) ? shg[up * (8 * T.NT) + 8 * t0 + q] : float4{0.f, 0.f, 0.f, 0.f};
    }
    // phi step, double-buffered row groups
    for (int tc0 = 0; tc0 < ntc; tc0 += 2 * kRG) {
      const bool more = tc0 + kRG < ntc;
      if (more) load_rows(vb, src, tc0 + kRG, ntc, rstride, uoff, nk);
      phi_rows(va, tc0);
      if (more) {
        if (tc0 + 2 * kRG < ntc) load_rows(va, src, tc0 + 2 * kRG, ntc, rstride, uoff, nk);
        phi_rows(vb, tc0 + kRG);
      }
    }
#pragma unroll
    for (int i = 0; i < (SH / 2 + 63) / 64; ++i) {
      const int e = lane + 64 * i;
      if (e < SH / 2) reinterpret_cast<float4*>(ShL)[e] = shv[i];
    }
    wave_lds_sync();
    if (ch + 1 < ch1) load_rows(va, child_src(ch + 1), 0, ntc, rstride, uoff, nk);
    // theta step per row tile and slot batch, then shift and accumulate
#pragma unroll
    for (int t = 0; t < NT; ++t) {
      const int nkt = (t0 + t < T.NT) ? T.nkt[t0 + t] : 0;
#pragma unroll
      for (int s0 = 0; s0 < S; s0 += SB) {
        f4 d2[SB];
#pragma unroll
        for (int i = 0; i < SB; ++i) d2[i] = f4{0.f, 0.f, 0.f, 0.f};
        for (int kk = 0; kk < nkt; ++kk) {
          const int code = tcode[(t * T.ktmax + kk) * 4 + g];
          const float a = tAl[(t * T.ktmax + kk) * 64 + lane];
          // reflected inputs read the partner slot s ^ S2 of the same row
          const int rfo = (code >> 16) ? 16 * S2 : 0;
          const float* lo = O + (code & 0xffff) * RS + n + rfo;
          const float* hi = O + (code & 0xffff) * RS + n - rfo;
#pragma unroll
          for (int i = 0; i < SB; ++i) {
            const int s = s0 + i;
            d2[i] = mma(a, (s < S2 ? lo : hi)[s * 16], d2[i]);
          }
        }
#pragma unroll
        for (int i = 0; i < SB; ++i) {
          const int s = s0 + i;
          if ((s % S2) < h) {
            const float4* sp = reinterpret_cast<const float4*>(ShL + s * (16 * NT) + 16 * t + 4 * g);
            const float4 s01 = sp[0], s23 = sp[1];
            const float sx[4] = {s01.x, s01.z, s23.x, s23.z};
            const float sy[4] = {s01.y, s01.w, s23.y, s23.w};
#pragma unroll
            for (int j = 0; j < 4; ++j) {
              const float v = d2[i][j], vp = pair_swap(v);
              acc[t][s][j] = fmaf(sx[j], v, fmaf(sg * sy[j], vp, acc[t][s][j]));
            }
          }
        }
      }
    }
    wave_lds_sync();
  }
  float* dst = Sp + ((int64_t)m * 2 + comp) * Kp * ld2 + lcol;
#pragma unroll
  for (int t = 0; t < NT; ++t)
#pragma unroll
    for (int s = 0; s < S; ++s) {
      if ((s % S2) >= h) continue;
      const int up = u0 + (s % S2) + (s / S2) * T.half;
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int tp = 16 * (t0 + t) + 4 * g + j;
        if (tp < ntp) {
          float* o = dst + ((int64_t)tp * npp + up) * ld2;
          if (accum)
            unsafeAtomicAdd(o, acc[t][s][j]);   // single writer per element: a plain read-add-write
          else
            *o = acc[t][s][j];
        }
      }
    }
}

// Anterpolation parent level -> child level, one child box (and slot chunk
// over the child phi grid, and group of NT child theta row tiles) per block:
// conj(shift) times the parent pattern,
// the transposed phi step (parent phi -> child slots) into LDS, the
// transposed theta step with the child-grid reflection, stored into the child
// rows (add != 0: added onto them).  The block stages the chunk's shift
// values for the child's octant (zg: [chunk][octant][parent theta row][4
// kmax], in K-step key order) and the theta tables in LDS; the parent-row
// loads are double-buffered in groups of kRG rows.
// A sweep batch (sw) maps column tiles to slots as the interpolation does;
// each wave then needs its own slot's phase values: a per-wave LDS copy, or
// where a chunk's table is small (sw.zg_global) reads straight from global
// memory (L1/L2), which saves the copies' LDS and occupancy.
template <int NT, int S2, int kMK, int kRG, int kW>
__global__ void __launch_bounds__(256, kW) k_anterp_mf(const float* __restrict__ Gp, float* __restrict__ Gc,
                                                   const int32_t* __restrict__ parent,
                                                   const int8_t* __restrict__ octant, MfD T,
                                                   const float2* __restrict__ zg, int ntc, int npc, int ntp,
                                                   int npp, int nchild, int nc, int ldp, int add, SweepSlots sw) {
  constexpr int S = 2 * S2, RS = 16 * S + 16;
  extern __shared__ float lds[];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int b = (blockIdx.x & 7) * (gridDim.x >> 3) + (blockIdx.x >> 3);
  if (b >= nchild * T.nchunk) return;   // whole block
  const int ch = b / T.nchunk, c = b - ch * T.nchunk;
  const int kz = 4 * T.kmax;
  const int t0 = blockIdx.z * NT;   // first child theta row tile of this block
  int* tcode = reinterpret_cast<int*>(lds);
  float* tAl = lds + NT * T.ktmax * 4;
  float2* Z0 = reinterpret_cast<float2*>(tAl + NT * T.ktmax * 64);
  const bool zl = sw.on && !sw.zg_global;                          // per-wave LDS copies
  const int nz = sw.on ? (zl ? (int)(blockDim.x >> 6) : 0) : 1;   // phase tables in LDS
  stage_theta_tables(T, t0, NT, tcode, tAl);
  if (!sw.on) {
    const float4* zs = reinterpret_cast<const float4*>(zg + ((size_t)c * 8 + octant[ch]) * ntp * kz);
    float4* zd = reinterpret_cast<float4*>(Z0);
    for (int e = threadIdx.x; e < ntp * kz / 2; e += blockDim.x) zd[e] = zs[e];
  }
  __syncthreads();
  const int cpt = nc >> 3;
  const int tile = blockIdx.y * (int)(blockDim.x >> 6) + w;
  if (tile >= (sw.on ? sw.n : 2 * cpt)) return;
  const float2* zslot =
      sw.on ? zg + (int64_t)sw.k[tile] * sw.stride + ((size_t)c * 8 + octant[ch]) * ntp * kz : zg;
  if (zl) {
    const float4* zs = reinterpret_cast<const float4*>(zslot);
    float4* zd = reinterpret_cast<float4*>(Z0 + (size_t)w * ntp * kz);
    for (int e = lane; e < ntp * kz / 2; e += 64) zd[e] = zs[e];
    wave_lds_sync();
  }
  float* O = reinterpret_cast<float*>(Z0 + (size_t)nz * ntp * kz) + w * ntp * RS;
  const int m = parent[ch];
  const int g = lane >> 4, n = lane & 15;
  int comp, lcol;   // this lane's component and float offset within a row of that component
  if (sw.on) {
    comp = n >> 3;
    lcol = 8 * tile + (n & 7);
  } else {
    comp = tile / cpt;
    lcol = 16 * (tile - comp * cpt) + n;
  }
  const int ld2 = 2 * ldp;
  const int64_t Kc = (int64_t)ntc * npc, Kp = (int64_t)ntp * npp;
  const unsigned coff = (unsigned)comp * (unsigned)(Kp * ld2) + (unsigned)lcol;
  const int u0 = T.chunk[2 * c], h = T.chunk[2 * c + 1];
  const int nk = T.nk[c];
  unsigned poff[kMK];
  float pa[kMK];
#pragma unroll
  for (int kk = 0; kk < kMK; ++kk) {
    poff[kk] = 0;
    pa[kk] = 0.f;
    if (kk < nk) {
      poff[kk] = (unsigned)T.kidx[(c * T.kmax + kk) * 4 + g] * (unsigned)ld2 + coff;
      pa[kk] = T.kA[(c * T.kmax + kk) * 64 + lane];
    }
  }
  const float* par = Gp + (int64_t)m * 2 * Kp * ld2;
  const int64_t rstride = (int64_t)npp * ld2;
  const float sg = (n & 1) ? -1.f : 1.f;   // (sx - i sy)(re + i im): re lane +sy*im, im lane -sy*re
  auto phiT_rows = [&](const float2* Z, const float (&v)[kRG][kMK], int r0) {
    f4 d[kRG];
#pragma unroll
    for (int r = 0; r < kRG; ++r) d[r] = f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int k2 = 0; k2 < kMK; k2 += 2)
      if (k2 < nk) {
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
          for (int r = 0; r < kRG; ++r) {
            const float2 z = Z[min(r0 + r, ntp - 1) * kz + (k2 + i) * 4 + g];
            const float x = v[r][k2 + i];
            d[r] = mma(pa[k2 + i], fmaf(z.x, x, sg * z.y * pair_swap(x)), d[r]);
          }
      }
#pragma unroll
    for (int r = 0; r < kRG; ++r)
      if (r0 + r < ntp) {
#pragma unroll
        for (int j = 0; j < 4; ++j)
          if (4 * g + j < S) O[(r0 + r) * RS + (4 * g + j) * 16 + n] = d[r][j];
      }
  };
  // transposed phi step over the parent rows, double-buffered row groups;
  // the phase values come from the block's LDS copy, or in a sweep batch
  // (one wavenumber per wave) straight from the slot's table (L1/L2)
  float va[kRG][kMK], vb[kRG][kMK];
  auto phi_pass = [&](const float2* Z) {
    load_rows(va, par, 0, ntp, rstride, poff, nk);
    for (int tp0 = 0; tp0 < ntp; tp0 += 2 * kRG) {
      const bool more = tp0 + kRG < ntp;
      if (more) load_rows(vb, par, tp0 + kRG, ntp, rstride, poff, nk);
      phiT_rows(Z, va, tp0);
      if (more) {
        if (tp0 + 2 * kRG < ntp) load_rows(va, par, tp0 + 2 * kRG, ntp, rstride, poff, nk);
        phiT_rows(Z, vb, tp0 + kRG);
      }
    }
  };
  if (sw.on && !zl)
    phi_pass(zslot);
  else
    phi_pass(zl ? Z0 + (size_t)w * ntp * kz : Z0);
  wave_lds_sync();
  // transposed theta step
  f4 acc[NT][S];
#pragma unroll
  for (int t = 0; t < NT; ++t)
#pragma unroll
    for (int s = 0; s < S; ++s) acc[t][s] = f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int t = 0; t < NT; ++t) {
    const int nkt = (t0 + t < T.NT) ? T.nkt[t0 + t] : 0;
    for (int kk = 0; kk < nkt; ++kk) {
      const int code = tcode[(t * T.ktmax + kk) * 4 + g];
      const float a = tAl[(t * T.ktmax + kk) * 64 + lane];
      const int rfo = (code >> 16) ? 16 * S2 : 0;
      const float* lo = O + (code & 0xffff) * RS + n + rfo;
      const float* hi = O + (code & 0xffff) * RS + n - rfo;
#pragma unroll
      for (int s = 0; s < S; ++s) acc[t][s] = mma(a, (s < S2 ? lo : hi)[s * 16], acc[t][s]);
    }
  }
  float* dst = Gc + ((int64_t)ch * 2 + comp) * Kc * ld2;
  const unsigned rstep = (unsigned)npc * (unsigned)ld2;
  const unsigned loff = 4u * g * rstep + (unsigned)lcol;
#pragma unroll
  for (int t = 0; t < NT; ++t)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      if (16 * (t0 + t) + 4 * g + j >= ntc) continue;
      const unsigned ro = loff + (unsigned)(16 * (t0 + t) + j) * rstep;
#pragma unroll
      for (int s = 0; s < S; ++s) {
        if ((s % S2) >= h) continue;
        const unsigned o = ro + (unsigned)(u0 + (s % S2) + (s / S2) * T.half) * (unsigned)ld2;
        if (add)
          unsafeAtomicAdd(dst + o, acc[t][s][j]);   // single writer per element: a plain read-add-write
        else
          dst[o] = acc[t][s][j];
      }
    }
}

// Leaf aggregation S_box[row][c] = sum_i V_i[row] x_i[c] over the unknowns i
// of a leaf box (rows: component x direction, 2K of them): a complex product
// on the matrix cores as two real MFMAs, C += Re(A) B + Im(A) B~, where B~ is
// B with each (re, im) column pair swapped and the new re negated.  One wave
// owns MTW row tiles of 16 and NTL column tiles of 16 reals; K runs over the
// box's unknowns four at a time.  Grid: waves box-major, 256 threads.
template <int MTW, int NTL>
__global__ void __launch_bounds__(256) k_aggregate_mf(const float2* __restrict__ V, const float* __restrict__ xi,
                                                      int ldx, float* __restrict__ S, int ldS,
                                                      const int32_t* __restrict__ box_start, int nbox, int K2, int nc,
                                                      int wpb, int cvf, SlotTabs st) {
  const int z = (int)blockIdx.x % st.n, bx = (int)blockIdx.x / st.n;
  if (z) {
    V = (const float2*)st.t0[z];
    xi += z * st.in_off;
    S += z * st.out_off;
  }
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int g = lane >> 4, r = lane & 15;
  const int wid = bx * 4 + w;
  const int box = wid / wpb, m0 = (wid - box * wpb) * MTW * 16;
  if (box >= nbox || m0 >= K2) return;
  const int i0 = box_start[box], i1 = box_start[box + 1];
  const int ntiles = nc >> 3;
  const float sg = (r & 1) ? 1.f : -1.f;
  for (int nt0 = 0; nt0 < ntiles; nt0 += NTL) {
    f4 acc[MTW][NTL];
#pragma unroll
    for (int mt = 0; mt < MTW; ++mt)
#pragma unroll
      for (int nt = 0; nt < NTL; ++nt) acc[mt][nt] = f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll 2
    for (int i = i0; i < i1; i += 4) {
      const int ii = i + g;
      const bool ok = ii < i1;
      float2 a[MTW];
      float bq[NTL];
#pragma unroll
      for (int mt = 0; mt < MTW; ++mt) {
        const int row = m0 + 16 * mt + r;
        a[mt] = (ok && row < K2) ? V[(int64_t)ii * K2 + row] : make_float2(0.f, 0.f);
      }
#pragma unroll
      for (int nt = 0; nt < NTL; ++nt)
        bq[nt] = (ok && nt0 + nt < ntiles && 16 * (nt0 + nt) + r < cvf) ? xi[(int64_t)ii * 2 * ldx + 16 * (nt0 + nt) + r]
                                                                         : 0.f;
#pragma unroll
      for (int nt = 0; nt < NTL; ++nt) {
        const float bs = sg * pair_swap(bq[nt]);
#pragma unroll
        for (int mt = 0; mt < MTW; ++mt) {
          acc[mt][nt] = mma(a[mt].x, bq[nt], acc[mt][nt]);
          acc[mt][nt] = mma(a[mt].y, bs, acc[mt][nt]);
        }
      }
    }
#pragma unroll
    for (int mt = 0; mt < MTW; ++mt)
#pragma unroll
      for (int nt = 0; nt < NTL; ++nt) {
        if (nt0 + nt >= ntiles) continue;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const int row = m0 + 16 * mt + 4 * g + j;
          if (row < K2 && 16 * (nt0 + nt) + r < cvf)
            S[((int64_t)box * K2 + row) * 2 * ldS + 16 * (nt0 + nt) + r] = acc[mt][nt][j];
        }
      }
  }
}

// Leaf disaggregation y_i = yi_i + sum_row w_q conj(V_i[row]) G_box[row] (the
// far-field part of every unknown of a box), optionally conjugated, written
// at perm[i] (internal position i without perm).  One block per leaf box: its
// four waves split the 2K rows, each accumulating all the box's unknowns (MTU
// tiles of 16) times NTL column tiles on the matrix cores in one pass over
// the box's leaf patterns; the partial sums meet in LDS, two column tiles at
// a time (so the reduction buffer stays at 4 waves x MTU x 2 x 4 floats per
// lane).
template <int MTU, int NTL>
__global__ void __launch_bounds__(256) k_disagg_mf(const float2* __restrict__ V, const float* __restrict__ G, int ldp,
                                                   const float* __restrict__ qwc, const float* __restrict__ yi,
                                                   const int32_t* __restrict__ box_start,
                                                   const int32_t* __restrict__ perm, int K, int nc,
                                                   float* __restrict__ y, int64_t ld, int conj_out, int cvf,
                                                   int ldyi, SlotTabs st) {
  const int z = (int)blockIdx.x % st.n;
  if (z) {
    V = (const float2*)st.t0[z];
    qwc = (const float*)st.t1[z];
    G += z * st.in_off;
    yi += z * st.aux_off;
    y += z * st.out_off;
  }
  constexpr int NR = MTU * 2 * 4;     // floats per lane of one reduction round (two column tiles)
  extern __shared__ float red[];      // [4 waves][NR][64]
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int g = lane >> 4, r = lane & 15;
  const int box = (int)blockIdx.x / st.n;
  const int i0 = box_start[box], i1 = box_start[box + 1];
  const int K2 = 2 * K, nks = (K2 + 3) / 4;
  const int ks0 = w * nks / 4, ks1 = (w + 1) * nks / 4;
  const int ntiles = nc >> 3;
  const float sg = (r & 1) ? 1.f : -1.f;
  const float* gb = G + (int64_t)box * K2 * 2 * ldp;
  for (int nt0 = 0; nt0 < ntiles; nt0 += NTL) {
    f4 acc[MTU][NTL];
#pragma unroll
    for (int mt = 0; mt < MTU; ++mt)
#pragma unroll
      for (int nt = 0; nt < NTL; ++nt) acc[mt][nt] = f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll 2
    for (int ks = ks0; ks < ks1; ++ks) {
      const int row = 4 * ks + g;
      const bool rok = row < K2;
      const float wq = rok ? qwc[row < K ? row : row - K] : 0.f;
      float2 a[MTU];
      float bq[NTL];
#pragma unroll
      for (int mt = 0; mt < MTU; ++mt) {
        const int i = i0 + 16 * mt + r;
        const float2 v = (rok && i < i1) ? V[(int64_t)i * K2 + row] : make_float2(0.f, 0.f);
        a[mt] = make_float2(wq * v.x, -wq * v.y);   // w_q conj(V)
      }
#pragma unroll
      for (int nt = 0; nt < NTL; ++nt)
        bq[nt] = (rok && nt0 + nt < ntiles && 16 * (nt0 + nt) + r < cvf)
                     ? gb[(int64_t)row * 2 * ldp + 16 * (nt0 + nt) + r]
                     : 0.f;
#pragma unroll
      for (int nt = 0; nt < NTL; ++nt) {
        const float bs = sg * pair_swap(bq[nt]);
#pragma unroll
        for (int mt = 0; mt < MTU; ++mt)
          if (16 * mt < i1 - i0) {   // unknown tiles past the box's last unknown are zero: skipped
            acc[mt][nt] = mma(a[mt].x, bq[nt], acc[mt][nt]);
            acc[mt][nt] = mma(a[mt].y, bs, acc[mt][nt]);
          }
      }
    }
#pragma unroll
    for (int np = 0; np < NTL; np += 2) {
      __syncthreads();   // the previous round's reads of red are done
#pragma unroll
      for (int mt = 0; mt < MTU; ++mt)
#pragma unroll
        for (int h = 0; h < 2; ++h)
#pragma unroll
          for (int j = 0; j < 4; ++j)
            red[(w * NR + (mt * 2 + h) * 4 + j) * 64 + lane] = (np + h < NTL) ? acc[mt][np + h][j] : 0.f;
      __syncthreads();
      for (int e = threadIdx.x; e < NR * 64; e += 256) {
        const int v = e >> 6, l = e & 63;
        const int j = v & 3, h = (v >> 2) & 1, mt = (v >> 2) >> 1;
        const int nt = np + h;
        const int i = i0 + 16 * mt + 4 * (l >> 4) + j;
        const int colf = 16 * (nt0 + nt) + (l & 15);
        if (i >= i1 || nt >= NTL || nt0 + nt >= ntiles || colf >= cvf) continue;
        float sum = red[e] + red[NR * 64 + e] + red[2 * NR * 64 + e] + red[3 * NR * 64 + e];
        sum += yi[(int64_t)i * 2 * ldyi + colf];
        if (conj_out && (colf & 1)) sum = -sum;
        y[(int64_t)(perm ? perm[i] : i) * 2 * ld + colf] = sum;
      }
    }
  }
}

bool mf_aggregate(const void* V, const float2* xi, int ldx, float2* S, int ldS, const int32_t* box_start, int nbox,
                  int K, int nc, hipStream_t s, int ncv, const SlotTabs* st, int nslot) {
  if (nc % 8 != 0 || nslot < 1 || nslot > kMaxSlots || (nslot > 1 && !st)) return false;
  if (ncv < 0) ncv = nc;
  SlotTabs sv = st ? *st : SlotTabs();
  sv.n = nslot;
  constexpr int MTW = 3;
  const int K2 = 2 * K;
  const int wpb = (K2 + 16 * MTW - 1) / (16 * MTW);
  const int64_t waves = (int64_t)nbox * wpb;
  // four column tiles per pass over the leaf patterns, one for a single tile
  // (no matrix-core steps on empty tiles)
  const dim3 grid((unsigned)((waves + 3) / 4 * nslot));
  if (nc <= 8)
    hipLaunchKernelGGL((k_aggregate_mf<MTW, 1>), grid, dim3(256), 0, s, (const float2*)V, (const float*)xi, ldx,
                       (float*)S, ldS, box_start, nbox, K2, nc, wpb, 2 * ncv, sv);
  else
    hipLaunchKernelGGL((k_aggregate_mf<MTW, 4>), grid, dim3(256), 0, s, (const float2*)V, (const float*)xi, ldx,
                       (float*)S, ldS, box_start, nbox, K2, nc, wpb, 2 * ncv, sv);
  return true;
}

bool mf_disagg(const void* V, const float2* G, int ldp, const float* qwc, const float2* yi, const int32_t* box_start,
               int nbox, int max_box, const int32_t* perm, int K, int nc, float2* y, int64_t ld, int conj,
               hipStream_t s, int ncv, int ldyi, const SlotTabs* st, int nslot) {
  if (nc % 8 != 0 || max_box > 64 || nslot < 1 || nslot > kMaxSlots || (nslot > 1 && !st)) return false;
  if (ncv < 0) ncv = nc;
  if (ldyi < 0) ldyi = nc;
  SlotTabs sv = st ? *st : SlotTabs();
  sv.n = nslot;
  // four column tiles per pass over the leaf patterns (each read once for
  // 32 columns), reduced two tiles at a time: the LDS buffer (4 waves x MTU
  // x 2 x 4 floats per lane) leaves room for four blocks per CU
  // (one column tile per pass for a single tile)
#define CM_DIS(MTU, NTL)                                                                                       \
  hipLaunchKernelGGL((k_disagg_mf<MTU, NTL>), dim3(nbox * nslot), dim3(256), (size_t)4 * MTU * 2 * 4 * 64 * 4,   \
                     s, (const float2*)V, (const float*)G, ldp, qwc, (const float*)yi, box_start, perm, K, nc,    \
                     (float*)y, ld, conj, 2 * ncv, ldyi, sv)
#define CM_DIS_N(MTU)  \
  if (nc <= 8)         \
    CM_DIS(MTU, 1);    \
  else                 \
    CM_DIS(MTU, 4);
  if (max_box <= 16) {
    CM_DIS_N(1)
  } else if (max_box <= 32) {
    CM_DIS_N(2)
  } else if (max_box <= 48) {
    CM_DIS_N(3)
  } else {
    CM_DIS_N(4)
  }
#undef CM_DIS_N
#undef CM_DIS
  return true;
}

typedef double d4 __attribute__((ext_vector_type(4)));

// v_mfma_f64_16x16x4f64: A and B lanes as in the FP32 form (lane 16 k + m,
// lane 16 k + n); result register j of lane 16 g + n holds row 4 j + g.
__device__ __forceinline__ d4 mma64(double a, double b, d4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ double pair_swap64(double v) {
  const long long u = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_mov_dpp((int)(u & 0xffffffffll), 0xB1, 0xF, 0xF, true);
  const int hi = __builtin_amdgcn_mov_dpp((int)(u >> 32), 0xB1, 0xF, 0xF, true);
  return __longlong_as_double(((long long)(unsigned)hi << 32) | (unsigned)lo);
}

// Near-field product y_i = sum_t Z_near[i, t] x[col_t] (mode 1: Re Z_near on
// the box's own columns, mode 2: Im Z_near) on the FP64 matrix cores.  Each
// leaf box takes (2 / MT) x (4 / NW) waves: a wave owns MT of every two row
// tiles of 16 (rows 32 k + 16 h .. for its half h when MT = 1) times NW of
// the four column tiles of 16 reals (x rows gathered from memory and
// converted to FP64), so each near-field value is loaded by 4 / NW waves.
// Complex steps as in the leaf aggregation: C += Re(A) B + Im(A) B~.
// Columns beyond 32 take further blocks (grid y); nc <= 64.
template <typename R, int MODE, int MT, int NW>
__global__ void __launch_bounds__(256) k_near_mf(const int64_t* __restrict__ row_ptr,
                                                 const int32_t* __restrict__ box_start,
                                                 const int32_t* __restrict__ bcol_ptr,
                                                 const int32_t* __restrict__ bcol,
                                                 const int32_t* __restrict__ self_off, const double2* __restrict__ Zn,
                                                 const R* __restrict__ xi, R* __restrict__ yi, int nleaf, int nc,
                                                 int xcap, SlotTabs st) {
  if (blockIdx.z) {
    Zn = (const double2*)st.t0[blockIdx.z];
    xi += blockIdx.z * st.in_off;
    yi += blockIdx.z * st.out_off;
  }
  extern __shared__ int32_t xoff_all[];   // per wave: the box's column rows as offsets into x (floats)
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int g = lane >> 4, r = lane & 15;
  constexpr int WM = 2 / MT, WB = WM * (4 / NW);   // waves per box (row halves x column groups)
  const int b = blockIdx.x * (4 / WB) + w / WB;
  const int mh = (MT == 1) ? 16 * (w % WM) : 0;    // first row of this wave's tile in each 32
  // first column tile of this wave (grid y: groups of four column tiles, 32 columns)
  const int n0 = 4 * (int)blockIdx.y + NW * ((w % WB) / WM);
  if (b >= nleaf) return;
  int32_t* xoff = xoff_all + w * xcap;
  const int r0 = box_start[b], nb = box_start[b + 1] - r0;
  const int32_t* cols = bcol + bcol_ptr[b];
  int t0 = 0, t1 = bcol_ptr[b + 1] - bcol_ptr[b];
  if (MODE == 1) {
    t0 = self_off[b];
    t1 = t0 + nb;
  }
  const int nc2 = 2 * nc, ntiles = nc >> 3;
  // K steps of four columns in groups of two, the same count on every lane
  const int ngrp = (t1 - t0 + 7) / 8;
  for (int e = lane; e < 8 * ngrp; e += 64) xoff[e] = (t0 + e < t1) ? cols[t0 + e] * nc2 : -1;
  wave_lds_sync();
  const int tlast = t1 - t0 - 1;
  const double sg = (r & 1) ? 1.0 : -1.0;
  for (int m0 = mh; m0 < nb; m0 += 32) {
    // this lane's A-operand rows (one per row tile); every load is in bounds
    // (padding reads a valid entry and is zeroed afterwards)
    bool iok[MT];
    const double2* zrow[MT];
#pragma unroll
    for (int mt = 0; mt < MT; ++mt) {
      iok[mt] = m0 + 16 * mt + r < nb;
      zrow[mt] = Zn + row_ptr[r0 + (iok[mt] ? m0 + 16 * mt + r : 0)] + t0;
    }
    d4 acc[MT][NW];
#pragma unroll
    for (int mt = 0; mt < MT; ++mt)
#pragma unroll
      for (int nt = 0; nt < NW; ++nt) acc[mt][nt] = d4{0.0, 0.0, 0.0, 0.0};
    auto load = [&](int gi, double2 (&z)[2][MT], R (&xv)[2][NW]) {
#pragma unroll
      for (int u = 0; u < 2; ++u) {
        const int tt = 8 * gi + 4 * u + g;
        const int xo = xoff[tt];
#pragma unroll
        for (int mt = 0; mt < MT; ++mt) z[u][mt] = zrow[mt][min(tt, tlast)];
#pragma unroll
        for (int nt = 0; nt < NW; ++nt)
          xv[u][nt] = (n0 + nt < ntiles) ? xi[(xo >= 0 ? xo : 0) + 16 * (n0 + nt) + r] : (R)0;
      }
    };
    auto step = [&](int gi, double2 (&z)[2][MT], R (&xv)[2][NW]) {
#pragma unroll
      for (int u = 0; u < 2; ++u) {
        const bool ok = xoff[8 * gi + 4 * u + g] >= 0;
#pragma unroll
        for (int nt = 0; nt < NW; ++nt) {
          if (n0 + nt >= ntiles) continue;
          const double bv = ok ? (double)xv[u][nt] : 0.0;
          const double bs = sg * pair_swap64(bv);
#pragma unroll
          for (int mt = 0; mt < MT; ++mt) {
            const double2 zz = (iok[mt] && ok) ? z[u][mt] : make_double2(0.0, 0.0);
            acc[mt][nt] = mma64((MODE == 2) ? zz.y : zz.x, bv, acc[mt][nt]);
            if (MODE == 0) acc[mt][nt] = mma64(zz.y, bs, acc[mt][nt]);
          }
        }
      }
    };
    double2 za[2][MT], zb[2][MT];
    R xa[2][NW], xb[2][NW];
    load(0, za, xa);
    for (int gi = 0; gi < ngrp; gi += 2) {
      if (gi + 1 < ngrp) load(gi + 1, zb, xb);
      step(gi, za, xa);
      if (gi + 1 < ngrp) {
        if (gi + 2 < ngrp) load(gi + 2, za, xa);
        step(gi + 1, zb, xb);
      }
    }
#pragma unroll
    for (int mt = 0; mt < MT; ++mt)
#pragma unroll
      for (int nt = 0; nt < NW; ++nt) {
        if (n0 + nt >= ntiles) continue;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const int ii = m0 + 16 * mt + 4 * j + g;   // FP64 16x16x4 result: row 4 j + lane / 16
          if (ii < nb) yi[(int64_t)(r0 + ii) * nc2 + 16 * (n0 + nt) + r] = (R)acc[mt][nt][j];
        }
      }
  }
}

// FP32 form of the near-field product for the FP32 applies: near-field values
// rounded to FP32 once at set-up, FP32 matrix-core steps (v_mfma_f32_16x16x4:
// about three times the FP64 rate), same work layout as k_near_mf.
template <int MODE>
__global__ void __launch_bounds__(256) k_near_mf32(const int64_t* __restrict__ row_ptr,
                                                   const int32_t* __restrict__ box_start,
                                                   const int32_t* __restrict__ bcol_ptr,
                                                   const int32_t* __restrict__ bcol,
                                                   const int32_t* __restrict__ self_off,
                                                   const float2* __restrict__ Zn, const float* __restrict__ xi,
                                                   float* __restrict__ yi, int nleaf, int nc, int xcap) {
  extern __shared__ int32_t xoff_all[];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int g = lane >> 4, r = lane & 15;
  const int b = blockIdx.x * 4 + w;
  if (b >= nleaf) return;
  int32_t* xoff = xoff_all + w * xcap;
  const int r0 = box_start[b], nb = box_start[b + 1] - r0;
  const int32_t* cols = bcol + bcol_ptr[b];
  int t0 = 0, t1 = bcol_ptr[b + 1] - bcol_ptr[b];
  if (MODE == 1) {
    t0 = self_off[b];
    t1 = t0 + nb;
  }
  const int nc2 = 2 * nc, ntiles = nc >> 3;
  const int ngrp = (t1 - t0 + 7) / 8;
  for (int e = lane; e < 8 * ngrp; e += 64) xoff[e] = (t0 + e < t1) ? cols[t0 + e] * nc2 : -1;
  wave_lds_sync();
  const int tlast = t1 - t0 - 1;
  const float sg = (r & 1) ? 1.f : -1.f;
  for (int m0 = 0; m0 < nb; m0 += 32) {
    bool iok[2];
    const float2* zrow[2];
#pragma unroll
    for (int mt = 0; mt < 2; ++mt) {
      iok[mt] = m0 + 16 * mt + r < nb;
      zrow[mt] = Zn + row_ptr[r0 + (iok[mt] ? m0 + 16 * mt + r : 0)] + t0;
    }
    f4 acc[2][4];
#pragma unroll
    for (int mt = 0; mt < 2; ++mt)
#pragma unroll
      for (int nt = 0; nt < 4; ++nt) acc[mt][nt] = f4{0.f, 0.f, 0.f, 0.f};
    auto load = [&](int gi, float2 (&z)[2][2], float (&xv)[2][4]) {
#pragma unroll
      for (int u = 0; u < 2; ++u) {
        const int tt = 8 * gi + 4 * u + g;
        const int xo = xoff[tt];
#pragma unroll
        for (int mt = 0; mt < 2; ++mt) z[u][mt] = zrow[mt][min(tt, tlast)];
#pragma unroll
        for (int nt = 0; nt < 4; ++nt) xv[u][nt] = (nt < ntiles) ? xi[(xo >= 0 ? xo : 0) + 16 * nt + r] : 0.f;
      }
    };
    auto step = [&](int gi, float2 (&z)[2][2], float (&xv)[2][4]) {
#pragma unroll
      for (int u = 0; u < 2; ++u) {
        const bool ok = xoff[8 * gi + 4 * u + g] >= 0;
#pragma unroll
        for (int nt = 0; nt < 4; ++nt) {
          if (nt >= ntiles) continue;
          const float bv = ok ? xv[u][nt] : 0.f;
          const float bs = sg * pair_swap(bv);
#pragma unroll
          for (int mt = 0; mt < 2; ++mt) {
            const float2 zz = (iok[mt] && ok) ? z[u][mt] : make_float2(0.f, 0.f);
            acc[mt][nt] = mma((MODE == 2) ? zz.y : zz.x, bv, acc[mt][nt]);
            if (MODE == 0) acc[mt][nt] = mma(zz.y, bs, acc[mt][nt]);
          }
        }
      }
    };
    float2 za[2][2], zb[2][2];
    float xa[2][4], xb[2][4];
    load(0, za, xa);
    for (int gi = 0; gi < ngrp; gi += 2) {
      if (gi + 1 < ngrp) load(gi + 1, zb, xb);
      step(gi, za, xa);
      if (gi + 1 < ngrp) {
        if (gi + 2 < ngrp) load(gi + 2, za, xa);
        step(gi + 1, zb, xb);
      }
    }
#pragma unroll
    for (int mt = 0; mt < 2; ++mt)
#pragma unroll
      for (int nt = 0; nt < 4; ++nt) {
        if (nt >= ntiles) continue;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const int ii = m0 + 16 * mt + 4 * g + j;
          if (ii < nb) yi[(int64_t)(r0 + ii) * nc2 + 16 * nt + r] = acc[mt][nt][j];
        }
      }
  }
}

bool mf_near32(const int64_t* row_ptr, const int32_t* box_start, const int32_t* bcol_ptr, const int32_t* bcol,
               const int32_t* self_off, const float2* Zn, const float2* xi, float2* yi, int nleaf,
               int max_cols_box, int nc, int mode, hipStream_t s) {
  if (!Zn || nc % 8 != 0 || nc > 32 || max_cols_box > 4096) return false;
  const int xcap = (max_cols_box + 8 + 7) / 8 * 8;
  const size_t sh = (size_t)4 * xcap * sizeof(int32_t);
  const dim3 grid((unsigned)((nleaf + 3) / 4));
#define CM_NEAR(M)                                                                                                   \
  hipLaunchKernelGGL((k_near_mf32<M>), grid, dim3(256), sh, s, row_ptr, box_start, bcol_ptr, bcol, self_off, Zn,    \
                     (const float*)xi, (float*)yi, nleaf, nc, xcap)
  if (mode == 0)
    CM_NEAR(0);
  else if (mode == 1)
    CM_NEAR(1);
  else
    CM_NEAR(2);
#undef CM_NEAR
  return true;
}

template <typename R>
bool mf_near(const int64_t* row_ptr, const int32_t* box_start, const int32_t* bcol_ptr, const int32_t* bcol,
             const int32_t* self_off, const double2* Zn, const void* xi, void* yi, int nleaf, int max_box,
             int max_cols_box, int nc, int mode, hipStream_t s, const SlotTabs* st, int nslot) {
  if (nc % 8 != 0 || nc > 64 || max_cols_box > 4096) return false;
  if (nslot < 1 || nslot > kMaxSlots || (nslot > 1 && !st)) return false;
  const SlotTabs none;
  const SlotTabs& sv = st ? *st : none;
  const int xcap = (max_cols_box + 8 + 7) / 8 * 8;
  const size_t sh = (size_t)4 * xcap * sizeof(int32_t);
  (void)max_box;
  // one row tile and two column tiles per wave: four waves per leaf box
  // (0.53 ms for the 32-column product at N = 122,880 against 0.73 ms with
  // one wave per box); a batch of one column tile takes two waves per box
  // with all four column slots each, so that every value is loaded once
  constexpr int MT = 1;
#define CM_NEAR_W(M, NW)                                                                                       \
  {                                                                                                            \
    constexpr int BPB = 4 / ((2 / MT) * (4 / NW));                                                             \
    const dim3 grid((unsigned)((nleaf + BPB - 1) / BPB), (unsigned)((nc + 31) / 32), (unsigned)nslot);        \
    hipLaunchKernelGGL((k_near_mf<R, M, MT, NW>), grid, dim3(256), sh, s, row_ptr, box_start, bcol_ptr, bcol,  \
                       self_off, Zn, (const R*)xi, (R*)yi, nleaf, nc, xcap, sv);                               \
  }
#define CM_NEAR(M)        \
  if (nc <= 8)            \
    CM_NEAR_W(M, 4)       \
  else                    \
    CM_NEAR_W(M, 2)
  if (mode == 0) {
    CM_NEAR(0)
  } else if (mode == 1) {
    CM_NEAR(1)
  } else {
    CM_NEAR(2)
  }
#undef CM_NEAR
#undef CM_NEAR_W
  return true;
}
template bool mf_near<float>(const int64_t*, const int32_t*, const int32_t*, const int32_t*, const int32_t*,
                             const double2*, const void*, void*, int, int, int, int, int, hipStream_t,
                             const SlotTabs*, int);
template bool mf_near<double>(const int64_t*, const int32_t*, const int32_t*, const int32_t*, const int32_t*,
                              const double2*, const void*, void*, int, int, int, int, int, hipStream_t,
                              const SlotTabs*, int);

static void lds_limit(const void* f, size_t bytes) {
  if (bytes > 64 * 1024) {
    hipError_t e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
    if (e != hipSuccess) throw Error(-4, std::string("hipFuncSetAttribute: ") + hipGetErrorString(e));
  }
}

static bool lds_fits(size_t bytes) { return bytes <= 160 * 1024; }

// theta row tiles per block: all of them up to four, else split evenly over
// ceil(NT / 4) blocks
static int nt_block(const MfD& T) {
  const int groups = (T.NT + 3) / 4;
  return (T.NT + groups - 1) / groups;
}
static int nt_groups(const MfD& T) { return (T.NT + nt_block(T) - 1) / nt_block(T); }

// LDS of a block of wpb waves (each wave keeps its own phi-step rows)
static size_t interp_lds(const MfD& T, int ntc, int wpb) {
  const int nb = nt_block(T), S = 2 * T.S2, RS = 16 * S + 16, SH = S * 16 * nb;
  return (size_t)nb * T.ktmax * 68 * 4 + (size_t)wpb * (ntc * RS + 2 * SH) * 4;
}
// a sweep batch reads a chunk's phase values from global memory when the
// chunk's table is at most this size (measured on the 122,880-unknown sphere:
// faster than per-wave LDS copies at levels 4 and 5, slower at level 3)
constexpr size_t kZgGlobalMax = 12 * 1024;
static bool zg_global(const MfD& T, int ntp) { return (size_t)ntp * 4 * T.kmax * 8 <= kZgGlobalMax; }
static size_t anterp_lds(const MfD& T, int ntp, int wpb, bool sweep) {
  const int S = 2 * T.S2, RS = 16 * S + 16;
  const int nz = sweep ? (zg_global(T, ntp) ? 0 : wpb) : 1;
  return (size_t)nt_block(T) * T.ktmax * 68 * 4 + (size_t)nz * ntp * 4 * T.kmax * 8 + (size_t)wpb * ntp * RS * 4;
}
// waves per block: four (one column tile each), fewer where the rows of four
// waves do not fit in LDS (large angular grids at coarse levels); 0: none fits
static int interp_wpb(const MfD& T, int ntc) {
  for (int w = 4; w >= 1; w /= 2)
    if (lds_fits(interp_lds(T, ntc, w))) return w;
  return 0;
}
static int anterp_wpb(const MfD& T, int ntp, bool sweep) {
  for (int w = 4; w >= 1; w /= 2)
    if (lds_fits(anterp_lds(T, ntp, w, sweep))) return w;
  return 0;
}

// Rows per double-buffered load group: by default from the K-step register
// budget (two rows up to 8 K steps, one row at 16), or the autotuner's choice
// for the level (LevelD::rg_ip / rg_at; 4 rows only up to 8 K steps).  The
// code's bit 8 selects the variant compiled for at least three waves per
// SIMD (register file capped at 168 per lane; 1 or 2 rows only).
constexpr int kRgW3 = 8;
static int rg_default(int mk) { return mk <= 8 ? 2 : 1; }
static bool rg_valid(int mk, int rg) {
  const int r = rg & ~kRgW3;
  if (rg & kRgW3) return r == 1 || r == 2;
  return r == 1 || r == 2 || (r == 4 && mk <= 8);
}

template <int NT, int S2, int MK, int RG, int W>
static void launch_interp_rg(const LevelD<float>& Lp, const LevelD<float>& Lc, const float2* Sc, float2* Sp, int nc,
                             int ldp, int accum, const void* shiftT, const SweepSlots& sw, hipStream_t s) {
  const MfD& T = Lp.mip;
  const int nb = (Lp.nbox * T.nchunk + 7) / 8 * 8;
  const int ntiles = nc / 4;   // 2 components x nc/8, or the slots of a sweep batch
  const int wpb = interp_wpb(T, Lc.nt);
  const size_t sh = interp_lds(T, Lc.nt, wpb);
  lds_limit((const void*)k_interp_mf<NT, S2, MK, RG, W>, sh);
  hipLaunchKernelGGL((k_interp_mf<NT, S2, MK, RG, W>), dim3(nb, (ntiles + wpb - 1) / wpb, nt_groups(T)), dim3(64 * wpb),
                     sh, s,
                     (const float*)Sc,
                     (float*)Sp, Lp.child_ptr, Lc.octant, T, (const float2*)shiftT, Lc.nt, Lc.np, Lp.nt, Lp.np,
                     Lp.nbox, nc, ldp, accum, sw);
}

template <int NT, int S2, int MK>
static void launch_interp(const LevelD<float>& Lp, const LevelD<float>& Lc, const float2* Sc, float2* Sp, int nc,
                          int ldp, int accum, const void* shiftT, int rg, const SweepSlots& sw, hipStream_t s) {
  if constexpr (MK <= 8)
    if (rg == 4) return launch_interp_rg<NT, S2, MK, 4, 1>(Lp, Lc, Sc, Sp, nc, ldp, accum, shiftT, sw, s);
  if (rg == (1 | kRgW3)) return launch_interp_rg<NT, S2, MK, 1, 3>(Lp, Lc, Sc, Sp, nc, ldp, accum, shiftT, sw, s);
  if (rg == (2 | kRgW3)) return launch_interp_rg<NT, S2, MK, 2, 3>(Lp, Lc, Sc, Sp, nc, ldp, accum, shiftT, sw, s);
  if (rg == 1) return launch_interp_rg<NT, S2, MK, 1, 1>(Lp, Lc, Sc, Sp, nc, ldp, accum, shiftT, sw, s);
  launch_interp_rg<NT, S2, MK, 2, 1>(Lp, Lc, Sc, Sp, nc, ldp, accum, shiftT, sw, s);
}

template <int NT, int S2, int MK, int RG, int W>
static void launch_anterp_rg(const LevelD<float>& Lp, const LevelD<float>& Lc, const float2* Gp, float2* Gc, int nc,
                             int ldp, int add, const void* zg, const SweepSlots& sw, hipStream_t s) {
  const MfD& T = Lp.mat;
  const int nb = (Lc.nbox * T.nchunk + 7) / 8 * 8;
  const int ntiles = nc / 4;
  const int wpb = anterp_wpb(T, Lp.nt, sw.on);
  const size_t sh = anterp_lds(T, Lp.nt, wpb, sw.on);
  SweepSlots sv = sw;
  sv.zg_global = sw.on && zg_global(T, Lp.nt);
  lds_limit((const void*)k_anterp_mf<NT, S2, MK, RG, W>, sh);
  hipLaunchKernelGGL((k_anterp_mf<NT, S2, MK, RG, W>), dim3(nb, (ntiles + wpb - 1) / wpb, nt_groups(T)), dim3(64 * wpb),
                     sh, s,
                     (const float*)Gp,
                     (float*)Gc, Lc.parent, Lc.octant, T, (const float2*)zg, Lc.nt, Lc.np, Lp.nt, Lp.np, Lc.nbox, nc,
                     ldp, add, sv);
}

template <int NT, int S2, int MK>
static void launch_anterp(const LevelD<float>& Lp, const LevelD<float>& Lc, const float2* Gp, float2* Gc, int nc,
                          int ldp, int add, const void* zg, int rg, const SweepSlots& sw, hipStream_t s) {
  if constexpr (MK <= 8)
    if (rg == 4) return launch_anterp_rg<NT, S2, MK, 4, 1>(Lp, Lc, Gp, Gc, nc, ldp, add, zg, sw, s);
  if (rg == (1 | kRgW3)) return launch_anterp_rg<NT, S2, MK, 1, 3>(Lp, Lc, Gp, Gc, nc, ldp, add, zg, sw, s);
  if (rg == (2 | kRgW3)) return launch_anterp_rg<NT, S2, MK, 2, 3>(Lp, Lc, Gp, Gc, nc, ldp, add, zg, sw, s);
  if (rg == 1) return launch_anterp_rg<NT, S2, MK, 1, 1>(Lp, Lc, Gp, Gc, nc, ldp, add, zg, sw, s);
  launch_anterp_rg<NT, S2, MK, 2, 1>(Lp, Lc, Gp, Gc, nc, ldp, add, zg, sw, s);
}

#define CM_MF_CASES(X)                                                    \
  X(1, 8, 4) X(1, 8, 8) X(1, 8, 16) X(1, 4, 4) X(1, 4, 8) X(1, 4, 16) \
  X(2, 8, 4) X(2, 8, 8) X(2, 8, 16) X(2, 4, 4) X(2, 4, 8) X(2, 4, 16) \
  X(3, 4, 4) X(3, 4, 8) X(3, 4, 16) X(4, 4, 4) X(4, 4, 8) X(4, 4, 16)

static int mk_of(const MfD& T) { return T.kmax <= 4 ? 4 : T.kmax <= 8 ? 8 : 16; }

static bool has_case(const MfD& T) {
  const int mk = mk_of(T), nb = nt_block(T);
#define X(a, b, c) \
  if (nb == a && T.S2 == b && mk == c) return true;
  CM_MF_CASES(X)
#undef X
  return false;
}

// columns per batch: tiles of eight, or slots of four in a sweep batch (at most kMaxSlots)
static bool cols_ok(int nc, bool sweep) {
  return sweep ? (nc % 4 == 0 && nc / 4 <= kMaxSlots) : nc % 8 == 0;
}

bool mf_interp_covers(const LevelD<float>& Lp, const LevelD<float>& Lc, int nc, bool sweep) {
  const MfD& T = Lp.mip;
  return T.ok && cols_ok(nc, sweep) && interp_wpb(T, Lc.nt) && has_case(T);
}

bool mf_interp(const LevelD<float>& Lp, const LevelD<float>& Lc, const float2* Sc, float2* Sp, int nc, int ldp,
               int accum, const void* shiftT, hipStream_t s, const SweepSlots* sw) {
  const MfD& T = Lp.mip;
  if (!shiftT || !mf_interp_covers(Lp, Lc, nc, sw != nullptr)) return false;
  if (sw && (!sw->on || sw->n * 4 != nc)) return false;
  const SweepSlots none;
  const SweepSlots& sv = sw ? *sw : none;
  const int mk = mk_of(T);
  const int rg = rg_valid(mk, Lp.rg_ip) ? Lp.rg_ip : rg_default(mk);
  const int nb = nt_block(T);
#define X(a, b, c)                                                               \
  if (nb == a && T.S2 == b && mk == c) {                                       \
    launch_interp<a, b, c>(Lp, Lc, Sc, Sp, nc, ldp, accum, shiftT, rg, sv, s);   \
    return true;                                                                 \
  }
  CM_MF_CASES(X)
#undef X
  return false;
}

bool mf_covers(const LevelD<float>& Lp, int nc, bool sweep) {
  const MfD& T = Lp.mat;
  return T.ok && cols_ok(nc, sweep) && Lp.zg && anterp_wpb(T, Lp.nt, sweep) && has_case(T);
}

bool mf_anterp(const LevelD<float>& Lp, const LevelD<float>& Lc, const float2* Gp, float2* Gc, int nc, int ldp,
               int add, const void* zg, hipStream_t s, const SweepSlots* sw) {
  const MfD& T = Lp.mat;
  if (!mf_covers(Lp, nc, sw != nullptr) || !zg) return false;
  if (sw && (!sw->on || sw->n * 4 != nc)) return false;
  const SweepSlots none;
  const SweepSlots& sv = sw ? *sw : none;
  const int mk = mk_of(T);
  const int rg = rg_valid(mk, Lp.rg_at) ? Lp.rg_at : rg_default(mk);
  const int nb = nt_block(T);
#define X(a, b, c)                                                           \
  if (nb == a && T.S2 == b && mk == c) {                                   \
    launch_anterp<a, b, c>(Lp, Lc, Gp, Gc, nc, ldp, add, zg, rg, sv, s);     \
    return true;                                                             \
  }
  CM_MF_CASES(X)
#undef X
  return false;
}

// Autotuning of the matrix-core interpolation and anterpolation per level:
// for each level, every valid combination of slot-chunk width (the plan's
// table or the alternate one) and rows per load group is timed on the
// workspace (one untimed and three timed launches at nc columns, HIP events
// on the stream) and the fastest is kept.  The choices change only the
// summation grouping, so results differ from the untuned handle by FP32
// rounding.  Returns the choices and times as a JSON array.
std::string mf_autotune(PrecD<float>& pd, int lf, const std::vector<void*>& S, const std::vector<void*>& G, int nc,
                        hipStream_t s) {
  std::ostringstream js;
  js << "[";
  // the two timing events, destroyed on every way out
  struct Events {
    hipEvent_t a = nullptr, b = nullptr;
    ~Events() {
      if (a) (void)hipEventDestroy(a);
      if (b) (void)hipEventDestroy(b);
    }
  } ev;
  if (hipEventCreate(&ev.a) != hipSuccess || hipEventCreate(&ev.b) != hipSuccess)
    throw Error(-4, "hipEventCreate (autotune)");
  hipEvent_t e0 = ev.a, e1 = ev.b;
  auto time_it = [&](auto&& launch) -> float {
    if (!launch()) return -1.f;
    if (hipEventRecord(e0, s) != hipSuccess) throw Error(-4, "hipEventRecord (autotune)");
    for (int i = 0; i < 3; ++i) launch();
    if (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess)
      throw Error(-4, "autotune timing");
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, e0, e1) != hipSuccess) throw Error(-4, "hipEventElapsedTime (autotune)");
    return ms / 3.f;
  };
  bool first = true;
  for (int l = 2; l < lf; ++l) {
    LevelD<float>& Lp = pd.lev[l];
    const LevelD<float>& Lc = pd.lev[l + 1];
    for (int kind = 0; kind < 2; ++kind) {      // 0 interpolation into l, 1 anterpolation from l
      MfD& cur = kind ? Lp.mat : Lp.mip;
      MfD& alt = kind ? Lp.mat_alt : Lp.mip_alt;
      int& rgsel = kind ? Lp.rg_at : Lp.rg_ip;
      float best = 1e30f;
      int best_alt = 0, best_rg = 0, best_s2 = 0;
      float base = -1.f;
      for (int a = 0; a < 2; ++a) {
        if (a) {
          std::swap(cur, alt);
          if (kind) {
            std::swap(Lp.zg, Lp.zg_alt);
            std::swap(Lp.dzg, Lp.dzg_alt);
          }
        }
        if (cur.ok) {
          const int mk = mk_of(cur);
          for (int rg : {1, 2, 4, 1 | kRgW3, 2 | kRgW3}) {
            if (!rg_valid(mk, rg)) continue;
            rgsel = rg;
            const float ms = kind ? time_it([&] {
              return mf_anterp(Lp, Lc, (const float2*)G[l], (float2*)G[l + 1], nc, nc, 1, Lp.zg, s);
            })
                                  : time_it([&] {
                                      return mf_interp(Lp, Lc, (const float2*)S[l + 1], (float2*)S[l], nc, nc, 0,
                                                       Lp.shiftT, s);
                                    });
            if (ms < 0.f) break;   // this table is not covered at all
            if (a == 0 && rg == rg_default(mk)) base = ms;
            if (ms < best) {
              best = ms;
              best_alt = a;
              best_rg = rg;
              best_s2 = cur.S2;
            }
          }
        }
        if (a) {   // back to the plan's table
          std::swap(cur, alt);
          if (kind) {
            std::swap(Lp.zg, Lp.zg_alt);
            std::swap(Lp.dzg, Lp.dzg_alt);
          }
        }
      }
      if (best >= 1e30f) {
        rgsel = 0;
        continue;
      }
      if (best_alt) {
        std::swap(cur, alt);
        if (kind) {
          std::swap(Lp.zg, Lp.zg_alt);
          std::swap(Lp.dzg, Lp.dzg_alt);
        }
      }
      rgsel = best_rg;
      js << (first ? "" : ", ") << "{\"stage\": \"" << (kind ? "anterp_l" : "interp_l") << (kind ? l + 1 : l)
         << "\", \"half_slots\": " << best_s2 << ", \"row_group\": " << (best_rg & ~kRgW3)
         << ", \"min_waves\": " << ((best_rg & kRgW3) ? 3 : 1) << ", \"ms\": " << best
         << ", \"default_ms\": " << base << "}";
      first = false;
    }
  }
  js << "]";
  return js.str();
}

}  // namespace cm
