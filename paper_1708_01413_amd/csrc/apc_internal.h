// Internal declarations shared by the HIP kernels and the host side of libapc.
#pragma once

#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <cstdint>

#include "apc.h"

namespace apc {

// Per-kernel timing without extra packets on the stream: when a pair of events
// is pending, the next timed launch takes it and records the two events from
// its own dispatch (the kernel's start and end), so timing adds no idle gap
// between kernels.  A launcher that enqueues nothing leaves the pair pending.
struct TimedLaunch {
  hipEvent_t start = nullptr;
  hipEvent_t stop = nullptr;
};
TimedLaunch& pending_timing();

#define APC_LAUNCH(kernel, grid, block, shmem, stream, ...)                                  \
  do {                                                                                      \
    ::apc::TimedLaunch& tl_ = ::apc::pending_timing();                                      \
    if (tl_.start) {                                                                        \
      hipExtLaunchKernelGGL(kernel, grid, block, shmem, stream, tl_.start, tl_.stop, 0,      \
                            __VA_ARGS__);                                                   \
      tl_ = ::apc::TimedLaunch{};                                                           \
    } else {                                                                                \
      hipLaunchKernelGGL(kernel, grid, block, shmem, stream, __VA_ARGS__);                  \
    }                                                                                       \
  } while (0)


constexpr int kThreads = 256;       // threads per workgroup for streaming kernels

// FP32 wave sum without LDS: DPP within each 16-lane row (pairs, quads, then
// rotations by 4 and 8 lanes give every lane its row's sum), then the four row
// sums read as scalars.  The result is uniform across the wave.
template <int CTRL>
__device__ inline float dpp_f32(float x) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), CTRL, 0xf, 0xf, false));
}
__device__ inline float wave_sum_dpp(float v) {
  v += dpp_f32<0xB1>(v);   // quad_perm(1, 0, 3, 2)
  v += dpp_f32<0x4E>(v);   // quad_perm(2, 3, 0, 1)
  v += dpp_f32<0x124>(v);  // row_ror:4
  v += dpp_f32<0x128>(v);  // row_ror:8
  const float r0 = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 0));
  const float r1 = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 16));
  const float r2 = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 32));
  const float r3 = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 48));
  return (r0 + r1) + (r2 + r3);
}
// The same for FP64: each DPP move carries the two 32-bit halves.
template <int CTRL>
__device__ inline double dpp_f64(double x) {
  const long long b = __double_as_longlong(x);
  const int lo = __builtin_amdgcn_update_dpp(0, static_cast<int>(b), CTRL, 0xf, 0xf, false);
  const int hi = __builtin_amdgcn_update_dpp(0, static_cast<int>(b >> 32), CTRL, 0xf, 0xf, false);
  return __longlong_as_double((static_cast<long long>(hi) << 32) |
                              static_cast<long long>(static_cast<unsigned>(lo)));
}
__device__ inline double lane_f64(double x, int l) {
  const long long b = __double_as_longlong(x);
  const int lo = __builtin_amdgcn_readlane(static_cast<int>(b), l);
  const int hi = __builtin_amdgcn_readlane(static_cast<int>(b >> 32), l);
  return __longlong_as_double((static_cast<long long>(hi) << 32) |
                              static_cast<long long>(static_cast<unsigned>(lo)));
}
__device__ inline double wave_sum_dpp(double v) {
  v += dpp_f64<0xB1>(v);
  v += dpp_f64<0x4E>(v);
  v += dpp_f64<0x124>(v);
  v += dpp_f64<0x128>(v);
  return (lane_f64(v, 0) + lane_f64(v, 16)) + (lane_f64(v, 32) + lane_f64(v, 48));
}

// Row sums of R rows at once, each row's partial spread over the 64 lanes of
// the wave (v[k] in every lane).  Instead of R separate wave sums, the rows are
// halved between lane halves: v_permlane32_swap pairs lane l with l ^ 32, which
// keeps rows k < R/2 in the low half and the others in the high half (one swap
// and one add per pair of rows, no selects); v_permlane16_swap does the same
// for l ^ 16, and for R = 8 a DPP rotate by 8 within each 16-lane row (with
// selects) for l ^ 8.  Each lane then holds one row's partial, summed within
// groups of 8 or 16 lanes by DPP, and the R results are read out with
// v_readlane.  The order of the additions is fixed, so results are
// reproducible.
__device__ inline double swap_add32(double& a, double& b) {
  const uint64_t ua = static_cast<uint64_t>(__double_as_longlong(a));
  const uint64_t ub = static_cast<uint64_t>(__double_as_longlong(b));
  const auto lo = __builtin_amdgcn_permlane32_swap(static_cast<unsigned>(ua), static_cast<unsigned>(ub),
                                                   false, false);
  const auto hi = __builtin_amdgcn_permlane32_swap(static_cast<unsigned>(ua >> 32),
                                                   static_cast<unsigned>(ub >> 32), false, false);
  const double na = __longlong_as_double(static_cast<long long>(
      (static_cast<uint64_t>(hi[0]) << 32) | static_cast<uint64_t>(lo[0])));
  const double nb = __longlong_as_double(static_cast<long long>(
      (static_cast<uint64_t>(hi[1]) << 32) | static_cast<uint64_t>(lo[1])));
  return na + nb;
}
__device__ inline double swap_add16(double& a, double& b) {
  const uint64_t ua = static_cast<uint64_t>(__double_as_longlong(a));
  const uint64_t ub = static_cast<uint64_t>(__double_as_longlong(b));
  const auto lo = __builtin_amdgcn_permlane16_swap(static_cast<unsigned>(ua), static_cast<unsigned>(ub),
                                                   false, false);
  const auto hi = __builtin_amdgcn_permlane16_swap(static_cast<unsigned>(ua >> 32),
                                                   static_cast<unsigned>(ub >> 32), false, false);
  const double na = __longlong_as_double(static_cast<long long>(
      (static_cast<uint64_t>(hi[0]) << 32) | static_cast<uint64_t>(lo[0])));
  const double nb = __longlong_as_double(static_cast<long long>(
      (static_cast<uint64_t>(hi[1]) << 32) | static_cast<uint64_t>(lo[1])));
  return na + nb;
}

template <int R>
__device__ inline void row_sums(double (&v)[R], double (&w)[R], int lane) {
  static_assert(R == 1 || R == 2 || R == 4 || R == 8, "rows per wave");
  double r;
  if constexpr (R == 1) {
    r = v[0];
  } else {
    // l ^ 32: the low half keeps rows [0, R/2), the high half [R/2, R).
    double h[R / 2];
#pragma unroll
    for (int k = 0; k < R / 2; ++k) h[k] = swap_add32(v[k], v[k + R / 2]);
    if constexpr (R == 2) {
      r = h[0];
    } else {
      // l ^ 16 within each half: even rows of 16 lanes keep the lower quarter.
      double g[R / 4];
#pragma unroll
      for (int k = 0; k < R / 4; ++k) g[k] = swap_add16(h[k], h[k + R / 4]);
      if constexpr (R == 4) {
        r = g[0];
      } else {
        // l ^ 8 (a rotate by 8 within 16 lanes): lanes with bit 3 clear keep g[0].
        const bool up = (lane & 8) != 0;
        const double send = up ? g[0] : g[1];
        const double keep = up ? g[1] : g[0];
        r = keep + dpp_f64<0x128>(send);
      }
    }
  }
  // Plain sums within groups of 8 lanes (R = 8) or 16 lanes (R < 8).
  r += dpp_f64<0xB1>(r);   // quad_perm(1, 0, 3, 2)
  r += dpp_f64<0x4E>(r);   // quad_perm(2, 3, 0, 1)
  r += dpp_f64<0x141>(r);  // row_half_mirror
  if constexpr (R < 8) r += dpp_f64<0x128>(r);  // row_ror:8
  if constexpr (R == 8) {
#pragma unroll
    for (int k = 0; k < 8; ++k) w[k] = lane_f64(r, 8 * k);
  } else if constexpr (R == 4) {
#pragma unroll
    for (int k = 0; k < 4; ++k) w[k] = lane_f64(r, 16 * k);
  } else if constexpr (R == 2) {
#pragma unroll
    for (int k = 0; k < 2; ++k) w[k] = lane_f64(r, 32 * k) + lane_f64(r, 32 * k + 16);
  } else {
    w[0] = (lane_f64(r, 0) + lane_f64(r, 16)) + (lane_f64(r, 32) + lane_f64(r, 48));
  }
}


constexpr int kRowTile = 16;        // rows per pass-A workgroup
constexpr int kLdAlign = 64;        // padded row stride of the internal factor (elements)
constexpr int kGramTile = 64;       // FP64 setup GEMM tile edge
constexpr int kMaxBlockRows = 2048; // largest p_i the setup Cholesky accepts
constexpr int kXcds = 8;            // XCDs per MI355X; workgroups are dealt round-robin

// ---------------------------------------------------------------------------
// Streaming kernels (hot path)
// ---------------------------------------------------------------------------

// out[split * out_stride + row] = sum_{j in split} C[row][j] * d_blk[j] for
// every row of every tile, accumulated in TA, where d_blk is d + blk*ldd when
// d is given, else va - vb[blk] (either may be null: 0) rounded to TA.
// Columns are split into nsplit ranges of split_cols (a multiple of the
// register chunk, rowdot_chunk<TQ>()).
template <typename TQ, typename TA = TQ>
struct RowdotArgs {
  const TQ* C;
  int64_t ldc;
  const int32_t* tile_row0;   // null: uniform tiling of rows_total rows
  const int32_t* tile_nrows;
  const int32_t* tile_blk;
  int32_t ntiles;              // tiles in this launch, starting at tile_begin
  int32_t rows_total;
  const double* va;
  const double* vb;
  int64_t ldvb;
  const TA* d;
  int64_t ldd;
  TA* out;
  int64_t out_stride;
  int32_t nsplit;
  int64_t split_cols;
  int32_t xcd_remap;          // 1: give each XCD a contiguous range of tiles;
                              // 2: walk the tiles from last to first
  int32_t rows_per_tile;      // 8, 16 or 32 (must match the tile lists)
  int32_t tile_begin;         // first tile of this launch (block-tile lists only)
  int32_t nt_loads = 1;       // 1: non-temporal loads of C
};

template <typename TQ>
constexpr int rowdot_unroll() { return 2; }
// Columns covered by one register chunk of pass A.
template <typename TQ>
constexpr int64_t rowdot_chunk() { return static_cast<int64_t>(kThreads) * (16 / sizeof(TQ)) * rowdot_unroll<TQ>(); }

// Pass B of eq. (2a): x_i += gamma (x_bar - x_i - Q_i w_i), with
// w = sum over pass A's nsplit partials (w + s * w_stride).
template <typename TQ>
struct PassBArgs {
  const TQ* C;
  int64_t ldc;
  const int64_t* off;
  int32_t m;                  // blocks in this launch, starting at blk_begin
  int32_t nslab;
  const TQ* w;
  int32_t nsplit;
  int64_t w_stride;
  double* x;
  int64_t ldx;
  double* xbar;
  double gamma;
  int32_t blk_begin;
  int32_t nt_loads;           // 1: non-temporal loads of C
  int32_t row_split = 1;      // 1: waves split the block's rows over a 64-lane slab;
                              // 0: every wave streams all rows over its own part of a
                              //    kThreads-lane slab
};

// Columns per pass-B slab for an element size and slab layout.
inline int pass_b_slab(int elem_bytes, int row_split) {
  return (row_split ? 64 : kThreads) * (16 / elem_bytes);
}

// y_i = beta * y_i + alpha * sum_{r in block i} w_r C[r][:], FP64 accumulation,
// w_r = sum over nsplit partials (w + s * w_stride).  off == null: a single
// block of rows_total rows.
template <typename TQ>
struct ExpandArgs {
  const TQ* C;
  int64_t ldc;
  const int64_t* off;
  int32_t m;
  int32_t nslab;              // ceil(ldc / (64 * 16 / sizeof(TQ)))
  int64_t rows_total;
  const double* w;
  int32_t nsplit;
  int64_t w_stride;
  double* y;
  int64_t ldy;
  double alpha;
  double beta;
  int32_t blk_begin;          // first block of this launch (off != null)
  const double* wsub = nullptr;  // optional per-row value subtracted from w_r
};

inline int expand_slab(int elem_bytes) { return 64 * (16 / elem_bytes); }

hipError_t launch_rowdot_f64(const RowdotArgs<double, double>& a, hipStream_t s);
hipError_t launch_rowdot_f32(const RowdotArgs<float, float>& a, hipStream_t s);
hipError_t launch_rowdot_f32x64(const RowdotArgs<float, double>& a, hipStream_t s);
hipError_t launch_pass_b_f64(const PassBArgs<double>& a, hipStream_t s);
hipError_t launch_pass_b_f32(const PassBArgs<float>& a, hipStream_t s);
hipError_t launch_expand_f64(const ExpandArgs<double>& a, hipStream_t s);
hipError_t launch_expand_f32(const ExpandArgs<float>& a, hipStream_t s);

// One pass over C for both halves of eq. (2a): every workgroup owns a tile of
// rows of one block and the whole row width.  For each row r it forms
// w_r = C[r][:] . d_blk (accumulated in TA) and adds w_r C[r][:] to its own
// partial sum, so each row is read once and used twice:
//   part[t * ldp + j] = sum_{r in tile t} (C[r][:] . d_blk) C[r][j],  j < ldc
// (zero for j >= n).
// d_blk = d + blk * ldd (ldd = 0: one vector for every tile); entries of d at
// j >= n are not read (taken as 0).  C is N x ldc, zero past column n, ldc a
// multiple of kLdAlign.  cpt: 16-byte chunks of a row per thread (ldc * sizeof(TQ)
// <= kThreads * 16 * cpt); g: rows per register group (two groups in flight).
template <typename TQ, typename TA = TQ>
struct FusedArgs {
  const TQ* C;
  int64_t ldc;
  int64_t n;
  const int32_t* tile_row0;
  const int32_t* tile_nrows;
  const int32_t* tile_blk;
  int32_t ntiles;
  const TA* d;
  int64_t ldd;
  TA* part;
  int64_t ldp;
  int32_t xcd_remap;          // 1: give each XCD a contiguous range of tiles
  const TA* wsub = nullptr;   // optional: w_r = C[r][:] . d_blk - wsub[r] (global row r)
};
// cpt for a row width: the smallest of 1, 2, 4, 8, 16 that covers it (0 when
// none does).  A launcher accepts g in 1, 2, 4 when fused_shape_ok: the two
// register groups, d_blk and the partial sum fit 256 registers per thread
// (q_bytes = sizeof(TQ), a_bytes = sizeof(TA)).
int fused_cpt(int64_t ldc, int elem_bytes);
bool fused_shape_ok(int q_bytes, int a_bytes, int cpt, int g);
hipError_t launch_fused_f32(const FusedArgs<float, float>& a, int g, hipStream_t s);
hipError_t launch_fused_f64(const FusedArgs<double, double>& a, int g, hipStream_t s);
// FP32 factor, FP64 vector and sums (the normal operator of the eigenvalue
// estimate).
hipError_t launch_fused_f32x64(const FusedArgs<float, double>& a, int g, hipStream_t s);
// out[i * ldo + j] = sum of block i's partial rows (tile_first[i] .. tile_first[i+1]-1,
// in order), j < ncols, every block i < m (FP64).
hipError_t launch_block_sum(const double* part, int64_t ldp, const int32_t* tile_first, int32_t m,
                            int64_t ncols, double* out, int64_t ldo, hipStream_t s);
// out[2i] = ||V_i - U_i||^2 and out[2i+1] = ||U_i||^2 over j < n, rows i < m of
// stride ld (FP64).
hipError_t launch_defect(const double* U, const double* V, int64_t ld, int32_t m, int64_t n,
                         double* out, hipStream_t s);
// h[2 i] = sum over block i's rows r of (w[r] + y[r])^2, h[2 i + 1] = sum of
// y[r]^2 (rows off[i] .. off[i + 1]), where w[r] adds the nsplit partials
// w + s * wstride in split order (fixed summation order throughout).
hipError_t launch_defect_rows(const double* w, int32_t nsplit, int64_t wstride, const double* y,
                              const int64_t* off, int32_t m, double* h, hipStream_t s);
// out[j] = alpha * sum over all ntiles partial rows part[t][j] (FP64), j < n.
hipError_t launch_fused_sum(const double* part, int64_t ldp, int32_t ntiles, int64_t n,
                            double alpha, double* out, hipStream_t s);
// The same over FP32 partial rows (summed in FP64).
hipError_t launch_fused_sum_f32(const float* part, int64_t ldp, int32_t ntiles, int64_t n,
                                double alpha, double* out, hipStream_t s);

// The rest of one update after the single-pass kernel, per column j < n:
//   x_i[j] += gamma (x_bar[j] - x_i[j] - sum_{t in block i} part[t][j])   (eq. 2a)
//   x_bar[j] <- alpha sum_i x_i[j] + beta x_bar[j]                         (eq. 2b)
//   d_i[j] = TD(x_bar[j] - x_i[j])                                         (next pass)
// The partials of block i are tiles tile_first[i] .. tile_first[i+1]-1, summed
// in FP64 in tile order; the block sum runs in a fixed order.
template <typename TD>
struct FusedCombineArgs {
  const TD* part;
  int64_t ldp;
  const int32_t* tile_first;
  double* x;
  int64_t ldx;
  int32_t m;
  int64_t n;
  double gamma;
  double alpha;
  double beta;
  double* xbar;
  TD* d;
  int64_t ldd;
  int32_t tpb = 0;            // > 0: every block has exactly tpb tiles (1, 2, 4 or 8)
};
hipError_t launch_fused_combine_f32(const FusedCombineArgs<float>& a, hipStream_t s);
hipError_t launch_fused_combine_f64(const FusedCombineArgs<double>& a, hipStream_t s);

// T updates of eq. (2a)-(2b) for k = 1 in ONE launch (FP64, small blocks): one
// workgroup per block keeps its rows of C in registers for the whole launch,
// and the m workgroups exchange their x_i once per update through tagged
// words to form x_bar.  The state (x, x_bar, d) is read at the start and written at the end
// in the layout the two-kernel update uses, so the two paths interleave.
// Needs every block to fit one workgroup's registers (resident_shape) and all
// m workgroups resident at once (m at most the device's CU count).
struct ResidentArgs {
  const double* C;
  int64_t ldc;
  int32_t n;
  const int64_t* off;         // m + 1 row offsets of the blocks in C
  int32_t m;
  double* x;                  // x_i at x + i*ldx
  int64_t ldx;
  double* xbar;
  double* d;                  // d_i = x_bar - x_i at d + i*ldd
  int64_t ldd;
  double gamma, alpha, beta;  // x_bar <- alpha sum_i x_i + beta x_bar
  int32_t T;
  uint64_t* xch;              // 2 parities x m x ldc x 2 tagged words (zero at setup)
  uint32_t* sync;             // [1] epoch base, [2] a poll timed out (zero at setup)
  int32_t stride;             // launched workgroups per block (the others exit at once)
  uint32_t spin_limit;        // polls of one exchanged word before the launch gives up
};
constexpr int kResidentThreads = 512;
// Register shape (rows per wave, 16-byte chunks per lane and row) for blocks
// of at most max_rows rows and a row stride of ldc doubles; false if none.
bool resident_shape(int64_t max_rows, int64_t ldc, int* rpw, int* cpl);
hipError_t launch_resident_f64(const ResidentArgs& a, int rpw, int cpl, hipStream_t s);

// ---------------------------------------------------------------------------
// k right-hand sides: streaming contractions on the matrix cores (apc_gemm.hip)
// ---------------------------------------------------------------------------

enum { kTnF64 = 0, kTnF32 = 1, kTnBF16 = 2 };
constexpr int kTnPad = 256;       // rows and K of every operand, zero-padded to a multiple of this
constexpr int kTnMaxSplit = 8;    // split-K factors the partial buffer holds

// part[(s*kp + c)*ldp + r] = sum_{j in [s*klen, min((s+1)*klen, K))} M[r*ldm + j] V[c*ldv + j]
// for r < rows and c < kp, accumulated in FP32 (f32, bf16 operands) or FP64.
// rows is a multiple of 64*rt, K and klen multiples of the step (256 bytes of
// a row), kp is 16, 32, 64 or a multiple of 128, M and V rows are 16-byte
// aligned and zero wherever they extend past the data.
// M: rows x K in the fragment-packed layout written by launch_tn_pack_frag
// (ldm = K); V: kp rows of K, stride ldv.
struct TnArgs {
  const void* M;
  int64_t ldm;
  int64_t rows;
  const void* V;
  int64_t ldv;
  int32_t kp;
  int64_t K;
  int32_t nsplit;
  int64_t klen;
  void* part;
  int64_t ldp;
  int32_t nt;   // 1: non-temporal loads of M
  int32_t waves = 4;  // waves per workgroup: 4, or 8 (bf16 / FP32, nt; rt 1, or rt 2 with pf <= 2)
};
// rt: 16-row tiles per wave (1, 2, 4; FP64 1, 2); pf: steps of M loaded ahead
// (1, 2; 3 and 4 with rt <= 2, non-temporal loads, not FP64).  A workgroup
// covers 16 * waves * rt rows.
hipError_t launch_tn(int type, int rt, int pf, const TnArgs& a, hipStream_t s);
int tn_step_elems(int type);
// out[c*ldo + r] = TQ(sum over the nsplit partials in split order), r < rows, c < kp.
hipError_t launch_tn_sum_cast(int type, const void* part, int32_t nsplit, int32_t kp, int64_t ldp,
                              int64_t rows, void* out, int64_t ldo, hipStream_t s);
// One update of APC in the (y, x_bar) form, over c < kp, j < n (state FP64 with
// stride ldx, z = the summed partials of C^T W):
//   y1 = (1 - gamma) y + gamma x_bar
//   u  = z / m (+ u_ref when anchored)                       (= X y1)
//   x_bar <- eta (x0 + y1 - u) + (1 - eta) x_bar,  y <- y1
//   yq = TQ((1 - gamma) y1 + gamma x_bar - y_ref)   (the next pass-A operand)
// mode 0: an update (y_ref, u_ref may be null: 0); mode 2: an anchor update,
// whose z was formed in FP64 from y1 itself: u_ref <- z / m, y_ref = y1;
// mode 1: the start, x0 = x_bar = z / m, y = 0 (y_ref = u_ref = 0),
// yq = TQ(gamma x0).
struct TnUpdateArgs {
  const void* part;
  int32_t nsplit;
  int32_t kp;
  int64_t ldp;
  int64_t n;
  double* x0;
  double* y;
  double* xb;
  int64_t ldx;
  void* yq;
  int64_t ldq;
  double gamma;
  double eta;
  double inv_m;
  int32_t mode;
  double* yref;
  double* uref;
};
// y_ref[e] = (1 - gamma) y[e] + gamma x_bar[e], e < count.
hipError_t launch_tn_anchor_vec(const double* y, const double* xb, int64_t count, double gamma,
                                double* yref, hipStream_t s);
hipError_t launch_tn_update(int type, int part_f64, const TnUpdateArgs& a, hipStream_t s);
// yq = TQ((1 - gamma) y + gamma x_bar), count entries (the pass-A operand for a
// restored state).
hipError_t launch_tn_prep(int type, const double* y, const double* xb, int64_t count, double gamma,
                          void* yq, hipStream_t s);

// One reverse step of the (y, x_bar) iteration (FP64 adjoints a = dL/dy(t+1),
// bh = dL/dx_bar(t+1); z = the summed partials of C^T C b_q, so X bh = z / m):
//   at = a + eta (bh - X bh)            (the adjoint of y(t+1), both paths)
//   dL/dgamma += <at, x_bar(t) - y(t)>,  dL/deta += <bh, x_bar(t+1) - x_bar(t)> / eta
//   g0 += eta bh                        (the adjoint of x_bar(0) through eq. (2b))
//   a <- (1 - gamma) at,  bh <- (1 - eta) bh + gamma at,  bq = TQ(bh)
// over c < kp, j < n (stride ldx); red holds 2 running sums per workgroup.
struct TnAdjointArgs {
  const void* part;
  int32_t nsplit;
  int32_t kp;
  int64_t ldp;
  int64_t n;
  double* a;
  double* bh;
  double* g0;
  const double* y_t;
  const double* xb_t;
  const double* xb_next;
  int64_t ldx;
  void* bq;
  int64_t ldq;
  double gamma;
  double eta;
  double inv_m;
  double* red;
};
constexpr int kTnAdjointBlocks = 512;
int tn_adjoint_blocks();
hipError_t launch_tn_adjoint(int type, const TnAdjointArgs& a, hipStream_t s);

// ---------------------------------------------------------------------------
// Many independent k = 1 systems (apc_batch.hip)
// ---------------------------------------------------------------------------

// One system of a batch: pointers into its own plan's workspace.
struct BatchSys {
  const void* C;        // factor in the projection precision, N x ldc
  void* d;              // differences x_bar - x_i, m x ldc (projection precision)
  void* w;              // pass-A output, N (projection precision)
  double* x;            // local solutions, m x ldc
  double* xbar;         // average, ldc
  const int64_t* off;   // device block offsets, m + 1
  const double* A;      // FP64 system matrix (residual), row stride lda
  int64_t lda;
  const double* b;      // right-hand side, entry stride ldb
  int64_t ldb;
  int64_t ldc;
  int64_t n;
  int64_t N;
  int32_t m;
  double gamma;
  double eta;
  double bnorm;
  // Single-pass update: the system's row tiles in the batch (row0, nrows, blk
  // at tiles, tiles + ntiles, tiles + 2 ntiles; block i's tiles from
  // tile_first[i]) and one FP32 partial row of ldc entries per tile (in the
  // plan's partial-row slice).
  const int32_t* tiles = nullptr;
  const int32_t* tile_first = nullptr;
  int32_t ntiles = 0;
  float* part = nullptr;
};
// Items: pass A (sys, first row, rows <= 8, block); pass B (sys, block, first
// column of a 256-column slab, 0); average (sys, first column of 256).
// Single pass (rows up to kBatchFusedCols wide): items (sys, tile) write the
// tile's partial row; items (sys, first of 64 columns) then apply the x_i
// update, the average and the next differences, as k = 1 single-system plans do.
constexpr int kBatchFusedCols = 1024;
hipError_t launch_batch_fused(int32_t grid, const BatchSys* sys, const int4* items, int32_t nitems,
                              const int32_t* active, hipStream_t s);
hipError_t launch_batch_fused_combine(int32_t grid, const BatchSys* sys, const int2* items,
                                      int32_t nitems, const int32_t* active, hipStream_t s);

// Mixed batches: k-RHS plans (the (y, x_bar) form with FP32 products and
// optional FP64 anchor updates) run in the same persistent launches as k = 1
// single-pass systems.  Per update four launches, each over one work list:
//   1. pass-A contraction tiles (W = C y; FP64 C with y_ref on anchor updates)
//   2. split sums of W (W64 on anchor updates)
//   3. pass-B contraction tiles (Z = C^T W)
//   4. (y, x_bar) update chunks (anchor update on anchor updates)
// preceded on anchor updates by one launch of y_ref chunks.  Each k = 1
// system's single-pass tiles go with launch 1 and its combine with launch 2,
// or with launches 3 and 4 (the systems are split between the two pairs).
// Items: int4 {kind | system << 8, descriptor (BatchSys or BatchGemm index),
// which / tile / column, block or chunk}.
struct BatchGemm {
  TnArgs tn[4];           // pass A, pass B (FP32 factor), anchor pass A, anchor pass B (FP64)
  int32_t tn_blocks[4];   // 64-row tiles x splits of each contraction
  const void* sum_part;   // split sums: partials, split count (FP32, FP64 anchor),
  int32_t sum_nsplit[2];  // stride, rows, outputs (W FP32, W64 FP64)
  int64_t sum_ldp;
  int64_t sum_rows;
  void* sum_out[2];
  int64_t sum_ldo;
  int32_t kp;
  TnUpdateArgs upd[2];    // update (FP32 partials), anchor update (FP64 partials)
  const double* y;        // y_ref = (1 - gamma) y + gamma x_bar before an anchor update
  const double* xbar;
  double* yref;
  int64_t state_count;    // kp * np
  double gamma;
};
enum BatchItemKind {
  kItemFused = 0, kItemCombine = 1, kItemTn32 = 2, kItemTn64 = 3, kItemSum32 = 4,
  kItemSum64 = 5, kItemUpd32 = 6, kItemUpd64 = 7, kItemAnchorVec = 8
};
constexpr int kBatchChunk = 2048;  // elements per split-sum / update / y_ref item
// nct = kp / 16 of the k-RHS plans (1, 2, 4 or 8).
hipError_t launch_batch_mixed(int32_t grid, int32_t nct, const BatchSys* sys, const BatchGemm* gemm,
                              const int4* items, int32_t nitems, const int32_t* active,
                              hipStream_t s);

hipError_t launch_batch_pass_a(int f64, int32_t grid, const BatchSys* sys, const int4* items,
                               int32_t nitems, const int32_t* active, hipStream_t s);
hipError_t launch_batch_pass_b(int f64, int32_t grid, const BatchSys* sys, const int4* items,
                               int32_t nitems, const int32_t* active, hipStream_t s);
hipError_t launch_batch_average(int f64, int32_t grid, const BatchSys* sys, const int2* items,
                                int32_t nitems, const int32_t* active, hipStream_t s);
// partial[item] = sum over the item's rows of (b_r - a_r . x_bar)^2 (pass-A items).
hipError_t launch_batch_resid(int32_t grid, const BatchSys* sys, const int4* items, int32_t nitems,
                              const int32_t* active, double* partial, hipStream_t s);
// relres[s] = sqrt(sum of system s's partials) / ||b_s||; active[s] = 0 once <= rtol.
hipError_t launch_batch_check(const BatchSys* sys, int32_t count, const int32_t* item_start,
                              const double* partial, double rtol, int32_t* active, double* relres,
                              hipStream_t s);

// R[c*ldr + r] = B[r*ldb + c] - sum of the FP64 partials, r < N, c < k.
hipError_t launch_tn_resid(const double* part, int32_t nsplit, int32_t kp, int64_t ldp, int64_t N,
                           int32_t k, const double* B, int64_t ldb, double* R, int64_t ldr,
                           hipStream_t s);
// dst (drows x ldd, element type of `type`) = src, or src^T when transpose,
// zero outside the FP64 source (srows x scols, stride lds).
hipError_t launch_tn_pack(int type, const double* src, int64_t lds, int64_t srows, int64_t scols,
                          int32_t transpose, void* dst, int64_t ldd, int64_t drows, hipStream_t s);
// The same into the fragment-packed layout of k_tn's M operand (rows x K,
// rows % 16 == 0, K a multiple of tn_step_elems(type)).
hipError_t launch_tn_pack_frag(int type, const double* src, int64_t lds, int64_t srows,
                               int64_t scols, int32_t transpose, void* dst, int64_t K,
                               int64_t rows, hipStream_t s);
// The same from one read of the source, also writing (when non-null) a second
// fragment-packed copy d2 of element type type2 (kTnF64 or kTnF32, not type)
// and, for a non-transposed pack, the row-major FP32 copy r32 (r32rows x
// r32cols of it, stride ldr; r32cols % 8 == 0, r32 16-byte aligned).
hipError_t launch_tn_pack_frag_multi(int type, const double* src, int64_t lds, int64_t srows,
                                     int64_t scols, int32_t transpose, void* dst, int64_t K,
                                     int64_t rows, void* d2, int type2, float* r32, int64_t ldr,
                                     int64_t r32rows, int64_t r32cols, hipStream_t s);

// Per block: out[col*ldo + r0 + r] = scale * sum_q Lop[r][q] in[col*ldi + r0 + q], col < kc,
// with Lop = Linv_i (q <= r) or, when trans, Linv_i^T (q >= r); pmax = max p_i.
hipError_t launch_linv_apply(const int64_t* off, const int64_t* goff, int32_t m, int64_t pmax,
                             const double* Linv, const double* in, int64_t ldi, double* out,
                             int64_t ldo, int32_t kc, int32_t trans, double scale, hipStream_t s);
hipError_t launch_axpy(int64_t count, double alpha, const double* x, double* y, hipStream_t s);
hipError_t launch_sumsq(const double* src, int64_t count, double* partial, hipStream_t s);
int sumsq_parts();

// Eq. (2b) and the next differences: xbar[j] = alpha * sum_{i<m} x[i*ldx + j]
// + beta * xbar[j] for j < n in a fixed order (wave w sums i = w, w+4, ...;
// then (s0 + s1) + (s2 + s3)); beta == 0 does not read xbar.  If d is not
// null, also d[i*ldd + j] = xbar[j] - x[i*ldx + j] rounded to its type.
hipError_t launch_combine_f64(const double* x, int64_t ldx, int32_t m, int64_t n, double alpha,
                              double beta, double* xbar, double* d, int64_t ldd, hipStream_t s);
hipError_t launch_combine_f32(const double* x, int64_t ldx, int32_t m, int64_t n, double alpha,
                              double beta, double* xbar, float* d, int64_t ldd, hipStream_t s);

// ---------------------------------------------------------------------------
// Setup kernels (FP64)
// ---------------------------------------------------------------------------

// C[r][j] = A[r*lda + j] (j < n), 0 for n <= j < ldc; the right-hand sides in
// RHS-major order: c[col*N + r] = B[r*ldb + col] for col < k, 0 up to kp.
hipError_t launch_copy_pad(const double* A, int64_t lda, const double* B, int64_t ldb, int64_t N,
                           int64_t n, double* C, int64_t ldc, double* c, int32_t k, int32_t kp,
                           hipStream_t s);
// G_i = C_i C_i^T for every block (tiles: (blk, ta, tb) with ta >= tb).
hipError_t launch_gram(const double* C, int64_t ldc, const int64_t* off, const int32_t* tiles,
                       int32_t ntiles, const int64_t* goff, double* G, hipStream_t s);
// Per block: Cholesky G_i = L L^T in place (lower triangle), Linv_i = L^{-1}
// (zeros above the diagonal); flags[0] <- 1 + (first block whose pivot fails
// the rank test).
hipError_t launch_chol_inv(const int64_t* off, const int64_t* goff, int32_t m, int64_t pmax,
                           double* G, double* Linv, int* flags, double rank_tol, hipStream_t s);
// G_i = C_i C_i^T on the FP64 matrix cores, both operands staged in LDS
// (512 threads per 64 x 64 tile of `tiles` and K range; ldc a multiple of 32).
// nsplit > 1 splits K into that many ranges: ranges 1.. write partial Grams
// into part (pstride = the total size of G, nsplit - 1 copies), then a second
// launch adds them to G in range order.
hipError_t launch_gram_lds(const double* C, int64_t ldc, const int64_t* off,
                           const int32_t* tiles, int32_t ntiles, const int64_t* goff, double* G,
                           int32_t nsplit, double* part, int64_t pstride, hipStream_t s);
// Out_i = Linv_i In_i on the FP64 matrix cores as kTrmmTile x kTrmmTile
// tiles with both operands staged in LDS (ldc a multiple of 64, pmax the
// largest block's rows, In and Out distinct).  out32 (optional, same layout as
// Out): the result also rounded to FP32.  Row sums (optional, tpart non-null):
// for an N-vector cx (and / or cy), the tile (block i, row tile t) writes
// sum over its rows r of cx[r] Out[r][:] to row toff[i] + t of tpart (cy: row
// toff[m] + toff[i] + t), toff[i] = the row tiles of the blocks before i;
// launch_tile_sum adds them up per block.
constexpr int kTrmmTile = 128;
hipError_t launch_trmm_lds(const double* In, double* Out, int64_t ldc, const int64_t* off,
                           int32_t m, int64_t pmax, const int64_t* goff, const double* Linv,
                           float* out32, const double* cx, const double* cy, const int64_t* toff,
                           double* tpart, hipStream_t s);
// out[i * ldo + c] = sum over t in [toff[i], toff[i + 1]) of part[t * ldc + c],
// in t order, for every block i < m and c < ldc.
hipError_t launch_tile_sum(const double* part, const int64_t* toff, int32_t m, int64_t ldc,
                           double* out, int64_t ldo, hipStream_t s);
// Out_i = Linv_i In_i for every block on the vector units (tiles: (blk, ta, tc)).
hipError_t launch_trmm(const double* In, double* Out, int64_t ldc, const int64_t* off,
                       const int32_t* tiles, int32_t ntiles, const int64_t* goff,
                       const double* Linv, hipStream_t s);
// dst[j*ldd + c] = src[c*lds + j] for j < n, c < k.
hipError_t launch_copy_t(const double* src, int64_t lds, double* dst, int64_t ldd, int64_t n,
                         int32_t k, hipStream_t s);
hipError_t launch_cast_f32(const double* src, float* dst, int64_t count, hipStream_t s);
// C <- A (N x n, row stride lda) in FP32 (f32 != 0) or FP64, zero-padded to ldc.
hipError_t launch_pad_cast(int f32, const double* A, int64_t lda, int64_t N, int64_t n, void* C,
                           int64_t ldc, hipStream_t s);
// Heavy-ball step: g = sum_i Y_i (block order), z <- beta z + g, x <- x - alpha z.
hipError_t launch_hbm_step(const double* Y, int64_t ldy, int32_t m, int64_t n, double alpha,
                           double beta, double* x, double* z, hipStream_t s);
hipError_t launch_fill_u32(unsigned* p, int64_t count, unsigned v, hipStream_t s);
hipError_t launch_copy_strided(const double* src, int64_t lds, double* dst, int64_t ldd,
                               int64_t rows, int64_t cols, hipStream_t s);

// One Lanczos step after the operator (twice classical Gram-Schmidt of w
// against V's rows 0..j, alpha_j, beta_j, V[j + 1] = w / beta_j), over column
// slabs of kLzSlab.  w is the operator's output, or, when part is non-null,
// scale * (the sum of ntiles partial rows of stride ldp, FP32 when part32).
constexpr int kLzSlab = 64;
constexpr int kLzMaxRows = 1024;  // basis rows a step can reorthogonalise against
struct LanczosArgs {
  const double* V;  // basis rows 0..j, row stride ldc
  int64_t ldc;
  int32_t j;
  int32_t nslab;    // ceil(ldc / kLzSlab)
  double* w;        // ldc entries, overwritten by the reorthogonalised vector
  double* hp;       // dot partials: pass q, slab s, row r at hp[(q * nslab + s) * hstride + r]
  int64_t hstride;  // >= j + 1
  double* np;       // nslab norm partials
  double* alpha;
  double* beta;
  double* vnext;    // V's row j + 1
  float* vnext32;   // optional FP32 copy of vnext
  double* host_ab;  // optional (host memory the device can write): alpha_j at [j], beta_j at [hstride + j]
};
hipError_t launch_lanczos_step(const LanczosArgs& a, const void* part, bool part32, int64_t ldp,
                               int32_t ntiles, double scale, hipStream_t s);
// v = the normalised splitmix64 start vector of n entries (zero up to ldc),
// and its FP32 rounding in v32 when non-null.
hipError_t launch_lanczos_start(uint64_t seed, int64_t n, int64_t ldc, double* v, float* v32,
                                hipStream_t s);

// ---------------------------------------------------------------------------
// Residual monitor (FP64)
// ---------------------------------------------------------------------------

// partial[t] = sum over rows of tile t of (b_r - a_r . x)^2 (x may be null: x = 0).
hipError_t launch_residual_partial(const double* A, int64_t lda, const double* B, int64_t ldb,
                                   int64_t N, int64_t n, const double* x, double* partial,
                                   int32_t* nparts, hipStream_t s);
// out[0] = sum_t partial[t] (fixed order).
hipError_t launch_sum_partials(const double* partial, int32_t count, double* out, hipStream_t s);

int residual_parts(int64_t N);

// ---------------------------------------------------------------------------
// Host-side helpers shared with entry points outside apc_host.cpp
// ---------------------------------------------------------------------------

// Sets the thread-local message of apc_last_error and returns st.
apc_status report(apc_status st, const char* fmt, ...);
// The device a plan was set up on.
int plan_device(const apc_plan_s* p);

// The allocation-free adjoint's fixed scratch (apc_noalloc.hip): its size, the
// one-time lookup of this device's copy (the device must be current), and the
// address found (NULL before the lookup).
size_t noalloc_scratch_bytes();
hipError_t noalloc_scratch_init(int device);
void* noalloc_scratch(int device);

}  // namespace apc
