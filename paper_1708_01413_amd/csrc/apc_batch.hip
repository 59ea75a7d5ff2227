// Many independent systems (k = 1 each), one persistent launch per pass.
//
// Every system keeps its own factor, local solutions and average in its own
// plan's workspace; a descriptor array points at them.  A pass is one launch
// over a work list that covers all systems: the grid is a fixed number of
// workgroups (chosen by timing), each looping over items i = blockIdx.x,
// blockIdx.x + gridDim.x, ...  Items of a system whose `active` flag is 0 are
// skipped, so converged systems stop costing bandwidth.
//
// Per update (eq. (2a)-(2b) for every system), when every plan updates in one
// pass and rows are at most 1024 wide:
//   single pass  items (system, row tile of one block): w_r = C_r . d_i and the
//                tile's partial row sum_r w_r C_r, one read of the factor
//   combine      items (system, 32 columns): x_i += gamma (x_bar - x_i - Q_i w_i),
//                x_bar <- (eta/m) sum_i x_i + (1-eta) x_bar, d_i = x_bar - x_i
// otherwise in two passes:
//   pass A   items (system, 16-row tile of one block): w_r = C_r . d_i
//   pass B   items (system, block, 256-column slab):   x_i += gamma (x_bar - x_i - Q_i w_i)
//   average  items (system, 256-column chunk):          x_bar <- (eta/m) sum_i x_i + (1-eta) x_bar,
//                                                       d_i = x_bar - x_i
// The arithmetic per system is the single-system k = 1 path's.

#include <hip/hip_runtime.h>

#include "apc_internal.h"
#include "apc_tn.h"

namespace apc {

namespace {

template <typename TQ>
__device__ inline float4 ld4(const TQ* p);
template <>
__device__ inline float4 ld4<float>(const float* p) { return *reinterpret_cast<const float4*>(p); }

// The factor is read once per pass: non-temporal loads.
typedef float bf32x4 __attribute__((ext_vector_type(4)));
__device__ inline float4 ld4_nt(const float* p) {
  const bf32x4 v = __builtin_nontemporal_load(reinterpret_cast<const bf32x4*>(p));
  return make_float4(v[0], v[1], v[2], v[3]);
}

template <typename T>
__device__ inline T wsum64(T v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Pass A: wave v takes rows v, v + 4, v + 8, v + 12 of the item's tile (up to
// 16 rows), with all its rows' loads in flight together.  Rows past the tile
// repeat the wave's first row and are not stored.
template <typename TQ>
__global__ __launch_bounds__(256) void k_batch_pass_a(const BatchSys* sys, const int4* items,
                                                      int32_t nitems, const int32_t* active) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  for (int32_t it = blockIdx.x; it < nitems; it += gridDim.x) {
    const int4 w = items[it];
    if (!active[w.x]) continue;
    if (wv >= w.z) continue;  // uniform per wave
    const BatchSys& S = sys[w.x];
    const TQ* C = static_cast<const TQ*>(S.C);
    const TQ* d = static_cast<const TQ*>(S.d) + static_cast<int64_t>(w.w) * S.ldc;
    TQ* out = static_cast<TQ*>(S.w);
    const int64_t r0 = w.y + wv;
    const TQ* row[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) row[q] = C + (wv + 4 * q < w.z ? r0 + 4 * q : r0) * S.ldc;
    TQ acc[4] = {0, 0, 0, 0};
    for (int64_t j = static_cast<int64_t>(lane) * 4; j < S.n; j += 256) {
      if (j + 4 <= S.n) {
        const float4 v = ld4(d + j);
        float4 c[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) c[q] = ld4_nt(row[q] + j);
#pragma unroll
        for (int q = 0; q < 4; ++q) acc[q] += c[q].x * v.x + c[q].y * v.y + c[q].z * v.z + c[q].w * v.w;
      } else {
        for (int64_t e = j; e < S.n; ++e)
#pragma unroll
          for (int q = 0; q < 4; ++q) acc[q] += row[q][e] * d[e];
      }
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) acc[q] = wsum64(acc[q]);
    if (lane == 0) {
#pragma unroll
      for (int q = 0; q < 4; ++q)
        if (wv + 4 * q < w.z) out[r0 + 4 * q] = acc[q];
    }
  }
}

// Pass B: lane l owns 4 columns of the item's 256-column slab; the 4 waves
// take interleaved rows of the block (4 rows in flight per wave) and combine
// in LDS; then one thread per column applies the FP64 update.
template <typename TQ>
__global__ __launch_bounds__(256) void k_batch_pass_b(const BatchSys* sys, const int4* items,
                                                      int32_t nitems, const int32_t* active) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  __shared__ float red[4][256];
  for (int32_t it = blockIdx.x; it < nitems; it += gridDim.x) {
    const int4 w = items[it];
    if (!active[w.x]) continue;  // uniform per workgroup
    const BatchSys& S = sys[w.x];
    const int blk = w.y;
    const int64_t r0 = S.off[blk], r1 = S.off[blk + 1];
    const int64_t j = w.z + static_cast<int64_t>(lane) * 4;
    const TQ* C = static_cast<const TQ*>(S.C);
    const TQ* wvec = static_cast<const TQ*>(S.w);
    float acc[4] = {0.f, 0.f, 0.f, 0.f};
    if (j + 4 <= S.ldc) {  // rows are padded to ldc (zeros past n)
      int64_t r = r0 + wv;
      for (; r + 12 < r1; r += 16) {
        const float4 c0 = ld4_nt(C + r * S.ldc + j), c1 = ld4_nt(C + (r + 4) * S.ldc + j);
        const float4 c2 = ld4_nt(C + (r + 8) * S.ldc + j), c3 = ld4_nt(C + (r + 12) * S.ldc + j);
        const float s0 = wvec[r], s1 = wvec[r + 4], s2 = wvec[r + 8], s3 = wvec[r + 12];
        acc[0] += (c0.x * s0 + c1.x * s1) + (c2.x * s2 + c3.x * s3);
        acc[1] += (c0.y * s0 + c1.y * s1) + (c2.y * s2 + c3.y * s3);
        acc[2] += (c0.z * s0 + c1.z * s1) + (c2.z * s2 + c3.z * s3);
        acc[3] += (c0.w * s0 + c1.w * s1) + (c2.w * s2 + c3.w * s3);
      }
      for (; r < r1; r += 4) {
        const float4 c0 = ld4_nt(C + r * S.ldc + j);
        const float s0 = wvec[r];
        acc[0] += c0.x * s0;
        acc[1] += c0.y * s0;
        acc[2] += c0.z * s0;
        acc[3] += c0.w * s0;
      }
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) red[wv][lane * 4 + q] = acc[q];
    __syncthreads();
    const int64_t jc = w.z + threadIdx.x;
    if (jc < S.n) {
      const float t = (red[0][threadIdx.x] + red[1][threadIdx.x]) +
                      (red[2][threadIdx.x] + red[3][threadIdx.x]);
      double* x = S.x + static_cast<int64_t>(blk) * S.ldc;
      const double xi = x[jc];
      x[jc] = xi + S.gamma * (S.xbar[jc] - xi - static_cast<double>(t));
    }
    __syncthreads();
  }
}

// Average, and the next differences.
template <typename TQ>
__global__ __launch_bounds__(256) void k_batch_average(const BatchSys* sys, const int2* items,
                                                       int32_t nitems, const int32_t* active) {
  for (int32_t it = blockIdx.x; it < nitems; it += gridDim.x) {
    const int2 w = items[it];
    if (!active[w.x]) continue;
    const BatchSys& S = sys[w.x];
    const int64_t j = w.y + threadIdx.x;
    if (j >= S.n) continue;
    double s = 0.0;
    for (int i = 0; i < S.m; ++i) s += S.x[static_cast<int64_t>(i) * S.ldc + j];
    const double xb = (S.eta / S.m) * s + (1.0 - S.eta) * S.xbar[j];
    S.xbar[j] = xb;
    TQ* d = static_cast<TQ*>(S.d);
    for (int i = 0; i < S.m; ++i)
      d[static_cast<int64_t>(i) * S.ldc + j] =
          static_cast<TQ>(xb - S.x[static_cast<int64_t>(i) * S.ldc + j]);
  }
}

// Single pass over one row tile of one system: w_r = C_r . d_blk for each row
// and the tile's partial row sum_r w_r C_r.  Lane l holds the 16-byte chunks
// l, l + 64, ... (CPL of them: rows up to 256 CPL wide), so a row's dot product
// needs only a wave sum.  A wave takes RF = 16 / CPL rows at a time (rows
// wv, wv + 4, ...), all their loads in flight, so short rows still keep 16
// loads per lane in flight.  The four waves' partial rows are added in LDS.
// Global-address-space view of a pointer read from a descriptor (its address
// space is otherwise unknown and the loads become flat loads).
typedef float g_f32x4 __attribute__((ext_vector_type(4)));
__device__ inline const __attribute__((address_space(1))) g_f32x4* gptr4(const float* p) {
  return reinterpret_cast<const __attribute__((address_space(1))) g_f32x4*>(
      reinterpret_cast<uintptr_t>(p));
}

template <int CPL, int INFLIGHT = 16>
__device__ __attribute__((always_inline)) inline void batch_tile_pass(const BatchSys& S, int64_t row0,
                                                                      int nrows, int blk,
                                                                      float (&red)[4][kBatchFusedCols]) {
  constexpr int RF = INFLIGHT / CPL;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const float* C = static_cast<const float*>(S.C);
  const float* d = static_cast<const float*>(S.d) + static_cast<int64_t>(blk) * S.ldc;
  // Every load below is issued without a branch: a chunk past the row (the
  // row stride ldc is a multiple of 64, so only lanes past ldc) reads the
  // row's last chunk, a row past the tile reads the tile's first row, and
  // their contributions are zeroed by selects (entries of d past n, the dot
  // products of such rows).  A load behind a branch makes the compiler wait
  // for every load in flight where the paths join.
  int64_t jc[CPL];
  float dv[CPL][4], acc[CPL][4];
#pragma unroll
  for (int c = 0; c < CPL; ++c) {
    const int64_t j = static_cast<int64_t>(lane + 64 * c) * 4;
    jc[c] = j < S.ldc ? j : S.ldc - 4;
    const g_f32x4 v = *gptr4(d + jc[c]);
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      dv[c][e] = j + e < S.n ? v[e] : 0.f;
      acc[c][e] = 0.f;
    }
  }
  for (int r = wv; r < nrows; r += 4 * RF) {
    g_f32x4 row[RF][CPL];
#pragma unroll
    for (int q = 0; q < RF; ++q) {
      const int64_t rr = row0 + (r + 4 * q < nrows ? r + 4 * q : 0);
#pragma unroll
      for (int c = 0; c < CPL; ++c) row[q][c] = __builtin_nontemporal_load(gptr4(C + rr * S.ldc + jc[c]));
    }
#pragma unroll
    for (int q = 0; q < RF; ++q) {
      float s = 0.f;
#pragma unroll
      for (int c = 0; c < CPL; ++c)
        s += (row[q][c][0] * dv[c][0] + row[q][c][1] * dv[c][1]) +
             (row[q][c][2] * dv[c][2] + row[q][c][3] * dv[c][3]);
      s = wave_sum_dpp(s);
      s = r + 4 * q < nrows ? s : 0.f;
#pragma unroll
      for (int c = 0; c < CPL; ++c)
#pragma unroll
        for (int e = 0; e < 4; ++e) acc[c][e] = fmaf(s, row[q][c][e], acc[c][e]);
    }
  }
#pragma unroll
  for (int c = 0; c < CPL; ++c)
#pragma unroll
    for (int e = 0; e < 4; ++e) red[wv][(lane + 64 * c) * 4 + e] = acc[c][e];
}

// One single-pass item: tile t of system S, its partial row written, with
// INFLIGHT 16-byte loads per lane in flight (16 measured best, also in the
// mixed kernel: 8 took 342 against 333 us per update of the 8192^2 k = 64
// system with the 256 systems).
template <int INFLIGHT = 16>
__device__ __attribute__((always_inline)) inline void fused_item(const BatchSys& S, int t, int64_t row0,
                                                                 int nrows, int blk,
                                                                 float (&red)[4][kBatchFusedCols]) {
  if (S.ldc <= 256) batch_tile_pass<1, INFLIGHT>(S, row0, nrows, blk, red);
  else if (S.ldc <= 512) batch_tile_pass<2, INFLIGHT>(S, row0, nrows, blk, red);
  else batch_tile_pass<4, INFLIGHT>(S, row0, nrows, blk, red);
  __syncthreads();
  float* out = S.part + static_cast<int64_t>(t) * S.ldc;
  for (int64_t j = threadIdx.x; j < S.ldc; j += 256)
    out[j] = (red[0][j] + red[1][j]) + (red[2][j] + red[3][j]);
  __syncthreads();
}

// The same with the tile's rows and block read from the system's tile lists.
template <int INFLIGHT = 16>
__device__ __attribute__((always_inline)) inline void fused_item(const BatchSys& S, int t,
                                                                 float (&red)[4][kBatchFusedCols]) {
  fused_item<INFLIGHT>(S, t, S.tiles[t], S.tiles[S.ntiles + t], S.tiles[2 * S.ntiles + t], red);
}

// Items (sys, row tile of the batch's tiles for that system, the tile's first
// row, (rows - 1) | block << 8): the tile's partial row, for rows up to
// kBatchFusedCols wide.  The item carries the tile so that its rows' loads
// wait only for the item and the system's descriptor.
__global__ __launch_bounds__(256) void k_batch_fused(const BatchSys* sys, const int4* items,
                                                     int32_t nitems, const int32_t* active) {
  __shared__ float red[4][kBatchFusedCols];
  for (int32_t it = blockIdx.x; it < nitems; it += gridDim.x) {
    const int4 w = items[it];
    if (!active[w.x]) continue;  // uniform per workgroup
    fused_item(sys[w.x], w.y, w.z, (w.w & 0xff) + 1, static_cast<int>(static_cast<uint32_t>(w.w) >> 8), red);
  }
}

// After k_batch_fused, items (sys, first of 64 columns): lane l of wave w
// takes column l and the blocks i = w (mod 4) -- x_i += gamma (x_bar - x_i -
// sum of block i's partial rows), x_bar <- (eta/m) sum_i x_i + (1 - eta)
// x_bar, d_i = x_bar - x_i.  A lane's blocks are loaded four at a time (their
// x_i and first four partial rows, clamped addresses and selects), and with
// m <= 16 their new x_i stay in registers for the differences.  A block's
// partial rows are added in tile order.
__device__ __attribute__((always_inline)) inline void combine_item(const BatchSys& S, int col,
                                                                   double (&part)[4][64],
                                                                   double (&xb)[64]) {
  constexpr int U = 4;
  const int lane = threadIdx.x & 63;
  const int bl = threadIdx.x >> 6;
  const int64_t j = col + lane;
  const bool ok = j < S.n;
  const int64_t jc = ok ? j : col;  // col < n
  double* x = S.x;
  const double xo = S.xbar[jc];
  const bool one = S.m <= 4 * U;
  double keep[U];
  double s = 0.0;
  for (int i0 = bl; i0 < S.m; i0 += 4 * U) {
    double xi[U];
    float v[U][4];
    int t0[U], t1[U];
#pragma unroll
    for (int q = 0; q < U; ++q) {
      const int i = i0 + 4 * q;
      const int ic = i < S.m ? i : i0;
      t0[q] = S.tile_first[ic];
      t1[q] = S.tile_first[ic + 1];
      xi[q] = x[static_cast<int64_t>(ic) * S.ldc + jc];
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const int t = min(t0[q] + k, t1[q] - 1);  // every block has a tile
        v[q][k] = S.part[static_cast<int64_t>(t) * S.ldc + jc];
      }
    }
#pragma unroll
    for (int q = 0; q < U; ++q) {
      const int i = i0 + 4 * q;
      double u = 0.0;
#pragma unroll
      for (int k = 0; k < 4; ++k) u += t0[q] + k < t1[q] ? static_cast<double>(v[q][k]) : 0.0;
      for (int t = t0[q] + 4; t < t1[q]; ++t)  // blocks of more than four tiles
        u += static_cast<double>(S.part[static_cast<int64_t>(t) * S.ldc + jc]);
      const double xn = xi[q] + S.gamma * ((xo - xi[q]) - u);
      keep[q] = xn;
      if (i < S.m && ok) {
        x[static_cast<int64_t>(i) * S.ldc + j] = xn;
        s += xn;
      }
    }
  }
  part[bl][lane] = s;
  __syncthreads();
  if (bl == 0 && ok) {
    const double tot = (part[0][lane] + part[1][lane]) + (part[2][lane] + part[3][lane]);
    const double v = (S.eta / S.m) * tot + (1.0 - S.eta) * S.xbar[j];
    S.xbar[j] = v;
    xb[lane] = v;
  }
  __syncthreads();
  if (ok) {
    float* d = static_cast<float*>(S.d);
    const double v = xb[lane];
    for (int i0 = bl; i0 < S.m; i0 += 4 * U) {
#pragma unroll
      for (int q = 0; q < U; ++q) {
        const int i = i0 + 4 * q;
        if (i < S.m) {
          const double xi = one ? keep[q] : x[static_cast<int64_t>(i) * S.ldc + j];
          d[static_cast<int64_t>(i) * S.ldc + j] = static_cast<float>(v - xi);
        }
      }
    }
  }
  __syncthreads();
}

__global__ __launch_bounds__(256) void k_batch_fused_combine(const BatchSys* sys, const int2* items,
                                                             int32_t nitems, const int32_t* active) {
  __shared__ double part[4][64];
  __shared__ double xb[64];
  for (int32_t it = blockIdx.x; it < nitems; it += gridDim.x) {
    const int2 w = items[it];
    if (!active[w.x]) continue;  // uniform per workgroup
    combine_item(sys[w.x], w.y, part, xb);
  }
}

// Residual partials: partial[item] = sum over the tile's rows of (b_r - a_r . x_bar)^2.
__global__ __launch_bounds__(256) void k_batch_resid(const BatchSys* sys, const int4* items,
                                                     int32_t nitems, const int32_t* active,
                                                     double* partial) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  __shared__ double ws[4];
  for (int32_t it = blockIdx.x; it < nitems; it += gridDim.x) {
    const int4 w = items[it];
    if (!active[w.x]) continue;  // uniform per workgroup
    const BatchSys& S = sys[w.x];
    double acc = 0.0;
    for (int rr = wv; rr < w.z; rr += 4) {
      const int64_t r = w.y + rr;
      const double* a = S.A + r * S.lda;
      double dot = 0.0;
      for (int64_t j = lane; j < S.n; j += 64) dot += a[j] * S.xbar[j];
      dot = wsum64(dot);
      const double res = S.b[r * S.ldb] - dot;
      acc += res * res;
    }
    if (lane == 0) ws[wv] = acc;
    __syncthreads();
    if (threadIdx.x == 0) partial[it] = (ws[0] + ws[1]) + (ws[2] + ws[3]);
    __syncthreads();
  }
}

// Per system: relres = sqrt(sum of its items' partials) / ||b||; a system whose
// relres <= rtol, or is not finite (it diverged), is deactivated.  One thread
// per system.
__global__ void k_batch_check(const BatchSys* sys, int32_t count, const int32_t* item_start,
                              const double* partial, double rtol, int32_t* active,
                              double* relres) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= count) return;
  if (!active[s]) return;
  double t = 0.0;
  for (int32_t i = item_start[s]; i < item_start[s + 1]; ++i) t += partial[i];
  const double bn = sys[s].bnorm;
  const double rr = bn > 0.0 ? sqrt(t) / bn : sqrt(t);
  relres[s] = rr;
  if (!(rr > rtol) || !isfinite(rr)) active[s] = 0;
}

// One launch of a mixed batch: every workgroup loops over the work list and
// runs each item with the matching device function (the contraction tile of
// k_tn with 64-row tiles, two steps of prefetch; the k = 1 single-pass tile
// and combine of the batch kernels above; the elementwise epilogues).  The
// item kinds share one LDS buffer.  Registers are capped for two workgroups
// per CU (one otherwise: 326 against 338 us per update for the 8192^2 k = 64
// system with the 256 systems; four steps of prefetch took 345; the k = 1
// tile as a called function instead of inlined, 395).
template <int NCT>
__global__ __launch_bounds__(256, 2) void k_batch_mixed(const BatchSys* sys, const BatchGemm* gemm,
                                                     const int4* items, int32_t nitems,
                                                     const int32_t* active) {
  constexpr size_t kTn = sizeof(TnStage<NCT>);
  constexpr size_t kRed = sizeof(float) * 4 * kBatchFusedCols;
  constexpr size_t kBytes = kTn > kRed ? kTn : kRed;
  __shared__ __attribute__((aligned(16))) unsigned char lds[kBytes];
  for (int32_t it = blockIdx.x; it < nitems; it += gridDim.x) {
    const int4 w = items[it];
    if (!active[w.x >> 8]) continue;  // uniform per workgroup
    const int kind = w.x & 0xff;
    if (kind == kItemFused) {
      fused_item(sys[w.y], w.z, *reinterpret_cast<float(*)[4][kBatchFusedCols]>(lds));
    } else if (kind == kItemCombine) {
      combine_item(sys[w.y], w.z, *reinterpret_cast<double(*)[4][64]>(lds),
                   *reinterpret_cast<double(*)[64]>(lds + sizeof(double) * 4 * 64));
    } else if (kind == kItemTn32 || kind == kItemTn64) {
      const TnArgs a = gemm[w.y].tn[w.z];
      // (The FP64 contraction, an anchor update's, loads one step ahead: with
      // two the kernel's union of work kinds spilled registers.)
      if (kind == kItemTn32)
        tn_block<float, 1, NCT, 2, 1>(a, w.w, *reinterpret_cast<TnStage<NCT>*>(lds));
      else
        tn_block<double, 1, NCT, 1, 0>(a, w.w, *reinterpret_cast<TnStage<NCT>*>(lds));
      __syncthreads();
    } else {
      // Elementwise items, four consecutive entries per thread: every row
      // length and stride of a k-RHS plan's operands is a multiple of 256
      // and every slice 256-byte aligned.
      const BatchGemm& G = gemm[w.y];
      const int64_t e0 = static_cast<int64_t>(w.w) * kBatchChunk;
      if (kind == kItemSum32 || kind == kItemSum64) {
        const int64_t total = static_cast<int64_t>(G.kp) * G.sum_rows;
        const int64_t e1 = min(total, e0 + kBatchChunk);
        const int64_t stride = static_cast<int64_t>(G.kp) * G.sum_ldp;
        for (int64_t e = e0 + 4 * threadIdx.x; e < e1; e += 4 * 256) {
          if (kind == kItemSum32)
            sum_cast4(static_cast<const float*>(G.sum_part), G.sum_nsplit[0], G.sum_ldp, G.sum_rows,
                      stride, static_cast<float*>(G.sum_out[0]), G.sum_ldo, e);
          else
            sum_cast4(static_cast<const double*>(G.sum_part), G.sum_nsplit[1], G.sum_ldp,
                      G.sum_rows, stride, static_cast<double*>(G.sum_out[1]), G.sum_ldo, e);
        }
      } else if (kind == kItemUpd32 || kind == kItemUpd64) {
        const TnUpdateArgs& u = G.upd[kind == kItemUpd64 ? 1 : 0];
        const int64_t e1 = min(static_cast<int64_t>(u.kp) * u.n, e0 + kBatchChunk);
        for (int64_t e = e0 + 4 * threadIdx.x; e < e1; e += 4 * 256) {
          if (kind == kItemUpd32) update4<float, float>(u, e);
          else update4<double, float>(u, e);
        }
      } else if (kind == kItemAnchorVec) {
        const int64_t e1 = min(G.state_count, e0 + kBatchChunk);
        for (int64_t e = e0 + 4 * threadIdx.x; e < e1; e += 4 * 256) {
          double y[4], xb[4], r[4];
          load4(G.y + e, y);
          load4(G.xbar + e, xb);
#pragma unroll
          for (int q = 0; q < 4; ++q) r[q] = (1.0 - G.gamma) * y[q] + G.gamma * xb[q];
          store4(G.yref + e, r);
        }
      }
    }
  }
}

}  // namespace

hipError_t launch_batch_mixed(int32_t grid, int32_t nct, const BatchSys* sys, const BatchGemm* gemm,
                              const int4* items, int32_t nitems, const int32_t* active,
                              hipStream_t s) {
  if (nitems <= 0) return hipSuccess;
  switch (nct) {
    case 1: k_batch_mixed<1><<<grid, 256, 0, s>>>(sys, gemm, items, nitems, active); break;
    case 2: k_batch_mixed<2><<<grid, 256, 0, s>>>(sys, gemm, items, nitems, active); break;
    case 4: k_batch_mixed<4><<<grid, 256, 0, s>>>(sys, gemm, items, nitems, active); break;
    case 8: k_batch_mixed<8><<<grid, 256, 0, s>>>(sys, gemm, items, nitems, active); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_batch_pass_a(int f64, int32_t grid, const BatchSys* sys, const int4* items,
                               int32_t nitems, const int32_t* active, hipStream_t s) {
  if (f64) return hipErrorInvalidValue;
  k_batch_pass_a<float><<<grid, 256, 0, s>>>(sys, items, nitems, active);
  return hipGetLastError();
}

hipError_t launch_batch_pass_b(int f64, int32_t grid, const BatchSys* sys, const int4* items,
                               int32_t nitems, const int32_t* active, hipStream_t s) {
  if (f64) return hipErrorInvalidValue;
  k_batch_pass_b<float><<<grid, 256, 0, s>>>(sys, items, nitems, active);
  return hipGetLastError();
}

hipError_t launch_batch_average(int f64, int32_t grid, const BatchSys* sys, const int2* items,
                                int32_t nitems, const int32_t* active, hipStream_t s) {
  if (f64) return hipErrorInvalidValue;
  k_batch_average<float><<<grid, 256, 0, s>>>(sys, items, nitems, active);
  return hipGetLastError();
}

hipError_t launch_batch_fused(int32_t grid, const BatchSys* sys, const int4* items, int32_t nitems,
                              const int32_t* active, hipStream_t s) {
  k_batch_fused<<<grid, 256, 0, s>>>(sys, items, nitems, active);
  return hipGetLastError();
}

hipError_t launch_batch_fused_combine(int32_t grid, const BatchSys* sys, const int2* items,
                                      int32_t nitems, const int32_t* active, hipStream_t s) {
  k_batch_fused_combine<<<grid, 256, 0, s>>>(sys, items, nitems, active);
  return hipGetLastError();
}

hipError_t launch_batch_resid(int32_t grid, const BatchSys* sys, const int4* items, int32_t nitems,
                              const int32_t* active, double* partial, hipStream_t s) {
  k_batch_resid<<<grid, 256, 0, s>>>(sys, items, nitems, active, partial);
  return hipGetLastError();
}

hipError_t launch_batch_check(const BatchSys* sys, int32_t count, const int32_t* item_start,
                              const double* partial, double rtol, int32_t* active, double* relres,
                              hipStream_t s) {
  k_batch_check<<<(count + 255) / 256, 256, 0, s>>>(sys, count, item_start, partial, rtol, active,
                                                    relres);
  return hipGetLastError();
}

}  // namespace apc
