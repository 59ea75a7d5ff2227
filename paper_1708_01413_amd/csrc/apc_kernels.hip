// HIP kernels (gfx950, wave64) for Accelerated Projection-based Consensus.
//
// Hot path, per update of eq. (2a)-(2b):
//   pass A  (k_rowdot)  w_i = Q_i^T d_i, d_i = x_bar - x_i: one dot product
//           per row of the stacked factor C = [Q_1^T; ...; Q_m^T] (N x ldc,
//           row-major), streamed once with 16-byte loads, the difference
//           vector held in registers, one wave-level reduction per row.
//   pass B  (k_pass_b)  x_i += gamma (x_bar - x_i - Q_i w_i): each workgroup
//           owns a 4 KB column slab of one block and streams that block's
//           rows once.
//   average (k_combine) x_bar <- (eta/m) sum_i x_i + (1 - eta) x_bar in a
//           fixed summation order, and d_i = x_bar - x_i for the next pass A.
// Both passes are HBM-bound (one FMA per streamed element), so they are
// written for coalescing and memory-level parallelism, not for MFMA.  The
// average is a launch of its own: folding it into pass B's epilogue needs a
// device-scope release per workgroup, which on a multi-XCD part writes back
// L2 and measured slower than the extra launch.
//
// Setup (FP64): CholeskyQR2 of every A_i^T -- Gram G_i = C_i C_i^T (LDS-tiled),
// per-block Cholesky + triangular inverse, C_i <- L_i^{-1} C_i -- applied
// twice; then x_i(0) = Q_i c_i and x_bar(0) = mean (Alg. 1 initialisation).

#include <hip/hip_runtime.h>

#include "apc_internal.h"

namespace apc {

namespace {

// ------------------------------------------------------------------ helpers

// 16-byte loads of the streamed factor.  Every element of C is read once per
// pass, so the loads are non-temporal: they do not displace the vectors that
// are reused (d_i, w, x_bar) from the caches, and streaming reads measured
// ~7.0 TB/s this way against ~6.3 TB/s with ordinary loads.
typedef float f32x4_t __attribute__((ext_vector_type(4)));
typedef double f64x2_t __attribute__((ext_vector_type(2)));
typedef double f64x4 __attribute__((ext_vector_type(4)));
template <typename T>
struct V16;
template <>
struct V16<float> {
  static constexpr int W = 4;
  template <bool NT = true>
  __device__ static inline void load(const float* p, float (&o)[4]) {
    const f32x4_t* q = reinterpret_cast<const f32x4_t*>(p);
    const f32x4_t v = NT ? __builtin_nontemporal_load(q) : *q;
    o[0] = v[0]; o[1] = v[1]; o[2] = v[2]; o[3] = v[3];
  }
};
template <>
struct V16<double> {
  static constexpr int W = 2;
  template <bool NT = true>
  __device__ static inline void load(const double* p, double (&o)[2]) {
    const f64x2_t* q = reinterpret_cast<const f64x2_t*>(p);
    const f64x2_t v = NT ? __builtin_nontemporal_load(q) : *q;
    o[0] = v[0]; o[1] = v[1];
  }
};

template <typename T>
__device__ inline T wave_sum(T v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

inline unsigned grid_for(int64_t work, int per) {
  int64_t g = (work + per - 1) / per;
  if (g < 1) g = 1;
  return static_cast<unsigned>(g);
}

// ------------------------------------------------------------------ pass A

// One workgroup per (row tile, column split).  The difference vector d of the
// tile's block is held in registers one chunk (U sweeps of 256 x 16 B) at a
// time; every row of the tile is streamed with 16-byte loads against it.
template <typename TQ, typename TA, int ROWS, int U, bool NT>
__global__ __launch_bounds__(kThreads) void k_rowdot(RowdotArgs<TQ, TA> a) {
  constexpr int W = V16<TQ>::W;
  constexpr int SWEEP = kThreads * W;
  constexpr int CH = SWEEP * U;

  const int total = a.ntiles * a.nsplit;
  int q = blockIdx.x;
  if (a.xcd_remap == 1) {
    const int per = (total + kXcds - 1) / kXcds;
    q = (blockIdx.x % kXcds) * per + blockIdx.x / kXcds;
  } else if (a.xcd_remap == 2) {
    q = total - 1 - static_cast<int>(blockIdx.x);
  }
  if (q < 0 || q >= total) return;
  const int Lrel = q / a.nsplit;
  const int split = q - Lrel * a.nsplit;
  const int L = a.tile_begin + Lrel;
  int row0, nrows, blk;
  if (a.tile_row0) {
    row0 = a.tile_row0[L];
    nrows = a.tile_nrows[L];
    blk = a.tile_blk[L];
  } else {
    row0 = Lrel * ROWS;
    nrows = min(ROWS, a.rows_total - row0);
    blk = 0;
  }
  const int64_t c0 = static_cast<int64_t>(split) * a.split_cols;
  const int64_t c1 = min(a.ldc, c0 + a.split_cols);
  const double* vb = a.vb ? a.vb + static_cast<int64_t>(blk) * a.ldvb : nullptr;
  const TA* dblk = a.d ? a.d + static_cast<int64_t>(blk) * a.ldd : nullptr;
  const int tcol = threadIdx.x * W;

  TA acc[ROWS];
#pragma unroll
  for (int r = 0; r < ROWS; ++r) acc[r] = TA(0);

  for (int64_t base = c0; base < c1; base += CH) {
    TA d[U][W];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int64_t j = base + u * SWEEP + tcol;
      if (dblk) {
#pragma unroll
        for (int e = 0; e < W; ++e) d[u][e] = j < c1 ? dblk[j + e] : TA(0);
      } else {
#pragma unroll
        for (int e = 0; e < W; ++e) {
          double v = 0.0;
          if (j < c1) {
            v = a.va ? a.va[j + e] : 0.0;
            if (vb) v -= vb[j + e];
          }
          d[u][e] = static_cast<TA>(v);
        }
      }
    }
#pragma unroll
    for (int r = 0; r < ROWS; ++r) {
      if (r < nrows) {
        const TQ* crow = a.C + static_cast<int64_t>(row0 + r) * a.ldc;
#pragma unroll
        for (int u = 0; u < U; ++u) {
          const int64_t j = base + u * SWEEP + tcol;
          if (j < c1) {
            TQ qv[W];
            V16<TQ>::template load<NT>(crow + j, qv);
#pragma unroll
            for (int e = 0; e < W; ++e) acc[r] = fma(static_cast<TA>(qv[e]), d[u][e], acc[r]);
          }
        }
      }
    }
  }

  __shared__ TA red[kThreads / 64][ROWS];
  const int lane = threadIdx.x & 63;
  const int wv = threadIdx.x >> 6;
#pragma unroll
  for (int r = 0; r < ROWS; ++r) {
    const TA v = wave_sum(acc[r]);
    if (lane == 0) red[wv][r] = v;
  }
  __syncthreads();
  if (static_cast<int>(threadIdx.x) < nrows) {
    const int r = threadIdx.x;
    a.out[static_cast<int64_t>(split) * a.out_stride + row0 + r] =
        (red[0][r] + red[1][r]) + (red[2][r] + red[3][r]);
  }
}

// ------------------------------------------------------------------ pass B

// One workgroup per (block i, 256 x 16-byte column slab): every wave streams
// all rows of the block over its own 64 x 16 B of the slab, so each row read
// by the workgroup is 4 KB contiguous and no cross-wave combine is needed.
// w_r is the sum of pass A's column-split partials, added in split order.
// NT selects non-temporal loads of C.
template <typename TQ, int RU, bool NT>
__global__ __launch_bounds__(kThreads) void k_pass_b(PassBArgs<TQ> a) {
  constexpr int W = V16<TQ>::W;
  constexpr int SW = kThreads * W;  // columns per slab
  const int s = blockIdx.x % a.nslab;
  const int i = a.blk_begin + static_cast<int>(blockIdx.x / a.nslab);
  const int64_t r0 = a.off[i];
  const int64_t r1 = a.off[i + 1];
  const int64_t col = static_cast<int64_t>(s) * SW + threadIdx.x * W;
  if (col >= a.ldc) return;

  auto coef = [&](int64_t r) {
    TQ v = a.w[r];
    for (int sp = 1; sp < a.nsplit; ++sp) v += a.w[sp * a.w_stride + r];
    return v;
  };
  TQ acc[W];
#pragma unroll
  for (int e = 0; e < W; ++e) acc[e] = TQ(0);
  int64_t r = r0;
  for (; r + RU - 1 < r1; r += RU) {
    TQ qv[RU][W];
    TQ wr[RU];
#pragma unroll
    for (int u = 0; u < RU; ++u) {
      wr[u] = coef(r + u);
      V16<TQ>::template load<NT>(a.C + (r + u) * a.ldc + col, qv[u]);
    }
#pragma unroll
    for (int u = 0; u < RU; ++u)
#pragma unroll
      for (int e = 0; e < W; ++e) acc[e] = fma(wr[u], qv[u][e], acc[e]);
  }
  for (; r < r1; ++r) {
    TQ qv[W];
    const TQ wr = coef(r);
    V16<TQ>::template load<NT>(a.C + r * a.ldc + col, qv);
#pragma unroll
    for (int e = 0; e < W; ++e) acc[e] = fma(wr, qv[e], acc[e]);
  }

  double* xi = a.x + static_cast<int64_t>(i) * a.ldx;
#pragma unroll
  for (int e = 0; e < W; ++e) {
    const double xo = xi[col + e];
    const double d = a.xbar[col + e] - xo;
    xi[col + e] = xo + a.gamma * (d - static_cast<double>(acc[e]));
  }
}

// The same update with the block's rows split over the waves: one workgroup
// per (block i, 64 x 16-byte column slab); wave v streams rows r0+v, r0+v+4,
// ... (1 KB contiguous per row), the four partial sums are added in LDS in a
// fixed order, then one thread per column applies the FP64 update.  Four times
// as many workgroups as the layout above at the same shape.
template <typename TQ, bool NT>
__global__ __launch_bounds__(kThreads) void k_pass_b_rows(PassBArgs<TQ> a) {
  constexpr int W = V16<TQ>::W;
  constexpr int SW = 64 * W;  // columns per slab
  const int s = blockIdx.x % a.nslab;
  const int i = a.blk_begin + static_cast<int>(blockIdx.x / a.nslab);
  const int lane = threadIdx.x & 63;
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int64_t r0 = a.off[i];
  const int64_t r1 = a.off[i + 1];
  const int64_t col = static_cast<int64_t>(s) * SW + lane * W;
  TQ acc[W];
#pragma unroll
  for (int e = 0; e < W; ++e) acc[e] = TQ(0);
  if (col < a.ldc) {
    for (int64_t r = r0 + wv; r < r1; r += 4) {
      TQ wr = a.w[r];
      for (int sp = 1; sp < a.nsplit; ++sp) wr += a.w[sp * a.w_stride + r];
      TQ q[W];
      V16<TQ>::template load<NT>(a.C + r * a.ldc + col, q);
#pragma unroll
      for (int e = 0; e < W; ++e) acc[e] = fma(wr, q[e], acc[e]);
    }
  }
  __shared__ TQ red[kThreads / 64][SW];
#pragma unroll
  for (int e = 0; e < W; ++e) red[wv][lane * W + e] = acc[e];
  __syncthreads();
  double* xi = a.x + static_cast<int64_t>(i) * a.ldx;
  for (int t = threadIdx.x; t < SW; t += kThreads) {
    const int64_t j = static_cast<int64_t>(s) * SW + t;
    if (j >= a.ldc) break;
    const TQ v = (red[0][t] + red[1][t]) + (red[2][t] + red[3][t]);
    const double xo = xi[j];
    xi[j] = xo + a.gamma * ((a.xbar[j] - xo) - static_cast<double>(v));
  }
}

// ------------------------------------------------------------------ FP64 refinement

// Per block i: out[c*ldo + r0 + r] = scale * sum_q Lop[r][q] in[c*ldi + r0 + q] for
// r < p_i, c < kc, with Lop = Linv_i (lower triangular, q <= r) or, for TRANS,
// Linv_i^T (q >= r).  Grid: (row tiles of 64) x (column tiles of 64) x blocks;
// 16 x 16 threads, 4 x 4 outputs each, 32-wide K chunks staged in LDS.
template <bool TRANS>
__global__ __launch_bounds__(256) void k_tri_apply(const int64_t* off, const int64_t* goff,
                                                   const double* Linv, const double* in,
                                                   int64_t ldi, double* out, int64_t ldo,
                                                   int32_t kc, double scale) {
  const int blk = blockIdx.z;
  const int64_t r0 = off[blk];
  const int p = static_cast<int>(off[blk + 1] - r0);
  const int rt0 = blockIdx.x * 64, ct0 = blockIdx.y * 64;
  if (rt0 >= p || ct0 >= kc) return;
  const double* Lb = Linv + goff[blk];
  __shared__ double Ls[64][33];
  __shared__ double Is[32][65];
  const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
  double acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = 0.0;
  const int qbeg = TRANS ? rt0 : 0;
  const int qend = TRANS ? p : min(p, rt0 + 64);
  for (int q0 = qbeg; q0 < qend; q0 += 32) {
    for (int e = threadIdx.x; e < 64 * 32; e += 256) {
      int rr, qq;
      if (TRANS) { rr = e & 63; qq = e >> 6; }  // Linv[q][r]: consecutive r
      else { qq = e & 31; rr = e >> 5; }        // Linv[r][q]: consecutive q
      const int r = rt0 + rr, q = q0 + qq;
      double v = 0.0;
      if (r < p && q < qend && (TRANS ? q >= r : q <= r))
        v = TRANS ? Lb[static_cast<int64_t>(q) * p + r] : Lb[static_cast<int64_t>(r) * p + q];
      Ls[rr][qq] = v;
    }
    for (int e = threadIdx.x; e < 32 * 64; e += 256) {
      const int qq = e & 31, cc = e >> 5;
      const int q = q0 + qq, c = ct0 + cc;
      Is[qq][cc] = (q < qend && c < kc) ? in[static_cast<int64_t>(c) * ldi + r0 + q] : 0.0;
    }
    __syncthreads();
#pragma unroll 4
    for (int qq = 0; qq < 32; ++qq) {
      double av[4], bv[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) av[i] = Ls[tx * 4 + i][qq];
#pragma unroll
      for (int j = 0; j < 4; ++j) bv[j] = Is[qq][ty * 4 + j];
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] += av[i] * bv[j];
    }
    __syncthreads();
  }
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const int c = ct0 + ty * 4 + j;
    if (c >= kc) continue;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int r = rt0 + tx * 4 + i;
      if (r < p) out[static_cast<int64_t>(c) * ldo + r0 + r] = scale * acc[i][j];
    }
  }
}

// y[e] = alpha * x[e] + y[e].
__global__ void k_axpy(int64_t count, double alpha, const double* x, double* y) {
  for (int64_t e = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; e < count;
       e += static_cast<int64_t>(gridDim.x) * blockDim.x)
    y[e] += alpha * x[e];
}

// partial[b] = sum of squares of src over a fixed grid-stride assignment.
__global__ __launch_bounds__(256) void k_sumsq(const double* src, int64_t count, double* partial) {
  __shared__ double part[4];
  double s = 0.0;
  for (int64_t e = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; e < count;
       e += static_cast<int64_t>(gridDim.x) * blockDim.x)
    s = fma(src[e], src[e], s);
  s = wave_sum(s);
  if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) partial[blockIdx.x] = (part[0] + part[1]) + (part[2] + part[3]);
}

// ------------------------------------------------------------------ average

// Eq. (2b) over a 64-column stripe: wave w sums blocks w, w+4, ... in order,
// the four partial sums are added as (s0 + s1) + (s2 + s3), then
// x_bar <- alpha * sum + beta * x_bar (beta == 0 does not read x_bar).  When
// d is given, the next pass A's differences d_i = x_bar - x_i are written,
// rounded to the projection precision.
template <typename TD>
__global__ __launch_bounds__(256) void k_combine(const double* x, int64_t ldx, int32_t m,
                                                 int64_t n, double alpha, double beta,
                                                 double* xbar, TD* d, int64_t ldd) {
  __shared__ double part[4][64];
  __shared__ double xb[64];
  const int lane = threadIdx.x & 63;
  const int wv = threadIdx.x >> 6;
  const int64_t j = static_cast<int64_t>(blockIdx.x) * 64 + lane;
  double s = 0.0;
  if (j < n)
    for (int i = wv; i < m; i += 4) s += x[static_cast<int64_t>(i) * ldx + j];
  part[wv][lane] = s;
  __syncthreads();
  if (wv == 0 && j < n) {
    const double tot = (part[0][lane] + part[1][lane]) + (part[2][lane] + part[3][lane]);
    const double v = beta == 0.0 ? alpha * tot : alpha * tot + beta * xbar[j];
    xbar[j] = v;
    xb[lane] = v;
  }
  if (!d) return;
  __syncthreads();
  if (j < n)
    for (int i = wv; i < m; i += 4)
      d[static_cast<int64_t>(i) * ldd + j] =
          static_cast<TD>(xb[lane] - x[static_cast<int64_t>(i) * ldx + j]);
}

// ------------------------------------------------------------------ single pass

// Stores of one thread's 16-byte runs (W elements of TA per chunk of C).
template <typename T, int W>
__device__ inline void store_run(T* p, const T (&v)[W]) {
  if constexpr (sizeof(T) == 4 && W == 4) {
    *reinterpret_cast<f32x4_t*>(p) = f32x4_t{v[0], v[1], v[2], v[3]};
  } else if constexpr (sizeof(T) == 8 && W % 2 == 0) {
#pragma unroll
    for (int h = 0; h < W; h += 2) *reinterpret_cast<f64x2_t*>(p + h) = f64x2_t{v[h], v[h + 1]};
  } else {
#pragma unroll
    for (int e = 0; e < W; ++e) p[e] = v[e];
  }
}

// Both halves of eq. (2a) in one pass over C.  One workgroup per row tile of
// one block, all of the row's width: thread t owns the 16-byte chunks t,
// t + 256, ... of every row, so the tile's d_blk and the running sum of
// w_r C[r][:] stay in its registers.  Rows go in groups of G.  While one
// group's dot products are reduced across the workgroup (a wave sum each, then
// the four wave values through LDS), the next group's loads are in flight; the
// LDS slot alternates between groups, so one barrier per group is enough.
template <typename TQ, typename TA, int CPT, int G>
__global__ __launch_bounds__(kThreads) void k_fused(FusedArgs<TQ, TA> a) {
  constexpr int W = V16<TQ>::W;
  int q = blockIdx.x;
  if (a.xcd_remap == 1) {
    const int per = (a.ntiles + kXcds - 1) / kXcds;
    q = (blockIdx.x % kXcds) * per + blockIdx.x / kXcds;
  }
  if (q >= a.ntiles) return;
  const int row0 = a.tile_row0[q];
  const int nrows = a.tile_nrows[q];
  const TA* dblk = a.d + static_cast<int64_t>(a.tile_blk[q]) * a.ldd;

  // A chunk takes part when it starts before column n; C is zero from n to
  // ldc (a multiple of W), so the chunk's loads stay inside the row.
  bool ok[CPT];
  TA dv[CPT][W], acc[CPT][W];
#pragma unroll
  for (int c = 0; c < CPT; ++c) {
    const int64_t j = static_cast<int64_t>(threadIdx.x + c * kThreads) * W;
    ok[c] = j < a.n;
#pragma unroll
    for (int e = 0; e < W; ++e) {
      dv[c][e] = j + e < a.n ? dblk[j + e] : TA(0);
      acc[c][e] = TA(0);
    }
  }

  const TQ* base = a.C + static_cast<int64_t>(row0) * a.ldc + threadIdx.x * W;
  auto load = [&](TQ (&b)[G][CPT][W], int r0) {
#pragma unroll
    for (int r = 0; r < G; ++r) {
      const bool row_ok = r0 + r < nrows;
#pragma unroll
      for (int c = 0; c < CPT; ++c) {
        if (row_ok && ok[c]) {
          V16<TQ>::template load<true>(base + static_cast<int64_t>(r0 + r) * a.ldc + c * kThreads * W,
                                       b[r][c]);
        } else {
#pragma unroll
          for (int e = 0; e < W; ++e) b[r][c][e] = TQ(0);
        }
      }
    }
  };

  __shared__ TA red[2][kThreads / 64][G];
  const int lane = threadIdx.x & 63;
  const int wv = threadIdx.x >> 6;
  // Rows past the tile were loaded as zeros, so their w is 0 and they add nothing.
  auto step = [&](const TQ (&b)[G][CPT][W], int r0, int slot) {
    TA sum[G];
#pragma unroll
    for (int r = 0; r < G; ++r) {
      sum[r] = TA(0);
#pragma unroll
      for (int c = 0; c < CPT; ++c)
#pragma unroll
        for (int e = 0; e < W; ++e) sum[r] = fma(static_cast<TA>(b[r][c][e]), dv[c][e], sum[r]);
    }
#pragma unroll
    for (int r = 0; r < G; ++r) {
      const TA v = wave_sum_dpp(sum[r]);
      if (lane == 0) red[slot][wv][r] = v;
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < G; ++r) {
      TA w = (red[slot][0][r] + red[slot][1][r]) + (red[slot][2][r] + red[slot][3][r]);
      if (a.wsub && r0 + r < nrows) w -= a.wsub[row0 + r0 + r];
#pragma unroll
      for (int c = 0; c < CPT; ++c)
#pragma unroll
        for (int e = 0; e < W; ++e) acc[c][e] = fma(w, static_cast<TA>(b[r][c][e]), acc[c][e]);
    }
  };

  TQ b0[G][CPT][W], b1[G][CPT][W];
  load(b0, 0);
  for (int r0 = 0; r0 < nrows; r0 += 2 * G) {
    load(b1, r0 + G);
    step(b0, r0, 0);
    load(b0, r0 + 2 * G);
    step(b1, r0 + G, 1);
  }

  // Every chunk inside the padded row is written (zeros past n), so a partial
  // row is defined on all of [0, ldc).
  TA* out = a.part + static_cast<int64_t>(q) * a.ldp + threadIdx.x * W;
#pragma unroll
  for (int c = 0; c < CPT; ++c)
    if (static_cast<int64_t>(threadIdx.x + c * kThreads) * W < a.ldc)
      store_run<TA, W>(out + c * kThreads * W, acc[c]);
}

// The x_i update, the average and the next differences after k_fused.  A
// workgroup owns kCombineCols = 16 columns; its 16 lanes per column take every
// sixteenth block, U blocks at a time with all their loads issued before any
// store.  16 columns rather than 32 give twice the workgroups, two waves per
// SIMD at 16384 x 8192 (5.8 -> 5.3 us there; 8 columns, with 32-byte pieces
// of the partial rows per load, took 9.1).  TPB > 0: every block has exactly
// TPB tiles (tile t of block i is i TPB + t), so a block's partials are
// loaded together; TPB = 0 reads the tile ranges.  Both sum a block's
// partials in tile order.
constexpr int kCombineCols = 16;
template <typename TD, int TPB>
__global__ __launch_bounds__(256) void k_fused_combine(FusedCombineArgs<TD> a) {
  constexpr int U = 4;
  constexpr int CL = kCombineCols, BL = 256 / kCombineCols;
  __shared__ double part[BL][CL];
  __shared__ double xb[CL];
  const int lane = threadIdx.x % CL;
  const int bl = threadIdx.x / CL;
  const int64_t j = static_cast<int64_t>(blockIdx.x) * CL + lane;
  const TD* pp = a.part;
  double* x = a.x;
  double s = 0.0;
  // The first two rounds' new x_i stay in registers for the differences
  // below (m <= 2 BL U = 128 needs no re-read); later rounds read them back.
  double keep[2][U];
  auto round = [&](int i0, double xo, double (&kx)[U]) {
    double u[U], xi[U];
#pragma unroll
    for (int q = 0; q < U; ++q) {
      const int i = i0 + BL * q;
      u[q] = 0.0;
      xi[q] = 0.0;
      if (i < a.m) {
        if constexpr (TPB > 0) {
          double v[TPB];
#pragma unroll
          for (int t = 0; t < TPB; ++t)
            v[t] = static_cast<double>(pp[static_cast<int64_t>(i * TPB + t) * a.ldp + j]);
#pragma unroll
          for (int t = 0; t < TPB; ++t) u[q] += v[t];
        } else {
          for (int t = a.tile_first[i]; t < a.tile_first[i + 1]; ++t)
            u[q] += static_cast<double>(pp[static_cast<int64_t>(t) * a.ldp + j]);
        }
        xi[q] = x[static_cast<int64_t>(i) * a.ldx + j];
      }
    }
#pragma unroll
    for (int q = 0; q < U; ++q) {
      const int i = i0 + BL * q;
      kx[q] = 0.0;
      if (i < a.m) {
        const double xn = xi[q] + a.gamma * ((xo - xi[q]) - u[q]);
        x[static_cast<int64_t>(i) * a.ldx + j] = xn;
        s += xn;
        kx[q] = xn;
      }
    }
  };
  if (j < a.n) {
    const double xo = a.xbar[j];
    if (bl < a.m) round(bl, xo, keep[0]);
    if (bl + BL * U < a.m) round(bl + BL * U, xo, keep[1]);
    for (int i0 = bl + 2 * BL * U; i0 < a.m; i0 += BL * U) {
      double tmp[U];
      round(i0, xo, tmp);
    }
  }
  part[bl][lane] = s;
  __syncthreads();
  if (bl == 0 && j < a.n) {
    double tot = part[0][lane];
#pragma unroll
    for (int b = 1; b < BL; ++b) tot += part[b][lane];  // block-lane order
    const double v = a.beta == 0.0 ? a.alpha * tot : a.alpha * tot + a.beta * a.xbar[j];
    a.xbar[j] = v;
    xb[lane] = v;
  }
  __syncthreads();
  if (j < a.n) {
    const double v = xb[lane];
#pragma unroll
    for (int r = 0; r < 2; ++r) {
#pragma unroll
      for (int q = 0; q < U; ++q) {
        const int i = bl + BL * U * r + BL * q;
        if (i < a.m) a.d[static_cast<int64_t>(i) * a.ldd + j] = static_cast<TD>(v - keep[r][q]);
      }
    }
    for (int i0 = bl + 2 * BL * U; i0 < a.m; i0 += BL * U) {
      double xi[U];
#pragma unroll
      for (int q = 0; q < U; ++q) {
        const int i = i0 + BL * q;
        xi[q] = i < a.m ? x[static_cast<int64_t>(i) * a.ldx + j] : 0.0;
      }
#pragma unroll
      for (int q = 0; q < U; ++q) {
        const int i = i0 + BL * q;
        if (i < a.m) a.d[static_cast<int64_t>(i) * a.ldd + j] = static_cast<TD>(v - xi[q]);
      }
    }
  }
}

// out[j] = alpha sum_t part[t][j] over all tiles (summed in FP64, fixed order), j < n:
// the sum over blocks of the normal operator after k_fused with one shared
// vector.  32 columns per workgroup, 8 lanes per column, each lane four
// independent running sums.
template <typename TP>
__global__ __launch_bounds__(256) void k_fused_sum(const TP* part, int64_t ldp, int32_t ntiles,
                                                   int64_t n, double alpha, double* out) {
  __shared__ double red[8][32];
  const int lane = threadIdx.x & 31;
  const int bl = threadIdx.x >> 5;
  const int64_t j = static_cast<int64_t>(blockIdx.x) * 32 + lane;
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  if (j < n) {
    for (int t0 = bl; t0 < ntiles; t0 += 32) {
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int t = t0 + 8 * q;
        if (t < ntiles) acc[q] += static_cast<double>(part[static_cast<int64_t>(t) * ldp + j]);
      }
    }
  }
  red[bl][lane] = (acc[0] + acc[1]) + (acc[2] + acc[3]);
  __syncthreads();
  if (bl == 0 && j < n)
    out[j] = alpha * (((red[0][lane] + red[1][lane]) + (red[2][lane] + red[3][lane])) +
                      ((red[4][lane] + red[5][lane]) + (red[6][lane] + red[7][lane])));
}

// out[i * ldo + j] = sum over block i's partial rows (tiles tile_first[i] ..
// tile_first[i + 1] - 1, in order) of part[t][j], j < ncols.  Grid: (column
// chunks of 256, blocks).
__global__ __launch_bounds__(256) void k_block_sum(const double* part, int64_t ldp,
                                                   const int32_t* tile_first, int64_t ncols,
                                                   double* out, int64_t ldo) {
  const int i = blockIdx.y;
  const int64_t j = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x;
  if (j >= ncols) return;
  double s = 0.0;
  for (int t = tile_first[i]; t < tile_first[i + 1]; ++t) s += part[static_cast<int64_t>(t) * ldp + j];
  out[static_cast<int64_t>(i) * ldo + j] = s;
}

// Per block i: out[2i] = ||V_i - U_i||^2, out[2i + 1] = ||U_i||^2 over j < n.
__global__ __launch_bounds__(256) void k_defect(const double* U, const double* V, int64_t ld,
                                                int64_t n, double* out) {
  __shared__ double ra[4], rb[4];
  const int i = blockIdx.x;
  double a = 0.0, b = 0.0;
  for (int64_t j = threadIdx.x; j < n; j += 256) {
    const double u = U[static_cast<int64_t>(i) * ld + j];
    const double d = V[static_cast<int64_t>(i) * ld + j] - u;
    a += d * d;
    b += u * u;
  }
  a = wave_sum(a);
  b = wave_sum(b);
  if ((threadIdx.x & 63) == 0) {
    ra[threadIdx.x >> 6] = a;
    rb[threadIdx.x >> 6] = b;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    out[2 * i] = (ra[0] + ra[1]) + (ra[2] + ra[3]);
    out[2 * i + 1] = (rb[0] + rb[1]) + (rb[2] + rb[3]);
  }
}

// Per block: ||w_i + y_i||^2 and ||y_i||^2 over the block's rows (w = -C s,
// the sum of nsplit column-split partials, with s_i = C_i^T y_i, so
// w_i + y_i = -(C_i C_i^T - I) y_i).
__global__ __launch_bounds__(256) void k_defect_rows(const double* w, int32_t nsplit,
                                                     int64_t wstride, const double* y,
                                                     const int64_t* off, int32_t m, double* h) {
  __shared__ double ra[4], rb[4];
  for (int32_t i = blockIdx.x; i < m; i += gridDim.x) {
    double a = 0.0, b = 0.0;
    for (int64_t r = off[i] + threadIdx.x; r < off[i + 1]; r += 256) {
      double wr = w[r];
      for (int32_t sp = 1; sp < nsplit; ++sp) wr += w[sp * wstride + r];
      const double e = wr + y[r];
      a = fma(e, e, a);
      b = fma(y[r], y[r], b);
    }
    a = wave_sum(a);
    b = wave_sum(b);
    if ((threadIdx.x & 63) == 0) {
      ra[threadIdx.x >> 6] = a;
      rb[threadIdx.x >> 6] = b;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      h[2 * i] = (ra[0] + ra[1]) + (ra[2] + ra[3]);
      h[2 * i + 1] = (rb[0] + rb[1]) + (rb[2] + rb[3]);
    }
    __syncthreads();
  }
}

// ------------------------------------------------------------------ expand (FP64)

// y_i = beta * y_i + alpha * sum_{r in block i} w_r C[r][:], FP64 accumulation.
// A workgroup owns a 64-lane column slab of one block; its 4 waves take
// interleaved rows and combine in LDS.  w_r sums nsplit partials in order.
template <typename TQ>
__global__ __launch_bounds__(kThreads) void k_expand(ExpandArgs<TQ> a) {
  constexpr int W = V16<TQ>::W;
  constexpr int SW = 64 * W;
  const int s = blockIdx.x % a.nslab;
  const int i = a.blk_begin + static_cast<int>(blockIdx.x / a.nslab);
  const int lane = threadIdx.x & 63;
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int64_t r0 = a.off ? a.off[i] : 0;
  const int64_t r1 = a.off ? a.off[i + 1] : a.rows_total;
  const int64_t col = static_cast<int64_t>(s) * SW + lane * W;
  double acc[W];
#pragma unroll
  for (int e = 0; e < W; ++e) acc[e] = 0.0;
  if (col < a.ldc) {
    for (int64_t r = r0 + wv; r < r1; r += 4) {
      double wr = a.w[r];
      for (int sp = 1; sp < a.nsplit; ++sp) wr += a.w[sp * a.w_stride + r];
      if (a.wsub) wr -= a.wsub[r];
      TQ q[W];
      V16<TQ>::load(a.C + r * a.ldc + col, q);
#pragma unroll
      for (int e = 0; e < W; ++e) acc[e] = fma(wr, static_cast<double>(q[e]), acc[e]);
    }
  }
  __shared__ double red[kThreads / 64][SW];
#pragma unroll
  for (int e = 0; e < W; ++e) red[wv][lane * W + e] = acc[e];
  __syncthreads();
  for (int t = threadIdx.x; t < SW; t += kThreads) {
    const int64_t j = static_cast<int64_t>(s) * SW + t;
    if (j >= a.ldc) break;
    const double v = (red[0][t] + red[1][t]) + (red[2][t] + red[3][t]);
    double* yi = a.y + static_cast<int64_t>(i) * a.ldy;
    yi[j] = (a.beta == 0.0 ? 0.0 : a.beta * yi[j]) + a.alpha * v;
  }
}

// ------------------------------------------------------------------ setup

// C <- A zero-padded to ldc columns; c <- B in RHS-major order
// (c[col * N + r] = B[r * ldb + col]), zero for k <= col < kp.
__global__ void k_copy_pad(const double* A, int64_t lda, const double* B, int64_t ldb, int64_t N,
                           int64_t n, double* C, int64_t ldc, double* c, int32_t k, int32_t kp) {
  for (int64_t r = blockIdx.x; r < N; r += gridDim.x) {
    if (C)
      for (int64_t j = threadIdx.x; j < ldc; j += blockDim.x) C[r * ldc + j] = j < n ? A[r * lda + j] : 0.0;
    for (int col = threadIdx.x; col < kp; col += blockDim.x)
      c[static_cast<int64_t>(col) * N + r] = col < k ? B[r * ldb + col] : 0.0;
  }
}

// 64x64 tile of G_i = C_i C_i^T; 256 threads, 4x4 outputs each; K staged in
// LDS 32 columns at a time (256-byte row segments).
constexpr int GK = 32;
__global__ __launch_bounds__(256) void k_gram(const double* C, int64_t ldc, const int64_t* off,
                                              const int32_t* tiles, const int64_t* goff,
                                              double* G) {
  const int blk = tiles[3 * blockIdx.x + 0];
  const int ta = tiles[3 * blockIdx.x + 1];
  const int tb = tiles[3 * blockIdx.x + 2];
  const int64_t r0 = off[blk];
  const int p = static_cast<int>(off[blk + 1] - r0);
  __shared__ double As[GK][kGramTile + 1];
  __shared__ double Bs[GK][kGramTile + 1];
  const int tx = threadIdx.x % 16;
  const int ty = threadIdx.x / 16;
  double acc[4][4] = {};
  for (int64_t k0 = 0; k0 < ldc; k0 += GK) {
    for (int e = threadIdx.x; e < kGramTile * GK; e += 256) {
      const int rr = e / GK;
      const int kk = e % GK;
      const int ra = ta * kGramTile + rr;
      const int rb = tb * kGramTile + rr;
      const int64_t kc = k0 + kk;
      As[kk][rr] = (ra < p && kc < ldc) ? C[(r0 + ra) * ldc + kc] : 0.0;
      Bs[kk][rr] = (rb < p && kc < ldc) ? C[(r0 + rb) * ldc + kc] : 0.0;
    }
    __syncthreads();
#pragma unroll 8
    for (int kk = 0; kk < GK; ++kk) {
      double av[4], bv[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        av[u] = As[kk][ty * 4 + u];
        bv[u] = Bs[kk][tx * 4 + u];
      }
#pragma unroll
      for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int v = 0; v < 4; ++v) acc[u][v] = fma(av[u], bv[v], acc[u][v]);
    }
    __syncthreads();
  }
  double* Gb = G + goff[blk];
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const int ra = ta * kGramTile + ty * 4 + u;
    if (ra >= p) continue;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int rb = tb * kGramTile + tx * 4 + v;
      if (rb >= p) continue;
      Gb[static_cast<int64_t>(ra) * p + rb] = acc[u][v];
      if (ta != tb) Gb[static_cast<int64_t>(rb) * p + ra] = acc[u][v];
    }
  }
}

// Blocked Cholesky G_i = L L^T and the diagonal blocks of Linv_i = L^{-1}, one
// workgroup per block.  Panels of 32 columns: wave 0 factors and inverts the
// 32 x 32 diagonal block in registers (lane i holds row i; broadcasts by
// shuffles), all threads then solve the panel below it (rows times L_kk^{-T})
// and update the trailing lower triangle from an LDS copy of the panel.
// Linv's strict upper triangle is written as zeros (the tiled products read
// whole tiles); its blocks below the diagonal are k_tri_inv's.  flags[0] <-
// 1 + (first block whose pivot fails the rank test).
constexpr int kNB = 32;
constexpr int kPanelRows = 384;  // panels of up to this many rows are kept in LDS

__global__ __launch_bounds__(512) void k_chol_inv(const int64_t* off, const int64_t* goff,
                                                   double* G, double* Linv, int* flags,
                                                   double rank_tol) {
  const int blk = blockIdx.x;
  const int p = static_cast<int>(off[blk + 1] - off[blk]);
  double* Gb = G + goff[blk];
  double* Lb = Linv + goff[blk];
  const int tid = threadIdx.x, nt = blockDim.x;
  const int lane = tid & 63, wv = tid >> 6;
  __shared__ double dl[kNB][kNB + 1];   // L_kk, then (column-solve input)
  __shared__ double di[kNB][kNB + 1];   // L_kk^{-1}
  __shared__ double pan[kPanelRows][kNB + 2];  // stride 34: conflict-free MFMA fragment reads
  __shared__ double red[1024 / 64];  // per-wave maxima (up to 16 waves)
  __shared__ int bad;

  // Largest diagonal entry (rank test scale) and the zero upper triangle of Linv.
  double mx = 0.0;
  for (int k = tid; k < p; k += nt) mx = fmax(mx, Gb[static_cast<int64_t>(k) * p + k]);
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) mx = fmax(mx, __shfl_xor(mx, o, 64));
  if (lane == 0) red[wv] = mx;
  if (tid == 0) bad = 0;
  for (int r = wv; r < p; r += nt / 64)
    for (int c = r + 1 + lane; c < p; c += 64) Lb[static_cast<int64_t>(r) * p + c] = 0.0;
  __syncthreads();
  double maxdiag = 0.0;
  for (int w = 0; w < nt / 64; ++w) maxdiag = fmax(maxdiag, red[w]);

  for (int kb = 0; kb < p; kb += kNB) {
    const int nb = min(kNB, p - kb);
    // (1) diagonal block: Cholesky and its inverse in wave 0's registers.
    if (wv == 0) {
      double a[kNB];
#pragma unroll
      for (int j = 0; j < kNB; ++j) {
        double v = (lane == j) ? 1.0 : 0.0;  // identity past nb
        if (lane < nb && j < nb && j <= lane) v = Gb[static_cast<int64_t>(kb + lane) * p + kb + j];
        a[j] = v;
      }
      // Column j and the pivot pass between lanes by lane reads (scalar
      // broadcasts: the source lanes are compile-time constants).
#pragma unroll
      for (int j = 0; j < kNB; ++j) {
        double piv = lane_f64(a[j], j);
        if (j < nb && !(piv > rank_tol * maxdiag)) {  // also catches NaN
          if (lane == 0) bad = 1;
          piv = maxdiag > 0.0 ? maxdiag : 1.0;
        }
        const double d = sqrt(piv);
        if (lane > j) a[j] /= d;
        if (lane == j) a[j] = d;
#pragma unroll
        for (int jj = j + 1; jj < kNB; ++jj) {
          const double ljj = lane_f64(a[j], jj);
          if (lane >= jj) a[jj] -= a[j] * ljj;
        }
      }
      if (lane < kNB) {
#pragma unroll
        for (int j = 0; j < kNB; ++j) dl[lane][j] = (j <= lane) ? a[j] : 0.0;
      }
      __builtin_amdgcn_wave_barrier();
      // Inverse of L_kk: lane c forms column c by right-looking forward
      // substitution, x_i = s_i / L_ii and then s_k -= L_ki x_i for k > i
      // (L's entries broadcast from LDS: a wave's LDS accesses complete in
      // order).  The dependent chain is one multiply and one FMA per step.
      double sv[kNB];
#pragma unroll
      for (int k = 0; k < kNB; ++k) sv[k] = (lane == k) ? 1.0 : 0.0;
#pragma unroll
      for (int i = 0; i < kNB; ++i) {
        const double x = sv[i] * (1.0 / dl[i][i]);
        sv[i] = x;
#pragma unroll
        for (int k = i + 1; k < kNB; ++k) sv[k] -= dl[k][i] * x;
      }
      if (lane < kNB) {
#pragma unroll
        for (int i = 0; i < kNB; ++i) di[i][lane] = (i < lane) ? 0.0 : sv[i];
      }
    }
    __syncthreads();
    // Write L_kk and L_kk^{-1} back.
    for (int e = tid; e < nb * nb; e += nt) {
      const int i = e / nb, j = e % nb;
      if (j <= i) {
        Gb[static_cast<int64_t>(kb + i) * p + kb + j] = dl[i][j];
        Lb[static_cast<int64_t>(kb + i) * p + kb + j] = di[i][j];
      }
    }
    // (2) panel below: P = rows times L_kk^{-T} (a panel exists only below a
    // full 32-column block) on the FP64 matrix cores.  Wave w takes the
    // 16-row tiles I = w (mod 8) and both 16-column output tiles of each:
    // lane (li, g) supplies A[li][g] = G[row 16 I + li][4 kk + g] (all eight K
    // steps loaded before anything is written: the result replaces those
    // rows) and B[g][li] = Linv_kk[16 J + li][4 kk + g], and receives
    // P[16 I + g + 4 q][16 J + li].
    const int T = p - kb - nb;
    const bool in_lds = T <= kPanelRows;
    if (T > 0) {
      const int nT = (T + 15) / 16;
      const int li = lane & 15, g = lane >> 4;
      for (int I = wv; I < nT; I += nt / 64) {
        const int ra = 16 * I + li;
        const double* arow = Gb + static_cast<int64_t>(kb + nb + min(ra, T - 1)) * p + kb;
        double av[kNB / 4];
#pragma unroll
        for (int kk = 0; kk < kNB / 4; ++kk) {
          const double v = arow[4 * kk + g];
          av[kk] = ra < T ? v : 0.0;
        }
        f64x4 acc0 = f64x4{}, acc1 = f64x4{};
#pragma unroll
        for (int kk = 0; kk < kNB / 4; ++kk) {
          acc0 = __builtin_amdgcn_mfma_f64_16x16x4f64(av[kk], di[li][4 * kk + g], acc0, 0, 0, 0);
          acc1 = __builtin_amdgcn_mfma_f64_16x16x4f64(av[kk], di[16 + li][4 * kk + g], acc1, 0, 0, 0);
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int row = 16 * I + g + 4 * q;
          if (row < T) {
            double* orow = Gb + static_cast<int64_t>(kb + nb + row) * p + kb;
            orow[li] = acc0[q];
            orow[16 + li] = acc1[q];
            if (in_lds) {
              pan[row][li] = acc0[q];
              pan[row][16 + li] = acc1[q];
            }
          }
        }
      }
    }
    __syncthreads();
    // (3) trailing update G22 -= P P^T of the lower triangle.  With the panel
    // in LDS: 16 x 16 tiles (I >= J) on the FP64 matrix cores, dealt to the
    // waves round-robin, 8 MFMA 16x16x4 per tile (K = nb = 32: a trailing
    // block exists only after a full panel).  Lane (li, g) supplies
    // A[li][g] = -P[16 I + li][k] and B[g][li] = P[16 J + li][k] and holds
    // D[g + 4 q][li]; rows past T read a clamped row and are zeroed.
    if (in_lds) {
      // Tile t = I (I + 1) / 2 + J goes to wave t mod (waves); a wave loads
      // the G entries of kTrail of its tiles before it multiplies any, so the
      // loads' latencies overlap instead of adding up tile after tile.
      const int nT = (T + 15) / 16;
      const int ntile = nT * (nT + 1) / 2;
      const int nw = nt / 64;
      const int li = lane & 15, g = lane >> 4;
      constexpr int kTrail = 8;
      for (int t0 = wv; t0 < ntile; t0 += kTrail * nw) {
        f64x4 acc[kTrail];
        int tI[kTrail], tJ[kTrail];
#pragma unroll
        for (int u = 0; u < kTrail; ++u) {
          const int t = t0 + u * nw;
          int I = static_cast<int>((sqrt(8.0 * t + 1.0) - 1.0) * 0.5);
          while ((I + 1) * (I + 2) / 2 <= t) ++I;
          while (I * (I + 1) / 2 > t) --I;
          tI[u] = I;
          tJ[u] = t - I * (I + 1) / 2;
          const int col = 16 * tJ[u] + li;
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            const int row = 16 * I + g + 4 * q;
            const double v = Gb[static_cast<int64_t>(kb + nb + min(row, T - 1)) * p + kb + nb +
                                min(col, T - 1)];
            acc[u][q] = (t < ntile && row < T && col <= row) ? v : 0.0;
          }
        }
#pragma unroll
        for (int u = 0; u < kTrail; ++u) {
          if (t0 + u * nw >= ntile) break;  // uniform per wave
          const int I = tI[u], J = tJ[u];
          const int col = 16 * J + li;
          const int ra = 16 * I + li, rb = 16 * J + li;
          const int ca = min(ra, T - 1), cb = min(rb, T - 1);
#pragma unroll
          for (int kk = 0; kk < kNB / 4; ++kk) {
            const int k = 4 * kk + g;
            const double av = pan[ca][k], bv = pan[cb][k];
            const double a = ra < T ? -av : 0.0;
            const double b = rb < T ? bv : 0.0;
            acc[u] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc[u], 0, 0, 0);
          }
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            const int row = 16 * I + g + 4 * q;
            if (row < T && col <= row)
              Gb[static_cast<int64_t>(kb + nb + row) * p + kb + nb + col] = acc[u][q];
          }
        }
      }
    } else {
      for (int64_t e = tid; e < static_cast<int64_t>(T) * T; e += nt) {
        const int rr = static_cast<int>(e / T), cc = static_cast<int>(e % T);
        if (cc > rr) continue;
        const double* pr = Gb + static_cast<int64_t>(kb + nb + rr) * p + kb;
        const double* pc = Gb + static_cast<int64_t>(kb + nb + cc) * p + kb;
        double sacc = 0.0;
        for (int q = 0; q < nb; ++q) sacc += pr[q] * pc[q];
        Gb[static_cast<int64_t>(kb + nb + rr) * p + kb + nb + cc] -= sacc;
      }
    }
    __syncthreads();
  }

  if (tid == 0 && bad) atomicCAS(flags, 0, blk + 1);
}

// Off-diagonal blocks of L^{-1} after k_chol_inv (which leaves L in the lower
// triangle of G and the inverses of L's 32 x 32 diagonal blocks in Linv).  One
// 512-thread workgroup per (block column J, block): block column J of L^{-1}
// depends on no other column, so the columns of all blocks run in parallel.
// Going down the column, for block row I > J,
//   Linv[I][J] = -Linv_II sum_{K=J}^{I-1} L[I][K] Linv[K][J],
// each term a 32 x 32 product through LDS; the Linv[K][J] it reads were written
// by this workgroup earlier in the column (or are the diagonal block, K = J).
// Thread (i, column pair): i = tid / 16, columns 2 (tid % 16) and 2 (tid % 16) + 1.
__global__ __launch_bounds__(512) void k_tri_inv(const int64_t* off, const int64_t* goff,
                                                 const double* G, double* Linv) {
  const int blk = blockIdx.y;
  const int p = static_cast<int>(off[blk + 1] - off[blk]);
  const int J0 = static_cast<int>(blockIdx.x) * kNB;
  if (J0 + kNB >= p) return;  // the last block column has no block below it
  const double* Gb = G + goff[blk];
  double* Lb = Linv + goff[blk];
  const int tid = threadIdx.x;
  const int ti = tid >> 4, tc2 = (tid & 15) * 2;
  __shared__ double dl[kNB][kNB + 1];
  __shared__ double di[kNB][kNB + 1];
  __shared__ double pan[kNB][kNB + 1];
  // The steps (I0, K0) -- row blocks I0 = J0 + 32, ..., K0 = J0 .. I0 - 32 --
  // run in order; the next step's two blocks are loaded into registers while
  // the current one is multiplied (thread t stages entries t and t + 512 of
  // each: row e / 32, column e % 32).  A step reads Linv[K0][J0] with K0 < I0,
  // written by this workgroup at the end of an earlier row; the last step of
  // a row, which reads the block the previous row wrote, is loaded during the
  // step before it, after that write.
  const int sr = tid >> 5, sq = tid & 31;
  double vl[2], vp[2];
  auto load_step = [&](int I, int K) {
    const int nb = min(kNB, p - I);
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      const int r = sr + 16 * u;
      vl[u] = Gb[static_cast<int64_t>(I + min(r, nb - 1)) * p + K + sq];
      vp[u] = Lb[static_cast<int64_t>(K + r) * p + J0 + sq];
    }
  };
  int I0 = J0 + kNB, K0 = J0;
  load_step(I0, K0);
  double t0 = 0.0, t1 = 0.0;
  for (;;) {
    const int nbI = min(kNB, p - I0);
    __syncthreads();
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      const int r = sr + 16 * u;
      dl[r][sq] = r < nbI ? vl[u] : 0.0;
      pan[r][sq] = vp[u];
    }
    if (K0 == J0) {
      // L_II^{-1} into LDS (zero-padded to 32 x 32).
      for (int e = tid; e < kNB * kNB; e += 512) {
        const int i = e / kNB, q = e % kNB;
        di[i][q] = (i < nbI && q <= i) ? Lb[static_cast<int64_t>(I0 + i) * p + I0 + q] : 0.0;
      }
    }
    __syncthreads();
    int nI = I0, nK = K0 + kNB;
    const bool row_end = nK >= I0;
    if (row_end) {
      nI = I0 + kNB;
      nK = J0;
    }
    const bool more = nI < p;
    load_step(more ? nI : I0, more ? nK : K0);  // past the end: reload, unused
#pragma unroll 8
    for (int k = 0; k < kNB; ++k) {
      const double l = dl[ti][k];
      t0 = fma(l, pan[k][tc2], t0);
      t1 = fma(l, pan[k][tc2 + 1], t1);
    }
    if (row_end) {
      // Linv[I][J] = -L_II^{-1} (the row's sum).
      __syncthreads();
      dl[ti][tc2] = t0;
      dl[ti][tc2 + 1] = t1;
      __syncthreads();
      double o0 = 0.0, o1 = 0.0;
#pragma unroll 8
      for (int q = 0; q < kNB; ++q) {
        const double d = di[ti][q];  // zero above the diagonal
        o0 = fma(d, dl[q][tc2], o0);
        o1 = fma(d, dl[q][tc2 + 1], o1);
      }
      if (ti < nbI) {
        Lb[static_cast<int64_t>(I0 + ti) * p + J0 + tc2] = -o0;
        Lb[static_cast<int64_t>(I0 + ti) * p + J0 + tc2 + 1] = -o1;
      }
      t0 = 0.0;
      t1 = 0.0;
      if (!more) break;
    }
    I0 = nI;
    K0 = nK;
  }
}

// 64x64 tile of Out_i = Linv_i In_i (Linv lower triangular: K runs to the
// tile's last row).
__global__ __launch_bounds__(256) void k_trmm(const double* In, double* Out, int64_t ldc,
                                              const int64_t* off, const int32_t* tiles,
                                              const int64_t* goff, const double* Linv) {
  const int blk = tiles[3 * blockIdx.x + 0];
  const int ta = tiles[3 * blockIdx.x + 1];
  const int tc = tiles[3 * blockIdx.x + 2];
  const int64_t r0 = off[blk];
  const int p = static_cast<int>(off[blk + 1] - r0);
  const double* Lb = Linv + goff[blk];
  __shared__ double As[GK][kGramTile + 1];
  __shared__ double Bs[GK][kGramTile + 1];
  const int tx = threadIdx.x % 16;
  const int ty = threadIdx.x / 16;
  double acc[4][4] = {};
  const int kend = min(p, (ta + 1) * kGramTile);
  const int64_t c0 = static_cast<int64_t>(tc) * kGramTile;
  for (int k0 = 0; k0 < kend; k0 += GK) {
    for (int e = threadIdx.x; e < kGramTile * GK; e += 256) {
      const int rr = e / GK;
      const int kk = e % GK;
      const int ra = ta * kGramTile + rr;
      const int kc = k0 + kk;
      As[kk][rr] = (ra < p && kc < p) ? Lb[static_cast<int64_t>(ra) * p + kc] : 0.0;
      const int kb = e / kGramTile;
      const int cc = e % kGramTile;
      const int kr = k0 + kb;
      Bs[kb][cc] = (kr < p && c0 + cc < ldc) ? In[(r0 + kr) * ldc + c0 + cc] : 0.0;
    }
    __syncthreads();
#pragma unroll 8
    for (int kk = 0; kk < GK; ++kk) {
      double av[4], bv[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        av[u] = As[kk][ty * 4 + u];
        bv[u] = Bs[kk][tx * 4 + u];
      }
#pragma unroll
      for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int v = 0; v < 4; ++v) acc[u][v] = fma(av[u], bv[v], acc[u][v]);
    }
    __syncthreads();
  }
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const int ra = ta * kGramTile + ty * 4 + u;
    if (ra >= p) continue;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int64_t cc = c0 + tx * 4 + v;
      if (cc < ldc) Out[(r0 + ra) * ldc + cc] = acc[u][v];
    }
  }
}


__global__ void k_cast_f32(const double* src, float* dst, int64_t count) {
  for (int64_t e = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; e < count;
       e += static_cast<int64_t>(gridDim.x) * blockDim.x)
    dst[e] = static_cast<float>(src[e]);
}

__global__ void k_fill_u32(unsigned* p, int64_t count, unsigned v) {
  for (int64_t e = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; e < count;
       e += static_cast<int64_t>(gridDim.x) * blockDim.x)
    p[e] = v;
}

// C <- A zero-padded to ldc columns, converted to T.
template <typename T>
__global__ void k_pad_cast(const double* A, int64_t lda, int64_t N, int64_t n, T* C, int64_t ldc) {
  for (int64_t r = blockIdx.x; r < N; r += gridDim.x)
    for (int64_t j = threadIdx.x; j < ldc; j += blockDim.x)
      C[r * ldc + j] = j < n ? static_cast<T>(A[r * lda + j]) : T(0);
}

// Heavy-ball step (Sec. 4.3) after the block pass: g = sum_i Y_i with the
// blocks added in the same fixed order as the APC average, then
// z <- beta z + g, x <- x - alpha z.  One column per lane of wave 0.
__global__ __launch_bounds__(256) void k_hbm_step(const double* Y, int64_t ldy, int32_t m,
                                                  int64_t n, double alpha, double beta, double* x,
                                                  double* z) {
  __shared__ double part[4][64];
  const int lane = threadIdx.x & 63;
  const int wv = threadIdx.x >> 6;
  const int64_t j = static_cast<int64_t>(blockIdx.x) * 64 + lane;
  double s = 0.0;
  if (j < n)
    for (int i = wv; i < m; i += 4) s += Y[static_cast<int64_t>(i) * ldy + j];
  part[wv][lane] = s;
  __syncthreads();
  if (wv == 0 && j < n) {
    const double g = (part[0][lane] + part[1][lane]) + (part[2][lane] + part[3][lane]);
    const double zn = beta * z[j] + g;
    z[j] = zn;
    x[j] -= alpha * zn;
  }
}

__global__ void k_copy_strided(const double* src, int64_t lds, double* dst, int64_t ldd,
                               int64_t rows, int64_t cols) {
  if (cols == 1) {
    for (int64_t r = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; r < rows;
         r += static_cast<int64_t>(gridDim.x) * blockDim.x)
      dst[r * ldd] = src[r * lds];
    return;
  }
  for (int64_t r = blockIdx.x; r < rows; r += gridDim.x)
    for (int64_t j = threadIdx.x; j < cols; j += blockDim.x) dst[r * ldd + j] = src[r * lds + j];
}

// dst[j * ldd + c] = src[c * lds + j] for j < n, c < k (RHS-major -> row-major).
__global__ void k_copy_t(const double* src, int64_t lds, double* dst, int64_t ldd, int64_t n,
                         int32_t k) {
  const int64_t total = n * k;
  for (int64_t e = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; e < total;
       e += static_cast<int64_t>(gridDim.x) * blockDim.x) {
    const int64_t j = e / k;
    const int c = static_cast<int>(e - j * k);
    dst[j * ldd + c] = src[c * lds + j];
  }
}

// ------------------------------------------------------------------ Lanczos step

// One Lanczos step after the operator: twice classical Gram-Schmidt of w
// against the basis rows V[0..j], then beta_j = ||w||, V[j + 1] = w / beta_j,
// in three launches over column slabs of kLzSlab = 64 columns, one workgroup
// of kLzWaves waves per slab.  Lane l of every wave owns the slab's column l;
// the waves split the rows (or the partial-row tiles) r = wv, wv + 8, ...
// Every step local to a column -- the operator's sum over partial rows,
// w -= sum_r h_r V[r], the scaling -- runs in the slab that owns it; only the
// dot products and the norm cross slabs, as per-slab partials that every
// workgroup of the next launch sums in slab order (so nothing depends on
// scheduling).  Rows go eight per wave at a time: their loads are issued
// together and their eight wave sums reduced at once (row_sums), so a step
// costs a few memory round trips instead of one per row; each thread's
// entries of the first 64 basis rows are loaded once per launch, before the
// loads they do not depend on have returned.  Columns past ldc contribute
// zero.  The norm after the second pass is taken by Pythagoras: with V's rows
// orthonormal, ||w1 - V^T h2||^2 = ||w1||^2 - ||h2||^2 for h2 = V w1 (to
// rounding, h2 being of the order of the first pass's rounding), so the
// second pass and the normalisation share a launch.
constexpr int kLzWaves = 8;
constexpr int kLzRows = 8 * kLzWaves;  // basis rows one pass over the workgroup covers

// v[k] = V[r][c] for the first kLzRows rows this wave takes (r = wv + 8 k,
// clamped to j; rows past j are never used).
__device__ inline void lz_first_rows(const LanczosArgs& a, int64_t c, bool ok, double (&v)[8]) {
  const int wv = threadIdx.x >> 6;
  const int64_t cc = ok ? c : 0;
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    const int r = wv + kLzWaves * k;
    v[k] = a.V[static_cast<int64_t>(r <= a.j ? r : a.j) * a.ldc + cc];
  }
}

// hp[blockIdx.x * hstride + r] = sum over the slab's columns of V[r][c] x, r <= j.
// v0: the thread's entries of the first kLzRows rows (lz_first_rows).
__device__ inline void lz_dots(const LanczosArgs& a, int64_t c, bool ok, double x, double* hp,
                               const double (&v0)[8]) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int64_t cc = ok ? c : 0;
  for (int r0 = 0; r0 <= a.j; r0 += kLzRows) {
    double p[8], t[8];
    if (r0 == 0) {
#pragma unroll
      for (int k = 0; k < 8; ++k) p[k] = v0[k];
    } else {
      // Clamped addresses and a select after the load keep the eight loads
      // free of branches, so they are all in flight at once.
#pragma unroll
      for (int k = 0; k < 8; ++k) {
        const int r = r0 + wv + kLzWaves * k;
        p[k] = a.V[static_cast<int64_t>(r <= a.j ? r : a.j) * a.ldc + cc];
      }
    }
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      const int r = r0 + wv + kLzWaves * k;
      p[k] = ok && r <= a.j ? p[k] * x : 0.0;
    }
    row_sums<8>(p, t, lane);
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      const int r = r0 + wv + kLzWaves * k;
      if (lane == k && r <= a.j) hp[static_cast<int64_t>(blockIdx.x) * a.hstride + r] = t[k];
    }
  }
}

// hs[r] = sum over the slabs of hp[s * hstride + r], r <= j: lane l takes the
// slabs s = l (mod 64) of eight rows at a time, then one row_sums.
__device__ inline void lz_gather(const LanczosArgs& a, const double* hp, double* hs) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  for (int r0 = 0; r0 <= a.j; r0 += kLzRows) {
    double p[8], t[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) p[k] = 0.0;
    for (int sl = lane; sl < a.nslab; sl += 64) {
      double v[8];
#pragma unroll
      for (int k = 0; k < 8; ++k) {
        const int r = r0 + wv + kLzWaves * k;
        v[k] = hp[static_cast<int64_t>(sl) * a.hstride + (r <= a.j ? r : a.j)];
      }
#pragma unroll
      for (int k = 0; k < 8; ++k) p[k] += r0 + wv + kLzWaves * k <= a.j ? v[k] : 0.0;
    }
    row_sums<8>(p, t, lane);
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      const int r = r0 + wv + kLzWaves * k;
      if (lane == k && r <= a.j) hs[r] = t[k];
    }
  }
  __syncthreads();
}

__device__ inline double lz_tree(const double (*acc)[64], int lane) {
  return ((acc[0][lane] + acc[1][lane]) + (acc[2][lane] + acc[3][lane])) +
         ((acc[4][lane] + acc[5][lane]) + (acc[6][lane] + acc[7][lane]));
}

// w - sum_{r <= j} hs[r] V[r][c]: each wave sums its rows (eight loads in
// flight), the eight partial sums meet in LDS (acc, 8 x 64).  Returns the new
// w of the lane's column in every wave.  v0 as in lz_dots.
__device__ inline double lz_subtract(const LanczosArgs& a, int64_t c, bool ok, double w,
                                     const double* hs, double (*acc)[64], const double (&v0)[8]) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int64_t cc = ok ? c : 0;
  double s = 0.0;
  for (int r0 = 0; r0 <= a.j; r0 += kLzRows) {
    double v[8];
    if (r0 == 0) {
#pragma unroll
      for (int k = 0; k < 8; ++k) v[k] = v0[k];
    } else {
#pragma unroll
      for (int k = 0; k < 8; ++k) {
        const int r = r0 + wv + kLzWaves * k;
        v[k] = a.V[static_cast<int64_t>(r <= a.j ? r : a.j) * a.ldc + cc];
      }
    }
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      const int r = r0 + wv + kLzWaves * k;
      const int rc = r <= a.j ? r : a.j;
      s = fma(r <= a.j ? hs[rc] : 0.0, ok ? v[k] : 0.0, s);
    }
  }
  acc[wv][lane] = s;
  __syncthreads();
  return w - lz_tree(acc, lane);
}

// Sum of nslab per-slab values in slab order (wave 0 of the workgroup; the
// same order in every workgroup).
__device__ inline double lz_slab_sum(const double* v, int32_t nslab, int lane) {
  double t = 0.0;
  for (int sl = lane; sl < nslab; sl += 64) t += v[sl];
  return wave_sum_dpp(t);
}

// Launch 1: w (the operator's output, or first its sum scale * sum_t part[t]
// over the single pass's partial rows, in FP64: wave wv takes tiles t = wv
// (mod 8), sixteen loads in flight) and the first Gram-Schmidt pass's dot
// partials.
template <typename TP>
__global__ __launch_bounds__(64 * kLzWaves) void k_lz_first(LanczosArgs a, const TP* part,
                                                            int64_t ldp, int32_t ntiles,
                                                            double scale) {
  __shared__ double acc[kLzWaves][64];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int64_t c = static_cast<int64_t>(blockIdx.x) * kLzSlab + lane;
  const bool ok = c < a.ldc;
  double v0[8];
  lz_first_rows(a, c, ok, v0);
  double w = 0.0;
  if (part) {
    double s = 0.0;
    const int64_t cc = ok ? c : 0;
    if (ntiles > 0) {
      for (int t0 = wv; t0 < ntiles; t0 += 16 * kLzWaves) {
        double v[16];
#pragma unroll
        for (int q = 0; q < 16; ++q) {
          const int t = t0 + kLzWaves * q;
          v[q] = static_cast<double>(part[static_cast<int64_t>(t < ntiles ? t : ntiles - 1) * ldp + cc]);
        }
#pragma unroll
        for (int q = 0; q < 16; ++q) v[q] = ok && t0 + kLzWaves * q < ntiles ? v[q] : 0.0;
        double u[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) u[q] = (v[4 * q] + v[4 * q + 1]) + (v[4 * q + 2] + v[4 * q + 3]);
        s += (u[0] + u[1]) + (u[2] + u[3]);
      }
    }
    acc[wv][lane] = s;
    __syncthreads();
    w = scale * lz_tree(acc, lane);
    if (ok && wv == 0) a.w[c] = w;
  } else if (ok) {
    w = a.w[c];
  }
  lz_dots(a, c, ok, w, a.hp, v0);
}

// Launch 2: w1 = w - V^T h (first pass), the second pass's dot partials and
// the slab's part of ||w1||^2.
__global__ __launch_bounds__(64 * kLzWaves) void k_lz_second(LanczosArgs a) {
  __shared__ double hs[kLzMaxRows];
  __shared__ double acc[kLzWaves][64];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int64_t c = static_cast<int64_t>(blockIdx.x) * kLzSlab + lane;
  const bool ok = c < a.ldc;
  double v0[8];
  lz_first_rows(a, c, ok, v0);
  const double wc = ok ? a.w[c] : 0.0;
  lz_gather(a, a.hp, hs);
  const double w = lz_subtract(a, c, ok, wc, hs, acc, v0);
  lz_dots(a, c, ok, w, a.hp + static_cast<int64_t>(a.nslab) * a.hstride, v0);
  if (wv == 0) {
    if (ok) a.w[c] = w;
    const double t = wave_sum_dpp(ok ? w * w : 0.0);
    if (lane == 0) a.np[blockIdx.x] = t;
  }
}

// Launch 3: w2 = w1 - V^T h2 (second pass), beta_j = sqrt(||w1||^2 - ||h2||^2)
// (every workgroup sums the slab norms and h2 in the same order), alpha_j =
// both passes' coefficients of V[j] (workgroup 0), V[j + 1] = w2 / beta_j and
// its FP32 rounding when vnext32 is non-null.
__global__ __launch_bounds__(64 * kLzWaves) void k_lz_third(LanczosArgs a) {
  __shared__ double hs[kLzMaxRows];
  __shared__ double acc[kLzWaves][64];
  __shared__ double beta_sh;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int64_t c = static_cast<int64_t>(blockIdx.x) * kLzSlab + lane;
  const bool ok = c < a.ldc;
  double v0[8];
  lz_first_rows(a, c, ok, v0);
  const double wc = ok ? a.w[c] : 0.0;
  lz_gather(a, a.hp + static_cast<int64_t>(a.nslab) * a.hstride, hs);
  if (wv == 0) {
    double h2 = 0.0;
    for (int r = lane; r <= a.j; r += 64) h2 = fma(hs[r], hs[r], h2);
    h2 = wave_sum_dpp(h2);
    const double n1 = lz_slab_sum(a.np, a.nslab, lane);
    const double b = sqrt(fmax(n1 - h2, 0.0));
    if (lane == 0) beta_sh = b;
    if (blockIdx.x == 0) {
      double a1 = 0.0;
      for (int sl = lane; sl < a.nslab; sl += 64) a1 += a.hp[static_cast<int64_t>(sl) * a.hstride + a.j];
      a1 = wave_sum_dpp(a1);
      if (lane == 0) {
        const double al = a1 + hs[a.j];
        a.beta[a.j] = b;
        a.alpha[a.j] = al;
        if (a.host_ab) {
          a.host_ab[a.j] = al;
          a.host_ab[a.hstride + a.j] = b;
        }
      }
    }
  }
  // (lz_subtract's barrier also publishes beta_sh.)
  const double w = lz_subtract(a, c, ok, wc, hs, acc, v0);
  const double b = beta_sh;
  const double inv = b > 0.0 ? 1.0 / b : 0.0;
  if (wv == 0 && ok) {
    const double v = w * inv;
    a.vnext[c] = v;
    if (a.vnext32) a.vnext32[c] = static_cast<float>(v);
  }
}

// The Lanczos start vector: v[c] = u_c - 1/2 for c < n, u_c the top 53 bits of
// splitmix64(seed + c) as a fraction of 2^53, zero for n <= c < ldc; then
// v /= ||v||.  One workgroup (the norm in a fixed order).
__device__ inline double lz_start_value(uint64_t seed, int64_t c) {
  uint64_t x = seed + static_cast<uint64_t>(c) + 0x9E3779B97F4A7C15ull;
  x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ull;
  x = (x ^ (x >> 27)) * 0x94D049BB133111EBull;
  x ^= x >> 31;
  return static_cast<double>(x >> 11) * (1.0 / 9007199254740992.0) - 0.5;
}
__global__ __launch_bounds__(1024) void k_lz_start(uint64_t seed, int64_t n, int64_t ldc, double* v,
                                                   float* v32) {
  __shared__ double part[1024 / 64];
  __shared__ double inv_sh;
  double s = 0.0;
  for (int64_t c = threadIdx.x; c < n; c += 1024) {
    const double x = lz_start_value(seed, c);
    s = fma(x, x, s);
  }
  s = wave_sum_dpp(s);
  if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int w = 0; w < 1024 / 64; ++w) t += part[w];
    inv_sh = 1.0 / sqrt(t);
  }
  __syncthreads();
  const double inv = inv_sh;
  for (int64_t c = threadIdx.x; c < ldc; c += 1024) {
    const double x = c < n ? lz_start_value(seed, c) * inv : 0.0;
    v[c] = x;
    if (v32) v32[c] = static_cast<float>(x);
  }
}

// ------------------------------------------------------------------ residual

constexpr int kResRows = 8;
__global__ __launch_bounds__(256) void k_residual_partial(const double* A, int64_t lda,
                                                          const double* B, int64_t ldb, int64_t N,
                                                          int64_t n, const double* x,
                                                          double* partial) {
  __shared__ double red[4][kResRows];
  const int lane = threadIdx.x & 63;
  const int wv = threadIdx.x >> 6;
  const int64_t row0 = static_cast<int64_t>(blockIdx.x) * kResRows;
  double acc[kResRows];
#pragma unroll
  for (int r = 0; r < kResRows; ++r) acc[r] = 0.0;
  if (x) {
    for (int64_t j = threadIdx.x; j < n; j += 256) {
      const double xj = x[j];
#pragma unroll
      for (int r = 0; r < kResRows; ++r)
        if (row0 + r < N) acc[r] = fma(A[(row0 + r) * lda + j], xj, acc[r]);
    }
  }
#pragma unroll
  for (int r = 0; r < kResRows; ++r) {
    const double v = wave_sum(acc[r]);
    if (lane == 0) red[wv][r] = v;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double s = 0.0;
    for (int r = 0; r < kResRows; ++r) {
      if (row0 + r >= N) break;
      const double ax = (red[0][r] + red[1][r]) + (red[2][r] + red[3][r]);
      const double res = B[(row0 + r) * ldb] - ax;
      s = fma(res, res, s);
    }
    partial[blockIdx.x] = s;
  }
}

__global__ __launch_bounds__(256) void k_sum_partials(const double* partial, int32_t count,
                                                      double* out) {
  __shared__ double part[4];
  double s = 0.0;
  for (int e = threadIdx.x; e < count; e += 256) s += partial[e];
  s = wave_sum(s);
  if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) out[0] = (part[0] + part[1]) + (part[2] + part[3]);
}

}  // namespace

// ------------------------------------------------------------------ launchers

template <typename TQ, typename TA>
static hipError_t rowdot_impl(const RowdotArgs<TQ, TA>& a, hipStream_t s) {
  if (a.ntiles <= 0) return hipSuccess;
  const int total = a.ntiles * a.nsplit;
  unsigned grid = static_cast<unsigned>(total);
  if (a.xcd_remap == 1) grid = static_cast<unsigned>(((total + kXcds - 1) / kXcds) * kXcds);
  constexpr int U = rowdot_unroll<TQ>();
#define APC_ROWDOT_CASE(R)                                                                  \
  case R:                                                                                   \
    if (a.nt_loads)                                                                         \
      APC_LAUNCH((k_rowdot<TQ, TA, R, U, true>), dim3(grid), dim3(kThreads), 0, s, a);  \
    else                                                                                    \
      APC_LAUNCH((k_rowdot<TQ, TA, R, U, false>), dim3(grid), dim3(kThreads), 0, s, a); \
    break;
  switch (a.rows_per_tile) {
    APC_ROWDOT_CASE(8)
    APC_ROWDOT_CASE(16)
    APC_ROWDOT_CASE(32)
    default:
      return hipErrorInvalidValue;
  }
#undef APC_ROWDOT_CASE
  return hipGetLastError();
}

hipError_t launch_rowdot_f64(const RowdotArgs<double, double>& a, hipStream_t s) { return rowdot_impl(a, s); }
hipError_t launch_rowdot_f32(const RowdotArgs<float, float>& a, hipStream_t s) { return rowdot_impl(a, s); }
hipError_t launch_rowdot_f32x64(const RowdotArgs<float, double>& a, hipStream_t s) { return rowdot_impl(a, s); }

template <typename TQ>
static hipError_t pass_b_impl(const PassBArgs<TQ>& a, hipStream_t s) {
  const unsigned grid = static_cast<unsigned>(a.nslab) * static_cast<unsigned>(a.m);
  if (grid == 0) return hipSuccess;
  if (a.row_split) {
    if (a.nt_loads)
      APC_LAUNCH((k_pass_b_rows<TQ, true>), dim3(grid), dim3(kThreads), 0, s, a);
    else
      APC_LAUNCH((k_pass_b_rows<TQ, false>), dim3(grid), dim3(kThreads), 0, s, a);
  } else if (a.nt_loads) {
    APC_LAUNCH((k_pass_b<TQ, 8, true>), dim3(grid), dim3(kThreads), 0, s, a);
  } else {
    APC_LAUNCH((k_pass_b<TQ, 8, false>), dim3(grid), dim3(kThreads), 0, s, a);
  }
  return hipGetLastError();
}

hipError_t launch_pass_b_f64(const PassBArgs<double>& a, hipStream_t s) { return pass_b_impl(a, s); }
hipError_t launch_pass_b_f32(const PassBArgs<float>& a, hipStream_t s) { return pass_b_impl(a, s); }

template <typename TD>
static hipError_t combine_impl(const double* x, int64_t ldx, int32_t m, int64_t n, double alpha,
                               double beta, double* xbar, TD* d, int64_t ldd, hipStream_t s) {
  APC_LAUNCH((k_combine<TD>), dim3(grid_for(n, 64)), dim3(256), 0, s, x, ldx, m, n, alpha,
                     beta, xbar, d, ldd);
  return hipGetLastError();
}

hipError_t launch_combine_f64(const double* x, int64_t ldx, int32_t m, int64_t n, double alpha,
                              double beta, double* xbar, double* d, int64_t ldd, hipStream_t s) {
  return combine_impl(x, ldx, m, n, alpha, beta, xbar, d, ldd, s);
}

hipError_t launch_combine_f32(const double* x, int64_t ldx, int32_t m, int64_t n, double alpha,
                              double beta, double* xbar, float* d, int64_t ldd, hipStream_t s) {
  return combine_impl(x, ldx, m, n, alpha, beta, xbar, d, ldd, s);
}

template <typename TQ>
static hipError_t expand_impl(const ExpandArgs<TQ>& a, hipStream_t s) {
  const unsigned grid = static_cast<unsigned>(a.nslab) * static_cast<unsigned>(a.m);
  if (grid == 0) return hipSuccess;
  hipLaunchKernelGGL((k_expand<TQ>), dim3(grid), dim3(kThreads), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_expand_f64(const ExpandArgs<double>& a, hipStream_t s) { return expand_impl(a, s); }

int fused_cpt(int64_t ldc, int elem_bytes) {
  const int64_t chunks = ldc * elem_bytes / 16;
  for (int c = 1; c <= 16; c *= 2)
    if (chunks <= static_cast<int64_t>(kThreads) * c) return c;
  return 0;
}

template <typename TQ, typename TA, int CPT, int G>
static hipError_t fused_launch(const FusedArgs<TQ, TA>& a, hipStream_t s) {
  const unsigned grid = a.xcd_remap == 1
                            ? static_cast<unsigned>((a.ntiles + kXcds - 1) / kXcds * kXcds)
                            : static_cast<unsigned>(a.ntiles);
  if (grid == 0) return hipSuccess;
  APC_LAUNCH((k_fused<TQ, TA, CPT, G>), dim3(grid), dim3(kThreads), 0, s, a);
  return hipGetLastError();
}

// Register estimate of a (cpt, g) shape per thread, in 32-bit registers: two
// groups of g rows x cpt chunks of 16 bytes, plus d_blk and the partial sum
// (cpt chunks of 16 / sizeof(TQ) elements of TA each).  Shapes over 256 spill
// or leave no room for addresses, so launchers refuse them.
constexpr int fused_regs(int q_bytes, int a_bytes, int cpt, int g) {
  return 8 * g * cpt + 2 * cpt * (16 / q_bytes) * a_bytes / 4;
}
bool fused_shape_ok(int q_bytes, int a_bytes, int cpt, int g) {
  return cpt >= 1 && (g == 1 || g == 2 || g == 4) && fused_regs(q_bytes, a_bytes, cpt, g) <= 256;
}

template <typename TQ, typename TA, int CPT>
static hipError_t fused_g(const FusedArgs<TQ, TA>& a, int g, hipStream_t s) {
  constexpr int q = sizeof(TQ), e = sizeof(TA);
  switch (g) {
    case 1:
      if constexpr (fused_regs(q, e, CPT, 1) <= 256) return fused_launch<TQ, TA, CPT, 1>(a, s);
      break;
    case 2:
      if constexpr (fused_regs(q, e, CPT, 2) <= 256) return fused_launch<TQ, TA, CPT, 2>(a, s);
      break;
    case 4:
      if constexpr (fused_regs(q, e, CPT, 4) <= 256) return fused_launch<TQ, TA, CPT, 4>(a, s);
      break;
    default: break;
  }
  return hipErrorInvalidValue;
}

template <typename TQ, typename TA>
static hipError_t fused_impl(const FusedArgs<TQ, TA>& a, int g, hipStream_t s) {
  switch (fused_cpt(a.ldc, sizeof(TQ))) {
    case 1: return fused_g<TQ, TA, 1>(a, g, s);
    case 2: return fused_g<TQ, TA, 2>(a, g, s);
    case 4: return fused_g<TQ, TA, 4>(a, g, s);
    case 8: return fused_g<TQ, TA, 8>(a, g, s);
    case 16: return fused_g<TQ, TA, 16>(a, g, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_fused_f32(const FusedArgs<float, float>& a, int g, hipStream_t s) {
  return fused_impl(a, g, s);
}
hipError_t launch_fused_f64(const FusedArgs<double, double>& a, int g, hipStream_t s) {
  return fused_impl(a, g, s);
}
hipError_t launch_fused_f32x64(const FusedArgs<float, double>& a, int g, hipStream_t s) {
  return fused_impl(a, g, s);
}

hipError_t launch_block_sum(const double* part, int64_t ldp, const int32_t* tile_first, int32_t m,
                            int64_t ncols, double* out, int64_t ldo, hipStream_t s) {
  if (m <= 0 || ncols <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_block_sum, dim3(grid_for(ncols, 256), static_cast<unsigned>(m)), dim3(256),
                     0, s, part, ldp, tile_first, ncols, out, ldo);
  return hipGetLastError();
}

hipError_t launch_defect(const double* U, const double* V, int64_t ld, int32_t m, int64_t n,
                         double* out, hipStream_t s) {
  if (m <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_defect, dim3(static_cast<unsigned>(m)), dim3(256), 0, s, U, V, ld, n, out);
  return hipGetLastError();
}

hipError_t launch_defect_rows(const double* w, int32_t nsplit, int64_t wstride, const double* y,
                              const int64_t* off, int32_t m, double* h, hipStream_t s) {
  if (m <= 0) return hipSuccess;
  if (nsplit < 1) return hipErrorInvalidValue;
  const unsigned grid = static_cast<unsigned>(std::min<int32_t>(m, 65536));
  hipLaunchKernelGGL(k_defect_rows, dim3(grid), dim3(256), 0, s, w, nsplit, wstride, y, off, m,
                     h);
  return hipGetLastError();
}

hipError_t launch_fused_sum(const double* part, int64_t ldp, int32_t ntiles, int64_t n,
                            double alpha, double* out, hipStream_t s) {
  APC_LAUNCH(k_fused_sum<double>, dim3(grid_for(n, 32)), dim3(256), 0, s, part, ldp, ntiles, n,
             alpha, out);
  return hipGetLastError();
}
hipError_t launch_fused_sum_f32(const float* part, int64_t ldp, int32_t ntiles, int64_t n,
                                double alpha, double* out, hipStream_t s) {
  APC_LAUNCH(k_fused_sum<float>, dim3(grid_for(n, 32)), dim3(256), 0, s, part, ldp, ntiles, n,
             alpha, out);
  return hipGetLastError();
}

template <typename TD>
static hipError_t fused_combine_impl(const FusedCombineArgs<TD>& a, hipStream_t s) {
  const dim3 grid(grid_for(a.n, kCombineCols));
  switch (a.tpb) {
    case 1: APC_LAUNCH((k_fused_combine<TD, 1>), grid, dim3(256), 0, s, a); break;
    case 2: APC_LAUNCH((k_fused_combine<TD, 2>), grid, dim3(256), 0, s, a); break;
    case 4: APC_LAUNCH((k_fused_combine<TD, 4>), grid, dim3(256), 0, s, a); break;
    case 8: APC_LAUNCH((k_fused_combine<TD, 8>), grid, dim3(256), 0, s, a); break;
    default: APC_LAUNCH((k_fused_combine<TD, 0>), grid, dim3(256), 0, s, a); break;
  }
  return hipGetLastError();
}
hipError_t launch_fused_combine_f32(const FusedCombineArgs<float>& a, hipStream_t s) {
  return fused_combine_impl(a, s);
}
hipError_t launch_fused_combine_f64(const FusedCombineArgs<double>& a, hipStream_t s) {
  return fused_combine_impl(a, s);
}

hipError_t launch_expand_f32(const ExpandArgs<float>& a, hipStream_t s) { return expand_impl(a, s); }

hipError_t launch_linv_apply(const int64_t* off, const int64_t* goff, int32_t m, int64_t pmax,
                             const double* Linv, const double* in, int64_t ldi, double* out,
                             int64_t ldo, int32_t kc, int32_t trans, double scale, hipStream_t s) {
  const dim3 grid(static_cast<unsigned>((pmax + 63) / 64), static_cast<unsigned>((kc + 63) / 64),
                  static_cast<unsigned>(m));
  if (trans)
    k_tri_apply<true><<<grid, 256, 0, s>>>(off, goff, Linv, in, ldi, out, ldo, kc, scale);
  else
    k_tri_apply<false><<<grid, 256, 0, s>>>(off, goff, Linv, in, ldi, out, ldo, kc, scale);
  return hipGetLastError();
}

hipError_t launch_axpy(int64_t count, double alpha, const double* x, double* y, hipStream_t s) {
  unsigned g = grid_for(count, 256);
  if (g > 8192) g = 8192;
  hipLaunchKernelGGL(k_axpy, dim3(g), dim3(256), 0, s, count, alpha, x, y);
  return hipGetLastError();
}

constexpr int kSumsqBlocks = 1024;
int sumsq_parts() { return kSumsqBlocks; }

hipError_t launch_sumsq(const double* src, int64_t count, double* partial, hipStream_t s) {
  hipLaunchKernelGGL(k_sumsq, dim3(kSumsqBlocks), dim3(256), 0, s, src, count, partial);
  return hipGetLastError();
}

hipError_t launch_copy_pad(const double* A, int64_t lda, const double* B, int64_t ldb, int64_t N,
                           int64_t n, double* C, int64_t ldc, double* c, int32_t k, int32_t kp,
                           hipStream_t s) {
  const unsigned g = N > 8192 ? 8192u : static_cast<unsigned>(N);
  hipLaunchKernelGGL(k_copy_pad, dim3(g), dim3(256), 0, s, A, lda, B, ldb, N, n, C, ldc, c, k, kp);
  return hipGetLastError();
}

hipError_t launch_gram(const double* C, int64_t ldc, const int64_t* off, const int32_t* tiles,
                       int32_t ntiles, const int64_t* goff, double* G, hipStream_t s) {
  if (ntiles <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_gram, dim3(ntiles), dim3(256), 0, s, C, ldc, off, tiles, goff, G);
  return hipGetLastError();
}

hipError_t launch_chol_inv(const int64_t* off, const int64_t* goff, int32_t m, int64_t pmax,
                           double* G, double* Linv, int* flags, double rank_tol, hipStream_t s) {
  hipLaunchKernelGGL(k_chol_inv, dim3(m), dim3(512), 0, s, off, goff, G, Linv, flags, rank_tol);
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const unsigned cols = static_cast<unsigned>((pmax + kNB - 1) / kNB);
  hipLaunchKernelGGL(k_tri_inv, dim3(cols, static_cast<unsigned>(m)), dim3(512), 0, s, off, goff,
                     G, Linv);
  return hipGetLastError();
}

hipError_t launch_trmm(const double* In, double* Out, int64_t ldc, const int64_t* off,
                       const int32_t* tiles, int32_t ntiles, const int64_t* goff,
                       const double* Linv, hipStream_t s) {
  if (ntiles <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_trmm, dim3(ntiles), dim3(256), 0, s, In, Out, ldc, off, tiles, goff, Linv);
  return hipGetLastError();
}

TimedLaunch& pending_timing() {
  static thread_local TimedLaunch t;
  return t;
}

hipError_t launch_pad_cast(int f32, const double* A, int64_t lda, int64_t N, int64_t n, void* C,
                           int64_t ldc, hipStream_t s) {
  const int grid = static_cast<int>(N > 65535 ? 65535 : N);
  if (grid <= 0) return hipSuccess;
  if (f32)
    hipLaunchKernelGGL(k_pad_cast<float>, dim3(grid), dim3(256), 0, s, A, lda, N, n,
                       static_cast<float*>(C), ldc);
  else
    hipLaunchKernelGGL(k_pad_cast<double>, dim3(grid), dim3(256), 0, s, A, lda, N, n,
                       static_cast<double*>(C), ldc);
  return hipGetLastError();
}

hipError_t launch_hbm_step(const double* Y, int64_t ldy, int32_t m, int64_t n, double alpha,
                           double beta, double* x, double* z, hipStream_t s) {
  const int64_t grid = (n + 63) / 64;
  if (grid <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_hbm_step, dim3(static_cast<unsigned>(grid)), dim3(256), 0, s, Y, ldy, m, n,
                     alpha, beta, x, z);
  return hipGetLastError();
}

hipError_t launch_cast_f32(const double* src, float* dst, int64_t count, hipStream_t s) {
  const unsigned g = grid_for(count, 256) > 4096 ? 4096 : grid_for(count, 256);
  hipLaunchKernelGGL(k_cast_f32, dim3(g), dim3(256), 0, s, src, dst, count);
  return hipGetLastError();
}

hipError_t launch_fill_u32(unsigned* p, int64_t count, unsigned v, hipStream_t s) {
  const unsigned g = grid_for(count, 256) > 1024 ? 1024 : grid_for(count, 256);
  hipLaunchKernelGGL(k_fill_u32, dim3(g), dim3(256), 0, s, p, count, v);
  return hipGetLastError();
}

hipError_t launch_copy_strided(const double* src, int64_t lds, double* dst, int64_t ldd,
                               int64_t rows, int64_t cols, hipStream_t s) {
  if (rows <= 0 || cols <= 0) return hipSuccess;
  unsigned g = cols == 1 ? grid_for(rows, 256) : static_cast<unsigned>(rows);
  if (g > 8192) g = 8192;
  hipLaunchKernelGGL(k_copy_strided, dim3(g), dim3(256), 0, s, src, lds, dst, ldd, rows, cols);
  return hipGetLastError();
}

hipError_t launch_copy_t(const double* src, int64_t lds, double* dst, int64_t ldd, int64_t n,
                         int32_t kcols, hipStream_t s) {
  unsigned g = grid_for(n * kcols, 256);
  if (g > 8192) g = 8192;
  hipLaunchKernelGGL(k_copy_t, dim3(g), dim3(256), 0, s, src, lds, dst, ldd, n, kcols);
  return hipGetLastError();
}

hipError_t launch_lanczos_step(const LanczosArgs& a, const void* part, bool part32, int64_t ldp,
                               int32_t ntiles, double scale, hipStream_t s) {
  if (a.j < 0 || a.j >= kLzMaxRows || a.nslab != (a.ldc + kLzSlab - 1) / kLzSlab)
    return hipErrorInvalidValue;
  const dim3 grid(static_cast<unsigned>(a.nslab)), block(64 * kLzWaves);
  if (part && part32)
    hipLaunchKernelGGL(k_lz_first<float>, grid, block, 0, s, a, static_cast<const float*>(part),
                       ldp, ntiles, scale);
  else
    hipLaunchKernelGGL(k_lz_first<double>, grid, block, 0, s, a, static_cast<const double*>(part),
                       ldp, ntiles, scale);
  hipLaunchKernelGGL(k_lz_second, grid, block, 0, s, a);
  hipLaunchKernelGGL(k_lz_third, grid, block, 0, s, a);
  return hipGetLastError();
}

hipError_t launch_lanczos_start(uint64_t seed, int64_t n, int64_t ldc, double* v, float* v32,
                                hipStream_t s) {
  hipLaunchKernelGGL(k_lz_start, dim3(1), dim3(1024), 0, s, seed, n, ldc, v, v32);
  return hipGetLastError();
}

int residual_parts(int64_t N) { return static_cast<int>((N + kResRows - 1) / kResRows); }

hipError_t launch_residual_partial(const double* A, int64_t lda, const double* B, int64_t ldb,
                                   int64_t N, int64_t n, const double* x, double* partial,
                                   int32_t* nparts, hipStream_t s) {
  const int g = residual_parts(N);
  *nparts = g;
  hipLaunchKernelGGL(k_residual_partial, dim3(g), dim3(256), 0, s, A, lda, B, ldb, N, n, x,
                     partial);
  return hipGetLastError();
}

hipError_t launch_sum_partials(const double* partial, int32_t count, double* out, hipStream_t s) {
  hipLaunchKernelGGL(k_sum_partials, dim3(1), dim3(256), 0, s, partial, count, out);
  return hipGetLastError();
}

}  // namespace apc
