// HIP kernels (gfx950, wave64) for Accelerated Projection-based Consensus.
//
// Hot path, per update of eq. (2a)-(2b):
//   pass A  (k_rowdot)  w_i = Q_i^T (x_bar - x_i): one dot product per row of
//           the stacked factor C = [Q_1^T; ...; Q_m^T] (N x ldc, row-major),
//           streamed once with 16-byte loads, the difference vector held in
//           registers, one wave-level reduction per row.
//   pass B  (k_pass_b)  x_i += gamma (x_bar - x_i - Q_i w_i): each workgroup
//           owns one column slab of one block and streams that block's rows
//           once; the momentum average of eq. (2b) is fused into the
//           epilogue: the last workgroup to finish a slab (atomic ticket)
//           sums the m new x_i of that slab in block order and writes x_bar.
// Both passes are HBM-bound (one FMA per streamed element), so they are
// written for coalescing and memory-level parallelism, not for MFMA.
//
// Setup (FP64): CholeskyQR2 of every A_i^T -- Gram G_i = C_i C_i^T (LDS-tiled),
// per-block Cholesky + triangular inverse, C_i <- L_i^{-1} C_i -- applied
// twice; then x_i(0) = Q_i c_i and x_bar(0) = mean (Alg. 1 initialisation).

#include <hip/hip_runtime.h>

#include "apc_internal.h"

namespace apc {

namespace {

// ------------------------------------------------------------------ helpers

template <typename T>
struct V16;
template <>
struct V16<float> {
  static constexpr int W = 4;
  __device__ static inline void load(const float* p, float (&o)[4]) {
    const float4 v = *reinterpret_cast<const float4*>(p);
    o[0] = v.x; o[1] = v.y; o[2] = v.z; o[3] = v.w;
  }
};
template <>
struct V16<double> {
  static constexpr int W = 2;
  __device__ static inline void load(const double* p, double (&o)[2]) {
    const double2 v = *reinterpret_cast<const double2*>(p);
    o[0] = v.x; o[1] = v.y;
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

template <typename TQ, int ROWS, int U>
__global__ __launch_bounds__(kThreads) void k_rowdot(RowdotArgs<TQ> a) {
  constexpr int W = V16<TQ>::W;
  constexpr int SWEEP = kThreads * W;
  constexpr int CH = SWEEP * U;

  int L = blockIdx.x;
  if (a.xcd_remap) {
    const int per = (a.ntiles + kXcds - 1) / kXcds;
    L = (blockIdx.x % kXcds) * per + blockIdx.x / kXcds;
  }
  if (L >= a.ntiles) return;
  int row0, nrows, blk;
  if (a.tile_row0) {
    row0 = a.tile_row0[L];
    nrows = a.tile_nrows[L];
    blk = a.tile_blk[L];
  } else {
    row0 = L * ROWS;
    nrows = min(ROWS, a.rows_total - row0);
    blk = 0;
  }
  const double* vb = a.vb ? a.vb + static_cast<int64_t>(blk) * a.ldvb : nullptr;
  const int tcol = threadIdx.x * W;

  TQ acc[ROWS];
#pragma unroll
  for (int r = 0; r < ROWS; ++r) acc[r] = TQ(0);

  for (int64_t base = 0; base < a.ldc; base += CH) {
    TQ d[U][W];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int64_t j = base + u * SWEEP + tcol;
#pragma unroll
      for (int e = 0; e < W; ++e) {
        double v = 0.0;
        if (j < a.ldc) {
          v = a.va[j + e];
          if (vb) v -= vb[j + e];
        }
        d[u][e] = static_cast<TQ>(v);
      }
    }
#pragma unroll
    for (int r = 0; r < ROWS; ++r) {
      if (r < nrows) {
        const TQ* crow = a.C + static_cast<int64_t>(row0 + r) * a.ldc;
#pragma unroll
        for (int u = 0; u < U; ++u) {
          const int64_t j = base + u * SWEEP + tcol;
          if (j < a.ldc) {
            TQ q[W];
            V16<TQ>::load(crow + j, q);
#pragma unroll
            for (int e = 0; e < W; ++e) acc[r] = fma(q[e], d[u][e], acc[r]);
          }
        }
      }
    }
  }

  __shared__ TQ red[kThreads / 64][ROWS];
  const int lane = threadIdx.x & 63;
  const int wv = threadIdx.x >> 6;
#pragma unroll
  for (int r = 0; r < ROWS; ++r) {
    const TQ v = wave_sum(acc[r]);
    if (lane == 0) red[wv][r] = v;
  }
  __syncthreads();
  if (static_cast<int>(threadIdx.x) < nrows) {
    const int r = threadIdx.x;
    a.out[row0 + r] = (red[0][r] + red[1][r]) + (red[2][r] + red[3][r]);
  }
}

// ------------------------------------------------------------------ pass B

template <typename TQ, int RU>
__global__ __launch_bounds__(kThreads) void k_pass_b(PassBArgs<TQ> a) {
  constexpr int W = V16<TQ>::W;
  constexpr int SW = 64 * W;  // columns per slab
  int s, i;
  if (a.order == 0) {
    s = blockIdx.x / a.m;
    i = blockIdx.x % a.m;
  } else {
    i = a.m - 1 - static_cast<int>(blockIdx.x / a.nslab);
    s = blockIdx.x % a.nslab;
  }
  const int lane = threadIdx.x & 63;
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int64_t r0 = a.off[i];
  const int64_t r1 = a.off[i + 1];
  const int64_t col = static_cast<int64_t>(s) * SW + lane * W;

  TQ acc[W];
#pragma unroll
  for (int e = 0; e < W; ++e) acc[e] = TQ(0);
  if (col < a.ldc) {
    int64_t r = r0 + wv;
    for (; r + 4 * (RU - 1) < r1; r += 4 * RU) {
      TQ q[RU][W];
      TQ wr[RU];
#pragma unroll
      for (int u = 0; u < RU; ++u) {
        wr[u] = a.w[r + 4 * u];
        V16<TQ>::load(a.C + (r + 4 * u) * a.ldc + col, q[u]);
      }
#pragma unroll
      for (int u = 0; u < RU; ++u)
#pragma unroll
        for (int e = 0; e < W; ++e) acc[e] = fma(wr[u], q[u][e], acc[e]);
    }
    for (; r < r1; r += 4) {
      TQ q[W];
      const TQ wr = a.w[r];
      V16<TQ>::load(a.C + r * a.ldc + col, q);
#pragma unroll
      for (int e = 0; e < W; ++e) acc[e] = fma(wr, q[e], acc[e]);
    }
  }

  __shared__ TQ red[kThreads / 64][SW];
  __shared__ unsigned ticket;
#pragma unroll
  for (int e = 0; e < W; ++e) red[wv][lane * W + e] = acc[e];
  __syncthreads();

  const int t = threadIdx.x;
  const int64_t j = static_cast<int64_t>(s) * SW + t;
  const bool mine = (t < SW) && (j < a.ldc);
  if (mine) {
    const TQ pr = (red[0][t] + red[1][t]) + (red[2][t] + red[3][t]);
    double* xi = a.x + static_cast<int64_t>(i) * a.ldx;
    const double xo = xi[j];
    const double d = a.xbar[j] - xo;
    xi[j] = xo + a.gamma * (d - static_cast<double>(pr));
  }

  // Fused eq. (2b): publish this block's slab, take a ticket; the last of the
  // m workgroups of the slab forms the average in block order.
  __threadfence();
  __syncthreads();
  if (t == 0) ticket = atomicAdd(&a.counters[s], 1u);
  __syncthreads();
  if (ticket == static_cast<unsigned>(a.m - 1)) {
    __threadfence();
    if (mine) {
      double sum = 0.0;
      for (int ii = 0; ii < a.m; ++ii) sum += a.x[static_cast<int64_t>(ii) * a.ldx + j];
      a.xbar[j] = (a.eta / a.m) * sum + (1.0 - a.eta) * a.xbar[j];
    }
    if (t == 0) atomicExch(&a.counters[s], 0u);
  }
}

// ------------------------------------------------------------------ expand (FP64)

template <int RU>
__global__ __launch_bounds__(kThreads) void k_expand(ExpandArgs a) {
  constexpr int W = 2;
  constexpr int SW = 64 * W;
  const int s = blockIdx.x % a.nslab;
  const int i = blockIdx.x / a.nslab;
  const int lane = threadIdx.x & 63;
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int64_t r0 = a.off ? a.off[i] : 0;
  const int64_t r1 = a.off ? a.off[i + 1] : a.rows_total;
  const int64_t col = static_cast<int64_t>(s) * SW + lane * W;
  double acc[W] = {0.0, 0.0};
  if (col < a.ldc) {
    for (int64_t r = r0 + wv; r < r1; r += 4) {
      double q[W];
      const double wr = a.w[r];
      V16<double>::load(a.C + r * a.ldc + col, q);
      acc[0] = fma(wr, q[0], acc[0]);
      acc[1] = fma(wr, q[1], acc[1]);
    }
  }
  __shared__ double red[kThreads / 64][SW];
  red[wv][lane * W + 0] = acc[0];
  red[wv][lane * W + 1] = acc[1];
  __syncthreads();
  const int t = threadIdx.x;
  const int64_t j = static_cast<int64_t>(s) * SW + t;
  if (t < SW && j < a.ldc) {
    const double v = (red[0][t] + red[1][t]) + (red[2][t] + red[3][t]);
    double* yi = a.y + static_cast<int64_t>(i) * a.ldy;
    yi[j] = (a.beta == 0.0 ? 0.0 : a.beta * yi[j]) + a.alpha * v;
  }
}

__global__ void k_block_sum(const double* y, int64_t ldy, int32_t m, int64_t n, double scale,
                            double* out) {
  const int64_t j = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (j >= n) return;
  double s = 0.0;
  for (int i = 0; i < m; ++i) s += y[static_cast<int64_t>(i) * ldy + j];
  out[j] = scale * s;
}

// ------------------------------------------------------------------ setup

__global__ void k_copy_pad(const double* A, int64_t lda, const double* B, int64_t ldb, int64_t N,
                           int64_t n, double* C, int64_t ldc, double* c) {
  for (int64_t r = blockIdx.x; r < N; r += gridDim.x) {
    for (int64_t j = threadIdx.x; j < ldc; j += blockDim.x) C[r * ldc + j] = j < n ? A[r * lda + j] : 0.0;
    if (threadIdx.x == 0) c[r] = B[r * ldb];
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

// One workgroup per block.  G_i (p x p, row-major, full symmetric) is
// factored in place (lower triangle = L), then Linv = L^{-1} is formed row by
// row (zeros above the diagonal), then c_out = Linv c_in.
__global__ __launch_bounds__(1024) void k_chol_inv(const int64_t* off, const int64_t* goff,
                                                   double* G, double* Linv, const double* c_in,
                                                   double* c_out, int* flags, double rank_tol) {
  const int blk = blockIdx.x;
  const int64_t r0 = off[blk];
  const int p = static_cast<int>(off[blk + 1] - r0);
  double* Gb = G + goff[blk];
  double* Lb = Linv + goff[blk];
  const int tid = threadIdx.x;
  const int nt = blockDim.x;
  __shared__ double maxdiag;
  __shared__ int bad;
  if (tid == 0) {
    double mx = 0.0;
    for (int k = 0; k < p; ++k) mx = fmax(mx, Gb[static_cast<int64_t>(k) * p + k]);
    maxdiag = mx;
    bad = 0;
  }
  __syncthreads();
  for (int k = 0; k < p; ++k) {
    double piv = Gb[static_cast<int64_t>(k) * p + k];
    if (!(piv > rank_tol * maxdiag)) {  // also catches NaN
      if (tid == 0) bad = 1;
      piv = maxdiag > 0.0 ? maxdiag : 1.0;  // keep going without NaNs; result is flagged
    }
    const double lkk = sqrt(piv);
    __syncthreads();
    for (int i = k + 1 + tid; i < p; i += nt) Gb[static_cast<int64_t>(i) * p + k] /= lkk;
    if (tid == 0) Gb[static_cast<int64_t>(k) * p + k] = lkk;
    __syncthreads();
    const int q = p - k - 1;
    for (int64_t e = tid; e < static_cast<int64_t>(q) * q; e += nt) {
      const int ii = k + 1 + static_cast<int>(e / q);
      const int jj = k + 1 + static_cast<int>(e % q);
      if (jj <= ii)
        Gb[static_cast<int64_t>(ii) * p + jj] -=
            Gb[static_cast<int64_t>(ii) * p + k] * Gb[static_cast<int64_t>(jj) * p + k];
    }
    __syncthreads();
  }
  for (int r = 0; r < p; ++r) {
    const double* Lr = Gb + static_cast<int64_t>(r) * p;
    for (int c = tid; c < p; c += nt) {
      double v = 0.0;
      if (c <= r) {
        double s = (r == c) ? 1.0 : 0.0;
        for (int k = c; k < r; ++k) s -= Lr[k] * Lb[static_cast<int64_t>(k) * p + c];
        v = s / Lr[r];
      }
      Lb[static_cast<int64_t>(r) * p + c] = v;
    }
    __syncthreads();
  }
  for (int r = tid; r < p; r += nt) {
    double s = 0.0;
    for (int k = 0; k <= r; ++k) s += Lb[static_cast<int64_t>(r) * p + k] * c_in[r0 + k];
    c_out[r0 + r] = s;
  }
  if (tid == 0 && bad) atomicCAS(flags, 0, blk + 1);
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

__global__ __launch_bounds__(1024) void k_lanczos_normalize(const double* y, int64_t n,
                                                            const double* h, const double* h2,
                                                            int32_t j, double* alpha,
                                                            double* beta, double* vnext) {
  __shared__ double part[1024 / 64];
  __shared__ double bsh;
  double s = 0.0;
  for (int64_t e = threadIdx.x; e < n; e += blockDim.x) s = fma(y[e], y[e], s);
  s = wave_sum(s);
  if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int w = 0; w < static_cast<int>(blockDim.x / 64); ++w) t += part[w];
    const double b = sqrt(t);
    bsh = b;
    beta[j] = b;
    alpha[j] = h[j] + h2[j];
  }
  __syncthreads();
  const double b = bsh;
  const double inv = b > 0.0 ? 1.0 / b : 0.0;
  for (int64_t e = threadIdx.x; e < n; e += blockDim.x) vnext[e] = y[e] * inv;
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

template <typename TQ>
static hipError_t rowdot_impl(const RowdotArgs<TQ>& a, hipStream_t s) {
  if (a.ntiles <= 0) return hipSuccess;
  unsigned grid = static_cast<unsigned>(a.ntiles);
  if (a.xcd_remap) grid = static_cast<unsigned>(((a.ntiles + kXcds - 1) / kXcds) * kXcds);
  constexpr int U = sizeof(TQ) == 4 ? 4 : 2;
  hipLaunchKernelGGL((k_rowdot<TQ, kRowTile, U>), dim3(grid), dim3(kThreads), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_rowdot_f64(const RowdotArgs<double>& a, hipStream_t s) { return rowdot_impl(a, s); }
hipError_t launch_rowdot_f32(const RowdotArgs<float>& a, hipStream_t s) { return rowdot_impl(a, s); }

template <typename TQ>
static hipError_t pass_b_impl(const PassBArgs<TQ>& a, hipStream_t s) {
  const unsigned grid = static_cast<unsigned>(a.nslab) * static_cast<unsigned>(a.m);
  if (grid == 0) return hipSuccess;
  hipLaunchKernelGGL((k_pass_b<TQ, 8>), dim3(grid), dim3(kThreads), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_pass_b_f64(const PassBArgs<double>& a, hipStream_t s) { return pass_b_impl(a, s); }
hipError_t launch_pass_b_f32(const PassBArgs<float>& a, hipStream_t s) { return pass_b_impl(a, s); }

hipError_t launch_expand(const ExpandArgs& a, hipStream_t s) {
  const unsigned grid = static_cast<unsigned>(a.nslab) * static_cast<unsigned>(a.m);
  if (grid == 0) return hipSuccess;
  hipLaunchKernelGGL((k_expand<4>), dim3(grid), dim3(kThreads), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_block_sum(const double* y, int64_t ldy, int32_t m, int64_t n, double scale,
                            double* out, hipStream_t s) {
  hipLaunchKernelGGL(k_block_sum, dim3(grid_for(n, 256)), dim3(256), 0, s, y, ldy, m, n, scale, out);
  return hipGetLastError();
}

hipError_t launch_copy_pad(const double* A, int64_t lda, const double* B, int64_t ldb, int64_t N,
                           int64_t n, double* C, int64_t ldc, double* c, hipStream_t s) {
  const unsigned g = N > 8192 ? 8192u : static_cast<unsigned>(N);
  hipLaunchKernelGGL(k_copy_pad, dim3(g), dim3(256), 0, s, A, lda, B, ldb, N, n, C, ldc, c);
  return hipGetLastError();
}

hipError_t launch_gram(const double* C, int64_t ldc, const int64_t* off, const int32_t* tiles,
                       int32_t ntiles, const int64_t* goff, double* G, hipStream_t s) {
  if (ntiles <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_gram, dim3(ntiles), dim3(256), 0, s, C, ldc, off, tiles, goff, G);
  return hipGetLastError();
}

hipError_t launch_chol_inv(const int64_t* off, const int64_t* goff, int32_t m, double* G,
                           double* Linv, const double* c_in, double* c_out, int* flags,
                           double rank_tol, hipStream_t s) {
  hipLaunchKernelGGL(k_chol_inv, dim3(m), dim3(1024), 0, s, off, goff, G, Linv, c_in, c_out, flags,
                     rank_tol);
  return hipGetLastError();
}

hipError_t launch_trmm(const double* In, double* Out, int64_t ldc, const int64_t* off,
                       const int32_t* tiles, int32_t ntiles, const int64_t* goff,
                       const double* Linv, hipStream_t s) {
  if (ntiles <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_trmm, dim3(ntiles), dim3(256), 0, s, In, Out, ldc, off, tiles, goff, Linv);
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

hipError_t launch_lanczos_normalize(const double* y, int64_t n, const double* h, const double* h2,
                                    int32_t j, double* alpha, double* beta, double* vnext,
                                    hipStream_t s) {
  hipLaunchKernelGGL(k_lanczos_normalize, dim3(1), dim3(1024), 0, s, y, n, h, h2, j, alpha, beta,
                     vnext);
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
