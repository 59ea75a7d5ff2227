// Internal declarations shared by the HIP kernels and the host side of libapc.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace apc {

constexpr int kThreads = 256;       // threads per workgroup for streaming kernels
constexpr int kRowTile = 16;        // rows per pass-A workgroup
constexpr int kLdAlign = 64;        // padded row stride of the internal factor (elements)
constexpr int kGramTile = 64;       // FP64 setup GEMM tile edge
constexpr int kMaxBlockRows = 2048; // largest p_i the setup Cholesky accepts
constexpr int kXcds = 8;            // XCDs per MI355X; workgroups are dealt round-robin

// ---------------------------------------------------------------------------
// Streaming kernels (hot path)
// ---------------------------------------------------------------------------

// out[row] = sum_j C[row][j] * d_blk[j] for every row of every tile, with
// d_blk = va - vb[blk] (vb may be null: d = va), rounded to TQ.
template <typename TQ>
struct RowdotArgs {
  const TQ* C;
  int64_t ldc;
  const int32_t* tile_row0;   // null: uniform tiling of rows_total rows
  const int32_t* tile_nrows;
  const int32_t* tile_blk;
  int32_t ntiles;
  int32_t rows_total;
  const double* va;
  const double* vb;
  int64_t ldvb;
  TQ* out;
  int32_t xcd_remap;          // 1: give each XCD a contiguous range of tiles
};

// Pass B of eq. (2a)-(2b): x_i += gamma (x_bar - x_i - Q_i w_i), then the
// last workgroup of each column slab forms x_bar <- (eta/m) sum_i x_i +
// (1 - eta) x_bar for that slab.
template <typename TQ>
struct PassBArgs {
  const TQ* C;
  int64_t ldc;
  const int64_t* off;
  int32_t m;
  int32_t nslab;
  const TQ* w;
  double* x;
  int64_t ldx;
  double* xbar;
  double gamma;
  double eta;
  unsigned* counters;
  int32_t order;              // 0: slab-major workgroup order, 1: reversed block-major
};

// y_i = beta * y_i + alpha * sum_{r in block i} w[r] C[r][:]  (FP64).
// off == null: a single block of rows_total rows.
struct ExpandArgs {
  const double* C;
  int64_t ldc;
  const int64_t* off;
  int32_t m;
  int32_t nslab;
  int64_t rows_total;
  const double* w;
  double* y;
  int64_t ldy;
  double alpha;
  double beta;
};

hipError_t launch_rowdot_f64(const RowdotArgs<double>& a, hipStream_t s);
hipError_t launch_rowdot_f32(const RowdotArgs<float>& a, hipStream_t s);
hipError_t launch_pass_b_f64(const PassBArgs<double>& a, hipStream_t s);
hipError_t launch_pass_b_f32(const PassBArgs<float>& a, hipStream_t s);
hipError_t launch_expand(const ExpandArgs& a, hipStream_t s);

// out[j] = scale * sum_{i<m} y[i*ldy + j] for j < n (fixed block order).
hipError_t launch_block_sum(const double* y, int64_t ldy, int32_t m, int64_t n, double scale,
                            double* out, hipStream_t s);

// ---------------------------------------------------------------------------
// Setup kernels (FP64)
// ---------------------------------------------------------------------------

// C[r][j] = A[r*lda + j] (j < n), 0 for n <= j < ldc; c[r] = B[r*ldb].
hipError_t launch_copy_pad(const double* A, int64_t lda, const double* B, int64_t ldb, int64_t N,
                           int64_t n, double* C, int64_t ldc, double* c, hipStream_t s);
// G_i = C_i C_i^T for every block (tiles: (blk, ta, tb) with ta >= tb).
hipError_t launch_gram(const double* C, int64_t ldc, const int64_t* off, const int32_t* tiles,
                       int32_t ntiles, const int64_t* goff, double* G, hipStream_t s);
// Per block: Cholesky G_i = L L^T in place, Linv_i = L^{-1}, c_out = Linv c_in;
// flags[0] <- 1 + (first block whose pivot fails the rank test).
hipError_t launch_chol_inv(const int64_t* off, const int64_t* goff, int32_t m, double* G,
                           double* Linv, const double* c_in, double* c_out, int* flags,
                           double rank_tol, hipStream_t s);
// Out_i = Linv_i In_i for every block (tiles: (blk, ta, tc)).
hipError_t launch_trmm(const double* In, double* Out, int64_t ldc, const int64_t* off,
                       const int32_t* tiles, int32_t ntiles, const int64_t* goff,
                       const double* Linv, hipStream_t s);
hipError_t launch_cast_f32(const double* src, float* dst, int64_t count, hipStream_t s);
hipError_t launch_fill_u32(unsigned* p, int64_t count, unsigned v, hipStream_t s);
hipError_t launch_copy_strided(const double* src, int64_t lds, double* dst, int64_t ldd,
                               int64_t rows, int64_t cols, hipStream_t s);

// Lanczos helpers: alpha[j] = h[j] + h2[j]; beta[j] = ||y||; V[j+1] = y / beta[j].
hipError_t launch_lanczos_normalize(const double* y, int64_t n, const double* h, const double* h2,
                                    int32_t j, double* alpha, double* beta, double* vnext,
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

}  // namespace apc
