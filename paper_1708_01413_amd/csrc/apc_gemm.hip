// Streaming contractions on the gfx950 matrix cores for k right-hand sides.
//
// With k > 1 every projection pass is a tall-skinny matrix product.  One
// kernel serves all of them:
//
//   part[s][c][r] = sum_{j in split s} M[r][j] * V[c][j]
//
// M (rows x K) is the large operand and is read exactly once: each lane loads
// four 16-byte pieces of a row per 256-byte step straight into MFMA operand
// registers (no LDS round trip).  V (one row per right-hand side, K
// contiguous) is small and re-read by every workgroup: one 256-byte-per-row
// step of it is staged in LDS and shared by the four waves.  Both operands
// are K-contiguous per row, so the per-update passes of the (y, x_bar) form
// of APC are
//
//   pass A:  W  = C  y     M = C   (N x n),  V = y^T (k x n)
//   pass B:  Z  = C^T W    M = C^T (n x N),  V = W^T (k x N)
//
// with C = [Q_1^T; ...; Q_m^T] kept in both orientations.  The same kernel in
// FP64 forms the minimum-norm start x_bar(0) = (1/m) C^T c and the
// refinement residual B - A X.
//
// K permutation: the MFMA instructions reduce over a K index that is only a
// label.  A step's 256 bytes of a row are sixteen 16-byte chunks; lane group g
// (lanes 16 g .. 16 g + 15) holds chunks g, 4 + g, 8 + g, 12 + g as pieces
// p = 0..3, and piece p feeds the p-th MFMA of the step (bf16: one 16x16x32,
// f32: four 16x16x4, f64: two 16x16x4).  In a row-major M one load instruction
// then reads 64 contiguous bytes of each of 16 rows, which measured 2-5 %
// faster than giving each lane one contiguous 64-byte run.  V is read from LDS
// with exactly the same (lane group, piece, element) -> K mapping, so the sum
// is over all of K.
//
// Fragment-packed M.  An MFMA operand gives each of 16 lanes its own row, so
// in a row-major M one load instruction touches 16 rows 32 KB apart and a
// step touches every row of the workgroup for 256 bytes only; a read-only
// probe of that pattern over 16384 x 16384 bf16 reached 4.6 TB/s.  M is
// therefore stored as tiles of 16 rows x one 256-byte step, each tile 4 KB
// contiguous in the order the lanes consume it: piece p of lane L (row L % 16,
// chunk 4 p + L / 16 of the step) at bytes (64 p + L) * 16 of the tile.  One
// load instruction then reads 1 KB contiguous, and the tiles are ordered by
// step, then row tile, so a workgroup's step is 16 RT KB contiguous per wave.
// The same probe reads this layout at 6.8-7.0 TB/s with non-temporal loads
// (each byte of M is read once per pass), which are the default for it; the
// tuner also times plain loads.  k_tn_pack writes it (frag = 1).
//
// Split-K partials are written per split and summed in a fixed order by the
// epilogue kernels, so results do not depend on timing.

#include <hip/hip_runtime.h>

#include <limits>

#include "apc_internal.h"
#include "apc_tn.h"

namespace apc {

namespace {

template <typename T, int RT, int NCT, int PF, int NT, int W>
__global__ __launch_bounds__(64 * W) void k_tn(TnArgs a) {
  __shared__ TnStage<NCT> vs;
  tn_block<T, RT, NCT, PF, NT, W>(a, blockIdx.x, vs);
}

template <typename T, int RT, int PF, int NT, int W>
hipError_t tn_nct_w(const TnArgs& a, hipStream_t s) {
  const int nct = a.kp >= 128 ? 8 : a.kp / 16;
  const int64_t ncg = a.kp / (16 * nct);
  const int64_t blocks = (a.rows / (16 * W * RT)) * ncg * a.nsplit;
  const dim3 grid(static_cast<unsigned>(blocks)), block(64 * W);
  switch (nct) {
    case 1:
      if constexpr (W == 4) APC_LAUNCH((k_tn<T, RT, 1, PF, NT, W>), grid, block, 0, s, a);
      else return hipErrorInvalidValue;
      break;
    case 2: APC_LAUNCH((k_tn<T, RT, 2, PF, NT, W>), grid, block, 0, s, a); break;
    case 4: APC_LAUNCH((k_tn<T, RT, 4, PF, NT, W>), grid, block, 0, s, a); break;
    case 8: APC_LAUNCH((k_tn<T, RT, 8, PF, NT, W>), grid, block, 0, s, a); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

// Eight-wave workgroups (two waves per SIMD where the registers allow) for
// bf16 / FP32 with non-temporal loads and one row tile per wave (up to four
// steps of prefetch) or two (up to two): twice the rows share each staged step
// of V.
template <typename T, int RT, int PF, int NT>
hipError_t tn_nct(const TnArgs& a, hipStream_t s) {
  if (a.waves == 8) {
    if constexpr (sizeof(T) <= 4 && (RT == 1 || (RT == 2 && PF <= 2)) && NT == 1)
      return tn_nct_w<T, RT, PF, NT, 8>(a, s);
    else
      return hipErrorInvalidValue;
  }
  return tn_nct_w<T, RT, PF, NT, 4>(a, s);
}

template <typename T, int PF, int NT>
hipError_t tn_rt(int rt, const TnArgs& a, hipStream_t s) {
  switch (rt) {
    case 1: return tn_nct<T, 1, PF, NT>(a, s);
    case 2: return tn_nct<T, 2, PF, NT>(a, s);
    case 4:
      if constexpr (sizeof(T) == 8) return hipErrorInvalidValue;
      else return tn_nct<T, 4, PF, NT>(a, s);
    default: return hipErrorInvalidValue;
  }
}

// Deeper prefetch (3 or 4 steps ahead) for shapes with one or two row tiles
// per wave, whose steps are short.
template <typename T, int PF, int NT>
hipError_t tn_rt_deep(int rt, const TnArgs& a, hipStream_t s) {
  if constexpr (sizeof(T) == 8) return hipErrorInvalidValue;  // FP64: registers
  else switch (rt) {
    case 1: return tn_nct<T, 1, PF, NT>(a, s);
    case 2: return tn_nct<T, 2, PF, NT>(a, s);
    default: return hipErrorInvalidValue;
  }
}

template <typename T>
hipError_t tn_pf(int rt, int pf, const TnArgs& a, hipStream_t s) {
  const int nt = a.nt ? 1 : 0;
  switch (pf * 2 + nt) {
    case 2: return tn_rt<T, 1, 0>(rt, a, s);
    case 3: return tn_rt<T, 1, 1>(rt, a, s);
    case 4: return tn_rt<T, 2, 0>(rt, a, s);
    case 5: return tn_rt<T, 2, 1>(rt, a, s);
    case 7: return tn_rt_deep<T, 3, 1>(rt, a, s);
    case 9: return tn_rt_deep<T, 4, 1>(rt, a, s);
    default: return hipErrorInvalidValue;
  }
}

// ------------------------------------------------------------------ epilogues

// out[c*ldo + r] = TQ(sum of the split partials), r < rows, c < kp.
template <typename P, typename TQ>
__global__ __launch_bounds__(256) void k_tn_sum_cast(const P* part, int32_t nsplit, int32_t kp,
                                                     int64_t ldp, int64_t rows, TQ* out, int64_t ldo) {
  const int64_t total = static_cast<int64_t>(kp) * rows;
  const int64_t stride = static_cast<int64_t>(kp) * ldp;
  for (int64_t e = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; e < total;
       e += static_cast<int64_t>(gridDim.x) * blockDim.x)
    sum_cast_elem(part, nsplit, ldp, rows, stride, out, ldo, e);
}

// The (y, x_bar) update, its start, or an anchor update; see TnUpdateArgs.
template <typename P, typename TQ>
__global__ __launch_bounds__(256) void k_tn_update(TnUpdateArgs a) {
  const int64_t total = static_cast<int64_t>(a.kp) * a.n;
  for (int64_t e = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; e < total;
       e += static_cast<int64_t>(gridDim.x) * blockDim.x)
    update_elem<P, TQ>(a, e);
}

// The same four entries per thread (every row length and stride a multiple of 4).
template <typename P, typename TQ>
__global__ __launch_bounds__(256) void k_tn_update4(TnUpdateArgs a) {
  const int64_t total = static_cast<int64_t>(a.kp) * a.n / 4;
  for (int64_t e = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; e < total;
       e += static_cast<int64_t>(gridDim.x) * blockDim.x)
    update4<P, TQ>(a, 4 * e);
}

template <typename P, typename TQ>
__global__ __launch_bounds__(256) void k_tn_sum_cast4(const P* part, int32_t nsplit, int32_t kp,
                                                      int64_t ldp, int64_t rows, TQ* out, int64_t ldo) {
  const int64_t total = static_cast<int64_t>(kp) * rows / 4;
  const int64_t stride = static_cast<int64_t>(kp) * ldp;
  for (int64_t e = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; e < total;
       e += static_cast<int64_t>(gridDim.x) * blockDim.x)
    sum_cast4(part, nsplit, ldp, rows, stride, out, ldo, 4 * e);
}

inline bool quad_ok(const void* p) { return reinterpret_cast<uintptr_t>(p) % 16 == 0; }

// y_ref = (1 - gamma) y + gamma x_bar (the vector the next update multiplies), FP64.
__global__ __launch_bounds__(256) void k_tn_anchor_vec(const double* y, const double* xb, int64_t count,
                                                       double gamma, double* yref) {
  for (int64_t e = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; e < count;
       e += static_cast<int64_t>(gridDim.x) * blockDim.x)
    yref[e] = (1.0 - gamma) * y[e] + gamma * xb[e];
}

// Operand yq = TQ((1 - gamma) y + gamma x_bar) after the state was restored.
template <typename TQ>
__global__ __launch_bounds__(256) void k_tn_prep(const double* y, const double* xb, int64_t count,
                                                 double gamma, TQ* yq) {
  for (int64_t e = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; e < count;
       e += static_cast<int64_t>(gridDim.x) * blockDim.x)
    yq[e] = cvt<TQ>((1.0 - gamma) * y[e] + gamma * xb[e]);
}

// One reverse step of the (y, x_bar) iteration; see TnAdjointArgs.  Each
// workgroup adds its own share of the dL/dgamma and dL/deta sums to red[2 b],
// red[2 b + 1] (grid fixed by the launcher, so the sums are deterministic).
template <typename P, typename TQ>
__global__ __launch_bounds__(256) void k_tn_adjoint(TnAdjointArgs a) {
  const int64_t total = static_cast<int64_t>(a.kp) * a.n;
  const int64_t stride = static_cast<int64_t>(a.kp) * a.ldp;
  const P* part = static_cast<const P*>(a.part);
  TQ* bq = static_cast<TQ*>(a.bq);
  const double g = a.gamma, eta = a.eta;
  double sg = 0.0, se = 0.0;
  for (int64_t e = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; e < total;
       e += static_cast<int64_t>(gridDim.x) * blockDim.x) {
    const int64_t c = e / a.n, j = e - c * a.n;
    const int64_t i = c * a.ldx + j;
    const double xbh = split_sum(part, a.nsplit, stride, c * a.ldp + j) * a.inv_m;  // X b
    const double bh = a.bh[i];
    const double at = a.a[i] + eta * (bh - xbh);
    sg += at * (a.xb_t[i] - a.y_t[i]);
    se += bh * (a.xb_next[i] - a.xb_t[i]);
    a.g0[i] += eta * bh;
    a.a[i] = (1.0 - g) * at;
    const double bn = (1.0 - eta) * bh + g * at;
    a.bh[i] = bn;
    bq[c * a.ldq + j] = cvt<TQ>(bn);
  }
  __shared__ double rs[2][256];
  rs[0][threadIdx.x] = sg;
  rs[1][threadIdx.x] = se;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) {
      rs[0][threadIdx.x] += rs[0][threadIdx.x + o];
      rs[1][threadIdx.x] += rs[1][threadIdx.x + o];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    a.red[2 * blockIdx.x] += rs[0][0];
    a.red[2 * blockIdx.x + 1] += rs[1][0] / eta;
  }
}

// R[c*ldr + r] = B[r*ldb + c] - sum of the FP64 split partials, r < N, c < k.
__global__ __launch_bounds__(256) void k_tn_resid(const double* part, int32_t nsplit, int32_t kp,
                                                  int64_t ldp, int64_t N, int32_t k, const double* B,
                                                  int64_t ldb, double* R, int64_t ldr) {
  const int64_t total = static_cast<int64_t>(k) * N;
  const int64_t stride = static_cast<int64_t>(kp) * ldp;
  for (int64_t e = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; e < total;
       e += static_cast<int64_t>(gridDim.x) * blockDim.x) {
    const int64_t r = e / k, c = e - r * k;  // B read row by row
    R[c * ldr + r] = B[r * ldb + c] - split_sum(part, nsplit, stride, c * ldp + r);
  }
}

// dst (drows x ldd, type TQ) = src or src^T (FP64, srows x scols, stride lds),
// zero outside the source.  64 x 64 tiles through LDS for the transpose.
// frag = 1 writes the fragment-packed layout of k_tn's M operand instead of
// row-major (then drows % 16 == 0 and ldd is a multiple of the step).
template <typename TQ>
__global__ __launch_bounds__(256) void k_tn_pack(const double* src, int64_t lds, int64_t srows,
                                                 int64_t scols, int32_t transpose, TQ* dst,
                                                 int64_t ldd, int64_t drows, int32_t frag) {
  __shared__ double tile[64][65];
  const int64_t tiles_c = (ldd + 63) / 64;
  const int64_t tr = blockIdx.x / tiles_c, tc = blockIdx.x % tiles_c;
  const int64_t r0 = tr * 64, c0 = tc * 64;  // destination tile origin
  const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
  auto at = [&](int64_t r, int64_t c) { return frag ? frag_index<TQ>(r, c, drows) : r * ldd + c; };
  if (!transpose) {
    for (int rr = ty; rr < 64; rr += 4) {
      const int64_t r = r0 + rr, c = c0 + tx;
      if (r >= drows || c >= ldd) continue;
      const double v = (r < srows && c < scols) ? src[r * lds + c] : 0.0;
      dst[at(r, c)] = cvt<TQ>(v);
    }
    return;
  }
  // dst[r][c] = src[c][r]: read src rows c0.. (coalesced along r), write dst rows r0..
  for (int cc = ty; cc < 64; cc += 4) {
    const int64_t sr = c0 + cc, sc = r0 + tx;
    tile[cc][tx] = (sr < srows && sc < scols) ? src[sr * lds + sc] : 0.0;
  }
  __syncthreads();
  for (int rr = ty; rr < 64; rr += 4) {
    const int64_t r = r0 + rr, c = c0 + tx;
    if (r < drows && c < ldd) dst[at(r, c)] = cvt<TQ>(tile[tx][rr]);
  }
}

// One destination row's eight consecutive entries (columns c0 .. c0 + 7,
// c0 % 8 == 0) as whole 16-byte pieces of the fragment-packed layout: one
// piece in bf16, two in FP32, four in FP64.
template <typename TQ>
__device__ inline void store_frag8(TQ* dst, int64_t r, int64_t c0, int64_t rows, const double (&v)[8]) {
  constexpr int kE = 16 / sizeof(TQ);
#pragma unroll
  for (int h = 0; h < 8 / kE; ++h) {
    TQ w[kE];
#pragma unroll
    for (int e = 0; e < kE; ++e) w[e] = cvt<TQ>(v[kE * h + e]);
    u32x4 piece;
    __builtin_memcpy(&piece, w, 16);
    *reinterpret_cast<u32x4*>(dst + frag_index<TQ>(r, c0 + kE * h, rows)) = piece;
  }
}

struct PackMultiArgs {
  const double* src;
  int64_t lds, srows, scols;
  int32_t transpose;
  int32_t vec;     // 16-byte source loads: src 16-byte aligned, lds and scols even
  void* dq;        // fragment-packed, element type of the kernel
  void* d2;        // a second fragment-packed copy (null: none), FP64 or FP32
  int32_t d2_f64;  // its element type: 1 FP64, 0 FP32
  float* r32;      // row-major FP32, non-transposed packs only (null: none)
  int64_t ldr, r32rows, r32cols;
  int64_t K, rows;  // packed outputs: rows x K, rows % 16 == 0, K % 128 == 0
};

// Fragment-packed copies of an FP64 matrix (or of its transpose) from a single
// read of it: dq in the element type TQ, optionally d2 in FP64 or FP32, and for a
// non-transposed pack optionally the row-major FP32 copy r32[r * ldr + c] of
// rows < r32rows and columns < r32cols (r32cols % 8 == 0).  Entries outside
// the source are zero.  A workgroup takes units of 16 destination rows x 128
// destination columns: the unit's source block goes to LDS through loads that
// are contiguous across lanes (16 bytes each when vec, 8 otherwise; addresses
// clamped into the source and the value selected afterwards, so that no load
// sits behind a branch), then thread (r, o) writes entries (r, 8 o .. 8 o + 7)
// of the unit as whole 16-byte pieces of every packed output, sixteen
// consecutive threads filling 256 contiguous bytes.
constexpr int kPkPitch = 128 + 2;  // LDS row pitch in doubles (16-byte aligned rows)
template <typename TQ>
__global__ __launch_bounds__(256) void k_tn_pack_multi(PackMultiArgs a) {
  __shared__ __align__(16) double tile[16][kPkPitch];
  const int t = threadIdx.x;
  const int64_t ucols = a.K / 128;
  const int64_t units = (a.rows / 16) * ucols;
  for (int64_t u = blockIdx.x; u < units; u += gridDim.x) {
    const int64_t R0 = (u / ucols) * 16, C0 = (u % ucols) * 128;
    // tile[r][c] = dest (R0 + r, C0 + c) = src[R0 + r][C0 + c] or src[C0 + c][R0 + r].
    if (!a.transpose) {
      const int r = t >> 4;
      const int64_t sr = R0 + r;
      const bool rok = sr < a.srows;
      const double* row = a.src + (rok ? sr : 0) * a.lds;
      if (a.vec) {
        f64x2 v[4];
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const int64_t c = C0 + 2 * ((t & 15) + 16 * e);
          v[e] = *reinterpret_cast<const f64x2*>(row + (c < a.scols ? c : 0));
        }
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const int cl = 2 * ((t & 15) + 16 * e);
          const bool ok = rok && C0 + cl < a.scols;
          *reinterpret_cast<f64x2*>(&tile[r][cl]) = ok ? v[e] : f64x2{0.0, 0.0};
        }
      } else {
        double v[8];
#pragma unroll
        for (int e = 0; e < 8; ++e) {
          const int64_t c = C0 + (t & 15) + 16 * e;
          v[e] = row[c < a.scols ? c : 0];
        }
#pragma unroll
        for (int e = 0; e < 8; ++e) {
          const int cl = (t & 15) + 16 * e;
          tile[r][cl] = rok && C0 + cl < a.scols ? v[e] : 0.0;
        }
      }
    } else if (a.vec) {
      // Thread: source rows C0 + t / 8 + 32 e, columns R0 + 2 (t % 8) + {0, 1}
      // (scols even: both or neither inside).
      const int64_t sc = R0 + 2 * (t & 7);
      const bool cok = sc < a.scols;
      f64x2 v[4];
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int64_t sr = C0 + (t >> 3) + 32 * e;
        v[e] = *reinterpret_cast<const f64x2*>(a.src + (sr < a.srows ? sr : 0) * a.lds + (cok ? sc : 0));
      }
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int cl = (t >> 3) + 32 * e;
        const bool ok = cok && C0 + cl < a.srows;
        tile[2 * (t & 7)][cl] = ok ? v[e][0] : 0.0;
        tile[2 * (t & 7) + 1][cl] = ok ? v[e][1] : 0.0;
      }
    } else {
      // Thread: source rows C0 + t / 16 + 16 e, column R0 + t % 16.
      const int64_t sc = R0 + (t & 15);
      const bool cok = sc < a.scols;
      double v[8];
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const int64_t sr = C0 + (t >> 4) + 16 * e;
        v[e] = a.src[(sr < a.srows ? sr : 0) * a.lds + (cok ? sc : 0)];
      }
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const int cl = (t >> 4) + 16 * e;
        tile[t & 15][cl] = cok && C0 + cl < a.srows ? v[e] : 0.0;
      }
    }
    __syncthreads();
    {
      const int r = t & 15, o = t >> 4;
      double v[8];
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const f64x2 w = *reinterpret_cast<const f64x2*>(&tile[r][8 * o + 2 * e]);
        v[2 * e] = w[0];
        v[2 * e + 1] = w[1];
      }
      store_frag8(static_cast<TQ*>(a.dq), R0 + r, C0 + 8 * o, a.rows, v);
      if (a.d2) {
        if (a.d2_f64) store_frag8(static_cast<double*>(a.d2), R0 + r, C0 + 8 * o, a.rows, v);
        else store_frag8(static_cast<float*>(a.d2), R0 + r, C0 + 8 * o, a.rows, v);
      }
    }
    if (a.r32) {
      // Row-major: thread (r = t / 16, o = t % 16), 32 contiguous bytes each.
      const int r = t >> 4, o = t & 15;
      const int64_t gr = R0 + r, gc = C0 + 8 * o;
      if (gr < a.r32rows && gc < a.r32cols) {
        f32x4 lo, hi;
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          lo[e] = static_cast<float>(tile[r][8 * o + e]);
          hi[e] = static_cast<float>(tile[r][8 * o + 4 + e]);
        }
        float* d = a.r32 + gr * a.ldr + gc;
        *reinterpret_cast<f32x4*>(d) = lo;
        *reinterpret_cast<f32x4*>(d + 4) = hi;
      }
    }
    __syncthreads();
  }
}

unsigned grid_stride_blocks(int64_t total) {
  int64_t b = (total + 255) / 256;
  return static_cast<unsigned>(std::max<int64_t>(1, std::min<int64_t>(b, 8192)));
}

}  // namespace

hipError_t launch_tn(int type, int rt, int pf, const TnArgs& a, hipStream_t s) {
  if (a.kp < 16 || (a.kp > 128 && a.kp % 128) || (a.kp <= 128 && (a.kp & (a.kp - 1))) ||
      a.rows % (16 * (a.waves == 8 ? 8 : 4) * rt) || a.nsplit < 1 || a.nsplit > kTnMaxSplit ||
      (a.waves != 4 && a.waves != 8))
    return hipErrorInvalidValue;
  switch (type) {
    case kTnF64: return tn_pf<double>(rt, pf, a, s);
    case kTnF32: return tn_pf<float>(rt, pf, a, s);
    case kTnBF16: return tn_pf<__bf16>(rt, pf, a, s);
    default: return hipErrorInvalidValue;
  }
}

int tn_step_elems(int type) { return type == kTnF64 ? 32 : type == kTnF32 ? 64 : 128; }

hipError_t launch_tn_sum_cast(int type, const void* part, int32_t nsplit, int32_t kp, int64_t ldp,
                              int64_t rows, void* out, int64_t ldo, hipStream_t s) {
  // Four entries per thread where every row starts 16-byte aligned.
  const bool four = rows % 4 == 0 && ldp % 4 == 0 && ldo % 4 == 0 && quad_ok(part) &&
                    reinterpret_cast<uintptr_t>(out) % 16 == 0;
  const unsigned g = grid_stride_blocks(static_cast<int64_t>(kp) * rows / (four ? 4 : 1));
#define APC_SUM_CAST(P, TQ)                                                                      \
  do {                                                                                           \
    if (four)                                                                                    \
      APC_LAUNCH((k_tn_sum_cast4<P, TQ>), dim3(g), dim3(256), 0, s, static_cast<const P*>(part), \
                 nsplit, kp, ldp, rows, static_cast<TQ*>(out), ldo);                             \
    else                                                                                         \
      APC_LAUNCH((k_tn_sum_cast<P, TQ>), dim3(g), dim3(256), 0, s, static_cast<const P*>(part),  \
                 nsplit, kp, ldp, rows, static_cast<TQ*>(out), ldo);                             \
  } while (0)
  switch (type) {
    case kTnF64: APC_SUM_CAST(double, double); break;
    case kTnF32: APC_SUM_CAST(float, float); break;
    case kTnBF16: APC_SUM_CAST(float, __bf16); break;
    default: return hipErrorInvalidValue;
  }
#undef APC_SUM_CAST
  return hipGetLastError();
}

hipError_t launch_tn_update(int type, int part_f64, const TnUpdateArgs& a, hipStream_t s) {
  const bool four = a.n % 4 == 0 && a.ldp % 4 == 0 && a.ldx % 4 == 0 && a.ldq % 4 == 0 &&
                    quad_ok(a.part) && quad_ok(a.x0) && quad_ok(a.y) && quad_ok(a.xb) &&
                    quad_ok(a.yq) && (!a.yref || (quad_ok(a.yref) && quad_ok(a.uref)));
  const unsigned g = grid_stride_blocks(static_cast<int64_t>(a.kp) * a.n / (four ? 4 : 1));
#define APC_UPDATE(P, TQ)                                                            \
  do {                                                                               \
    if (four) APC_LAUNCH((k_tn_update4<P, TQ>), dim3(g), dim3(256), 0, s, a);        \
    else APC_LAUNCH((k_tn_update<P, TQ>), dim3(g), dim3(256), 0, s, a);              \
  } while (0)
  if (part_f64) {
    switch (type) {
      case kTnF64: APC_UPDATE(double, double); break;
      case kTnF32: APC_UPDATE(double, float); break;
      case kTnBF16: APC_UPDATE(double, __bf16); break;
      default: return hipErrorInvalidValue;
    }
  } else {
    switch (type) {
      case kTnF32: APC_UPDATE(float, float); break;
      case kTnBF16: APC_UPDATE(float, __bf16); break;
      default: return hipErrorInvalidValue;
    }
  }
#undef APC_UPDATE
  return hipGetLastError();
}

hipError_t launch_tn_anchor_vec(const double* y, const double* xb, int64_t count, double gamma,
                               double* yref, hipStream_t s) {
  k_tn_anchor_vec<<<grid_stride_blocks(count), 256, 0, s>>>(y, xb, count, gamma, yref);
  return hipGetLastError();
}

hipError_t launch_tn_prep(int type, const double* y, const double* xb, int64_t count, double gamma,
                          void* yq, hipStream_t s) {
  const unsigned g = grid_stride_blocks(count);
  switch (type) {
    case kTnF64: k_tn_prep<double><<<g, 256, 0, s>>>(y, xb, count, gamma, static_cast<double*>(yq)); break;
    case kTnF32: k_tn_prep<float><<<g, 256, 0, s>>>(y, xb, count, gamma, static_cast<float*>(yq)); break;
    case kTnBF16: k_tn_prep<__bf16><<<g, 256, 0, s>>>(y, xb, count, gamma, static_cast<__bf16*>(yq)); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

int tn_adjoint_blocks() { return kTnAdjointBlocks; }

hipError_t launch_tn_adjoint(int type, const TnAdjointArgs& a, hipStream_t s) {
  switch (type) {
    case kTnF64: k_tn_adjoint<double, double><<<kTnAdjointBlocks, 256, 0, s>>>(a); break;
    case kTnF32: k_tn_adjoint<float, float><<<kTnAdjointBlocks, 256, 0, s>>>(a); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_tn_resid(const double* part, int32_t nsplit, int32_t kp, int64_t ldp, int64_t N,
                           int32_t k, const double* B, int64_t ldb, double* R, int64_t ldr,
                           hipStream_t s) {
  k_tn_resid<<<grid_stride_blocks(static_cast<int64_t>(k) * N), 256, 0, s>>>(part, nsplit, kp, ldp,
                                                                           N, k, B, ldb, R, ldr);
  return hipGetLastError();
}

namespace {

hipError_t tn_pack(int type, const double* src, int64_t lds, int64_t srows, int64_t scols,
                   int32_t transpose, void* dst, int64_t ldd, int64_t drows, int32_t frag,
                   hipStream_t s) {
  const int64_t blocks = ((drows + 63) / 64) * ((ldd + 63) / 64);
  if (blocks < 1) return hipSuccess;
  const dim3 grid(static_cast<unsigned>(blocks));
  switch (type) {
    case kTnF64:
      k_tn_pack<double><<<grid, 256, 0, s>>>(src, lds, srows, scols, transpose,
                                             static_cast<double*>(dst), ldd, drows, frag);
      break;
    case kTnF32:
      k_tn_pack<float><<<grid, 256, 0, s>>>(src, lds, srows, scols, transpose,
                                            static_cast<float*>(dst), ldd, drows, frag);
      break;
    case kTnBF16:
      k_tn_pack<__bf16><<<grid, 256, 0, s>>>(src, lds, srows, scols, transpose,
                                             static_cast<__bf16*>(dst), ldd, drows, frag);
      break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace

hipError_t launch_tn_pack(int type, const double* src, int64_t lds, int64_t srows, int64_t scols,
                          int32_t transpose, void* dst, int64_t ldd, int64_t drows, hipStream_t s) {
  return tn_pack(type, src, lds, srows, scols, transpose, dst, ldd, drows, 0, s);
}

hipError_t launch_tn_pack_frag(int type, const double* src, int64_t lds, int64_t srows,
                               int64_t scols, int32_t transpose, void* dst, int64_t K,
                               int64_t rows, hipStream_t s) {
  return launch_tn_pack_frag_multi(type, src, lds, srows, scols, transpose, dst, K, rows, nullptr,
                                   0, nullptr, 0, 0, 0, s);
}

hipError_t launch_tn_pack_frag_multi(int type, const double* src, int64_t lds, int64_t srows,
                                     int64_t scols, int32_t transpose, void* dst, int64_t K,
                                     int64_t rows, void* d2, int type2, float* r32, int64_t ldr,
                                     int64_t r32rows, int64_t r32cols, hipStream_t s) {
  if (rows % 16 || K % tn_step_elems(type)) return hipErrorInvalidValue;
  if (d2 && (type2 == type || (type2 != kTnF64 && type2 != kTnF32) || K % tn_step_elems(type2)))
    return hipErrorInvalidValue;
  if ((r32 && (transpose || r32cols % 8 || ldr % 4 ||
                                          reinterpret_cast<uintptr_t>(r32) % 16 ||
                                          r32rows > rows || r32cols > K)))
    return hipErrorInvalidValue;
  if (K % 128 || srows < 1 || scols < 1) {
    // Shapes the unit kernel does not take: the element-wise kernel, once per output.
    if (r32) return hipErrorInvalidValue;
    const hipError_t e = tn_pack(type, src, lds, srows, scols, transpose, dst, K, rows, 1, s);
    if (e != hipSuccess || !d2) return e;
    return tn_pack(type2, src, lds, srows, scols, transpose, d2, K, rows, 1, s);
  }
  PackMultiArgs a{src, lds, srows, scols, transpose, 0, dst, d2, type2 == kTnF64 ? 1 : 0,
                  r32, ldr, r32rows, r32cols, K, rows};
  a.vec = reinterpret_cast<uintptr_t>(src) % 16 == 0 && lds % 2 == 0 && scols % 2 == 0;
  const int64_t units = (rows / 16) * (K / 128);
  if (units < 1) return hipSuccess;
  // Eight 256-thread workgroups per CU (16.6 KB of LDS each), grid-stride over the units.
  const unsigned grid = static_cast<unsigned>(std::min<int64_t>(units, 256 * 8));
  switch (type) {
    case kTnF64: k_tn_pack_multi<double><<<grid, 256, 0, s>>>(a); break;
    case kTnF32: k_tn_pack_multi<float><<<grid, 256, 0, s>>>(a); break;
    case kTnBF16: k_tn_pack_multi<__bf16><<<grid, 256, 0, s>>>(a); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace apc

namespace apc {

// ------------------------------------------------------------------ FP64 setup products
//
// The two products of CholeskyQR on the FP64 matrix cores: the Gram matrix
// G_i = C_i C_i^T and the triangular product Out_i = L_i^{-1} In_i, both with
// their operands staged in LDS by eight-wave workgroups.

namespace {

// Workgroups are dealt round-robin to the 8 XCDs; giving each XCD a
// contiguous range of work items keeps the items of one block (which read the
// same rows) on one XCD, so they share its L2.  (At 16384 x 8192 this measured
// the same as the plain order: the Infinity Cache already serves the re-reads.)
__device__ inline int xcd_contiguous(int b, int total) {
  const int per = (total + kXcds - 1) / kXcds;
  return (b % kXcds) * per + b / kXcds;
}

// Out_i = Linv_i In_i as 128 x 128 output tiles on the FP64 matrix cores,
// one workgroup per (block, 128-row tile, 128-column tile).  K (the block's
// rows, cut at the tile's last row since Linv is lower triangular) goes in
// chunks of 32: both operands are staged in LDS K-major -- As[k][r] =
// Linv[R0 + r][kc + k], Bs[k][c] = In[kc + k][C0 + c] -- and each of the eight
// waves multiplies 32 rows x 64 columns as 2 x 4 MFMA 16x16x4 tiles (half the
// registers of four 64 x 64 quadrants: four waves per SIMD instead of two,
// 0.94 ms instead of 1.27 at 16384 x 8192).  The next chunk is loaded into
// registers while the current one is multiplied.  Row tiles entirely above
// the chunk's diagonal are skipped; a wave takes the 16-row tiles w and 7 - w
// of the 128 (not 32 contiguous rows), so every wave skips as many.  The LDS row stride (144 doubles, 1152
// bytes) puts the two half-waves of a fragment read on different banks.  The
// launch bounds ask for four waves per SIMD (at most 128 registers), which the
// optional row sums after the product would otherwise exceed.
constexpr int kTT = kTrmmTile;
constexpr int kTK = 32;
constexpr int kTS = kTT + 16;
__global__ __launch_bounds__(512, 4) void k_trmm_lds(const double* In, double* Out, int64_t ldc,
                                                  const int64_t* off, int32_t m, int32_t nrt,
                                                  int32_t nct, const int64_t* goff,
                                                  const double* Linv, float* Out32,
                                                  const double* cx, const double* cy,
                                                  const int64_t* toff, double* tpart) {
  const int total = m * nrt * nct;
  const int q = xcd_contiguous(static_cast<int>(blockIdx.x), total);
  if (q >= total) return;
  const int blk = q / (nrt * nct);
  const int rem = q - blk * nrt * nct;
  const int rt = rem / nct, ct = rem - rt * nct;
  const int64_t r0 = off[blk];
  const int p = static_cast<int>(off[blk + 1] - r0);
  const int R0 = rt * kTT;
  if (R0 >= p) return;  // uniform per workgroup
  const int64_t C0 = static_cast<int64_t>(ct) * kTT;
  const double* Lb = Linv + goff[blk];
  const int kend = min(p, R0 + kTT);
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int li = lane & 15, g = lane >> 4;
  const int wr = wv >> 1, wc = wv & 1;  // eight waves: 4 row pairs x 2 column halves of 64
  // The wave's two 16-row tiles of the 128: wr and 7 - wr, so that the
  // products skipped above the diagonal are spread evenly over the waves.
  const int tr16[2] = {wr, 7 - wr};
  __shared__ __align__(16) double As[kTK][kTS];
  __shared__ __align__(16) double Bs[kTK][kTS];
  // The row sums' weights for the tile's rows (0 past the block), loaded
  // before the product so that the sums after it wait on no global load.
  __shared__ double wts[2][kTT];
  if (tpart && threadIdx.x < 2 * kTT) {
    const int v = threadIdx.x / kTT, row = R0 + threadIdx.x % kTT;
    const double* cv = v == 0 ? cx : cy;
    wts[v][threadIdx.x % kTT] = cv && row < p ? cv[r0 + row] : 0.0;
  }

  // Staging: A -- thread t takes row t / 2 and 16 consecutive k (scalar loads:
  // Linv rows have stride p, which may be odd); B -- thread t takes row t / 8
  // of the chunk and 16 consecutive columns (16-byte loads: ldc is a multiple
  // of 64).  Entries past the block, past kend or past ldc are zero.
  // Loads read clamped in-range addresses unconditionally and the entries
  // outside the block are zeroed when stored to LDS, after the products: a
  // load behind a branch, or one whose value is selected at once, makes the
  // compiler wait for every load in flight there.
  const int ar = threadIdx.x >> 2, ak = (threadIdx.x & 3) * 8;
  const int bk = threadIdx.x >> 4, bc = (threadIdx.x & 15) * 8;
  const bool a_row_ok = R0 + ar < p;
  const bool b_col_ok = C0 + bc < ldc;
  const int64_t a_row = static_cast<int64_t>(a_row_ok ? R0 + ar : p - 1) * p;
  const int64_t b_col = b_col_ok ? C0 + bc : 0;
  double pa[8];
  f64x2 pb[4];
  int kc_loaded = 0;
  auto load_chunk = [&](int kc) {
    kc_loaded = kc;
#pragma unroll
    for (int j = 0; j < 8; ++j) pa[j] = Lb[a_row + min(kc + ak + j, p - 1)];
    const double* src = In + (r0 + min(kc + bk, p - 1)) * ldc + b_col;
#pragma unroll
    for (int j = 0; j < 4; ++j) pb[j] = *reinterpret_cast<const f64x2*>(src + 2 * j);
  };
  auto store_chunk = [&]() {
    const int kc = kc_loaded;
#pragma unroll
    for (int j = 0; j < 8; ++j) As[ak + j][ar] = (a_row_ok && kc + ak + j < kend) ? pa[j] : 0.0;
    const bool brow = kc + bk < kend && b_col_ok;
#pragma unroll
    for (int j = 0; j < 4; ++j)
      *reinterpret_cast<f64x2*>(&Bs[bk][bc + 2 * j]) = brow ? pb[j] : f64x2{0.0, 0.0};
  };

  f64x4 acc[2][4];
#pragma unroll
  for (int t = 0; t < 2; ++t)
#pragma unroll
    for (int u = 0; u < 4; ++u) acc[t][u] = f64x4{};
  load_chunk(0);
  store_chunk();
  __syncthreads();
  for (int kc = 0; kc < kend; kc += kTK) {
    const bool more = kc + kTK < kend;
    load_chunk(more ? kc + kTK : kc);  // the last chunk reloads itself, unused
#pragma unroll
    for (int kk = 0; kk < kTK / 4; ++kk) {
      const int k = 4 * kk + g;
      double b[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) b[u] = Bs[k][wc * 64 + u * 16 + li];
#pragma unroll
      for (int t = 0; t < 2; ++t) {
        // Rows of this 16-row tile all lie above column kc + 4 kk: zero.
        if (kc + 4 * kk > R0 + tr16[t] * 16 + 15) continue;  // uniform per wave
        const double a = As[k][tr16[t] * 16 + li];
#pragma unroll
        for (int u = 0; u < 4; ++u)
          acc[t][u] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b[u], acc[t][u], 0, 0, 0);
      }
    }
    __syncthreads();
    if (more) store_chunk();
    __syncthreads();
  }
  // acc[t][u][q] = D[g + 4 q][li] of the 16 x 16 tile (t, u).
#pragma unroll
  for (int t = 0; t < 2; ++t)
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
      for (int qq = 0; qq < 4; ++qq) {
        const int row = R0 + tr16[t] * 16 + g + 4 * qq;
        const int64_t col = C0 + wc * 64 + u * 16 + li;
        if (row < p && col < ldc) {
          const int64_t o = (r0 + row) * ldc + col;
          Out[o] = acc[t][u][qq];
          if (Out32) Out32[o] = static_cast<float>(acc[t][u][qq]);
        }
      }
  if (!tpart) return;  // uniform per workgroup
  // Row sums of the tile for the vectors given: each lane weights its eight
  // rows (weights from LDS; rows past the block have zero products and
  // weight 0), the four lane groups of a column are added by shuffles, the
  // four row-pair waves of a column half in LDS, in wave order.  As is free:
  // every wave has passed the loop's last barrier.
  double* red = &As[0][0];  // [2 vectors][4 waves][kTT columns]
  const int64_t T = toff[m];
#pragma unroll
  for (int v = 0; v < 2; ++v) {
    const double* cv = v == 0 ? cx : cy;
    if (!cv) continue;  // uniform
    double wgt[2][4];
#pragma unroll
    for (int t = 0; t < 2; ++t)
#pragma unroll
      for (int qq = 0; qq < 4; ++qq) wgt[t][qq] = wts[v][tr16[t] * 16 + g + 4 * qq];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      double sum = 0.0;
#pragma unroll
      for (int t = 0; t < 2; ++t)
#pragma unroll
        for (int qq = 0; qq < 4; ++qq) sum = fma(wgt[t][qq], acc[t][u][qq], sum);
      sum += __shfl_xor(sum, 16);
      sum += __shfl_xor(sum, 32);
      if (g == 0) red[(v * 4 + wr) * kTT + wc * 64 + u * 16 + li] = sum;
    }
  }
  __syncthreads();
  if (threadIdx.x < 2 * kTT) {
    const int v = threadIdx.x / kTT, c = threadIdx.x % kTT;
    if ((v == 0 ? cx : cy) && C0 + c < ldc) {
      const double* rv = red + v * 4 * kTT + c;
      const double sum = (rv[0] + rv[kTT]) + (rv[2 * kTT] + rv[3 * kTT]);
      tpart[(v * T + toff[blk] + rt) * ldc + C0 + c] = sum;
    }
  }
}

// G_i = C_i C_i^T as 64 x 64 tiles (ta >= tb) on the FP64 matrix cores with
// both operands staged in LDS: one workgroup of eight waves per tile, each
// wave a 16 x 32 quadrant (1 x 2 MFMA 16x16x4 tiles), so that four or more
// waves per SIMD hide the latencies.  K (the padded row length, a multiple of
// 32) goes in chunks of 32, K-major in LDS (As[k][r'] = C[row 64 ta + r][kc + k],
// Bs[k][c'] likewise for 64 tb + c); the next chunk is loaded into registers
// while the current one is multiplied.  Rows past the block read its last
// row: they only reach entries of G past the block, which are not stored.
// LDS banks: with the row stride of 80 doubles, rows k and k + 1 of one
// fragment read fall on opposite halves of the banks; the staging stores,
// where a half-wave writes four rows r at eight k four apart, would all land
// on four banks, so the row index is stored swizzled, r' = r ^ 4 ((k >> 2) & 7):
// the stores then cover every bank once and a fragment read's 16 consecutive
// r stay one aligned group of 16 (measured: bank-conflict cycles were about
// half the kernel's time before).
constexpr int kGT = 64;
constexpr int kGK = 32;
constexpr int kGS = kGT + 16;
__device__ __forceinline__ int gram_swz(int k, int r) { return r ^ (4 * ((k >> 2) & 7)); }
__global__ __launch_bounds__(512) void k_gram_lds(const double* C, int64_t ldc,
                                                 const int64_t* off, const int32_t* tiles,
                                                 int32_t ntiles, const int64_t* goff, double* G,
                                                 int32_t nsplit, int64_t klen, double* part,
                                                 int64_t pstride) {
  // Work item u = split * ntiles + tile: consecutive items (one XCD's share)
  // are tiles of the same blocks over the same K range, which share rows.
  const int total = ntiles * nsplit;
  const int item = xcd_contiguous(static_cast<int>(blockIdx.x), total);
  if (item >= total) return;
  const int split = item / ntiles;
  const int q = item - split * ntiles;
  const int blk = tiles[3 * q + 0];
  const int ta = tiles[3 * q + 1];
  const int tb = tiles[3 * q + 2];
  const int64_t r0 = off[blk];
  const int p = static_cast<int>(off[blk + 1] - r0);
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int li = lane & 15, g = lane >> 4;
  const int wr = wv >> 1, wc = wv & 1;
  __shared__ __align__(16) double As[kGK][kGS];
  __shared__ __align__(16) double Bs[kGK][kGS];
  // Staging: thread t takes row t / 8 of each operand tile and the four
  // consecutive k at 4 (t % 8) (two 16-byte loads each).
  const int sr = threadIdx.x >> 3, sk = (threadIdx.x & 7) * 4;
  const double* pa = C + (r0 + min(ta * kGT + sr, p - 1)) * ldc + sk;
  const double* pb = C + (r0 + min(tb * kGT + sr, p - 1)) * ldc + sk;
  f64x2 ra[2], rb[2];
  auto load_chunk = [&](int64_t kc) {
#pragma unroll
    for (int e = 0; e < 2; ++e) {
      ra[e] = *reinterpret_cast<const f64x2*>(pa + kc + 2 * e);
      rb[e] = *reinterpret_cast<const f64x2*>(pb + kc + 2 * e);
    }
  };
  const int ssr = gram_swz(sk, sr);  // the same for sk .. sk + 3
  auto store_chunk = [&]() {
#pragma unroll
    for (int e = 0; e < 2; ++e) {
      As[sk + 2 * e][ssr] = ra[e][0];
      As[sk + 2 * e + 1][ssr] = ra[e][1];
      Bs[sk + 2 * e][ssr] = rb[e][0];
      Bs[sk + 2 * e + 1][ssr] = rb[e][1];
    }
  };
  f64x4 acc[2] = {f64x4{}, f64x4{}};
  const int64_t k0 = static_cast<int64_t>(split) * klen;
  const int64_t kend = min(ldc, k0 + klen);  // > k0: the host sizes the splits
  load_chunk(k0);
  store_chunk();
  __syncthreads();
  for (int64_t kc = k0; kc < kend; kc += kGK) {
    const bool more = kc + kGK < kend;
    load_chunk(more ? kc + kGK : kc);  // the last chunk reloads itself, unused
#pragma unroll
    for (int kk = 0; kk < kGK / 4; ++kk) {
      const int k = 4 * kk + g;
      const double a = As[k][gram_swz(k, wr * 16 + li)];
      const double b0 = Bs[k][gram_swz(k, wc * 32 + li)];
      const double b1 = Bs[k][gram_swz(k, wc * 32 + 16 + li)];
      acc[0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b0, acc[0], 0, 0, 0);
      acc[1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b1, acc[1], 0, 0, 0);
    }
    __syncthreads();
    if (more) store_chunk();
    __syncthreads();
  }
  // acc[u][q] = G[64 ta + 16 wr + g + 4 q][64 tb + 32 wc + 16 u + li] (this
  // split's share; split s > 0 writes the same layout at part + (s - 1) pstride).
  double* Gb = (split == 0 ? G : part + (split - 1) * pstride) + goff[blk];
#pragma unroll
  for (int u = 0; u < 2; ++u)
#pragma unroll
    for (int qq = 0; qq < 4; ++qq) {
      const int ra_ = ta * kGT + wr * 16 + g + 4 * qq;
      const int rb_ = tb * kGT + wc * 32 + u * 16 + li;
      if (ra_ < p && rb_ < p) {
        Gb[static_cast<int64_t>(ra_) * p + rb_] = acc[u][qq];
        if (ta != tb) Gb[static_cast<int64_t>(rb_) * p + ra_] = acc[u][qq];
      }
    }
}

// Per-block sums of the triangular product's row-tile sums, in tile order.
__global__ __launch_bounds__(256) void k_tile_sum(const double* part, const int64_t* toff,
                                                 int32_t m, int64_t ldc, double* out,
                                                 int64_t ldo) {
  const int64_t c = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x;
  if (c >= ldc) return;
  for (int32_t i = blockIdx.y; i < m; i += gridDim.y) {
    double v = 0.0;
    for (int64_t t = toff[i]; t < toff[i + 1]; ++t) v += part[t * ldc + c];
    out[static_cast<int64_t>(i) * ldo + c] = v;
  }
}

// G += part[0] + part[1] + ... (split s > 0 at part + (s - 1) pstride), in
// split order, so the sum does not depend on scheduling.
__global__ __launch_bounds__(256) void k_gram_split_sum(double* G, const double* part,
                                                       int64_t pstride, int32_t nsplit) {
  for (int64_t e = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; e < pstride;
       e += static_cast<int64_t>(gridDim.x) * blockDim.x) {
    double v = G[e];
    for (int sp = 1; sp < nsplit; ++sp) v += part[(sp - 1) * pstride + e];
    G[e] = v;
  }
}

}  // namespace

hipError_t launch_gram_lds(const double* C, int64_t ldc, const int64_t* off,
                           const int32_t* tiles, int32_t ntiles, const int64_t* goff, double* G,
                           int32_t nsplit, double* part, int64_t pstride, hipStream_t s) {
  if (ntiles <= 0) return hipSuccess;
  if (ldc % kGK != 0 || nsplit < 1 || (nsplit > 1 && !part)) return hipErrorInvalidValue;
  // Every split non-empty: klen a whole number of chunks, (nsplit - 1) klen < ldc
  // (fewer splits where the chunks do not divide so).
  int64_t klen = 0;
  for (;; --nsplit) {
    klen = (ldc / kGK + nsplit - 1) / nsplit * kGK;
    if (nsplit == 1 || (nsplit - 1) * klen < ldc) break;
  }
  const int64_t total = static_cast<int64_t>(ntiles) * nsplit;
  if (total > std::numeric_limits<int32_t>::max() / 2) return hipErrorInvalidValue;
  const unsigned grid = static_cast<unsigned>((total + kXcds - 1) / kXcds * kXcds);
  k_gram_lds<<<grid, 512, 0, s>>>(C, ldc, off, tiles, ntiles, goff, G, nsplit, klen, part, pstride);
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess || nsplit == 1) return e;
  k_gram_split_sum<<<grid_stride_blocks(pstride), 256, 0, s>>>(G, part, pstride, nsplit);
  return hipGetLastError();
}

hipError_t launch_trmm_lds(const double* In, double* Out, int64_t ldc, const int64_t* off,
                           int32_t m, int64_t pmax, const int64_t* goff, const double* Linv,
                           float* out32, const double* cx, const double* cy, const int64_t* toff,
                           double* tpart, hipStream_t s) {
  if (m <= 0) return hipSuccess;
  if (ldc % 64 != 0) return hipErrorInvalidValue;
  if (tpart && (!toff || (!cx && !cy))) return hipErrorInvalidValue;
  const int64_t nrt = (pmax + kTT - 1) / kTT, nct = (ldc + kTT - 1) / kTT;
  const int64_t items = static_cast<int64_t>(m) * nrt * nct;
  if (items > std::numeric_limits<int32_t>::max() / 2) return hipErrorInvalidValue;
  const unsigned grid = static_cast<unsigned>((items + kXcds - 1) / kXcds * kXcds);
  k_trmm_lds<<<grid, 512, 0, s>>>(In, Out, ldc, off, m, static_cast<int32_t>(nrt),
                                  static_cast<int32_t>(nct), goff, Linv, out32, cx, cy, toff,
                                  tpart);
  return hipGetLastError();
}

hipError_t launch_tile_sum(const double* part, const int64_t* toff, int32_t m, int64_t ldc,
                           double* out, int64_t ldo, hipStream_t s) {
  if (m <= 0 || ldc <= 0) return hipSuccess;
  const int64_t gx = (ldc + 255) / 256;
  if (gx > std::numeric_limits<int32_t>::max()) return hipErrorInvalidValue;
  const dim3 grid(static_cast<unsigned>(gx), static_cast<unsigned>(std::min<int32_t>(m, 65535)));
  k_tile_sum<<<grid, 256, 0, s>>>(part, toff, m, ldc, out, ldo);
  return hipGetLastError();
}

}  // namespace apc
