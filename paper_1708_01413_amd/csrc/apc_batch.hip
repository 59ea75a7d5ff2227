// Many independent systems (k = 1 each), one persistent launch per pass.
//
// Every system keeps its own factor, local solutions and average in its own
// plan's workspace; a descriptor array points at them.  A pass is one launch
// over a work list that covers all systems: the grid is a fixed number of
// workgroups (chosen by timing), each looping over items i = blockIdx.x,
// blockIdx.x + gridDim.x, ...  Items of a system whose `active` flag is 0 are
// skipped, so converged systems stop costing bandwidth.
//
// Per update (eq. (2a)-(2b) for every system):
//   pass A   items (system, 16-row tile of one block): w_r = C_r . d_i
//   pass B   items (system, block, 256-column slab):   x_i += gamma (x_bar - x_i - Q_i w_i)
//   average  items (system, 256-column chunk):          x_bar <- (eta/m) sum_i x_i + (1-eta) x_bar,
//                                                       d_i = x_bar - x_i
// The arithmetic per system is the single-system k = 1 path's.

#include <hip/hip_runtime.h>

#include "apc_internal.h"

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
// relres <= rtol (or is not finite) is deactivated.  One thread per system.
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
  if (!(rr > rtol)) active[s] = 0;
}

}  // namespace

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
