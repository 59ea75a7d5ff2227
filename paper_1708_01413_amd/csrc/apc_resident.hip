// T updates of eq. (2a)-(2b) in one launch, for k = 1 in FP64 when every block
// is small enough to live in one workgroup's registers (up to 64 rows of up to
// 1024 columns).
//
// At these sizes an update moves a few MiB at most, and two kernel launches per
// update (the single pass and its combine) cost more than the arithmetic.  Here
// workgroup i owns block i for the whole launch: its rows of C are loaded once
// into registers, x_i and x_bar stay in registers, and per update
//   1. w_r = C[r] . d_i for the block's rows (each wave owns whole rows: a wave
//      sum, no LDS),
//   2. u = sum_r w_r C[r] (per-wave partials, summed across the 8 waves in LDS),
//   3. x_i <- x_i + gamma ((x_bar - x_i) - u), published to an exchange buffer,
//   4. x_bar <- alpha sum_i x_i + beta x_bar from the m published x_i (every
//      workgroup forms the same sum in the same order) and d_i = x_bar - x_i.
//
// The exchange carries its own validity, so no barrier or cache flush is
// needed: every double is published as two 64-bit words, each a 32-bit half of
// the value under a 32-bit epoch, stored and loaded with single-copy-atomic
// agent-scope accesses (coherent across XCDs).  A reader polls a word until it
// shows the current epoch.  Epochs run on across launches: update t of a launch
// carries sync[1] + t + 1, and workgroup 0 stores the next base after reading
// the launch's last update (which every workgroup publishes after reading the
// base); the next launch on the stream starts after this one has ended.  The buffer alternates between two halves by update
// parity: a workgroup publishes update t + 2 only after it has read update
// t + 1 from every block, which each block publishes after reading update t,
// so no word is overwritten before every reader has seen it.
//
// Polls are bounded: after spin_limit of them (the library passes 2^22,
// seconds) a thread records the time-out in sync[2]; its workgroup sets x_bar
// to NaN and leaves, and so, waiting on it, do the others; later launches on
// the same buffers stop at once the same way, so no wait can hang the device.
// The host reads sync[2] with the residual.

#include "apc_internal.h"

namespace apc {
namespace {

typedef double f64x2_t __attribute__((ext_vector_type(2)));

constexpr int kWaves = kResidentThreads / 64;

__device__ inline double tree8(const double (&p)[8]) {
  return ((p[0] + p[1]) + (p[2] + p[3])) + ((p[4] + p[5]) + (p[6] + p[7]));
}

__device__ inline uint64_t word_load(uint64_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ inline void word_store(uint64_t* p, uint64_t v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ inline uint64_t tag(uint32_t epoch, uint32_t half) {
  return (static_cast<uint64_t>(epoch) << 32) | half;
}
__device__ inline bool tagged(uint64_t w, uint32_t epoch) {
  return static_cast<uint32_t>(w >> 32) == epoch;
}
__device__ inline double untag(uint64_t lo, uint64_t hi) {
  return __longlong_as_double(static_cast<long long>((hi << 32) | (lo & 0xffffffffull)));
}

// RPW rows per wave (rows wave + 8k of the block), CPL 16-byte chunks per lane
// and row (chunk lane + 64c, i.e. columns 2(lane + 64c) and the next one).
// The owner layout for x_i, x_bar and the column sums: thread t owns columns
// t, t + 512, ...
template <int RPW, int CPL>
__global__ __launch_bounds__(kResidentThreads, 1) void k_resident(ResidentArgs a) {
  constexpr int NCOL = 128 * CPL;
  constexpr int NOWN = (NCOL + kResidentThreads - 1) / kResidentThreads;
  __shared__ double red[kWaves][NCOL];
  __shared__ double dsh[NCOL];
  __shared__ int flag;
  __shared__ uint32_t base;
  if (blockIdx.x % a.stride != 0) return;
  const int i = static_cast<int>(blockIdx.x / a.stride);
  if (i >= a.m) return;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;

  if (threadIdx.x == 0) {
    flag = __hip_atomic_load(a.sync + 2, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0;
    base = __hip_atomic_load(a.sync + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
  __syncthreads();
  if (flag) {
    if (i == 0)
      for (int j = tid; j < a.n; j += kResidentThreads) a.xbar[j] = __builtin_nan("");
    return;
  }
  const uint32_t epoch0 = base;

  const int64_t r0 = a.off[i];
  const int64_t p = a.off[i + 1] - r0;
  double cr[RPW][CPL][2];
#pragma unroll
  for (int k = 0; k < RPW; ++k) {
    const int64_t row = wv + kWaves * k;
#pragma unroll
    for (int c = 0; c < CPL; ++c) {
      const int64_t col = 2 * (lane + 64 * c);
      if (row < p && col < a.ldc) {
        const f64x2_t v = __builtin_nontemporal_load(
            reinterpret_cast<const f64x2_t*>(a.C + (r0 + row) * a.ldc + col));
        cr[k][c][0] = v[0];
        cr[k][c][1] = v[1];
      } else {
        cr[k][c][0] = 0.0;
        cr[k][c][1] = 0.0;
      }
    }
  }

  // Owned columns: j = tid + 512 q.  Columns at or past n hold d = 0, so the
  // zero padding of C meets zeros.
  double xi[NOWN], xb[NOWN];
#pragma unroll
  for (int q = 0; q < NOWN; ++q) {
    const int j = tid + kResidentThreads * q;
    xi[q] = 0.0;
    xb[q] = 0.0;
    if (j < a.n) {
      xi[q] = a.x[static_cast<int64_t>(i) * a.ldx + j];
      xb[q] = a.xbar[j];
      dsh[j] = a.d[static_cast<int64_t>(i) * a.ldd + j];
    } else if (j < NCOL) {
      dsh[j] = 0.0;
    }
  }
  __syncthreads();

  bool ok = true;
  for (int t = 0; t < a.T; ++t) {
    double dl[CPL][2];
#pragma unroll
    for (int c = 0; c < CPL; ++c) {
      const f64x2_t v = *reinterpret_cast<const f64x2_t*>(&dsh[2 * (lane + 64 * c)]);
      dl[c][0] = v[0];
      dl[c][1] = v[1];
    }
    double s[RPW], w[RPW];
#pragma unroll
    for (int k = 0; k < RPW; ++k) {
      s[k] = 0.0;
#pragma unroll
      for (int c = 0; c < CPL; ++c) {
        s[k] = fma(cr[k][c][0], dl[c][0], s[k]);
        s[k] = fma(cr[k][c][1], dl[c][1], s[k]);
      }
    }
    row_sums<RPW>(s, w, lane);
#pragma unroll
    for (int c = 0; c < CPL; ++c) {
      double u0 = 0.0, u1 = 0.0;
#pragma unroll
      for (int k = 0; k < RPW; ++k) {
        u0 = fma(w[k], cr[k][c][0], u0);
        u1 = fma(w[k], cr[k][c][1], u1);
      }
      *reinterpret_cast<f64x2_t*>(&red[wv][2 * (lane + 64 * c)]) = f64x2_t{u0, u1};
    }
    __syncthreads();

    // Publish x_i: column j as two tagged words at xo + 2 (i ldc + j).
    const uint32_t ep = epoch0 + static_cast<uint32_t>(t) + 1u;
    uint64_t* xo = a.xch + 2 * static_cast<int64_t>(t & 1) * a.m * a.ldc;
#pragma unroll
    for (int q = 0; q < NOWN; ++q) {
      const int j = tid + kResidentThreads * q;
      if (j < a.n) {
        double r[8];
#pragma unroll
        for (int v = 0; v < 8; ++v) r[v] = red[v][j];
        const double u = tree8(r);
        xi[q] = xi[q] + a.gamma * ((xb[q] - xi[q]) - u);
        const uint64_t bits = static_cast<uint64_t>(__double_as_longlong(xi[q]));
        uint64_t* w = xo + 2 * (static_cast<int64_t>(i) * a.ldc + j);
        word_store(w, tag(ep, static_cast<uint32_t>(bits)));
        word_store(w + 1, tag(ep, static_cast<uint32_t>(bits >> 32)));
      }
    }

    // Every workgroup sums the m published x_i in the same order: block i
    // into running sum i mod 8 (ascending i), then a fixed tree of the eight.
    bool late = false;
#pragma unroll
    for (int q = 0; q < NOWN; ++q) {
      const int j = tid + kResidentThreads * q;
      if (j < a.n && !late) {
        double ps[8];
#pragma unroll
        for (int v = 0; v < 8; ++v) ps[v] = 0.0;
        for (int i0 = 0; i0 < a.m && !late; i0 += 8) {
          uint64_t lo[8], hi[8];
#pragma unroll
          for (int v = 0; v < 8; ++v) {
            uint64_t* w = xo + 2 * (static_cast<int64_t>(i0 + v) * a.ldc + j);
            lo[v] = i0 + v < a.m ? word_load(w) : tag(ep, 0);
            hi[v] = i0 + v < a.m ? word_load(w + 1) : tag(ep, 0);
          }
          // Poll until all eight blocks show this update's epoch; a retry
          // reloads every word still missing at once, so a poll costs one
          // round trip however many are missing.
          uint32_t polls = 0;
          for (;;) {
            bool all = true;
#pragma unroll
            for (int v = 0; v < 8; ++v) all = all && tagged(lo[v], ep) && tagged(hi[v], ep);
            if (all) break;
            if (++polls > a.spin_limit) {
              late = true;
              break;
            }
            __builtin_amdgcn_s_sleep(1);
#pragma unroll
            for (int v = 0; v < 8; ++v) {
              uint64_t* w = xo + 2 * (static_cast<int64_t>(i0 + v) * a.ldc + j);
              if (!tagged(lo[v], ep)) lo[v] = word_load(w);
              if (!tagged(hi[v], ep)) hi[v] = word_load(w + 1);
            }
          }
#pragma unroll
          for (int v = 0; v < 8; ++v)
            if (i0 + v < a.m) ps[v] += untag(lo[v], hi[v]);
        }
        const double tot = tree8(ps);
        xb[q] = a.beta == 0.0 ? a.alpha * tot : a.alpha * tot + a.beta * xb[q];
        dsh[j] = xb[q] - xi[q];
      }
    }
    if (late) {
      __hip_atomic_store(a.sync + 2, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      flag = 1;
    }
    __syncthreads();
    if (flag) {
      ok = false;
      break;
    }
  }

  if (!ok) {
    for (int j = tid; j < a.n; j += kResidentThreads) a.xbar[j] = __builtin_nan("");
    return;
  }
#pragma unroll
  for (int q = 0; q < NOWN; ++q) {
    const int j = tid + kResidentThreads * q;
    if (j < a.n) {
      a.x[static_cast<int64_t>(i) * a.ldx + j] = xi[q];
      a.d[static_cast<int64_t>(i) * a.ldd + j] = dsh[j];
      if (i == 0) a.xbar[j] = xb[q];
    }
  }
  if (i == 0 && tid == 0)
    __hip_atomic_store(a.sync + 1, epoch0 + static_cast<uint32_t>(a.T), __ATOMIC_RELAXED,
                       __HIP_MEMORY_SCOPE_AGENT);
}

template <int RPW, int CPL>
hipError_t launch_shape(const ResidentArgs& a, hipStream_t s) {
  const unsigned grid = static_cast<unsigned>(a.m) * static_cast<unsigned>(a.stride);
  APC_LAUNCH((k_resident<RPW, CPL>), dim3(grid), dim3(kResidentThreads), 0, s, a);
  return hipGetLastError();
}

template <int RPW>
hipError_t launch_rpw(const ResidentArgs& a, int cpl, hipStream_t s) {
  switch (cpl) {
    case 1: return launch_shape<RPW, 1>(a, s);
    case 2: return launch_shape<RPW, 2>(a, s);
    case 4: return launch_shape<RPW, 4>(a, s);
    case 8:
      if constexpr (RPW * 8 <= 32) return launch_shape<RPW, 8>(a, s);
      break;
    default: break;
  }
  return hipErrorInvalidValue;
}

}  // namespace

bool resident_shape(int64_t max_rows, int64_t ldc, int* rpw, int* cpl) {
  if (max_rows < 1 || ldc < 2) return false;
  int r = 1, c = 1;
  while (kWaves * r < max_rows) r *= 2;
  while (128 * c < ldc) c *= 2;
  if (r > 8 || c > 8 || r * c > 32) return false;
  *rpw = r;
  *cpl = c;
  return true;
}

hipError_t launch_resident_f64(const ResidentArgs& a, int rpw, int cpl, hipStream_t s) {
  if (a.m <= 0 || a.T <= 0) return hipSuccess;
  if (a.stride < 1 || a.n < 1 || a.ldc < a.n || a.ldc % 2 != 0 || 128 * cpl < a.ldc)
    return hipErrorInvalidValue;
  switch (rpw) {
    case 1: return launch_rpw<1>(a, cpl, s);
    case 2: return launch_rpw<2>(a, cpl, s);
    case 4: return launch_rpw<4>(a, cpl, s);
    case 8: return launch_rpw<8>(a, cpl, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace apc
