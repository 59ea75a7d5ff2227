// Device building blocks of the matrix-core contraction (see apc_gemm.hip for
// the layout of its operands) and of its elementwise epilogues.  Shared by the
// single-plan kernels (apc_gemm.hip) and the persistent batch kernel that mixes
// k-RHS contractions with k = 1 systems (apc_batch.hip).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "apc_internal.h"

namespace apc {

namespace {

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef double f64x4 __attribute__((ext_vector_type(4)));
typedef double f64x2 __attribute__((ext_vector_type(2)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef unsigned u32x4 __attribute__((ext_vector_type(4)));

template <typename T>
struct TnTraits;
template <>
struct TnTraits<__bf16> {
  using Acc = f32x4;
  using Part = float;
};
template <>
struct TnTraits<float> {
  using Acc = f32x4;
  using Part = float;
};
template <>
struct TnTraits<double> {
  using Acc = f64x4;
  using Part = double;
};

// MFMA over one 16-byte piece of A (lane's row) and B (lane's right-hand side).
__device__ inline void mma_piece(const u32x4& a, const u32x4& b, f32x4& c, __bf16*) {
  c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, a),
                                              __builtin_bit_cast(bf16x8, b), c, 0, 0, 0);
}
__device__ inline void mma_piece(const u32x4& a, const u32x4& b, f32x4& c, float*) {
  const f32x4 av = __builtin_bit_cast(f32x4, a);
  const f32x4 bv = __builtin_bit_cast(f32x4, b);
#pragma unroll
  for (int e = 0; e < 4; ++e) c = __builtin_amdgcn_mfma_f32_16x16x4f32(av[e], bv[e], c, 0, 0, 0);
}
__device__ inline void mma_piece(const u32x4& a, const u32x4& b, f64x4& c, double*) {
  const f64x2 av = __builtin_bit_cast(f64x2, a);
  const f64x2 bv = __builtin_bit_cast(f64x2, b);
#pragma unroll
  for (int e = 0; e < 2; ++e) c = __builtin_amdgcn_mfma_f64_16x16x4f64(av[e], bv[e], c, 0, 0, 0);
}

// V staging of one workgroup: two 256-byte-per-row steps of 16 NCT rows, 16
// pieces per row + 1 pad (conflict-free fragment reads).
template <int NCT>
struct TnStage {
  u32x4 v[2][NCT * 16][17];
  __device__ u32x4 (&operator[](int b))[NCT * 16][17] { return v[b]; }
};

// Element offset of (row r, column c) in the fragment-packed layout of a
// rows x K operand (rows % 16 == 0, K a multiple of the step).
template <typename T>
__host__ __device__ inline int64_t frag_index(int64_t r, int64_t c, int64_t rows) {
  constexpr int kE = 16 / sizeof(T);
  constexpr int kStep = 16 * kE;
  const int64_t ks = c / kStep;
  const int kc = static_cast<int>((c % kStep) / kE);   // 16-byte chunk in the step
  const int lane = static_cast<int>(r % 16) + 16 * (kc % 4);
  return (ks * (rows / 16) + r / 16) * (16 * kStep) + (64 * (kc / 4) + lane) * kE + c % kE;
}

// Workgroup: W waves (4 or 8), wave w owns RT consecutive 16-row tiles, all
// 16*NCT right-hand sides of its column group.  Grid: (rows / (16 W RT)) x ncg x nsplit,
// with the split index fastest so that, dealt round-robin over the 8 XCDs, one
// XCD works on one split (nsplit | 8) and keeps that split's V in its L2.
template <typename T, int RT, int NCT, int PF, int NT, int W = 4>
__device__ inline void tn_block(const TnArgs& a, int bid, TnStage<NCT>& vs) {
  static_assert((W == 4 || W == 8) && (4 * NCT) % W == 0, "waves per workgroup");
  constexpr int VU = 4 * NCT / W;     // V rows each thread stages per step: 4 W rows at a time
  using Acc = typename TnTraits<T>::Acc;
  using Part = typename TnTraits<T>::Part;
  constexpr int kE = 16 / sizeof(T);  // elements per 16-byte piece
  constexpr int kStep = 16 * kE;      // elements per row per step (256 bytes)
  const int ncg = a.kp / (16 * NCT);
  int q = bid;
  const int split = q % a.nsplit;
  q /= a.nsplit;
  const int cg = q % ncg;
  const int64_t rtile = q / ncg;
  const int lane = threadIdx.x & 63;
  const int wv = threadIdx.x >> 6;
  const int li = lane & 15, g = lane >> 4;
  const int64_t kb0 = static_cast<int64_t>(split) * a.klen;
  const int64_t kend = min(a.K, kb0 + a.klen);
  const int nsteps = kend > kb0 ? static_cast<int>((kend - kb0) / kStep) : 0;
  const T* M = static_cast<const T*>(a.M);
  const T* V = static_cast<const T*>(a.V) + static_cast<int64_t>(cg) * NCT * 16 * a.ldv + kb0;
  const int64_t rb = rtile * 16 * W * RT + static_cast<int64_t>(wv) * 16 * RT;

  // Fragment-packed M: this wave's tile t of step s starts at
  // ((kb0 / kStep + s) * rows / 16 + rb / 16 + t) * 16 * kStep, and lane L's
  // piece p sits (64 p + L) * kE further on.
  const int64_t sstride = a.rows * kStep;
  const T* mrow[RT];
#pragma unroll
  for (int t = 0; t < RT; ++t)
    mrow[t] = M + (kb0 / kStep) * sstride + (rb + 16 * t) * kStep + lane * kE;
  const int vr = threadIdx.x >> 4, vp = threadIdx.x & 15;
  const T* vsrc = V + static_cast<int64_t>(vr) * a.ldv + vp * kE;

  Acc acc[RT][NCT];
#pragma unroll
  for (int t = 0; t < RT; ++t)
#pragma unroll
    for (int ct = 0; ct < NCT; ++ct) acc[t][ct] = Acc{};
  // Ring of PF + 1 register sets for M: the loads for step s + PF are issued
  // while step s computes.  The step loop is unrolled by the ring size so that
  // every slot index is a compile-time constant.
  constexpr int D = PF + 1;
  u32x4 mr[D][RT][4], vst[VU];
  auto load_m = [&](u32x4 (&dst)[RT][4], int step) {
    const int64_t o = static_cast<int64_t>(step) * sstride;
#pragma unroll
    for (int t = 0; t < RT; ++t)
#pragma unroll
      for (int p = 0; p < 4; ++p) {
        const u32x4* src = reinterpret_cast<const u32x4*>(mrow[t] + o + p * 64 * kE);
        dst[t][p] = NT ? __builtin_nontemporal_load(src) : *src;
      }
  };
  auto load_v = [&](int step) {
    const int64_t o = static_cast<int64_t>(step) * kStep;
#pragma unroll
    for (int u = 0; u < VU; ++u)
      vst[u] = *reinterpret_cast<const u32x4*>(vsrc + static_cast<int64_t>(4 * W * u) * a.ldv + o);
  };
  // A split past the end of K (from rounding its length up to whole steps)
  // writes zero partials.  Otherwise every load below is issued without a
  // branch, so that the compiler can count the loads in flight (see the main
  // part); a step past the split's end is replaced by its last step.
  if (nsteps > 0) {
#pragma unroll
  for (int s0 = 0; s0 < PF; ++s0) load_m(mr[s0], min(s0, nsteps - 1));
  load_v(0);
#pragma unroll
  for (int u = 0; u < VU; ++u) vs[0][vr + 4 * W * u][vp] = vst[u];
  __syncthreads();
  // One step: V's next step and M's step + PF are loaded, step `step` is
  // multiplied from ring slot i, V's next step goes to the other LDS buffer.
  // V is loaded before M: loads complete in order, so the wait for V at the
  // end of the step does not also wait for the newest M loads, which keep PF
  // steps in flight.
  auto body = [&](int step, int i, bool more, bool load_ahead) {
    const int buf = step & 1;
    if (more) load_v(step + 1);
    if (load_ahead) load_m(mr[(i + PF) % D], step + PF);
    // Keep the loads at the top of the step: moved down among the products
    // they would be waited for as soon as they are issued.
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int p = 0; p < 4; ++p) {
      u32x4 bf[NCT];
#pragma unroll
      for (int ct = 0; ct < NCT; ++ct) bf[ct] = vs[buf][ct * 16 + li][4 * p + g];
#pragma unroll
      for (int t = 0; t < RT; ++t)
#pragma unroll
        for (int ct = 0; ct < NCT; ++ct)
          mma_piece(mr[i][t][p], bf[ct], acc[t][ct], static_cast<T*>(nullptr));
    }
    if (more) {
#pragma unroll
      for (int u = 0; u < VU; ++u) vs[buf ^ 1][vr + 4 * W * u][vp] = vst[u];
    }
    __syncthreads();
  };
  // Main part: every step of the chunk has step + PF < nsteps, so both loads
  // are issued without a branch.  A load behind a branch makes the compiler
  // wait for every load in flight where the paths join (it cannot count the
  // loads issued after V's), which would drain the prefetch each step.
  int step0 = 0;
  // (Both loops are unrolled by the ring size, so every slot index is a
  // compile-time constant.)
  for (; step0 + D - 1 + PF < nsteps; step0 += D) {
#pragma unroll
    for (int i = 0; i < D; ++i) body(step0 + i, i, true, true);
  }
  // Tail: the last steps, loads only where they exist (uniform branches).
  for (; step0 < nsteps; step0 += D) {
#pragma unroll
    for (int i = 0; i < D; ++i)
      if (step0 + i < nsteps) body(step0 + i, i, step0 + i + 1 < nsteps, step0 + i + PF < nsteps);
  }
  }  // nsteps > 0

  // Result layout: f32 accumulators hold D[4 g + q][li]; f64 ones D[g + 4 q][li].
  Part* part = static_cast<Part*>(a.part);
#pragma unroll
  for (int t = 0; t < RT; ++t)
#pragma unroll
    for (int ct = 0; ct < NCT; ++ct) {
      const int c = cg * NCT * 16 + ct * 16 + li;
      Part* dst = part + (static_cast<int64_t>(split) * a.kp + c) * a.ldp + rb + 16 * t;
      if constexpr (sizeof(Part) == 8) {
#pragma unroll
        for (int qq = 0; qq < 4; ++qq) dst[g + 4 * qq] = acc[t][ct][qq];
      } else {
        *reinterpret_cast<f32x4*>(dst + 4 * g) = acc[t][ct];
      }
    }
}


template <typename T>
__device__ inline T cvt(double v);
template <>
__device__ inline double cvt<double>(double v) { return v; }
template <>
__device__ inline float cvt<float>(double v) { return static_cast<float>(v); }
template <>
__device__ inline __bf16 cvt<__bf16>(double v) { return static_cast<__bf16>(static_cast<float>(v)); }

template <typename P>
__device__ inline double split_sum(const P* part, int32_t nsplit, int64_t split_stride, int64_t idx) {
  P s = part[idx];
  for (int sp = 1; sp < nsplit; ++sp) s += part[sp * split_stride + idx];
  return static_cast<double>(s);
}

// out[c*ldo + r] = TQ(sum of the split partials) for element e = c * rows + r.
template <typename P, typename TQ>
__device__ inline void sum_cast_elem(const P* part, int32_t nsplit, int64_t ldp, int64_t rows,
                                     int64_t stride, TQ* out, int64_t ldo, int64_t e) {
  const int64_t c = e / rows, r = e - c * rows;
  P s = part[c * ldp + r];
  for (int sp = 1; sp < nsplit; ++sp) s += part[sp * stride + c * ldp + r];
  out[c * ldo + r] = static_cast<TQ>(s);
}

// Four consecutive entries as one or two 16-byte accesses (8 bytes for bf16);
// the address is a multiple of four entries, 16-byte aligned.
template <typename T>
__device__ inline void load4(const T* p, T (&v)[4]) {
  if constexpr (sizeof(T) == 4) {
    const f32x4 w = *reinterpret_cast<const f32x4*>(p);
    __builtin_memcpy(v, &w, 16);
  } else {
    const f64x2 w0 = reinterpret_cast<const f64x2*>(p)[0];
    const f64x2 w1 = reinterpret_cast<const f64x2*>(p)[1];
    v[0] = w0[0];
    v[1] = w0[1];
    v[2] = w1[0];
    v[3] = w1[1];
  }
}
template <typename T>
__device__ inline void store4(T* p, const T (&v)[4]) {
  if constexpr (sizeof(T) == 2) {
    uint2 w;
    __builtin_memcpy(&w, v, 8);
    *reinterpret_cast<uint2*>(p) = w;
  } else if constexpr (sizeof(T) == 4) {
    f32x4 w;
    __builtin_memcpy(&w, v, 16);
    *reinterpret_cast<f32x4*>(p) = w;
  } else {
    reinterpret_cast<f64x2*>(p)[0] = f64x2{v[0], v[1]};
    reinterpret_cast<f64x2*>(p)[1] = f64x2{v[2], v[3]};
  }
}

// sum_cast_elem for the four entries e .. e + 3 (e, rows, ldp and ldo
// multiples of 4: the four share one right-hand side).
template <typename P, typename TQ>
__device__ inline void sum_cast4(const P* part, int32_t nsplit, int64_t ldp, int64_t rows,
                                 int64_t stride, TQ* out, int64_t ldo, int64_t e) {
  const int64_t c = e / rows, r = e - c * rows;
  P s[4];
  load4(part + c * ldp + r, s);
  for (int sp = 1; sp < nsplit; ++sp) {
    P t[4];
    load4(part + sp * stride + c * ldp + r, t);
#pragma unroll
    for (int q = 0; q < 4; ++q) s[q] += t[q];
  }
  TQ o[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) o[q] = static_cast<TQ>(s[q]);
  store4(out + c * ldo + r, o);
}

// The (y, x_bar) update, its start, or an anchor update (see TnUpdateArgs)
// for element e = c * n + j.
template <typename P, typename TQ>
__device__ inline void update_elem(const TnUpdateArgs& a, int64_t e) {
  const int64_t stride = static_cast<int64_t>(a.kp) * a.ldp;
  const P* part = static_cast<const P*>(a.part);
  TQ* yq = static_cast<TQ*>(a.yq);
  const double g = a.gamma, omg = 1.0 - a.gamma, eta = a.eta, ome = 1.0 - a.eta;
  const int64_t c = e / a.n, j = e - c * a.n;
  const double z = split_sum(part, a.nsplit, stride, c * a.ldp + j);
  const int64_t i = c * a.ldx + j;
  if (a.mode == 1) {
    const double x0 = z * a.inv_m;
    a.x0[i] = x0;
    a.xb[i] = x0;
    a.y[i] = 0.0;
    if (a.yref) {
      a.yref[i] = 0.0;
      a.uref[i] = 0.0;
    }
    yq[c * a.ldq + j] = cvt<TQ>(g * x0);
    return;
  }
  const double xb = a.xb[i];
  // y1 = (1 - gamma) y + gamma x_bar; an anchor update reads the copy its
  // FP64 product was formed from.
  const double y1 = a.mode == 2 ? a.yref[i] : omg * a.y[i] + g * xb;
  double u = z * a.inv_m;
  double ref = 0.0;
  if (a.mode == 2) {  // z = m X y1 in FP64: new anchor
    a.uref[i] = u;
    ref = y1;
  } else if (a.yref) {  // z = m X~ (y1 - y_ref)
    u += a.uref[i];
    ref = a.yref[i];
  }
  const double xn = eta * (a.x0[i] + y1 - u) + ome * xb;
  a.y[i] = y1;
  a.xb[i] = xn;
  yq[c * a.ldq + j] = cvt<TQ>(omg * y1 + g * xn - ref);
}

// update_elem for the four entries e .. e + 3 (e, n, ldp, ldx and ldq
// multiples of 4), the same arithmetic per entry.
template <typename P, typename TQ>
__device__ inline void update4(const TnUpdateArgs& a, int64_t e) {
  const int64_t stride = static_cast<int64_t>(a.kp) * a.ldp;
  const P* part = static_cast<const P*>(a.part);
  TQ* yq = static_cast<TQ*>(a.yq);
  const double g = a.gamma, omg = 1.0 - a.gamma, eta = a.eta, ome = 1.0 - a.eta;
  const int64_t c = e / a.n, j = e - c * a.n;
  P zs[4];
  load4(part + c * a.ldp + j, zs);
  for (int sp = 1; sp < a.nsplit; ++sp) {
    P t[4];
    load4(part + sp * stride + c * a.ldp + j, t);
#pragma unroll
    for (int q = 0; q < 4; ++q) zs[q] += t[q];
  }
  const int64_t i = c * a.ldx + j;
  TQ qv[4];
  if (a.mode == 1) {
    double x0[4], zero[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      x0[q] = static_cast<double>(zs[q]) * a.inv_m;
      qv[q] = cvt<TQ>(g * x0[q]);
    }
    store4(a.x0 + i, x0);
    store4(a.xb + i, x0);
    store4(a.y + i, zero);
    if (a.yref) {
      store4(a.yref + i, zero);
      store4(a.uref + i, zero);
    }
    store4(yq + c * a.ldq + j, qv);
    return;
  }
  double xb[4], x0[4], y[4] = {0.0, 0.0, 0.0, 0.0}, yr[4] = {0.0, 0.0, 0.0, 0.0},
         ur[4] = {0.0, 0.0, 0.0, 0.0};
  load4(a.xb + i, xb);
  load4(a.x0 + i, x0);
  if (a.mode == 2) {
    load4(a.yref + i, yr);
  } else {
    load4(a.y + i, y);
    if (a.yref) {
      load4(a.yref + i, yr);
      load4(a.uref + i, ur);
    }
  }
  double yo[4], xo[4], uo[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const double y1 = a.mode == 2 ? yr[q] : omg * y[q] + g * xb[q];
    double u = static_cast<double>(zs[q]) * a.inv_m;
    double ref = 0.0;
    if (a.mode == 2) {
      uo[q] = u;
      ref = y1;
    } else if (a.yref) {
      u += ur[q];
      ref = yr[q];
    }
    const double xn = eta * (x0[q] + y1 - u) + ome * xb[q];
    yo[q] = y1;
    xo[q] = xn;
    qv[q] = cvt<TQ>(omg * y1 + g * xn - ref);
  }
  if (a.mode == 2) store4(a.uref + i, uo);
  store4(a.y + i, yo);
  store4(a.xb + i, xo);
  store4(yq + c * a.ldq + j, qv);
}

}  // namespace

}  // namespace apc
