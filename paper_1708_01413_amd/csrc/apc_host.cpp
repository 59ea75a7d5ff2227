// Host side of libapc: argument validation, workspace layout, setup and
// iteration orchestration, the Lanczos eigenvalue estimate and the C ABI.
//
// The library never allocates device memory: every device buffer is a slice
// of the caller's workspace.  The plan itself is a small host object.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <limits>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "apc.h"
#include "apc_internal.h"

using namespace apc;

namespace {

thread_local std::string g_last_error;

apc_status fail(apc_status st, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_last_error = buf;
  return st;
}

#define HIP_TRY(expr)                                                                     \
  do {                                                                                    \
    hipError_t e_ = (expr);                                                               \
    if (e_ != hipSuccess)                                                                 \
      return fail(APC_EHIP, "%s failed: %s (%s:%d)", #expr, hipGetErrorString(e_), __FILE__, \
                  __LINE__);                                                              \
  } while (0)

#define ST_TRY(expr)              \
  do {                            \
    apc_status s_ = (expr);       \
    if (s_ != APC_OK) return s_;  \
  } while (0)

constexpr int64_t kAlign = 256;
constexpr int kLanczosMax = 1024;   // Lanczos steps cap (full reorthogonalisation)
static_assert(kLanczosMax <= kLzMaxRows, "a Lanczos step reorthogonalises against at most kLzMaxRows rows");
constexpr int kLanczosWindow = 4;   // steps over which a Ritz value's change is measured
constexpr int kAnchorEvery = 16;    // default anchor spacing of the FP32 k-RHS iteration

int64_t round_up(int64_t v, int64_t a) { return (v + a - 1) / a * a; }

// ------------------------------------------------------------------ layout

struct Layout {
  int64_t ldc = 0, kmax = 0, S = 0;
  int32_t ntiles_a = 0, ntiles_g = 0, ntiles_t = 0, nparts = 0;
  int32_t ntiles_fmax = 0;  // single-pass row tiles the workspace holds
  size_t tiles_f = 0, fpart = 0, v32 = 0;
  // k-RHS path: rows/K padding of its operands (N and n rounded up to kTnPad)
  int64_t Np = 0, np = 0;
  size_t Cq, CqT, C64T, C32T, Apad, yq, Wq, tnpart, x0, ys, c64p, Xs, Rb, cw, Linv2, ssq;
  size_t C64p, yref, uref, W64;  // FP64 anchor of the FP32 / bf16 k-RHS iteration
  size_t C64a, C64b, C32, x, xbar, dv, w, ca, cb, Y, vtmp, V, h, alpha, beta, G, Linv, flags, scal, partial, tiles_a, tiles_g, tiles_t, doff, goff, total;
  size_t toff, tpart;  // triangular product's row-tile sums (setup)
  size_t xch, rsync;  // single-launch k = 1 path: exchange buffer, epoch and time-out words
};

struct Tiles {
  std::vector<int32_t> a_row0, a_nrows, a_blk;  // pass-A row tiles, aligned to block starts
  std::vector<int32_t> g;                        // Gram tiles (blk, ta, tb), ta >= tb
  std::vector<int32_t> t;                        // TRMM tiles (blk, ta, tc)
  std::vector<int64_t> goff;                     // offset of G_i in the packed Gram storage
  std::vector<int64_t> toff;                     // triangular-product row tiles before block i (m+1)
  std::vector<int32_t> f_row0, f_nrows, f_blk;  // single-pass row tiles (k = 1)
  std::vector<int32_t> f_first;                 // first single-pass tile of every block (m+1)
};

constexpr int kFusedMinRows = 16;  // the workspace holds single-pass tiles of this height or more

void build_fused_tiles(const int64_t* off, int32_t m, int rows_per_tile, Tiles* T) {
  T->f_first.assign(1, 0);
  for (int i = 0; i < m; ++i) {
    const int64_t p = off[i + 1] - off[i];
    for (int64_t r = 0; r < p; r += rows_per_tile) {
      T->f_row0.push_back(static_cast<int32_t>(off[i] + r));
      T->f_nrows.push_back(static_cast<int32_t>(std::min<int64_t>(rows_per_tile, p - r)));
      T->f_blk.push_back(i);
    }
    T->f_first.push_back(static_cast<int32_t>(T->f_row0.size()));
  }
}

// Default single-pass shape: two rows per register group (one at the widest
// rows, where two spill), and tiles of 64 rows, fewer when that leaves under
// about one workgroup per CU.  At 16384 x 8192 in FP32, 64 rows and groups of
// two measured best (85.5 us per launch against 88-145 us for 16-128 rows and
// groups of one to four).
void fused_shape(int64_t N, int elem, int cpt, int32_t* rows, int32_t* g) {
  *g = fused_shape_ok(elem, elem, cpt, 2) ? 2 : 1;
  int32_t r = 64;
  while (r > kFusedMinRows && N / r < 256) r /= 2;
  *rows = r;
}

constexpr int kMinRowTile = 8;  // the workspace holds pass-A tile lists of this height or more
constexpr int kPassARows = 8;   // default rows per pass-A workgroup
constexpr int kMaxSplit = 8;    // pass-A column splits the workspace holds partials for

void build_tiles(const int64_t* off, int32_t m, int64_t ldc, int rows_per_tile, Tiles* T) {
  int64_t g = 0;
  const int64_t ctiles = (ldc + kGramTile - 1) / kGramTile;
  for (int i = 0; i < m; ++i) {
    const int64_t p = off[i + 1] - off[i];
    for (int64_t r = 0; r < p; r += rows_per_tile) {
      T->a_row0.push_back(static_cast<int32_t>(off[i] + r));
      T->a_nrows.push_back(static_cast<int32_t>(std::min<int64_t>(rows_per_tile, p - r)));
      T->a_blk.push_back(i);
    }
    const int64_t pt = (p + kGramTile - 1) / kGramTile;
    for (int64_t a = 0; a < pt; ++a) {
      for (int64_t b = 0; b <= a; ++b) {
        T->g.push_back(i);
        T->g.push_back(static_cast<int32_t>(a));
        T->g.push_back(static_cast<int32_t>(b));
      }
      for (int64_t c = 0; c < ctiles; ++c) {
        T->t.push_back(i);
        T->t.push_back(static_cast<int32_t>(a));
        T->t.push_back(static_cast<int32_t>(c));
      }
    }
    T->goff.push_back(g);
    g += p * p;
  }
  T->toff.assign(1, 0);
  for (int i = 0; i < m; ++i)
    T->toff.push_back(T->toff.back() + (off[i + 1] - off[i] + kTrmmTile - 1) / kTrmmTile);
}

// k > 1 (and the mixed-precision mode) run the (y, x_bar) form on the matrix
// cores; k = 1 in FP64/FP32 keeps every block's x_i.
int32_t base_precision(int32_t prec) { return prec & ~static_cast<int32_t>(APC_REDUCED_FORM); }
bool uses_gemm(int32_t k, int32_t prec) {
  return k > 1 || base_precision(prec) == APC_BF16_IR || (prec & APC_REDUCED_FORM) != 0;
}

// Right-hand sides the k-RHS state holds: 16, 32, 64, then multiples of 128
// (one matrix-core column group); the extra columns stay zero.
int32_t padded_rhs(int32_t k, int32_t prec) {
  if (!uses_gemm(k, prec)) return 1;
  if (k <= 16) return 16;
  if (k <= 32) return 32;
  if (k <= 64) return 64;
  return static_cast<int32_t>(round_up(k, 128));
}

// k = 1 FP64 plans whose blocks fit one workgroup's registers can run T
// updates in one launch (k_resident); the workspace then holds its exchange
// buffer.  Whether a plan uses it also depends on the device (m workgroups
// resident at once), which the workspace size does not.
bool resident_candidate(const int64_t* off, int32_t m, int64_t ldc, int32_t k, int32_t flags,
                        int* rpw, int* cpl) {
  if (k != 1 || uses_gemm(k, flags) || base_precision(flags) != APC_F64) return false;
  int64_t pmax = 0;
  for (int i = 0; i < m; ++i) pmax = std::max(pmax, off[i + 1] - off[i]);
  return resident_shape(pmax, ldc, rpw, cpl);
}

Layout make_layout(int64_t N, int64_t n, const int64_t* off, int32_t m, int32_t k, int32_t flags,
                   const Tiles& T) {
  Layout L;
  const int64_t kp = padded_rhs(k, flags);
  const int32_t prec = base_precision(flags);
  L.ldc = round_up(n, kLdAlign);
  L.kmax = std::min<int64_t>(n, kLanczosMax);
  for (int i = 0; i < m; ++i) L.S += (off[i + 1] - off[i]) * (off[i + 1] - off[i]);
  int64_t max_tiles_a = 0;  // tile lists of the smallest height
  for (int i = 0; i < m; ++i) max_tiles_a += (off[i + 1] - off[i] + kMinRowTile - 1) / kMinRowTile;
  L.ntiles_a = static_cast<int32_t>(T.a_row0.size());
  L.ntiles_g = static_cast<int32_t>(T.g.size() / 3);
  L.ntiles_t = static_cast<int32_t>(T.t.size() / 3);
  L.nparts = residual_parts(N);
  size_t cur = 0;
  auto take = [&](int64_t bytes) {
    const size_t at = cur;
    cur += static_cast<size_t>(round_up(std::max<int64_t>(bytes, 1), kAlign));
    return at;
  };
  const int64_t d = sizeof(double);
  const bool gemm = uses_gemm(k, flags);
  const bool bf = prec == APC_BF16_IR;
  const int64_t kq = k == 1 ? 1 : kp;        // k = 1 state columns
  L.C64a = take(N * L.ldc * d);
  L.C64b = take(N * L.ldc * d);
  L.C32 = take(prec == APC_F32 && !gemm ? N * L.ldc * 4 : 0);
  L.x = take(gemm ? 0 : m * kq * L.ldc * d);
  L.dv = take(gemm ? 0 : m * kq * L.ldc * d);
  L.w = take(kMaxSplit * N * d);
  L.ca = take(N * kp * d);
  L.cb = take(N * kp * d);
  L.Y = take(m * L.ldc * d);
  L.vtmp = take(L.ldc * d);
  L.V = take((L.kmax + 1) * L.ldc * d);
  // Lanczos step: two passes' dot partials per column slab, then the slab norms.
  const int64_t nlz = (L.ldc + kLzSlab - 1) / kLzSlab;
  L.h = take((2 * nlz * (L.kmax + 1) + nlz) * d);
  L.alpha = take((L.kmax + 1) * d);
  L.beta = take((L.kmax + 1) * d);
  L.G = take(L.S * d);
  L.Linv = take(L.S * d);
  L.Linv2 = take(L.S * d);  // both inverse CholeskyQR factors: c = L2^-1 L1^-1 b and back
  L.flags = take(4 * 4);
  L.scal = take(8 * d);
  L.partial = take(L.nparts * kq * d);
  // k-RHS path: the factor in the iteration's precision in both orientations
  // (C: Np x np, C^T: np x Np), its FP64 transpose for x_bar(0) = (1/m) C^T c
  // (the FP64 mode iterates on it), a padded FP64 copy of A for the residual,
  // the operands y and W, split-K partials, the FP64 state x0, y, x_bar.
  L.Np = gemm ? round_up(N, kTnPad) : 0;
  L.np = gemm ? round_up(n, kTnPad) : 0;
  const int64_t sq = prec == APC_F64 ? 8 : prec == APC_F32 ? 4 : 2;
  L.Cq = take(gemm ? L.Np * L.np * sq : 0);
  L.CqT = take(gemm ? L.np * L.Np * sq : 0);
  L.C64T = take(gemm && prec != APC_F64 ? L.np * L.Np * d : 0);
  // bf16: C^T in FP32 for the inner solves' starts (x_bar(0) = (1/m) C^T c).
  L.C32T = take(bf ? L.np * L.Np * 4 : 0);
  L.Apad = take(gemm ? L.Np * L.np * d : 0);
  L.yq = take(gemm ? kp * L.np * sq : 0);
  L.Wq = take(gemm ? kp * L.Np * sq : 0);
  L.tnpart = take(gemm ? static_cast<int64_t>(kTnMaxSplit) * kp * std::max(L.Np, L.np) * d : 0);
  L.xbar = take((gemm ? kp * L.np : kq * L.ldc) * d);
  L.x0 = take(gemm ? kp * L.np * d : 0);
  L.ys = take(gemm ? kp * L.np * d : 0);
  L.c64p = take(gemm ? kp * L.Np * d : 0);
  L.Xs = take(bf ? kp * L.np * d : 0);
  // Anchor updates (FP32 and bf16 iterations): the FP64 factor as pass-A
  // operand, the anchor y_ref, u_ref = X y_ref, and the FP64 W.
  const bool anc = gemm && prec != APC_F64;
  L.C64p = take(anc ? L.Np * L.np * d : 0);
  L.yref = take(anc ? kp * L.np * d : 0);
  L.uref = take(anc ? kp * L.np * d : 0);
  L.W64 = take(anc ? kp * L.Np * d : 0);
  L.Rb = take(gemm ? kp * N * d : 0);
  L.cw = take(bf ? kp * N * d : 0);
  L.ssq = take(sumsq_parts() * d);
  L.tiles_a = take(3 * max_tiles_a * 4);
  // Single-pass k = 1 iteration: its tile lists and one partial row per tile.
  // Also for FP32 / bf16 k-RHS plans, whose eigenvalue estimate runs the
  // FP32 single-pass kernel on a temporary FP32 copy of the factor.
  if ((!gemm && k == 1) || (gemm && prec != APC_F64)) {
    int64_t nf = 0;
    for (int i = 0; i < m; ++i) nf += (off[i + 1] - off[i] + kFusedMinRows - 1) / kFusedMinRows;
    L.ntiles_fmax = static_cast<int32_t>(nf);
  }
  L.tiles_f = take((3 * static_cast<int64_t>(L.ntiles_fmax) + m + 1) * 4);
  // FP64 entries: the normal operator of the eigenvalue estimate sums in FP64.
  L.fpart = take(static_cast<int64_t>(L.ntiles_fmax) * L.ldc * 8);
  L.v32 = take(L.ntiles_fmax > 0 ? L.ldc * 4 : 0);  // FP32 copy of an operator's vector
  L.tiles_g = take(3 * static_cast<int64_t>(L.ntiles_g) * 4);
  L.tiles_t = take(3 * static_cast<int64_t>(L.ntiles_t) * 4);
  L.doff = take((m + 1) * 8);
  L.goff = take(m * 8);
  // The triangular product's row-tile sums (the start x_i(0) = C_i^T c_i and
  // the orthogonality estimate's C_i^T y_i), then the estimate's random
  // N-vector y and its per-block norms (2 m).
  L.toff = take((m + 1) * 8);
  L.tpart = take((2 * T.toff.back() * L.ldc + N + 2 * m) * 8);
  {
    int rpw = 0, cpl = 0;
    const bool res = resident_candidate(off, m, L.ldc, k, flags, &rpw, &cpl);
    L.xch = take(res ? 2 * m * L.ldc * 16 : 0);  // two tagged 64-bit words per double
    L.rsync = take(4 * 4);
  }
  L.total = cur;
  return L;
}

apc_status validate(int64_t N, int64_t n, const int64_t* off, int32_t m, int32_t k,
                    int32_t prec) {
  if (n < 1 || N < n) return fail(APC_EINVAL, "need N >= n >= 1 (got N=%lld n=%lld)", (long long)N, (long long)n);
  if (m < 1 || m > N) return fail(APC_EINVAL, "need 1 <= m <= N (got m=%d)", m);
  if (!off) return fail(APC_EINVAL, "off is NULL");
  if (k < 1 || k > 1024) return fail(APC_EINVAL, "need 1 <= k <= 1024 (got %d)", k);
  const int32_t base = base_precision(prec);
  if (base != APC_F64 && base != APC_F32 && base != APC_BF16_IR)
    return fail(APC_EINVAL, "unknown precision %d", prec);
  if (off[0] != 0 || off[m] != N) return fail(APC_EINVAL, "off[0] must be 0 and off[m] must be N");
  const int64_t pmax = std::min<int64_t>(n, kMaxBlockRows);
  for (int i = 0; i < m; ++i) {
    const int64_t p = off[i + 1] - off[i];
    if (p < 1) return fail(APC_EINVAL, "block %d is empty or offsets decrease", i);
    if (p > n) return fail(APC_EINVAL, "block %d has p_i=%lld > n=%lld rows", i, (long long)p, (long long)n);
    if (p > pmax) return fail(APC_EUNSUPPORTED, "block %d has p_i=%lld > %d rows", i, (long long)p, kMaxBlockRows);
  }
  if (N > std::numeric_limits<int32_t>::max() / 2) return fail(APC_EINVAL, "N too large");
  return APC_OK;
}

// ------------------------------------------------------------------ tridiagonal eigen

// Number of eigenvalues of the symmetric tridiagonal (a, b) smaller than x.
int sturm_count(const std::vector<double>& a, const std::vector<double>& b, int k, double x) {
  int cnt = 0;
  double q = a[0] - x;
  if (q < 0) ++cnt;
  for (int i = 1; i < k; ++i) {
    if (q == 0.0) q = std::numeric_limits<double>::min();
    q = a[i] - x - b[i - 1] * b[i - 1] / q;
    if (q < 0) ++cnt;
  }
  return cnt;
}

// The idx-th smallest eigenvalue (0-based) by bisection on the Sturm count.
double tridiag_eig(const std::vector<double>& a, const std::vector<double>& b, int k, int idx) {
  double lo = a[0], hi = a[0];
  for (int i = 0; i < k; ++i) {
    const double r = (i > 0 ? std::fabs(b[i - 1]) : 0.0) + (i + 1 < k ? std::fabs(b[i]) : 0.0);
    lo = std::min(lo, a[i] - r);
    hi = std::max(hi, a[i] + r);
  }
  for (int it = 0; it < 200; ++it) {
    const double mid = 0.5 * (lo + hi);
    if (mid <= lo || mid >= hi) break;
    if (sturm_count(a, b, k, mid) > idx) hi = mid; else lo = mid;
  }
  return 0.5 * (lo + hi);
}

// Last component of the unit eigenvector of T for an extreme eigenvalue theta,
// by inverse iteration with a shift just outside the spectrum (the shifted
// matrix is definite, so elimination without pivoting is stable).
double last_component(const std::vector<double>& a, const std::vector<double>& b, int k,
                      double theta, bool top) {
  const double scale = std::max(std::fabs(theta), 1e-300);
  const double sigma = top ? theta + 1e-12 * scale + 1e-300 : theta - 1e-12 * scale - 1e-300;
  std::vector<double> s(k, 1.0 / std::sqrt(static_cast<double>(k))), dd(k), rr(k);
  for (int it = 0; it < 4; ++it) {
    // Thomas algorithm on (T - sigma I) z = s.
    dd[0] = a[0] - sigma;
    rr[0] = s[0];
    for (int i = 1; i < k; ++i) {
      const double l = b[i - 1] / dd[i - 1];
      dd[i] = a[i] - sigma - l * b[i - 1];
      rr[i] = s[i] - l * rr[i - 1];
    }
    s[k - 1] = rr[k - 1] / dd[k - 1];
    for (int i = k - 2; i >= 0; --i) s[i] = (rr[i] - b[i] * s[i + 1]) / dd[i];
    double nrm = 0.0;
    for (int i = 0; i < k; ++i) nrm += s[i] * s[i];
    nrm = std::sqrt(nrm);
    if (!(nrm > 0.0) || !std::isfinite(nrm)) return 1.0;  // unusable: report a loose bound
    for (int i = 0; i < k; ++i) s[i] /= nrm;
  }
  return s[k - 1];
}

// Theorem 1's optimum for a spectrum enclosed in [lo, hi].  With
// s = eta*gamma = 4/(sqrt(hi)+sqrt(lo))^2 and rho = (sqrt(hi)-sqrt(lo))/
// (sqrt(hi)+sqrt(lo)), u = gamma-1 and v = eta-1 satisfy u v = rho^2 and
// u + v = s - 1 - rho^2; u is the smaller root, formed without cancellation.
void optimum(double lo, double hi, double* gamma, double* eta, double* rho) {
  const double a = std::sqrt(hi), c = std::sqrt(lo);
  const double r = (a - c) / (a + c);
  const double s = 4.0 / ((a + c) * (a + c));
  const double sum = s - 1.0 - r * r;  // u + v >= 2 r >= 0
  const double disc = std::sqrt(std::max(sum * sum - 4.0 * r * r, 0.0));
  const double v = 0.5 * (sum + disc);
  const double u = v > 0.0 ? (r * r) / v : 0.0;
  *gamma = 1.0 + u;
  *eta = 1.0 + v;
  *rho = r;
}


}  // namespace

// ------------------------------------------------------------------ the plan

// Launch shape of one streaming contraction (rows per workgroup = 64 rt).
struct TnChoice {
  int rt = 2;
  int nsplit = 1;
  float us = 0.f;  // measured time per launch when tuned
  int pf = 1;      // steps of the streamed operand loaded ahead
  int nt = 1;      // non-temporal loads of the streamed operand
  int waves = 4;   // waves per workgroup (rows per workgroup = 16 waves rt)
};

struct apc_plan_s {
  int device = 0;
  hipStream_t stream = nullptr;
  int64_t N = 0, n = 0;
  int32_t m = 0, k = 1, kp = 1, prec = APC_F64;
  std::vector<int64_t> off;
  Layout L;
  char* ws = nullptr;
  const double* A = nullptr;
  int64_t lda = 0;
  const double* B = nullptr;
  int64_t ldb = 0;
  double gamma = 0, eta = 0;
  double mu_min = NAN, mu_max = NAN, rho = NAN;
  int64_t iters = 0;
  double bnorm = 0;
  int lanczos_steps = 0;
  int32_t xcd_remap = 1, passa_rows = kRowTile, nsplit = 1;
  int64_t split_cols = 0;
  int32_t group_blocks = 0;            // blocks per pass-A/pass-B group (MALL reuse)
  bool gemm = false;                   // k-RHS path: (y, x_bar) form on the matrix cores
  bool bf16 = false;                   // mixed precision: bf16 inner solver + FP64 refinement
  int tq = kTnF64;                     // element type of the k-RHS factor copies
  TnChoice tnA, tnB, tnX0, tnR;        // launch shapes: pass A, pass B, x_bar(0), residual
  int anchor_every = 0;                // k-RHS FP32/bf16: every this many updates one in FP64
  bool c64p_ready = false;             // the FP64 factor in pass-A orientation is packed
  bool c64t_ready = false;             // ... and in pass-B orientation (FP32 / bf16 plans)
  int64_t pmax = 1;                    // largest block
  int32_t passb_nt = 1;                // k = 1 pass B: non-temporal loads of C
  int32_t passb_rows = 1;              // k = 1 pass B: waves split the block's rows
  int32_t passa_nt = 1;                // k = 1 pass A: non-temporal loads of C
  bool fused = false;                  // k = 1: both halves of eq. (2a) in one pass over C
  int32_t fused_rows = 0, fused_g = 0, ntiles_f = 0;
  int64_t ntiles_tr = 0;               // triangular-product row tiles over all blocks
  int32_t fused_tpb = 0;               // > 0: every block has this many single-pass tiles
  bool resident = false;               // k = 1 FP64: T updates in one launch (k_resident)
  int32_t res_rpw = 0, res_cpl = 0, res_stride = 1;
  uint32_t res_spin = 1u << 22;        // polls of one exchanged word before it gives up
  int32_t qr_passes = 2;               // CholeskyQR passes setup took (1: see setup_impl)
  double qr_defect = NAN;              // estimated ||Q_i^T Q_i - I|| after the first pass
  double* pinned = nullptr;            // pinned host staging (Lanczos coefficients, setup readbacks)
  size_t pinned_n = 0;                 // its size in doubles
  hipEvent_t check_ev = nullptr;       // recorded after their copy
  int64_t since_start = 0;             // k-RHS updates since the last start
  int refinements = 0;
  bool inner_pending = false;          // APC_BF16_IR: the inner solve must restart on
                                       // B - A X before the next update
  std::vector<int32_t> tile_start;     // first pass-A tile of every block (m+1)
  std::vector<hipEvent_t> events;
  // Captured graphs of T updates (apc_iterate_graph), keyed by (T, the anchor
  // phase of the k-RHS form); their launches carry gamma and eta by value, so
  // apc_set_params and apc_set_anchor drop them.
  std::map<std::pair<int32_t, int32_t>, std::pair<hipGraph_t, hipGraphExec_t>> graphs;
  void drop_graphs() {
    for (auto& kv : graphs) {
      (void)hipGraphExecDestroy(kv.second.second);
      (void)hipGraphDestroy(kv.second.first);
    }
    graphs.clear();
  }

  template <typename T>
  T* at(size_t o) const { return reinterpret_cast<T*>(ws + o); }
  double* C64() const { return at<double>(L.C64a); }
  double* x() const { return at<double>(L.x); }
  double* xbar() const { return at<double>(L.xbar); }
  int64_t* doff() const { return at<int64_t>(L.doff); }
  int32_t* ta(int which) const { return at<int32_t>(L.tiles_a) + which * L.ntiles_a; }
  int32_t* tf(int which) const { return at<int32_t>(L.tiles_f) + which * ntiles_f; }
  int32_t slab_cols() const { return pass_b_slab(prec == APC_F32 ? 4 : 8, passb_rows); }
  int64_t state_ld() const { return static_cast<int64_t>(kp) * L.ldc; }  // block stride of x, d
};

namespace {

// Pass A over blocks [i0, i1) for right-hand side col: w = C d with
// d_i = x_bar - x_i precomputed by the previous average (or by setup).
apc_status pass_a(apc_plan_s* P, int i0, int i1, int col) {
  const int32_t t0 = P->tile_start[i0], nt = P->tile_start[i1] - t0;
  const int64_t coff = static_cast<int64_t>(col) * P->L.ldc;
  const int64_t woff = static_cast<int64_t>(col) * P->nsplit * P->N;
  if (P->prec == APC_F32) {
    RowdotArgs<float> a{P->at<float>(P->L.C32), P->L.ldc, P->ta(0), P->ta(1), P->ta(2), nt, 0,
                        nullptr, nullptr, 0, P->at<float>(P->L.dv) + coff, P->state_ld(),
                        P->at<float>(P->L.w) + woff, P->N, P->nsplit, P->split_cols,
                        P->xcd_remap, P->passa_rows, t0, P->passa_nt};
    HIP_TRY(launch_rowdot_f32(a, P->stream));
  } else {
    RowdotArgs<double> a{P->C64(), P->L.ldc, P->ta(0), P->ta(1), P->ta(2), nt, 0, nullptr,
                         nullptr, 0, P->at<double>(P->L.dv) + coff, P->state_ld(),
                         P->at<double>(P->L.w) + woff, P->N, P->nsplit, P->split_cols,
                         P->xcd_remap, P->passa_rows, t0, P->passa_nt};
    HIP_TRY(launch_rowdot_f64(a, P->stream));
  }
  return APC_OK;
}

// x_bar <- alpha sum_i x_i + beta x_bar, and the differences d_i for pass A.
apc_status average(apc_plan_s* P, double alpha, double beta) {
  const int64_t ld = P->state_ld();  // the average is elementwise over each block's state
  if (P->prec == APC_F32)
    HIP_TRY(launch_combine_f32(P->x(), ld, P->m, ld, alpha, beta, P->xbar(),
                               P->at<float>(P->L.dv), ld, P->stream));
  else
    HIP_TRY(launch_combine_f64(P->x(), ld, P->m, ld, alpha, beta, P->xbar(),
                               P->at<double>(P->L.dv), ld, P->stream));
  return APC_OK;
}

// Pass B over blocks [i0, i1) for right-hand side col:
// x_i += gamma (x_bar - x_i - Q_i w_i).
apc_status pass_b(apc_plan_s* P, int i0, int i1, int col) {
  const int32_t nslab = static_cast<int32_t>((P->L.ldc + P->slab_cols() - 1) / P->slab_cols());
  const int64_t coff = static_cast<int64_t>(col) * P->L.ldc;
  const int64_t woff = static_cast<int64_t>(col) * P->nsplit * P->N;
  if (P->prec == APC_F32) {
    PassBArgs<float> a{P->at<float>(P->L.C32), P->L.ldc, P->doff(), i1 - i0, nslab,
                       P->at<float>(P->L.w) + woff, P->nsplit, P->N, P->x() + coff,
                       P->state_ld(), P->xbar() + coff, P->gamma, i0, P->passb_nt,
                       P->passb_rows};
    HIP_TRY(launch_pass_b_f32(a, P->stream));
  } else {
    PassBArgs<double> a{P->C64(), P->L.ldc, P->doff(), i1 - i0, nslab,
                        P->at<double>(P->L.w) + woff, P->nsplit, P->N, P->x() + coff,
                        P->state_ld(), P->xbar() + coff, P->gamma, i0, P->passb_nt,
                       P->passb_rows};
    HIP_TRY(launch_pass_b_f64(a, P->stream));
  }
  return APC_OK;
}

// Both halves of eq. (2a) in one pass over C (k = 1): every single-pass tile
// writes its part of Q_i w_i, w = C_i d_i formed row by row on the way.
apc_status fused_pass(apc_plan_s* P) {
  const Layout& L = P->L;
  const int32_t remap = P->xcd_remap == 1 ? 1 : 0;
  if (P->prec == APC_F32) {
    FusedArgs<float, float> a{P->at<float>(L.C32), L.ldc, P->n, P->tf(0), P->tf(1), P->tf(2),
                              P->ntiles_f, P->at<float>(L.dv), P->state_ld(),
                              P->at<float>(L.fpart), L.ldc, remap};
    HIP_TRY(launch_fused_f32(a, P->fused_g, P->stream));
  } else {
    FusedArgs<double, double> a{P->C64(), L.ldc, P->n, P->tf(0), P->tf(1), P->tf(2),
                                P->ntiles_f, P->at<double>(L.dv), P->state_ld(),
                                P->at<double>(L.fpart), L.ldc, remap};
    HIP_TRY(launch_fused_f64(a, P->fused_g, P->stream));
  }
  return APC_OK;
}

// After fused_pass: x_i += gamma (x_bar - x_i - Q_i w_i), the average of
// eq. (2b) with weights (alpha, beta), and the next d_i.
apc_status fused_combine(apc_plan_s* P, double alpha, double beta) {
  const Layout& L = P->L;
  const int64_t ld = P->state_ld();
  if (P->prec == APC_F32) {
    FusedCombineArgs<float> a{P->at<float>(L.fpart), L.ldc, P->tf(3), P->x(), ld, P->m, P->n,
                              P->gamma, alpha, beta, P->xbar(), P->at<float>(L.dv), ld,
                              P->fused_tpb};
    HIP_TRY(launch_fused_combine_f32(a, P->stream));
  } else {
    FusedCombineArgs<double> a{P->at<double>(L.fpart), L.ldc, P->tf(3), P->x(), ld, P->m, P->n,
                               P->gamma, alpha, beta, P->xbar(), P->at<double>(L.dv), ld,
                               P->fused_tpb};
    HIP_TRY(launch_fused_combine_f64(a, P->stream));
  }
  return APC_OK;
}

// Departure from orthonormality of every block's rows of the FP64 factor C,
// Pinned host staging of at least n doubles, kept for the plan's life.
apc_status pinned_at_least(apc_plan_s* P, size_t n) {
  if (P->pinned && P->pinned_n >= n) return APC_OK;
  if (P->pinned) {
    HIP_TRY(hipHostFree(P->pinned));
    P->pinned = nullptr;
    P->pinned_n = 0;
  }
  void* hp = nullptr;
  // Coherent: the Lanczos step's kernel writes its coefficients here directly.
  HIP_TRY(hipHostMalloc(&hp, n * sizeof(double), hipHostMallocCoherent));
  P->pinned = static_cast<double*>(hp);
  P->pinned_n = n;
  return APC_OK;
}

apc_status expand_blocks(apc_plan_s* P, const double* w, double* y, double alpha, double beta,
                         const double* C = nullptr);
apc_status rowdot64(apc_plan_s* P, const double* va, const double* vb, int64_t ldvb, double* out,
                    const double* C = nullptr);

// max_i ||C_i C_i^T - I||, estimated with one random vector z: with
// C_i C_i^T = I + E_i, u_i = C_i^T C_i z and v_i = C_i^T C_i u_i differ by
// C_i^T E_i C_i z, so ||v_i - u_i|| / ||u_i|| estimates ||E_i|| (within a factor
// up to sqrt(p_i) when E_i is concentrated in one direction).  Two single passes
// over C when its rows fit the single-pass kernel (k = 1 plans), else two
// row-dot and two expansion passes; synchronises the stream.  Scratch: the Y
// and vtmp slices, and for the second vector the x slice (k = 1) or the padded
// copy of A's slice (k-RHS plans, before setup fills it), plus w.  flags (4
// ints) and scal (2 doubles), when non-null, are read back from the plan's
// slices in the same synchronisation.
apc_status read_defect(apc_plan_s* P, const double* out, double* defect, int* flags,
                       double* scal);
apc_status orthogonality_defect(apc_plan_s* P, const double* C, double* defect, int* flags = nullptr,
                                double* scal = nullptr) {
  const Layout& L = P->L;
  hipStream_t st = P->stream;
  double* zd = P->at<double>(L.vtmp);
  // z: the splitmix64 vector of the Lanczos start, normalised (the estimate is
  // a ratio), generated on the GPU.
  HIP_TRY(launch_lanczos_start(0x0a7ull * 1000003ull, P->n, L.ldc, zd, nullptr, st));
  double* U = P->at<double>(L.Y);
  double* V = P->gemm ? P->at<double>(L.Apad) : P->x();
  double* out = P->at<double>(L.w);
  // (k-RHS FP32 / bf16 plans have single-pass tiles for their eigenvalue estimate.)
  if (fused_cpt(L.ldc, 8) > 0 && (!P->gemm || P->ntiles_f > 0)) {
    double* part = P->at<double>(L.fpart);
    const int g = fused_cpt(L.ldc, 8) >= 16 ? 1 : 2;
    const int32_t remap = P->xcd_remap == 1 ? 1 : 0;
    for (int app = 0; app < 2; ++app) {
      FusedArgs<double, double> a{C, L.ldc, P->n, P->tf(0), P->tf(1), P->tf(2), P->ntiles_f,
                                  app == 0 ? zd : U, app == 0 ? 0 : L.ldc, part, L.ldc, remap};
      HIP_TRY(launch_fused_f64(a, g, st));
      HIP_TRY(launch_block_sum(part, L.ldc, P->tf(3), P->m, L.ldc, app == 0 ? U : V, L.ldc, st));
    }
  } else {
    // w = C z, U_i = C_i^T w_i; then w = C (0 - U_blk) = -C_i U_i, V_i = -C_i^T w_i.
    ST_TRY(rowdot64(P, zd, nullptr, 0, out, C));
    ST_TRY(expand_blocks(P, out, U, 1.0, 0.0, C));
    ST_TRY(rowdot64(P, nullptr, U, L.ldc, out, C));
    ST_TRY(expand_blocks(P, out, V, -1.0, 0.0, C));
  }
  HIP_TRY(launch_defect(U, V, L.ldc, P->m, P->n, out, st));
  return read_defect(P, out, defect, flags, scal);
}

// The same estimate from the other side, when the triangular product that
// wrote C also left the row-tile sums of C_i^T y_i for a random N-vector y
// (row toff[m] + t of the tpart slice): s_i = C_i^T y_i, then one row-dot
// pass w = -C s (in the plan's pass-A column splits, summed in split order),
// and C_i C_i^T y_i - y_i = -(w_i + y_i), so ||w_i + y_i|| / ||y_i||
// estimates ||E_i|| within the same factor.  One pass over C instead of two.
// y and the norms sit after the row sums in the tpart slice.
double* defect_vector(apc_plan_s* P) {
  return P->at<double>(P->L.tpart) + 2 * P->ntiles_tr * P->L.ldc;
}
apc_status orthogonality_defect_rows(apc_plan_s* P, const double* C, double* defect, int* flags,
                                     double* scal) {
  const Layout& L = P->L;
  hipStream_t st = P->stream;
  double* U = P->at<double>(L.Y);
  double* out = P->at<double>(L.w);
  const double* y = defect_vector(P);
  double* h = defect_vector(P) + P->N;
  const int64_t* toff = P->at<int64_t>(L.toff);
  HIP_TRY(launch_tile_sum(P->at<double>(L.tpart) + P->ntiles_tr * L.ldc, toff, P->m, L.ldc, U,
                          L.ldc, st));
  RowdotArgs<double> a{C, L.ldc, P->ta(0), P->ta(1), P->ta(2), L.ntiles_a, 0, nullptr, U, L.ldc,
                       nullptr, 0, out, P->N, P->nsplit, P->split_cols, P->xcd_remap,
                       P->passa_rows, 0};
  HIP_TRY(launch_rowdot_f64(a, st));
  HIP_TRY(launch_defect_rows(out, P->nsplit, P->N, y, P->doff(), P->m, h, st));
  return read_defect(P, h, defect, flags, scal);
}

// Reads the per-block norms (and flags, scal) back in one synchronisation;
// defect = max_i sqrt(h[2 i] / h[2 i + 1]).
apc_status read_defect(apc_plan_s* P, const double* out, double* defect, int* flags,
                       double* scal) {
  const Layout& L = P->L;
  hipStream_t st = P->stream;
  const size_t nh = 2 * static_cast<size_t>(P->m);
  // (sized for the Lanczos coefficients too, which come next)
  ST_TRY(pinned_at_least(P, std::max<size_t>(nh + 4, 2 * static_cast<size_t>(L.kmax + 1))));
  double* h = P->pinned;
  HIP_TRY(hipMemcpyAsync(h, out, nh * sizeof(double), hipMemcpyDeviceToHost, st));
  if (flags) HIP_TRY(hipMemcpyAsync(h + nh, P->at<int>(L.flags), 4 * sizeof(int), hipMemcpyDeviceToHost, st));
  if (scal) HIP_TRY(hipMemcpyAsync(h + nh + 2, P->at<double>(L.scal), 2 * sizeof(double), hipMemcpyDeviceToHost, st));
  HIP_TRY(hipStreamSynchronize(st));
  if (flags) std::memcpy(flags, h + nh, 4 * sizeof(int));
  if (scal) std::memcpy(scal, h + nh + 2, 2 * sizeof(double));
  double worst = 0.0;
  for (int i = 0; i < P->m; ++i) {
    const double e = h[2 * i + 1] > 0.0 ? std::sqrt(h[2 * i] / h[2 * i + 1]) : INFINITY;
    worst = std::isnan(e) ? INFINITY : std::max(worst, e);
  }
  *defect = worst;
  return APC_OK;
}

// ------------------------------------------------------------------ k right-hand sides
//
// For k > 1 the plan keeps APC in its (y, x_bar) form.  With the minimum-norm
// start x_i(0) = Q_i c_i (so P_i x_i(0) = 0), eq. (2a) keeps every local
// iterate at x_i(t) = x_i(0) + P_i y(t) with y(0) = 0 and
// y(t+1) = (1 - gamma) y(t) + gamma x_bar(t), so the average in eq. (2b) is
// (1/m) sum_i x_i(t+1) = x_bar(0) + y(t+1) - X y(t+1),  X = (1/m) C^T C.
// An update is then pass A (W = C y), pass B (Z = C^T W) and an elementwise
// step; no per-block state is streamed.

TnArgs tn_args(const void* M, int64_t ldm, int64_t rows, const void* V, int64_t ldv, int32_t kp,
               int64_t K, const TnChoice& ch, int type, void* part, int64_t ldp) {
  TnArgs a{M, ldm, rows, V, ldv, kp, K, ch.nsplit, 0, part, ldp, ch.nt, ch.waves};
  a.klen = round_up((K + ch.nsplit - 1) / ch.nsplit, tn_step_elems(type));
  return a;
}

TnArgs pass_a_args(const apc_plan_s* P) {
  const Layout& L = P->L;
  return tn_args(P->ws + L.Cq, L.np, L.Np, P->ws + L.yq, L.np, P->kp, L.np, P->tnA, P->tq,
                 P->ws + L.tnpart, L.Np);
}
TnArgs pass_b_args(const apc_plan_s* P) {
  const Layout& L = P->L;
  return tn_args(P->ws + L.CqT, L.Np, L.np, P->ws + L.Wq, L.Np, P->kp, L.Np, P->tnB, P->tq,
                 P->ws + L.tnpart, L.np);
}
// The start's contraction x_bar(0) = (1/m) C^T c: FP64 (the FP32 and FP64
// iterations), FP32 in the mixed-precision mode, whose inner solves only
// need the start to a relative 1e-7 or so (the FP64 residual of the
// refinement corrects the rest); its operand c then sits in the same slice
// as FP32.
int x0_type(const apc_plan_s* P) { return P->bf16 ? kTnF32 : kTnF64; }
TnArgs x0_args(const apc_plan_s* P) {
  const Layout& L = P->L;
  const void* Mt = P->tq == kTnF64 ? P->ws + L.CqT : P->bf16 ? P->ws + L.C32T : P->ws + L.C64T;
  return tn_args(Mt, L.Np, L.np, P->ws + L.c64p, L.Np, P->kp, L.Np, P->tnX0, x0_type(P),
                 P->ws + L.tnpart, L.np);
}
TnArgs resid_args(const apc_plan_s* P, const double* X) {
  const Layout& L = P->L;
  return tn_args(P->ws + L.Apad, L.np, L.Np, X, L.np, P->kp, L.np, P->tnR, kTnF64,
                 P->ws + L.tnpart, L.Np);
}

// The FP64 factor C (from the plan's FP64 slice) in the fragment-packed pass-A
// layout (C64p), once.
apc_status pack_c64p(apc_plan_s* P) {
  if (P->tq == kTnF64) return APC_OK;
  const Layout& L = P->L;
  if (!P->c64p_ready)
    HIP_TRY(launch_tn_pack_frag(kTnF64, P->C64(), L.ldc, P->N, P->n, 0, P->ws + L.C64p, L.np, L.Np,
                                P->stream));
  P->c64p_ready = true;
  // (A bf16 plan's anchor updates also need C^T in FP64.)
  if (!P->c64t_ready)
    HIP_TRY(launch_tn_pack_frag(kTnF64, P->C64(), L.ldc, P->N, P->n, 1, P->ws + L.C64T, L.Np, L.np,
                                P->stream));
  P->c64t_ready = true;
  return APC_OK;
}

TnUpdateArgs update_args(const apc_plan_s* P, const TnChoice& ch, int mode) {
  const Layout& L = P->L;
  // The start zeroes y_ref and u_ref whenever they exist (with both zero an
  // update is the same as an unanchored one).
  const bool anc = P->prec != APC_F64 && (P->anchor_every > 0 || mode == 1);
  return TnUpdateArgs{P->ws + L.tnpart, ch.nsplit, P->kp, L.np, L.np, P->at<double>(L.x0),
                      P->at<double>(L.ys), P->xbar(), L.np, P->ws + L.yq, L.np, P->gamma, P->eta,
                      1.0 / P->m, mode, anc ? P->at<double>(L.yref) : nullptr,
                      anc ? P->at<double>(L.uref) : nullptr};
}

// One update of the (y, x_bar) form.  In the FP32 and bf16 iterations every
// anchor_every-th update (the first after a start included) forms X y in FP64
// and keeps it as the anchor: u_ref = X y_ref.  The low-precision updates in
// between multiply only y - y_ref, which shrinks as the iteration converges,
// so their rounding (and the rounding of the stored factor) stops limiting
// the attainable accuracy.  *nev receives the number of events recorded.
// Timed updates: ev holds two events per timed kernel (start, end), kinds its
// pass (0 = A, 1 = B, 2 = average / epilogue).  time_next hands the next pair to
// the launcher (pending_timing); timed_done checks that the launch took it, and
// records the pair back to back when the launcher enqueued nothing.
void time_next(apc_plan_s*, hipEvent_t* ev, int* kinds, int* e, int kind) {
  if (!ev) return;
  pending_timing() = TimedLaunch{ev[2 * *e], ev[2 * *e + 1]};
  kinds[*e] = kind;
  ++*e;
}

apc_status timed_done(apc_plan_s* P, hipEvent_t* ev, int e) {
  if (!ev) return APC_OK;
  TimedLaunch& t = pending_timing();
  if (t.start) {
    t = TimedLaunch{};
    HIP_TRY(hipEventRecord(ev[2 * (e - 1)], P->stream));
    HIP_TRY(hipEventRecord(ev[2 * (e - 1) + 1], P->stream));
  }
  return APC_OK;
}

apc_status update_gemm(apc_plan_s* P, hipEvent_t* ev, int* kinds, int* nev) {
  const Layout& L = P->L;
  int e = 0;
  void* part = P->ws + L.tnpart;
  const bool anchor = P->anchor_every > 0 && P->since_start % P->anchor_every == 0;
  if (anchor) {
    const int64_t cnt = static_cast<int64_t>(P->kp) * L.np;
    HIP_TRY(launch_tn_anchor_vec(P->at<double>(L.ys), P->xbar(), cnt, P->gamma,
                                 P->at<double>(L.yref), P->stream));
    TnArgs a = tn_args(P->ws + L.C64p, L.np, L.Np, P->ws + L.yref, L.np, P->kp, L.np, P->tnR,
                       kTnF64, part, L.Np);
    time_next(P, ev, kinds, &e, 0);
    HIP_TRY(launch_tn(kTnF64, P->tnR.rt, P->tnR.pf, a, P->stream));
    ST_TRY(timed_done(P, ev, e));
    time_next(P, ev, kinds, &e, 2);
    HIP_TRY(launch_tn_sum_cast(kTnF64, part, P->tnR.nsplit, P->kp, L.Np, L.Np, P->ws + L.W64,
                               L.Np, P->stream));
    ST_TRY(timed_done(P, ev, e));
    // (A bf16 plan's start shape is an FP32 one: its anchors take the residual's.)
    const TnChoice& cb = P->bf16 ? P->tnR : P->tnX0;
    TnArgs b = tn_args(P->ws + L.C64T, L.Np, L.np, P->ws + L.W64, L.Np, P->kp, L.Np, cb, kTnF64,
                       part, L.np);
    time_next(P, ev, kinds, &e, 1);
    HIP_TRY(launch_tn(kTnF64, cb.rt, cb.pf, b, P->stream));
    ST_TRY(timed_done(P, ev, e));
    time_next(P, ev, kinds, &e, 2);
    HIP_TRY(launch_tn_update(P->tq, 1, update_args(P, cb, 2), P->stream));
    ST_TRY(timed_done(P, ev, e));
  } else {
    time_next(P, ev, kinds, &e, 0);
    HIP_TRY(launch_tn(P->tq, P->tnA.rt, P->tnA.pf, pass_a_args(P), P->stream));
    ST_TRY(timed_done(P, ev, e));
    time_next(P, ev, kinds, &e, 2);
    HIP_TRY(launch_tn_sum_cast(P->tq, part, P->tnA.nsplit, P->kp, L.Np, L.Np, P->ws + L.Wq, L.Np,
                               P->stream));
    ST_TRY(timed_done(P, ev, e));
    time_next(P, ev, kinds, &e, 1);
    HIP_TRY(launch_tn(P->tq, P->tnB.rt, P->tnB.pf, pass_b_args(P), P->stream));
    ST_TRY(timed_done(P, ev, e));
    time_next(P, ev, kinds, &e, 2);
    HIP_TRY(launch_tn_update(P->tq, P->tq == kTnF64, update_args(P, P->tnB, 0), P->stream));
    ST_TRY(timed_done(P, ev, e));
  }
  ++P->since_start;
  if (nev) *nev = e;
  return APC_OK;
}

// Starts the (y, x_bar) iteration for the right-hand sides whose transformed
// values c = R^{-T} b (RHS-major, stride N, zero past k) are given:
// x_bar(0) = (1/m) C^T c (FP64, or FP32 in the mixed-precision mode, see
// x0_args), y(0) = 0.
apc_status start_gemm(apc_plan_s* P, const double* c_rhs) {
  const Layout& L = P->L;
  const int t = x0_type(P);
  HIP_TRY(launch_tn_pack(t, c_rhs, P->N, P->kp, P->N, 0, P->ws + L.c64p, L.Np, P->kp, P->stream));
  HIP_TRY(launch_tn(t, P->tnX0.rt, P->tnX0.pf, x0_args(P), P->stream));
  HIP_TRY(launch_tn_update(P->tq, t == kTnF64, update_args(P, P->tnX0, 1), P->stream));
  P->since_start = 0;
  return APC_OK;
}

// R = B - A X (X: kp x np FP64, RHS-major) into R (RHS-major, stride N), k columns.
apc_status gemm_residual(apc_plan_s* P, const double* X, double* R) {
  const Layout& L = P->L;
  HIP_TRY(launch_tn(kTnF64, P->tnR.rt, P->tnR.pf, resid_args(P, X), P->stream));
  HIP_TRY(launch_tn_resid(P->at<double>(L.tnpart), P->tnR.nsplit, P->kp, L.Np, P->N, P->k, P->B,
                          P->ldb, R, P->N, P->stream));
  return APC_OK;
}

// Chooses the launch shape of one contraction by timing the candidates on the
// plan's operands (the partial buffer is scratch here).  Shapes are cached per
// (type, rows, K, kp) for the life of the process, so repeated plans of one
// shape launch identically and give identical results.
// scrub (optional): a contraction launched before each timed one, so that the
// candidate streams its operand the way an update does, right after the other
// orientation's pass has streamed its own (in a loop over one operand alone,
// part of it would still be in the 256 MB last-level cache).
struct TnScrub {
  TnArgs args;
  int type;
  TnChoice choice;
};
apc_status tn_tune(apc_plan_s* P, int type, TnArgs base, TnChoice* out,
                   const TnScrub* scrub = nullptr) {
  struct Key {
    int type;
    int64_t rows, K;
    int32_t kp;
    bool operator<(const Key& o) const {
      return std::tie(type, rows, K, kp) < std::tie(o.type, o.rows, o.K, o.kp);
    }
  };
  const int64_t ncg = base.kp >= 128 ? base.kp / 128 : 1;
  auto blocks = [&](int rt, int ns, int w = 4) { return (base.rows / (16 * w * rt)) * ncg * ns; };
  const int splits[4] = {1, 2, 4, 8};
  const char* fix_rt = std::getenv("APC_TN_RT");
  const char* fix_ns = std::getenv("APC_TN_SPLIT");
  const char* tune = std::getenv("APC_TN_TUNE");
  if (fix_rt || fix_ns || std::getenv("APC_TN_PF") || std::getenv("APC_TN_NT") ||
      (tune && std::atoi(tune) == 0)) {
    // Fixed shape (not cached): 128 rows per workgroup, the smallest split
    // with >= 512 workgroups, unless the environment names them.
    TnChoice c;
    c.rt = fix_rt ? std::atoi(fix_rt) : 2;
    if (c.rt != 1 && c.rt != 2 && c.rt != 4) c.rt = 2;
    if (type == kTnF64 && c.rt == 4) c.rt = 2;
    if (base.rows % (64 * c.rt)) c.rt = 1;
    c.nsplit = 8;
    for (int ns : splits)
      if (blocks(c.rt, ns) >= 512) { c.nsplit = ns; break; }
    if (fix_ns) c.nsplit = std::max(1, std::min(kTnMaxSplit, std::atoi(fix_ns)));
    if (const char* e = std::getenv("APC_TN_PF")) c.pf = std::max(1, std::min(4, std::atoi(e)));
    if (c.pf > 2 && (c.rt > 2 || type == kTnF64)) c.pf = 2;
    if (c.pf > 2) c.nt = 1;
    if (const char* e = std::getenv("APC_TN_NT")) c.nt = std::atoi(e) != 0;
    if (const char* e = std::getenv("APC_TN_WAVES"))
      if (std::atoi(e) == 8 && type != kTnF64 && (c.rt == 1 || (c.rt == 2 && c.pf <= 2)) && c.nt &&
          base.rows % (128 * c.rt) == 0)
        c.waves = 8;
    *out = c;
    return APC_OK;
  }
  static std::mutex mu;
  static std::map<Key, TnChoice> cache;
  const Key key{type, base.rows, base.K, base.kp};
  {
    std::lock_guard<std::mutex> lk(mu);
    auto it = cache.find(key);
    if (it != cache.end()) {
      *out = it->second;
      return APC_OK;
    }
  }
  std::vector<TnChoice> cand;
  const int rts[3] = {1, 2, 4};
  for (int rt : rts) {
    if (type == kTnF64 && rt == 4) continue;
    if (base.rows % (64 * rt)) continue;
    for (int ns : splits) {
      if (blocks(rt, ns) < 64 && !(rt == 1 && ns == 8)) continue;
      if (static_cast<int64_t>(ns) * tn_step_elems(type) > base.K && ns > 1) continue;
      for (int pf = 1; pf <= 4; ++pf)
        for (int nt = 0; nt <= 1; ++nt) {
          // Three and four steps ahead: non-temporal only, one or two tiles.
          if (pf > 2 && (nt == 0 || rt > 2 || type == kTnF64)) continue;
          TnChoice c;
          c.rt = rt;
          c.nsplit = ns;
          c.pf = pf;
          c.nt = nt;
          cand.push_back(c);
          // The same with eight waves per workgroup.
          // (Two tiles, two steps ahead and 128 right-hand sides spill there.)
          if (type != kTnF64 && (rt == 1 || (rt == 2 && pf <= 2)) && nt == 1 &&
              base.rows % (128 * rt) == 0 &&
              base.kp >= 32 && blocks(rt, ns, 8) >= 32 && !(rt == 2 && pf == 2 && base.kp >= 128)) {
            c.waves = 8;
            cand.push_back(c);
          }
        }
    }
  }
  if (cand.empty()) cand.push_back(TnChoice{1, 1, 0.f, 1, 1});
  TnChoice best;
  {
    // Each timed launch takes a pair of events recorded from its own dispatch.
    constexpr int kReps = 3;
    hipEvent_t ev[2 * kReps] = {};
    for (hipEvent_t& e : ev) HIP_TRY(hipEventCreate(&e));
    auto destroy = [&]() {
      for (hipEvent_t& e : ev) (void)hipEventDestroy(e);
    };
    auto run_scrub = [&]() -> hipError_t {
      if (!scrub) return hipSuccess;
      return launch_tn(scrub->type, scrub->choice.rt, scrub->choice.pf, scrub->args, P->stream);
    };
    float best_ms = 0.f;
    bool have = false;
    for (const TnChoice& c : cand) {
      TnArgs a = base;
      a.nsplit = c.nsplit;
      a.nt = c.nt;
      a.waves = c.waves;
      a.klen = round_up((a.K + c.nsplit - 1) / c.nsplit, tn_step_elems(type));
      hipError_t err = run_scrub();
      if (err == hipSuccess) err = launch_tn(type, c.rt, c.pf, a, P->stream);  // warm-up
      for (int r = 0; err == hipSuccess && r < kReps; ++r) {
        err = run_scrub();
        if (err != hipSuccess) break;
        pending_timing() = TimedLaunch{ev[2 * r], ev[2 * r + 1]};
        err = launch_tn(type, c.rt, c.pf, a, P->stream);
        if (pending_timing().start) {  // not taken: record back to back (never expected)
          pending_timing() = TimedLaunch{};
          err = hipErrorInvalidValue;
        }
      }
      float ms = 0.f;
      if (err == hipSuccess) err = hipEventSynchronize(ev[2 * kReps - 1]);
      for (int r = 0; err == hipSuccess && r < kReps; ++r) {
        float t = 0.f;
        err = hipEventElapsedTime(&t, ev[2 * r], ev[2 * r + 1]);
        ms += t;
      }
      if (err != hipSuccess) {
        pending_timing() = TimedLaunch{};
        destroy();
        return fail(APC_EHIP, "tuning launch failed: %s", hipGetErrorString(err));
      }
      ms /= static_cast<float>(kReps);
      if (!have || ms < best_ms) {
        best = c;
        best_ms = ms;
        have = true;
      }
    }
    destroy();
    best.us = best_ms * 1e3f;
  }
  std::lock_guard<std::mutex> lk(mu);
  cache[key] = best;
  *out = best;
  return APC_OK;
}

// One update of eq. (2a)-(2b).  k = 1, single pass: fused_pass, then
// fused_combine.  k = 1, two passes: for each group of blocks, pass A then
// pass B (pass B of a block needs only that block's w, so a group's rows of C
// are re-read while they are still in the Infinity Cache), then the average.
// With ev non-null, every kernel takes a pair of events (time_next) and its
// kind (0 pass A, 1 pass B, 2 average/epilogue) is appended to kinds; *nev
// receives the number of timed kernels (at most launches_per_update).
apc_status update(apc_plan_s* P, hipEvent_t* ev, int* kinds, int* nev) {
  if (P->gemm) return update_gemm(P, ev, kinds, nev);
  if (P->fused) {
    int e = 0;
    time_next(P, ev, kinds, &e, 0);
    ST_TRY(fused_pass(P));
    ST_TRY(timed_done(P, ev, e));
    time_next(P, ev, kinds, &e, 2);
    ST_TRY(fused_combine(P, P->eta / P->m, 1.0 - P->eta));
    ST_TRY(timed_done(P, ev, e));
    if (nev) *nev = e;
    return APC_OK;
  }
  const int g = P->group_blocks > 0 ? P->group_blocks : P->m;
  int e = 0;
  for (int i0 = 0; i0 < P->m; i0 += g) {
    const int i1 = std::min(P->m, i0 + g);
    time_next(P, ev, kinds, &e, 0);
    ST_TRY(pass_a(P, i0, i1, 0));
    ST_TRY(timed_done(P, ev, e));
    time_next(P, ev, kinds, &e, 1);
    ST_TRY(pass_b(P, i0, i1, 0));
    ST_TRY(timed_done(P, ev, e));
  }
  time_next(P, ev, kinds, &e, 2);
  ST_TRY(average(P, P->eta / P->m, 1.0 - P->eta));
  ST_TRY(timed_done(P, ev, e));
  if (nev) *nev = e;
  return APC_OK;
}

// T updates: one k_resident launch when the plan has that path, else T
// updates of the kernels above.
apc_status advance(apc_plan_s* P, int32_t T) {
  if (T <= 0) return APC_OK;
  if (P->resident) {
    const int64_t ld = P->state_ld();
    ResidentArgs a{P->C64(), P->L.ldc, static_cast<int32_t>(P->n), P->doff(), P->m, P->x(), ld,
                   P->xbar(), P->at<double>(P->L.dv), ld, P->gamma, P->eta / P->m,
                   1.0 - P->eta, T, P->at<uint64_t>(P->L.xch), P->at<uint32_t>(P->L.rsync),
                   P->res_stride, P->res_spin};
    HIP_TRY(launch_resident_f64(a, P->res_rpw, P->res_cpl, P->stream));
    return APC_OK;
  }
  for (int32_t t = 0; t < T; ++t) ST_TRY(update(P, nullptr, nullptr, nullptr));
  return APC_OK;
}

int launches_per_update(const apc_plan_s* P) {
  if (P->gemm) return 4;
  if (P->fused) return 2;
  const int g = P->group_blocks > 0 ? P->group_blocks : P->m;
  return 2 * ((P->m + g - 1) / g) + 1;
}

// y_i = alpha * C_i^T w_i + beta * y_i over all blocks of an FP64 factor C
// (the plan's, unless given).
apc_status expand_blocks(apc_plan_s* P, const double* w, double* y, double alpha, double beta,
                         const double* C) {
  ExpandArgs<double> e{C ? C : P->C64(), P->L.ldc, P->doff(), P->m,
                       static_cast<int32_t>((P->L.ldc + expand_slab(8) - 1) / expand_slab(8)),
                       P->N, w, 1, 0, y, P->L.ldc, alpha, beta, 0};
  HIP_TRY(launch_expand_f64(e, P->stream));
  return APC_OK;
}

// FP64 out = C d over the block tiles, d_i = va - vb_i (va or vb may be null),
// for an FP64 factor C (the plan's, unless given).
apc_status rowdot64(apc_plan_s* P, const double* va, const double* vb, int64_t ldvb,
                    double* out, const double* C) {
  RowdotArgs<double> a{C ? C : P->C64(), P->L.ldc, P->ta(0), P->ta(1), P->ta(2), P->L.ntiles_a, 0,
                       va, vb, ldvb, nullptr, 0, out, 0, 1, P->L.ldc, 0, P->passa_rows, 0};
  HIP_TRY(launch_rowdot_f64(a, P->stream));
  return APC_OK;
}

// X v for the eigenvalue estimate, through the factor the iteration uses
// (FP64, or FP32 storage with FP64 accumulation): u = C v, Y_i = Q_i u_i,
// out = (1/m) sum_i Y_i.
// A symmetric operator v -> scale * sum_i C_i^T (C_i v) over the plan's row
// blocks, for a row-major N x ldc matrix C streamed in FP32 or FP64: the
// plan's X (C = the factor, scale 1/m), or A^T A (C = a padded copy of A).
struct NormalOp {
  const void* C;
  bool f32;
  double scale;
};

NormalOp x_operator(const apc_plan_s* P) {
  const bool f32 = P->prec == APC_F32 && !P->gemm;  // the k = 1 FP32 factor; else the FP64 one
  return NormalOp{f32 ? static_cast<const void*>(P->at<float>(P->L.C32))
                      : static_cast<const void*>(P->C64()),
                  f32, 1.0 / P->m};
}

// out = op(v), FP64 vectors and accumulation.  v32_ready: the plan's FP32
// operator vector already holds v rounded to FP32.
// The single pass's partial rows, left for the caller to sum (the Lanczos step
// sums them in its first launch).
struct DeferredSum {
  const void* part = nullptr;
  bool f32 = false;
  int64_t ldp = 0;
  int32_t ntiles = 0;
  double scale = 1.0;
};

apc_status normal_matvec(apc_plan_s* P, const NormalOp& op, const double* v, double* out,
                         bool v32_ready = false, DeferredSum* defer = nullptr) {
  const Layout& L = P->L;
  // One pass over C (the plan's single-pass tiles, v shared by every tile),
  // then the FP64 sum of the tiles' partial rows.  Through the FP32 factor the
  // pass runs in FP32 like the iteration's (v rounded to FP32, FP32 partial
  // rows): the operator then carries a relative error ~1e-7, far below the
  // eigenvalue estimate's stopping tolerances (3e-4 and 1e-2).
  const int cpt64 = fused_cpt(L.ldc, 8);
  if (P->ntiles_f > 0 && (op.f32 || cpt64 > 0)) {
    double* part = P->at<double>(L.fpart);
    const int32_t remap = P->xcd_remap == 1 ? 1 : 0;
    if (op.f32) {
      float* v32 = P->at<float>(L.v32);
      float* part32 = P->at<float>(L.fpart);
      if (!v32_ready) HIP_TRY(launch_cast_f32(v, v32, L.ldc, P->stream));
      FusedArgs<float, float> a{static_cast<const float*>(op.C), L.ldc, P->n, P->tf(0), P->tf(1),
                                P->tf(2), P->ntiles_f, v32, 0, part32, L.ldc, remap};
      HIP_TRY(launch_fused_f32(a, P->fused_g, P->stream));
      if (defer) {
        *defer = DeferredSum{part32, true, L.ldc, P->ntiles_f, op.scale};
        return APC_OK;
      }
      HIP_TRY(launch_fused_sum_f32(part32, L.ldc, P->ntiles_f, L.ldc, op.scale, out, P->stream));
      return APC_OK;
    } else {
      FusedArgs<double, double> a{static_cast<const double*>(op.C), L.ldc, P->n, P->tf(0),
                                  P->tf(1), P->tf(2), P->ntiles_f, v, 0, part, L.ldc, remap};
      HIP_TRY(launch_fused_f64(a, cpt64 >= 16 ? 1 : 2, P->stream));
    }
    if (defer) {
      *defer = DeferredSum{part, false, L.ldc, P->ntiles_f, op.scale};
      return APC_OK;
    }
    HIP_TRY(launch_fused_sum(part, L.ldc, P->ntiles_f, L.ldc, op.scale, out, P->stream));
    return APC_OK;
  }
  double* u = P->at<double>(L.w);
  double* Y = P->at<double>(L.Y);
  const int g = P->group_blocks > 0 ? P->group_blocks : P->m;
  for (int i0 = 0; i0 < P->m; i0 += g) {
    const int i1 = std::min(P->m, i0 + g);
    const int32_t t0 = P->tile_start[i0], nt = P->tile_start[i1] - t0;
    if (op.f32) {
      const float* C = static_cast<const float*>(op.C);
      RowdotArgs<float, double> a{C, L.ldc, P->ta(0), P->ta(1), P->ta(2), nt, 0,
                                  v, nullptr, 0, nullptr, 0, u, 0, 1, L.ldc, P->xcd_remap,
                                  P->passa_rows, t0};
      HIP_TRY(launch_rowdot_f32x64(a, P->stream));
      ExpandArgs<float> e{C, L.ldc, P->doff(), i1 - i0,
                          static_cast<int32_t>((L.ldc + expand_slab(4) - 1) / expand_slab(4)),
                          P->N, u, 1, 0, Y, L.ldc, 1.0, 0.0, i0};
      HIP_TRY(launch_expand_f32(e, P->stream));
    } else {
      const double* C = static_cast<const double*>(op.C);
      RowdotArgs<double, double> a{C, L.ldc, P->ta(0), P->ta(1), P->ta(2), nt, 0, v,
                                   nullptr, 0, nullptr, 0, u, 0, 1, L.ldc, P->xcd_remap,
                                   P->passa_rows, t0};
      HIP_TRY(launch_rowdot_f64(a, P->stream));
      ExpandArgs<double> e{C, L.ldc, P->doff(), i1 - i0,
                           static_cast<int32_t>((L.ldc + expand_slab(8) - 1) / expand_slab(8)),
                           P->N, u, 1, 0, Y, L.ldc, 1.0, 0.0, i0};
      HIP_TRY(launch_expand_f64(e, P->stream));
    }
  }
  HIP_TRY(launch_combine_f64(Y, L.ldc, P->m, L.ldc, op.scale, 0.0, out, nullptr, 0, P->stream));
  return APC_OK;
}

// Lanczos with full (twice classical Gram-Schmidt) reorthogonalisation on a
// NormalOp (the plan's X v = (1/m) sum_i Q_i (Q_i^T v), or A^T A v for the
// heavy-ball comparison), on the GPU in FP64 arithmetic.  Returns an interval
// [lo, hi] (hi capped at `cap`: X's spectrum lies in [0, 1]) for the closed
// forms of the optimal parameters.  Ritz values lie inside the
// spectrum, and a spectrum that pokes out of [lo, hi] costs far more than a
// slightly wide interval: an eigenvalue delta outside turns the roots of p_i
// real and raises the rate by ~sqrt(delta), while widening the interval by
// delta raises it by O(delta).  So both ends are pushed outwards by a margin
// that covers the Ritz values' remaining movement.
apc_status lanczos(apc_plan_s* P, const NormalOp& op, double cap, double* lo_out, double* hi_out,
                   int* steps_out) {
  const int64_t ldc = P->L.ldc, n = P->n;
  const int kmax = static_cast<int>(P->L.kmax);
  const int64_t hstride = P->L.kmax + 1;
  double* V = P->at<double>(P->L.V);
  double* vt = P->at<double>(P->L.vtmp);
  double* hp = P->at<double>(P->L.h);
  double* al = P->at<double>(P->L.alpha);
  double* be = P->at<double>(P->L.beta);

  const int32_t nlz = static_cast<int32_t>((ldc + kLzSlab - 1) / kLzSlab);
  double* np = hp + 2 * static_cast<int64_t>(nlz) * hstride;

  double th_lo = 0, th_hi = 0, bd_lo = INFINITY, bd_hi = INFINITY;
  double d_lo = INFINITY, d_hi = INFINITY;
  // The extreme Ritz values after each step (index k - 1), for their change
  // over the last kLanczosWindow steps.
  std::vector<double> hist_lo, hist_hi;
  // The coefficients of the first k steps, in pinned host memory, decide
  // whether to stop after k steps.  The event after step k is awaited after
  // step k + 1 has been enqueued, so the GPU runs that step while the host
  // waits and decides; stopping then leaves one step unused.  Every step is
  // checked.
  ST_TRY(pinned_at_least(P, 2 * static_cast<size_t>(hstride)));
  if (!P->check_ev) HIP_TRY(hipEventCreateWithFlags(&P->check_ev, hipEventDisableTiming));
  double* ha = P->pinned;
  double* hb = P->pinned + hstride;
  std::vector<double> a, b;
  // Convergence test on T_k (alpha, beta of the first k steps in ha, hb).
  auto converged = [&](int k) -> apc_status {
    a.assign(ha, ha + k);
    b.assign(hb, hb + k);
    for (int i = 0; i < k; ++i)
      if (!std::isfinite(a[i]) || !std::isfinite(b[i]))
        return fail(APC_EDIVERGED, "non-finite value in the Lanczos recurrence");
    // A (numerically) zero beta_i means the Krylov space became invariant at
    // step i+1: T's leading block then holds exact eigenvalues of X, and with
    // a generic start vector it holds every distinct one.
    double scale = 0.0;
    for (int i = 0; i < k; ++i) scale = std::max(scale, std::fabs(a[i]));
    int kk = k;
    for (int i = 0; i < k; ++i)
      if (b[i] <= 1e-13 * scale) { kk = i + 1; break; }
    th_lo = tridiag_eig(a, b, kk, 0);
    th_hi = tridiag_eig(a, b, kk, kk - 1);
    const double bk = b[kk - 1];
    bd_hi = std::fabs(bk * last_component(a, b, kk, th_hi, true));
    bd_lo = std::fabs(bk * last_component(a, b, kk, th_lo, false));
    const bool exhausted = (kk < k) || (k == n) || (bk <= 1e-13 * std::max(th_hi, 1e-300));
    if (exhausted) {
      bd_lo = std::min(bd_lo, 1e-13 * th_hi);
      bd_hi = std::min(bd_hi, 1e-13 * th_hi);
    }
    // Converged ends: a small residual bound, or a Ritz value whose change
    // over the last four steps is below 3e-4 (top) or 1e-2 (bottom) of its
    // value, with a loose bound as a guard against an early plateau.  The
    // margins below cover the remaining movement (about 5x the last change for
    // the convergence rates seen at the spectral edges here) with a factor of
    // 4 to spare.  The enclosing interval is then a few 1e-3 wide above mu_max
    // and ~10 % below mu_min, which raises rho by O(width) only: at the
    // 16384 x 8192 benchmark shape 37 steps (each costs about 1.2 updates)
    // instead of 76 for about two more updates to 1e-6.
    hist_lo.resize(k, NAN);
    hist_hi.resize(k, NAN);
    hist_lo[k - 1] = th_lo;
    hist_hi[k - 1] = th_hi;
    const int kw = k - kLanczosWindow;
    const double prev_lo = kw >= 1 ? hist_lo[kw - 1] : NAN;
    const double prev_hi = kw >= 1 ? hist_hi[kw - 1] : NAN;
    d_lo = std::isnan(prev_lo) ? INFINITY : std::fabs(th_lo - prev_lo);
    d_hi = std::isnan(prev_hi) ? INFINITY : std::fabs(th_hi - prev_hi);
    const bool hi_ok = bd_hi <= 1e-10 * th_hi || (d_hi <= 3e-4 * th_hi && bd_hi <= 1e-2 * th_hi);
    const bool lo_ok = bd_lo <= 1e-6 * th_lo || (d_lo <= 1e-2 * th_lo && bd_lo <= 0.5 * th_lo);
    return (exhausted || (hi_ok && lo_ok)) ? APC_OK : APC_ENOCONV;
  };
  // The normalisation kernel also stores alpha_j, beta_j in the pinned buffer
  // (coherent host memory), so a check needs only an event, no copy.
  double* hab = nullptr;
  HIP_TRY(hipHostGetDevicePointer(reinterpret_cast<void**>(&hab), P->pinned, 0));
  auto issue_copy = [&](int) -> apc_status {
    HIP_TRY(hipEventRecord(P->check_ev, P->stream));
    return APC_OK;
  };
  auto decide = [&](int k, bool* stop) -> apc_status {
    HIP_TRY(hipEventSynchronize(P->check_ev));
    const apc_status c = converged(k);
    if (c != APC_OK && c != APC_ENOCONV) return c;
    *stop = c == APC_OK;
    return APC_OK;
  };
  // The FP32 operator reads the vector's FP32 copy, which the normalisation
  // writes for the next step.
  float* v32 = op.f32 && P->ntiles_f > 0 ? P->at<float>(P->L.v32) : nullptr;
  HIP_TRY(launch_lanczos_start(0x5eedull * 1000003ull, n, ldc, V, v32, P->stream));
  bool done = false;
  int steps = 0, pending = 0;
  for (int j = 0; j < kmax && !done; ++j) {
    DeferredSum ds;
    ST_TRY(normal_matvec(P, op, V + static_cast<int64_t>(j) * ldc, vt, v32 != nullptr, &ds));
    const LanczosArgs la{V,  ldc, j,  nlz, vt, hp, hstride, np, al, be,
                         V + static_cast<int64_t>(j + 1) * ldc, v32, hab};
    HIP_TRY(launch_lanczos_step(la, ds.part, ds.f32, ds.ldp, ds.ntiles, ds.scale, P->stream));
    const int k = j + 1;
    if (pending) {
      ST_TRY(decide(pending, &done));
      if (done) {
        steps = pending;
        break;
      }
      pending = 0;
    }
    steps = k;
    {
      ST_TRY(issue_copy(k));
      pending = k;
      if (k == kmax) {
        ST_TRY(decide(k, &done));
        pending = 0;
      }
    }
  }
  *steps_out = steps;
  if (!done)
    return fail(APC_ENOCONV, "eigenvalue estimate did not converge in %d Lanczos steps "
                "(theta in [%g, %g], bounds %g, %g); pass gamma and eta explicitly", kmax,
                th_lo, th_hi, bd_lo, bd_hi);
  if (!(th_lo > n * std::numeric_limits<double>::epsilon() * th_hi))
    return fail(APC_ESINGULAR, "smallest eigenvalue ~ 0 (Ritz value %g, largest %g): no unique "
                "solution", th_lo, th_hi);
  // The top end, where an underestimate of mu_max is the divergent side of
  // Theorem 1, takes the whole residual bound |beta_k s_k| (some eigenvalue
  // lies within it of the top Ritz value, which approaches mu_max from
  // below).  The bottom end, where an overestimate only slows the iteration,
  // takes at most 20 times its last change.
  const double m_lo = std::max(std::min(bd_lo, 20.0 * d_lo), 1e-13 * th_hi);
  const double m_hi = std::max(bd_hi, 1e-13 * th_hi);
  *lo_out = std::max(th_lo - m_lo, 0.5 * th_lo);
  *hi_out = std::min(th_hi + m_hi, cap);
  return APC_OK;
}

// ||B - A X||_F^2 into out_dev (X in RHS-major state layout, or null for ||B||^2).
// k = 1: row-dot kernel; k-RHS path: the FP64 matrix-core residual into R,
// then a fixed-order sum of squares.
apc_status residual_norm2(apc_plan_s* P, const double* x, double* out_dev) {
  int32_t parts = 0;
  double* partial = P->at<double>(P->L.partial);
  if (x && P->gemm) {
    ST_TRY(gemm_residual(P, x, P->at<double>(P->L.Rb)));
    HIP_TRY(launch_sumsq(P->at<double>(P->L.Rb), static_cast<int64_t>(P->k) * P->N,
                         P->at<double>(P->L.ssq), P->stream));
    HIP_TRY(launch_sum_partials(P->at<double>(P->L.ssq), sumsq_parts(), out_dev, P->stream));
    return APC_OK;
  }
  if (!x && P->ldb == P->k) {
    // ||B||_F^2 of a contiguous B: one sum of squares instead of a launch per
    // right-hand side.
    HIP_TRY(launch_sumsq(P->B, static_cast<int64_t>(P->k) * P->N, P->at<double>(P->L.ssq),
                         P->stream));
    HIP_TRY(launch_sum_partials(P->at<double>(P->L.ssq), sumsq_parts(), out_dev, P->stream));
    return APC_OK;
  }
  for (int col = 0; col < P->k; ++col)
    HIP_TRY(launch_residual_partial(P->A, P->lda, P->B + col, P->ldb, P->N, P->n,
                                    x ? x + static_cast<int64_t>(col) * P->L.ldc : nullptr,
                                    partial + static_cast<int64_t>(col) * P->L.nparts, &parts,
                                    P->stream));
  HIP_TRY(launch_sum_partials(partial, parts * P->k, out_dev, P->stream));
  return APC_OK;
}

// The current estimate in RHS-major layout: x_bar, or in the mixed-precision
// mode the committed solution plus the inner solve's x_bar (formed in cw).
apc_status current_solution(apc_plan_s* P, const double** out) {
  if (!P->bf16) {
    *out = P->xbar();
    return APC_OK;
  }
  // c64p (kp x Np >= kp x np) is free outside the start of an inner solve.
  double* cw = P->at<double>(P->L.c64p);
  const int64_t cnt = static_cast<int64_t>(P->kp) * P->L.np;
  HIP_TRY(launch_copy_strided(P->xbar(), 1, cw, 1, cnt, 1, P->stream));
  HIP_TRY(launch_axpy(cnt, 1.0, P->at<double>(P->L.Xs), cw, P->stream));
  *out = cw;
  return APC_OK;
}

apc_status check_device(int* dev) {
  int count = 0;
  if (hipGetDeviceCount(&count) != hipSuccess || count < 1)
    return fail(APC_ENODEV, "no HIP device available");
  HIP_TRY(hipGetDevice(dev));
  hipDeviceProp_t prop;
  HIP_TRY(hipGetDeviceProperties(&prop, *dev));
  if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0)
    return fail(APC_ENODEV, "libapc is built for gfx950 only (device is %s)", prop.gcnArchName);
  return APC_OK;
}

apc_status setup_impl(apc_plan_s* P, const Tiles& T) {
  const Layout& L = P->L;
  hipStream_t st = P->stream;
  const int64_t N = P->N, n = P->n, ldc = L.ldc;
  const int m = P->m;

  // Device copies of the block structure and tile lists.
  std::vector<int32_t> ta;
  ta.insert(ta.end(), T.a_row0.begin(), T.a_row0.end());
  ta.insert(ta.end(), T.a_nrows.begin(), T.a_nrows.end());
  ta.insert(ta.end(), T.a_blk.begin(), T.a_blk.end());
  HIP_TRY(hipMemcpyAsync(P->at<int32_t>(L.tiles_a), ta.data(), ta.size() * 4, hipMemcpyHostToDevice, st));
  HIP_TRY(hipMemcpyAsync(P->at<int32_t>(L.tiles_g), T.g.data(), T.g.size() * 4, hipMemcpyHostToDevice, st));
  std::vector<int32_t> tf;
  if (P->ntiles_f > 0) {
    tf.insert(tf.end(), T.f_row0.begin(), T.f_row0.end());
    tf.insert(tf.end(), T.f_nrows.begin(), T.f_nrows.end());
    tf.insert(tf.end(), T.f_blk.begin(), T.f_blk.end());
    tf.insert(tf.end(), T.f_first.begin(), T.f_first.end());
    HIP_TRY(hipMemcpyAsync(P->at<int32_t>(L.tiles_f), tf.data(), tf.size() * 4, hipMemcpyHostToDevice, st));
  }
  HIP_TRY(hipMemcpyAsync(P->at<int32_t>(L.tiles_t), T.t.data(), T.t.size() * 4, hipMemcpyHostToDevice, st));
  HIP_TRY(hipMemcpyAsync(P->doff(), P->off.data(), (m + 1) * 8, hipMemcpyHostToDevice, st));
  HIP_TRY(hipMemcpyAsync(P->at<int64_t>(L.goff), T.goff.data(), m * 8, hipMemcpyHostToDevice, st));
  HIP_TRY(hipMemcpyAsync(P->at<int64_t>(L.toff), T.toff.data(), (m + 1) * 8, hipMemcpyHostToDevice, st));
  HIP_TRY(launch_fill_u32(P->at<unsigned>(L.flags), 4, 0u, st));
  HIP_TRY(launch_fill_u32(P->at<unsigned>(L.rsync), 4, 0u, st));
  if (P->resident)
    HIP_TRY(launch_fill_u32(P->at<unsigned>(L.xch), 8 * P->m * L.ldc, 0u, st));

  // ||b||^2 for the residual monitor.
  ST_TRY(residual_norm2(P, nullptr, P->at<double>(L.scal) + 1));

  // CholeskyQR2 of every A_i^T: C <- L^{-1} C twice, c <- L^{-1} c alongside.
  double* Ca = P->at<double>(L.C64a);
  double* Cb = P->at<double>(L.C64b);
  double* ca = P->at<double>(L.ca);
  double* cb = P->at<double>(L.cb);
  // The Gram and triangular products run on the FP64 matrix cores
  // (APC_SETUP_MFMA=0 selects the vector kernels).
  bool mfma = true;
  if (const char* e = std::getenv("APC_SETUP_MFMA")) mfma = std::atoi(e) != 0;
  // When A's rows are already the factor's padded rows (n a multiple of 64,
  // lda = n, 16-byte aligned), the first pass reads A in place and only b is
  // copied (the matrix-core kernels never read past a block's rows).
  // The Gram product's K range is split so that the launch has about 2048
  // workgroups (four per CU fit at once) when the blocks alone give few
  // tiles, each range keeping at least 1024 columns (shorter rows gain
  // nothing); the partial Grams go to the factor slice the pass writes next,
  // which is free until the triangular product.
  int64_t gsize = 0;
  for (int i = 0; i < m; ++i) gsize += (P->off[i + 1] - P->off[i]) * (P->off[i + 1] - P->off[i]);
  int32_t gsplit = static_cast<int32_t>((2048 + L.ntiles_g - 1) / std::max(1, L.ntiles_g));
  if (const char* e = std::getenv("APC_GRAM_SPLIT")) gsplit = std::atoi(e);
  gsplit = static_cast<int32_t>(std::max<int64_t>(
      1, std::min<int64_t>({gsplit, 8, ldc / 1024, 1 + N * ldc / std::max<int64_t>(1, gsize)})));
  const bool in_place = mfma && n == ldc && P->lda == ldc &&
                        reinterpret_cast<uintptr_t>(P->A) % 16 == 0;
  HIP_TRY(launch_copy_pad(P->A, P->lda, P->B, P->ldb, N, n, in_place ? nullptr : Ca, ldc, ca,
                          P->k, P->kp, st));
  int64_t pmax = 1;
  for (int i = 0; i < m; ++i) pmax = std::max(pmax, P->off[i + 1] - P->off[i]);
  const double rank_tol = 32.0 * std::numeric_limits<double>::epsilon() *
                          static_cast<double>(std::max<int64_t>(pmax, 32));
  // An FP32 or bf16 plan rounds the factor to FP32 / bf16 for its products
  // (relative 6e-8 / 4e-3 per entry), so a second CholeskyQR pass, which takes
  // the rows' departure from orthonormality from the first pass's
  // ~kappa(A_i)^2 eps down to ~eps, changes nothing those products see when
  // that departure is already far below their rounding; the FP64 uses of the
  // factor (anchor updates, the k-RHS start, refinement restarts) then carry a
  // departure of at most the same 1e-10, below their tolerances.  The second
  // pass (about a quarter of setup at 16384 x 8192) is skipped when the
  // measured departure, times sqrt(p_max) for the estimate's worst case, is at
  // most 1e-10; FP64 plans and APC_QR_PASSES=2 always take two.
  bool may_skip = P->prec != APC_F64 && (P->gemm || P->fused);
  int flags[4] = {0, 0, 0, 0};
  double scal[2] = {0, 0};
  bool have_flags = false;  // read with the orthogonality estimate
  if (const char* e = std::getenv("APC_QR_PASSES")) may_skip = may_skip && std::atoi(e) != 2;
  // On the matrix-core path the triangular product also sums its rows: the
  // k = 1 start x_i(0) = C_i^T c_i (each pass; the last one's is used) and,
  // in a first pass that may be the only one, C_i^T y_i for the orthogonality
  // estimate's random N-vector y (the splitmix64 vector of the Lanczos start,
  // normalised; the estimate is a ratio), so that neither needs a pass of its
  // own over the factor.
  const bool x0_rows = mfma && !P->gemm && P->k == 1;
  double* yv = defect_vector(P);
  if (mfma && may_skip) HIP_TRY(launch_lanczos_start(0x0a7ull * 1000003ull, N, N, yv, nullptr, st));
  for (int pass = 0; pass < 2; ++pass) {
    const double* src = pass == 0 ? (in_place ? P->A : Ca) : Cb;
    double* dst = pass == 0 ? Cb : Ca;
    const double* cs = pass == 0 ? ca : cb;
    double* cd = pass == 0 ? cb : ca;
    if (mfma)
      HIP_TRY(launch_gram_lds(src, ldc, P->doff(), P->at<int32_t>(L.tiles_g), L.ntiles_g,
                              P->at<int64_t>(L.goff), P->at<double>(L.G), gsplit, dst, gsize, st));
    else
      HIP_TRY(launch_gram(src, ldc, P->doff(), P->at<int32_t>(L.tiles_g), L.ntiles_g,
                          P->at<int64_t>(L.goff), P->at<double>(L.G), st));
    // Both inverse factors are kept: refinement and apc_restart form
    // c = L2^{-1} L1^{-1} r, the adjoint applies L1^{-T} L2^{-T}.
    double* Li = pass == 1 ? P->at<double>(L.Linv2) : P->at<double>(L.Linv);
    HIP_TRY(launch_chol_inv(P->doff(), P->at<int64_t>(L.goff), m, P->pmax, P->at<double>(L.G), Li,
                            P->at<int>(L.flags), rank_tol, st));
    HIP_TRY(launch_linv_apply(P->doff(), P->at<int64_t>(L.goff), m, P->pmax, Li, cs, N, cd, N,
                              P->kp, 0, 1.0, st));
    // An FP32 k = 1 plan's factor copy is written by the same launch.
    float* dst32 = (P->prec == APC_F32 && !P->gemm) ? P->at<float>(L.C32) : nullptr;
    const bool est_rows = mfma && pass == 0 && may_skip;
    if (mfma) {
      const double* cx = x0_rows ? cd : nullptr;
      const double* cy = est_rows ? yv : nullptr;
      HIP_TRY(launch_trmm_lds(src, dst, ldc, P->doff(), m, P->pmax, P->at<int64_t>(L.goff), Li,
                              dst32, cx, cy, P->at<int64_t>(L.toff),
                              cx || cy ? P->at<double>(L.tpart) : nullptr, st));
    } else {
      HIP_TRY(launch_trmm(src, dst, ldc, P->doff(), P->at<int32_t>(L.tiles_t), L.ntiles_t,
                          P->at<int64_t>(L.goff), Li, st));
    }
    if (pass == 0 && may_skip) {
      if (est_rows)
        ST_TRY(orthogonality_defect_rows(P, dst, &P->qr_defect, flags, scal));
      else
        ST_TRY(orthogonality_defect(P, dst, &P->qr_defect, flags, scal));
      if (P->qr_defect * std::sqrt(static_cast<double>(pmax)) <= 1e-10) {
        have_flags = true;
        // The factor and c stay where the first pass left them: the plan's
        // layout names those slices from here on.
        P->qr_passes = 1;
        std::swap(P->L.C64a, P->L.C64b);
        std::swap(P->L.ca, P->L.cb);
        std::swap(Ca, Cb);
        std::swap(ca, cb);
        break;
      }
    }
  }
  if (!have_flags) {
    HIP_TRY(hipMemcpyAsync(flags, P->at<int>(L.flags), sizeof flags, hipMemcpyDeviceToHost, st));
    HIP_TRY(hipMemcpyAsync(scal, P->at<double>(L.scal), sizeof scal, hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
  }
  if (flags[0] != 0)
    return fail(APC_ERANK, "block %d is not of full row rank (Cholesky pivot below %g of the largest)",
                flags[0] - 1, rank_tol);
  P->bnorm = std::sqrt(scal[1]);

  if (P->gemm) {
    // Factor copies for the matrix cores (C and C^T in the iteration's
    // precision, C^T in FP64, C in FP64 for the anchor updates and the FP32
    // adjoint), the padded FP64 copy of A, zeroed operands.  Every one of them
    // is a streamed operand of the contraction kernel and is stored in its
    // fragment-packed layout; the copies of one orientation are written from a
    // single read of the FP64 factor.  A bf16 plan without anchors packs the
    // FP64 C when apc_set_anchor turns them on.
    const int64_t Np = L.Np, np = L.np;
    // FP32 / bf16: the eigenvalue estimate runs through a row-major FP32 copy
    // of the factor, written by the same read into the slice the padded copy
    // of A takes afterwards (one single pass over 4 bytes per entry per step
    // instead of two passes over 8).
    const bool est = P->ntiles_f > 0 && (std::isnan(P->gamma) || std::isnan(P->eta));
    float* c32 = est ? reinterpret_cast<float*>(P->ws + L.Apad) : nullptr;
    const bool pack64 = P->tq != kTnF64 && (P->anchor_every > 0 || !P->bf16) && !P->c64p_ready;
    HIP_TRY(launch_tn_pack_frag_multi(P->tq, Ca, ldc, N, n, 0, P->ws + L.Cq, np, Np,
                                      pack64 ? P->at<double>(L.C64p) : nullptr, kTnF64, c32, ldc,
                                      N, ldc, st));
    if (pack64) P->c64p_ready = true;
    // C^T: FP64 beside an FP32 iteration's copy; FP32 beside a bf16 one (its
    // starts), the FP64 one then packed with the anchors' operands if asked for.
    void* t2 = P->tq == kTnF64 ? nullptr : P->bf16 ? P->ws + L.C32T : P->ws + L.C64T;
    HIP_TRY(launch_tn_pack_frag_multi(P->tq, Ca, ldc, N, n, 1, P->ws + L.CqT, Np, np, t2,
                                      P->bf16 ? kTnF32 : kTnF64, nullptr, 0, 0, 0, st));
    if (P->tq != kTnF64 && !P->bf16) P->c64t_ready = true;
    if (P->bf16 && P->anchor_every > 0) ST_TRY(pack_c64p(P));
    if (est) {
      double lo = 0, hi = 0;
      ST_TRY(lanczos(P, NormalOp{c32, true, 1.0 / m}, 1.0, &lo, &hi, &P->lanczos_steps));
      P->mu_min = lo;
      P->mu_max = hi;
      optimum(lo, hi, &P->gamma, &P->eta, &P->rho);
    }
    HIP_TRY(launch_tn_pack_frag(kTnF64, P->A, P->lda, N, n, 0, P->ws + L.Apad, np, Np, st));
    const int64_t sq = P->tq == kTnF64 ? 8 : P->tq == kTnF32 ? 4 : 2;
    HIP_TRY(launch_fill_u32(P->at<unsigned>(L.yq), P->kp * np * sq / 4, 0u, st));
    HIP_TRY(launch_fill_u32(P->at<unsigned>(L.Wq), P->kp * Np * sq / 4, 0u, st));
    HIP_TRY(launch_fill_u32(P->at<unsigned>(L.c64p), 2 * P->kp * Np, 0u, st));
    HIP_TRY(launch_fill_u32(P->at<unsigned>(L.xbar), 2 * P->kp * np, 0u, st));
    HIP_TRY(launch_fill_u32(P->at<unsigned>(L.Rb), 2 * P->kp * N, 0u, st));
    if (P->bf16) {
      HIP_TRY(launch_fill_u32(P->at<unsigned>(L.cw), 2 * P->kp * N, 0u, st));
      HIP_TRY(launch_fill_u32(P->at<unsigned>(L.Xs), 2 * P->kp * np, 0u, st));
    }
    // The two passes alternate in an update: each is tuned right after the
    // other has streamed its operand (pass B first in a default shape).
    {
      TnChoice dflt;
      dflt.rt = 1;
      dflt.nsplit = 4;
      TnScrub sb{tn_args(P->ws + L.CqT, L.Np, L.np, P->ws + L.Wq, L.Np, P->kp, L.Np, dflt, P->tq,
                         P->ws + L.tnpart, L.np),
                 P->tq, dflt};
      ST_TRY(tn_tune(P, P->tq, pass_a_args(P), &P->tnA, &sb));
      const TnScrub sa{pass_a_args(P), P->tq, P->tnA};
      ST_TRY(tn_tune(P, P->tq, pass_b_args(P), &P->tnB, &sa));
    }
    ST_TRY(tn_tune(P, x0_type(P), x0_args(P), &P->tnX0));
    ST_TRY(tn_tune(P, kTnF64, resid_args(P, P->xbar()), &P->tnR));
  } else {
    // Alg. 1 initialisation: x_i(0) = Q_i c_i (minimum-norm local solutions),
    // x_bar(0) = (1/m) sum_i x_i(0).  The matrix-core triangular product left
    // x_i(0)'s row-tile sums.
    if (x0_rows)
      HIP_TRY(launch_tile_sum(P->at<double>(L.tpart), P->at<int64_t>(L.toff), m, ldc, P->x(),
                              P->state_ld(), st));
    for (int col = 0; col < (x0_rows ? 0 : P->k); ++col) {
      ExpandArgs<double> e{Ca, ldc, P->doff(), m,
                           static_cast<int32_t>((ldc + expand_slab(8) - 1) / expand_slab(8)), N,
                           ca + static_cast<int64_t>(col) * N, 1, 0,
                           P->x() + static_cast<int64_t>(col) * ldc, P->state_ld(), 1.0, 0.0, 0};
      HIP_TRY(launch_expand_f64(e, st));
    }
    ST_TRY(average(P, 1.0 / m, 0.0));
    if (P->prec == APC_F32 && !mfma) HIP_TRY(launch_cast_f32(Ca, P->at<float>(L.C32), N * ldc, st));
  }

  // Parameters: caller's, or Theorem 1's optimum from the estimated spectrum
  // (k-RHS FP32 / bf16 plans estimated it right after the QR).
  if (std::isnan(P->gamma) || std::isnan(P->eta)) {
    double lo = 0, hi = 0;
    ST_TRY(lanczos(P, x_operator(P), 1.0, &lo, &hi, &P->lanczos_steps));
    P->mu_min = lo;
    P->mu_max = hi;
    optimum(lo, hi, &P->gamma, &P->eta, &P->rho);
  }
  // The k-RHS start needs gamma (its first operand is y(1) = gamma x_bar(0)).
  // The mixed-precision mode's first inner solve has right-hand sides B and
  // committed solution X = 0.
  if (P->gemm) ST_TRY(start_gemm(P, ca));
  HIP_TRY(hipStreamSynchronize(st));
  return APC_OK;
}

}  // namespace

// ------------------------------------------------------------------ C ABI

extern "C" {

size_t apc_workspace_bytes(int64_t N, int64_t n, const int64_t* off, int32_t m, int32_t k,
                           int32_t precision) {
  if (validate(N, n, off, m, k, precision) != APC_OK) return 0;
  Tiles T;
  build_tiles(off, m, round_up(n, kLdAlign), kPassARows, &T);
  return make_layout(N, n, off, m, k, precision, T).total;
}

apc_status apc_setup(apc_plan* out, const double* A, int64_t lda, const double* B, int64_t ldb,
                     int64_t N, int64_t n, const int64_t* off, int32_t m, int32_t k,
                     int32_t precision, double gamma, double eta, void* workspace,
                     size_t ws_bytes, void* stream) {
  if (!out) return fail(APC_EINVAL, "out is NULL");
  *out = nullptr;
  apc_status st = validate(N, n, off, m, k, precision);
  if (st != APC_OK) return st;
  if (!A || !B) return fail(APC_EINVAL, "A and B must be device pointers");
  if (lda < n) return fail(APC_EINVAL, "lda=%lld < n=%lld", (long long)lda, (long long)n);
  if (ldb < 1) return fail(APC_EINVAL, "ldb must be >= 1");
  if (!workspace) return fail(APC_EINVAL, "workspace is NULL");
  if (reinterpret_cast<uintptr_t>(workspace) % kAlign != 0)
    return fail(APC_EINVAL, "workspace must be 256-byte aligned");
  const bool given = !std::isnan(gamma) && !std::isnan(eta);
  if (given && (!std::isfinite(gamma) || !std::isfinite(eta)))
    return fail(APC_EINVAL, "gamma and eta must be finite (or NaN for the optimum)");
  // Launch-shape knobs (defaults are the tuned ones; the environment may override).
  int32_t xcd_remap = 1, passa_rows = kPassARows, nsplit_req = 0, group_blocks = -1;
  if (const char* e = std::getenv("APC_XCD_REMAP")) xcd_remap = std::max(0, std::min(2, std::atoi(e)));
  int32_t passa_nt = 1;
  if (const char* e = std::getenv("APC_PASSA_NT")) passa_nt = std::atoi(e) != 0;
  if (const char* e = std::getenv("APC_PASSA_SPLIT")) nsplit_req = std::atoi(e);
  if (const char* e = std::getenv("APC_GROUP_BLOCKS")) group_blocks = std::atoi(e);
  int32_t passb_nt = 1;
  if (const char* e = std::getenv("APC_PASSB_NT")) passb_nt = std::atoi(e) != 0;
  int32_t passb_rows = 1;
  if (const char* e = std::getenv("APC_PASSB_ROWS")) passb_rows = std::atoi(e) != 0;
  if (const char* e = std::getenv("APC_PASSA_ROWS")) {
    const int r = std::atoi(e);
    if (r == 8 || r == 16 || r == 32) passa_rows = r;
  }
  Tiles T;
  build_tiles(off, m, round_up(n, kLdAlign), passa_rows, &T);
  // k = 1 FP64/FP32: one pass over C per update when a row fits the
  // single-pass kernel (n up to 16384 in FP32, 8192 in FP64).
  const int32_t base_prec = base_precision(precision);
  const int elem = base_prec == APC_F32 ? 4 : 8;
  const int cpt = fused_cpt(round_up(n, kLdAlign), elem);
  bool fused = !uses_gemm(k, precision) && k == 1 && cpt > 0;
  if (const char* e = std::getenv("APC_FUSED")) fused = fused && std::atoi(e) != 0;
  // FP32 / bf16 k-RHS plans: single-pass tiles for the eigenvalue operator
  // through an FP32 copy of the factor.
  const int cpt32 = fused_cpt(round_up(n, kLdAlign), 4);
  const bool op_tiles = uses_gemm(k, precision) && base_prec != APC_F64 && cpt32 > 0 &&
                        fused_shape_ok(4, 4, cpt32, 1);
  int32_t fused_rows = 0, fused_g = 0;
  if (op_tiles) {
    fused_shape(N, 4, cpt32, &fused_rows, &fused_g);
    build_fused_tiles(off, m, fused_rows, &T);
  }
  if (fused) {
    fused_shape(N, elem, cpt, &fused_rows, &fused_g);
    if (const char* e = std::getenv("APC_FUSED_ROWS")) {
      const int r = std::atoi(e);
      if (r == 16 || r == 32 || r == 64 || r == 128) fused_rows = r;
    }
    if (const char* e = std::getenv("APC_FUSED_G")) {
      const int g = std::atoi(e);
      if (fused_shape_ok(elem, elem, cpt, g)) fused_g = g;
    }
    build_fused_tiles(off, m, fused_rows, &T);
  }
  const Layout L = make_layout(N, n, off, m, k, precision, T);
  if (ws_bytes < L.total)
    return fail(APC_EINVAL, "workspace has %zu bytes, needs %zu", ws_bytes, L.total);

  int dev = 0;
  st = check_device(&dev);
  if (st != APC_OK) return st;
  // Once per device: the address of this GPU's copy of the allocation-free
  // adjoint's scratch.
  HIP_TRY(noalloc_scratch_init(dev));

  apc_plan_s* P = new (std::nothrow) apc_plan_s();
  if (!P) return fail(APC_EINVAL, "out of host memory");
  P->device = dev;
  P->stream = static_cast<hipStream_t>(stream);
  P->N = N;
  P->n = n;
  P->m = m;
  P->k = k;
  P->kp = padded_rhs(k, precision);
  P->prec = base_precision(precision);
  P->off.assign(off, off + m + 1);
  for (int i = 0; i < m; ++i) P->pmax = std::max(P->pmax, off[i + 1] - off[i]);
  P->L = L;
  P->ws = static_cast<char*>(workspace);
  P->A = A;
  P->lda = lda;
  P->B = B;
  P->ldb = ldb;
  P->gamma = given ? gamma : NAN;
  P->eta = given ? eta : NAN;
  P->xcd_remap = xcd_remap;
  P->passb_nt = passb_nt;
  P->passb_rows = passb_rows;
  P->passa_nt = passa_nt;
  P->passa_rows = passa_rows;
  P->fused = fused;
  P->fused_rows = fused_rows;
  P->fused_g = fused_g;
  P->ntiles_f = static_cast<int32_t>(T.f_row0.size());
  P->ntiles_tr = T.toff.back();
  {
    // At eight or more 16-byte chunks per thread, two-row register groups
    // take every register of a wave, one workgroup per CU: tiles beyond the
    // CU count then run as a second round of their own.  Between one and two
    // tiles per CU, one-row groups (two workgroups per CU) run them at once.
    int cus = 0;
    HIP_TRY(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    const int ce = fused ? elem : 4, cc = fused ? cpt : cpt32;
    const bool fixed = std::getenv("APC_FUSED_G") != nullptr;
    if (!fixed && P->fused_g == 2 && cc >= 8 && P->ntiles_f > cus && P->ntiles_f <= 2 * cus &&
        fused_shape_ok(ce, ce, cc, 1))
      P->fused_g = 1;
  }
  if (fused) {
    const int32_t t0 = T.f_first[1];
    bool same = true;
    for (int i = 0; i < m; ++i) same = same && T.f_first[i + 1] - T.f_first[i] == t0;
    if (same && (t0 == 1 || t0 == 2 || t0 == 4 || t0 == 8)) P->fused_tpb = t0;
  }
  {
    // One launch for T updates when every block fits one workgroup and the
    // device holds all m workgroups at once (one per CU).
    int rpw = 0, cpl = 0, cus = 0;
    HIP_TRY(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    bool res = resident_candidate(off, m, L.ldc, k, precision, &rpw, &cpl) && m <= cus;
    if (const char* e = std::getenv("APC_RESIDENT")) res = res && std::atoi(e) != 0;
    P->resident = res;
    P->res_rpw = rpw;
    P->res_cpl = cpl;
    // Stride 8 launches 8 workgroups per block and keeps every eighth, which
    // the dispatcher deals to one XCD; all m must then fit that XCD's CUs.
    if (const char* e = std::getenv("APC_RESIDENT_STRIDE")) {
      const int s = std::atoi(e);
      if (s == 1 || (s == kXcds && m <= cus / kXcds)) P->res_stride = s;
    }
    // Failure-path tests shorten the bounded wait from the host.
    if (const char* e = std::getenv("APC_RESIDENT_SPIN"))
      P->res_spin = static_cast<uint32_t>(std::strtoul(e, nullptr, 10));
  }
  P->tile_start.assign(1, 0);
  for (int i = 0; i < m; ++i)
    P->tile_start.push_back(P->tile_start.back() +
                            static_cast<int32_t>((off[i + 1] - off[i] + passa_rows - 1) / passa_rows));
  P->group_blocks = group_blocks >= 0 ? group_blocks : 0;
  P->gemm = uses_gemm(k, precision);
  P->bf16 = P->prec == APC_BF16_IR;
  P->tq = P->prec == APC_F64 ? kTnF64 : P->prec == APC_F32 ? kTnF32 : kTnBF16;
  // FP32 k-RHS: an FP64 anchor update every kAnchorEvery updates; the bf16 inner solver
  // is corrected by the outer refinement instead (0 = never).
  P->anchor_every = (P->gemm && P->prec == APC_F32) ? kAnchorEvery : 0;
  if (const char* e = std::getenv("APC_ANCHOR_EVERY"))
    if (P->gemm && P->prec != APC_F64) P->anchor_every = std::max(0, std::atoi(e));
  {
    // Column splits of pass A: about 4096 workgroups (16 per CU, measured best
    // for streaming at the 16384 x 8192 shape), each split at least one
    // register chunk wide.
    const int64_t chunk = P->prec == APC_F32 ? rowdot_chunk<float>() : rowdot_chunk<double>();
    const int64_t max_split = std::max<int64_t>(1, (L.ldc + chunk - 1) / chunk);
    int64_t want = nsplit_req > 0 ? nsplit_req
                                  : (4096 + L.ntiles_a - 1) / std::max<int32_t>(L.ntiles_a, 1);
    want = std::max<int64_t>(1, std::min<int64_t>({want, max_split, kMaxSplit}));
    P->split_cols = round_up((L.ldc + want - 1) / want, chunk);
    P->nsplit = static_cast<int32_t>((L.ldc + P->split_cols - 1) / P->split_cols);
  }
  st = setup_impl(P, T);
  if (st != APC_OK) {
    (void)hipStreamSynchronize(P->stream);
    delete P;
    return st;
  }
  *out = P;
  return APC_OK;
}

}  // extern "C"

namespace {
apc_status resume_refinement(apc_plan_s* p);
}  // namespace

extern "C" {

apc_status apc_iterate(apc_plan p, int32_t T) {
  if (!p) return fail(APC_EINVAL, "plan is NULL");
  if (T < 0) return fail(APC_EINVAL, "T must be >= 0");
  if (T > 0) ST_TRY(resume_refinement(p));
  ST_TRY(advance(p, T));
  p->iters += T;
  return APC_OK;
}

apc_status apc_iterate_graph(apc_plan p, int32_t T) {
  if (!p) return fail(APC_EINVAL, "plan is NULL");
  if (T < 0) return fail(APC_EINVAL, "T must be >= 0");
  if (T == 0) return APC_OK;
  if (p->stream == nullptr) return fail(APC_EINVAL, "graph capture needs a non-default stream");
  ST_TRY(resume_refinement(p));
  const int32_t phase = p->gemm && p->anchor_every > 0
                            ? static_cast<int32_t>(p->since_start % p->anchor_every) : 0;
  const auto key = std::make_pair(T, phase);
  auto itg = p->graphs.find(key);
  if (itg == p->graphs.end()) {
    // Capture T updates.  Nothing runs during capture: the update counter of
    // the k-RHS form (which places the anchor updates) is put back after it.
    const int64_t since = p->since_start;
    hipGraph_t g = nullptr;
    HIP_TRY(hipStreamBeginCapture(p->stream, hipStreamCaptureModeThreadLocal));
    const apc_status st = advance(p, T);
    const hipError_t e = hipStreamEndCapture(p->stream, &g);
    p->since_start = since;
    if (st != APC_OK) {
      if (g) (void)hipGraphDestroy(g);
      return st;
    }
    HIP_TRY(e);
    hipGraphExec_t ex = nullptr;
    const hipError_t ei = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
    if (ei != hipSuccess) {
      (void)hipGraphDestroy(g);
      HIP_TRY(ei);
    }
    itg = p->graphs.emplace(key, std::make_pair(g, ex)).first;
  }
  HIP_TRY(hipGraphLaunch(itg->second.second, p->stream));
  if (p->gemm) p->since_start += T;
  p->iters += T;
  return APC_OK;
}

apc_status apc_iterate_timed(apc_plan p, int32_t T, float* ms_total, float* ms_pass_a,
                             float* ms_pass_b, float* ms_average) {
  if (!p) return fail(APC_EINVAL, "plan is NULL");
  if (T < 0) return fail(APC_EINVAL, "T must be >= 0");
  if (T > 0) ST_TRY(resume_refinement(p));
  const int per = launches_per_update(p);
  // Two bracketing events for the whole run, two per timed kernel.
  const size_t kern = static_cast<size_t>(T) * per;
  const size_t need = 2 * kern + 2;
  while (p->events.size() < need) {
    hipEvent_t e = nullptr;
    HIP_TRY(hipEventCreate(&e));
    p->events.push_back(e);
  }
  std::vector<int> kinds(kern + 1, -1);
  hipEvent_t* kev = p->events.data() + 2;
  size_t used = 0;
  if (T > 0) HIP_TRY(hipEventRecord(p->events[0], p->stream));
  for (int32_t t = 0; t < T; ++t) {
    int nev = 0;
    ST_TRY(update(p, kev + 2 * used, kinds.data() + used, &nev));
    used += static_cast<size_t>(nev);
  }
  p->iters += T;
  float sums[3] = {0.f, 0.f, 0.f}, tot = 0.f;
  if (T > 0) {
    HIP_TRY(hipEventRecord(p->events[1], p->stream));
    HIP_TRY(hipEventSynchronize(p->events[1]));
    for (size_t e = 0; e < used; ++e) {
      float ms = 0.f;
      HIP_TRY(hipEventElapsedTime(&ms, kev[2 * e], kev[2 * e + 1]));
      sums[kinds[e]] += ms;
    }
    HIP_TRY(hipEventElapsedTime(&tot, p->events[0], p->events[1]));
  }
  if (ms_total) *ms_total = tot;
  if (ms_pass_a) *ms_pass_a = sums[0];
  if (ms_pass_b) *ms_pass_b = sums[1];
  if (ms_average) *ms_average = sums[2];
  return APC_OK;
}

apc_status apc_residual(apc_plan p, double* relres) {
  if (!p || !relres) return fail(APC_EINVAL, "NULL argument");
  double* dst = p->at<double>(p->L.scal);
  const double* x = nullptr;
  ST_TRY(current_solution(p, &x));
  ST_TRY(residual_norm2(p, x, dst));
  double r2 = 0;
  uint32_t timed_out = 0;
  HIP_TRY(hipMemcpyAsync(&r2, dst, sizeof r2, hipMemcpyDeviceToHost, p->stream));
  if (p->resident)
    HIP_TRY(hipMemcpyAsync(&timed_out, p->at<uint32_t>(p->L.rsync) + 2, sizeof timed_out,
                           hipMemcpyDeviceToHost, p->stream));
  HIP_TRY(hipStreamSynchronize(p->stream));
  *relres = p->bnorm > 0 ? std::sqrt(r2) / p->bnorm : std::sqrt(r2);
  if (timed_out)
    return fail(APC_EHIP, "the single-launch update gave up waiting for its %d workgroups "
                "(the device did not hold them all at once); x_bar is NaN", p->m);
  return APC_OK;
}

namespace {

// Restarts the inner solve of the refinement on the residual R (FP64,
// RHS-major, stride N, k columns) of the committed solution X: the
// minimum-norm start of the correction equation, c = L2^{-1} L1^{-1} r per
// block (padded columns of R are zeroed first).
apc_status restart_inner(apc_plan_s* p, double* Rb) {
  const Layout& L = p->L;
  double* cw = p->at<double>(L.cw);
  if (p->kp > p->k)
    HIP_TRY(launch_fill_u32(reinterpret_cast<unsigned*>(Rb + static_cast<int64_t>(p->k) * p->N),
                            2 * (p->kp - p->k) * p->N, 0u, p->stream));
  HIP_TRY(launch_linv_apply(p->doff(), p->at<int64_t>(L.goff), p->m, p->pmax,
                            p->at<double>(L.Linv), Rb, p->N, cw, p->N, p->kp, 0, 1.0, p->stream));
  if (p->qr_passes == 2)
    HIP_TRY(launch_linv_apply(p->doff(), p->at<int64_t>(L.goff), p->m, p->pmax,
                              p->at<double>(L.Linv2), cw, p->N, Rb, p->N, p->kp, 0, 1.0, p->stream));
  else
    HIP_TRY(launch_copy_strided(cw, 1, Rb, 1, static_cast<int64_t>(p->kp) * p->N, 1, p->stream));
  ST_TRY(start_gemm(p, Rb));
  p->inner_pending = false;
  return APC_OK;
}

// A refined solve ends with the correction committed (X += x_bar, x_bar = 0)
// and no inner solve on the new residual.  Updates after it continue the
// refinement: R = B - A X in FP64, then the inner solve restarts on R.
apc_status resume_refinement(apc_plan_s* p) {
  if (!p->bf16 || !p->inner_pending) return APC_OK;
  double* Rb = p->at<double>(p->L.Rb);
  ST_TRY(gemm_residual(p, p->at<double>(p->L.Xs), Rb));
  return restart_inner(p, Rb);
}

// Mixed precision: iterative refinement around the bf16 inner solver.  Each
// step runs `inner` updates of the current inner solve, commits X += x_bar,
// forms R = B - A X in FP64 on matrix cores, and (unless done) restarts the
// inner solve on R.
apc_status solve_refined(apc_plan_s* p, double rtol, int32_t max_iters, int32_t* done_out,
                         double* rr_out) {
  const Layout& L = p->L;
  int inner = 25;
  if (std::isfinite(p->rho) && p->rho > 0.0 && p->rho < 1.0)
    inner = static_cast<int>(std::ceil(std::log(1e-3) / std::log(p->rho)));
  inner = std::max(8, std::min(inner, 200));
  int32_t done = 0;
  double rr = 0.0;
  double* Rb = p->at<double>(L.Rb);
  double* dst = p->at<double>(L.scal);
  for (;;) {
    const int32_t T = std::min(inner, max_iters - done);
    if (T > 0) ST_TRY(apc_iterate(p, T));
    done += T;
    // Commit the correction and form R = B - A X in FP64.
    const int64_t cnt = static_cast<int64_t>(p->kp) * L.np;
    HIP_TRY(launch_axpy(cnt, 1.0, p->xbar(), p->at<double>(L.Xs), p->stream));
    HIP_TRY(launch_fill_u32(reinterpret_cast<unsigned*>(p->xbar()), 2 * cnt, 0u, p->stream));
    ST_TRY(gemm_residual(p, p->at<double>(L.Xs), Rb));
    HIP_TRY(launch_sumsq(Rb, static_cast<int64_t>(p->k) * p->N, p->at<double>(L.ssq), p->stream));
    HIP_TRY(launch_sum_partials(p->at<double>(L.ssq), sumsq_parts(), dst, p->stream));
    double r2 = 0.0;
    HIP_TRY(hipMemcpyAsync(&r2, dst, sizeof r2, hipMemcpyDeviceToHost, p->stream));
    HIP_TRY(hipStreamSynchronize(p->stream));
    rr = p->bnorm > 0 ? std::sqrt(r2) / p->bnorm : std::sqrt(r2);
    ++p->refinements;
    if (!std::isfinite(rr)) {
      *done_out = done;
      *rr_out = rr;
      return fail(APC_EDIVERGED, "residual became non-finite after %d refinement steps",
                  p->refinements);
    }
    if (rr <= rtol || done >= max_iters) {
      // The inner state still belongs to the correction just committed;
      // the next update restarts it on the current residual.
      p->inner_pending = true;
      break;
    }
    ST_TRY(restart_inner(p, Rb));
  }
  *done_out = done;
  *rr_out = rr;
  return APC_OK;
}

}  // namespace

apc_status apc_solve(apc_plan p, double rtol, int32_t max_iters, double* Xbar, int64_t ldx,
                     int32_t* iters_out, double* relres_out) {
  if (!p || !Xbar) return fail(APC_EINVAL, "NULL argument");
  if (ldx < 1 || max_iters < 0 || !(rtol >= 0)) return fail(APC_EINVAL, "bad ldx/max_iters/rtol");
  double rr = 0;
  int32_t done = 0;
  apc_status st = APC_OK;
  if (p->bf16) {
    st = solve_refined(p, rtol, max_iters, &done, &rr);
    if (st != APC_OK && st != APC_EDIVERGED) return st;
  } else {
    ST_TRY(apc_residual(p, &rr));
    while (rr > rtol && done < max_iters) {
      const int32_t T = std::min(8, max_iters - done);
      ST_TRY(apc_iterate(p, T));
      done += T;
      ST_TRY(apc_residual(p, &rr));
      if (!std::isfinite(rr)) {
        st = fail(APC_EDIVERGED, "residual became non-finite after %d updates", done);
        break;
      }
    }
  }
  if (st == APC_OK && rr > rtol)
    st = fail(APC_ENOCONV, "relative residual %g > %g after %d updates", rr, rtol, done);
  apc_status cs = apc_get_xbar(p, Xbar, ldx);
  if (cs != APC_OK) return cs;
  HIP_TRY(hipStreamSynchronize(p->stream));
  if (iters_out) *iters_out = done;
  if (relres_out) *relres_out = rr;
  return st;
}

apc_status apc_get_xbar(apc_plan p, double* Xbar, int64_t ldx) {
  if (!p || !Xbar || ldx < (p->k == 1 ? 1 : p->k)) return fail(APC_EINVAL, "bad argument");
  const double* x = nullptr;
  ST_TRY(current_solution(p, &x));
  if (!p->gemm)
    HIP_TRY(launch_copy_strided(x, 1, Xbar, ldx, p->n, 1, p->stream));
  else
    HIP_TRY(launch_copy_t(x, p->L.np, Xbar, ldx, p->n, p->k, p->stream));
  return APC_OK;
}

apc_status apc_get_local(apc_plan p, double* X, int64_t ldx) {
  if (!p || !X) return fail(APC_EINVAL, "bad argument");
  if (p->bf16) return fail(APC_EUNSUPPORTED, "local solutions are not kept in the mixed-precision mode");
  if (!p->gemm) {
    if (ldx < p->n) return fail(APC_EINVAL, "ldx < n");
    HIP_TRY(launch_copy_strided(p->x(), p->L.ldc, X, ldx, p->m, p->n, p->stream));
    return APC_OK;
  }
  if (ldx < (p->k == 1 ? p->n : p->k)) return fail(APC_EINVAL, "ldx < k (k = 1: ldx < n)");
  // x_i(t) = x_i(0) + P_i y(t) = y + Q_i (c_i - Q_i^T y), per right-hand side,
  // in FP64 on the FP64 factor.
  const Layout& L = p->L;
  double* w = p->at<double>(L.w);
  double* r = p->at<double>(L.cb);
  double* Y = p->at<double>(L.Y);
  for (int col = 0; col < p->k; ++col) {
    const double* y = p->at<double>(L.ys) + static_cast<int64_t>(col) * L.np;
    ST_TRY(rowdot64(p, y, nullptr, 0, w));
    HIP_TRY(launch_copy_strided(p->at<double>(L.ca) + static_cast<int64_t>(col) * p->N, 1, r, 1,
                                p->N, 1, p->stream));
    HIP_TRY(launch_axpy(p->N, -1.0, w, r, p->stream));
    HIP_TRY(launch_copy_strided(y, 0, Y, L.ldc, p->m, L.ldc, p->stream));
    ST_TRY(expand_blocks(p, r, Y, 1.0, 1.0));
    for (int i = 0; i < p->m; ++i) {
      // k = 1: row i at X + i*ldx; k > 1: entry (i, j, c) at X[(i*n + j)*ldx + c].
      double* dst = p->k == 1 ? X + i * ldx : X + i * p->n * ldx + col;
      HIP_TRY(launch_copy_t(Y + static_cast<int64_t>(i) * L.ldc, 0, dst, p->k == 1 ? 1 : ldx,
                            p->n, 1, p->stream));
    }
  }
  return APC_OK;
}

apc_status apc_project(apc_plan p, const double* V, double* Out, int64_t ldv) {
  if (!p || !V || !Out || ldv < p->n) return fail(APC_EINVAL, "bad argument");
  if (p->k != 1) return fail(APC_EUNSUPPORTED, "apc_project needs a plan with k = 1");
  const Layout& L = p->L;
  double* Y = p->at<double>(L.Y);
  // Y_i <- V_i zero-padded to ldc; w = Q_i^T (0 - Y_i) = -Q_i^T V_i; Y_i += Q_i w.
  HIP_TRY(launch_fill_u32(reinterpret_cast<unsigned*>(Y), 2 * p->m * L.ldc, 0u, p->stream));
  HIP_TRY(launch_copy_strided(V, ldv, Y, L.ldc, p->m, p->n, p->stream));
  ST_TRY(rowdot64(p, nullptr, Y, L.ldc, p->at<double>(L.w)));
  ST_TRY(expand_blocks(p, p->at<double>(L.w), Y, 1.0, 1.0));
  HIP_TRY(launch_copy_strided(Y, L.ldc, Out, ldv, p->m, p->n, p->stream));
  return APC_OK;
}

apc_status apc_get_params(apc_plan p, double* gamma, double* eta, double* mu_min, double* mu_max,
                          double* rho) {
  if (!p) return fail(APC_EINVAL, "plan is NULL");
  if (gamma) *gamma = p->gamma;
  if (eta) *eta = p->eta;
  if (mu_min) *mu_min = p->mu_min;
  if (mu_max) *mu_max = p->mu_max;
  if (rho) *rho = p->rho;
  return APC_OK;
}

apc_status apc_optimal_params(double mu_min, double mu_max, double* gamma, double* eta,
                              double* rho) {
  if (!(mu_min > 0.0) || !(mu_max >= mu_min) || !(mu_max <= 1.0 + 1e-12))
    return fail(APC_EINVAL, "need 0 < mu_min <= mu_max <= 1 (got %g, %g)", mu_min, mu_max);
  double g = 0, e = 0, r = 0;
  optimum(mu_min, std::min(mu_max, 1.0), &g, &e, &r);
  if (gamma) *gamma = g;
  if (eta) *eta = e;
  if (rho) *rho = r;
  return APC_OK;
}

apc_status apc_tridiag_extremes(const double* alpha, const double* beta, int32_t k,
                                int32_t with_bounds, double* lo, double* hi, double* bound_lo,
                                double* bound_hi) {
  if (k < 1 || !alpha || (k > 1 && !beta) || (with_bounds && !beta))
    return fail(APC_EINVAL, "bad tridiagonal arguments");
  std::vector<double> a(alpha, alpha + k), b(k, 0.0);
  for (int i = 0; i + 1 < k; ++i) b[i] = beta[i];
  if (with_bounds) b[k - 1] = beta[k - 1];
  const double tl = tridiag_eig(a, b, k, 0);
  const double th = tridiag_eig(a, b, k, k - 1);
  if (lo) *lo = tl;
  if (hi) *hi = th;
  if (bound_lo) *bound_lo = with_bounds ? std::fabs(b[k - 1] * last_component(a, b, k, tl, false)) : 0.0;
  if (bound_hi) *bound_hi = with_bounds ? std::fabs(b[k - 1] * last_component(a, b, k, th, true)) : 0.0;
  return APC_OK;
}

apc_status apc_get_info(apc_plan p, int32_t* lanczos_steps, int32_t* rows_per_tile,
                        int32_t* column_splits, int32_t* block_groups, int32_t* refinements) {
  if (!p) return fail(APC_EINVAL, "plan is NULL");
  if (refinements) *refinements = p->refinements;
  if (lanczos_steps) *lanczos_steps = p->lanczos_steps;
  if (rows_per_tile) *rows_per_tile = p->passa_rows;
  if (column_splits) *column_splits = p->nsplit;
  if (block_groups) *block_groups = (launches_per_update(p) - 1) / 2;
  return APC_OK;
}

apc_status apc_get_setup(apc_plan p, int32_t* qr_passes, double* qr_defect) {
  if (!p) return fail(APC_EINVAL, "plan is NULL");
  if (qr_passes) *qr_passes = p->qr_passes;
  if (qr_defect) *qr_defect = p->qr_defect;
  return APC_OK;
}

apc_status apc_get_launch(apc_plan p, int32_t which, int32_t* rows_per_wg, int32_t* splits,
                          float* tuned_us) {
  if (!p) return fail(APC_EINVAL, "plan is NULL");
  if (which == 4) {
    if (!p->fused) return fail(APC_EUNSUPPORTED, "the plan does not use the single-pass k = 1 update");
    if (rows_per_wg) *rows_per_wg = p->fused_rows;
    if (splits) *splits = p->fused_g;
    if (tuned_us) *tuned_us = 0.f;
    return APC_OK;
  }
  if (which == 5) {
    if (!p->resident) return fail(APC_EUNSUPPORTED, "the plan does not use the single-launch update");
    if (rows_per_wg) *rows_per_wg = 8 * p->res_rpw;
    if (splits) *splits = 128 * p->res_cpl;
    if (tuned_us) *tuned_us = 0.f;
    return APC_OK;
  }
  if (which < 0 || which > 3) return fail(APC_EINVAL, "which must be 0..5");
  if (!p->gemm) return fail(APC_EUNSUPPORTED, "launch shapes are reported for the k-RHS path only");
  const TnChoice& c = which == 0 ? p->tnA : which == 1 ? p->tnB : which == 2 ? p->tnX0 : p->tnR;
  if (rows_per_wg) *rows_per_wg = 16 * c.waves * c.rt;
  if (splits) *splits = c.nsplit;
  if (tuned_us) *tuned_us = c.us;
  return APC_OK;
}

apc_status apc_set_anchor(apc_plan p, int32_t every) {
  if (!p) return fail(APC_EINVAL, "plan is NULL");
  if (every < 0) return fail(APC_EINVAL, "every must be >= 0");
  if (!p->gemm || p->prec == APC_F64)
    return fail(APC_EUNSUPPORTED, "anchor updates exist for FP32 / bf16 plans with the k-RHS form");
  if (p->since_start != 0)
    return fail(APC_EINVAL, "set the anchor spacing before the first update after setup");
  if (every > 0) ST_TRY(pack_c64p(p));
  if (every != p->anchor_every) {
    (void)hipStreamSynchronize(p->stream);  // no captured graph may still be running
    p->drop_graphs();
  }
  p->anchor_every = every;
  return APC_OK;
}

apc_status apc_set_params(apc_plan p, double gamma, double eta) {
  if (!p) return fail(APC_EINVAL, "plan is NULL");
  if (!std::isfinite(gamma) || !std::isfinite(eta))
    return fail(APC_EINVAL, "gamma and eta must be finite");
  if (gamma != p->gamma || eta != p->eta) {
    (void)hipStreamSynchronize(p->stream);  // no captured graph may still be running
    p->drop_graphs();
  }
  p->gamma = gamma;
  p->eta = eta;
  return APC_OK;
}

namespace {

// New right-hand sides (or the stored ones): c = L2^{-1} L1^{-1} b per block
// (L1^{-1} b after a one-pass setup), then the start of Alg. 1 again.
apc_status restart_impl(apc_plan_s* P, const double* B, int64_t ldb) {
  const Layout& L = P->L;
  hipStream_t st = P->stream;
  if (B) {
    P->B = B;
    P->ldb = ldb;
    double* cb = P->at<double>(L.cb);
    double* ca = P->at<double>(L.ca);
    // RHS-major copy of B (columns k..kp zero), then the two inverse factors.
    HIP_TRY(launch_tn_pack(kTnF64, B, ldb, P->N, P->k, 1, cb, P->N, P->kp, st));
    HIP_TRY(launch_linv_apply(P->doff(), P->at<int64_t>(L.goff), P->m, P->pmax,
                              P->at<double>(L.Linv), cb, P->N, ca, P->N, P->kp, 0, 1.0, st));
    if (P->qr_passes == 2) {
      HIP_TRY(launch_linv_apply(P->doff(), P->at<int64_t>(L.goff), P->m, P->pmax,
                                P->at<double>(L.Linv2), ca, P->N, cb, P->N, P->kp, 0, 1.0, st));
      HIP_TRY(launch_copy_strided(cb, 1, ca, 1, static_cast<int64_t>(P->kp) * P->N, 1, st));
    }
    ST_TRY(residual_norm2(P, nullptr, P->at<double>(L.scal) + 1));
    double b2 = 0;
    HIP_TRY(hipMemcpyAsync(&b2, P->at<double>(L.scal) + 1, sizeof b2, hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    P->bnorm = std::sqrt(b2);
  }
  const double* ca = P->at<double>(L.ca);
  if (P->gemm) {
    if (P->bf16)
      HIP_TRY(launch_fill_u32(P->at<unsigned>(L.Xs), 2 * static_cast<int64_t>(P->kp) * L.np, 0u, st));
    ST_TRY(start_gemm(P, ca));
  } else {
    ExpandArgs<double> e{P->C64(), L.ldc, P->doff(), P->m,
                         static_cast<int32_t>((L.ldc + expand_slab(8) - 1) / expand_slab(8)), P->N,
                         ca, 1, 0, P->x(), P->state_ld(), 1.0, 0.0, 0};
    HIP_TRY(launch_expand_f64(e, st));
    ST_TRY(average(P, 1.0 / P->m, 0.0));
  }
  P->iters = 0;
  P->refinements = 0;
  P->inner_pending = false;
  return APC_OK;
}

// Slices of the caller's backward workspace.
struct BwdLayout {
  size_t ck, seg, a, bh, g0, bq, red, total;
};

BwdLayout bwd_layout(const apc_plan_s* P, int32_t T, int32_t ckpt) {
  BwdLayout B{};
  const int64_t st = static_cast<int64_t>(P->kp) * P->L.np * 8;  // one FP64 state vector set
  const int64_t nck = T > 0 ? (T + ckpt - 1) / ckpt : 0;
  const int64_t sq = P->tq == kTnF64 ? 8 : 4;
  size_t cur = 0;
  auto take = [&](int64_t bytes) {
    const size_t at = cur;
    cur += static_cast<size_t>(round_up(std::max<int64_t>(bytes, 1), kAlign));
    return at;
  };
  B.ck = take((nck + 1) * 2 * st);             // (y, x_bar) at t = 0, ckpt, 2 ckpt, ... and T
  B.seg = take((std::min<int64_t>(ckpt, std::max(T, 1)) + 1) * 2 * st);  // one segment
  B.a = take(st);
  B.bh = take(st);
  B.g0 = take(st);
  B.bq = take(static_cast<int64_t>(P->kp) * P->L.np * sq);
  B.red = take(2 * static_cast<int64_t>(tn_adjoint_blocks()) * 8);
  B.total = cur;
  return B;
}

apc_status copy_state(apc_plan_s* P, double* y_dst, double* xb_dst, const double* y_src,
                      const double* xb_src) {
  const int64_t cnt = static_cast<int64_t>(P->kp) * P->L.np;
  HIP_TRY(launch_copy_strided(y_src, 1, y_dst, 1, cnt, 1, P->stream));
  HIP_TRY(launch_copy_strided(xb_src, 1, xb_dst, 1, cnt, 1, P->stream));
  return APC_OK;
}

// Put a saved (y, x_bar) back as the plan's state; the next update is an
// anchor update when anchoring is on, else its operand is formed here.
apc_status restore_state(apc_plan_s* P, const double* y, const double* xb) {
  const Layout& L = P->L;
  ST_TRY(copy_state(P, P->at<double>(L.ys), P->xbar(), y, xb));
  HIP_TRY(launch_tn_prep(P->tq, P->at<double>(L.ys), P->xbar(),
                         static_cast<int64_t>(P->kp) * L.np, P->gamma, P->ws + L.yq, P->stream));
  P->since_start = 0;
  return APC_OK;
}

}  // namespace

apc_status apc_restart(apc_plan p, const double* B, int64_t ldb) {
  if (!p) return fail(APC_EINVAL, "plan is NULL");
  if (B && ldb < (p->k == 1 ? 1 : p->k)) return fail(APC_EINVAL, "ldb < k");
  return restart_impl(p, B, ldb);
}

size_t apc_backward_workspace_bytes(apc_plan p, int32_t T, int32_t ckpt_every) {
  if (!p || !p->gemm || T < 0 || ckpt_every < 1) return 0;
  return bwd_layout(p, T, ckpt_every).total;
}

apc_status apc_backward(apc_plan p, const double* dXbar, int64_t ldd, int32_t T,
                        int32_t ckpt_every, double* dB, int64_t lddb, double* dgamma, double* deta,
                        void* bwd_ws, size_t bwd_bytes) {
  if (!p || !dXbar || !dB) return fail(APC_EINVAL, "NULL argument");
  if (!p->gemm || p->bf16)
    return fail(APC_EUNSUPPORTED, "the adjoint needs an FP64/FP32 plan in the (y, x_bar) form "
                "(k > 1 or APC_REDUCED_FORM)");
  if (T < 0 || ckpt_every < 1) return fail(APC_EINVAL, "need T >= 0 and ckpt_every >= 1");
  const int64_t kmin = p->k == 1 ? 1 : p->k;
  if (ldd < kmin || lddb < kmin) return fail(APC_EINVAL, "ldd and lddb must be >= k");
  const BwdLayout BL = bwd_layout(p, T, ckpt_every);
  if (!bwd_ws || bwd_bytes < BL.total)
    return fail(APC_EINVAL, "backward workspace has %zu bytes, needs %zu", bwd_bytes, BL.total);
  if (reinterpret_cast<uintptr_t>(bwd_ws) % kAlign != 0)
    return fail(APC_EINVAL, "backward workspace must be 256-byte aligned");
  apc_plan_s* P = p;
  const Layout& L = P->L;
  hipStream_t st = P->stream;
  char* bw = static_cast<char*>(bwd_ws);
  const int64_t cnt = static_cast<int64_t>(P->kp) * L.np;
  auto ck = [&](int64_t s) { return reinterpret_cast<double*>(bw + BL.ck) + 2 * s * cnt; };
  auto seg = [&](int64_t s) { return reinterpret_cast<double*>(bw + BL.seg) + 2 * s * cnt; };
  double* a = reinterpret_cast<double*>(bw + BL.a);
  double* bh = reinterpret_cast<double*>(bw + BL.bh);
  double* g0 = reinterpret_cast<double*>(bw + BL.g0);
  void* bq = bw + BL.bq;
  double* red = reinterpret_cast<double*>(bw + BL.red);
  double* ys = P->at<double>(L.ys);
  double* xb = P->xbar();
  const int64_t nck = T > 0 ? (T + ckpt_every - 1) / ckpt_every : 0;

  // Forward from the start, keeping (y, x_bar) every ckpt_every updates and at T.
  ST_TRY(restart_impl(P, nullptr, 0));
  for (int32_t t = 0; t < T; ++t) {
    if (t % ckpt_every == 0) ST_TRY(copy_state(P, ck(t / ckpt_every), ck(t / ckpt_every) + cnt, ys, xb));
    ST_TRY(update(P, nullptr, nullptr, nullptr));
  }
  ST_TRY(copy_state(P, ck(nck), ck(nck) + cnt, ys, xb));

  // Adjoint start: dL/dx_bar(T) = dXbar, dL/dy(T) = 0.
  HIP_TRY(launch_fill_u32(reinterpret_cast<unsigned*>(a), 2 * cnt, 0u, st));
  HIP_TRY(launch_fill_u32(reinterpret_cast<unsigned*>(g0), 2 * cnt, 0u, st));
  HIP_TRY(launch_fill_u32(reinterpret_cast<unsigned*>(red), 4 * tn_adjoint_blocks(), 0u, st));
  HIP_TRY(launch_tn_pack(kTnF64, dXbar, ldd, P->n, P->k, 1, bh, L.np, P->kp, st));
  HIP_TRY(launch_tn_prep(P->tq, a, bh, cnt, 1.0, bq, st));  // bq = TQ(bh)

  void* part = P->ws + L.tnpart;
  for (int64_t sgi = nck - 1; sgi >= 0; --sgi) {
    const int32_t t0 = static_cast<int32_t>(sgi * ckpt_every);
    const int32_t t1 = std::min(T, t0 + ckpt_every);
    // Recompute the segment's states.
    ST_TRY(restore_state(P, ck(sgi), ck(sgi) + cnt));
    ST_TRY(copy_state(P, seg(0), seg(0) + cnt, ys, xb));
    for (int32_t t = t0; t < t1; ++t) {
      ST_TRY(update(P, nullptr, nullptr, nullptr));
      ST_TRY(copy_state(P, seg(t - t0 + 1), seg(t - t0 + 1) + cnt, ys, xb));
    }
    // Reverse through it: X bh by the same two contractions as an update.
    for (int32_t t = t1 - 1; t >= t0; --t) {
      TnArgs pa = tn_args(P->ws + L.Cq, L.np, L.Np, bq, L.np, P->kp, L.np, P->tnA, P->tq, part, L.Np);
      HIP_TRY(launch_tn(P->tq, P->tnA.rt, P->tnA.pf, pa, st));
      HIP_TRY(launch_tn_sum_cast(P->tq, part, P->tnA.nsplit, P->kp, L.Np, L.Np, P->ws + L.Wq, L.Np, st));
      HIP_TRY(launch_tn(P->tq, P->tnB.rt, P->tnB.pf, pass_b_args(P), st));
      const double* s_t = seg(t - t0);
      const double* s_n = seg(t - t0 + 1);
      TnAdjointArgs ad{part, P->tnB.nsplit, P->kp, L.np, L.np, a, bh, g0, s_t, s_t + cnt,
                       s_n + cnt, L.np, bq, L.np, P->gamma, P->eta, 1.0 / P->m, red};
      HIP_TRY(launch_tn_adjoint(P->tq, ad, st));
    }
  }
  // x_bar(0) = x0 itself: its adjoint gets dL/dx_bar(0) too.
  HIP_TRY(launch_axpy(cnt, 1.0, bh, g0, st));
  // dL/dc = (1/m) C g0 in FP64, then dL/db_i = L1^{-T} L2^{-T} dL/dc_i.
  const void* C64 = P->tq == kTnF64 ? static_cast<const void*>(P->ws + L.Cq)
                                    : static_cast<const void*>(P->ws + L.C64p);
  double* W64 = P->tq == kTnF64 ? P->at<double>(L.Wq) : P->at<double>(L.W64);
  TnArgs pc = tn_args(C64, L.np, L.Np, g0, L.np, P->kp, L.np, P->tnR, kTnF64, part, L.Np);
  HIP_TRY(launch_tn(kTnF64, P->tnR.rt, P->tnR.pf, pc, st));
  HIP_TRY(launch_tn_sum_cast(kTnF64, part, P->tnR.nsplit, P->kp, L.Np, L.Np, W64, L.Np, st));
  double* t1b = P->at<double>(L.Rb);
  double* t2b = P->at<double>(L.cb);
  if (P->qr_passes == 2) {
    HIP_TRY(launch_linv_apply(P->doff(), P->at<int64_t>(L.goff), P->m, P->pmax,
                              P->at<double>(L.Linv2), W64, L.Np, t1b, P->N, P->kp, 1, 1.0 / P->m, st));
    HIP_TRY(launch_linv_apply(P->doff(), P->at<int64_t>(L.goff), P->m, P->pmax,
                              P->at<double>(L.Linv), t1b, P->N, t2b, P->N, P->kp, 1, 1.0, st));
  } else {  // one CholeskyQR pass: c = L1^{-1} b only
    HIP_TRY(launch_linv_apply(P->doff(), P->at<int64_t>(L.goff), P->m, P->pmax,
                              P->at<double>(L.Linv), W64, L.Np, t2b, P->N, P->kp, 1, 1.0 / P->m, st));
  }
  HIP_TRY(launch_copy_t(t2b, P->N, dB, lddb, P->N, P->k, st));
  // The plan is left at x_bar(T) of the forward run.
  ST_TRY(restore_state(P, ck(nck), ck(nck) + cnt));
  P->since_start = 0;
  P->iters = T;
  std::vector<double> hr(2 * static_cast<size_t>(tn_adjoint_blocks()));
  HIP_TRY(hipMemcpyAsync(hr.data(), red, hr.size() * sizeof(double), hipMemcpyDeviceToHost, st));
  HIP_TRY(hipStreamSynchronize(st));
  double sg = 0.0, se = 0.0;
  for (int b = 0; b < tn_adjoint_blocks(); ++b) {
    sg += hr[2 * b];
    se += hr[2 * b + 1];
  }
  if (dgamma) *dgamma = sg;
  if (deta) *deta = se;
  return APC_OK;
}

int64_t apc_iterations(apc_plan p) { return p ? p->iters : -1; }

void apc_destroy(apc_plan p) {
  if (!p) return;
  if (!p->graphs.empty()) {
    (void)hipStreamSynchronize(p->stream);
    p->drop_graphs();
  }
  for (hipEvent_t e : p->events) (void)hipEventDestroy(e);
  if (p->check_ev) (void)hipEventDestroy(p->check_ev);
  if (p->pinned) (void)hipHostFree(p->pinned);
  delete p;
}

const char* apc_last_error(void) { return g_last_error.c_str(); }

}  // extern "C"

// ------------------------------------------------------------------ batches of systems

struct apc_batch_s {
  std::vector<apc_plan_s*> plans;
  int32_t count = 0;
  hipStream_t stream = nullptr;
  char* ws = nullptr;
  BatchSys* sys = nullptr;
  int4* itemsA = nullptr;
  int4* itemsB = nullptr;
  int2* itemsV = nullptr;
  int32_t nA = 0, nB = 0, nV = 0;
  bool fused = false;                  // single pass: items F (sys, tile), W (sys, 64 columns)
  int4* itemsF = nullptr;
  int2* itemsW = nullptr;
  int32_t nF = 0, nW = 0;
  int32_t* active = nullptr;
  int32_t* item_start = nullptr;
  double* partial = nullptr;
  double* relres = nullptr;
  int32_t gridA = 1024, gridB = 1024, gridV = 1024;
  float tuned_us = 0.f;
  std::vector<int32_t> h_active;
  std::map<std::pair<int32_t, int32_t>, std::pair<hipGraph_t, hipGraphExec_t>> graphs;
  // Mixed batch (k-RHS plans with k = 1 systems): per-update work lists of
  // the four launches, for ordinary [0] and anchor [1] updates, and the
  // anchor prologue; the k-RHS plans' descriptors and their anchor cycle.
  bool mixed = false;
  BatchGemm* gemm = nullptr;
  std::vector<int32_t> gemm_sys;       // system index of each k-RHS plan
  std::vector<int32_t> gemm_slot;      // its residual slot in `partial`
  int4* itemsL[2][4] = {};
  int32_t nL[2][4] = {};
  int4* itemsL0 = nullptr;
  int32_t nL0 = 0;
  int32_t nct = 1;
  int32_t anchor_every = 0;
  int64_t since = 0;                   // updates of the k-RHS plans' anchor cycle
};

namespace {

struct BatchPlanItems {
  std::vector<int4> A, B;
  std::vector<int2> V;
  std::vector<int4> F;     // single pass (when every plan has it and rows fit):
                           // (sys, tile, first row, (rows - 1) | block << 8)
  std::vector<int2> W;
  std::vector<int4> L[2][4], L0;  // mixed batch work lists
  std::vector<BatchGemm> gemm;
  std::vector<int32_t> gemm_sys, gemm_slot;
  // Single pass: every system's row tiles (up to tile_rows rows of one
  // block) as row0[t], nrows[t], blk[t], then first[i] (m + 1), concatenated;
  // tile_at[s] is system s's offset in that array, tile_n[s] its tile count.
  std::vector<int32_t> tiles;
  std::vector<size_t> tile_at;
  std::vector<int32_t> tile_n;
  int tile_rows = 0;
  std::vector<int32_t> start;
};

// Rows per single-pass tile: each item streams long enough to cover the
// chain of dependent loads that starts it (the 256-system pass took 72 us
// with 64-row items, 67 with 128, 65 with 256).  Next to contraction tiles in
// a mixed batch the shorter items balance better, so 128 there.
constexpr int kBatchTileRows = 256;
constexpr int kBatchTileRowsMixed = 128;

// A batch updates in one pass over every factor when each plan does (k = 1
// single-pass tiles) and every row fits the batch kernel's registers.
bool batch_single_pass(const apc_plan* plans, int32_t count) {
  if (const char* e = std::getenv("APC_FUSED"))
    if (std::atoi(e) == 0) return false;
  for (int32_t s = 0; s < count; ++s) {
    if (plans[s]->gemm) continue;
    // The single-pass items carry the block index in 24 bits.
    if (!plans[s]->fused || plans[s]->L.ldc > kBatchFusedCols || plans[s]->m >= (1 << 24)) return false;
  }
  return true;
}

// The descriptor of a k-RHS plan in a mixed batch: its four contractions
// (arguments as update_gemm forms them), split sums and updates.
BatchGemm batch_gemm_desc(apc_plan_s* P) {
  const Layout& L = P->L;
  void* part = P->ws + L.tnpart;
  BatchGemm G{};
  G.tn[0] = pass_a_args(P);
  G.tn[1] = pass_b_args(P);
  G.tn[2] = tn_args(P->ws + L.C64p, L.np, L.Np, P->ws + L.yref, L.np, P->kp, L.np, P->tnR, kTnF64,
                    part, L.Np);
  G.tn[3] = tn_args(P->ws + L.C64T, L.Np, L.np, P->ws + L.W64, L.Np, P->kp, L.Np, P->tnX0, kTnF64,
                    part, L.np);
  // The batch kernel runs one 16-row tile per wave in four-wave workgroups.
  for (int q = 0; q < 4; ++q) {
    G.tn[q].waves = 4;
    G.tn_blocks[q] = static_cast<int32_t>((G.tn[q].rows / 64) * (P->kp / (16 * std::min(8, P->kp / 16))) *
                                          G.tn[q].nsplit);
  }
  G.sum_part = part;
  G.sum_nsplit[0] = P->tnA.nsplit;
  G.sum_nsplit[1] = P->tnR.nsplit;
  G.sum_ldp = L.Np;
  G.sum_rows = L.Np;
  G.sum_out[0] = P->ws + L.Wq;
  G.sum_out[1] = P->ws + L.W64;
  G.sum_ldo = L.Np;
  G.kp = P->kp;
  G.upd[0] = update_args(P, P->tnB, 0);
  G.upd[1] = update_args(P, P->tnX0, 2);
  G.y = P->at<double>(L.ys);
  G.xbar = P->xbar();
  G.yref = P->anchor_every > 0 ? P->at<double>(L.yref) : nullptr;
  G.state_count = static_cast<int64_t>(P->kp) * L.np;
  G.gamma = P->gamma;
  return G;
}

apc_status batch_items(const apc_plan* plans, int32_t count, BatchPlanItems* it) {
  it->start.push_back(0);
  for (int32_t s = 0; s < count; ++s) {
    const apc_plan_s* P = plans[s];
    if (P->gemm) {
      // One residual slot, filled by the plan's own FP64 residual (an empty
      // pass-A item keeps the slot's index in the per-system ranges).
      it->gemm_slot.push_back(static_cast<int32_t>(it->A.size()));
      it->A.push_back(make_int4(s, 0, 0, 0));
      it->start.push_back(static_cast<int32_t>(it->A.size()));
      continue;
    }
    for (int i = 0; i < P->m; ++i) {
      const int64_t r0 = P->off[i], p = P->off[i + 1] - r0;
      for (int64_t r = 0; r < p; r += 16)
        it->A.push_back(make_int4(s, static_cast<int>(r0 + r), static_cast<int>(std::min<int64_t>(16, p - r)), i));
      for (int64_t j = 0; j < P->n; j += 256) it->B.push_back(make_int4(s, i, static_cast<int>(j), 0));
    }
    for (int64_t j = 0; j < P->n; j += 256) it->V.push_back(make_int2(s, static_cast<int>(j)));
    it->start.push_back(static_cast<int32_t>(it->A.size()));
  }
  bool any_gemm = false;
  for (int32_t s = 0; s < count; ++s) any_gemm = any_gemm || plans[s]->gemm;
  if (batch_single_pass(plans, count)) {
    const int tr = any_gemm ? kBatchTileRowsMixed : kBatchTileRows;
    it->tile_rows = tr;
    // (weight, item) pairs, ordered below.
    std::vector<std::pair<int64_t, int4>> fw;
    std::vector<std::pair<int64_t, int2>> ww;
    for (int32_t s = 0; s < count; ++s) {
      const apc_plan_s* P = plans[s];
      if (P->gemm) {
        it->tile_at.push_back(it->tiles.size());
        it->tile_n.push_back(0);
        continue;
      }
      std::vector<int32_t> r0, nr, bk, first(1, 0);
      for (int i = 0; i < P->m; ++i) {
        const int64_t p = P->off[i + 1] - P->off[i];
        for (int64_t r = 0; r < p; r += tr) {
          r0.push_back(static_cast<int32_t>(P->off[i] + r));
          nr.push_back(static_cast<int32_t>(std::min<int64_t>(tr, p - r)));
          bk.push_back(i);
        }
        first.push_back(static_cast<int32_t>(r0.size()));
      }
      it->tile_at.push_back(it->tiles.size());
      it->tile_n.push_back(static_cast<int32_t>(r0.size()));
      for (auto* v : {&r0, &nr, &bk, &first}) it->tiles.insert(it->tiles.end(), v->begin(), v->end());
      for (size_t t = 0; t < r0.size(); ++t)
        fw.emplace_back(static_cast<int64_t>(nr[t]) * P->L.ldc,
                        make_int4(s, static_cast<int>(t), r0[t], (nr[t] - 1) | (bk[t] << 8)));
      for (int64_t j = 0; j < P->n; j += 64)
        ww.emplace_back(static_cast<int64_t>(r0.size()) + P->m, make_int2(s, static_cast<int>(j)));
    }
    // Largest items first: workgroups take items in launch order, so the big
    // tiles start early and small ones fill the end of the pass, instead of a
    // few big tiles running alone at its end.  Every item writes only its own
    // partial row or columns (partial rows are summed later in tile order), so
    // the order changes no result.
    auto by_weight = [](const auto& a, const auto& b) { return a.first > b.first; };
    std::stable_sort(fw.begin(), fw.end(), by_weight);
    std::stable_sort(ww.begin(), ww.end(), by_weight);
    for (const auto& f : fw) it->F.push_back(f.second);
    for (const auto& w : ww) it->W.push_back(w.second);
  }
  // Mixed batch: the k-RHS plans' contraction tiles and epilogue chunks next
  // to the k = 1 items, one list per launch.  Contraction tiles first (they
  // take longest), then the k = 1 work.
  if (!any_gemm) return APC_OK;
  auto item = [](int kind, int sys, int desc, int z, int w) { return make_int4(kind | (sys << 8), desc, z, w); };
  for (int32_t s = 0; s < count; ++s) {
    apc_plan_s* P = plans[s];
    if (!P->gemm) continue;
    const int g = static_cast<int>(it->gemm.size());
    it->gemm.push_back(batch_gemm_desc(P));
    it->gemm_sys.push_back(s);
    const BatchGemm& G = it->gemm.back();
    auto chunks = [](int64_t total) { return static_cast<int>((total + kBatchChunk - 1) / kBatchChunk); };
    for (int v = 0; v < 2; ++v) {
      const int tnk = v ? kItemTn64 : kItemTn32;
      for (int b = 0; b < G.tn_blocks[v ? 2 : 0]; ++b) it->L[v][0].push_back(item(tnk, s, g, v ? 2 : 0, b));
      const int nsum = chunks(static_cast<int64_t>(G.kp) * G.sum_rows);
      for (int c = 0; c < nsum; ++c) it->L[v][1].push_back(item(v ? kItemSum64 : kItemSum32, s, g, v, c));
      for (int b = 0; b < G.tn_blocks[v ? 3 : 1]; ++b) it->L[v][2].push_back(item(tnk, s, g, v ? 3 : 1, b));
      const int nupd = chunks(static_cast<int64_t>(G.upd[v].kp) * G.upd[v].n);
      for (int c = 0; c < nupd; ++c) it->L[v][3].push_back(item(v ? kItemUpd64 : kItemUpd32, s, g, v, c));
    }
    if (G.yref)
      for (int c = 0; c < chunks(G.state_count); ++c) it->L0.push_back(item(kItemAnchorVec, s, g, 0, c));
  }
  // The k = 1 systems are split between the two contraction launches (single
  // pass with pass A, combine with the split sums; or single pass with pass B,
  // combine with the update), balanced by the bytes of their factors, so that
  // neither launch carries all of them next to a full contraction.
  std::vector<int> side(count, 0);
  int64_t load[2] = {0, 0};
  std::vector<int32_t> order;
  for (int32_t s = 0; s < count; ++s)
    if (!plans[s]->gemm) order.push_back(s);
  std::sort(order.begin(), order.end(), [&](int32_t a, int32_t b) {
    return plans[a]->N * plans[a]->L.ldc > plans[b]->N * plans[b]->L.ldc;
  });
  for (int32_t s : order) {
    const int q = load[0] <= load[1] ? 0 : 1;
    side[s] = q;
    load[q] += plans[s]->N * plans[s]->L.ldc;
  }
  for (int v = 0; v < 2; ++v) {
    for (const int4& f : it->F) it->L[v][side[f.x] ? 2 : 0].push_back(item(kItemFused, f.x, f.x, f.y, 0));
    for (const int2& w : it->W) it->L[v][side[w.x] ? 3 : 1].push_back(item(kItemCombine, w.x, w.x, w.y, 0));
  }
  return APC_OK;
}

struct BatchLayout {
  size_t sys, A, B, V, F, W, T, active, start, partial, relres, gemm, L[2][4], L0, total;
};

BatchLayout batch_layout(int32_t count, const BatchPlanItems& it) {
  BatchLayout L{};
  size_t cur = 0;
  auto take = [&](int64_t bytes) {
    const size_t at = cur;
    cur += static_cast<size_t>(round_up(std::max<int64_t>(bytes, 1), kAlign));
    return at;
  };
  L.sys = take(static_cast<int64_t>(count) * sizeof(BatchSys));
  L.A = take(static_cast<int64_t>(it.A.size()) * sizeof(int4));
  L.B = take(static_cast<int64_t>(it.B.size()) * sizeof(int4));
  L.V = take(static_cast<int64_t>(it.V.size()) * sizeof(int2));
  L.F = take(static_cast<int64_t>(it.F.size()) * sizeof(int4));
  L.W = take(static_cast<int64_t>(it.W.size()) * sizeof(int2));
  L.T = take(static_cast<int64_t>(it.tiles.size()) * 4);
  L.active = take(static_cast<int64_t>(count) * 4);
  L.start = take(static_cast<int64_t>(count + 1) * 4);
  L.partial = take(static_cast<int64_t>(it.A.size()) * 8);
  L.relres = take(static_cast<int64_t>(count) * 8);
  L.gemm = take(static_cast<int64_t>(it.gemm.size()) * sizeof(BatchGemm));
  for (int v = 0; v < 2; ++v)
    for (int q = 0; q < 4; ++q) L.L[v][q] = take(static_cast<int64_t>(it.L[v][q].size()) * sizeof(int4));
  L.L0 = take(static_cast<int64_t>(it.L0.size()) * sizeof(int4));
  L.total = cur;
  return L;
}

apc_status batch_check_plans(const apc_plan* plans, int32_t count) {
  if (!plans || count < 1) return fail(APC_EINVAL, "need at least one plan");
  for (int32_t s = 0; s < count; ++s) {
    const apc_plan_s* P = plans[s];
    if (!P) return fail(APC_EINVAL, "plan %d is NULL", s);
    if (P->prec != APC_F32 || P->bf16 || (P->gemm && P->tq != kTnF32) || (!P->gemm && P->k != 1))
      return fail(APC_EUNSUPPORTED, "plan %d: batches take FP32 plans (k = 1 per-block form, or the "
                  "k-RHS form with FP32 products)", s);
    if (P->gemm && P->kp > 128)
      return fail(APC_EUNSUPPORTED, "plan %d: k-RHS plans in a batch need k <= 128", s);
    if (s >= (1 << 23)) return fail(APC_EINVAL, "too many plans");
    if (P->stream != plans[0]->stream) return fail(APC_EINVAL, "plans must share one stream");
    if (P->n > (1 << 30) || P->N > (1 << 30)) return fail(APC_EINVAL, "plan %d too large", s);
  }
  // k-RHS plans share one launch shape and one anchor cycle, and k = 1 plans
  // next to them must update in one pass.
  const apc_plan_s* first = nullptr;
  for (int32_t s = 0; s < count; ++s) {
    const apc_plan_s* P = plans[s];
    if (!P->gemm) continue;
    if (!first) { first = P; continue; }
    if (P->kp != first->kp || P->anchor_every != first->anchor_every || P->since_start != first->since_start)
      return fail(APC_EUNSUPPORTED, "k-RHS plans in one batch need the same padded k, anchor spacing "
                  "and number of updates since their start");
  }
  if (first && !batch_single_pass(plans, count))
    return fail(APC_EUNSUPPORTED, "k = 1 plans next to k-RHS plans must update in one pass "
                "(rows up to %d wide)", kBatchFusedCols);
  return APC_OK;
}

apc_status batch_update(apc_batch_s* B) {
  if (B->mixed) {
    const int v = B->anchor_every > 0 && B->since % B->anchor_every == 0 ? 1 : 0;
    if (v) HIP_TRY(launch_batch_mixed(B->gridA, B->nct, B->sys, B->gemm, B->itemsL0, B->nL0, B->active,
                                      B->stream));
    for (int q = 0; q < 4; ++q)
      HIP_TRY(launch_batch_mixed(B->gridA, B->nct, B->sys, B->gemm, B->itemsL[v][q], B->nL[v][q],
                                 B->active, B->stream));
    ++B->since;
    return APC_OK;
  }
  if (B->fused) {
    HIP_TRY(launch_batch_fused(B->gridA, B->sys, B->itemsF, B->nF, B->active, B->stream));
    HIP_TRY(launch_batch_fused_combine(B->gridV, B->sys, B->itemsW, B->nW, B->active, B->stream));
    return APC_OK;
  }
  HIP_TRY(launch_batch_pass_a(0, B->gridA, B->sys, B->itemsA, B->nA, B->active, B->stream));
  HIP_TRY(launch_batch_pass_b(0, B->gridB, B->sys, B->itemsB, B->nB, B->active, B->stream));
  HIP_TRY(launch_batch_average(0, B->gridV, B->sys, B->itemsV, B->nV, B->active, B->stream));
  return APC_OK;
}

void batch_count(apc_batch_s* B, int32_t T) {
  for (int32_t s = 0; s < B->count; ++s)
    if (B->h_active[s]) {
      B->plans[s]->iters += T;
      if (B->plans[s]->gemm) B->plans[s]->since_start += T;
    }
}

}  // namespace

extern "C" {

size_t apc_batch_workspace_bytes(const apc_plan* plans, int32_t count) {
  if (batch_check_plans(plans, count) != APC_OK) return 0;
  BatchPlanItems it;
  batch_items(plans, count, &it);
  return batch_layout(count, it).total;
}

apc_status apc_batch_create(apc_batch* out, const apc_plan* plans, int32_t count, void* workspace,
                            size_t ws_bytes) {
  if (!out) return fail(APC_EINVAL, "out is NULL");
  *out = nullptr;
  ST_TRY(batch_check_plans(plans, count));
  if (!workspace || reinterpret_cast<uintptr_t>(workspace) % kAlign != 0)
    return fail(APC_EINVAL, "workspace must be a 256-byte aligned device pointer");
  BatchPlanItems it;
  batch_items(plans, count, &it);
  const BatchLayout L = batch_layout(count, it);
  if (ws_bytes < L.total) return fail(APC_EINVAL, "workspace has %zu bytes, needs %zu", ws_bytes, L.total);
  if (it.A.size() > static_cast<size_t>(std::numeric_limits<int32_t>::max()))
    return fail(APC_EINVAL, "too many work items");
  apc_batch_s* B = new (std::nothrow) apc_batch_s();
  if (!B) return fail(APC_EINVAL, "out of host memory");
  std::unique_ptr<apc_batch_s> guard(B);
  B->plans.assign(plans, plans + count);
  B->count = count;
  B->stream = plans[0]->stream;
  B->ws = static_cast<char*>(workspace);
  B->sys = reinterpret_cast<BatchSys*>(B->ws + L.sys);
  B->itemsA = reinterpret_cast<int4*>(B->ws + L.A);
  B->itemsB = reinterpret_cast<int4*>(B->ws + L.B);
  B->itemsV = reinterpret_cast<int2*>(B->ws + L.V);
  B->active = reinterpret_cast<int32_t*>(B->ws + L.active);
  B->item_start = reinterpret_cast<int32_t*>(B->ws + L.start);
  B->partial = reinterpret_cast<double*>(B->ws + L.partial);
  B->relres = reinterpret_cast<double*>(B->ws + L.relres);
  B->nA = static_cast<int32_t>(it.A.size());
  B->nB = static_cast<int32_t>(it.B.size());
  B->nV = static_cast<int32_t>(it.V.size());
  B->fused = !it.F.empty();
  B->mixed = !it.gemm.empty();
  if (B->mixed) {
    B->gemm = reinterpret_cast<BatchGemm*>(B->ws + L.gemm);
    B->gemm_sys = it.gemm_sys;
    B->gemm_slot = it.gemm_slot;
    for (int v = 0; v < 2; ++v)
      for (int q = 0; q < 4; ++q) {
        B->itemsL[v][q] = reinterpret_cast<int4*>(B->ws + L.L[v][q]);
        B->nL[v][q] = static_cast<int32_t>(it.L[v][q].size());
      }
    B->itemsL0 = reinterpret_cast<int4*>(B->ws + L.L0);
    B->nL0 = static_cast<int32_t>(it.L0.size());
    const apc_plan_s* G0 = plans[it.gemm_sys[0]];
    B->nct = std::min(8, G0->kp / 16);
    B->anchor_every = G0->anchor_every;
    B->since = G0->since_start;
  }
  B->itemsF = reinterpret_cast<int4*>(B->ws + L.F);
  B->itemsW = reinterpret_cast<int2*>(B->ws + L.W);
  B->nF = static_cast<int32_t>(it.F.size());
  B->nW = static_cast<int32_t>(it.W.size());
  std::vector<BatchSys> hs(count);
  for (int32_t s = 0; s < count; ++s) {
    apc_plan_s* P = plans[s];
    BatchSys& d = hs[s];
    d.C = P->at<float>(P->L.C32);
    d.d = P->at<float>(P->L.dv);
    d.w = P->at<float>(P->L.w);
    d.x = P->x();
    d.xbar = P->xbar();
    d.off = P->doff();
    d.A = P->A;
    d.lda = P->lda;
    d.b = P->B;
    d.ldb = P->ldb;
    d.ldc = P->L.ldc;
    d.n = P->n;
    d.N = P->N;
    d.m = P->m;
    d.gamma = P->gamma;
    d.eta = P->eta;
    d.bnorm = P->bnorm;
    if (B->fused && !P->gemm) {
      // The plan's partial-row slice holds at least one FP64 row per 16 rows
      // of a block, so one FP32 row per tile of 128 or more rows fits.
      const int32_t* tl = reinterpret_cast<const int32_t*>(B->ws + L.T) + it.tile_at[s];
      const int32_t nt = it.tile_n[s];
      d.tiles = tl;
      d.tile_first = tl + 3 * nt;
      d.ntiles = nt;
      d.part = P->at<float>(P->L.fpart);
    }
  }
  B->h_active.assign(count, 1);
  hipStream_t st = B->stream;
  HIP_TRY(hipMemcpyAsync(B->sys, hs.data(), hs.size() * sizeof(BatchSys), hipMemcpyHostToDevice, st));
  HIP_TRY(hipMemcpyAsync(B->itemsA, it.A.data(), it.A.size() * sizeof(int4), hipMemcpyHostToDevice, st));
  HIP_TRY(hipMemcpyAsync(B->itemsB, it.B.data(), it.B.size() * sizeof(int4), hipMemcpyHostToDevice, st));
  HIP_TRY(hipMemcpyAsync(B->itemsV, it.V.data(), it.V.size() * sizeof(int2), hipMemcpyHostToDevice, st));
  if (B->fused) {
    HIP_TRY(hipMemcpyAsync(B->ws + L.T, it.tiles.data(), it.tiles.size() * 4, hipMemcpyHostToDevice, st));
    HIP_TRY(hipMemcpyAsync(B->itemsF, it.F.data(), it.F.size() * sizeof(int4), hipMemcpyHostToDevice, st));
    HIP_TRY(hipMemcpyAsync(B->itemsW, it.W.data(), it.W.size() * sizeof(int2), hipMemcpyHostToDevice, st));
  }
  if (B->mixed) {
    HIP_TRY(hipMemcpyAsync(B->gemm, it.gemm.data(), it.gemm.size() * sizeof(BatchGemm),
                           hipMemcpyHostToDevice, st));
    for (int v = 0; v < 2; ++v)
      for (int q = 0; q < 4; ++q)
        HIP_TRY(hipMemcpyAsync(B->itemsL[v][q], it.L[v][q].data(), it.L[v][q].size() * sizeof(int4),
                               hipMemcpyHostToDevice, st));
    HIP_TRY(hipMemcpyAsync(B->itemsL0, it.L0.data(), it.L0.size() * sizeof(int4), hipMemcpyHostToDevice, st));
  }
  HIP_TRY(hipMemcpyAsync(B->active, B->h_active.data(), count * 4, hipMemcpyHostToDevice, st));
  HIP_TRY(hipMemcpyAsync(B->item_start, it.start.data(), it.start.size() * 4, hipMemcpyHostToDevice, st));
  // Persistent grid: time the pass over the factors for a few workgroup
  // counts and use the fastest for every pass, unless the environment fixes it.
  if (const char* e = std::getenv("APC_BATCH_GRID")) {
    const int g = std::max(1, std::atoi(e));
    B->gridA = B->gridB = B->gridV = g;
  } else {
    hipEvent_t e0 = nullptr, e1 = nullptr;
    HIP_TRY(hipEventCreate(&e0));
    HIP_TRY(hipEventCreate(&e1));
    const int cands[5] = {256, 512, 1024, 2048, 4096};
    float best = 0.f;
    for (int c : cands) {
      // The pass that streams the factors (it writes only scratch: w, or the
      // partial rows).
      auto stream_pass = [&]() {
        if (B->mixed)
          return launch_batch_mixed(c, B->nct, B->sys, B->gemm, B->itemsL[0][0], B->nL[0][0],
                                    B->active, st);
        return B->fused ? launch_batch_fused(c, B->sys, B->itemsF, B->nF, B->active, st)
                        : launch_batch_pass_a(0, c, B->sys, B->itemsA, B->nA, B->active, st);
      };
      hipError_t err = stream_pass();
      if (err == hipSuccess) err = hipEventRecord(e0, st);
      for (int r = 0; err == hipSuccess && r < 3; ++r) err = stream_pass();
      if (err == hipSuccess) err = hipEventRecord(e1, st);
      if (err == hipSuccess) err = hipEventSynchronize(e1);
      float ms = 0.f;
      if (err == hipSuccess) err = hipEventElapsedTime(&ms, e0, e1);
      if (err != hipSuccess) {
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        return fail(APC_EHIP, "batch tuning failed: %s", hipGetErrorString(err));
      }
      if (c == cands[0] || ms < best) {
        best = ms;
        B->gridA = B->gridB = B->gridV = c;
      }
    }
    B->tuned_us = best * 1e3f / 3.f;
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
  }
  HIP_TRY(hipStreamSynchronize(st));
  *out = guard.release();
  return APC_OK;
}

apc_status apc_batch_iterate(apc_batch b, int32_t T) {
  if (!b || T < 0) return fail(APC_EINVAL, "bad argument");
  for (int32_t t = 0; t < T; ++t) ST_TRY(batch_update(b));
  batch_count(b, T);
  return APC_OK;
}

apc_status apc_batch_iterate_graph(apc_batch b, int32_t T) {
  if (!b || T < 0) return fail(APC_EINVAL, "bad argument");
  if (T == 0) return APC_OK;
  if (b->stream == nullptr) return fail(APC_EINVAL, "graph capture needs a non-default stream");
  const int32_t phase = b->mixed && b->anchor_every > 0
                            ? static_cast<int32_t>(b->since % b->anchor_every) : 0;
  const auto key = std::make_pair(T, phase);
  auto itg = b->graphs.find(key);
  if (itg == b->graphs.end()) {
    // Nothing runs during capture: the anchor cycle is put back after it.
    const int64_t since = b->since;
    hipGraph_t g = nullptr;
    HIP_TRY(hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal));
    apc_status st = APC_OK;
    for (int32_t t = 0; t < T && st == APC_OK; ++t) st = batch_update(b);
    hipError_t e = hipStreamEndCapture(b->stream, &g);
    b->since = since;
    if (st != APC_OK) {
      if (g) (void)hipGraphDestroy(g);
      return st;
    }
    HIP_TRY(e);
    hipGraphExec_t ex = nullptr;
    e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
    if (e != hipSuccess) {
      (void)hipGraphDestroy(g);
      HIP_TRY(e);
    }
    itg = b->graphs.emplace(key, std::make_pair(g, ex)).first;
  }
  HIP_TRY(hipGraphLaunch(itg->second.second, b->stream));
  b->since += T;
  batch_count(b, T);
  return APC_OK;
}

apc_status apc_batch_residuals(apc_batch b, double rtol, double* relres, int32_t* active) {
  if (!b) return fail(APC_EINVAL, "batch is NULL");
  HIP_TRY(launch_batch_resid(b->gridA, b->sys, b->itemsA, b->nA, b->active, b->partial, b->stream));
  // k-RHS plans: ||B - A X_bar||_F^2 in FP64 by the plan's own residual, into
  // the system's slot.
  for (size_t g = 0; g < b->gemm_sys.size(); ++g) {
    apc_plan_s* P = b->plans[b->gemm_sys[g]];
    double* Rb = P->at<double>(P->L.Rb);
    ST_TRY(gemm_residual(P, P->xbar(), Rb));
    HIP_TRY(launch_sumsq(Rb, static_cast<int64_t>(P->k) * P->N, P->at<double>(P->L.ssq), b->stream));
    HIP_TRY(launch_sum_partials(P->at<double>(P->L.ssq), sumsq_parts(), b->partial + b->gemm_slot[g],
                                b->stream));
  }
  HIP_TRY(launch_batch_check(b->sys, b->count, b->item_start, b->partial, rtol, b->active,
                             b->relres, b->stream));
  std::vector<double> rr(b->count);
  HIP_TRY(hipMemcpyAsync(rr.data(), b->relres, b->count * 8, hipMemcpyDeviceToHost, b->stream));
  HIP_TRY(hipMemcpyAsync(b->h_active.data(), b->active, b->count * 4, hipMemcpyDeviceToHost, b->stream));
  HIP_TRY(hipStreamSynchronize(b->stream));
  if (relres) std::copy(rr.begin(), rr.end(), relres);
  if (active) std::copy(b->h_active.begin(), b->h_active.end(), active);
  return APC_OK;
}

apc_status apc_batch_activate(apc_batch b) {
  if (!b) return fail(APC_EINVAL, "batch is NULL");
  b->h_active.assign(b->count, 1);
  HIP_TRY(hipMemcpyAsync(b->active, b->h_active.data(), b->count * 4, hipMemcpyHostToDevice, b->stream));
  HIP_TRY(hipStreamSynchronize(b->stream));
  return APC_OK;
}

apc_status apc_batch_solve(apc_batch b, double rtol, int32_t max_iters, int32_t check_every,
                           int32_t use_graph, int32_t* iters_out, double* relres_out) {
  if (!b || max_iters < 0 || check_every < 1 || !(rtol >= 0)) return fail(APC_EINVAL, "bad argument");
  // Every system is checked afresh: a flag left clear by an earlier check with
  // another tolerance says nothing about this one.
  b->h_active.assign(b->count, 1);
  HIP_TRY(hipMemcpyAsync(b->active, b->h_active.data(), b->count * 4, hipMemcpyHostToDevice, b->stream));
  std::vector<int64_t> start(b->count);
  for (int32_t s = 0; s < b->count; ++s) start[s] = b->plans[s]->iters;
  std::vector<double> rr(b->count, 0.0);
  int32_t done = 0;
  for (;;) {
    ST_TRY(apc_batch_residuals(b, rtol, rr.data(), nullptr));
    int32_t left = 0;
    for (int32_t s = 0; s < b->count; ++s) left += b->h_active[s];
    if (left == 0 || done >= max_iters) break;
    const int32_t T = std::min(check_every, max_iters - done);
    if (use_graph) ST_TRY(apc_batch_iterate_graph(b, T));
    else ST_TRY(apc_batch_iterate(b, T));
    done += T;
  }
  for (int32_t s = 0; s < b->count; ++s) {
    if (iters_out) iters_out[s] = static_cast<int32_t>(b->plans[s]->iters - start[s]);
    if (relres_out) relres_out[s] = rr[s];
  }
  for (int32_t s = 0; s < b->count; ++s)
    if (!std::isfinite(rr[s]))
      return fail(APC_EDIVERGED, "system %d: residual became non-finite", s);
  for (int32_t s = 0; s < b->count; ++s)
    if (rr[s] > rtol)
      return fail(APC_ENOCONV, "system %d did not reach %g in %d updates (relres %g)", s, rtol,
                  max_iters, rr[s]);
  return APC_OK;
}

apc_status apc_batch_get_launch(apc_batch b, int32_t* grid, int32_t* items_a, int32_t* items_b,
                                int32_t* items_avg, float* tuned_us) {
  if (!b) return fail(APC_EINVAL, "batch is NULL");
  if (grid) *grid = b->gridA;
  if (b->mixed) {
    // Items of the launches of an ordinary update: pass A with the k = 1
    // single pass, pass B, and the split sums with the k = 1 combine.
    if (items_a) *items_a = b->nL[0][0];
    if (items_b) *items_b = b->nL[0][2];
    if (items_avg) *items_avg = b->nL[0][1];
  } else {
    if (items_a) *items_a = b->fused ? b->nF : b->nA;
    if (items_b) *items_b = b->fused ? 0 : b->nB;
    if (items_avg) *items_avg = b->fused ? b->nW : b->nV;
  }
  if (tuned_us) *tuned_us = b->tuned_us;
  return APC_OK;
}

void apc_batch_destroy(apc_batch b) {
  if (!b) return;
  (void)hipStreamSynchronize(b->stream);  // no captured graph may still be running
  for (auto& kv : b->graphs) {
    (void)hipGraphExecDestroy(kv.second.second);
    (void)hipGraphDestroy(kv.second.first);
  }
  delete b;
}

}  // extern "C"

// ------------------------------------------------------------------ heavy-ball comparison

// D-HBM (Sec. 4.3) on the plan's row blocks, plain or on Sec. 6's
// preconditioned blocks (realised as [Q_i^T, c_i], which has the same
// gradient).  The object keeps its own x, z and scratch; the plan's iterates
// are not touched (its Lanczos scratch is reused at creation only).
struct apc_hbm_s {
  apc_plan_s* P = nullptr;
  int32_t kind = 0;
  char* ws = nullptr;
  double* x = nullptr;      // ldc
  double* z = nullptr;      // ldc
  double* Y = nullptr;      // m x ldc per-block sums
  double* w = nullptr;      // kMaxSplit x N row-pass partials
  void* C = nullptr;        // the streamed matrix (plan's factor, or the copy of A)
  const double* d = nullptr;  // per-row right-hand side (c or b)
  double alpha = 0, beta = 0, lam_min = NAN, lam_max = NAN, rho = NAN;
  int lanczos_steps = 0;
  int64_t iters = 0;
};

namespace {

struct HbmLayout {
  size_t x, z, Y, w, A, b, total;
};

HbmLayout hbm_layout(const apc_plan_s* P, int32_t kind) {
  HbmLayout H{};
  size_t cur = 0;
  auto take = [&](int64_t bytes) {
    const size_t at = cur;
    cur += static_cast<size_t>(round_up(std::max<int64_t>(bytes, 1), kAlign));
    return at;
  };
  const int64_t ldc = P->L.ldc, d = sizeof(double);
  H.x = take(ldc * d);
  H.z = take(ldc * d);
  H.Y = take(static_cast<int64_t>(P->m) * ldc * d);
  H.w = take(static_cast<int64_t>(kMaxSplit) * P->N * d);
  const int64_t sq = P->prec == APC_F32 ? 4 : 8;
  H.A = take(kind == APC_HBM_PLAIN ? P->N * ldc * sq : 0);
  H.b = take(kind == APC_HBM_PLAIN ? P->N * d : 0);
  H.total = cur;
  return H;
}

apc_status hbm_check(const apc_plan_s* P, int32_t kind) {
  if (!P) return fail(APC_EINVAL, "plan is NULL");
  if (kind != APC_HBM_PLAIN && kind != APC_HBM_PRECONDITIONED)
    return fail(APC_EINVAL, "unknown heavy-ball kind %d", kind);
  if (P->gemm || P->k != 1 || (P->prec != APC_F32 && P->prec != APC_F64))
    return fail(APC_EUNSUPPORTED, "the heavy-ball comparison takes k = 1 APC_F64 / APC_F32 plans "
                "in the per-block form");
  return APC_OK;
}

// x(0) = the plan's x_bar(0) = (1/m) sum_i Q_i c_i (Alg. 1 initialisation,
// recomputed from the stored c so the plan's state is not needed), z(0) = 0.
apc_status hbm_start(apc_hbm_s* H) {
  apc_plan_s* P = H->P;
  const Layout& L = P->L;
  ExpandArgs<double> e{P->C64(), L.ldc, P->doff(), P->m,
                       static_cast<int32_t>((L.ldc + expand_slab(8) - 1) / expand_slab(8)), P->N,
                       P->at<double>(L.ca), 1, 0, H->Y, L.ldc, 1.0, 0.0, 0};
  HIP_TRY(launch_expand_f64(e, P->stream));
  HIP_TRY(launch_combine_f64(H->Y, L.ldc, P->m, L.ldc, 1.0 / P->m, 0.0, H->x, nullptr, 0,
                             P->stream));
  HIP_TRY(launch_fill_u32(reinterpret_cast<unsigned*>(H->z), 2 * L.ldc, 0u, P->stream));
  H->iters = 0;
  return APC_OK;
}

// One update: w_r = C_r . x (row pass, FP64 accumulation, the plan's pass-A
// tiling and column splits), Y_i = sum_{r in block i} (w_r - d_r) C_r (block
// pass), then the heavy-ball step over the blocks' sums.
apc_status hbm_update(apc_hbm_s* H) {
  apc_plan_s* P = H->P;
  const Layout& L = P->L;
  const int32_t nt = P->tile_start[P->m];
  const bool f32 = P->prec == APC_F32;
  // Single pass (the plan's tiles): every tile's partial of sum_r (C_r x - d_r) C_r,
  // their sum (the gradient), then the heavy-ball step.
  const int cpt32 = fused_cpt(L.ldc, 4), cpt64 = fused_cpt(L.ldc, 8);
  if (P->fused && (f32 ? fused_shape_ok(4, 8, cpt32, 1) : cpt64 > 0)) {
    double* part = P->at<double>(L.fpart);
    const int32_t remap = P->xcd_remap == 1 ? 1 : 0;
    if (f32) {
      FusedArgs<float, double> a{static_cast<const float*>(H->C), L.ldc, P->n, P->tf(0),
                                 P->tf(1), P->tf(2), P->ntiles_f, H->x, 0, part, L.ldc, remap,
                                 H->d};
      HIP_TRY(launch_fused_f32x64(a, 1, P->stream));
    } else {
      FusedArgs<double, double> a{static_cast<const double*>(H->C), L.ldc, P->n, P->tf(0),
                                  P->tf(1), P->tf(2), P->ntiles_f, H->x, 0, part, L.ldc, remap,
                                  H->d};
      HIP_TRY(launch_fused_f64(a, cpt64 >= 16 ? 1 : 2, P->stream));
    }
    HIP_TRY(launch_fused_sum(part, L.ldc, P->ntiles_f, L.ldc, 1.0, H->Y, P->stream));
    HIP_TRY(launch_hbm_step(H->Y, L.ldc, 1, P->n, H->alpha, H->beta, H->x, H->z, P->stream));
    return APC_OK;
  }
  if (f32) {
    const float* C = static_cast<const float*>(H->C);
    RowdotArgs<float, double> a{C, L.ldc, P->ta(0), P->ta(1), P->ta(2), nt, 0, H->x, nullptr, 0,
                                nullptr, 0, H->w, P->N, P->nsplit, P->split_cols, P->xcd_remap,
                                P->passa_rows, 0, P->passa_nt};
    HIP_TRY(launch_rowdot_f32x64(a, P->stream));
    ExpandArgs<float> e{C, L.ldc, P->doff(), P->m,
                        static_cast<int32_t>((L.ldc + expand_slab(4) - 1) / expand_slab(4)), P->N,
                        H->w, P->nsplit, P->N, H->Y, L.ldc, 1.0, 0.0, 0, H->d};
    HIP_TRY(launch_expand_f32(e, P->stream));
  } else {
    const double* C = static_cast<const double*>(H->C);
    RowdotArgs<double, double> a{C, L.ldc, P->ta(0), P->ta(1), P->ta(2), nt, 0, H->x, nullptr, 0,
                                 nullptr, 0, H->w, P->N, P->nsplit, P->split_cols, P->xcd_remap,
                                 P->passa_rows, 0, P->passa_nt};
    HIP_TRY(launch_rowdot_f64(a, P->stream));
    ExpandArgs<double> e{C, L.ldc, P->doff(), P->m,
                         static_cast<int32_t>((L.ldc + expand_slab(8) - 1) / expand_slab(8)), P->N,
                         H->w, P->nsplit, P->N, H->Y, L.ldc, 1.0, 0.0, 0, H->d};
    HIP_TRY(launch_expand_f64(e, P->stream));
  }
  HIP_TRY(launch_hbm_step(H->Y, L.ldc, P->m, P->n, H->alpha, H->beta, H->x, H->z, P->stream));
  return APC_OK;
}

}  // namespace

extern "C" {

size_t apc_hbm_workspace_bytes(apc_plan p, int32_t kind) {
  if (hbm_check(p, kind) != APC_OK) return 0;
  return hbm_layout(p, kind).total;
}

apc_status apc_hbm_create(apc_hbm* out, apc_plan p, int32_t kind, double alpha, double beta,
                          void* workspace, size_t ws_bytes) {
  if (!out) return fail(APC_EINVAL, "out is NULL");
  *out = nullptr;
  ST_TRY(hbm_check(p, kind));
  if (!workspace || reinterpret_cast<uintptr_t>(workspace) % kAlign != 0)
    return fail(APC_EINVAL, "workspace must be a 256-byte aligned device pointer");
  const HbmLayout L = hbm_layout(p, kind);
  if (ws_bytes < L.total) return fail(APC_EINVAL, "workspace has %zu bytes, needs %zu", ws_bytes, L.total);
  const bool given = !std::isnan(alpha) && !std::isnan(beta);
  if (given && !(alpha > 0.0 && beta >= 0.0 && beta < 1.0 && std::isfinite(alpha)))
    return fail(APC_EINVAL, "need alpha > 0 and 0 <= beta < 1 (got %g, %g)", alpha, beta);
  std::unique_ptr<apc_hbm_s> H(new apc_hbm_s);
  H->P = p;
  H->kind = kind;
  H->ws = static_cast<char*>(workspace);
  H->x = reinterpret_cast<double*>(H->ws + L.x);
  H->z = reinterpret_cast<double*>(H->ws + L.z);
  H->Y = reinterpret_cast<double*>(H->ws + L.Y);
  H->w = reinterpret_cast<double*>(H->ws + L.w);
  const bool f32 = p->prec == APC_F32;
  if (kind == APC_HBM_PLAIN) {
    H->C = H->ws + L.A;
    double* b = reinterpret_cast<double*>(H->ws + L.b);
    HIP_TRY(launch_pad_cast(f32 ? 1 : 0, p->A, p->lda, p->N, p->n, H->C, p->L.ldc, p->stream));
    HIP_TRY(launch_copy_strided(p->B, p->ldb, b, 1, p->N, 1, p->stream));
    H->d = b;
  } else {
    H->C = f32 ? static_cast<void*>(p->at<float>(p->L.C32)) : static_cast<void*>(p->C64());
    H->d = p->at<double>(p->L.ca);
  }
  if (given) {
    H->alpha = alpha;
    H->beta = beta;
  } else {
    double lo = 0, hi = 0;
    if (kind == APC_HBM_PRECONDITIONED) {
      // sum_i Q_i Q_i^T = m X: the plan's enclosure of X's spectrum, or a new
      // one when the plan was given its parameters.
      if (std::isnan(p->mu_min) || std::isnan(p->mu_max)) {
        ST_TRY(lanczos(p, x_operator(p), 1.0, &lo, &hi, &H->lanczos_steps));
      } else {
        lo = p->mu_min;
        hi = p->mu_max;
      }
      lo *= p->m;
      hi *= p->m;
    } else {
      ST_TRY(lanczos(p, NormalOp{H->C, f32, 1.0}, std::numeric_limits<double>::infinity(), &lo,
                     &hi, &H->lanczos_steps));
    }
    const double a = std::sqrt(hi), c = std::sqrt(lo);
    H->alpha = 4.0 / ((a + c) * (a + c));
    H->rho = (a - c) / (a + c);
    H->beta = H->rho * H->rho;
    H->lam_min = lo;
    H->lam_max = hi;
  }
  ST_TRY(hbm_start(H.get()));
  HIP_TRY(hipStreamSynchronize(p->stream));
  *out = H.release();
  return APC_OK;
}

apc_status apc_hbm_iterate(apc_hbm h, int32_t T) {
  if (!h) return fail(APC_EINVAL, "heavy-ball run is NULL");
  if (T < 0) return fail(APC_EINVAL, "T must be >= 0");
  for (int32_t t = 0; t < T; ++t) ST_TRY(hbm_update(h));
  h->iters += T;
  return APC_OK;
}

apc_status apc_hbm_restart(apc_hbm h) {
  if (!h) return fail(APC_EINVAL, "heavy-ball run is NULL");
  return hbm_start(h);
}

apc_status apc_hbm_get_x(apc_hbm h, double* x, int64_t ldx) {
  if (!h || !x || ldx < 1) return fail(APC_EINVAL, "bad argument");
  HIP_TRY(launch_copy_strided(h->x, 1, x, ldx, h->P->n, 1, h->P->stream));
  return APC_OK;
}

apc_status apc_hbm_residual(apc_hbm h, double* relres) {
  if (!h || !relres) return fail(APC_EINVAL, "NULL argument");
  apc_plan_s* P = h->P;
  double* dst = P->at<double>(P->L.scal);
  ST_TRY(residual_norm2(P, h->x, dst));
  double r2 = 0;
  HIP_TRY(hipMemcpyAsync(&r2, dst, sizeof r2, hipMemcpyDeviceToHost, P->stream));
  HIP_TRY(hipStreamSynchronize(P->stream));
  *relres = P->bnorm > 0 ? std::sqrt(r2) / P->bnorm : std::sqrt(r2);
  return APC_OK;
}

apc_status apc_hbm_get_params(apc_hbm h, double* alpha, double* beta, double* lam_min,
                              double* lam_max, double* rho, int32_t* lanczos_steps,
                              int64_t* iters) {
  if (!h) return fail(APC_EINVAL, "heavy-ball run is NULL");
  if (alpha) *alpha = h->alpha;
  if (beta) *beta = h->beta;
  if (lam_min) *lam_min = h->lam_min;
  if (lam_max) *lam_max = h->lam_max;
  if (rho) *rho = h->rho;
  if (lanczos_steps) *lanczos_steps = h->lanczos_steps;
  if (iters) *iters = h->iters;
  return APC_OK;
}

void apc_hbm_destroy(apc_hbm h) { delete h; }

}  // extern "C"

// ------------------------------------------------------------------ helpers for other files

namespace apc {

apc_status report(apc_status st, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_last_error = buf;
  return st;
}

int plan_device(const apc_plan_s* p) { return p ? p->device : -1; }

}  // namespace apc
