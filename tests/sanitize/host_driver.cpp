// Drives the host-side C++ of libapc through its C ABI without a GPU: argument
// validation, workspace sizing, the closed-form helpers and every error path
// that returns before device work.  Built with AddressSanitizer and
// UndefinedBehaviorSanitizer on the host code (tests/test_host_sanitizers.py);
// any report aborts the run.  Exit status 0 when every check held.
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <limits>
#include <vector>

#include "apc.h"

static int failures = 0;
#define CHECK(cond)                                                         \
  do {                                                                      \
    if (!(cond)) {                                                          \
      std::fprintf(stderr, "check failed at line %d: %s\n", __LINE__, #cond); \
      ++failures;                                                           \
    }                                                                       \
  } while (0)

int main() {
  const double nan = std::numeric_limits<double>::quiet_NaN();
  // Workspace sizing: valid, uneven, k-RHS, mixed precision; invalid offsets.
  const int64_t off_even[5] = {0, 64, 128, 192, 256};
  const int64_t off_uneven[4] = {0, 100, 101, 257};
  const int64_t off_bad[4] = {0, 100, 90, 257};
  CHECK(apc_workspace_bytes(256, 256, off_even, 4, 1, APC_F64) > 0);
  CHECK(apc_workspace_bytes(256, 200, off_even, 4, 1, APC_F32) > 0);
  CHECK(apc_workspace_bytes(257, 257, off_uneven, 3, 1, APC_F32) > 0);
  CHECK(apc_workspace_bytes(256, 256, off_even, 4, 37, APC_F32) > 0);
  CHECK(apc_workspace_bytes(256, 256, off_even, 4, 130, APC_F64) > 0);
  CHECK(apc_workspace_bytes(256, 256, off_even, 4, 8, APC_BF16_IR) > 0);
  CHECK(apc_workspace_bytes(256, 256, off_even, 4, 1, APC_F32 | APC_REDUCED_FORM) > 0);
  CHECK(apc_workspace_bytes(257, 257, off_bad, 3, 1, APC_F64) == 0);
  CHECK(apc_workspace_bytes(256, 256, nullptr, 4, 1, APC_F64) == 0);
  CHECK(apc_workspace_bytes(256, 32, off_even, 4, 1, APC_F64) == 0);   // p_i = 64 > n
  CHECK(apc_workspace_bytes(256, 256, off_even, 4, 0, APC_F64) == 0);  // k = 0
  CHECK(apc_workspace_bytes(256, 256, off_even, 4, 1, 99) == 0);       // precision
  CHECK(apc_workspace_bytes(256, 256, off_even, 0, 1, APC_F64) == 0);  // m = 0

  // apc_setup: every argument error is found on the host; with valid
  // arguments and no GPU it reports APC_ENODEV (or APC_EHIP), never crashes.
  std::vector<char> fake(1 << 20);
  void* ws = reinterpret_cast<void*>((reinterpret_cast<uintptr_t>(fake.data()) + 255) & ~uintptr_t(255));
  const double* A = reinterpret_cast<const double*>(ws);
  apc_plan p = reinterpret_cast<apc_plan>(0x1);
  CHECK(apc_setup(nullptr, A, 256, A, 1, 256, 256, off_even, 4, 1, APC_F64, nan, nan, ws, 1, nullptr) == APC_EINVAL);
  CHECK(apc_setup(&p, A, 256, A, 1, 256, 256, off_even, 4, 1, APC_F64, nan, nan, ws, 1, nullptr) == APC_EINVAL);
  CHECK(p == nullptr);
  CHECK(apc_setup(&p, nullptr, 256, A, 1, 256, 256, off_even, 4, 1, APC_F64, nan, nan, ws, size_t(1) << 40, nullptr) == APC_EINVAL);
  CHECK(apc_setup(&p, A, 100, A, 1, 256, 256, off_even, 4, 1, APC_F64, nan, nan, ws, size_t(1) << 40, nullptr) == APC_EINVAL);
  CHECK(apc_setup(&p, A, 256, A, 1, 256, 256, off_bad, 3, 1, APC_F64, nan, nan, ws, size_t(1) << 40, nullptr) == APC_EINVAL);
  CHECK(apc_setup(&p, A, 256, A, 1, 256, 256, off_even, 4, 1, APC_F64, 1.0, INFINITY, ws, size_t(1) << 40, nullptr) == APC_EINVAL);
  CHECK(apc_setup(&p, A, 256, A, 1, 256, 256, off_even, 4, 1, APC_F64, nan, nan,
                  static_cast<char*>(ws) + 8, size_t(1) << 40, nullptr) == APC_EINVAL);
  const apc_status st = apc_setup(&p, A, 256, A, 1, 256, 256, off_even, 4, 1, APC_F64, nan, nan,
                                  ws, size_t(1) << 40, nullptr);
  CHECK(st == APC_ENODEV || st == APC_EHIP);
  CHECK(p == nullptr);
  CHECK(std::strlen(apc_last_error()) > 0);

  // NULL plans everywhere.
  double d = 0;
  int32_t i32 = 0;
  CHECK(apc_iterate(nullptr, 1) == APC_EINVAL);
  CHECK(apc_iterate_graph(nullptr, 1) == APC_EINVAL);
  CHECK(apc_residual(nullptr, &d) == APC_EINVAL);
  CHECK(apc_solve(nullptr, 1e-6, 10, nullptr, 1, &i32, &d) == APC_EINVAL);
  CHECK(apc_get_xbar(nullptr, nullptr, 1) == APC_EINVAL);
  CHECK(apc_get_params(nullptr, &d, &d, &d, &d, &d) == APC_EINVAL);
  CHECK(apc_set_params(nullptr, 1.0, 1.0) == APC_EINVAL);
  CHECK(apc_restart(nullptr, nullptr, 1) == APC_EINVAL);
  CHECK(apc_backward_workspace_bytes(nullptr, 10, 2) == 0);
  CHECK(apc_backward(nullptr, nullptr, 1, 1, 1, nullptr, 1, &d, &d, nullptr, 0) == APC_EINVAL);
  CHECK(apc_backward_noalloc(nullptr, nullptr, 1, 1, 1, nullptr, 1, &d, &d) == APC_EINVAL);
  CHECK(apc_iterations(nullptr) == -1);
  apc_destroy(nullptr);
  CHECK(apc_batch_workspace_bytes(nullptr, 0) == 0);
  apc_batch b = reinterpret_cast<apc_batch>(0x1);
  CHECK(apc_batch_create(&b, nullptr, 0, ws, 1) != APC_OK);
  CHECK(b == nullptr);
  CHECK(apc_batch_iterate(nullptr, 1) == APC_EINVAL);
  apc_batch_destroy(nullptr);
  CHECK(apc_hbm_workspace_bytes(nullptr, 0) == 0);

  // Theorem 1's closed form and its argument checks.
  double g = 0, e = 0, r = 0;
  CHECK(apc_optimal_params(0.01, 0.5, &g, &e, &r) == APC_OK);
  CHECK(g > 1.0 && e > g && r > 0.0 && r < 1.0);
  // mu_max (eta gamma) = (1 + r)^2 and mu_min (eta gamma) = (1 - r)^2
  CHECK(std::fabs(0.5 * e * g - (1 + r) * (1 + r)) < 1e-12);
  CHECK(std::fabs(0.01 * e * g - (1 - r) * (1 - r)) < 1e-12);
  CHECK(apc_optimal_params(1.0, 1.0, &g, &e, &r) == APC_OK && std::fabs(g - 1) < 1e-12 && r < 1e-7);
  CHECK(apc_optimal_params(0.5, 0.1, &g, &e, &r) == APC_EINVAL);
  CHECK(apc_optimal_params(0.0, 0.5, &g, &e, &r) == APC_EINVAL);
  CHECK(apc_optimal_params(nan, 0.5, &g, &e, &r) == APC_EINVAL);

  // Tridiagonal extremes with residual bounds, on sizes 1 .. 300.
  for (int k : {1, 2, 3, 17, 64, 300}) {
    std::vector<double> a(k), be(k);
    for (int i = 0; i < k; ++i) {
      a[i] = 2.0 + std::sin(0.37 * i);
      be[i] = 0.5 + 0.25 * std::cos(0.11 * i);
    }
    double lo = 0, hi = 0, bl = 0, bh = 0;
    CHECK(apc_tridiag_extremes(a.data(), be.data(), k, 1, &lo, &hi, &bl, &bh) == APC_OK);
    CHECK(lo <= hi && bl >= 0 && bh >= 0);
    // Gershgorin: a_i in [1, 3] and |beta_i| <= 0.75 on each side put every
    // eigenvalue in [-0.5, 4.5].
    CHECK(lo >= -0.5 - 1e-12 && hi <= 4.5 + 1e-12);
  }
  CHECK(apc_tridiag_extremes(nullptr, nullptr, 3, 0, &g, &e, nullptr, nullptr) == APC_EINVAL);
  CHECK(apc_tridiag_extremes(&g, &e, 0, 0, &g, &e, nullptr, nullptr) == APC_EINVAL);

  std::printf("host driver: %d failed checks\n", failures);
  return failures == 0 ? 0 : 1;
}
