"""AddressSanitizer + UndefinedBehaviorSanitizer on the host C++ layer (CPU only).

apc_host.cpp (and the allocation-free entry point's host side) is compiled with both
sanitizers on the host code only (each -fsanitize= after -Xarch_host), the kernel
sources as usual, and tests/sanitize/host_driver.cpp drives every host path that needs
no GPU: argument validation, workspace sizing, Theorem 1's closed form, the
tridiagonal helper, NULL plans and batches, and apc_setup failing cleanly without a
device.  Any sanitizer report aborts the driver (UBSan without recovery)."""

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1708_01413_amd", "csrc")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

SAN = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
       "-Xarch_host", "-fno-sanitize-recover=undefined", "-fno-omit-frame-pointer", "-g"]
COMMON = ["-O1", "-std=c++17", "-fPIC", "--offload-arch=gfx950",
          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
          "-I", os.path.join(ROOT, "include"), "-I", CSRC]


def _run(cmd):
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError(f"{' '.join(cmd)}\n{res.stdout}\n{res.stderr}")


@pytest.mark.skipif(not os.path.exists(HIPCC), reason="hipcc not available")
def test_host_layer_under_asan_and_ubsan(tmp_path):
    kernels = ["apc_kernels.hip", "apc_gemm.hip", "apc_batch.hip", "apc_noalloc.hip",
               "apc_resident.hip"]
    jobs = [[HIPCC, *COMMON, "-c", os.path.join(CSRC, k), "-o", str(tmp_path / (k + ".o"))]
            for k in kernels]
    jobs.append([HIPCC, *COMMON, *SAN, "-c", os.path.join(CSRC, "apc_host.cpp"),
                 "-o", str(tmp_path / "apc_host.o")])
    jobs.append([HIPCC, *COMMON, *SAN, "-c", os.path.join(ROOT, "tests", "sanitize", "host_driver.cpp"),
                 "-o", str(tmp_path / "driver.o")])
    with ThreadPoolExecutor(max_workers=len(jobs)) as ex:
        for f in [ex.submit(_run, j) for j in jobs]:
            f.result()
    exe = str(tmp_path / "host_driver")
    _run([HIPCC, "--offload-arch=gfx950", *SAN, str(tmp_path / "driver.o"),
          str(tmp_path / "apc_host.o"), *[str(tmp_path / (k + ".o")) for k in kernels], "-o", exe])
    env = dict(os.environ)
    # The HIP runtime keeps allocations until exit: leak checking is for our code's
    # own lifetime errors, which ASan reports as use-after-free / overflow anyway.
    env["ASAN_OPTIONS"] = "detect_leaks=0:abort_on_error=1"
    env["UBSAN_OPTIONS"] = "print_stacktrace=1:halt_on_error=1"
    env["HIP_VISIBLE_DEVICES"] = env.get("HIP_VISIBLE_DEVICES", "")
    res = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=300)
    sys.stdout.write(res.stdout)
    sys.stderr.write(res.stderr[-4000:])
    assert "ERROR: AddressSanitizer" not in res.stderr
    assert "runtime error" not in res.stderr
    assert res.returncode == 0, res.stderr[-2000:]
    assert "0 failed checks" in res.stdout
