"""Host code under AddressSanitizer with LeakSanitizer, and under UndefinedBehaviorSanitizer
(opt-in: FDLB_RUN_ASAN=1, a few minutes each).

The library is rebuilt with host-side instrumentation only (-Xarch_host -fsanitize=...; the
device code is not instrumented) and tests/asan/harness.c drives every host-only entry point:
quadrature of every order, seeded valid and invalid problem descriptions, batches, networks,
hybrid channels, tile descriptions and error messages.  No GPU call is made."""
import glob
import os
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

pytestmark = pytest.mark.skipif(os.environ.get("FDLB_RUN_ASAN") != "1",
                                reason="set FDLB_RUN_ASAN=1 to build the instrumented library (minutes)")


@pytest.mark.parametrize("san,runtime", [("address", "asan"), ("undefined", "ubsan_standalone")])
def test_host_entry_points_are_clean_under_sanitizers(tmp_path, san, runtime):
    csrc = os.path.join(ROOT, "paper_1308_0692_amd", "csrc")
    rt = glob.glob(f"/opt/rocm*/lib/llvm/lib/clang/*/lib/linux/libclang_rt.{runtime}-x86_64.so")
    assert rt, f"clang's {runtime} runtime not found"
    lib = str(tmp_path / "libfdlb_san.so")
    srcs = sorted(glob.glob(os.path.join(csrc, "*.cpp")) + glob.glob(os.path.join(csrc, "*.hip")))
    flags = ["-Xarch_host", f"-fsanitize={san}", "-Xarch_host", "-fno-sanitize-recover=all",
             "-Xarch_host", "-fno-omit-frame-pointer", "-shared-libsan"]
    subprocess.run(["hipcc", "-std=c++17", "-O1", "-g", "-fPIC", "-shared", "--offload-arch=gfx950",
                    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", *flags,
                    "-I", csrc, "-I", os.path.join(ROOT, "include"), "-o", lib, *srcs], check=True)
    exe = str(tmp_path / "harness")
    subprocess.run(["/opt/rocm/llvm/bin/clang", "-g", "-O1", f"-fsanitize={san}", "-fno-sanitize-recover=all",
                    "-shared-libsan", "-I", os.path.join(ROOT, "include"), "-o", exe,
                    os.path.join(ROOT, "tests", "asan", "harness.c"), "-L", str(tmp_path), "-lfdlb_san",
                    f"-Wl,-rpath,{tmp_path}", f"-Wl,-rpath,{os.path.dirname(rt[0])}", "-lm"], check=True)
    r = subprocess.run([exe], capture_output=True, text=True, timeout=600,
                       env=dict(os.environ, ASAN_OPTIONS="detect_leaks=1", UBSAN_OPTIONS="print_stacktrace=1"))
    assert r.returncode == 0, r.stdout + r.stderr
    assert "Sanitizer" not in r.stderr and "runtime error" not in r.stderr, r.stderr
    assert "host harness done, 0 problems" in r.stdout
