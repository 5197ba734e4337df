"""The CPU oracle built with AddressSanitizer and UndefinedBehaviorSanitizer
(gcc), and a cross-section of its pins run against that build in a child
process: any out-of-bounds access, use after free, misaligned access,
signed overflow or other undefined behaviour in the oracle aborts the run.
Also the library's host runtime under the same sanitizers (the C-ABI driver
tests/abi_check.cpp, built with the library): here, without a device, the
paths that need none (a failing sdq_create, NULL contexts, the strings).
CPU only."""
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

# pins that together call every exported oracle routine
SUBSET = ("expk_generator or cpqr_properties or udt_reconstructs or chain_kinds or free_fermions "
          "or uniform_field or tdisp_boundaries or nonsymmetric or stabilization_interval or "
          "gradient_sum_rule or symmetric_slices_naive or jacobi_svd_factors or dense_slices_plain "
          "or complex_udt_matches or complex_udt_properties or complex_chain_of_real or "
          "complex_chain_conjugate or recompute or inv_sum_fails or rejects_bad_arguments")


def _lib(name):
    out = subprocess.run(["gcc", f"-print-file-name={name}"], capture_output=True, text=True).stdout.strip()
    return out if os.path.isabs(out) and os.path.exists(out) else None


@pytest.mark.skipif(shutil.which("gcc") is None or _lib("libasan.so") is None, reason="gcc with libasan needed")
def test_oracle_pins_under_asan_and_ubsan(tmp_path):
    pkg = tmp_path / "oracle"
    pkg.mkdir()
    for f in ("__init__.py", "sdq_oracle.h"):
        shutil.copy(os.path.join(ROOT, "oracle", f), pkg / f)
    subprocess.check_call(["gcc", "-O1", "-g", "-fno-omit-frame-pointer", "-std=c99", "-fPIC", "-shared",
                           "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
                           "-o", str(pkg / "liboracle_sdq.so"), os.path.join(ROOT, "oracle", "sdq_oracle.c"),
                           "-lm"])
    env = dict(os.environ)
    env["LD_PRELOAD"] = _lib("libasan.so")
    env["ASAN_OPTIONS"] = "detect_leaks=0:abort_on_error=1"
    env["UBSAN_OPTIONS"] = "halt_on_error=1:print_stacktrace=1"
    env["PYTHONPATH"] = f"{tmp_path}{os.pathsep}{ROOT}"
    r = subprocess.run([sys.executable, "-m", "pytest", os.path.join(ROOT, "tests", "test_oracle_pins.py"),
                        "-c", os.path.join(ROOT, "pytest.ini"), "-q", "-p", "no:cacheprovider", "-x",
                        "-k", SUBSET],
                       cwd=str(tmp_path), env=env, capture_output=True, text=True, timeout=900)
    out = r.stdout + r.stderr
    assert "AddressSanitizer" not in out and "runtime error:" not in out, out[-4000:]
    assert r.returncode == 0, out[-4000:]
    assert " passed" in out
    # the sanitized build was the one loaded
    chk = subprocess.run([sys.executable, "-c", "import oracle; print(oracle.__file__)"], cwd=str(tmp_path),
                         env=env, capture_output=True, text=True)
    assert str(tmp_path) in chk.stdout


ABI_CHECK = os.path.join(ROOT, "tests", "_bin", "sdq_abi_check")


def abi_check_env():
    env = dict(os.environ)
    env["ASAN_OPTIONS"] = "detect_leaks=1:abort_on_error=1"
    env["UBSAN_OPTIONS"] = "halt_on_error=1:print_stacktrace=1"
    env["LSAN_OPTIONS"] = "suppressions=" + os.path.join(ROOT, "tests", "lsan_rocm.supp")
    return env


def _abi_check_binary():
    if os.path.exists(ABI_CHECK):
        return ABI_CHECK
    from paper_2003_05286_amd import build as B
    objs = [os.path.join(B.BUILD, f) for f in sorted(os.listdir(B.BUILD))] if os.path.isdir(B.BUILD) else []
    objs = [o for o in objs if o.endswith(".o") and "_san" not in os.path.basename(o)]
    if not any(os.path.basename(o) == "sdq_dispatch.o" for o in objs):
        pytest.skip("the library's objects are not built (run __graft_entry__.build())")
    return B.build_abi_check(objs)


@pytest.mark.skipif(shutil.which("g++") is None, reason="g++ needed")
def test_c_abi_host_runtime_under_asan_and_ubsan_without_a_device():
    exe = _abi_check_binary()
    r = subprocess.run([exe], env=abi_check_env(), capture_output=True, text=True, timeout=300)
    out = r.stdout + r.stderr
    assert "AddressSanitizer" not in out and "runtime error:" not in out and "LeakSanitizer" not in out, out[-4000:]
    assert r.returncode == 0, out[-4000:]
    assert "checks passed" in out, out[-2000:]
