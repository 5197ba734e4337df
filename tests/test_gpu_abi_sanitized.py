"""Every entry point of the C ABI driven from C++ (tests/abi_check.cpp) on
the device, with the library's host runtime built under AddressSanitizer,
UndefinedBehaviorSanitizer and LeakSanitizer (host code only): argument
checks, batch plans of mixed sizes (one-workgroup, n = 144 and gang
classes), graphs captured and replayed, checkpoint handles, profiling
tables, the autotune cache, the allocation-free entry point, the SVD
stabilizer, dense and complex slices, the UDTs and the Monte Carlo drivers,
then two contexts destroyed.  Any memory error, undefined behaviour or leak
in the runtime (outside the ROCm libraries' own, tests/lsan_rocm.supp), a
failing status or an inconsistent result ends the program with a nonzero
exit."""
import os
import subprocess

import pytest

from _gpu import say
from test_sanitizers import ABI_CHECK, abi_check_env

pytestmark = pytest.mark.gpu


def test_c_abi_under_host_sanitizers_on_the_device():
    assert os.path.exists(ABI_CHECK), "tests/_bin/sdq_abi_check is built by __graft_entry__.build()"
    say("[gpu] sdq_abi_check --require-gpu (ASan + UBSan + LSan host runtime, every entry point)")
    r = subprocess.run([ABI_CHECK, "--require-gpu"], env=abi_check_env(), capture_output=True, text=True,
                       timeout=280)
    out = r.stdout + r.stderr
    say(out[-600:])
    assert "AddressSanitizer" not in out and "runtime error:" not in out and "LeakSanitizer" not in out, out[-4000:]
    assert r.returncode == 0, out[-4000:]
    assert "checks passed on device 0" in out
