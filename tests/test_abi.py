"""Host-side checks of the C ABI: the library loads without a GPU and
exports every function include/sdq.h declares; the binding's validation
errors are raised before anything reaches the device.  CPU only."""
import ctypes
import os
import re

import pytest

from paper_2003_05286_amd import binding

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    text = open(os.path.join(ROOT, "include", "sdq.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(sdq_[a-z_]+)\s*\(", text)))


def test_header_declares_expected_calls():
    names = declared_functions()
    assert set(names) == set(binding.EXPORTS)


def test_library_exports_every_declared_symbol():
    lib = binding.load_library()
    for name in declared_functions():
        assert hasattr(lib, name), name
    assert binding.version().startswith("sdq ")


def test_null_context_is_rejected():
    lib = binding.load_library()
    assert lib.sdq_greens(None, None, 0, 0, None, None, None, None) == binding.SDQ_EINVAL
    assert lib.sdq_greens_noalloc(None, None, 0, 0, None, None, None, None) == binding.SDQ_EINVAL
    assert lib.sdq_sync(None) == binding.SDQ_EINVAL
    assert lib.sdq_last_error(None) == b"null context"
    out = ctypes.c_void_p()
    # an invalid device index never creates a context
    assert lib.sdq_create(ctypes.byref(out), -1, None) == binding.SDQ_EINVAL
    assert out.value is None


def test_instance_struct_layout():
    # matches sdq_instance: 4 int32, 3 pointers, 1 double
    assert ctypes.sizeof(binding._Instance) == 16 + 3 * 8 + 8
    assert binding._Instance.alpha.offset == 40


def test_bench_rejects_more_than_one_gpu():
    """The benchmark measures one GPU; asking for more exits with status 2
    and says so, before touching any device."""
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    r = subprocess.run([sys.executable, os.path.join(root, "bench.py"), "--gpus", "4"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU only" in r.stderr and r.stdout == ""
