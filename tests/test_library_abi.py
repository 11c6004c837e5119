"""The C-ABI library loads, exports every declared entry point and rejects bad input (no GPU)."""

import ctypes as C
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "sbfem.h")
LIB = os.path.join(ROOT, "paper_2103_09100_amd", "libsbfem.so")


def declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(sbfem_[a-z_0-9]+)\s*\(", text)))


@pytest.fixture(scope="module")
def binding():
    if not os.path.exists(LIB):
        pytest.fail("libsbfem.so not built (python -m paper_2103_09100_amd.build)")
    from paper_2103_09100_amd import binding as b
    return b


def test_every_declared_symbol_is_exported(binding):
    lib = C.CDLL(LIB)
    names = declared()
    assert len(names) >= 12
    for n in names:
        assert hasattr(lib, n), n
    assert set(binding.EXPORTS) <= set(names)


def test_argument_validation_without_device(binding):
    lib = binding._lib
    h = C.c_void_p()
    # bad ndof is rejected before any device call
    nd = np.array([25], dtype=np.int32)
    K = np.zeros(25 * 25)
    m = np.ones(25)
    w = np.ones(1)
    st = lib.sbfem_upload_patterns(C.byref(h), 1, nd.ctypes.data, K.ctypes.data, m.ctypes.data,
                                   w.ctypes.data, None)
    assert st == binding.EINVAL and "ndof" in binding.last_error()
    st = lib.sbfem_upload_patterns(C.byref(h), 0, None, None, None, None, None)
    assert st == binding.EINVAL
    d = binding.MeshDesc()
    st = lib.sbfem_create_mesh(C.byref(h), None, C.byref(d), None)
    assert st == binding.EINVAL
    st = lib.sbfem_step_n(None, 1, None)
    assert st == binding.EINVAL
    st = lib.sbfem_read_state(None, 0, None, None, None)
    assert st == binding.EINVAL


def test_one_hip_runtime_per_process():
    """Importing the binding (before or after torch) maps exactly one HIP runtime."""
    import subprocess
    import sys
    code = ("import {first}\nimport {second}\n"
            "paths = set(l.split()[-1] for l in open('/proc/self/maps') if 'libamdhip64' in l)\n"
            "print(len(paths))\n")
    for first, second in (("paper_2103_09100_amd.binding", "torch"), ("torch", "paper_2103_09100_amd.binding")):
        out = subprocess.run([sys.executable, "-c", code.format(first=first, second=second)], cwd=ROOT,
                             capture_output=True, text=True, timeout=300)
        assert out.returncode == 0, out.stderr
        assert out.stdout.split()[-1] == "1", (first, second, out.stdout)


def test_allocator_hook_validation_without_device(binding):
    lib = binding._lib
    st = lib.sbfem_set_allocator(binding.ALLOC_FN(lambda n, u: None), binding.RELEASE_FN(), None)
    assert st == binding.EINVAL and "both" in binding.last_error()
    binding.set_allocator(lambda n: 0, lambda p: None)  # accepted; nothing allocated here
    binding.set_allocator(None, None)
