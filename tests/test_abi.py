"""The C-ABI library loads on the CPU host, exports every symbol its headers
declare, and rejects bad arguments before touching a device."""
import ctypes
import glob
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_functions():
    names = set()
    for h in glob.glob(os.path.join(ROOT, "include", "*.h")):
        src = open(h).read()
        src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
        src = re.sub(r"//[^\n]*", "", src)
        for m in re.finditer(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_]*\s*\**\s+\**([a-z_][a-z0-9_]*)\s*\(", src, flags=re.M):
            names.add(m.group(1))
    return sorted(names)


@pytest.fixture(scope="module")
def mcs():
    import paper_2008_08654_amd as m
    if not os.path.exists(m.LIB_PATH):
        pytest.fail("libmcs.so not built (run __graft_entry__.build())")
    return m


def test_headers_declare_the_core_api():
    names = _declared_functions()
    for n in ("cs_create", "cs_update", "cs_estimate_f2", "mersenne_divmod", "mersenne_div", "mersenne_mod",
              "cs_destroy", "cs_last_error"):
        assert n in names


def test_every_declared_symbol_is_exported(mcs):
    lib = mcs.lib()
    missing = [n for n in _declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


def test_argument_errors_without_device(mcs):
    lib = mcs.lib()
    h = ctypes.c_void_p()
    assert lib.cs_create(0, 1024, mcs.CS_P61, 1, ctypes.byref(h)) == mcs.CS_EINVAL
    assert b"rows" in lib.cs_last_error()
    assert lib.cs_create(5, 1000, mcs.CS_P61, 1, ctypes.byref(h)) == mcs.CS_EINVAL
    assert lib.cs_create(5, 1024, mcs.CS_P64_59, 1, ctypes.byref(h)) == mcs.CS_EINVAL
    assert lib.cs_create(5, 1 << 31, mcs.CS_P61, 1, ctypes.byref(h)) == mcs.CS_EINVAL
    assert lib.cs_create_ex(5, 1024, mcs.CS_P61, 1, 7, 4, ctypes.byref(h)) == mcs.CS_EINVAL
    assert lib.cs_create_ex(5, 1024, mcs.CS_P61, 1, 0, 3, ctypes.byref(h)) == mcs.CS_EINVAL
    assert lib.cs_update(None, None, mcs.CS_U32, None, mcs.CS_I64, 10, None) == mcs.CS_EINVAL
    assert lib.mersenne_divmod(9, None, 10, None, None, None) == mcs.CS_EINVAL
    lib.cs_destroy(None)


def test_package_has_no_cpu_fallback():
    """The binding never imports the oracle and has no compute of its own."""
    pkg = os.path.join(ROOT, "paper_2008_08654_amd")
    for path in glob.glob(os.path.join(pkg, "*.py")):
        src = open(path).read()
        assert "import oracle" not in src and "from oracle" not in src, path


def test_hip_error_status_mapping(mcs):
    """Out of memory is CS_ENOMEM; every other HIP error, such as the fault an earlier
    kernel leaves behind (which later runtime calls, allocations included, keep
    returning), is CS_EDEVICE rather than a misleading CS_ENOMEM."""
    f = mcs.lib().cs_status_from_hip_error
    assert f(0) == mcs.CS_OK
    assert f(2) == mcs.CS_ENOMEM          # hipErrorOutOfMemory
    assert f(1) == mcs.CS_EDEVICE         # hipErrorInvalidValue
    assert f(700) == mcs.CS_EDEVICE       # hipErrorIllegalAddress
    assert f(719) == mcs.CS_EDEVICE       # hipErrorLaunchFailure
