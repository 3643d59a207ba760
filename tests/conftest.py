import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU")


def gpu_available():
    try:
        import torch
        return torch.cuda.is_available()
    except Exception:
        return False


@pytest.fixture(scope="session")
def rocrand_ref(tmp_path_factory):
    """ctypes handle of a host build of rocRAND's Philox4x32-10 engine."""
    import ctypes
    import subprocess
    src = os.path.join(ROOT, "tests", "rocrand_ref", "rocrand_ref.cpp")
    hdr = "/opt/rocm/include/rocrand/rocrand_philox4x32_10.h"
    if not os.path.exists(hdr):
        pytest.skip("rocRAND headers not installed")
    out = str(tmp_path_factory.mktemp("rr") / "rr.so")
    subprocess.check_call(["g++", "-O1", "-shared", "-fPIC", "-D__HIP_PLATFORM_AMD__",
                           "-I/opt/rocm/include", src, "-o", out])
    lib = ctypes.CDLL(out)
    lib.rr_philox_next4.argtypes = [ctypes.c_ulonglong] * 3 + [ctypes.c_void_p]
    lib.rr_philox_next4.restype = None
    return lib
