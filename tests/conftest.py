import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HELPERS = os.path.join(ROOT, "tests", "helpers")


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: a longer statistical test")


@pytest.fixture(scope="session")
def orc():
    """The CPU oracle (built on first use if the shared library is missing)."""
    import oracle

    oracle.lib()
    return oracle


def _build_rocrand_helper() -> str:
    so = os.path.join(HELPERS, "librocrand_philox_ref.so")
    src = os.path.join(HELPERS, "rocrand_philox_ref.cpp")
    if not os.path.exists(so) or os.path.getmtime(so) < os.path.getmtime(src):
        subprocess.check_call(["hipcc", "-O1", "-fPIC", "-shared", "-o", so, src])
    return so


@pytest.fixture(scope="session")
def rocrand_philox():
    """Philox4x32-10 evaluated by rocRAND's engine (an independent implementation)."""
    import ctypes

    import numpy as np

    try:
        so = _build_rocrand_helper()
    except (OSError, subprocess.CalledProcessError) as exc:  # pragma: no cover
        pytest.skip(f"rocRAND helper could not be built: {exc}")
    h = ctypes.CDLL(so)

    def f(ctr, key):
        c = np.ascontiguousarray(ctr, dtype=np.uint32)
        k = np.ascontiguousarray(key, dtype=np.uint32)
        out = np.zeros(4, dtype=np.uint32)
        h.rr_philox4x32_10(c.ctypes.data_as(ctypes.c_void_p), k.ctypes.data_as(ctypes.c_void_p),
                           out.ctypes.data_as(ctypes.c_void_p))
        return out

    return f
