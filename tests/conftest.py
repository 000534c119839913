import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def ensure_library():
    """Builds liblbm.so if it is missing (a fresh checkout holds sources only);
    the package refuses to import without it."""
    lib = os.path.join(ROOT, "paper_2009_13426_amd", "liblbm.so")
    if not os.path.exists(lib):
        import importlib.util
        spec = importlib.util.spec_from_file_location(
            "_lbm_build", os.path.join(ROOT, "paper_2009_13426_amd", "build.py"))
        m = importlib.util.module_from_spec(spec)
        spec.loader.exec_module(m)
        m.build()


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (HIP device) to run")
    config.addinivalue_line("markers", "slow: takes more than a few seconds on the CPU")


@pytest.fixture(scope="session")
def orc():
    import oracle
    from oracle import build
    build.build()          # always rebuild: the library is tiny and must match the source
    oracle._lib = None
    oracle.lib()
    return oracle
