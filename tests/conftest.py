import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)
ORACLE_DIR = os.path.join(ROOT, "oracle")
if ORACLE_DIR not in sys.path:
    sys.path.insert(0, ORACLE_DIR)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU")
    config.addinivalue_line("markers", "slow: long-running CPU test")


def _ensure_oracle():
    lib = os.path.join(ORACLE_DIR, "liboracle.so")
    src = os.path.join(ORACLE_DIR, "oracle.c")
    hdr = os.path.join(ORACLE_DIR, "oracle.h")
    if (not os.path.exists(lib) or os.path.getmtime(lib) < os.path.getmtime(src)
            or os.path.getmtime(lib) < os.path.getmtime(hdr)):
        subprocess.run([sys.executable, os.path.join(ORACLE_DIR, "build.py")],
                       check=True)


_ensure_oracle()


@pytest.fixture(scope="session")
def O():
    import oracle as mod
    return mod


@pytest.fixture(scope="session")
def W():
    from paper_2401_10878_amd import workloads
    return workloads


@pytest.fixture(scope="session")
def H():
    from paper_2401_10878_amd import hlbm
    return hlbm
