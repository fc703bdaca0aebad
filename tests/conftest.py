import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU")
    config.addinivalue_line("markers", "slow: long CPU test")


def _ensure_cpu_libs():
    # The gcc-built libraries (inputs and oracle) are cheap to build; build
    # them only when absent.  The HIP library is built by __graft_entry__.build().
    import synth
    import oracle
    for mod in (synth, oracle):
        so = mod._LIB_PATH
        if not os.path.exists(so):
            subprocess.check_call(mod.build_cmd())


_ensure_cpu_libs()


@pytest.fixture(scope="session")
def orc():
    import oracle
    return oracle.oracle()
