import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

GOLDEN = os.path.join(ROOT, "tests", "golden")


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU")
    config.addinivalue_line("markers", "slow: takes more than a few seconds on the CPU")


def _ensure_c_libs():
    # the plain-C generator and oracle libraries build in a second with gcc;
    # build them only when nothing is built yet
    import oracle.solve as osv
    import workloads.grids as wg
    if not os.path.exists(wg._LIB_PATH):
        wg.build()
    if not os.path.exists(osv._LIB_PATH):
        osv.build()


_ensure_c_libs()


@pytest.fixture(scope="session")
def golden():
    import json

    def load(name):
        with open(os.path.join(GOLDEN, name)) as f:
            return json.load(f)
    return load
