import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) and the built HIP library")
    config.addinivalue_line("markers", "slow: larger CPU oracle cases")


TINY = dict(cfg_id=90, coarse=(2, 2, 2), dense=(2, 2, 2), n_ao=8, nv=2, nc=2, n_aux=12, r_cut=None)
SMALL = dict(cfg_id=91, coarse=(2, 2, 2), dense=(3, 2, 2), n_ao=10, nv=2, nc=3, n_aux=16, r_cut=None)


@pytest.fixture(scope="session")
def tiny_cfg():
    return dict(TINY)


@pytest.fixture(scope="session")
def small_cfg():
    return dict(SMALL)
