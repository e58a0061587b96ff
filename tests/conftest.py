import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

GOLDEN = os.path.join(ROOT, "tests", "golden")


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs through the HIP library)")
    config.addinivalue_line("markers", "slow: long CPU test")


def read_table(name):
    """Parse a golden table file: returns (header dict, list of row token lists)."""
    header, rows = {}, []
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            tok = line.split()
            if tok[0] in ("n", "Q", "best"):
                header[tok[0]] = tok[1:]
            else:
                rows.append(tok)
    return header, rows


@pytest.fixture(scope="session")
def orc():
    import oracle
    oracle.build(force=False)
    return oracle


def check_fp32(orc, Q, got, E_star, idx_star=None):
    """Accept an fp32 answer only on the oracle's own rescoring of the returned state.

    Reading of the fp32 path (fixed point, then a float64 rescore of the
    returned state): the oracle's float64 energy of ``got.index`` must equal
    the reported energy (up to float64 summation order), lie within
    ``got.tol`` of the oracle minimum ``E_star``, and ``got.tol`` must meet
    the 1e-5 * sum|Q| bound.  A different index is accepted only as such a
    near-tie.
    """
    import numpy as np
    scale = float(np.abs(np.asarray(Q, dtype=np.float64)).sum())
    e = orc.energy(Q, got.index)
    assert abs(e - got.energy) <= 1e-9 * scale + 1e-12, (got, e)
    assert e <= E_star + got.tol, (got, e, E_star)
    assert abs(got.energy - E_star) <= got.tol, (got, E_star)
    assert got.tol <= 1e-5 * scale, (got.tol, scale)
    if idx_star is not None and got.index != idx_star:
        assert e - E_star <= got.tol


@pytest.fixture(scope="session", autouse=True)
def _torch_before_library(request):
    """Sessions that run GPU tests initialise torch's HIP runtime before any
    test loads the library: torch ships its own copy of the runtime, and that
    copy finds no device when it starts after the library's."""
    if any(item.get_closest_marker("gpu") for item in request.session.items):
        import torch
        if torch.cuda.is_available():
            torch.cuda.init()
    yield
