import os
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

GOLDEN = os.path.join(ROOT, "tests", "golden")


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs the HIP library)")


def load_golden(name):
    """Stored eigenvalues (and residual/bound columns when present)."""
    path = os.path.join(GOLDEN, f"{name}_eig.txt")
    rows = [l.split() for l in open(path) if l.strip() and not l.startswith("#")]
    arr = np.array([[float(x) for x in r] for r in rows])
    return arr[:, 1], (arr[:, 2:] if arr.shape[1] > 2 else None)


@pytest.fixture(scope="session")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


_problem_cache = {}


@pytest.fixture(scope="session")
def oracle_problem():
    """(workload, miller, dense H or None, MatFreeH) per workload name, cached."""
    from oracle import pw, matfree
    from workloads import make_workload

    def get(name, dense=True):
        key = (name, dense)
        if key not in _problem_cache:
            w = make_workload(name)
            mil = pw.sphere(w.cell, w.kfrac, w.ecut)
            H = (pw.dense_hamiltonian(w.cell, w.kfrac, mil, w.vgrid, w.pos, w.lm, w.D)
                 if dense else None)
            mf = matfree.MatFreeH(w.cell, w.kfrac, mil, w.vgrid, w.pos, w.lm, w.D)
            _problem_cache[key] = (w, mil, H, mf)
        return _problem_cache[key]
    return get


def pytest_runtest_setup(item):
    # name the case before it touches the GPU, unbuffered, so that a run that
    # ends abruptly still says which test was running
    sys.__stderr__.write(f"[start] {item.nodeid}\n")
    sys.__stderr__.flush()
