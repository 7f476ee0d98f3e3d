"""symhss_factor_solve: factor then solve in one call.

With the factorisation pipelined during compress, the call runs the solve's
sweep up the levels while the top-level LU is still being computed, so its
result must equal that of symhss_factor followed by symhss_solve: the same
kernels on the same data, only overlapped (checked to 1e-13 relative, and
to the dense oracle at 1e-8).  Without pipelining, and for several
right-hand sides through device pointers, it is the two calls one after the
other.  A context factored this way accepts later solves.
"""

import numpy as np
import pytest

import workloads
from oracle import dense
from tests.gpu_common import make_solver, oracle_system, rel

pytestmark = pytest.mark.gpu


def _star(n=2048):
    # order of the top-level system above the blocked-substitution limit (512)
    return workloads.scaled_config(workloads.config2(), n, leaf=64)


@pytest.mark.parametrize("pipeline", [True, False])
def test_factor_solve_matches_factor_then_solve(pipeline):
    wl = _star()
    _, _, A, b = oracle_system(wl)
    out = []
    for fused in (False, True):
        s = make_solver(wl)
        s.configure(pipeline=pipeline)
        s.compress()
        if fused:
            x = s.factor_solve(b)
        else:
            s.factor()
            x = s.solve(b)
        out.append((x, s.stats()["root_size"]))
        if fused:
            # the context is factored: a plain solve gives the same result
            assert rel(s.solve(b), x) < 1e-13
    (x0, r0), (x1, r1) = out
    e = rel(x1, x0)
    ed = rel(x1, dense.solve_dense(A, b))
    print("pipeline", pipeline, "root order", r1, "fused vs separate", e, "vs dense", ed)
    assert r0 == r1
    assert e < 1e-13
    assert ed < 1e-8


def test_factor_solve_device_several_rhs():
    import torch
    wl = _star(1500)
    s = make_solver(wl)
    s.compress()
    n2 = 2 * s.n
    rng = np.random.default_rng(11)
    B = rng.standard_normal((n2, 3)) + 1j * rng.standard_normal((n2, 3))
    dev = torch.device("cuda:0")
    bd = torch.from_numpy(np.asfortranarray(B).T.copy()).to(dev)  # column-major 2N x 3 = row-major 3 x 2N
    xd = torch.zeros_like(bd)
    torch.cuda.synchronize()
    s.factor_solve_device(bd.data_ptr(), xd.data_ptr(), 3)
    torch.cuda.synchronize()
    X = xd.cpu().numpy().T
    X2 = s.solve(B)
    assert rel(X, X2) < 1e-13
