"""The OpenMP build of the oracle (used only to time the threaded CPU
baseline) computes what the serial build computes, up to summation order."""

import numpy as np
import pytest

import oracle


def _poly(shape, seed):
    rng = np.random.default_rng(seed)
    n = int(np.prod(shape))
    C = np.zeros((4, 6, 6))
    for p in range(3):
        A = rng.standard_normal((6, 6))
        C[p] = A @ A.T + 6 * np.eye(6)
    phase = rng.integers(0, 4, n).astype(np.int32)  # phase 3 is a void
    return phase, C


@pytest.mark.skipif(not oracle.threaded_available(), reason="no OpenMP compiler")
@pytest.mark.parametrize("shape", [(6, 5, 4), (5, 7, 9), (4, 4, 3), (3, 4, 2)])
def test_threaded_build_matches_serial(shape):
    phase, C = _poly(shape, sum(shape))
    P1 = oracle.Problem(shape, phase, C)
    P4 = oracle.Problem(shape, phase, C, threads=4)
    x = np.random.default_rng(1).standard_normal((3, P1.n))
    y1, y4 = P1.apply(x), P4.apply(x)
    assert np.abs(y1 - y4).max() <= 1e-12 * np.abs(y1).max()
    assert np.array_equal(P1.precond(), P4.precond())
    e6 = [1e-3, 0, 0, 0, 5e-4, 0]
    r1 = P1.solve(e6, tol=1e-12, maxit=3000)
    r4 = P4.solve(e6, tol=1e-12, maxit=3000)
    assert r1["status"] == r4["status"] == oracle.CONVERGED
    assert abs(r1["iters"] - r4["iters"]) <= 2
    s1, _ = P1.stress(e6, r1["w"])
    s4, _ = P4.stress(e6, r4["w"])
    assert np.abs(s1 - s4).max() <= 1e-8 * np.abs(s1).max()
