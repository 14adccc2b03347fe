"""Serving (continuous batching): served results against the CPU oracle, and
a request the library refuses in the middle of a mix."""

import dataclasses

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)


@pytest.fixture(scope="module")
def E():
    from paper_2602_07354_amd import elas3d
    elas3d.lib()
    return elas3d


def _rel(a, b):
    d = a - b
    return max(np.linalg.norm(d) / max(np.linalg.norm(b), 1e-300), np.abs(d).max() / max(np.abs(b).max(), 1e-300))


# serving-stream requests of edge 32 (1, 2 and 2 load cases): small enough for
# the oracle to solve every case to 1e-12
SEEDS = (971, 913, 930)


@pytest.mark.parametrize("engine", ["group", "streams"])
def test_served_results_match_oracle(E, orc, engine):
    """Every served request, mixed precision and FP64 side by side in one mix,
    solved to a true relative residual of 1e-12: each load case's voxel stress
    and displacement (mean over active nodes removed) within 1e-8 of the
    oracle's FP64 PCG solution (element-wise and normwise)."""
    from paper_2602_07354_amd import serve
    reqs = [serve.Request(k, serve.synth.serving_request(s), 1e-12,
                          E.PREC_FP64 if k == 2 else E.PREC_MIXED) for k, s in enumerate(SEEDS)]
    srv = (serve.GroupServer(max_concurrency=4, keep_fields=True) if engine == "group"
           else serve.Server(max_concurrency=4, keep_fields=True))
    try:
        res = serve.run_stream(reqs, srv)
    finally:
        srv.close()
    assert [r.rid for r in res] == [0, 1, 2]
    for req, r in zip(reqs, res):
        ms = req.micro
        say("case: served request", SEEDS[r.rid], ms.shape, ms.nrhs, "precision", req.precision, engine)
        assert r.status == E.OK and r.error is None and max(r.relres_true) <= 1e-12
        P = orc.Problem.from_micro(ms)
        active = np.any(np.abs(P.precond()).reshape(ms.n, 9) > 0, axis=1)
        for c in range(ms.nrhs):
            ro = P.solve(ms.strain[c], tol=1e-12)
            assert ro["status"] == orc.CONVERGED
            so, avg_o = P.stress(ms.strain[c], ro["w"])
            assert _rel(r.sigma[c], so) <= 1e-8
            assert np.allclose(r.sigma_avg[c], avg_o, rtol=1e-8, atol=1e-10 * np.abs(avg_o).max())
            w, wo = r.w[c][:, active], ro["w"][:, active]
            assert _rel(w - w.mean(axis=1, keepdims=True), wo - wo.mean(axis=1, keepdims=True)) <= 1e-8


@pytest.mark.parametrize("engine", ["group", "streams"])
def test_refused_request_does_not_disturb_the_mix(E, engine):
    """A request whose phase map holds an id out of range is refused by setup
    (EBADARG, before any device call): it comes back as an error result, its
    memory and slot are released, drain() returns, and the other requests'
    results are bit for bit those they have alone."""
    from paper_2602_07354_amd import serve
    good = [serve.Request(k, serve.synth.serving_request(s), 1e-8) for k, s in enumerate((913, 921))]
    bad_ms = serve.synth.serving_request(955)
    ph = bad_ms.phase.copy()
    ph[123] = bad_ms.nphase + 5
    bad = serve.Request(2, dataclasses.replace(bad_ms, phase=ph), 1e-8)
    alone = [serve.solve_one(r) for r in good]
    srv = serve.GroupServer(max_concurrency=4) if engine == "group" else serve.Server(max_concurrency=4)
    try:
        res = serve.run_stream([good[0], bad, good[1]], srv)
        again = serve.run_stream(good, srv)  # the server still serves after the refusal
    finally:
        srv.close()
    say("case: refused request in the mix,", engine, [r.status for r in res])
    assert [r.rid for r in res] == [0, 1, 2]
    assert res[2].status == E.EBADARG and res[2].error and "phase" in res[2].error.lower()
    for a, m, s in zip(alone, res[:2], again):
        assert a.status == m.status == s.status == E.OK
        assert a.iters == m.iters == s.iters
        assert np.array_equal(a.sigma_avg, m.sigma_avg) and np.array_equal(a.sigma_avg, s.sigma_avg)
