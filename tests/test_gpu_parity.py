"""GPU parity: the HIP path through the C-ABI against the CPU oracle on the
same seeded inputs.

Tolerances (FP64 everywhere):
* operator, load vector, preconditioner: element-wise, normwise relative
  1e-12 (both sides are exact formulas; they differ only in summation order
  and in the element evaluation: 2x2x2 Gauss on the oracle side, the modal
  split on the GPU side);
* solves to a true relative residual of 1e-12: displacement (mean over the
  nodes removed) and voxel stress, normwise relative <= 1e-8;
* iteration counts within 2 of the oracle's (same recursion, different
  rounding).
"""

import numpy as np
import pytest

from paper_2602_07354_amd import synth

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)


@pytest.fixture(scope="module")
def E():
    from paper_2602_07354_amd import elas3d
    elas3d.lib()
    return elas3d


def _rel(a, b):
    """The larger of the normwise relative error and the largest element
    error relative to the largest reference element, so that a localised
    error cannot hide in the norm of a large field."""
    a, b = np.asarray(a), np.asarray(b)
    nb, mb = np.linalg.norm(b), np.abs(b).max() if b.size else 0.0
    d = a - b
    return max(np.linalg.norm(d) / (nb if nb > 0 else 1.0),
               (np.abs(d).max() if d.size else 0.0) / (mb if mb > 0 else 1.0))


def _small_poly(shape, seed, porosity=0.02, grains=12):
    ms = synth.polycrystal(shape, grains, seed,
                           [dict(kind="sphere", fraction=porosity, median=1.5, sigma=0.3)],
                           np.array([[2e-4, -1e-4, 1e-3, 3e-4, -2e-4, 1e-4]]))
    return ms


SHAPES = [(4, 4, 4), (17, 19, 23), (33, 31, 20), (40, 40, 40)]


@pytest.mark.parametrize("shape", SHAPES)
def test_operator_load_precond_parity(E, orc, shape):
    say("case: operator/load/precond parity", shape)
    ms = _small_poly(shape, 100 + shape[0])
    P = orc.Problem.from_micro(ms)
    rng = np.random.default_rng(shape[0])
    x = rng.standard_normal((3, ms.n))
    with E.Context.from_micro(ms) as ctx:
        y = ctx.apply(x)
        assert _rel(y, P.apply(x)) <= 1e-12
        b = ctx.load(0)
        bo, _ = P.load(ms.strain[0])
        assert _rel(b, bo) <= 1e-12
        M = ctx.precond()
        Mo = P.precond()
        assert _rel(M, Mo) <= 1e-12
        assert np.array_equal(np.all(M == 0, axis=(1, 2)), np.all(Mo == 0, axis=(1, 2)))


@pytest.mark.parametrize("precond", [True, False])
def test_eshelby_solve_parity(E, orc, precond):
    say("case: eshelby 20^3 solve parity, precond =", precond)
    ms = synth.eshelby_inclusion(20)
    P = orc.Problem.from_micro(ms)
    ro = P.solve(ms.strain[0], tol=1e-12, preconditioned=precond)
    opts = {} if precond else {"preconditioner": E.PRECOND_NONE}
    with E.Context.from_micro(ms, **opts) as ctx:
        st, info = ctx.solve(1e-12, 10000)
        assert st == E.OK and info["relres_true"][0] <= 1e-12
        assert abs(info["iters"][0] - ro["iters"]) <= 2
        w = ctx.solution(0)
        out = ctx.stress(0)
    wo = ro["w"]
    assert _rel(w - w.mean(axis=1, keepdims=True), wo - wo.mean(axis=1, keepdims=True)) <= 1e-8
    so, avg_o = P.stress(ms.strain[0], wo)
    assert _rel(out["sigma"], so) <= 1e-8
    assert np.allclose(out["avg"], avg_o, rtol=1e-9, atol=1e-12)
    assert np.isclose(out["energy"], P.energy(ms.strain[0], wo), rtol=1e-9)


@pytest.mark.parametrize("shape", [(24, 20, 18), (32, 32, 32)])
def test_polycrystal_solve_parity(E, orc, shape):
    say("case: polycrystal solve parity", shape)
    ms = _small_poly(shape, 7 + shape[0], grains=20)
    P = orc.Problem.from_micro(ms)
    ro = P.solve(ms.strain[0], tol=1e-12)
    with E.Context.from_micro(ms) as ctx:
        st, info = ctx.solve(1e-12, 20000)
        assert st == E.OK and info["relres_true"][0] <= 1e-12
        assert abs(info["iters"][0] - ro["iters"]) <= 2
        w = ctx.solution(0)
        out = ctx.stress(0)
    so, _ = P.stress(ms.strain[0], ro["w"])
    assert _rel(out["sigma"], so) <= 1e-8
    active = np.any(np.abs(P.precond()).reshape(ms.n, 9) > 0, axis=1)
    d1 = w[:, active] - w[:, active].mean(axis=1, keepdims=True)
    d0 = ro["w"][:, active] - ro["w"][:, active].mean(axis=1, keepdims=True)
    assert _rel(d1, d0) <= 1e-8


def test_paper_criterion_matches_oracle(E, orc):
    say("case: paper criterion")
    ms = synth.eshelby_inclusion(16, radius=4.0)
    P = orc.Problem.from_micro(ms)
    ro = P.solve(ms.strain[0], tol=1e-6, mode=1)
    with E.Context.from_micro(ms, convergence=E.CONV_PAPER) as ctx:
        st, info = ctx.solve(1e-6, 10000)
    assert st == E.OK and abs(info["iters"][0] - ro["iters"]) <= 1
    assert info["relres_precond"][0] < 1e-6


def test_void_timing_case_parity(E, orc):
    """The paper's timing case (a void of radius 0.04 of the edge in an
    isotropic matrix, eps_33 = 1e-3) at 50^3: the solve to 1e-12 matches the
    oracle's stress and iteration count, zero stress in the void, and with the
    paper's criterion at 1e-8 the iteration count matches the oracle's."""
    say("case: void timing case at 50^3")
    ms = synth.workload("void500", scale=50)
    P = orc.Problem.from_micro(ms)
    ro = P.solve(ms.strain[0], tol=1e-12)
    rp = P.solve(ms.strain[0], tol=1e-8, mode=1)
    with E.Context.from_micro(ms) as ctx:
        st, info = ctx.solve(1e-12, 20000)
        assert st == E.OK and info["relres_true"][0] <= 1e-12
        assert abs(info["iters"][0] - ro["iters"]) <= 2
        sig = ctx.stress(0)["sigma"]
    so, _ = P.stress(ms.strain[0], ro["w"])
    assert _rel(sig, so) <= 1e-8
    assert np.all(sig[:, ms.phase == 1] == 0.0)
    with E.Context.from_micro(ms, convergence=E.CONV_PAPER) as ctx:
        st, info = ctx.solve(1e-8, 20000)
    assert st == E.OK and abs(info["iters"][0] - rp["iters"]) <= 1
    assert info["relres_precond"][0] < 1e-8


def test_config_poly100_metric_and_sampled_parity(E, orc):
    """100^3 polycrystal with 1 % pores, eps_xx = 1e-3, tol 1e-10: sampled
    node parity at full size plus properties that hold at any size."""
    say("case: poly100 full size")
    ms = synth.workload("poly100")
    P = orc.Problem.from_micro(ms)
    rng = np.random.default_rng(5)
    sel = rng.choice(ms.n, 200, replace=False)
    x = rng.standard_normal((3, ms.n))
    with E.Context.from_micro(ms) as ctx:
        y = ctx.apply(x)
        assert _rel(y[:, sel], P.apply_at(x, sel)) <= 1e-12
        b = ctx.load(0)
        assert _rel(b[:, sel], P.load_at(ms.strain[0], sel)) <= 1e-12
        assert _rel(ctx.precond()[sel], P.precond_at(sel)) <= 1e-12
        st, info = ctx.solve(1e-10, 20000)
        say("poly100 iterations", info["iters"][0], "relres", info["relres_true"][0])
        assert st == E.OK and info["relres_true"][0] <= 1e-10
        w = ctx.solution(0)
        out = ctx.stress(0)
        g = ctx.apply(w) + b
    # Hill-Mandel: 2 Pi = N E_hat.<sigma> + w.g
    eh = np.r_[ms.strain[0][:3], 2 * ms.strain[0][3:]]
    lhs = 2 * out["energy"]
    rhs = ms.n * eh @ out["avg"] + np.sum(w * g)
    assert abs(lhs - rhs) <= 1e-10 * abs(lhs)
    assert np.linalg.norm(g) <= 1e-10 * np.linalg.norm(b) * 1.01
    # stress vanishes in the pores
    void = ms.phase == ms.nphase - 1
    assert np.all(out["sigma"][:, void] == 0.0)


def test_config_poly500_bench_launch_sampled_parity(E, orc):
    """The benchmark's own configuration: poly500 generated on the device,
    phase ids device-resident, autotuned sweep geometry.  Sampled nodes of
    the operator, load and M^-1 against the oracle; the M^-1 dictionary's
    size; FP64 and mixed-precision solves to 1e-8 with properties that hold
    at any size (true residual, Hill-Mandel, zero stress in pores, the two
    precisions agreeing)."""
    import torch
    from paper_2602_07354_amd import generate
    say("case: poly500 in the benchmark's launch configuration")
    rec = synth.workload_recipe("poly500")
    dev = torch.device("cuda:0")
    phase = torch.empty(int(np.prod(rec["shape"])), dtype=torch.int32, device=dev)
    ms = generate.workload("poly500", phase=phase)
    torch.cuda.synchronize()
    host = synth.Microstructure(ms.shape, phase.cpu().numpy(), ms.C, ms.strain, ms.meta)
    P = orc.Problem.from_micro(host)
    rng = np.random.default_rng(500)
    sel = np.sort(rng.choice(host.n, 300, replace=False))
    eh = np.r_[ms.strain[0][:3], 2 * ms.strain[0][3:]]
    void = host.phase == host.nphase - 1
    avg = {}
    for prec in (E.PREC_FP64, E.PREC_MIXED):
        opts = E.options_init(inputs_on_device=1, autotune=1, device=0, precision=prec)
        h = E.setup(ms.shape, phase, ms.C, ms.strain[:1], opts)
        try:
            if prec == E.PREC_FP64:
                x = rng.standard_normal((3, host.n))
                y = np.empty_like(x)
                E.apply(h, x, y)
                assert _rel(y[:, sel], P.apply_at(x, sel)) <= 1e-12
                del x, y
                b = np.empty((3, host.n))
                E.get_load(h, 0, b)
                assert _rel(b[:, sel], P.load_at(ms.strain[0], sel)) <= 1e-12
                M = np.empty((6, host.n))
                E.get_precond(h, M)
                Mo = P.precond_at(sel)
                Ms = np.stack([M[q][sel] for q in (0, 5, 4, 5, 1, 3, 4, 3, 2)], axis=1).reshape(-1, 3, 3)
                assert _rel(Ms, Mo) <= 1e-12
                del M
            st, info = E.solve(h, 1e-8, 50000, 1)
            say("  ", "fp64" if prec == E.PREC_FP64 else "mixed", "iterations", info.iters[0],
                "relres", info.relres_true[0], "tile", list(info.op_tile))
            assert st == E.OK and info.relres_true[0] <= 1e-8
            assert tuple(info.op_tile[:2]) in E.TILE_SHAPES
            sig = np.empty((6, host.n))
            a6, en = np.empty(6), np.empty(1)
            assert E.lib().elas3d_stress(h, 0, sig.ctypes.data, a6.ctypes.data, None, en.ctypes.data) == 0
            assert np.all(sig[:, void] == 0.0)
            del sig
            avg[prec] = a6
            if prec == E.PREC_FP64:
                assert info.precond_rows == host.nphase + _boundary_nodes(host)
                w = np.empty((3, host.n))
                E.get_solution(h, 0, w)
                g = np.empty_like(w)
                E.apply(h, w, g)
                g += b
                assert np.linalg.norm(g) <= 1e-8 * np.linalg.norm(b) * 1.01
                # Hill-Mandel: 2 Pi = N E_hat.<sigma> + w.g
                lhs, rhs = 2 * en[0], host.n * eh @ a6 + np.sum(w * g)
                assert abs(lhs - rhs) <= 1e-9 * abs(lhs)
                del w, g, b
        finally:
            E.destroy(h)
    assert _rel(avg[E.PREC_MIXED], avg[E.PREC_FP64]) <= 1e-6


def test_config_poly800_capacity_sampled_parity(E, orc):
    """The 800^3 capacity point in the benchmark's launch configuration:
    sampled operator, load and M^-1 nodes against the oracle, the M^-1
    dictionary size, and after 20 iterations the residual recomputed from
    the returned w (A w + b) against the recursion's, which ties the
    deferred w updates to the operator at full size."""
    import torch
    from paper_2602_07354_amd import generate
    say("case: poly800 capacity point")
    rec = synth.workload_recipe("poly800")
    dev = torch.device("cuda:0")
    phase = torch.empty(int(np.prod(rec["shape"])), dtype=torch.int32, device=dev)
    ms = generate.workload("poly800", phase=phase)
    torch.cuda.synchronize()
    host = synth.Microstructure(ms.shape, phase.cpu().numpy(), ms.C, ms.strain, ms.meta)
    P = orc.Problem.from_micro(host)
    rng = np.random.default_rng(800)
    sel = np.sort(rng.choice(host.n, 200, replace=False))
    opts = E.options_init(inputs_on_device=1, autotune=1, device=0)
    h = E.setup(ms.shape, phase, ms.C, ms.strain[:1], opts)
    try:
        v = np.empty((3, host.n))
        x = rng.standard_normal((3, host.n))
        E.apply(h, x, v)
        assert _rel(v[:, sel], P.apply_at(x, sel)) <= 1e-12
        del x
        b = np.empty((3, host.n))
        E.get_load(h, 0, b)
        assert _rel(b[:, sel], P.load_at(ms.strain[0], sel)) <= 1e-12
        M = np.empty((6, host.n))
        E.get_precond(h, M)
        Ms = np.stack([M[q][sel] for q in (0, 5, 4, 5, 1, 3, 4, 3, 2)], axis=1).reshape(-1, 3, 3)
        del M
        assert _rel(Ms, P.precond_at(sel)) <= 1e-12
        st, info = E.solve(h, 1e-30, 20, 1)
        say("   20 iterations, recursive rel-res", info.relres_recursive[0], "tile", list(info.op_tile))
        assert st == E.NOT_CONVERGED and info.iters[0] == 20
        assert info.precond_rows == host.nphase + _boundary_nodes(host)
        E.get_solution(h, 0, v)
        g = np.empty_like(v)
        E.apply(h, v, g)
        g += b
        rel = np.linalg.norm(g) / np.linalg.norm(b)
        assert abs(rel - info.relres_recursive[0]) <= 1e-6 * info.relres_recursive[0]
    finally:
        E.destroy(h)


def test_edge_cases(E, orc):
    say("case: edge cases")
    # the smallest grids (2 nodes in a dimension: both neighbours are the same
    # node through the periodic wrap) against the oracle
    for shape in [(2, 3, 2), (2, 2, 2), (3, 2, 5)]:
        say("  grid", shape)
        ms2 = _small_poly(shape, 31 + shape[2], porosity=0.0, grains=3)
        P2 = orc.Problem.from_micro(ms2)
        ro = P2.solve(ms2.strain[0], tol=1e-12)
        with E.Context.from_micro(ms2) as ctx:
            st, info = ctx.solve(1e-12, 1000)
            assert st == E.OK and abs(info["iters"][0] - ro["iters"]) <= 2
            so, _ = P2.stress(ms2.strain[0], ro["w"])
            assert _rel(ctx.stress(0)["sigma"], so) <= 1e-8
            x = np.random.default_rng(1).standard_normal((3, ms2.n))
            assert _rel(ctx.apply(x), P2.apply(x)) <= 1e-12
    iso = synth.isotropic_stiffness(200, .3)
    C = np.stack([iso, np.zeros((6, 6))])
    strain = np.array([[1e-3, 0, 0, 0, 0, 0]])
    # all void: nothing to solve
    with E.Context((5, 4, 3), np.ones(60, np.int32), C, strain) as ctx:
        st, info = ctx.solve(1e-10, 100)
        assert st == E.OK and info["iters"][0] == 0
        assert np.all(ctx.stress(0)["sigma"] == 0)
    # homogeneous: exact uniform strain, zero iterations
    with E.Context((6, 5, 4), np.zeros(120, np.int32), C, strain) as ctx:
        st, info = ctx.solve(1e-10, 100)
        assert st == E.OK and info["iters"][0] == 0
        assert np.allclose(ctx.stress(0)["sigma"], (iso @ [1e-3, 0, 0, 0, 0, 0])[:, None], rtol=1e-13)
    # one solid voxel in a void box: floppy cluster, still a consistent solve
    ph = np.ones(64, np.int32)
    ph[21] = 0
    with E.Context((4, 4, 4), ph, C, strain) as ctx:
        st, info = ctx.solve(1e-10, 100)
        assert st == E.OK
        s = ctx.stress(0)["sigma"]
        assert np.abs(s).max() <= 1e-9 * np.abs(iso).max() * 1e-3
    # maxit = 1 -> not converged, outputs still valid
    ms = synth.eshelby_inclusion(12, radius=3.0)
    with E.Context.from_micro(ms) as ctx:
        st, info = ctx.solve(1e-10, 1)
        assert st == E.NOT_CONVERGED and info["iters"][0] == 1
        ctx.stress(0)
    # maxit = 0: no iteration, not converged, outputs valid
    with E.Context.from_micro(ms) as ctx:
        st, info = ctx.solve(1e-10, 0)
        assert st == E.NOT_CONVERGED and info["iters"][0] == 0
        ctx.stress(0)
    # stress before solve is an ordering error
    with E.Context.from_micro(ms) as ctx:
        with pytest.raises(E.Elas3dError) as ei:
            ctx.stress(0)
        assert ei.value.code == E.EORDER
    # tiny memory budget
    with pytest.raises(E.Elas3dError) as ei:
        E.Context.from_micro(ms, hbm_budget_bytes=1e5)
    assert ei.value.code == E.ENOMEM


def _boundary_nodes(ms):
    """Nodes whose eight voxels (i-a, j-b, k-c), a, b, c in {0, 1}, do not all
    have one phase (periodic), counted on the host."""
    nx, ny, nz = ms.shape
    p = ms.phase.reshape(nz, ny, nx)
    same = np.ones(p.shape, dtype=bool)
    for c in (0, 1):
        for b in (0, 1):
            for a in (0, 1):
                same &= np.roll(p, (c, b, a), axis=(0, 1, 2)) == p
    return int((~same).sum())


@pytest.mark.parametrize("shape", [(17, 19, 23), (2, 3, 2), (40, 40, 40)])
def test_precond_dictionary_rows(E, orc, shape):
    """M^-1 is stored as one row per phase and one per phase-boundary node;
    its rows expand to the oracle's per-node blocks (also for plain CG)."""
    say("case: M^-1 dictionary", shape)
    ms = _small_poly(shape, 53, grains=9)
    P = orc.Problem.from_micro(ms)
    for cg in (False, True):
        kw = dict(preconditioner=E.PRECOND_NONE) if cg else {}
        with E.Context.from_micro(ms, **kw) as ctx:
            st, info = ctx.solve(1e-6, 5)
            assert info["precond_rows"] == ms.nphase + _boundary_nodes(ms)
            M = ctx.precond()
        Mo = P.precond(identity=cg)
        assert _rel(M, Mo) <= (0.0 if cg else 1e-12)
        assert np.array_equal(np.all(M == 0, axis=(1, 2)), np.all(Mo == 0, axis=(1, 2)))


def test_runs_cut_after_k_iterations_match_oracle_iterates(E, orc):
    """w owes the last step or two of a run until a direction sweep or the
    end of the run pays them; after exactly k iterations (k = 1..5 covers a
    run ending with one and with two owed steps, after a paying sweep and
    not) the iterate equals the oracle's k-th PCG iterate, for a single case
    and for each case of a batched run."""
    say("case: iterates after k iterations")
    ms = _small_poly((17, 19, 23), 29)
    ms2 = synth.polycrystal((17, 19, 23), 12, 29, [dict(kind="sphere", fraction=0.02, median=1.5, sigma=0.3)],
                            synth.unit_load_cases()[[2, 4]])
    P = orc.Problem.from_micro(ms)
    P2 = orc.Problem.from_micro(ms2)
    for k in range(1, 6):
        ro = P.solve(ms.strain[0], tol=1e-30, maxit=k)
        assert ro["iters"] == k
        with E.Context.from_micro(ms) as ctx:
            st, info = ctx.solve(1e-30, k)
            assert st == E.NOT_CONVERGED and info["iters"][0] == k
            assert _rel(ctx.solution(0), ro["w"]) <= 1e-11, k
        with E.Context.from_micro(ms2, batched=1) as ctx:
            st, info = ctx.solve(1e-30, k)
            for r in range(2):
                assert info["iters"][r] == k
                ro2 = P2.solve(ms2.strain[r], tol=1e-30, maxit=k)
                assert _rel(ctx.solution(r), ro2["w"]) <= 1e-11, (k, r)


def test_deterministic_and_device_inputs(E):
    say("case: determinism and device-resident inputs")
    import torch
    ms = _small_poly((20, 18, 16), 3)
    with E.Context.from_micro(ms) as c1:
        c1.solve(1e-10, 5000)
        w1 = c1.solution(0)
    with E.Context.from_micro(ms) as c2:
        c2.solve(1e-10, 5000)
        w2 = c2.solution(0)
    assert np.array_equal(w1, w2)
    dev = torch.device("cuda:0")
    ph = torch.from_numpy(ms.phase).to(dev)
    w3 = torch.empty((3, ms.n), dtype=torch.float64, device=dev)
    opts = E.options_init(inputs_on_device=1, outputs_on_device=1)
    h = E.setup(ms.shape, ph, ms.C, ms.strain, opts)
    try:
        st, info = E.solve(h, 1e-10, 5000)
        E.get_solution(h, 0, w3)
        torch.cuda.synchronize()
    finally:
        E.destroy(h)
    assert np.array_equal(w3.cpu().numpy(), w1)
    bad = ph.clone()
    bad[7] = ms.nphase
    with pytest.raises(E.Elas3dError) as ei:
        E.setup(ms.shape, bad, ms.C, ms.strain, opts)
    assert ei.value.code == E.EBADARG


@pytest.mark.parametrize("case", ["eshelby", "poly"])
def test_mixed_precision_refinement_matches_oracle(E, orc, case):
    """FP32 inner PCG inside FP64 refinement, driven to a true FP64 residual of
    1e-12: displacement and stress match the FP64 oracle to the FP64 bar."""
    say("case: mixed precision", case)
    ms = synth.eshelby_inclusion(20) if case == "eshelby" else _small_poly((28, 24, 20), 41, grains=16)
    P = orc.Problem.from_micro(ms)
    ro = P.solve(ms.strain[0], tol=1e-12)
    with E.Context.from_micro(ms, precision=E.PREC_MIXED) as ctx:
        st, info = ctx.solve(1e-12, 20000)
        say("mixed", info["iters"][0], "inner iterations,", info["restarts"][0], "cycles, fallback",
            info["fp64_fallback"][0], "oracle", ro["iters"])
        assert st == E.OK and info["relres_true"][0] <= 1e-12
        w = ctx.solution(0)
        out = ctx.stress(0)
    so, _ = P.stress(ms.strain[0], ro["w"])
    assert _rel(out["sigma"], so) <= 1e-8
    active = np.any(np.abs(P.precond()).reshape(ms.n, 9) > 0, axis=1)
    d1 = w[:, active] - w[:, active].mean(axis=1, keepdims=True)
    d0 = ro["w"][:, active] - ro["w"][:, active].mean(axis=1, keepdims=True)
    assert _rel(d1, d0) <= 1e-8


def test_mixed_precision_metric_tolerance_poly100(E):
    """Mixed precision at the metric tolerance on the 100^3 polycrystal: the
    FP64 true residual meets 1e-8 and the stress agrees with the FP64 solve."""
    say("case: mixed precision poly100")
    ms = synth.workload("poly100")
    with E.Context.from_micro(ms) as c64:
        st, i64 = c64.solve(1e-10, 20000)
        s64 = c64.stress(0)
    with E.Context.from_micro(ms, precision=E.PREC_MIXED) as c32:
        st, i32 = c32.solve(1e-8, 20000)
        s32 = c32.stress(0)
    say("fp64 iters", i64["iters"][0], "mixed iters", i32["iters"][0], "cycles", i32["restarts"][0])
    assert st == E.OK and i32["relres_true"][0] <= 1e-8
    assert np.allclose(s32["avg"], s64["avg"], rtol=1e-7, atol=1e-12)


@pytest.mark.parametrize("precision", [0, 1])
def test_batched_six_load_cases_equal_sequential(E, precision):
    """The six homogenisation load cases solved in one lockstep batch give
    bit-identical fields to six sequential solves; C_eff is symmetric."""
    say("case: batched multi-RHS, precision", precision)
    ms = _small_poly((24, 20, 18), 77, grains=10)
    ms.strain = synth.unit_load_cases()
    with E.Context.from_micro(ms, precision=precision) as cs:
        st, i_seq = cs.solve(1e-10, 20000)
        w_seq = [cs.solution(r) for r in range(6)]
        avg = np.array([cs.stress(r, voxel=False)["avg"] for r in range(6)])
    with E.Context.from_micro(ms, precision=precision, batched=1) as cb:
        st, i_bat = cb.solve(1e-10, 20000)
        w_bat = [cb.solution(r) for r in range(6)]
    say("iters seq", i_seq["iters"], "batched", i_bat["iters"])
    assert st == E.OK and max(i_bat["relres_true"]) <= 1e-10
    assert i_seq["iters"] == i_bat["iters"]
    for r in range(6):
        assert np.array_equal(w_seq[r], w_bat[r]), r
    Ceff = avg.T / 1e-3  # column j: mean stress of unit strain j
    assert np.abs(Ceff - Ceff.T).max() <= 1e-6 * np.abs(Ceff).max()


def test_config_poly300_six_cases_mixed_batched_full_size(E, orc):
    """The six-case homogenisation configuration at full size (poly300 on
    the device, mixed precision, one batched launch sequence, autotuned
    geometry): sampled operator nodes against the oracle, every case to a
    true relative residual of 1e-8, and C_eff symmetric and positive
    definite."""
    import torch
    from paper_2602_07354_amd import generate
    say("case: poly300, six cases, mixed + batched, full size")
    rec = synth.workload_recipe("poly300")
    dev = torch.device("cuda:0")
    phase = torch.empty(int(np.prod(rec["shape"])), dtype=torch.int32, device=dev)
    ms = generate.workload("poly300", phase=phase)
    torch.cuda.synchronize()
    host = synth.Microstructure(ms.shape, phase.cpu().numpy(), ms.C, ms.strain, ms.meta)
    assert ms.nrhs == 6
    P = orc.Problem.from_micro(host)
    rng = np.random.default_rng(300)
    sel = np.sort(rng.choice(host.n, 300, replace=False))
    opts = E.options_init(inputs_on_device=1, autotune=1, device=0, precision=E.PREC_MIXED, batched=1)
    h = E.setup(ms.shape, phase, ms.C, ms.strain, opts)
    try:
        x = rng.standard_normal((3, host.n))
        y = np.empty_like(x)
        E.apply(h, x, y)
        assert _rel(y[:, sel], P.apply_at(x, sel)) <= 1e-12
        del x, y
        st, info = E.solve(h, 1e-8, 50000, 6)
        say("   iterations", list(info.iters), "relres", max(info.relres_true[:6]), "tile", list(info.op_tile))
        assert st == E.OK and max(info.relres_true[:6]) <= 1e-8
        avg = np.empty((6, 6))
        for r in range(6):
            assert E.lib().elas3d_stress(h, r, None, avg[r].ctypes.data, None, None) == 0
    finally:
        E.destroy(h)
    Ceff = avg.T / 1e-3  # column j: mean stress of unit strain j
    assert np.abs(Ceff - Ceff.T).max() <= 1e-6 * np.abs(Ceff).max()
    assert np.linalg.eigvalsh(0.5 * (Ceff + Ceff.T)).min() > 0


def test_homogeneous_effective_stiffness_is_C(E):
    say("case: homogeneous C_eff")
    rng = np.random.default_rng(3)
    A = rng.standard_normal((6, 6))
    C = A @ A.T + 6 * np.eye(6)
    with E.Context((6, 5, 4), np.zeros(120, np.int32), C[None], synth.unit_load_cases(),
                   batched=1) as ctx:
        st, info = ctx.solve(1e-10, 100)
        avg = np.array([ctx.stress(r, voxel=False)["avg"] for r in range(6)])
    assert st == E.OK and info["iters"] == [0] * 6
    assert np.allclose(avg.T / 1e-3, C, rtol=1e-12)


@pytest.mark.parametrize("engine", ["group", "streams"])
def test_serving_results_same_alone_and_in_the_mix(E, engine):
    """Continuous batching: requests of uneven size admitted by memory budget
    and solved together (one launch per sweep for the whole mix, or one
    stream per request) give bit-identical results to the same requests
    solved alone."""
    say("case: serving mix vs alone,", engine)
    from paper_2602_07354_amd import serve
    pool = [r for r in serve.make_pool(12, seed0=900) if r.micro.shape[0] <= 96][:5]
    alone = [serve.solve_one(r) for r in pool]
    srv = serve.GroupServer(max_concurrency=4) if engine == "group" else serve.Server(max_concurrency=4)
    try:
        # all queued at once (concurrent), then a staggered stream
        mixed = serve.run_stream(pool, srv)
        import dataclasses
        stag = serve.run_stream([dataclasses.replace(r, arrival=0.01 * i) for i, r in enumerate(pool)], srv)
    finally:
        srv.close()
    for a, m, s in zip(alone, mixed, stag):
        assert a.status == 0 and max(a.relres_true) <= 1e-8
        assert a.iters == m.iters == s.iters
        assert np.array_equal(a.sigma_avg, m.sigma_avg) and np.array_equal(a.sigma_avg, s.sigma_avg)


def test_graph_replay_matches_eager_launches(E):
    """Iteration batches replayed from a captured HIP graph give the same
    iterates as eager launches (many replays per solve, host syncs between)."""
    say("case: graphs vs eager")
    ms = _small_poly((20, 18, 16), 5)
    out = []
    for graphs in (0, 1):
        with E.Context.from_micro(ms, graphs=graphs, poll_interval=4) as ctx:
            st, info = ctx.solve(1e-10, 5000)
            out.append((info["iters"], ctx.solution(0)))
    assert out[0][0] == out[1][0] and np.array_equal(out[0][1], out[1][1])


@pytest.mark.parametrize("tile", [0, 1, 2, 3, 4])  # 5: test_wave_specialised_sweep_matches_oracle
def test_every_sweep_tile_shape_matches_oracle(E, orc, tile):
    """Each workgroup shape of the fused direction+operator sweep (the
    autotuner's candidates) solves to the oracle's solution; ragged sizes so
    that every shape has partial tiles in x and y."""
    say("case: sweep tile shape", tile)
    ms = _small_poly((37, 29, 21), 41, grains=15)
    P = orc.Problem.from_micro(ms)
    ro = P.solve(ms.strain[0], tol=1e-12)
    for precision in (E.PREC_FP64, E.PREC_MIXED):
        with E.Context.from_micro(ms, tile=tile, precision=precision) as ctx:
            st, info = ctx.solve(1e-12 if precision == E.PREC_FP64 else 1e-10, 20000)
            assert st == E.OK
            assert info["op_tile"][:2] == list(E.TILE_SHAPES[tile])
            if precision == E.PREC_FP64:
                assert abs(info["iters"][0] - ro["iters"]) <= 2
            out = ctx.stress(0)
        so, _ = P.stress(ms.strain[0], ro["w"])
        assert _rel(out["sigma"], so) <= (1e-8 if precision == E.PREC_FP64 else 1e-7)


def test_fixed_z_chunking_matches_oracle(E, orc):
    """options.zchunk fixes the z planes per workgroup of the fused sweep
    (values above nz mean nz); every choice solves to the oracle's answer."""
    say("case: fixed z chunking")
    ms = _small_poly((37, 29, 21), 47, grains=15)
    P = orc.Problem.from_micro(ms)
    ro = P.solve(ms.strain[0], tol=1e-12)
    so, _ = P.stress(ms.strain[0], ro["w"])
    for zc in (1, 5, 21, 100):
        with E.Context.from_micro(ms, tile=4, zchunk=zc) as ctx:
            st, info = ctx.solve(1e-12, 20000)
            assert st == E.OK and info["op_tile"] == [64, 8, min(zc, 21)]
            assert abs(info["iters"][0] - ro["iters"]) <= 2
            assert _rel(ctx.stress(0)["sigma"], so) <= 1e-8
    # the wave-specialised sweep takes its plane steps two per loop trip:
    # chunks of an odd and an even number of steps (zchunk + 1), and a grid
    # whose last chunk is shorter than the others
    say("case: fixed z chunking, wave-specialised")
    ms = _small_poly((38, 29, 21), 47, grains=15)
    P = orc.Problem.from_micro(ms)
    ro = P.solve(ms.strain[0], tol=1e-12)
    so, _ = P.stress(ms.strain[0], ro["w"])
    for zc in (1, 2, 4, 21):
        with E.Context.from_micro(ms, tile=5, zchunk=zc, autotune=2) as ctx:
            st, info = ctx.solve(1e-12, 20000)
            assert st == E.OK and info["op_tile"] == [64, 6, zc] and info["apply_tile"] == [64, 6, zc]
            assert abs(info["iters"][0] - ro["iters"]) <= 2
            assert _rel(ctx.stress(0)["sigma"], so) <= 1e-8
    # the FP32-only 64x8 shape in mixed precision (its FP64 sweeps on 64x8 lanes)
    ms = _small_poly((40, 29, 21), 47, grains=15)
    P = orc.Problem.from_micro(ms)
    ro = P.solve(ms.strain[0], tol=1e-12)
    so, _ = P.stress(ms.strain[0], ro["w"])
    for zc in (1, 2, 21):
        say("case: fixed z chunking, FP32 64x8 shape, zchunk", zc)
        with E.Context.from_micro(ms, tile=6, zchunk=zc, autotune=2, precision=E.PREC_MIXED) as ctx:
            st, info = ctx.solve(1e-10, 20000)
            assert st == E.OK and info["op_tile"] == [64, 8, zc] and info["op_shape"] == 6
            assert info["apply_tile"] == [64, 8, zc]
            assert _rel(ctx.stress(0)["sigma"], so) <= 1e-7


def test_update_sweep_forms_are_bitwise_equal(E, orc):
    """The plain and the non-temporal form of the update sweep compute the
    same arithmetic: on the same grid their solves agree bit for bit (FP64,
    mixed, three batched cases), and they solve to the oracle."""
    ms = _small_poly((40, 36, 30), 71, grains=24)
    ms3 = synth.polycrystal((40, 36, 33), 20, 72, [dict(kind="sphere", fraction=0.02, median=1.5, sigma=0.3)],
                            synth.unit_load_cases()[:3])
    P = orc.Problem.from_micro(ms)
    ro = P.solve(ms.strain[0], tol=1e-12)
    cases = [("fp64", ms, dict(), 1e-12), ("mixed", ms, dict(precision=E.PREC_MIXED), 1e-10),
             ("fp64 x3 batched", ms3, dict(batched=1), 1e-10)]
    for name, m, kw, tol in cases:
        for blocks in (32768, 37):
            say("case: update forms,", name, "update grid", blocks)
            out = []
            for nt in (0, 1):
                with E.Context.from_micro(m, update_blocks=blocks, update_nontemporal=nt, **kw) as ctx:
                    st, info = ctx.solve(tol, 20000)
                    assert st == E.OK and max(info["relres_true"]) <= tol
                    assert info["update_blocks"] == blocks and info["update_nontemporal"] == nt
                    out.append((info["iters"], [ctx.solution(r) for r in range(m.nrhs)],
                                [ctx.stress(r)["sigma"] for r in range(m.nrhs)]))
            assert out[0][0] == out[1][0]
            for a, b in zip(out[0][1] + out[0][2], out[1][1] + out[1][2]):
                assert np.array_equal(a, b)
            if name == "fp64":
                assert abs(out[0][0][0] - ro["iters"]) <= 2
                so, _ = P.stress(ms.strain[0], ro["w"])
                assert _rel(out[0][2][0], so) <= 1e-8


def test_autotuned_geometry_solves_and_is_cached(E, orc):
    """Autotuning picks one of the candidate geometries, solves to the same
    answer (to rounding) as the default geometry, and a second context of the
    same size reuses the choice."""
    say("case: autotune")
    ms = _small_poly((45, 38, 30), 43, grains=18)
    P = orc.Problem.from_micro(ms)
    ro = P.solve(ms.strain[0], tol=1e-12)
    so, _ = P.stress(ms.strain[0], ro["w"])
    infos = []
    for _ in range(2):
        with E.Context.from_micro(ms, autotune=1) as ctx:
            st, info = ctx.solve(1e-12, 20000)
            assert st == E.OK and info["relres_true"][0] <= 1e-12
            assert tuple(info["op_tile"][:2]) in E.TILE_SHAPES
            assert info["update_blocks"] in (1024, 2048, 4096, 8192, 16384, 32768)
            assert info["update_nontemporal"] in (0, 1)
            assert abs(info["iters"][0] - ro["iters"]) <= 2
            assert _rel(ctx.stress(0)["sigma"], so) <= 1e-8
            infos.append(info)
    for k in ("op_tile", "update_blocks", "update_nontemporal"):
        assert infos[0][k] == infos[1][k], k
    with E.Context.from_micro(ms, autotune=1, precision=E.PREC_MIXED) as ctx:
        st, info = ctx.solve(1e-10, 20000)
        assert st == E.OK and info["relres_true"][0] <= 1e-10
    # autotune = 2: the update sweep is tuned, the operator sweep keeps the
    # geometry the options fix
    say("case: autotune of the update sweep only, 64x8 fixed")
    with E.Context.from_micro(ms, tile=4) as ctx:
        _, fixed = ctx.solve(1e-12, 20000)
    with E.Context.from_micro(ms, autotune=2, tile=4) as ctx:
        st, info = ctx.solve(1e-12, 20000)
        assert st == E.OK and info["relres_true"][0] <= 1e-12
        assert info["op_tile"] == fixed["op_tile"] and tuple(info["op_tile"][:2]) == (64, 8)
        assert info["update_blocks"] in (1024, 2048, 4096, 8192, 16384, 32768)
        assert abs(info["iters"][0] - ro["iters"]) <= 2
        assert _rel(ctx.stress(0)["sigma"], so) <= 1e-8


from test_oracle_pins import BREAKDOWN_CASES  # noqa: E402


@pytest.mark.parametrize("poll", [0, 1])
@pytest.mark.parametrize("case", BREAKDOWN_CASES, ids=lambda c: "k%d" % c[-1])
def test_breakdown_matches_oracle(E, orc, case, poll):
    """Indefinite grid (a phase with -C): the step size of Algorithm 2 meets
    h.Ah <= 0 at iteration k (pinned on the oracle by the Krylov projection).
    The GPU stops with BREAKDOWN at the same iteration, and the iterate it
    returns (every step owed to w paid, none of the breaking iteration) is the
    oracle's.  k = 1, 2, 3, 8, 13 covers a breakdown with no step owed, with
    one owed and with two just paid by the sweep; poll 1 looks at the flags
    after every iteration, 0 after batches of 16 replayed as graphs."""
    shape, seed, frac, eneg, k = case
    say("case: breakdown", case, "poll", poll)
    ms = synth.indefinite_grid(shape, seed, frac, eneg)
    P = orc.Problem.from_micro(ms)
    ro = P.solve(ms.strain[0], tol=1e-12, maxit=500)
    assert ro["status"] == orc.BREAKDOWN and ro["iters"] == k
    with E.Context.from_micro(ms, poll_interval=poll) as ctx:
        st, info = ctx.solve(1e-12, 500)
        w = ctx.solution(0)
    assert st == E.BREAKDOWN and info["status"][0] == E.BREAKDOWN
    assert info["iters"][0] == k
    if k == 1:
        assert np.all(w == 0.0)
    else:
        assert _rel(w, ro["w"]) <= 1e-10


@pytest.mark.parametrize("tile", [5, 6])
def test_wave_specialised_sweep_matches_oracle(E, orc, tile):
    """The wave-specialised fused sweep (loader wavefronts streaming node
    planes into an LDS ring): solves to the oracle's solution in FP64 and
    mixed precision on a grid with partial tiles in x (68 = 63 + 5) and y,
    and on one narrower than a tile (nx = 8: the patch rows wrap around the
    periodic box several times); the iterates after k = 1..5 iterations
    equal the oracle's, single case and batched."""
    for shape, grains in (((68, 29, 21), 20), ((8, 6, 5), 4)):
        say("case: wave-specialised sweep, tile", tile, shape)
        ms = _small_poly(shape, 61 + shape[0], grains=grains)
        P = orc.Problem.from_micro(ms)
        ro = P.solve(ms.strain[0], tol=1e-12)
        so, _ = P.stress(ms.strain[0], ro["w"])
        for precision in ((E.PREC_MIXED,) if tile in E.WS_FP32_ONLY else (E.PREC_FP64, E.PREC_MIXED)):
            with E.Context.from_micro(ms, tile=tile, precision=precision) as ctx:
                st, info = ctx.solve(1e-12 if precision == E.PREC_FP64 else 1e-10, 20000)
                assert st == E.OK
                assert info["op_tile"][:2] == list(E.TILE_SHAPES[tile]) and info["op_shape"] == tile
                if precision == E.PREC_FP64:
                    assert abs(info["iters"][0] - ro["iters"]) <= 2
                out = ctx.stress(0)
            assert _rel(out["sigma"], so) <= (1e-8 if precision == E.PREC_FP64 else 1e-7)
    if tile in E.WS_FP32_ONLY:
        # two load cases batched in lockstep (case-major workgroups of one
        # launch) in mixed precision: each reaches the oracle's stress
        say("case: FP32-only shape, two load cases batched")
        shape = (40, 19, 23)
        ms2 = synth.polycrystal(shape, 12, 37, [dict(kind="sphere", fraction=0.02, median=1.5, sigma=0.3)],
                                synth.unit_load_cases()[[1, 5]])
        P2 = orc.Problem.from_micro(ms2)
        with E.Context.from_micro(ms2, batched=1, tile=tile, precision=E.PREC_MIXED) as ctx:
            st, info = ctx.solve(1e-10, 20000)
            assert st == E.OK and info["op_shape"] == tile
            for r in range(2):
                ro2 = P2.solve(ms2.strain[r], tol=1e-12)
                so2, _ = P2.stress(ms2.strain[r], ro2["w"])
                assert _rel(ctx.stress(r)["sigma"], so2) <= 1e-7, r
        return  # (the iterates below are FP64's)
    say("case: wave-specialised sweep iterates, tile", tile)
    shape = (20, 19, 23)
    ms = _small_poly(shape, 29)
    ms2 = synth.polycrystal(shape, 12, 29, [dict(kind="sphere", fraction=0.02, median=1.5, sigma=0.3)],
                            synth.unit_load_cases()[[2, 4]])
    P = orc.Problem.from_micro(ms)
    P2 = orc.Problem.from_micro(ms2)
    for k in range(1, 6):
        ro = P.solve(ms.strain[0], tol=1e-30, maxit=k)
        with E.Context.from_micro(ms, tile=tile) as ctx:
            st, info = ctx.solve(1e-30, k)
            assert st == E.NOT_CONVERGED and info["iters"][0] == k
            assert _rel(ctx.solution(0), ro["w"]) <= 1e-11, k
        with E.Context.from_micro(ms2, batched=1, tile=tile) as ctx:
            st, info = ctx.solve(1e-30, k)
            for r in range(2):
                ro2 = P2.solve(ms2.strain[r], tol=1e-30, maxit=k)
                assert _rel(ctx.solution(r), ro2["w"]) <= 1e-11, (k, r)


def test_wave_specialised_sweep_on_a_grid_of_several_workgroup_groups(E, orc):
    """A grid with more workgroups than the XCDs hold at once (432 at
    4-plane chunks: one whole group of 8 x 32 and a tail), so that both parts
    of the workgroup-to-tile map run: the iterates after k = 1..3 iterations
    equal the oracle's, for the fused sweep and the residual sweep."""
    shape = (128, 60, 48)
    ms = _small_poly(shape, 83, grains=40)
    P = orc.Problem.from_micro(ms)
    b, _ = P.load(ms.strain[0])
    for k in (1, 2, 3):
        say("case: wave-specialised sweep, several workgroup groups, k =", k)
        ro = P.solve(ms.strain[0], tol=1e-30, maxit=k)
        with E.Context.from_micro(ms, tile=5, zchunk=4, autotune=2) as ctx:
            st, info = ctx.solve(1e-30, k)
            assert st == E.NOT_CONVERGED and info["iters"][0] == k
            assert info["op_tile"] == [64, 6, 4] and info["apply_tile"] == [64, 6, 4]
            w = ctx.solution(0)
            assert _rel(w, ro["w"]) <= 1e-11, k
            rel = np.linalg.norm(P.apply(w) + b) / np.linalg.norm(b)
            assert abs(info["relres_true"][0] - rel) <= 1e-9 * rel, (info["relres_true"][0], rel)


def _many_phase_grid(shape, nphase, seed):
    """Every voxel its own random draw among nphase rotated 316L crystals: a
    64-voxel row meets far more distinct phases than a grain structure does."""
    rng = synth.rng_for(seed)
    C = synth.rotate_stiffness(synth.cubic_stiffness(*synth.SS316L_CUBIC), synth.random_rotations(rng, nphase))
    phase = rng.integers(0, nphase, int(np.prod(shape))).astype(np.int32)
    return synth.Microstructure(tuple(shape), phase, C,
                                np.array([[2e-4, -1e-4, 1e-3, 3e-4, -2e-4, 1e-4]]), {"workload": "many_phase"})


def test_sweep_with_many_phases_per_box(E, orc):
    """A grid whose rows hold dozens of distinct phases, so that a
    wave-specialised workgroup box holds more than its phase dictionary: the
    forced wave-specialised shape is refused at setup, and with autotuning
    another shape is chosen and solves to the oracle's solution.  (Parity of
    the classic sweep on it: test_sweep_with_many_phases_per_row_matches_oracle.)"""
    ms = _many_phase_grid((72, 13, 11), 300, 7)
    for tile in E.WS_TILES:
        for prec in ((E.PREC_MIXED,) if tile in E.WS_FP32_ONLY else (E.PREC_FP64, E.PREC_MIXED)):
            with pytest.raises(E.Elas3dError) as ei:
                E.Context.from_micro(ms, tile=tile, precision=prec)
            assert ei.value.code == E.EBADARG and "distinct phases" in str(ei.value)
    P = orc.Problem.from_micro(ms)
    ro = P.solve(ms.strain[0], tol=1e-12)
    with E.Context.from_micro(ms, autotune=1) as ctx:
        st, info = ctx.solve(1e-12, 20000)
        assert st == E.OK and abs(info["iters"][0] - ro["iters"]) <= 2
        assert info["op_shape"] not in E.WS_TILES
        assert _rel(ctx.solution(0), ro["w"]) <= 1e-9


@pytest.mark.parametrize("tile", [5, 6])
def test_wave_specialised_sweep_with_a_full_dictionary(E, orc, tile):
    """Every voxel draws one of exactly 96 phases (a workgroup box holds all
    of them: the phase dictionary is full, ranks 0..95 in use): the
    wave-specialised sweep's iterates after k = 1..3 iterations equal the
    oracle's, and the FP64 and mixed-precision solves reach its stress (the
    FP32-only shape: the mixed-precision solve)."""
    ms = _many_phase_grid((72, 13, 11), 96, 11)
    assert len(np.unique(ms.phase)) == 96
    P = orc.Problem.from_micro(ms)
    fp64 = tile not in E.WS_FP32_ONLY
    for k in range(1, 4) if fp64 else ():
        say("case: full dictionary, iterations", k)
        ro = P.solve(ms.strain[0], tol=1e-30, maxit=k)
        with E.Context.from_micro(ms, tile=tile) as ctx:
            st, info = ctx.solve(1e-30, k)
            assert st == E.NOT_CONVERGED and info["iters"][0] == k
            assert _rel(ctx.solution(0), ro["w"]) <= 1e-11, k
    ro = P.solve(ms.strain[0], tol=1e-12)
    so, _ = P.stress(ms.strain[0], ro["w"])
    for precision in (E.PREC_FP64, E.PREC_MIXED) if fp64 else (E.PREC_MIXED,):
        say("case: full dictionary, converged, precision", precision)
        with E.Context.from_micro(ms, tile=tile, precision=precision) as ctx:
            st, info = ctx.solve(1e-12 if precision == E.PREC_FP64 else 1e-10, 20000)
            assert st == E.OK and info["op_shape"] == tile
            out = ctx.stress(0)
        assert _rel(out["sigma"], so) <= (1e-8 if precision == E.PREC_FP64 else 1e-7)


@pytest.mark.parametrize("tile", [4])
def test_sweep_with_many_phases_per_row_matches_oracle(E, orc, tile):
    """A grid whose rows hold dozens of distinct phases (every voxel its own
    draw): the iterates after k = 1..4 iterations and the converged stress
    equal the oracle's in FP64, and the mixed-precision solve reaches the
    oracle's solution."""
    ms = _many_phase_grid((72, 13, 11), 300, 7)
    rows = ms.phase.reshape(11, 13, 72)
    assert min(len(np.unique(rows[k, j, :64])) for k in range(11) for j in range(13)) > 32
    P = orc.Problem.from_micro(ms)
    for k in range(1, 5):
        say("case: many phases per row, tile", tile, "iterations", k)
        ro = P.solve(ms.strain[0], tol=1e-30, maxit=k)
        with E.Context.from_micro(ms, tile=tile) as ctx:
            st, info = ctx.solve(1e-30, k)
            assert st == E.NOT_CONVERGED and info["iters"][0] == k
            assert _rel(ctx.solution(0), ro["w"]) <= 1e-11, k
    say("case: many phases per row, converged, tile", tile)
    ro = P.solve(ms.strain[0], tol=1e-12)
    so, _ = P.stress(ms.strain[0], ro["w"])
    for precision in (E.PREC_FP64, E.PREC_MIXED):
        with E.Context.from_micro(ms, tile=tile, precision=precision) as ctx:
            st, info = ctx.solve(1e-12 if precision == E.PREC_FP64 else 1e-10, 20000)
            assert st == E.OK
            if precision == E.PREC_FP64:
                assert abs(info["iters"][0] - ro["iters"]) <= 2
            out = ctx.stress(0)
        assert _rel(out["sigma"], so) <= (1e-8 if precision == E.PREC_FP64 else 1e-7)


def test_wave_specialised_operator_gives_the_true_residual(E, orc):
    """With the wave-specialised shape forced (autotune = 2), the residual
    sweep (y = A w + b, the true residual of the stopping test) and the mixed
    refinement sweep (w += d, then r = A w + b stored in FP32 with ||r||^2 in
    FP64) run in their wave-specialised forms: the relative true residual the
    GPU reports equals the oracle's ||A w + b|| / ||b|| of the returned w, in
    FP64 and in mixed precision (whose refinement cycles each take one), and
    mixed precision refined to 1e-12 reaches the FP64 oracle's solution."""
    ms = _small_poly((68, 29, 21), 131, grains=20)
    P = orc.Problem.from_micro(ms)
    b, _ = P.load(ms.strain[0])
    for precision in (E.PREC_FP64, E.PREC_MIXED):
        say("case: wave-specialised residual sweep, precision", precision)
        with E.Context.from_micro(ms, tile=5, autotune=2, precision=precision) as ctx:
            st, info = ctx.solve(1e-6, 20000)
            assert st == E.OK
            assert info["apply_tile"][:2] == [64, 6] and info["op_shape"] == 5
            w = ctx.solution(0)
        rel = np.linalg.norm(P.apply(w) + b) / np.linalg.norm(b)
        assert 0 < rel <= 1e-6
        assert abs(info["relres_true"][0] - rel) <= 1e-6 * rel, (info["relres_true"][0], rel)
    say("case: wave-specialised refinement sweep to 1e-12")
    ro = P.solve(ms.strain[0], tol=1e-12)
    so, _ = P.stress(ms.strain[0], ro["w"])
    with E.Context.from_micro(ms, tile=5, autotune=2, precision=E.PREC_MIXED) as ctx:
        st, info = ctx.solve(1e-12, 20000)
        say("mixed", info["iters"][0], "inner iterations,", info["restarts"][0], "cycles, fallback",
            info["fp64_fallback"][0])
        assert st == E.OK and info["fp64_fallback"][0] == 0 and info["restarts"][0] >= 1
        assert info["apply_tile"][:2] == [64, 6]
        w = ctx.solution(0)
        out = ctx.stress(0)
    rel = np.linalg.norm(P.apply(w) + b) / np.linalg.norm(b)
    # at 1e-12 the two residuals differ by rounding of order 1e-16 ||b||
    assert rel <= 1.05e-12 and abs(info["relres_true"][0] - rel) <= 1e-2 * rel, (info["relres_true"][0], rel)
    assert _rel(out["sigma"], so) <= 1e-8
    active = np.any(np.abs(P.precond()).reshape(ms.n, 9) > 0, axis=1)
    d1 = w[:, active] - w[:, active].mean(axis=1, keepdims=True)
    d0 = ro["w"][:, active] - ro["w"][:, active].mean(axis=1, keepdims=True)
    assert _rel(d1, d0) <= 1e-8


def test_wave_specialised_shape_needs_whole_chunks(E):
    """Forcing a wave-specialised shape on a grid whose rows are not a whole
    number of 16-byte chunks is refused at setup (before any device work)."""
    ms = _small_poly((37, 29, 21), 41, grains=15)
    for prec in (E.PREC_FP64, E.PREC_MIXED):
        with pytest.raises(E.Elas3dError) as ei:
            E.Context.from_micro(ms, tile=5, precision=prec)
        assert ei.value.code == E.EBADARG and "multiple" in str(ei.value)
    ms2 = _small_poly((38, 29, 21), 41, grains=15)  # even: FP64 fine, mixed needs 4
    E.Context.from_micro(ms2, tile=5).close()
    with pytest.raises(E.Elas3dError):
        E.Context.from_micro(ms2, tile=5, precision=E.PREC_MIXED)
