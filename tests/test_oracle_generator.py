"""Pins of the oracle's microstructure generator and von Mises output
(Sec. 2.2, Eq. ellipsoid_dist; Sec. 2.2.3 pore overwrite; Table 1) against
closed forms, a library routine and exact invariances."""

import numpy as np
import pytest

import oracle


def _rng(seed):
    return np.random.default_rng(seed)


def test_two_seeds_split_the_box_at_the_bisector():
    # equal isotropic grains at x = L/4 and 3L/4: the periodic bisectors are
    # x = L/2 and x = 0, so voxel i belongs to grain 1 iff i >= L/2
    L, M = 12, 5
    seeds = np.array([[L / 4, 2.3, 1.1], [3 * L / 4, 2.3, 1.1]])
    ph = oracle.grains((L, M, M), seeds).reshape(M, M, L)
    expect = (np.arange(L) >= L // 2).astype(np.int32)
    assert np.array_equal(ph, np.broadcast_to(expect, (M, M, L)))


def test_unit_radii_is_the_periodic_voronoi_of_a_kd_tree():
    from scipy.spatial import cKDTree
    shape = (20, 17, 13)
    box = np.array(shape, dtype=float)
    seeds = _rng(1).random((30, 3)) * box
    ph = oracle.grains(shape, seeds)
    k, j, i = np.meshgrid(np.arange(13), np.arange(17), np.arange(20), indexing="ij")
    pts = np.stack([i.ravel() + 0.5, j.ravel() + 0.5, k.ravel() + 0.5], axis=1)
    _, idx = cKDTree(seeds, boxsize=box).query(pts)
    assert np.array_equal(ph, idx.astype(np.int32))


def test_weighted_grain_owns_its_apollonius_sphere():
    # two isotropic grains with radii r0 > r1 far from the box faces: grain 1
    # owns exactly the points with |x - s1| / r1 < |x - s0| / r0, the ball of
    # centre (s1 - k^2 s0) / (1 - k^2) and radius k |s1 - s0| / (1 - k^2),
    # k = r1 / r0 (Apollonius).  Only voxels clear of the sphere surface are
    # compared.
    L = 40
    s0 = np.array([20.3, 19.7, 20.1])
    s1 = np.array([25.9, 20.4, 19.6])
    r0, r1 = 2.0, 1.0
    k = r1 / r0
    c = (s1 - k * k * s0) / (1 - k * k)
    rho = k * np.linalg.norm(s1 - s0) / (1 - k * k)
    ph = oracle.grains((L, L, L), np.stack([s0, s1]), np.array([[r0, r0], [r1, r1]])).reshape(L, L, L)
    kk, jj, ii = np.meshgrid(np.arange(L), np.arange(L), np.arange(L), indexing="ij")
    dist = np.sqrt((ii + 0.5 - c[0]) ** 2 + (jj + 0.5 - c[1]) ** 2 + (kk + 0.5 - c[2]) ** 2)
    clear = np.abs(dist - rho) > 1e-6
    assert rho + np.abs(c - L / 2).max() < L / 2  # no periodic image interferes
    assert np.array_equal((ph == 1)[clear], (dist < rho)[clear])
    assert (ph == 1).sum() > 100


def test_longitudinal_radius_acts_along_z():
    # grain 0 (rt = 1, rl = 2) and grain 1 (1, 1) on one z-line: the x-y terms
    # cancel and the boundary is |z - z0| = 2 |z - z1|, the plane
    # z = (z0 + 2 z1) / 3 between them (no wrap: both near the middle)
    L = 24
    z0, z1 = 8.2, 14.5
    seeds = np.array([[12.0, 12.0, z0], [12.0, 12.0, z1]])
    ph = oracle.grains((L, L, L), seeds, np.array([[1.0, 2.0], [1.0, 1.0]])).reshape(L, L, L)
    zc = np.arange(L) + 0.5
    zb = (z0 + 2 * z1) / 3
    between = (zc > z0) & (zc < z1)
    for kz in np.nonzero(between)[0]:
        assert np.all(ph[kz] == (0 if zc[kz] < zb else 1))


def test_assignment_is_invariant_to_radius_scale_and_relabelling():
    shape = (15, 18, 11)
    rng = _rng(2)
    seeds = rng.random((25, 3)) * np.array(shape)
    semi = np.exp(0.3 * rng.standard_normal((25, 2)))
    ph = oracle.grains(shape, seeds, semi)
    # doubling every semi-axis scales every D^2 by exactly 1/4
    assert np.array_equal(ph, oracle.grains(shape, seeds, 2.0 * semi))
    perm = rng.permutation(25)
    ph_p = oracle.grains(shape, seeds[perm], semi[perm])
    assert np.array_equal(perm[ph_p], ph)


def _pore(c, a, R=None):
    return np.concatenate([c, a, (np.eye(3) if R is None else R).ravel()])


def test_sphere_pore_covers_the_lattice_points_of_its_ball():
    # a sphere centred on a voxel centre covers the voxels whose integer
    # offsets lie in the ball (counted here directly)
    L = 16
    for r in (1.0, 2.0, 2.5, 3.7):
        ph, used, nvoid = oracle.carve((L, L, L), np.zeros(L ** 3, np.int32), 9,
                                       _pore(np.array([8.5, 8.5, 8.5]), np.array([r, r, r])))
        o = np.arange(-8, 8)
        a, b, cc = np.meshgrid(o, o, o, indexing="ij")
        assert nvoid == int(np.count_nonzero(a * a + b * b + cc * cc <= r * r)), r
        assert used == 1


def test_rotation_by_a_quarter_turn_swaps_the_semi_axes():
    L = 14
    c = np.array([6.2, 7.9, 5.4])
    Rz = np.array([[0.0, -1.0, 0.0], [1.0, 0.0, 0.0], [0.0, 0.0, 1.0]])
    ph_r, _, n_r = oracle.carve((L, L, L), np.zeros(L ** 3, np.int32), 1, _pore(c, np.array([3.0, 2.0, 1.5]), Rz))
    ph_a, _, n_a = oracle.carve((L, L, L), np.zeros(L ** 3, np.int32), 1, _pore(c, np.array([2.0, 3.0, 1.5])))
    assert n_r == n_a > 0
    assert np.array_equal(ph_r, ph_a)


def test_pore_wraps_around_the_periodic_box():
    L = 10
    ph, _, n = oracle.carve((L, L, L), np.zeros(L ** 3, np.int32), 1,
                            _pore(np.array([0.1, 9.9, 5.0]), np.array([1.6, 1.6, 1.6])))
    ph = ph.reshape(L, L, L)
    assert ph[5, 9, 0] == 1 and ph[4, 0, 9] == 1 and ph[5, 0, 0] == 1
    assert n == int(ph.sum())


def test_carving_stops_at_the_first_pore_reaching_the_target():
    L = 20
    rng = _rng(3)
    pores = np.stack([_pore(rng.random(3) * L, np.full(3, 1.0 + 2 * rng.random())) for _ in range(40)])
    base = np.zeros(L ** 3, np.int32)
    base[:37] = 5  # already void: counted, never carved again
    target = 0.05 * L ** 3
    ph, used, nvoid = oracle.carve((L, L, L), base, 5, pores, target)
    assert nvoid >= target
    _, _, n_before = oracle.carve((L, L, L), base, 5, pores[: used - 1])
    _, _, n_all = oracle.carve((L, L, L), base, 5, pores[:used])
    assert n_before < target <= n_all == nvoid
    assert np.count_nonzero(ph == 5) == nvoid
    # nothing to do when the target is already met
    _, used0, n0 = oracle.carve((L, L, L), base, 5, pores, 37.0)
    assert used0 == 0 and n0 == 37


def test_von_mises_closed_forms_and_invariance():
    s, t, p = 3.0, 2.0, 7.0
    sig = np.array([[s, 0, 0, 0, 0, 0],        # uniaxial: |s|
                    [0, 0, 0, 0, 0, t],        # pure shear: sqrt(3) |t|
                    [p, p, p, 0, 0, 0],        # hydrostatic: 0
                    [s, -s, 0, 0, 0, 0]]).T    # in-plane pure shear: sqrt(3) s
    vm = oracle.von_mises(sig)
    assert np.allclose(vm, [s, np.sqrt(3) * t, 0.0, np.sqrt(3) * s], rtol=1e-15, atol=1e-15)
    # invariant under rotation of the stress tensor
    rng = _rng(4)
    S = rng.standard_normal((3, 3))
    S = S + S.T
    Q, _ = np.linalg.qr(rng.standard_normal((3, 3)))
    def voigt(T):
        return np.array([T[0, 0], T[1, 1], T[2, 2], T[1, 2], T[0, 2], T[0, 1]])
    a = oracle.von_mises(voigt(S)[:, None])
    b = oracle.von_mises(voigt(Q @ S @ Q.T)[:, None])
    assert np.allclose(a, b, rtol=1e-13)
    # sqrt(3 J2) with J2 from the deviator
    D = S - np.trace(S) / 3 * np.eye(3)
    assert np.isclose(a[0], np.sqrt(1.5 * np.sum(D * D)), rtol=1e-13)


def _probe_voxels(shape, rng, count):
    """Random voxels plus every corner and a voxel on each face of the box
    (the places where the periodic minimum image wraps)."""
    nx, ny, nz = shape
    corners = [i + nx * (j + ny * k) for i in (0, nx - 1) for j in (0, ny - 1) for k in (0, nz - 1)]
    faces = [0 + nx * (ny // 2 + ny * (nz // 2)), nx - 1 + nx * (ny // 2 + ny * (nz // 2)),
             nx // 2 + nx * (0 + ny * (nz // 2)), nx // 2 + nx * (ny - 1 + ny * (nz // 2)),
             nx // 2 + nx * (ny // 2 + ny * 0), nx // 2 + nx * (ny // 2 + ny * (nz - 1))]
    return np.concatenate([rng.integers(0, nx * ny * nz, count), corners, faces]).astype(np.int64)


@pytest.mark.parametrize("shape", [(13, 7, 5), (9, 16, 11), (4, 3, 17)])
def test_grains_at_samples_the_full_assignment(shape):
    # the sampled helper is Eq. (ellipsoid_dist) evaluated at chosen voxels:
    # it must agree with the full brute-force map (pinned above by closed
    # forms and the periodic k-d tree) wherever it is asked, weighted or not
    rng = _rng(11 + shape[0])
    box = np.array(shape, dtype=float)
    seeds = rng.random((23, 3)) * box
    semi = np.stack([0.6 + rng.random(23), 0.6 + 2.0 * rng.random(23)], axis=1)
    idx = _probe_voxels(shape, rng, 200)
    for s in (None, semi):
        full = oracle.grains(shape, seeds, s)
        assert np.array_equal(oracle.grains_at(shape, seeds, s, idx), full[idx])


@pytest.mark.parametrize("shape", [(15, 11, 9), (8, 19, 6)])
def test_covered_at_is_the_void_mask_of_carving_every_pore(shape):
    # a voxel is covered iff carving all pores (no target) makes it void
    # (Sec. 2.2.3 pore overwrite; the carving is pinned above by lattice
    # counts, a quarter-turn symmetry and periodic wrap)
    rng = _rng(23 + shape[1])
    box = np.array(shape, dtype=float)
    pores = []
    for t in range(9):
        Q, _ = np.linalg.qr(rng.standard_normal((3, 3)))
        c = rng.random(3) * box
        if t == 0:
            c = np.array([0.05, box[1] - 0.05, box[2] - 0.1])  # straddles a corner of the box
        pores.append(_pore(c, 0.7 + 2.5 * rng.random(3), Q))
    pores = np.stack(pores)
    n = int(np.prod(shape))
    ph, used, nvoid = oracle.carve(shape, np.zeros(n, np.int32), 7, pores)
    assert used == len(pores) and 0 < nvoid < n
    idx = np.concatenate([_probe_voxels(shape, rng, 300), np.flatnonzero(ph == 7)[:50]])
    got = oracle.covered_at(shape, pores, idx)
    assert np.array_equal(got, (ph[idx] == 7).astype(np.int32))
    assert got.sum() > 0 and got.sum() < idx.size
