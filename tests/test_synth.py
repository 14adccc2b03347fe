"""Seeded input generator: reproducibility, recipe statistics, orientation sampling."""

import numpy as np
import pytest

from paper_2602_07354_amd import synth


def test_seed_reproducible_and_recipe():
    a = synth.workload("poly100", scale=40)
    b = synth.workload("poly100", scale=40)
    assert np.array_equal(a.phase, b.phase) and np.array_equal(a.C, b.C)
    assert a.phase.dtype == np.int32 and a.phase.size == 40 ** 3
    ng = a.meta["n_grains"]
    assert a.nphase == ng + 1
    assert np.all(a.C[ng] == 0.0)            # shared void phase
    assert a.void_fraction() >= 0.01        # stop rule: first pore reaching 1 %
    assert a.phase.min() >= 0 and a.phase.max() <= ng
    full = synth.workload("poly100")
    assert full.meta["n_grains"] == 500 and 0.01 <= full.void_fraction() < 0.0115


def test_eshelby_inclusion_voxel_count():
    ms = synth.eshelby_inclusion(20)
    assert ms.meta["inclusion_voxels"] == 552
    assert np.array_equal(ms.phase.reshape(20, 20, 20), ms.phase.reshape(20, 20, 20)[::-1, ::-1, ::-1])


def test_periodic_voronoi_wraps():
    # one seed just inside the +x face: the voxel at the -x face is closer to it
    seeds = np.array([[9.9, 2.5, 2.5], [4.0, 2.5, 2.5]])
    ph = synth.periodic_voronoi((10, 5, 5), seeds).reshape(5, 5, 10)
    assert ph[2, 2, 0] == 0 and ph[2, 2, 9] == 0 and ph[2, 2, 4] == 1


def test_carve_sphere_wraps_and_counts():
    ph = np.zeros(8 * 8 * 8, np.int32)
    fresh = synth.carve_spheres(ph, (8, 8, 8), np.array([[0.0, 0.0, 0.0]]), np.array([1.0]), 7)
    v = ph.reshape(8, 8, 8)
    assert fresh == 8 and v[0, 0, 0] == 7 and v[7, 7, 7] == 7 and v[0, 0, 7] == 7


def test_rotations_orthonormal_and_uniform():
    rng = synth.rng_for(3)
    R = synth.random_rotations(rng, 20000)
    assert np.allclose(R @ np.swapaxes(R, 1, 2), np.eye(3), atol=1e-12)
    assert np.allclose(np.linalg.det(R), 1.0, atol=1e-12)
    # Haar measure: the rotation angle has density (1 - cos t)/pi on [0, pi]
    t = np.arccos(np.clip((np.trace(R, axis1=1, axis2=2) - 1) / 2, -1, 1))
    edges = np.linspace(0, np.pi, 11)
    cdf = lambda x: (x - np.sin(x)) / np.pi
    expect = np.diff(cdf(edges)) * len(t)
    obs, _ = np.histogram(t, edges)
    chi2 = np.sum((obs - expect) ** 2 / expect)
    assert chi2 < 30.0  # 9 dof, p ~ 4e-4
    # rotated z axes are isotropic: mean of each component ~ 0, second moment 1/3
    z = R[:, :, 2]
    assert np.abs(z.mean(axis=0)).max() < 0.03
    assert np.allclose((z ** 2).mean(axis=0), 1 / 3, atol=0.02)


def test_rodrigues_fallback_and_roundtrip():
    q = np.array([[0.0, 0.0, 0.0, 1.0]])  # 180 degrees about z
    rho = synth.quaternion_to_rodrigues(q)
    assert np.allclose(rho, [[0, 0, 1e9]])
    R = synth.rodrigues_to_rotation(rho)[0]
    assert np.allclose(R, np.diag([-1, -1, 1]), atol=1e-8)
    # 90 degrees about x: rho = tan(45 deg) e_x
    R = synth.rodrigues_to_rotation(np.array([[1.0, 0, 0]]))[0]
    assert np.allclose(R @ [0, 1, 0], [0, 0, 1])


def test_isotropic_stiffness_unchanged_by_rotation_and_cubic_by_90deg():
    Ci = synth.isotropic_stiffness(200.0, 0.3)
    R = synth.random_rotations(synth.rng_for(5), 3)
    assert np.allclose(synth.rotate_stiffness(Ci, R), Ci[None], atol=1e-10)
    Cc = synth.cubic_stiffness(206, 133, 119)
    Rz = np.array([[0.0, -1, 0], [1, 0, 0], [0, 0, 1]])
    assert np.allclose(synth.rotate_stiffness(Cc, Rz), Cc, atol=1e-12)


@pytest.mark.parametrize("n", [32, 64])
def test_serving_request_recipe(n):
    for seed in range(40):
        ms = synth.serving_request(seed)
        if ms.shape[0] == n:
            assert ms.meta["n_grains"] == n ** 3 // 2000
            assert 1 <= ms.nrhs <= 6
            assert ms.void_fraction() < 0.03
            return
    pytest.skip("no request of that size in the first seeds")


def test_void_sphere_is_the_papers_timing_case():
    """Sec. 3.1: E = 194 GPa, nu = 0.2934 around a zero-stiffness spherical
    void of radius 2 um in a 50 um cube (0.04 of the edge), eps_33 = 1e-3.
    The void is every voxel whose centre lies within the radius, counted here
    by brute force."""
    n = 50
    ms = synth.workload("void500", scale=n)
    assert ms.shape == (n, n, n) and ms.nphase == 2
    r = 0.04 * n
    c = (np.arange(n) + 0.5 - n / 2.0) ** 2
    inside = (c[:, None, None] + c[None, :, None] + c[None, None, :]) <= r * r
    assert np.array_equal(ms.phase.reshape(n, n, n) == 1, inside)
    assert np.all(ms.C[1] == 0.0)
    lam = 194.0 * 0.2934 / ((1 + 0.2934) * (1 - 2 * 0.2934))
    mu = 194.0 / (2 * (1 + 0.2934))
    assert np.isclose(ms.C[0][2, 2], lam + 2 * mu) and np.isclose(ms.C[0][3, 3], mu)
    assert np.isclose(ms.C[0][0, 1], lam)
    assert np.array_equal(ms.strain, [[0, 0, 1e-3, 0, 0, 0]])
