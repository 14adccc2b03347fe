"""Seeded synthetic microstructures for the periodic voxel elasticity solve.

This module makes the inputs of a solve and nothing else: a phase map, one
6x6 stiffness per phase and the applied macroscopic strains.  It holds none
of the solver's arithmetic (element stiffness, load vector, operator,
preconditioner, conjugate gradients, stress).  Both the HIP library and the
CPU oracle consume what it produces.

Conventions shared with the C-ABI:

* Grid: ``nx, ny, nz`` voxels, periodic in all three directions.  Voxel
  ``(i, j, k)`` is flattened as ``m = i + nx*(j + ny*k)`` (x fastest); its
  centre is at ``(i+1/2, j+1/2, k+1/2)`` in voxel units.
* Stiffness: 6x6 Voigt matrix in the order (11, 22, 33, 23, 13, 12) that
  maps engineering strain (shear components doubled) to stress.  A phase
  whose 36 entries are all zero is void.
* Strain: tensor components (E11, E22, E33, E23, E13, E12).

Paper passages followed (ELAS3D-Xtal, arXiv 2602.07354):

* isotropic stiffness from (E, nu): Sec. 2.1.1, Eq. (2)-(3);
* cubic crystal stiffness and its rotation by a Rodrigues vector through a
  Bond matrix: Sec. 2.1.1, Eq. (anisotropic_rotation) and Algorithm 1;
* random orientations by Shoemake's method, quaternion -> Rodrigues with
  the 1e9 fallback when |q_w| < 1e-8: Sec. 2.2.3, its quaternion equation
  and Algorithm 6 (random branch);
* nearest-seed grain assignment: Sec. 2.2.2, Eq. (ellipsoid_dist) with equal
  semi-axes (plain Voronoi), made periodic by the minimum-image distance;
* pore overwrite with one shared void id, "inside" meaning distance <= r:
  Sec. 2.2.3, Algorithm 5 (extended to ellipsoids).
"""

from __future__ import annotations

import dataclasses
import math
import os
from typing import Optional, Sequence

import numpy as np

__all__ = [
    "Microstructure",
    "isotropic_stiffness",
    "cubic_stiffness",
    "shoemake_quaternions",
    "quaternion_to_rodrigues",
    "rodrigues_to_rotation",
    "bond_stress_matrix",
    "rotate_stiffness",
    "random_rotations",
    "periodic_voronoi",
    "carve_spheres", "draw_pore", "workload_recipe",
    "carve_ellipsoids",
    "eshelby_inclusion",
    "polycrystal",
    "workload",
    "WORKLOADS",
    "unit_load_cases",
    "rng_for",
    "indefinite_grid",
    "serving_recipe",
]

SS316L_CUBIC = (206.0, 133.0, 119.0)  # C11, C12, C44 in GPa (Table 5)


@dataclasses.dataclass
class Microstructure:
    """Inputs of one solve (see module docstring for layouts)."""

    shape: tuple  # (nx, ny, nz)
    phase: np.ndarray  # int32, nx*ny*nz, x fastest
    C: np.ndarray  # float64, (nphase, 6, 6)
    strain: np.ndarray  # float64, (nrhs, 6) tensor components
    meta: dict

    @property
    def n(self) -> int:
        nx, ny, nz = self.shape
        return nx * ny * nz

    @property
    def nphase(self) -> int:
        return int(self.C.shape[0])

    @property
    def nrhs(self) -> int:
        return int(self.strain.shape[0])

    def void_fraction(self) -> float:
        void = np.all(self.C.reshape(self.nphase, 36) == 0.0, axis=1)
        return float(void[self.phase].mean())


def rng_for(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(int(seed)))


# ---------------------------------------------------------------- stiffness

def isotropic_stiffness(E: float, nu: float) -> np.ndarray:
    """Voigt 6x6 of the isotropic tensor with Lame constants of Eq. (2)-(3)."""
    lam = E * nu / ((1.0 + nu) * (1.0 - 2.0 * nu))
    mu = E / (2.0 * (1.0 + nu))
    C = np.zeros((6, 6))
    C[:3, :3] = lam
    C[0, 0] = C[1, 1] = C[2, 2] = lam + 2.0 * mu
    C[3, 3] = C[4, 4] = C[5, 5] = mu
    return C


def cubic_stiffness(C11: float, C12: float, C44: float) -> np.ndarray:
    """Crystal-frame cubic stiffness (Algorithm 1, step 1)."""
    C = np.zeros((6, 6))
    C[:3, :3] = C12
    C[0, 0] = C[1, 1] = C[2, 2] = C11
    C[3, 3] = C[4, 4] = C[5, 5] = C44
    return C


# ---------------------------------------------------------------- orientations

def shoemake_quaternions(rng: np.random.Generator, n: int) -> np.ndarray:
    """Uniform unit quaternions, labelled (q_w, q_x, q_y, q_z) as in Algorithm 6."""
    u1, u2, u3 = rng.random(n), rng.random(n), rng.random(n)
    a, b = np.sqrt(1.0 - u1), np.sqrt(u1)
    return np.stack(
        [a * np.sin(2 * np.pi * u2), a * np.cos(2 * np.pi * u2),
         b * np.sin(2 * np.pi * u3), b * np.cos(2 * np.pi * u3)], axis=1)


def quaternion_to_rodrigues(q: np.ndarray) -> np.ndarray:
    """rho = q_xyz / q_w, or q_xyz * 1e9 when |q_w| < 1e-8 (Algorithm 6)."""
    q = np.atleast_2d(np.asarray(q, dtype=np.float64))
    qw, qv = q[:, 0], q[:, 1:]
    small = np.abs(qw) < 1e-8
    safe = np.where(small, 1.0, qw)
    return np.where(small[:, None], qv * 1e9, qv / safe[:, None])


def rodrigues_to_rotation(rho: np.ndarray) -> np.ndarray:
    """Active rotation matrix of a Rodrigues vector tan(theta/2) n.

    R = I + 2/(1 + rho.rho) ([rho]_x + [rho]_x^2), which is the Euler-Rodrigues
    formula with sin(theta) and 1-cos(theta) written through tan(theta/2).
    """
    rho = np.atleast_2d(np.asarray(rho, dtype=np.float64))
    n = rho.shape[0]
    K = np.zeros((n, 3, 3))
    K[:, 0, 1], K[:, 0, 2] = -rho[:, 2], rho[:, 1]
    K[:, 1, 0], K[:, 1, 2] = rho[:, 2], -rho[:, 0]
    K[:, 2, 0], K[:, 2, 1] = -rho[:, 1], rho[:, 0]
    f = 2.0 / (1.0 + np.einsum("ni,ni->n", rho, rho))
    return np.eye(3)[None] + f[:, None, None] * (K + K @ K)


_VOIGT_PAIRS = ((0, 0), (1, 1), (2, 2), (1, 2), (0, 2), (0, 1))


def bond_stress_matrix(R: np.ndarray) -> np.ndarray:
    """6x6 Bond matrix M with sigma'_V = M sigma_V for sigma' = R sigma R^T.

    Voigt order (11, 22, 33, 23, 13, 12); stress components are not scaled.
    """
    R = np.asarray(R, dtype=np.float64)
    M = np.zeros(R.shape[:-2] + (6, 6))
    for I, (i, j) in enumerate(_VOIGT_PAIRS):
        for J, (k, l) in enumerate(_VOIGT_PAIRS):
            if k == l:
                M[..., I, J] = R[..., i, k] * R[..., j, l]
            else:
                M[..., I, J] = R[..., i, k] * R[..., j, l] + R[..., i, l] * R[..., j, k]
    return M


def rotate_stiffness(C_local: np.ndarray, R: np.ndarray) -> np.ndarray:
    """Sample-frame stiffness M C M^T for active rotation(s) R (crystal -> sample).

    The paper writes the product as Q C Q^T in Eq. (anisotropic_rotation) and
    as M^T C M in Algorithm 1; with M the Bond stress matrix of the active
    rotation, M C M^T is the tensor rotation C'_ijkl = R_ip R_jq R_kr R_ls C_pqrs.
    """
    M = bond_stress_matrix(R)
    C = M @ C_local @ np.swapaxes(M, -1, -2)
    return 0.5 * (C + np.swapaxes(C, -1, -2))


def random_rotations(rng: np.random.Generator, n: int) -> np.ndarray:
    """Uniform SO(3) samples via Shoemake -> Rodrigues -> matrix."""
    return rodrigues_to_rotation(quaternion_to_rodrigues(shoemake_quaternions(rng, n)))


# ---------------------------------------------------------------- geometry

def _workers() -> int:
    return max(1, min(16, os.cpu_count() or 1))


def periodic_voronoi(shape: Sequence[int], seeds: np.ndarray,
                     slab: int = 1 << 22) -> np.ndarray:
    """Nearest-seed id per voxel centre under the periodic minimum-image distance.

    Equal semi-axes turn Eq. (ellipsoid_dist) into Euclidean distance; exact
    ties (measure zero for continuous seeds) would go to the lower seed index.
    """
    from scipy.spatial import cKDTree

    nx, ny, nz = (int(s) for s in shape)
    box = np.array([nx, ny, nz], dtype=np.float64)
    tree = cKDTree(np.mod(seeds, box), boxsize=box)
    plane = nx * ny
    kz = max(1, slab // plane)
    out = np.empty(nx * ny * nz, dtype=np.int32)
    xi = (np.arange(nx) + 0.5)
    yj = (np.arange(ny) + 0.5)
    X, Y = np.meshgrid(xi, yj, indexing="xy")
    X, Y = X.ravel(), Y.ravel()
    for k0 in range(0, nz, kz):
        k1 = min(nz, k0 + kz)
        nk = k1 - k0
        pts = np.empty((nk * plane, 3))
        pts[:, 0] = np.tile(X, nk)
        pts[:, 1] = np.tile(Y, nk)
        pts[:, 2] = np.repeat(np.arange(k0, k1) + 0.5, plane)
        _, idx = tree.query(pts, k=1, workers=_workers())
        out[k0 * plane:k1 * plane] = idx.astype(np.int32)
    return out


def _min_image(x: np.ndarray, s: float, L: int) -> np.ndarray:
    """Minimum-image offset of voxel centres x from s, rounded once:
    x - s, or (x -+ L) - s when |x - s| > L/2."""
    d = x - s
    return np.where(d > 0.5 * L, (x - L) - s, np.where(d < -0.5 * L, (x + L) - s, d))


def _box_offsets(shape, centre, half):
    """Voxel indices (wrapped) near a point and the minimum-image offsets of
    their centres."""
    axes = []
    for d in range(3):
        n = shape[d]
        lo = int(math.floor(centre[d] - half[d] - 0.5))
        hi = int(math.ceil(centre[d] + half[d] - 0.5))
        idx = np.arange(n) if hi - lo + 1 >= n else np.mod(np.arange(lo, hi + 1), n)
        axes.append((idx, _min_image(idx + 0.5, float(centre[d]), n)))
    return axes


def carve_ellipsoids(phase: np.ndarray, shape: Sequence[int], centres: np.ndarray,
                     semi_axes: np.ndarray, rotations: Optional[np.ndarray],
                     void_id: int) -> int:
    """Overwrite voxels whose centre lies in an ellipsoid (<= 1) with ``void_id``.

    ``rotations[p]`` maps the ellipsoid's own axes to the sample frame; None
    means axis-aligned.  Distances use the periodic minimum image.  Returns
    the number of voxels that were not void before.
    """
    nx, ny, nz = (int(s) for s in shape)
    view = phase.reshape(nz, ny, nx)
    fresh = 0
    for p in range(len(centres)):
        c = centres[p]
        ax = np.asarray(semi_axes[p], dtype=np.float64)
        half = np.full(3, ax.max())
        (ix, dx), (iy, dy), (iz, dz) = _box_offsets((nx, ny, nz), c, half)
        d0, d1, d2 = np.meshgrid(dx, dy, dz, indexing="ij")  # [x, y, z]
        R = np.eye(3) if rotations is None else np.asarray(rotations[p], dtype=np.float64)
        # offsets in the ellipsoid's own axes, each product and sum rounded on
        # its own (the order fixed by the pore-overwrite definition)
        s = None
        for j in range(3):
            q = ((d0 * R[0, j] + d1 * R[1, j]) + d2 * R[2, j]) / ax[j]
            s = q * q if s is None else s + q * q
        inside = (s <= 1.0 + 1e-12).transpose(2, 1, 0)  # [z, y, x]
        if inside.any():
            sub = view[np.ix_(iz, iy, ix)]
            fresh += int(np.count_nonzero(sub[inside] != void_id))
            sub[inside] = void_id
            view[np.ix_(iz, iy, ix)] = sub
    return fresh


def carve_spheres(phase, shape, centres, radii, void_id) -> int:
    radii = np.asarray(radii, dtype=np.float64)
    return carve_ellipsoids(phase, shape, centres, np.repeat(radii[:, None], 3, axis=1),
                     None, void_id)


# ---------------------------------------------------------------- workloads

def unit_load_cases(magnitude: float = 1e-3) -> np.ndarray:
    """Six homogenisation load cases: Voigt unit strains times ``magnitude``.

    Shear cases have engineering shear ``magnitude``, i.e. tensor component
    E_ij = E_ji = magnitude / 2.
    """
    E = np.zeros((6, 6))
    for c in range(3):
        E[c, c] = magnitude
    for c in range(3, 6):
        E[c, c] = 0.5 * magnitude
    return E


def eshelby_inclusion(n: int = 20, radius: Optional[float] = None,
                      E_m: float = 200.0, nu_m: float = 0.3,
                      E_i: float = 400.0, nu_i: float = 0.25,
                      strain: Sequence[float] = (1e-3, 0, 0, 0, 0, 0)) -> Microstructure:
    """Isotropic matrix (phase 0) with one centred spherical inclusion (phase 1)."""
    r = n / 4.0 if radius is None else float(radius)
    c = n / 2.0
    idx = np.arange(n) + 0.5 - c
    Z, Y, X = np.meshgrid(idx, idx, idx, indexing="ij")
    inside = (X * X + Y * Y + Z * Z) <= r * r
    phase = inside.astype(np.int32).ravel()
    C = np.stack([isotropic_stiffness(E_m, nu_m), isotropic_stiffness(E_i, nu_i)])
    return Microstructure((n, n, n), phase, C, np.array([strain], dtype=np.float64),
                          {"workload": f"eshelby_{n}", "inclusion_voxels": int(inside.sum()),
                           "radius": r})


def void_sphere(n: int = 500) -> Microstructure:
    """The paper's Eshelby benchmark, timed in its Table 4 (Sec. 3.1): an
    isotropic matrix (E = 194 GPa, nu = 0.2934) around a centred spherical
    void of radius 0.04 n voxels (2 um in a 50 um cube at 500^3), strained
    1e-3 along X3.  The void is phase 1 with C = 0."""
    ms = eshelby_inclusion(n, radius=0.04 * n, E_m=194.0, nu_m=0.2934, E_i=0.0, nu_i=0.0,
                           strain=(0, 0, 1e-3, 0, 0, 0))
    ms.meta["workload"] = f"void{n}"
    return ms


def indefinite_grid(shape: Sequence[int], seed: int, neg_fraction: float, e_neg: float) -> Microstructure:
    """Two isotropic phases (E = 200 and 120 GPa) mixed voxel by voxel, with a
    fraction of voxels of a third phase whose stiffness is the negative of an
    isotropic one (-C(e_neg, 0.3)).  Such a C is symmetric and finite, so setup
    accepts it, but the operator is indefinite: a test input for the step-size
    breakdown of Algorithm 2 (h.Ah <= 0)."""
    rng = rng_for(seed)
    n = int(np.prod(shape))
    C = np.stack([isotropic_stiffness(200.0, 0.3), isotropic_stiffness(120.0, 0.25),
                  -isotropic_stiffness(float(e_neg), 0.3)])
    phase = (rng.random(n) < 0.5).astype(np.int32)
    phase[rng.random(n) < neg_fraction] = 2
    return Microstructure(tuple(int(v) for v in shape), phase, C,
                          np.array([[1e-3, 0, 0, 0, 0, 0]], dtype=np.float64),
                          {"workload": f"indefinite_{seed}", "neg_voxels": int((phase == 2).sum())})


def _lognormal_radii(rng, median, sigma, n):
    return median * np.exp(sigma * rng.standard_normal(n))


def draw_pore(rng: np.random.Generator, pop: dict, box: np.ndarray):
    """Next pore of a population: (centre, semi-axes, rotation or None).

    The draws (centre, then the shape's own) are the whole random stream of
    a pore, so a generator that carves on the device can replay it."""
    kind = pop["kind"]
    c = rng.random(3) * box
    if kind == "sphere":
        r = float(_lognormal_radii(rng, pop.get("median", 2.0), pop.get("sigma", 0.4), 1)[0])
        return c, np.array([r, r, r]), None
    if kind == "oblate":
        return c, np.asarray(pop.get("axes", (4.0, 4.0, 1.0)), dtype=np.float64), random_rotations(rng, 1)[0]
    if kind == "prolate_z":
        return c, np.asarray(pop.get("axes", (5.0 / 3.0, 5.0 / 3.0, 5.0)), dtype=np.float64), None
    raise ValueError(f"unknown pore kind {kind!r}")


def polycrystal(shape: Sequence[int], n_grains: int, seed: int,
                pores: Sequence[dict] = (), strain: Optional[np.ndarray] = None,
                cubic: Sequence[float] = SS316L_CUBIC) -> Microstructure:
    """Periodic Voronoi polycrystal of rotated cubic grains with void pores.

    ``pores`` is a list of populations, each a dict with ``kind`` in
    {"sphere", "oblate", "prolate_z"} and ``fraction`` (target void fraction
    added by that population; populations are carved in order and each adds
    pores until the running void fraction reaches the running target).
    Sphere populations take ``median`` and ``sigma`` of a lognormal radius.
    Grain ids are 0..n_grains-1; the void id is n_grains.
    """
    nx, ny, nz = (int(s) for s in shape)
    rng = rng_for(seed)
    box = np.array([nx, ny, nz], dtype=np.float64)
    seeds = rng.random((n_grains, 3)) * box
    phase = periodic_voronoi((nx, ny, nz), seeds)
    R = random_rotations(rng, n_grains)
    C = np.zeros((n_grains + 1, 6, 6))
    C[:n_grains] = rotate_stiffness(cubic_stiffness(*cubic), R)
    void_id = n_grains
    N = nx * ny * nz
    target = 0.0
    n_void = 0
    counts = {}
    for pop in pores:
        target += float(pop["fraction"])
        kind = pop["kind"]
        added = 0
        while n_void < target * N:
            c, a, Q = draw_pore(rng, pop, box)
            n_void += carve_ellipsoids(phase, (nx, ny, nz), c[None], a[None],
                                       None if Q is None else Q[None], void_id)
            added += 1
        counts[kind] = counts.get(kind, 0) + added
    if strain is None:
        strain = np.array([[1e-3, 0, 0, 0, 0, 0]], dtype=np.float64)
    strain = np.atleast_2d(np.asarray(strain, dtype=np.float64))
    return Microstructure((nx, ny, nz), phase, C, strain,
                          {"n_grains": n_grains, "seed": seed, "pores": counts,
                           "void_fraction": n_void / N})


def _poly_recipe(name: str):
    """Recipes of the synthetic workloads (grid, grains, pores, load)."""
    if name == "poly100":
        return dict(shape=(100, 100, 100), n_grains=500, seed=2000,
                    pores=[dict(kind="sphere", fraction=0.01, median=2.0, sigma=0.4)],
                    strain=[[1e-3, 0, 0, 0, 0, 0]])
    if name == "poly300":
        return dict(shape=(300, 300, 300), n_grains=3000, seed=3000,
                    pores=[dict(kind="sphere", fraction=0.005, median=2.0, sigma=0.4),
                           dict(kind="oblate", fraction=0.005, axes=(4.0, 4.0, 1.0))],
                    strain=unit_load_cases())
    if name in ("poly500", "poly800"):
        n = 500 if name == "poly500" else 800
        grains = 8000 if n == 500 else 32768
        return dict(shape=(n, n, n), n_grains=grains, seed=5000 + n,
                    pores=[dict(kind="sphere", fraction=0.02 / 3, median=3.0, sigma=0.4),
                           dict(kind="oblate", fraction=0.02 / 3, axes=(4.0, 4.0, 1.0)),
                           dict(kind="prolate_z", fraction=0.02 / 3,
                                axes=(5.0 / 3.0, 5.0 / 3.0, 5.0))],
                    strain=[[0, 0, 1e-3, 0, 0, 0]])
    raise KeyError(name)


WORKLOADS = ("eshelby20", "poly100", "poly300", "poly500", "poly800", "void500")


def workload_recipe(name: str, scale: Optional[int] = None) -> dict:
    """Recipe of a polycrystal workload; ``scale`` re-sizes it to ``scale``^3
    voxels keeping its grain density and pore recipe."""
    rec = _poly_recipe(name)
    if scale is not None:
        n0 = rec["shape"][0]
        rec["n_grains"] = max(1, int(round(rec["n_grains"] * (scale / n0) ** 3)))
        rec["shape"] = (scale, scale, scale)
        rec["seed"] = rec["seed"] + scale
    return rec


def workload(name: str, scale: Optional[int] = None, nrhs: Optional[int] = None) -> Microstructure:
    """Named synthetic workload; ``scale`` re-sizes a polycrystal to ``scale``^3
    voxels keeping its grain density and pore recipe (for bounded samples)."""
    if name == "eshelby20":
        return eshelby_inclusion(20)
    if name == "void500":
        return void_sphere(500 if scale is None else scale)
    rec = workload_recipe(name, scale)
    strain = np.array(rec["strain"], dtype=np.float64)
    if nrhs is not None:
        strain = strain[:nrhs]
    ms = polycrystal(rec["shape"], rec["n_grains"], rec["seed"], rec["pores"], strain)
    ms.meta["workload"] = name if scale is None else f"{name}@{scale}^3"
    return ms


def serving_recipe(seed: int) -> dict:
    """Draws of one request of the serving stream: grid edge uniform over
    {32, 64, 96, 128}, grain count voxels/2000, porosity U[0, 2%] spheres,
    1-6 load cases (the arguments of ``polycrystal``)."""
    rng = rng_for(seed)
    n = int(rng.choice([32, 64, 96, 128]))
    grains = max(1, (n ** 3) // 2000)
    por = float(rng.uniform(0.0, 0.02))
    nrhs = int(rng.integers(1, 7))
    return {"shape": (n, n, n), "n_grains": grains, "seed": seed * 7919 + 1,
            "pores": [dict(kind="sphere", fraction=por, median=2.0, sigma=0.4)],
            "strain": unit_load_cases()[:nrhs], "workload": f"serving_{n}"}


def serving_request(seed: int) -> Microstructure:
    """One request of the serving stream (``serving_recipe``), built on the host."""
    rec = serving_recipe(seed)
    ms = polycrystal(rec["shape"], rec["n_grains"], rec["seed"], rec["pores"], rec["strain"])
    ms.meta["workload"] = rec["workload"]
    return ms
