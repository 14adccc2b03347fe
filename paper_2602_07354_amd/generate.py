"""Polycrystal microstructures generated on the GPU (Sec. 2.2).

Draws the same random stream as ``synth.polycrystal`` (grain seeds, grain
rotations, then the pores of each population one by one), but assigns the
grains (``elas3d_generate_grains``) and carves the pores
(``elas3d_carve_pores``) with the library's kernels.  The pore populations
keep their sequential rule (each adds pores until the running void fraction
reaches its running target): candidates are drawn in batches, the device
finds how many of them the rule uses, and the random generator is rewound to
the state after the last used pore before the next population.
"""

from __future__ import annotations

from typing import Optional, Sequence

import numpy as np

from . import elas3d as E
from . import synth


def _pore_rows(cands) -> np.ndarray:
    rows = np.empty((len(cands), E.PORE_STRIDE))
    for q, (c, a, R) in enumerate(cands):
        rows[q, 0:3] = c
        rows[q, 3:6] = a
        rows[q, 6:15] = (np.eye(3) if R is None else R).reshape(9)
    return rows


def polycrystal(shape: Sequence[int], n_grains: int, seed: int, pores: Sequence[dict] = (),
                strain: Optional[np.ndarray] = None, cubic: Sequence[float] = synth.SS316L_CUBIC,
                phase=None, batch: int = 4096) -> synth.Microstructure:
    """The ``synth.polycrystal`` recipe with grain assignment and pore carving
    on the device.  ``phase``: optional device buffer of N int32 to fill
    (the Microstructure then holds it instead of a host array)."""
    nx, ny, nz = (int(s) for s in shape)
    N = nx * ny * nz
    rng = synth.rng_for(seed)
    box = np.array([nx, ny, nz], dtype=np.float64)
    seeds = rng.random((n_grains, 3)) * box
    opts = E.options_init(outputs_on_device=1 if phase is not None else 0)
    phase = E.generate_grains((nx, ny, nz), seeds, None, phase, opts)
    R = synth.random_rotations(rng, n_grains)
    C = np.zeros((n_grains + 1, 6, 6))
    C[:n_grains] = synth.rotate_stiffness(synth.cubic_stiffness(*cubic), R)
    void_id = n_grains
    target = 0.0
    n_void = 0
    counts = {}
    carved = []  # rows of the pores carved, in order
    for pop in pores:
        target += float(pop["fraction"])
        added = 0
        while n_void < target * N:
            states, cands = [], []
            for _ in range(batch):
                states.append(rng.bit_generator.state)
                cands.append(synth.draw_pore(rng, pop, box))
            rows = _pore_rows(cands)
            used, n_void = E.carve_pores((nx, ny, nz), phase, void_id, rows, target * N, opts)
            added += used
            carved.append(rows[:used])
            if used < len(cands):
                rng.bit_generator.state = states[used]  # the stream after the last used pore
                break
        counts[pop["kind"]] = counts.get(pop["kind"], 0) + added
    if strain is None:
        strain = np.array([[1e-3, 0, 0, 0, 0, 0]], dtype=np.float64)
    strain = np.atleast_2d(np.asarray(strain, dtype=np.float64))
    return synth.Microstructure((nx, ny, nz), phase, C, strain,
                                {"n_grains": n_grains, "seed": seed, "pores": counts,
                                 "void_fraction": n_void / N, "generated_on": "device",
                                 "seeds": seeds,
                                 "pores_carved": np.concatenate(carved) if carved else np.empty((0, 15))})


def workload(name: str, scale: Optional[int] = None, nrhs: Optional[int] = None,
             phase=None) -> synth.Microstructure:
    """Named polycrystal workload (``synth.workload`` recipes) generated on the device."""
    rec = synth.workload_recipe(name, scale)
    strain = np.array(rec["strain"], dtype=np.float64)
    if nrhs is not None:
        strain = strain[:nrhs]
    ms = polycrystal(rec["shape"], rec["n_grains"], rec["seed"], rec["pores"], strain, phase=phase)
    ms.meta["workload"] = name if scale is None else f"{name}@{scale}^3"
    return ms


def serving_request(seed: int) -> synth.Microstructure:
    """One request of the serving stream (``synth.serving_recipe``) generated
    on the device (host phase array)."""
    rec = synth.serving_recipe(seed)
    ms = polycrystal(rec["shape"], rec["n_grains"], rec["seed"], rec["pores"], rec["strain"])
    ms.meta["workload"] = rec["workload"]
    return ms
