"""C-ABI checks that need no GPU: the library loads, exports every symbol the
header declares, the ctypes structs match the C layout, and argument
validation rejects bad input before any device call."""

import ctypes
import os
import re
import subprocess

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "elas3d.h")


@pytest.fixture(scope="module")
def E():
    from paper_2602_07354_amd import elas3d
    elas3d.lib()
    return elas3d


def test_library_exports_every_declared_symbol(E):
    text = open(HEADER).read()
    declared = set(re.findall(r"\b(elas3d_[a-z_]+)\s*\(", text))
    assert declared, "no declarations found"
    assert declared == set(E.EXPORTS)
    L = E.lib()
    for name in declared:
        assert hasattr(L, name), name
    assert "gfx950" in E.version()


def test_struct_layout_matches_c(E, tmp_path):
    src = tmp_path / "layout.c"
    src.write_text(
        '#include <stdio.h>\n#include <stddef.h>\n#include "elas3d.h"\n'
        "int main(void){\n"
        'printf("%zu %zu %zu %zu %zu %zu\\n", sizeof(elas3d_options), offsetof(elas3d_options, hbm_budget_bytes),'
        " offsetof(elas3d_options, stream), offsetof(elas3d_options, graphs),"
        " sizeof(elas3d_info), offsetof(elas3d_info, relres_true));\n"
        'printf("%zu %zu %zu %zu %zu %zu\\n", offsetof(elas3d_info, t_operator_ms), offsetof(elas3d_info, n_update),'
        ' offsetof(elas3d_info, fp64_fallback), offsetof(elas3d_info, op_tile),'
        ' offsetof(elas3d_info, update_blocks), offsetof(elas3d_options, autotune));\n'
        'printf("%zu %zu %zu %zu\\n", offsetof(elas3d_options, tile), offsetof(elas3d_options, zchunk),'
        ' offsetof(elas3d_info, precond_rows), offsetof(elas3d_info, update_nontemporal));\n'
        'printf("%zu %zu %zu %zu\\n", offsetof(elas3d_options, update_blocks),'
        ' offsetof(elas3d_options, update_nontemporal), offsetof(elas3d_info, apply_tile),'
        ' offsetof(elas3d_info, op_shape));\n'
        "return 0;}\n")
    exe = tmp_path / "layout"
    subprocess.check_call(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)])
    out = subprocess.check_output([str(exe)]).decode().split()
    c = [int(v) for v in out]
    py = [ctypes.sizeof(E.Options), E.Options.hbm_budget_bytes.offset, E.Options.stream.offset,
          E.Options.graphs.offset, ctypes.sizeof(E.Info), E.Info.relres_true.offset,
          E.Info.t_operator_ms.offset, E.Info.n_update.offset, E.Info.fp64_fallback.offset,
          E.Info.op_tile.offset, E.Info.update_blocks.offset, E.Options.autotune.offset,
          E.Options.tile.offset, E.Options.zchunk.offset, E.Info.precond_rows.offset,
          E.Info.update_nontemporal.offset, E.Options.update_blocks.offset,
          E.Options.update_nontemporal.offset, E.Info.apply_tile.offset, E.Info.op_shape.offset]
    assert c == py


def _good():
    from paper_2602_07354_amd import synth
    C = np.stack([synth.isotropic_stiffness(200, .3), np.zeros((6, 6))])
    phase = np.zeros(4 * 4 * 4, np.int32)
    strain = np.array([[1e-3, 0, 0, 0, 0, 0]])
    return (4, 4, 4), phase, C, strain


@pytest.mark.parametrize("mutate,needle", [
    (lambda a: a.update(shape=(1, 4, 4)), "grid dimensions"),
    (lambda a: a.update(phase=None), "phase is NULL"),
    (lambda a: a.update(C=np.zeros((0, 6, 6))), "nphase"),
    (lambda a: a.update(strain=np.zeros((7, 6))), "nrhs"),
    (lambda a: a["phase"].__setitem__(5, 2), "out of range"),
    (lambda a: a["phase"].__setitem__(5, -1), "out of range"),
    (lambda a: a["C"].__setitem__((0, 0, 1), np.nan), "not finite"),
    (lambda a: a["C"].__setitem__((0, 0, 1), 1.0), "not symmetric"),
    (lambda a: a["strain"].__setitem__((0, 2), np.inf), "strain"),
])
def test_setup_rejects_bad_arguments(E, mutate, needle):
    shape, phase, C, strain = _good()
    args = {"shape": shape, "phase": phase, "C": C, "strain": strain}
    mutate(args)
    if args["phase"] is None:
        h = ctypes.c_void_p()
        rc = E.lib().elas3d_setup(ctypes.byref(h), 4, 4, 4, None, 2, args["C"].ctypes.data, 1,
                                  args["strain"].ctypes.data, None)
        assert rc == E.EBADARG and needle in E.last_error()
        return
    with pytest.raises(E.Elas3dError) as ei:
        E.setup(args["shape"], args["phase"], args["C"], args["strain"])
    assert ei.value.code == E.EBADARG
    assert needle in str(ei.value)


def test_setup_rejects_bad_options(E):
    shape, phase, C, strain = _good()
    for kw in ({"precision": 7}, {"convergence": 3}, {"preconditioner": -1},
               {"poll_interval": -2}, {"hbm_budget_bytes": -1.0}, {"inner_tol": 2.0},
               {"tile": 7}, {"tile": -1}, {"zchunk": -3}, {"update_blocks": -1},
               {"update_blocks": 32769}, {"update_nontemporal": 2}):
        with pytest.raises(E.Elas3dError) as ei:
            E.setup(shape, phase, C, strain, E.options_init(**kw))
        assert ei.value.code == E.EBADARG


def test_setup_rejects_a_forced_shape_the_grid_cannot_run(E):
    """The wave-specialised shapes need rows of whole 16-byte chunks: an odd
    nx (FP64) or one not a multiple of 4 (mixed precision) is refused before
    any device call."""
    from paper_2602_07354_amd import synth
    C = synth.isotropic_stiffness(200, .3)[None]
    strain = np.array([[1e-3, 0, 0, 0, 0, 0]])
    for shape, kw in (((5, 4, 4), {"tile": 5}), ((6, 4, 4), {"tile": 5, "precision": 1})):
        phase = np.zeros(int(np.prod(shape)), np.int32)
        with pytest.raises(E.Elas3dError) as ei:
            E.setup(shape, phase, C, strain, E.options_init(**kw))
        assert ei.value.code == E.EBADARG and "multiple" in str(ei.value)


def test_setup_rejects_the_fp32_only_shape_in_fp64(E):
    """Shape 6 (64x8 lanes + two loaders) is built for the FP32 sweep only:
    forcing it on an FP64 context is refused before any device call."""
    from paper_2602_07354_amd import synth
    C = synth.isotropic_stiffness(200, .3)[None]
    strain = np.array([[1e-3, 0, 0, 0, 0, 0]])
    assert E.WS_FP32_ONLY == (6,) and 6 in E.WS_TILES
    with pytest.raises(E.Elas3dError) as ei:
        E.setup((8, 4, 4), np.zeros(128, np.int32), C, strain, E.options_init(tile=6))
    assert ei.value.code == E.EBADARG and "FP32 sweep only" in str(ei.value)


def test_null_context_calls_are_rejected(E):
    L = E.lib()
    assert L.elas3d_solve(None, 1e-8, 10, 1, None) == E.EBADARG
    assert L.elas3d_stress(None, 0, None, None, None, None) == E.EBADARG
    assert L.elas3d_apply(None, None, None) == E.EBADARG
    L.elas3d_destroy(None)
    assert "ctx is NULL" in E.last_error()


def test_device_bytes_plan(E):
    b1 = E.device_bytes((500, 500, 500), 8001, 1)
    assert 25e9 < b1 < 30e9  # ~220 B per node in FP64 with one load case
    assert E.device_bytes((500, 500, 500), 8001, 6) > b1
    # a flat grid has far more workgroups than z chunks: the partial sums grow
    flat = E.device_bytes((6000, 6000, 2), 2, 1)
    assert flat > 220 * 6000 * 6000 * 2
    # sizes setup would reject
    assert E.device_bytes((1000, 1000, 1000), 2, 1) == 0.0
    # a fixed one-plane z chunking launches a workgroup per tile and plane:
    # its partial sums are part of the plan
    one = E.device_bytes((500, 500, 500), 8001, 1, E.options_init(tile=0, zchunk=1))
    assert one > b1 + 8.0 * 17 * 72 * 500 * 2


def test_generator_rejects_bad_arguments(E):
    seeds = np.array([[1.0, 1.0, 1.0], [2.5, 0.5, 3.9]])
    bad = [
        dict(seeds=np.array([[1.0, 1.0, 4.0]])),              # outside [0, n)
        dict(seeds=np.array([[-0.1, 1.0, 1.0]])),
        dict(seeds=np.empty((0, 3))),                        # no grains
        dict(seeds=seeds, semi=np.array([[1.0, 0.0], [1.0, 1.0]])),
        dict(seeds=seeds, semi=np.array([[1.0, np.nan], [1.0, 1.0]])),
    ]
    for kw in bad:
        with pytest.raises(E.Elas3dError) as ei:
            E.generate_grains((4, 4, 4), kw["seeds"], kw.get("semi"))
        assert ei.value.code == E.EBADARG
    pore = np.concatenate([[1.0, 1.0, 1.0], [1.0, 1.0, 1.0], np.eye(3).ravel()])
    phase = np.zeros(64, np.int32)
    for mutate in (lambda p: p.__setitem__(0, 4.0), lambda p: p.__setitem__(4, 0.0),
                   lambda p: p.__setitem__(8, np.inf)):
        p = pore.copy()
        mutate(p)
        with pytest.raises(E.Elas3dError) as ei:
            E.carve_pores((4, 4, 4), phase, 1, p[None])
        assert ei.value.code == E.EBADARG
    with pytest.raises(E.Elas3dError):
        E.carve_pores((4, 4, 4), phase, 1, pore[None], float("nan"))
    assert E.lib().elas3d_von_mises(None, 0, None, None, None) == E.EBADARG


def test_stream_probe_rejects_bad_arguments(E):
    """Every argument is checked before the probe touches a device."""
    for kw in (dict(nbytes=(1 << 20) - 16), dict(nbytes=(1 << 20) + 8), dict(blocks=0),
               dict(blocks=(1 << 24) + 1), dict(reps=0), dict(reps=10001)):
        args = dict(nbytes=1 << 20, blocks=64, reps=1)
        args.update(kw)
        with pytest.raises(E.Elas3dError) as ei:
            E.stream_bandwidth(**args)
        assert ei.value.code == E.EBADARG
    L = E.lib()
    assert L.elas3d_stream_bandwidth(1 << 20, 64, 1, 2, np.zeros(3).ctypes.data, None) == E.EBADARG
    assert "nontemporal" in E.last_error()
    assert L.elas3d_stream_bandwidth(1 << 20, 64, 1, 0, None, None) == E.EBADARG
    assert "gbs is NULL" in E.last_error()
