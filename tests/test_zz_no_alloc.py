"""The allocation-free grain assignment (elas3d_generate_grains_static)
against the allocating one, through the C-ABI: bit-identical grain maps on
two calls in a row, the second with a smaller grid and fewer grains (the
static work area keeps the first call's contents), plus its argument limits."""

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


def _seeds(shape, ngrain, seed, weighted):
    rng = np.random.default_rng(seed)
    seeds = rng.random((ngrain, 3)) * np.array(shape, dtype=float)
    semi = np.stack([0.7 + rng.random(ngrain), 0.7 + 2.0 * rng.random(ngrain)], axis=1) if weighted else None
    return seeds, semi


def test_static_grain_assignment_equals_the_allocating_one(E):
    import torch
    dev = torch.device("cuda:0")
    opts = E.options_init(outputs_on_device=1, device=0)
    # two calls in a row, the second smaller (fewer grains and cells): it must
    # not see the first call's leftovers in the shared work area
    for shape, ngrain, seed, weighted in [((96, 80, 72), 4000, 1, True), ((37, 29, 41), 150, 2, False),
                                          ((128, 128, 128), 65536, 3, False)]:
        say("case: static grain assignment", shape, ngrain, "weighted" if weighted else "voronoi")
        seeds, semi = _seeds(shape, ngrain, seed, weighted)
        n = int(np.prod(shape))
        ref = E.generate_grains(shape, seeds, semi)  # allocating entry point, host output
        out = torch.full((n,), -7, dtype=torch.int32, device=dev)
        E.generate_grains_static(shape, seeds, semi, out, opts)
        got = out.cpu().numpy()
        assert np.array_equal(got, ref)
        assert got.min() >= 0 and got.max() < ngrain


def test_static_grain_assignment_limits(E):
    import torch
    out = torch.empty(8 * 8 * 8, dtype=torch.int32, device="cuda:0")
    seeds = np.full((3, 3), 1.5)
    with pytest.raises(E.Elas3dError) as ei:  # host output is not supported
        E.generate_grains_static((8, 8, 8), seeds, None, out, E.options_init(outputs_on_device=0))
    assert ei.value.code == E.EBADARG and "outputs_on_device" in str(ei.value)
    big = np.random.default_rng(0).random((65537, 3)) * 64
    out2 = torch.empty(64 ** 3, dtype=torch.int32, device="cuda:0")
    with pytest.raises(E.Elas3dError) as ei:
        E.generate_grains_static((64, 64, 64), big, None, out2, E.options_init(outputs_on_device=1))
    assert ei.value.code == E.EBADARG and "65536" in str(ei.value)
