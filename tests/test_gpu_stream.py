"""Streaming-bandwidth probe (elas3d_stream_bandwidth): plain and non-temporal
copy, read and write kernels run on the device and report finite rates of
the right order (a sanity check of the figure the benchmark divides by)."""

import math

import pytest

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)


@pytest.fixture(scope="module")
def E():
    from paper_2602_07354_amd import elas3d
    elas3d.lib()
    return elas3d


def test_stream_probe_rates(E):
    import torch
    for nt in (False, True):
        say("case: stream probe, 256 MiB, 4096 workgroups, nontemporal", nt)
        r = E.stream_bandwidth(256 << 20, blocks=4096, reps=3, nontemporal=nt)
        say("  ", r)
        for k in ("copy", "read", "write"):
            assert math.isfinite(r[k]) and 100.0 < r[k] < 50000.0, (k, r[k])
    # on a caller's stream, with the smallest buffer and grid allowed
    say("case: stream probe on the current torch stream, 1 MiB, 1 workgroup")
    opts = E.options_init(device=0)
    opts.stream = torch.cuda.current_stream().cuda_stream
    r = E.stream_bandwidth(1 << 20, blocks=1, reps=1, options=opts)
    assert all(math.isfinite(v) and v > 0.0 for v in r.values())
    torch.cuda.synchronize()
