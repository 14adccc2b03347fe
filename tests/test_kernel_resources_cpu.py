"""Register, scratch and LDS budgets of the iteration sweeps, from the
compiler's own kernel metadata for gfx950 (cross-compiled on the CPU with the
library's flags).  The sweeps are built to run with no scratch memory and no
vector-register spills, and the wave-specialised shapes to hold one workgroup per CU
(8 wavefronts for 64x6, 10 for the FP32 64x8): a change that breaks one of these (a value whose address
escapes, a larger live range) slows the sweep without changing its results,
so it is caught here."""

import os
import re
import shutil
import subprocess

import pytest

from paper_2602_07354_amd import build as B

HIPCC = B.HIPCC


def _metadata(tmp_path):
    out = str(tmp_path / "kernels.s")
    flags = [f for f in B.FLAGS if f != "-fPIC"]
    cmd = [HIPCC, *flags, "--offload-device-only", "-S", os.path.join(B.CSRC, "elas3d_kernels.hip"), "-o", out]
    r = subprocess.run(cmd, capture_output=True, text=True, timeout=900)
    assert r.returncode == 0, r.stderr[-4000:]
    text = open(out).read()
    kernels = {}
    # the code-object metadata lists each kernel's .name and its resource fields
    for block in re.split(r"\n  - \.", text[text.index("amdhsa.kernels:"):]):
        m = re.search(r"\.name:\s+(\S+)", block)
        if not m:
            continue
        fields = dict(re.findall(r"\.(\w+):\s+(\d+)\n", block))
        kernels[m.group(1)] = {k: int(v) for k, v in fields.items()}
    return kernels


@pytest.mark.skipif(not shutil.which(HIPCC) and not os.path.exists(HIPCC), reason="needs hipcc")
def test_iteration_sweeps_use_no_scratch_and_fit_their_occupancy(tmp_path):
    ks = _metadata(tmp_path)
    sweeps = {n: v for n, v in ks.items() if re.search(r"op_kernel|update_precond_kernel|op_group_kernel|"
                                                       r"update_group_kernel", n)}
    assert len(sweeps) >= 30, sorted(ks)
    for name, v in sweeps.items():
        assert v.get("private_segment_fixed_size", 0) == 0, (name, v)
        # (SGPR spills go to VGPR lanes, not to memory, and are allowed)
        assert v.get("vgpr_spill_count", 0) == 0, (name, v)
        assert v["vgpr_count"] <= 256, (name, v)
    ws = {n: v for n, v in sweeps.items() if "op_kernel_ws" in n}
    # fused: light and paying forms, FP64 and FP32 (64x6), FP32 (64x8); FP64 operator with and without
    # add; refinement
    assert len(ws) == 9, sorted(ws)
    for name, v in ws.items():
        # 8 wavefronts (6 compute + 2 loaders) per CU: 2 per SIMD, at most 256 VGPRs each; 10 for
        # 64x8 (3 on two SIMDs: at most 168); the ring, row exchange and dictionary inside the
        # 160 KB of LDS
        assert v["group_segment_fixed_size"] <= 160 * 1024, (name, v)
        if "op_kernel_wsILi64ELi8" in name:
            assert v["vgpr_count"] <= 168, (name, v)
