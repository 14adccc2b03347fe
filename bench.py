"""Benchmark of the PCG hot path on one MI355X.

One step = one pass of the whole path over one synthetic microstructure
already resident in HBM: elas3d_setup (coefficient tables, load vector,
block-Jacobi inverse), elas3d_solve to a true relative residual of `tol`,
elas3d_stress (voxel stress planes, mean stress, energy) and destroy.

Prints one JSON line with the throughput in Gdof*iterations/s over the
whole step, the roofline of the dominant kernel (the fused
direction + operator sweep, timed with HIP events on its own stream) and
the CPU oracle timed on a bounded sample of the same recipe.

The microstructure is generated on the device (same recipe and random
stream as the host generator) before anything is timed.  The measured HBM
traffic of the dominant kernel comes from the committed rocprofv3 counter
summary when that summary was taken on the current kernel source (else null).
"""

from __future__ import annotations

import argparse
import hashlib
import json
import os
import re
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, GB/s
COUNTERS = os.path.join(ROOT, "profiles", "op_kernel_poly500_fp64_counters.txt")
VALU_COUNTERS = os.path.join(ROOT, "profiles", "op_kernel_poly500_valu_counters.txt")
VALU_PEAK_TFLOPS = {"fp64": 78.6, "fp32": 157.3}  # MI355X vector peaks
KERNEL_SOURCES = ("paper_2602_07354_amd/csrc/elas3d_kernels.hip", "paper_2602_07354_amd/csrc/elas3d_internal.h")
# Algorithmic HBM bytes per node of the fused direction+operator sweep, the
# mean of its two alternating forms: read z, h_old and the phase id, write
# h_new and Ah (4 x 3 values + 4 bytes); every other iteration it also pays
# the two steps w owes (read w and the older direction, write w: 3 x 3
# values).  Per launch: 5.5 vectors + phase.
OPERATOR_BYTES_PER_NODE_FP64 = (4 * 24 + 4 + 7 * 24 + 4) / 2  # 136
OPERATOR_BYTES_PER_NODE_FP32 = (4 * 12 + 4 + 7 * 12 + 4) / 2  # 70

WORKLOAD_TEXT = {
    "poly500": "500^3 periodic Voronoi polycrystal, 8000 rotated cubic SS316L grains "
               "(C11/C12/C44 = 206/133/119 GPa), 2% pores (spheres, oblate 4:4:1, z-prolate "
               "keyholes in thirds), eps_zz = 1e-3",
    "poly800": "800^3 periodic Voronoi polycrystal, 32768 rotated cubic SS316L grains (the 500^3 grain "
               "density), 2% pores (spheres, oblate 4:4:1, z-prolate keyholes in thirds), eps_zz = 1e-3",
    "poly300": "300^3 periodic Voronoi polycrystal, 3000 grains, 0.5% spheres + 0.5% oblate pores",
    "poly100": "100^3 periodic Voronoi polycrystal, 500 grains, 1% spherical pores, eps_xx = 1e-3",
    "eshelby20": "20^3 isotropic matrix with a stiff spherical inclusion, eps_xx = 1e-3",
    "void500": "the paper's Eshelby timing case: 500^3 isotropic matrix (E = 194 GPa, nu = 0.2934) around "
               "a centred spherical void of radius 20 voxels, eps_zz = 1e-3",
}
# workloads built on the host (the device generator makes polycrystals only)
HOST_WORKLOADS = ("eshelby20", "void500")


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="poly500", choices=sorted(WORKLOAD_TEXT))
    ap.add_argument("--scale", type=int, default=None, help="re-size the workload to scale^3")
    ap.add_argument("--tol", type=float, default=1e-8)
    ap.add_argument("--maxit", type=int, default=50000)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample", type=int, default=100, help="edge of the oracle sample grid")
    ap.add_argument("--cpu-iters", type=int, default=100)
    ap.add_argument("--calib-copy-gib", type=float, default=0.0,
                    help="run a plain device copy of this size first (counter calibration)")
    ap.add_argument("--no-autotune", action="store_true",
                    help="keep the default sweep geometry (32x8 workgroups) instead of autotuning it")
    ap.add_argument("--tile", type=int, default=None,
                    help="fix the workgroup shape of the fused sweep (index into elas3d.TILE_SHAPES) "
                         "instead of autotuning it (the update sweep is still autotuned)")
    ap.add_argument("--zchunk", type=int, default=0,
                    help="with --tile: z planes per workgroup (0 = automatic)")
    ap.add_argument("--nrhs", type=int, default=1, help="load cases solved per step (of the workload's)")
    ap.add_argument("--batched", action="store_true",
                    help="solve the load cases as one lockstep multi-RHS batch (else one after another)")
    ap.add_argument("--host-generator", action="store_true",
                    help="generate the microstructure on the host instead of the device")
    ap.add_argument("--precision", default="both", choices=["fp64", "mixed", "both"],
                    help="fp64: the paper's FP64 PCG; mixed: FP32 inner PCG in FP64 refinement; "
                         "both: time both (the headline value is FP64)")
    ap.add_argument("--criterion", default="residual", choices=["residual", "paper"],
                    help="stop on ||g||/||b|| confirmed by the true residual (default), or on the paper's "
                         "sqrt(z.g / z0.g0)")
    ap.add_argument("--stream-table", action="store_true",
                    help="print the stream probe's rates per grid and access kind, then exit")
    return ap.parse_args()


def source_code(text: str) -> str:
    """C++ source without comments, trailing blanks and empty lines (the
    kernel sources hold no string literal with a comment marker)."""
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    lines = (re.sub(r"//.*$", "", line).rstrip() for line in text.splitlines())
    return "\n".join(line for line in lines if line)


def kernel_source_hash() -> str:
    """Hash of the kernel sources' code, so that only code changes set the
    committed counter summaries aside."""
    h = hashlib.sha256()
    for rel in KERNEL_SOURCES:
        with open(os.path.join(ROOT, rel)) as f:
            h.update(source_code(f.read()).encode())
    return h.hexdigest()


def _counter_summary(path: str, workload: str, tile, tile_key: str = "op_tile"):
    """key: value lines of a committed counter summary, or None (with the
    reason) unless it was taken on this kernel source, workload and sweep
    geometry (lanes in x, y and z-chunk length; under tile_key)."""
    if not os.path.exists(path):
        return None, None
    kv = {}
    with open(path) as f:
        for line in f:
            if ":" in line and not line.startswith("#"):
                k, v = line.split(":", 1)
                kv[k.strip()] = v.strip()
    if (kv.get("kernel_source_sha256") != kernel_source_hash() or kv.get("workload") != workload
            or (tile_key is not None and kv.get(tile_key) != " ".join(str(v) for v in tile))):
        return None, "stale (kernel, workload or sweep geometry differs from the counters' run)"
    return kv, os.path.relpath(path, ROOT)


def measured_traffic(workload: str, tile) -> dict:
    """HBM bytes per launch of the fused sweep from the committed counter
    summary (see _counter_summary)."""
    kv, src = _counter_summary(COUNTERS, workload, tile)
    return {"bytes": float(kv["op_traffic_bytes_per_dispatch"]) if kv else None, "source": src}


def measured_valu(workload: str, tile, precision: str, op_ms: float, nz: int):
    """Achieved vector-ALU rate of the fused sweep: its counted flops per
    launch (committed summary) over the launch duration measured now,
    against the vector peak; and its MFMA count.  The summary must be of
    this kernel source, workload and workgroup shape; another z-chunk length
    kz changes only the element layers computed (nz plus one per chunk), and
    the flops are scaled by that count."""
    key = "op_tile" if precision == "fp64" else "fp32_op_tile"
    kv, src = _counter_summary(VALU_COUNTERS, workload, tile, key)
    scaled = False
    if not kv and src and os.path.exists(VALU_COUNTERS):
        kv, src = _counter_summary(VALU_COUNTERS, workload, None, None)
        if kv:
            tx, ty, kz0 = (int(v) for v in kv[key].split())
            if (tx, ty) != (int(tile[0]), int(tile[1])):
                return {"achieved": None, "source": "stale (workgroup shape differs from the counters' run)"}
            scaled = True
    if not kv:
        return {"achieved": None, "source": src}
    flops = float(kv[precision + "_flops_per_dispatch"])
    if scaled:
        layers = lambda kz: nz + -(-nz // kz)  # noqa: E731
        flops *= layers(int(tile[2])) / layers(kz0)
        src += " (scaled to z-chunk %d from %d)" % (int(tile[2]), kz0)
    achieved = flops / (op_ms * 1e-3) / 1e12
    peak = VALU_PEAK_TFLOPS[precision]
    return {"achieved": round(achieved, 2), "peak": peak, "unit": "TFLOP/s", "frac": round(achieved / peak, 4),
            "flops_per_launch": flops, "mfma_instructions": float(kv[precision + "_mfma_per_dispatch"]),
            "source": src}


def stream_rates(E, dev_index: int, gib: float = 4.0, table: bool = False) -> dict:
    """Best plain-stream rates on the device (GB/s), the practical HBM ceiling
    beside the datasheet peak: the library's copy, read-only and write-only
    probe kernels (16 B per lane), plain and non-temporal, over a few grids
    (each printed as a JSON line when table is set)."""
    best = {"copy": 0.0, "read": 0.0, "write": 0.0}
    opts = E.options_init(device=dev_index)
    for blocks in (2048, 8192, 32768, 131072):
        for nt in (False, True):
            r = E.stream_bandwidth(int(gib * (1 << 30)), blocks=blocks, reps=5, nontemporal=nt, options=opts)
            if table:
                print(json.dumps({"buffer_GiB": gib, "workgroups": blocks, "nontemporal": nt,
                                  **{k: round(v, 1) for k, v in r.items()}}), flush=True)
            for k in best:
                best[k] = max(best[k], r[k])
    return {k: round(v, 1) for k, v in best.items()}


def cpu_baseline(workload: str, edge: int, iters: int) -> dict:
    """The oracle (serial FP64 C) on a bounded sample: the same recipe at edge^3."""
    import oracle
    from paper_2602_07354_amd import synth

    ms = synth.workload(workload, scale=edge) if workload != "eshelby20" else synth.workload(workload)
    P = oracle.Problem.from_micro(ms)
    b, r2 = P.load(ms.strain[0])
    minv = P.precond()
    t0 = time.perf_counter()
    r = P.solve(ms.strain[0], tol=0.0, maxit=iters, b=b, minv=minv)
    dt = time.perf_counter() - t0
    n_it = max(1, r["iters"])
    return {
        "value": 3.0 * ms.n * n_it / dt / 1e9,
        "unit": "Gdof*iter/s",
        "cores": 1,
        "kind": "oracle",
        "sample": f"serial FP64 oracle PCG, {n_it} iterations on the {ms.meta['workload']} grid "
                  f"({ms.n} voxels, same grain density and pore recipe), {dt:.1f} s",
    }


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU only; sharding the solve over "
                                   "several GPUs is not implemented", "n_gpus": args.gpus}))
        sys.exit(2)

    import torch

    from paper_2602_07354_amd import elas3d as E
    from paper_2602_07354_amd import synth

    E.lib()
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    if args.stream_table:
        print(json.dumps({"best": stream_rates(E, 0, table=True)}), flush=True)
        return
    t_gen = time.perf_counter()
    if args.workload in HOST_WORKLOADS or args.host_generator:
        ms = synth.workload(args.workload, scale=args.scale) if args.workload != "eshelby20" \
            else synth.workload(args.workload)
        phase = torch.from_numpy(ms.phase).to(dev)
        void_fraction = ms.void_fraction()
    else:
        from paper_2602_07354_amd import generate
        rec = synth.workload_recipe(args.workload, args.scale)
        phase = torch.empty(int(np.prod(rec["shape"])), dtype=torch.int32, device=dev)
        ms = generate.workload(args.workload, scale=args.scale, phase=phase)
        void_fraction = ms.meta["void_fraction"]
    torch.cuda.synchronize()
    t_gen = time.perf_counter() - t_gen
    print(f"# generated {ms.meta.get('workload')} {ms.shape} in {t_gen:.1f} s "
          f"({'host' if ms.meta.get('generated_on') != 'device' else 'device'}), void {void_fraction:.4f}",
          file=sys.stderr, flush=True)
    try:
        streams = stream_rates(E, dev.index or 0)
    except E.Elas3dError as e:  # the benchmark stands without its context figure
        print(f"# stream probe failed: {e}", file=sys.stderr, flush=True)
        streams = {"copy": None, "read": None, "write": None}
    copy_gbs = streams["copy"]
    if args.calib_copy_gib > 0:
        # a plain elementwise kernel that reads and writes exactly this many
        # bytes once (HBM-counter calibration under rocprofv3 --pmc)
        nbytes = int(args.calib_copy_gib * (1 << 30))
        src = torch.empty(nbytes // 8, dtype=torch.float64, device=dev).fill_(1.0)
        dst = torch.empty(2 * (nbytes // 8), dtype=torch.float64, device=dev)  # evicts caches
        dst.fill_(0.0)
        dst = dst[: nbytes // 8]
        torch.mul(src, 2.0, out=dst)
        torch.cuda.synchronize()
        del src, dst
    nrhs = args.nrhs
    if not 1 <= nrhs <= ms.nrhs:
        sys.exit(f"--nrhs must be in [1, {ms.nrhs}] for {args.workload}")
    sigma = torch.empty((6, ms.n), dtype=torch.float64, device=dev)
    avg = np.empty(6)
    energy = np.empty(1)
    stream = torch.cuda.Stream(device=dev)
    torch.cuda.synchronize()

    def step(record, precision):
        opts = E.options_init(inputs_on_device=1, outputs_on_device=1, timing=1, device=0,
                              stream=stream.cuda_stream,
                              autotune=0 if args.no_autotune else (2 if args.tile is not None else 1),
                              tile=args.tile or 0, zchunk=args.zchunk if args.tile is not None else 0,
                              batched=1 if args.batched else 0,
                              convergence=E.CONV_PAPER if args.criterion == "paper" else E.CONV_RESIDUAL,
                              precision=E.PREC_MIXED if precision == "mixed" else E.PREC_FP64)
        h = E.setup(ms.shape, phase, ms.C, ms.strain[:nrhs], opts)
        try:
            st, info = E.solve(h, args.tol, args.maxit, nrhs)
            # voxel stress planes go to a device buffer; mean stress and energy to the host
            for r in range(nrhs):
                E.lib().elas3d_stress(h, r, sigma.data_ptr(), avg.ctypes.data, None, energy.ctypes.data)
        finally:
            E.destroy(h)
        if record is not None:
            record.append((st, info.as_dict()))

    def timed(precision):
        for _ in range(args.warmup):
            step(None, precision)
        torch.cuda.synchronize()
        print(f"# {precision}: warm-up done", file=sys.stderr, flush=True)
        recs = []
        t0 = time.perf_counter()
        for _ in range(args.steps):
            step(recs, precision)
            print(f"# {precision}: step done, {sum(recs[-1][1]['iters'])} iterations", file=sys.stderr, flush=True)
        torch.cuda.synchronize()
        return recs, time.perf_counter() - t0

    head = "mixed" if args.precision == "mixed" else "fp64"
    recs, dt = timed(head)
    mixed = None
    if args.precision == "both":
        mrecs, mdt = timed("mixed")
        m_iters = [sum(r[1]["iters"]) for r in mrecs]
        m_ms = 1e3 * mdt / args.steps
        m_tts = [r[1]["t_solve_s"] for r in mrecs]
        mixed = {
            "precision": "FP32 inner PCG + FP64 refinement (FP64 residual, update, dots, 3x3 inversions)",
            "ms_per_step": round(m_ms, 3),
            "time_to_solution_s": [round(t, 4) for t in m_tts],
            "inner_iters": [r[1]["iters"] for r in mrecs],
            "refinement_cycles": [r[1]["restarts"] for r in mrecs],
            "relres_true": [max(r[1]["relres_true"]) for r in mrecs],
            "fp64_fallback": [r[1]["fp64_fallback"] for r in mrecs],
            "gdof_iter_per_s": round(3.0 * ms.n * float(np.mean(m_iters)) / (m_ms / 1e3) / 1e9, 3),
            "operator_ms_avg": round(sum(r[1]["t_operator_ms"] for r in mrecs) /
                                     max(1, sum(r[1]["n_operator"] for r in mrecs)), 4),
            "update_ms_avg": round(sum(r[1]["t_update_ms"] for r in mrecs) /
                                   max(1, sum(r[1]["n_update"] for r in mrecs)), 4),
            "op_tile": mrecs[0][1]["op_tile"],
            "update_blocks": mrecs[0][1]["update_blocks"],
            "update_nontemporal": mrecs[0][1]["update_nontemporal"],
        }
        mixed["valu"] = measured_valu(ms.meta.get("workload"), mixed["op_tile"], "fp32", mixed["operator_ms_avg"],
                                      ms.shape[2])

    iters = [sum(r[1]["iters"]) for r in recs]  # summed over the load cases
    t_op = sum(r[1]["t_operator_ms"] for r in recs)
    n_op = sum(r[1]["n_operator"] for r in recs)
    t_up = sum(r[1]["t_update_ms"] for r in recs)
    n_up = sum(r[1]["n_update"] for r in recs)
    ms_step = 1e3 * dt / args.steps
    dof_iters = 3.0 * ms.n * float(np.mean(iters))
    value = dof_iters / (ms_step / 1e3) / 1e9
    op_ms = t_op / max(1, n_op)
    # a batched launch sweeps every RHS still running: RHS-sweeps per launch
    rhs_per_launch = (sum(iters) / max(1, n_op)) if args.batched else 1.0
    op_bytes = (OPERATOR_BYTES_PER_NODE_FP64 if head == "fp64" else OPERATOR_BYTES_PER_NODE_FP32) * ms.n * rhs_per_launch
    achieved = op_bytes / (op_ms / 1e3) / 1e9
    tile = recs[0][1]["op_tile"]
    traffic = (measured_traffic(ms.meta.get("workload"), tile) if head == "fp64" and nrhs == 1
               else {"bytes": None, "source": None})
    out = {
        "metric": ("Gdof*iterations/s of the block-Jacobi PCG solve to true rel-res 1e-8 "
                   if args.criterion == "residual" else
                   "Gdof*iterations/s of the block-Jacobi PCG solve to the paper's sqrt(z.g/z0.g0) < tol ")
                  + "(whole step: setup + solve + stress); FP64 vs mixed time-to-solution beside it",
        "value": round(value, 3),
        "unit": "Gdof*iter/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if head == "fp64" else "f32+f64",
        "data": "synthetic",
        "config": {
            "workload": ms.meta.get("workload"),
            "description": WORKLOAD_TEXT.get(args.workload, ""),
            "grid": list(ms.shape),
            "nphase": ms.nphase,
            "void_fraction": round(void_fraction, 5),
            "generator": ms.meta.get("generated_on", "host"),
            "tol": args.tol,
            "criterion": args.criterion,
            "precision": head,
            "nrhs": nrhs,
            "batched": bool(args.batched),
            "parallelism": "single GPU",
        },
        "iters": [r[1]["iters"] for r in recs] if nrhs > 1 else iters,
        "status": [r[0] for r in recs],
        "relres_true": [max(r[1]["relres_true"]) for r in recs],
        "refinement_cycles": [r[1]["restarts"] for r in recs] if head == "mixed" else None,
        "fp64_fallback": [r[1]["fp64_fallback"] for r in recs] if head == "mixed" else None,
        "time_to_solution_s": [round(r[1]["t_solve_s"], 4) for r in recs],
        "mixed": mixed,
        "mixed_speedup_time_to_solution": (
            round(float(np.mean([r[1]["t_solve_s"] for r in recs])) /
                  float(np.mean(mixed["time_to_solution_s"])), 3) if mixed else None),
        "precond_rows": recs[0][1]["precond_rows"],
        "operator_ms_avg": round(op_ms, 4),
        "update_ms_avg": round(t_up / max(1, n_up), 4),
        "roofline": {
            "kernel": "op_kernel<%d,%d,OP_FUSED,%s> (fused direction update + matrix-free operator + h.Ah)"
                      % (tile[0], tile[1], "double" if head == "fp64" else "float"),
            "bound": "hbm",
            "achieved": round(achieved, 1),
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": traffic["bytes"],
            "traffic_source": traffic["source"],
            "bytes_per_launch": round(op_bytes),
            "stream_GBs_measured": streams,
            "frac_of_copy": round(achieved / copy_gbs, 4) if copy_gbs else None,
            "op_tile": tile,
            "update_blocks": recs[0][1]["update_blocks"],
            "update_nontemporal": recs[0][1]["update_nontemporal"],
            "valu": (measured_valu(ms.meta.get("workload"), tile, "fp64" if head == "fp64" else "fp32", op_ms,
                                   ms.shape[2]) if nrhs == 1 else None),
        },
    }
    if not args.no_cpu_baseline:
        try:
            out["cpu_baseline"] = cpu_baseline(args.workload, args.cpu_sample, args.cpu_iters)
        except Exception as e:  # the GPU number stands without it
            out["cpu_baseline"] = {"error": repr(e)}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
