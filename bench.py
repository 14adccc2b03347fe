"""Benchmark of the PCG hot path on one MI355X.

One step = one pass of the whole path over one synthetic microstructure
already resident in HBM: elas3d_setup (coefficient tables, load vector,
block-Jacobi inverse), elas3d_solve for a fixed block of PCG iterations
(init, the iteration sweeps, the true residual), elas3d_stress (voxel
stress planes, mean stress, energy) and destroy.  The solve runs the
product path: iteration batches replayed as HIP graphs, sweep geometry
autotuned on the first step.  The value is Gdof*iterations/s over the whole
step (3N x iterations / step time).

Beside it, measured once per precision outside the timed steps:
  - time to solution: the same problem solved to a true relative residual
    of `tol` (FP64 PCG, and FP32 inner PCG inside FP64 refinement);
  - kernel durations: one extra step with HIP events recorded on the
    library's stream around every iteration sweep (eager launches, same
    geometry), which gives the roofline of the dominant kernel (the fused
    direction + operator sweep);
  - the CPU oracle on a bounded sample of the same recipe, serial and, when
    the OpenMP build of the oracle is present, on all host cores.

Progress goes to stderr; one JSON line goes to stdout at the end.  A
wall-clock budget skips the optional parts (mixed precision, time to
solution, CPU baseline) that would not fit, and says so in the line.

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
import platform
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
# mean of its two alternating forms: read z, h_old and the element's phase,
# write h_new and Ah (4 x 3 values + the phase); every other iteration it
# also pays the two steps w owes (read w and the older direction, write w:
# 3 x 3 values).  Per launch: 5.5 vectors + the phase, which the classic
# shapes read as a 4-byte id and the wave-specialised ones as a 1-byte rank
# in its workgroup's phase dictionary.
WS_SHAPES = (5, 6)  # options.tile of the wave-specialised shapes


def operator_bytes_per_node(precision: str, shape: int) -> float:
    v = 24 if precision == "fp64" else 12
    ph = 1 if shape in WS_SHAPES else 4
    return (4 * v + ph + 7 * v + ph) / 2
HOST_THREAD_CAP = 16  # host cores a one-GPU job may use

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


def parse(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="poly500", choices=sorted(WORKLOAD_TEXT))
    ap.add_argument("--scale", type=int, default=None, help="re-size the workload to scale^3")
    ap.add_argument("--tol", type=float, default=1e-8, help="tolerance of the time-to-solution solves")
    ap.add_argument("--block-iters", type=int, default=256,
                    help="PCG iterations of the solve in one timed step")
    ap.add_argument("--maxit", type=int, default=50000, help="iteration cap of the time-to-solution solves")
    ap.add_argument("--no-tts", action="store_true", help="skip the time-to-solution solves")
    ap.add_argument("--budget-s", type=float, default=420.0,
                    help="wall-clock seconds after which optional parts are skipped")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample", type=int, default=160, help="edge of the oracle's sample grid")
    ap.add_argument("--cpu-iters", type=int, default=0, help="oracle iterations timed (0 = automatic)")
    ap.add_argument("--cpu-tts", action="store_true",
                    help="also time the oracle's own solves of the benchmark problem to the tolerance, every "
                         "load case, threaded (grids of at most 2^21 nodes) and serial (at most 2^18)")
    ap.add_argument("--no-stream-probe", action="store_true")
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
                         "both: the FP64 steps are the headline, mixed precision is timed beside them")
    ap.add_argument("--criterion", default="residual", choices=["residual", "paper"],
                    help="stop on ||g||/||b|| confirmed by the true residual (default), or on the paper's "
                         "sqrt(z.g / z0.g0)")
    ap.add_argument("--stream-table", action="store_true",
                    help="print the stream probe's rates per grid and access kind, then exit")
    return ap.parse_args(argv)


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


def _counter_summary(path: str, workload: str, tile, tile_key: str = "op_tile", shape=None):
    """key: value lines of a committed counter summary, or None (with the
    reason) unless it was taken on this kernel source, workload and sweep
    geometry (lanes in x, y and z-chunk length under tile_key; the shape
    index under the matching *_shape key, when the file gives one)."""
    if not os.path.exists(path):
        return None, None
    kv = {}
    with open(path) as f:
        for line in f:
            if ":" in line and not line.startswith("#"):
                k, v = line.split(":", 1)
                kv[k.strip()] = v.strip()
    shape_key = tile_key.replace("tile", "shape") if tile_key else None
    if (kv.get("kernel_source_sha256") != kernel_source_hash() or kv.get("workload") != workload
            or (tile_key is not None and kv.get(tile_key) != " ".join(str(v) for v in tile))
            or (shape is not None and shape_key in kv and kv[shape_key] != str(shape))):
        return None, "stale (kernel, workload or sweep geometry differs from the counters' run)"
    return kv, os.path.relpath(path, ROOT)


def measured_traffic(workload: str, tile, shape=None) -> dict:
    """HBM bytes per launch of the fused sweep from the committed counter
    summary (see _counter_summary)."""
    kv, src = _counter_summary(COUNTERS, workload, tile, shape=shape)
    return {"bytes": float(kv["op_traffic_bytes_per_dispatch"]) if kv else None, "source": src}


def measured_valu(workload: str, tile, precision: str, op_ms: float, nz: int, shape=None):
    """Achieved vector-ALU rate of the fused sweep: its counted flops per
    launch (committed summary) over the launch duration measured now,
    against the vector peak; and its MFMA count.  The summary must be of
    this kernel source, workload and workgroup shape; another z-chunk length
    kz changes only the element layers computed (nz plus one per chunk), and
    the flops are scaled by that count."""
    key = "op_tile" if precision == "fp64" else "fp32_op_tile"
    kv, src = _counter_summary(VALU_COUNTERS, workload, tile, key, shape=shape)
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


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor() or "unknown"


def host_threads() -> int:
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(HOST_THREAD_CAP, n))


def _oracle_sample(workload: str, edge: int):
    """The workload's recipe at edge^3 (host arrays), and its name."""
    from paper_2602_07354_amd import synth
    if workload == "eshelby20":
        return synth.workload(workload)
    if workload in HOST_WORKLOADS:
        return synth.workload(workload, scale=edge)
    from paper_2602_07354_amd import generate
    return generate.workload(workload, scale=edge)


def _oracle_rate(P, strain, b, minv, iters: int, target_s: float, label: str = "oracle"):
    """Seconds per PCG iteration of the oracle: after one untimed run (cold
    caches), the time of a run of 1 + k iterations minus that of a run of 1
    (both pay the same start-up preconditioner apply, closing true residual
    and allocations), over k."""
    t0 = time.perf_counter()
    P.solve(strain, tol=0.0, maxit=0, b=b, minv=minv)
    t_warm = time.perf_counter() - t0
    t0 = time.perf_counter()
    P.solve(strain, tol=0.0, maxit=1, b=b, minv=minv)
    t_one = time.perf_counter() - t0
    if iters <= 0:  # about target_s of iterations
        iters = int(min(50, max(2, round(target_s / max(1e-3, t_one - 0.5 * t_warm)))))
    print(f"# {label}: a run of 1 iteration took {t_one:.2f} s; timing a run of {1 + iters}", file=sys.stderr,
          flush=True)
    t0 = time.perf_counter()
    r = P.solve(strain, tol=0.0, maxit=1 + iters, b=b, minv=minv)
    t_k = time.perf_counter() - t0
    k = max(1, r["iters"] - 1)
    return max(1e-9, (t_k - t_one) / k), k, t_warm + t_one + t_k


def cpu_baseline(workload: str, edge: int, iters: int, n_full: int, gpu_iters, time_left: float) -> dict:
    """The oracle (plain FP64 C, the same algorithm) on a bounded sample: the
    workload's recipe at edge^3, per-iteration time by difference of two
    runs, serial on one core and (OpenMP build) on the host's cores.  The
    time to solution of the full grid is extrapolated as seconds per
    iteration x (N_full / N_sample) x the GPU's FP64 iteration count."""
    import oracle

    ms = _oracle_sample(workload, edge)
    phase = np.asarray(ms.phase)
    strain = ms.strain[0]
    out = {"unit": "Gdof*iter/s", "kind": "oracle", "cpu_model": cpu_model(), "nproc": os.cpu_count(),
           "sample": f"the {workload} recipe at {ms.shape[0]}x{ms.shape[1]}x{ms.shape[2]} ({ms.n} voxels, "
                     f"same grain density and pores, generated with the same seeds), FP64 oracle PCG; "
                     f"seconds per iteration from a run of 1 + k iterations minus a run of 1"}
    legs = []
    threads = host_threads()
    if threads > 1 and oracle.threaded_available():
        legs.append(("threaded", threads))
    legs.append(("serial", 1))
    # seconds of timed iterations per leg, less when little time is left
    scale = max(0.25, min(1.0, time_left / 120.0))
    for name, nt in legs:
        t0 = time.perf_counter()
        P = oracle.Problem(ms.shape, phase, ms.C, threads=nt if name == "threaded" else 0)
        b, _ = P.load(strain)
        minv = P.precond()
        t_setup = time.perf_counter() - t0
        print(f"# oracle {name} ({nt} threads) on {ms.shape}: setup {t_setup:.1f} s", file=sys.stderr, flush=True)
        s_it, k, spent = _oracle_rate(P, strain, b, minv, iters, scale * (4.0 if name == "threaded" else 8.0),
                                      f"oracle {name}")
        leg = {"value": round(3.0 * ms.n / s_it / 1e9, 5), "threads": nt, "iters": k,
               "s_per_iter": round(s_it, 4), "setup_s": round(t_setup, 2), "timed_s": round(spent, 2)}
        if gpu_iters:
            leg["extrapolated_time_to_solution_s"] = round(s_it * (n_full / ms.n) * gpu_iters, 1)
        out[name] = leg
        del P, b, minv
    head = out.get("threaded") or out["serial"]
    out["value"] = head["value"]
    out["cores"] = head["threads"]
    if gpu_iters:
        out["extrapolation"] = (f"time to solution of the full grid ({n_full} voxels) extrapolated from the "
                                f"sample: s/iteration x {n_full / ms.n:.3g} (voxel ratio) x {gpu_iters} (the "
                                f"GPU's FP64 iterations to the tolerance); not a measured solve")
    return out


def cpu_time_to_solution(ms, tol: float, criterion: str, gpu: dict) -> dict:
    """The oracle's time to solution of the benchmark problem itself (same
    grid, phases, stiffnesses, load cases and stopping rule), every load case
    solved in turn, on the host's cores (OpenMP build) and on one core, beside
    the GPU's time for the same solves."""
    import oracle
    mode = 1 if criterion == "paper" else 0
    out = {"grid": list(ms.shape), "cases": int(ms.nrhs), "tol": tol, "criterion": criterion,
           "cpu_model": cpu_model(), "gpu": gpu}
    legs = [("serial", 1)] if ms.n <= (1 << 18) else []  # one core: small grids only
    threads = host_threads()
    if threads > 1 and oracle.threaded_available():
        legs.insert(0, ("threaded", threads))
    for name, nt in legs:
        phase = ms.phase.cpu().numpy() if hasattr(ms.phase, "cpu") else np.asarray(ms.phase)  # device-generated maps
        P = oracle.Problem(ms.shape, phase, np.asarray(ms.C), threads=nt if name == "threaded" else 0)
        t0 = time.perf_counter()
        iters = []
        for r in range(ms.nrhs):
            res = P.solve(ms.strain[r], tol=tol, mode=mode)
            iters.append(int(res["iters"]))
            print(f"# oracle {name}: case {r} solved in {iters[-1]} iterations", file=sys.stderr, flush=True)
        out[name] = {"threads": nt, "time_to_solution_s": round(time.perf_counter() - t0, 3), "iters": iters}
        del P
    return out


def main(argv=None):
    args = parse(argv)
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU only; sharding the solve over "
                                   "several GPUs is not implemented", "n_gpus": args.gpus}))
        sys.exit(2)
    t_start = time.perf_counter()

    def elapsed():
        return time.perf_counter() - t_start

    def note(msg):
        print(f"# [{elapsed():6.1f} s] {msg}", file=sys.stderr, flush=True)

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
    note(f"generated {ms.meta.get('workload')} {ms.shape} in {t_gen:.1f} s "
         f"({'host' if ms.meta.get('generated_on') != 'device' else 'device'}), void {void_fraction:.4f}")
    streams = {"copy": None, "read": None, "write": None}
    if not args.no_stream_probe:
        try:
            streams = stream_rates(E, dev.index or 0)
            note(f"stream probe {streams}")
        except E.Elas3dError as e:  # the benchmark stands without its context figure
            note(f"stream probe failed: {e}")
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

    def step(precision, maxit, timing=False):
        """setup + solve (at most maxit iterations per case) + stress + destroy;
        returns (status, info dict, {setup, solve, stress} in ms)."""
        opts = E.options_init(inputs_on_device=1, outputs_on_device=1, timing=1 if timing else 0, device=0,
                              stream=stream.cuda_stream,
                              autotune=0 if args.no_autotune else (2 if args.tile is not None else 1),
                              tile=args.tile or 0, zchunk=args.zchunk if args.tile is not None else 0,
                              batched=1 if args.batched else 0,
                              convergence=E.CONV_PAPER if args.criterion == "paper" else E.CONV_RESIDUAL,
                              precision=E.PREC_MIXED if precision == "mixed" else E.PREC_FP64)
        t0 = time.perf_counter()
        h = E.setup(ms.shape, phase, ms.C, ms.strain[:nrhs], opts)
        t1 = time.perf_counter()
        try:
            st, info = E.solve(h, args.tol, maxit, nrhs)
            t2 = time.perf_counter()
            # voxel stress planes go to a device buffer; mean stress and energy to the host
            for r in range(nrhs):
                E.stress(h, r, sigma, avg, None, energy)
            t3 = time.perf_counter()
        finally:
            E.destroy(h)
        return st, info.as_dict(), {"setup": 1e3 * (t1 - t0), "solve": 1e3 * (t2 - t1), "stress": 1e3 * (t3 - t2)}

    def timed_steps(precision):
        for _ in range(args.warmup):
            step(precision, args.block_iters)
        torch.cuda.synchronize()
        note(f"{precision}: {args.warmup} warm-up steps done")
        recs = []
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            recs.append(step(precision, args.block_iters))
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        note(f"{precision}: {args.steps} timed steps in {dt:.2f} s, "
             f"{sum(recs[-1][1]['iters'])} iterations per step")
        return recs, dt

    def kernel_times(precision):
        """Mean duration of the fused sweep and of the update sweep (each with
        its finalize), HIP events on the library's stream, over one step."""
        st, info, _ = step(precision, args.block_iters, timing=True)
        op_ms = info["t_operator_ms"] / max(1, info["n_operator"])
        up_ms = info["t_update_ms"] / max(1, info["n_update"])
        note(f"{precision}: kernel timing step, fused sweep {op_ms:.4f} ms, update {up_ms:.4f} ms "
             f"({info['n_operator']} launches)")
        return op_ms, up_ms, info

    def tts(precision):
        """Time to solution: one solve to tol from w = 0 (setup and stress apart)."""
        st, info, ms_ = step(precision, args.maxit)
        note(f"{precision}: solved to {args.tol:g} in {info['t_solve_s']:.3f} s, {sum(info['iters'])} iterations, "
             f"true rel-res {max(info['relres_true']):.2e}, status {st}")
        out = {"status": st, "time_to_solution_s": round(info["t_solve_s"], 4), "iters": info["iters"],
               "restarts": info["restarts"], "relres_true": info["relres_true"],
               "setup_ms": round(ms_["setup"], 2), "stress_ms": round(ms_["stress"], 2),
               "gdof_iter_per_s": round(3.0 * ms.n * sum(info["iters"]) / max(1e-9, info["t_solve_s"]) / 1e9, 3)}
        if precision == "mixed":
            out["fp64_fallback"] = info["fp64_fallback"]
        return out

    def leg_summary(recs, dt):
        iters = [sum(r[1]["iters"]) for r in recs]
        ms_step = 1e3 * dt / len(recs)
        parts = {k: round(float(np.median([r[2][k] for r in recs])), 3) for k in ("setup", "solve", "stress")}
        return {
            "ms_per_step": round(ms_step, 3),
            "iters_per_step": iters[0] if len(set(iters)) == 1 else iters,
            "gdof_iter_per_s": round(3.0 * ms.n * float(np.mean(iters)) / (ms_step / 1e3) / 1e9, 3),
            "median_ms": parts,
            "gdof_iter_per_s_solve_only": round(3.0 * ms.n * float(np.mean(iters)) / (parts["solve"] / 1e3) / 1e9, 3),
            "op_tile": recs[0][1]["op_tile"],
            "op_shape": recs[0][1]["op_shape"],
            "update_blocks": recs[0][1]["update_blocks"],
            "update_nontemporal": recs[0][1]["update_nontemporal"],
        }

    skipped = []
    head = "mixed" if args.precision == "mixed" else "fp64"
    recs, dt = timed_steps(head)
    main_leg = leg_summary(recs, dt)
    op_ms, up_ms, kinfo = kernel_times(head)
    mixed = None
    if args.precision == "both":
        if elapsed() < args.budget_s:
            mrecs, mdt = timed_steps("mixed")
            mixed = leg_summary(mrecs, mdt)
            m_op, m_up, _ = kernel_times("mixed")
            mixed["precision"] = "FP32 inner PCG + FP64 refinement (FP64 residual, update, dots, 3x3 inversions)"
            mixed["operator_ms_avg"] = round(m_op, 4)
            mixed["update_ms_avg"] = round(m_up, 4)
            mixed["valu"] = measured_valu(ms.meta.get("workload"), mixed["op_tile"], "fp32", m_op, ms.shape[2],
                                          shape=mixed["op_shape"])
        else:
            skipped.append("mixed steps")
    tts_out = {}
    if not args.no_tts:
        for prec in ([head, "mixed"] if args.precision == "both" else [head]):
            if elapsed() < args.budget_s:
                tts_out[prec] = tts(prec)
            else:
                skipped.append(f"{prec} time to solution")

    value = main_leg["gdof_iter_per_s"]
    rhs_per_launch = (sum(kinfo["iters"]) / max(1, kinfo["n_operator"])) if args.batched else 1.0
    op_bytes = (operator_bytes_per_node("fp64" if head == "fp64" else "fp32", main_leg["op_shape"]) * ms.n
                * rhs_per_launch)
    achieved = op_bytes / (op_ms / 1e3) / 1e9
    tile = main_leg["op_tile"]
    traffic = (measured_traffic(ms.meta.get("workload"), tile, main_leg["op_shape"]) if head == "fp64" and nrhs == 1
               else {"bytes": None, "source": None})
    out = {
        "metric": ("Gdof*iterations/s of the block-Jacobi PCG over whole steps (setup + "
                   f"{args.block_iters} PCG iterations + true residual + stress); time to true rel-res "
                   f"{args.tol:g}, FP64 vs mixed precision, beside it"),
        "value": value,
        "unit": "Gdof*iter/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": main_leg["ms_per_step"],
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
            "block_iters": args.block_iters,
            "criterion": args.criterion,
            "precision": head,
            "nrhs": nrhs,
            "batched": bool(args.batched),
            "graphs": True,
            "parallelism": "single GPU",
        },
        "step": main_leg,
        "status": [r[0] for r in recs],
        "time_to_solution": tts_out or None,
        "mixed": mixed,
        "mixed_speedup_time_to_solution": (
            round(tts_out[head]["time_to_solution_s"] / tts_out["mixed"]["time_to_solution_s"], 3)
            if head in tts_out and "mixed" in tts_out and head != "mixed" else None),
        "precond_rows": recs[0][1]["precond_rows"],
        "operator_ms_avg": round(op_ms, 4),
        "update_ms_avg": round(up_ms, 4),
        "roofline": {
            "kernel": (("op_kernel_ws<%d,%d,2 loader wavefronts,%s> (wave-specialised fused direction update + "
                        "matrix-free operator + h.Ah; its light and paying forms)"
                        % (tile[0], tile[1], "double" if head == "fp64" else "float"))
                       if main_leg["op_shape"] in WS_SHAPES else
                       "op_kernel<%d,%d,OP_FUSED,%s> (fused direction update + matrix-free operator + h.Ah)"
                       % (tile[0], tile[1], "double" if head == "fp64" else "float")),
            "bound": "hbm",
            "achieved": round(achieved, 1),
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": traffic["bytes"],
            "traffic_source": traffic["source"],
            "bytes_per_launch": round(op_bytes),
            "duration_source": "HIP events on the library stream around each fused-sweep launch (with its "
                               "finalize), over one extra step of the same geometry",
            "stream_GBs_measured": streams,
            "frac_of_copy": round(achieved / copy_gbs, 4) if copy_gbs else None,
            "op_tile": tile,
            "op_shape": main_leg["op_shape"],
            "update_blocks": main_leg["update_blocks"],
            "update_nontemporal": main_leg["update_nontemporal"],
            "valu": (measured_valu(ms.meta.get("workload"), tile, "fp64" if head == "fp64" else "fp32", op_ms,
                                   ms.shape[2], shape=main_leg["op_shape"]) if nrhs == 1 else None),
        },
        "skipped": skipped or None,
        "wall_s": None,
    }
    if not args.no_cpu_baseline:
        if elapsed() < args.budget_s:
            try:
                gpu_iters = sum(tts_out[head]["iters"]) if head in tts_out else None
                out["cpu_baseline"] = cpu_baseline(args.workload, args.cpu_sample, args.cpu_iters, ms.n,
                                                   gpu_iters, args.budget_s + 120 - elapsed())
                note("cpu baseline done")
            except Exception as e:  # the GPU number stands without it
                out["cpu_baseline"] = {"error": repr(e)}
        else:
            skipped.append("cpu baseline")
            out["skipped"] = skipped
    if args.cpu_tts:
        if ms.n > (1 << 21):
            out["cpu_time_to_solution"] = {"error": "grid above 2^21 nodes: the oracle's full solve is not timed"}
        elif head in tts_out:
            t = tts_out[head]
            out["cpu_time_to_solution"] = cpu_time_to_solution(
                ms, args.tol, args.criterion,
                {"precision": head, "time_to_solution_s": t["time_to_solution_s"], "iters": t["iters"]})
            note("cpu time to solution done")
    out["wall_s"] = round(elapsed(), 1)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
