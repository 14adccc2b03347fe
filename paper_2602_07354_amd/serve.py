"""Solve service with continuous batching of uneven requests on one GPU.

Requests are independent periodic voxel elasticity solves (their own grid,
phase map, stiffnesses and 1-6 load cases).  Queued requests are admitted as
soon as the device-memory budget and the concurrency cap allow, so requests
that arrive while others are on the GPU join as slots and memory free up.

Two engines:

* ``GroupServer`` (the default): one engine thread owns an elas3d group.
  Admitted requests are set up and added to it; every batch of iterations
  advances all of them with one launch per sweep over a work list of
  (request, workgroup) entries (four launches per PCG iteration for up to 8
  requests); finished requests leave between batches, new ones join.
* ``Server``: each admitted request runs elas3d_solve on a worker thread with
  its own HIP stream, and the solves overlap on the device.

Every kernel is deterministic and a request's sweeps are the same in either
engine, so a result is bit-identical whether its request runs alone or in the
mix.

``python -m paper_2602_07354_amd.serve`` measures the saturation throughput
and then p50/p99 latency under Poisson arrivals at fractions of it.
"""

from __future__ import annotations

import argparse
import dataclasses
import json
import sys
import threading
import time
from collections import deque
from concurrent.futures import FIRST_COMPLETED, ThreadPoolExecutor, wait
from typing import List, Optional

import numpy as np

from . import elas3d as E
from . import synth


@dataclasses.dataclass
class Request:
    rid: int
    micro: synth.Microstructure
    tol: float = 1e-8
    precision: int = E.PREC_MIXED
    arrival: float = 0.0  # seconds after the stream start


@dataclasses.dataclass
class Result:
    rid: int
    shape: tuple
    nrhs: int
    status: int
    iters: list
    relres_true: list
    sigma_avg: np.ndarray  # (nrhs, 6)
    t_arrival: float
    t_start: float
    t_end: float
    error: Optional[str] = None
    # with keep_fields: per load case the fluctuation displacement w (3 x N)
    # and the voxel stress (6 x N), host copies
    w: Optional[list] = None
    sigma: Optional[list] = None

    @property
    def latency(self) -> float:
        return self.t_end - self.t_arrival


def request_bytes(req: Request) -> float:
    o = E.options_init(precision=req.precision, batched=1)
    return E.device_bytes(req.micro.shape, req.micro.nphase, req.micro.nrhs, o)


def _collect(h, ms, keep_fields: bool):
    """Mean stress of every load case of a solved context (and, with
    keep_fields, its w and voxel stress planes)."""
    avg = np.empty((ms.nrhs, 6))
    ws, sigs = ([], []) if keep_fields else (None, None)
    for r in range(ms.nrhs):
        a = np.empty(6)
        sig = np.empty((6, ms.n)) if keep_fields else None
        E.stress(h, r, sig, a, None, None)
        avg[r] = a
        if keep_fields:
            w = np.empty((3, ms.n))
            E.get_solution(h, r, w)
            ws.append(w)
            sigs.append(sig)
    return avg, ws, sigs


def _code(e: BaseException) -> int:
    """Status of a failed request: the library's error code, else EDEVICE."""
    return int(getattr(e, "code", E.EDEVICE))


def _failed(req: Request, code: int, msg: str, t_arrival: float, t_start: float, t_end: float) -> Result:
    ms = req.micro
    return Result(req.rid, ms.shape, ms.nrhs, code, [], [], np.zeros((ms.nrhs, 6)), t_arrival, t_start, t_end,
                  msg)


def solve_one(req: Request, t_arrival: float = 0.0, t0: float = 0.0, device: int = 0,
              keep_fields: bool = False) -> Result:
    """Run one request to completion on the calling thread (own HIP stream)."""
    ms = req.micro
    t_start = time.perf_counter() - t0
    try:
        opts = E.options_init(precision=req.precision, batched=1, device=device)
        h = E.setup(ms.shape, ms.phase, ms.C, ms.strain, opts)
        try:
            st, info = E.solve(h, req.tol, 50000, ms.nrhs)
            avg, ws, sigs = _collect(h, ms, keep_fields)
        finally:
            E.destroy(h)
        d = info.as_dict()
        return Result(req.rid, ms.shape, ms.nrhs, st, d["iters"], d["relres_true"], avg, t_arrival,
                      t_start, time.perf_counter() - t0, None, ws, sigs)
    except Exception as e:  # noqa: BLE001 - a failed request is a result, not a crash
        return _failed(req, _code(e), str(e), t_arrival, t_start, time.perf_counter() - t0)


class Server:
    """Admission by memory budget and concurrency; workers overlap on the GPU."""

    def __init__(self, budget_bytes: Optional[float] = None, max_concurrency: int = 8,
                 device: int = 0, keep_fields: bool = False):
        if budget_bytes is None:
            import torch

            free, _ = torch.cuda.mem_get_info(device)
            budget_bytes = 0.8 * free
        self.budget = float(budget_bytes)
        self.max_conc = int(max_concurrency)
        self.device = device
        self.keep_fields = bool(keep_fields)
        self._lock = threading.Condition()
        self._queue: deque = deque()
        self._in_flight_bytes = 0.0
        self._in_flight = 0
        self._results: List[Result] = []
        self._stop = False
        self._t0 = time.perf_counter()
        self._dispatcher = threading.Thread(target=self._dispatch, daemon=True)
        self._dispatcher.start()

    def now(self) -> float:
        return time.perf_counter() - self._t0

    def submit(self, req: Request) -> None:
        nbytes = request_bytes(req)
        if nbytes > self.budget:
            raise ValueError(f"request {req.rid} needs {nbytes/1e9:.2f} GB, over the budget")
        with self._lock:
            self._queue.append((req, nbytes, self.now()))
            self._lock.notify_all()

    def _dispatch(self):
        while True:
            with self._lock:
                while not self._stop and not self._admissible():
                    self._lock.wait()
                if self._stop and not self._queue:
                    return
                if not self._admissible():
                    continue
                req, nbytes, t_arr = self._queue.popleft()  # FIFO: no overtaking
                self._in_flight_bytes += nbytes
                self._in_flight += 1
            threading.Thread(target=self._work, args=(req, nbytes, t_arr), daemon=True).start()

    def _admissible(self) -> bool:
        if not self._queue or self._in_flight >= self.max_conc:
            return False
        nbytes = self._queue[0][1]
        return self._in_flight_bytes + nbytes <= self.budget

    def _work(self, req: Request, nbytes: float, t_arr: float):
        res = solve_one(req, t_arr, self._t0, self.device, self.keep_fields)
        with self._lock:
            self._results.append(res)
            self._in_flight_bytes -= nbytes
            self._in_flight -= 1
            self._lock.notify_all()

    def drain(self) -> List[Result]:
        with self._lock:
            while self._queue or self._in_flight:
                self._lock.wait()
            out = sorted(self._results, key=lambda r: r.rid)
            self._results = []
            return out

    def close(self):
        with self._lock:
            self._stop = True
            self._lock.notify_all()
        self._dispatcher.join(timeout=5)


class GroupServer:
    """Continuous batching through an elas3d group: one engine thread runs the
    group; set-ups (copies, tables, load and preconditioner sweeps on each
    context's own stream) run on worker threads meanwhile."""

    def __init__(self, budget_bytes: Optional[float] = None, max_concurrency: int = 64,
                 poll: int = 8, device: int = 0, setup_workers: int = 4, keep_fields: bool = False):
        if budget_bytes is None:
            import torch

            free, _ = torch.cuda.mem_get_info(device)
            budget_bytes = 0.8 * free
        self.budget = float(budget_bytes)
        self.max_conc = int(max_concurrency)
        self.poll = int(poll)
        self.device = device
        self.setup_workers = int(setup_workers)
        self.keep_fields = bool(keep_fields)
        self._lock = threading.Condition()
        self._queue: deque = deque()
        self._results: List[Result] = []
        self._in_flight = {}  # context handle -> (request, bytes, arrival, start)
        self._in_flight_bytes = 0.0
        self._open = 0  # admitted and not finished (setting up or in the group)
        self._stop = False
        self._error: Optional[BaseException] = None
        self._t0 = time.perf_counter()
        self._engine = threading.Thread(target=self._run, daemon=True)
        self._engine.start()

    def now(self) -> float:
        return time.perf_counter() - self._t0

    def submit(self, req: Request) -> None:
        nbytes = request_bytes(req)
        if nbytes > self.budget:
            raise ValueError(f"request {req.rid} needs {nbytes/1e9:.2f} GB, over the budget")
        with self._lock:
            self._queue.append((req, nbytes, self.now()))
            self._lock.notify_all()

    def _setup(self, req: Request, nbytes: float, t_arr: float):
        """Set up a request's context; a request the library refuses comes
        back with h = None and the error instead of raising."""
        ms = req.micro
        t_start = self.now()
        try:
            opts = E.options_init(precision=req.precision, batched=1, device=self.device)
            return E.setup(ms.shape, ms.phase, ms.C, ms.strain, opts), (req, nbytes, t_arr, t_start), None
        except Exception as e:  # noqa: BLE001 - becomes the request's error result
            return None, (req, nbytes, t_arr, t_start), e

    def _admit(self, pool, pending: set) -> None:
        while True:
            with self._lock:
                if not self._queue or len(self._in_flight) + len(pending) >= self.max_conc:
                    return
                req, nbytes, t_arr = self._queue[0]
                if self._in_flight_bytes + nbytes > self.budget:
                    return
                self._queue.popleft()
                self._in_flight_bytes += nbytes
                self._open += 1
            pending.add(pool.submit(self._setup, req, nbytes, t_arr))

    def _release(self, res: Result, nbytes: float) -> None:
        with self._lock:
            self._results.append(res)
            self._in_flight_bytes -= nbytes
            self._open -= 1
            self._lock.notify_all()

    def _join(self, group, pending: set) -> None:
        for f in [f for f in pending if f.done()]:
            pending.discard(f)
            h, meta, err = f.result()
            req, nbytes, t_arr, t_start = meta
            if h is not None:
                try:
                    group.add(h, req.tol, 50000)
                    self._in_flight[h] = meta
                    continue
                except Exception as e:  # noqa: BLE001
                    err = e
                    E.destroy(h)
            self._release(_failed(req, _code(err), str(err), t_arr, t_start, self.now()), nbytes)

    def _finish(self, h, status, info, meta) -> None:
        req, nbytes, t_arr, t_start = meta
        ms = req.micro
        try:
            try:
                avg, ws, sigs = _collect(h, ms, self.keep_fields)
            finally:
                E.destroy(h)
            res = Result(req.rid, ms.shape, ms.nrhs, status, info["iters"], info["relres_true"], avg, t_arr,
                         t_start, self.now(), None, ws, sigs)
        except Exception as e:  # noqa: BLE001 - the slot is released whatever happened
            res = _failed(req, _code(e), str(e), t_arr, t_start, self.now())
        self._release(res, nbytes)

    def _run(self) -> None:
        try:
            with E.Group(E.options_init(device=self.device)) as group, \
                    ThreadPoolExecutor(self.setup_workers) as pool:
                pending: set = set()
                while True:
                    self._admit(pool, pending)
                    self._join(group, pending)
                    if not self._in_flight:
                        if pending:
                            wait(pending, timeout=0.05, return_when=FIRST_COMPLETED)
                            continue
                        with self._lock:
                            if self._stop and not self._queue:
                                return
                            if not self._queue:
                                self._lock.wait(0.05)
                        continue
                    done, _ = group.run(self.poll)
                    for h, st, info in done:  # stress and release off the engine thread
                        pool.submit(self._finish, h, st, info, self._in_flight.pop(h))
        except BaseException as e:  # surfaced by drain()
            with self._lock:
                self._error = e
                self._lock.notify_all()

    def drain(self) -> List[Result]:
        with self._lock:
            while (self._queue or self._open) and self._error is None:
                self._lock.wait(0.05)
            if self._error is not None:
                raise RuntimeError("group engine failed") from self._error
            out = sorted(self._results, key=lambda r: r.rid)
            self._results = []
            return out

    def close(self):
        with self._lock:
            self._stop = True
            self._lock.notify_all()
        self._engine.join(timeout=30)


def run_stream(requests: List[Request], server, progress: int = 0) -> List[Result]:
    """Submit requests at their arrival offsets (seconds) and wait for all;
    with progress > 0, a line on stderr every `progress` submissions."""
    start = server.now()
    for k, req in enumerate(sorted(requests, key=lambda r: r.arrival)):
        delay = start + req.arrival - server.now()
        if delay > 0:
            time.sleep(delay)
        server.submit(req)
        if progress and (k + 1) % progress == 0:
            print(f"# submitted {k + 1}/{len(requests)} at {server.now() - start:.1f} s",
                  file=sys.stderr, flush=True)
    return server.drain()


def latency_stats(results: List[Result], wall: float) -> dict:
    lat = np.array([r.latency for r in results])
    return {
        "n": len(results),
        "p50_s": float(np.percentile(lat, 50)),
        "p99_s": float(np.percentile(lat, 99)),
        "mean_s": float(lat.mean()),
        "solves_per_s": len(results) / wall,
        "failed": int(sum(1 for r in results if r.status != 0)),
    }


def make_pool(n: int, seed0: int = 0, precision: int = E.PREC_MIXED, tol: float = 1e-8,
              device_generator: bool = False):
    """n distinct seeded serving requests (seeds seed0 .. seed0 + n - 1; grid
    32^3..128^3, 1-6 cases), built on the host or with the device generator
    (same recipe and random stream)."""
    if device_generator:
        from . import generate
        make = generate.serving_request
    else:
        make = synth.serving_request
    return [Request(i, make(seed0 + i), tol, precision) for i in range(n)]


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--requests", type=int, default=500, help="distinct requests per arrival rate")
    ap.add_argument("--saturation-requests", type=int, default=200,
                    help="distinct requests of the closed-loop saturation run")
    ap.add_argument("--rates", type=float, nargs="+", default=[0.25, 0.5, 0.75, 0.9, 1.1])
    ap.add_argument("--concurrency", type=int, default=8)
    ap.add_argument("--precision", choices=["fp64", "mixed"], default="mixed")
    ap.add_argument("--seed", type=int, default=4000)
    ap.add_argument("--engine", choices=["group", "streams"], default="group",
                    help="group: one launch per sweep for all requests; streams: one stream per request")
    ap.add_argument("--poll", type=int, default=8, help="group: iterations between admissions")
    ap.add_argument("--saturation-only", action="store_true",
                    help="run the warm-up and the closed-loop saturation run only (for a kernel trace)")
    args = ap.parse_args(argv)

    import torch

    torch.cuda.set_device(0)
    E.lib()
    prec = E.PREC_MIXED if args.precision == "mixed" else E.PREC_FP64

    def pool(n, seed0):
        t0 = time.perf_counter()
        p = make_pool(n, seed0, prec, device_generator=True)
        print(f"# {n} requests (seeds {seed0}..{seed0 + n - 1}) generated in {time.perf_counter() - t0:.1f} s",
              file=sys.stderr, flush=True)
        return p

    srv = (GroupServer(max_concurrency=args.concurrency, poll=args.poll) if args.engine == "group"
           else Server(max_concurrency=args.concurrency))
    # warm-up, then saturation: closed loop, everything queued at t = 0
    run_stream(pool(16, args.seed + 900_000), srv)
    sat_pool = pool(args.saturation_requests, args.seed + 800_000)
    t0 = time.perf_counter()
    sat = run_stream(sat_pool, srv, progress=100)
    sat_rate = len(sat) / (time.perf_counter() - t0)
    print(f"# saturation {sat_rate:.2f} solves/s", file=sys.stderr, flush=True)
    if args.saturation_only:
        srv.close()
        print(json.dumps({"engine": args.engine, "precision": args.precision, "saturation_requests": len(sat),
                          "saturation_solves_per_s": round(sat_rate, 3)}), flush=True)
        return
    edges = [r.micro.shape[0] for r in sat_pool]
    out = {"metric": "p50/p99 solve latency under Poisson arrivals (continuous batching)",
           "engine": args.engine, "poll": args.poll if args.engine == "group" else None,
           "precision": args.precision, "tol": sat_pool[0].tol,
           "concurrency": args.concurrency, "requests_per_rate": args.requests,
           "requests": "distinct seeded requests per rate (none reused): edge uniform over "
                       "{32, 64, 96, 128}, voxels/2000 grains, U[0, 2 %] spherical pores, 1-6 load cases",
           "saturation_requests": len(sat), "saturation_edges": {str(e): edges.count(e) for e in sorted(set(edges))},
           "saturation_solves_per_s": round(sat_rate, 3), "rates": []}
    del sat_pool, sat
    rng = np.random.default_rng(args.seed)
    for k, frac in enumerate(args.rates):
        reqs = pool(args.requests, args.seed + 1_000_000 * (k + 1))
        lam = frac * sat_rate
        gaps = rng.exponential(1.0 / lam, len(reqs))
        arr = np.cumsum(gaps) - gaps[0]
        reqs = [dataclasses.replace(r, rid=i, arrival=float(arr[i])) for i, r in enumerate(reqs)]
        t0 = time.perf_counter()
        res = run_stream(reqs, srv, progress=100)
        st = latency_stats(res, time.perf_counter() - t0)
        st["arrival_rate_frac"] = frac
        st["arrival_rate_per_s"] = round(lam, 3)
        out["rates"].append({k2: (round(v, 4) if isinstance(v, float) else v) for k2, v in st.items()})
        print(json.dumps(out["rates"][-1]), file=sys.stderr, flush=True)
        del reqs, res
    srv.close()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
