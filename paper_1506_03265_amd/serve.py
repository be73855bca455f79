"""Request loop for decomposition + estimate jobs with continuous batching.

Requests (graph, tau, seed) arrive over time.  Graphs are resident in device
memory (CSR + packed arcs from cldiam_load_csr).  The loop admits a waiting
request as soon as a worker slot is free and the HBM budget can hold the
request's footprint (workspaces and outputs, from the library's size
queries), so requests that arrive while others run start immediately and
their kernels overlap on the device: every worker has its own HIP stream and
the library calls release the Python interpreter lock.  A request is done when
its estimate is on the host; its cluster ids and distance bounds stay in device
memory.

`serve(..., workers=1)` is the plain sequential baseline: one request at a
time, in arrival order.

`serve_engine` batches inside the device job instead: one long-lived
decomposition job (the cldiam_server_* calls) holds graph slots; a request
joins at the next sweep boundary when a slot and a node range of the job's
workspace are free, every admitted request advances in the same sweeps, and a
finished one leaves at once, its quotient and estimate built by worker threads
on their own streams.
"""
from __future__ import annotations

import threading
import time
from collections import deque
from dataclasses import dataclass, field

from . import (DRIVER_AUTO, DecomposeJob, EstimateJob, QuotientJob, _torch, load_library)


@dataclass
class Request:
    rid: int
    arrival_s: float
    graph: str         # key into the resident graph pool
    tau: int
    seed: int


@dataclass
class Result:
    rid: int
    arrival_s: float
    start_s: float
    done_s: float
    num_clusters: int
    radius: int
    phi_gc: int
    phi_approx: int
    stages: int
    cluster: object = None   # device tensor when kept
    D: object = None
    status: int = 0          # a decomposition status other than CLDIAM_OK leaves the estimate at 0

    @property
    def latency_s(self) -> float:
        return self.done_s - self.arrival_s


def footprint_bytes(g) -> int:
    """Device bytes one request on graph g needs beyond the resident graph."""
    lib = load_library()
    dec = lib.cldiam_decompose_workspace_size(g.n, 1)
    quo = lib.cldiam_quotient_workspace_size(g.n, g.m)
    outs = g.n * (4 + 8) + (g.n + 1) * 8 + g.n * 4 + max(g.m, 1) * (4 + 8)
    return int(dec + quo + outs + (1 << 20))


class _Budget:
    def __init__(self, total: int):
        self.total = total
        self.used = 0
        self.cv = threading.Condition()

    def fits(self, b: int) -> bool:
        return self.used + b <= self.total or self.used == 0

    def take(self, b: int):
        self.used += b

    def give(self, b: int):
        with self.cv:
            self.used -= b
            self.cv.notify_all()


def _run_one(req: Request, g, stream, keep: bool, driver: int) -> Result:
    torch = _torch()
    with torch.cuda.stream(stream):
        t0 = time.perf_counter()
        job = DecomposeJob([g], [(req.tau, req.seed, 0)], driver)
        st = job.run(stream)[0]
        q = QuotientJob(g).run(job.cluster[0], job.D[0], stream)
        phi, approx = EstimateJob(q.k, q.qm, g.row_ptr.device).run(q, st.radius, stream)
        t1 = time.perf_counter()
    return Result(req.rid, req.arrival_s, t0, t1, st.num_clusters, st.radius, phi, approx, st.stages,
                  job.cluster[0] if keep else None, job.D[0] if keep else None)


def serve(requests, graphs: dict, workers: int = 4, hbm_budget_bytes: int = 200 << 30, keep_outputs=False,
          driver: int = DRIVER_AUTO, time_scale: float = 1.0):
    """Runs the requests against resident graphs; returns (results sorted by
    request id, wall seconds).  Arrival times are honoured (scaled by
    time_scale); latency is measured from each request's arrival.
    keep_outputs: True keeps every request's cluster ids and distance bounds
    on the device, a set of request ids keeps only those."""
    torch = _torch()
    reqs = sorted(requests, key=lambda r: r.arrival_s)
    budget = _Budget(hbm_budget_bytes)
    foot = {k: footprint_bytes(g) for k, g in graphs.items()}
    pending = deque()
    results = []
    errors = []
    lock = threading.Lock()
    streams = [torch.cuda.Stream() for _ in range(workers)]
    idle = deque(range(workers))
    t_start = time.perf_counter()
    n_total = len(reqs)
    done_count = [0]

    def worker(slot: int, req: Request, nbytes: int):
        try:
            keep = keep_outputs if isinstance(keep_outputs, bool) else req.rid in keep_outputs
            r = _run_one(req, graphs[req.graph], streams[slot], keep, driver)
            r.arrival_s += t_start
            with lock:
                results.append(r)
        except BaseException as e:  # reported after the loop
            with lock:
                errors.append(e)
        finally:
            with budget.cv:
                budget.used -= nbytes
                idle.append(slot)
                done_count[0] += 1
                budget.cv.notify_all()

    i = 0
    threads = []
    with budget.cv:
        while done_count[0] < n_total:
            now = time.perf_counter() - t_start
            while i < n_total and reqs[i].arrival_s * time_scale <= now:
                pending.append(reqs[i])
                i += 1
            # admit in arrival order while a slot and the budget allow
            while pending and idle and budget.fits(foot[pending[0].graph]):
                req = pending.popleft()
                slot = idle.popleft()
                nbytes = foot[req.graph]
                budget.take(nbytes)
                req = Request(req.rid, req.arrival_s * time_scale, req.graph, req.tau, req.seed)
                th = threading.Thread(target=worker, args=(slot, req, nbytes), daemon=True)
                th.start()
                threads.append(th)
            if done_count[0] >= n_total:
                break
            wait = 0.05
            if i < n_total:
                wait = max(0.0, min(wait, reqs[i].arrival_s * time_scale - (time.perf_counter() - t_start)))
            budget.cv.wait(timeout=wait)
    for th in threads:
        th.join()
    wall = time.perf_counter() - t_start
    if errors:
        raise errors[0]
    for r in results:
        r.arrival_s -= t_start
        r.start_s -= t_start
        r.done_s -= t_start
    return sorted(results, key=lambda r: r.rid), wall


def percentile(xs, p: float) -> float:
    s = sorted(xs)
    if not s:
        return 0.0
    k = min(len(s) - 1, max(0, int(round(p / 100.0 * (len(s) - 1)))))
    return s[k]


def serve_engine(requests, graphs: dict, max_graphs: int = 64, node_capacity: int = 0, sweeps_per_step: int = 4,
                 workers: int = 4, keep_outputs: bool = False, time_scale: float = 1.0, local_rounds: int = -1,
                 split_nodes: int = 0):
    """Continuous batching inside device jobs: arrived requests are submitted
    to a cldiam server (admitted between sweeps as slots and node ranges free
    up, all admitted requests advancing in the same sweeps); finished
    decompositions go to `workers` threads that build the quotient and the
    estimate on their own streams.  With split_nodes > 0 there are two
    servers, each stepped by its own thread on its own stream: one for graphs
    of fewer nodes than split_nodes and one for the rest, so that the long
    sweeps of large graphs do not hold back small requests.  Returns (results
    sorted by request id, wall seconds)."""
    import queue as _queue

    from . import Server

    torch = _torch()
    reqs = sorted(requests, key=lambda r: r.arrival_s)
    classes = [lambda n: True] if split_nodes <= 0 else [lambda n: n < split_nodes, lambda n: n >= split_nodes]
    caps = []
    for member in classes:
        ns = sorted((g.n for g in graphs.values() if member(g.n)), reverse=True)
        caps.append(node_capacity if node_capacity > 0 else max(sum(ns[:8]), ns[0] if ns else 1, 1))
    servers = [Server(c, max_graphs, local_rounds=local_rounds) for c in caps]
    inboxes = [_queue.Queue() for _ in servers]
    work = _queue.Queue()
    results, errors = [], []
    lock = threading.Lock()
    by_id = {r.rid: r for r in reqs}
    t_start = time.perf_counter()

    def stepper(srv, inbox):
        closed = False
        try:
            while True:
                while True:
                    try:
                        item = inbox.get(block=not srv.outputs and not closed, timeout=0.05)
                    except _queue.Empty:
                        break
                    if item is None:
                        closed = True
                        break
                    g, tau, seed, rid = item
                    srv.submit(g, tau, seed, rid)
                if srv.outputs:
                    srv.step(sweeps_per_step)
                    t_dec = time.perf_counter()
                    for tag, st, g, cluster, D in srv.poll():
                        work.put((tag, st, g, cluster, D, t_dec))
                elif closed:
                    return
        except BaseException as e:
            with lock:
                errors.append(e)

    def worker():
        stream = torch.cuda.Stream()
        est = None
        while True:
            item = work.get()
            if item is None:
                return
            rid, st, g, cluster, D, t_dec = item
            try:
                req = by_id[rid]
                if st.status != 0:
                    r = Result(rid, req.arrival_s * time_scale, t_dec - t_start, time.perf_counter() - t_start, 0, 0,
                               0, 0, st.stages, status=st.status)
                    with lock:
                        results.append(r)
                    continue
                with torch.cuda.stream(stream):
                    q = QuotientJob(g).run(cluster, D, stream)
                    if est is None:
                        est = EstimateJob(q.k, q.qm, g.row_ptr.device)
                    phi, approx = est.run(q, st.radius, stream)
                t1 = time.perf_counter()
                r = Result(rid, req.arrival_s * time_scale, t_dec - t_start, t1 - t_start, st.num_clusters,
                           st.radius, phi, approx, st.stages, cluster if keep_outputs else None,
                           D if keep_outputs else None)
                with lock:
                    results.append(r)
            except BaseException as e:
                with lock:
                    errors.append(e)

    steppers = [threading.Thread(target=stepper, args=(srv, box), daemon=True) for srv, box in zip(servers, inboxes)]
    threads = [threading.Thread(target=worker, daemon=True) for _ in range(workers)]
    for th in steppers + threads:
        th.start()
    i, n_total = 0, len(reqs)
    try:
        while True:
            now = time.perf_counter() - t_start
            while i < n_total and reqs[i].arrival_s * time_scale <= now:
                r = reqs[i]
                g = graphs[r.graph]
                k = 0 if len(classes) == 1 or classes[0](g.n) else 1
                inboxes[k].put((g, r.tau, r.seed, r.rid))
                i += 1
            with lock:
                finished = len(results) + len(errors)
                failed = bool(errors)
            if finished >= n_total or failed:
                break
            wait = 0.0005
            if i < n_total:
                wait = max(0.0, min(0.002, reqs[i].arrival_s * time_scale - (time.perf_counter() - t_start)))
            time.sleep(wait)
    finally:
        for box in inboxes:
            box.put(None)
        for th in steppers:
            th.join()
        for _ in threads:
            work.put(None)
        for th in threads:
            th.join()
        for srv in servers:
            srv.close()
    wall = time.perf_counter() - t_start
    if errors:
        raise errors[0]
    return sorted(results, key=lambda r: r.rid), wall
