"""Benchmarks of the CL-DIAM hot path on one MI355X.

Default (``--workload road4096``): the line the contract asks for.  A step is
one pass of the whole path over the workload, inputs resident in HBM:
decomposition (CLUSTER, Algorithm 1), weighted quotient graph and the
diameter estimate (Section 4).  Ingest (validation + weight-sorted packing of
the CSR) runs once before the clock and is reported separately.  Workload:
the road-like 4096x4096 mesh (16.8M nodes, 64.1M arcs), tau = 4, seed 1,
initial Delta = mean arc weight.  Throughput is undirected input edges per
second of step time, in GTEPS.

The roofline object covers the dominant kernel, the decomposition's sweep
kernel: algorithmic bytes of one decomposition (work counts of the sequential
oracle run, stored by tests/golden/make_workload_counts.py) divided by the
device time of the decomposition's launch loop (all its sweep and control
launches), measured by the library with HIP events on the caller's stream,
against the 8 TB/s HBM peak.  The CPU baseline times the oracle on the host on
the same workload (single thread).

Other workloads (each prints its own JSON line):
  --workload rmat24   the same step on R-MAT scale 24 (social-like graph)
  --workload rgg256   256 random geometric graphs (sizes log-uniform in
                      [1e3, 1e6]) decomposed in one device job, against one
                      job per graph, with the schedule picked by the tuner
  --workload serve    a Poisson request stream (meshes and R-MAT graphs)
                      served with in-engine continuous batching, against a
                      pool of streams and sequential plain runs: p50/p99
                      latency and requests/s
  --workload sssp     the Delta-stepping SSSP competitor on the road-like
                      mesh, best of several bucket widths
  --workload variants CLUSTER, the literal step-synchronous variant and
                      CLUSTER2 on the road-like mesh
  --workload delta0   the initial-Delta experiment on a bimodal-weight mesh
  --workload stepcap  the growing-step cap on skewed graphs
  --workload ceilings random-access ceilings of the GPU (PyTorch kernels)
  --workload mesh29   the step on a 2^29-node mesh with 2.16G arcs (64-bit
                      row offsets), checked by properties that hold at any
                      size (the oracle cannot run it)

Only one GPU is supported.
"""
import argparse
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, HERE)

HBM_PEAK_GBS = 8000.0
METRIC = "decomposition GTEPS + % HBM roofline; p50/p99 latency served vs plain, bit-exact"


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def cpu_model():
    """The host CPU's model name (first processor entry), for the CPU baseline."""
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def code_digest(path):
    """SHA-256 of a source file's code: comments, trailing spaces and blank
    lines removed, so that stored counters stay tied to the code they were
    taken on and not to its comments."""
    import hashlib
    import re
    text = open(path).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    lines = [re.sub(r"//.*$", "", ln).rstrip() for ln in text.splitlines()]
    return hashlib.sha256("\n".join(ln for ln in lines if ln).encode()).hexdigest()


def step_bench(args, name):
    import torch

    import graphgen
    import paper_1506_03265_amd as cd

    counts = json.load(open(os.path.join(HERE, "tests", "golden", f"{name}_counts.json")))
    log(f"[bench] generating {name}")
    g = graphgen.road_like(4096, 1) if name == "road4096" else graphgen.rmat(24, seed=1)
    assert g.n == counts["n"] and g.m == counts["m_arcs"], "workload differs from the stored counts"
    torch.cuda.init()
    dev = torch.device("cuda", 0)

    torch.cuda.synchronize()
    t0 = time.perf_counter()
    dg = cd.cldiam_load_csr(g, dev)
    torch.cuda.synchronize()
    ingest_ms = (time.perf_counter() - t0) * 1e3
    log(f"[bench] ingest {ingest_ms:.1f} ms (H2D + validation + packing)")

    job = cd.DecomposeJob([dg], [(counts["tau"], counts["seed"], 0)], driver=args.driver,
                          local_rounds=args.local_rounds, grid_blocks=args.grid_blocks,
                          bucket_width=args.bucket_width, row_bucket_shift=args.row_shift,
                          chunk_factor=args.chunk_factor, wave_row_min=args.wave_row_min,
                          group_row_min=args.group_row_min, local_queue=args.local_queue,
                          local_cutoff=args.local_cutoff)
    qjob = cd.QuotientJob(dg)
    ejob = cd.EstimateJob(1, 1, dev)   # grows to the quotient's size on first use

    def step():
        ta = time.perf_counter()
        st = job.run()[0]
        tb = time.perf_counter()
        if args.decompose_only:
            return st, None, None, (tb - ta, 0.0, 0.0)
        q = qjob.run(job.cluster[0], job.D[0])
        tc = time.perf_counter()
        est = ejob.run(q, st.radius)
        td = time.perf_counter()
        return st, q, est, (tb - ta, tc - tb, td - tc)

    def check(st, q, est):
        ok = (st.num_clusters == counts["num_clusters"] and st.stages == counts["stages"]
              and st.delta_end == counts["delta_end"] and st.radius == counts["radius"]
              and (args.decompose_only or (q.k == counts["quotient_k"] and est[1] == counts["phi_approx"])))
        if not ok:
            log("[bench] result differs from the stored oracle values", st, est)
            sys.exit(1)

    for i in range(args.warmup):
        st, q, est, _ = step()
        log(f"[bench] warmup {i}: kernel {st.kernel_ms:.2f} ms, sweeps {st.sweeps}, iterations {st.iterations}")
    if args.warmup:
        check(st, q, est)

    torch.cuda.synchronize()
    t0 = time.perf_counter()
    kms, phases = [], []
    for i in range(args.steps):
        st, q, est, ph = step()
        kms.append(st.kernel_ms)
        phases.append(ph)
    torch.cuda.synchronize()
    check(st, q, est)
    elapsed = time.perf_counter() - t0
    ms_per_step = elapsed / args.steps * 1e3
    edges = counts["edges"]
    value = edges / (ms_per_step / 1e3) / 1e9
    kernel_ms = sum(kms) / len(kms)
    achieved = counts["bytes_decompose"] / (kernel_ms / 1e3) / 1e9
    dec_ms = sum(p[0] for p in phases) / len(phases) * 1e3
    quot_ms = sum(p[1] for p in phases) / len(phases) * 1e3
    est_ms = sum(p[2] for p in phases) / len(phases) * 1e3
    log(f"[bench] {args.steps} steps: {ms_per_step:.2f} ms/step (decompose {dec_ms:.2f}, quotient {quot_ms:.2f}, "
        f"estimate {est_ms:.2f}); decomposition kernel {kernel_ms:.2f} ms")

    cpu = None
    if not args.no_cpu_baseline:
        import oracle
        if name == "road4096":
            log("[bench] CPU baseline: oracle on the same workload, one thread")
            gs, what = g, "the full workload once"
        else:
            # the whole R-MAT 24 job takes the oracle about two minutes: time it on
            # the same generator and parameters at scale 21 (1/8 of the nodes)
            log("[bench] CPU baseline: oracle on R-MAT scale 21, one thread")
            gs = graphgen.rmat(21, seed=1)
            what = (f"R-MAT scale 21 from the same generator and parameters ({gs.n} nodes, {gs.m // 2} edges), "
                    f"tau={counts['tau']}, seed={counts['seed']}, once")
        tc0 = time.perf_counter()
        rdec = oracle.decompose(gs, counts["tau"], counts["seed"])
        tc1 = time.perf_counter()
        rq = oracle.quotient(gs, rdec)
        tc2 = time.perf_counter()
        rest = oracle.estimate(rq, rdec)
        tc = time.perf_counter() - tc0
        if gs is g:
            assert rest.phi_approx == counts["phi_approx"]
        cpu = {"value": round(gs.m // 2 / tc / 1e9, 6), "unit": "GTEPS", "cores": 1, "kind": "oracle",
               "sample": f"{what} (decompose + quotient + estimate, {tc:.1f} s single-threaded, "
                         f"host {os.cpu_count()} cpus visible)",
               "cpu_model": cpu_model(),
               "phase_s": {"decompose": round(tc1 - tc0, 3), "quotient": round(tc2 - tc1, 3),
                           "estimate": round(tc0 + tc - tc2, 3)}}

    src_sha = code_digest(os.path.join(HERE, "paper_1506_03265_amd", "csrc", "decompose.hip"))
    traffic = None
    tpath = os.path.join(HERE, "profiles", f"{name}_traffic.json")
    if os.path.exists(tpath):
        tr = json.load(open(tpath))
        if tr.get("code_sha256") == src_sha:
            traffic = tr["traffic_bytes"]   # counters taken on this very kernel code
    # random-access view: request counts of one decomposition (counters taken on
    # this kernel source) against the GPU's scattered-access ceilings
    random_access = None
    rpath = os.path.join(HERE, "profiles", f"{name}_requests.json")
    cpath = os.path.join(HERE, "profiles", "ceilings_bench.json")
    if os.path.exists(rpath) and os.path.exists(cpath):
        rq = json.load(open(rpath))
        ce = json.load(open(cpath))["config"]
        if rq.get("code_sha256") == src_sha:
            atom = rq["atomic_with_return"] + rq["atomic_without_return"]
            floor_s = atom / (ce["random_scatter_min_Gops"] * 1e9) + rq["read_requests"] / (ce["random_gather_Gops"] * 1e9)
            random_access = {"atomics": atom, "reads": rq["read_requests"], "writes": rq["write_requests"],
                             "atomics_per_s": round(atom / (kernel_ms / 1e3), 0),
                             "atomic_ceiling_per_s": ce["random_scatter_min_Gops"] * 1e9,
                             "gather_ceiling_per_s": ce["random_gather_Gops"] * 1e9,
                             "floor_ms": round(floor_s * 1e3, 3), "frac": round(floor_s * 1e3 / kernel_ms, 4)}

    return {
        "metric": METRIC,
        "value": round(value, 6),
        "unit": "GTEPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u64",
        "data": "synthetic",
        "config": {"workload": counts["text"] + f", tau={counts['tau']}, seed={counts['seed']}, "
                   "step = decompose + quotient + estimate" + (" (decompose only)" if args.decompose_only else ""),
                   "n": counts["n"], "m_arcs": counts["m_arcs"], "edges": edges,
                   "clusters": st.num_clusters, "phi_approx": None if est is None else est[1],
                   "ingest_ms": round(ingest_ms, 2), "decompose_ms": round(dec_ms, 3),
                   "quotient_ms": round(quot_ms, 3), "estimate_ms": round(est_ms, 3),
                   "decompose_gteps": round(edges / (dec_ms / 1e3) / 1e9, 4),
                   "sweeps": st.sweeps, "iterations": st.iterations, "grid_blocks": st.grid_blocks,
                   "arcs_relaxed": st.arcs_scanned,
                   "driver": "host-driven" if st.grid_blocks == 0 else "persistent"},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 2), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 5), "traffic": traffic,
                     "kernel": ("k_sweep+k_control launch loop" if st.grid_blocks == 0 else "k_persistent")
                               + " (one decomposition)", "kernel_ms": round(kernel_ms, 4),
                     "algorithmic_bytes": counts["bytes_decompose"], "random_access": random_access},
        "cpu_baseline": cpu,
    }


def batched_bench(args):
    import torch

    import graphgen
    import paper_1506_03265_amd as cd
    from paper_1506_03265_amd import tune

    count = args.graphs
    log(f"[bench] generating {count} random geometric graphs")
    graphs = graphgen.rgg_batch(count, seed=1)
    seeds = [(g_i << 32) | 1 for g_i in range(count)]
    params = [(1, s, 0) for s in seeds]
    dgs = [cd.cldiam_load_csr(g) for g in graphs]
    n_tot = sum(g.n for g in graphs)
    m_tot = sum(g.m for g in graphs)
    log(f"[bench] batch: {count} graphs, {n_tot} nodes, {m_tot} arcs")
    best = tune.tune_batch(dgs, params)
    log(f"[bench] tuner picked {best}")
    batch = cd.DecomposeJob(dgs, params, **best)
    singles = [cd.DecomposeJob([dg], [p], **best) for dg, p in zip(dgs, params)]
    for _ in range(args.warmup):
        batch.run()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        stats = batch.run()
    torch.cuda.synchronize()
    t_batch = (time.perf_counter() - t0) / args.steps
    for j in singles:
        j.run()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        for j in singles:
            j.run()
    torch.cuda.synchronize()
    t_single = (time.perf_counter() - t0) / args.steps
    same = all(bool((b == s.cluster[0]).all()) and bool((bd == s.D[0]).all())
               for b, bd, s in zip(batch.cluster, batch.D, singles))
    edges = m_tot // 2
    return {
        "metric": "batched decomposition throughput (one device job vs one job per graph)",
        "value": round(edges / t_batch / 1e9, 6), "unit": "GTEPS", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(t_batch * 1e3, 3), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "u64", "data": "synthetic",
        "config": {"workload": f"{count} random geometric graphs, sizes log-uniform in [1e3, 1e6], average "
                               "degree 8, w = round(1e4*len)+1, largest components, tau=1, seed_g=(g<<32)|1",
                   "graphs": count, "nodes": n_tot, "arcs": m_tot, "tuning": best,
                   "batched_ms": round(t_batch * 1e3, 3), "one_job_per_graph_ms": round(t_single * 1e3, 3),
                   "speedup": round(t_single / t_batch, 3), "graphs_per_s": round(count / t_batch, 1),
                   "batched_equals_single": same,
                   "sweeps": max(s.sweeps for s in stats), "iterations": stats[0].iterations},
    }


def serve_bench(args):
    import graphgen
    import paper_1506_03265_amd as cd
    from paper_1506_03265_amd import serve

    reqs_in = graphgen.serving_mix(args.requests, rate=args.rate, seed=1)

    # meshes are quantised to sides that are multiples of 256 so that the pool
    # of resident graphs stays small; R-MAT scales are 12..22
    def key(r):
        return f"grid{max(256, (r.size // 256) * 256)}" if r.kind == "grid" else f"rmat{r.size}"

    keys = sorted({key(r) for r in reqs_in})
    log(f"[bench] generating {len(keys)} resident graphs for {len(reqs_in)} requests")
    pool = {}
    sizes = {}
    for k in keys:
        if k.startswith("grid"):
            s = int(k[4:])
            g = graphgen.grid(s, s, 10000, s)
        else:
            g = graphgen.rmat(int(k[4:]), seed=int(k[4:]))
        pool[k] = cd.cldiam_load_csr(g)
        sizes[k] = (g.n, g.m)
    reqs = [serve.Request(r.rid, r.arrival_s, key(r), 1, r.rid) for r in reqs_in]
    # warm up every graph once
    serve.serve([serve.Request(i, 0.0, k, 1, 0) for i, k in enumerate(keys)], pool, workers=1)
    eng = dict(max_graphs=args.max_graphs, sweeps_per_step=args.sweeps_per_step, split_nodes=args.split_nodes)
    serve.serve_engine([serve.Request(i, 0.0, k, 1, 0) for i, k in enumerate(keys)], pool, **eng)
    log("[bench] engine run (in-engine continuous batching)")
    res_e, wall_e = serve.serve_engine(reqs, pool, workers=args.workers, **eng)
    log("[bench] stream-pool run")
    res_s, wall_s = serve.serve(reqs, pool, workers=args.workers, hbm_budget_bytes=200 << 30)
    log("[bench] plain sequential run")
    res_p, wall_p = serve.serve(reqs, pool, workers=1, hbm_budget_bytes=200 << 30)

    def same(xs, ys):
        return all((a.num_clusters, a.radius, a.phi_gc, a.phi_approx) == (b.num_clusters, b.radius, b.phi_gc,
                                                                         b.phi_approx) for a, b in zip(xs, ys))

    edges = sum(sizes[r.graph][1] // 2 for r in reqs)

    def summary(res, wall):
        lat = [r.latency_s * 1e3 for r in res]
        return {"p50_ms": round(serve.percentile(lat, 50), 3), "p99_ms": round(serve.percentile(lat, 99), 3),
                "req_per_s": round(len(res) / wall, 3), "wall_s": round(wall, 3),
                "gteps": round(edges / wall / 1e9, 4)}

    return {
        "metric": "served decompose+estimate: p50/p99 latency and requests/s, served vs plain",
        "value": round(len(reqs) / wall_s, 3), "unit": "req/s", "n_gpus": 1, "steps": len(reqs),
        "warmup": len(keys), "ms_per_step": round(wall_s / len(reqs) * 1e3, 4), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "u64", "data": "synthetic",
        "config": {"workload": f"{len(reqs)} Poisson requests at {args.rate}/s: half meshes (side 256-2048, "
                               "w in [1,1e4]), half R-MAT scale 12-22 (w in [1,2^20]), tau=1, seed=request id",
                   "resident_graphs": len(keys), "engine_slots": args.max_graphs,
                   "sweeps_per_step": args.sweeps_per_step, "engine_split_nodes": args.split_nodes,
                   "workers": args.workers, "hbm_budget_gb": 200,
                   "served": "stream_pool", "stream_pool": summary(res_s, wall_s), "engine": summary(res_e, wall_e),
                   "plain": summary(res_p, wall_p),
                   "engine_equals_plain": same(res_e, res_p), "stream_pool_equals_plain": same(res_s, res_p)},
    }


def _sssp_lower_bound(cd, dg, src, sweeps=4):
    """Iterated SSSP: each sweep starts from the farthest node of the previous
    one; the largest eccentricity found is a lower bound on the diameter."""
    import torch
    lb, s = 0, src
    for _ in range(sweeps):
        dist, mx = cd.cldiam_sssp_delta_stepping(dg, s, 0)
        lb = max(lb, int(mx))
        d = dist.to(torch.int64) & 0xFFFFFFFF
        d[d == 0xFFFFFFFF] = -1
        s = int(torch.argmax(d).item())
    return lb


def _pipeline(cd, dg, tau, seed, delta0=0, variant=0, step_cap=0, reps=3):
    """Best-of-reps time of decompose + quotient + estimate; returns (stats,
    (phi_gc, phi_approx), seconds, decompose seconds)."""
    import torch
    best = None
    for _ in range(reps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        c, D, st = cd.cldiam_decompose(dg, tau, seed, delta0=delta0, variant=variant, step_cap=step_cap)
        t1 = time.perf_counter()
        q = cd.cldiam_build_quotient(dg, c, D)
        est = cd.cldiam_estimate_diameter(q, st.radius)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        if best is None or t2 - t0 < best[2]:
            best = (st, est, t2 - t0, t1 - t0)
    return best


def variants_bench(args):
    """CLUSTER (fixpoint growth), the literal step-synchronous variant and
    CLUSTER2 on the road-like mesh: time, rounds/work, clusters and the
    estimate's ratio to an iterated-SSSP lower bound on the diameter."""
    import graphgen
    import oracle   # only for the SSSP source rule shared with the tests
    import paper_1506_03265_amd as cd
    counts = json.load(open(os.path.join(HERE, "tests", "golden", "road4096_counts.json")))
    log("[bench] generating road4096")
    g = graphgen.road_like(4096, 1)
    dg = cd.cldiam_load_csr(g)
    lb = _sssp_lower_bound(cd, dg, oracle.sssp_source(g.n, counts["seed"]))
    rows = {}
    for name, var in (("cluster", cd.VARIANT_FIXPOINT), ("steps", cd.VARIANT_STEPS),
                      ("cluster2", cd.VARIANT_CLUSTER2)):
        st, est, t, td = _pipeline(cd, dg, counts["tau"], counts["seed"], variant=var, reps=args.steps)
        ref = counts if name == "cluster" else counts[name]
        ok = st.num_clusters == ref["num_clusters"] and est[1] == ref["phi_approx"]
        if not ok:
            log(f"[bench] {name} differs from the stored oracle values")
            sys.exit(1)
        rows[name] = {"ms": round(t * 1e3, 3), "decompose_ms": round(td * 1e3, 3), "clusters": st.num_clusters,
                      "stages": st.stages, "levels": st.levels, "radius": st.radius, "phi_approx": est[1],
                      "ratio_to_lower_bound": round(est[1] / lb, 4), "sweeps": st.sweeps}
        if name == "steps":
            rows[name].update(rounds=st.rounds, messages=st.messages, updates=st.updates)
        if name == "cluster2":
            rows[name].update(radius1=st.radius1)
        log(f"[bench] {name}: {rows[name]}")
    t = rows["cluster"]["ms"]
    return {
        "metric": "CLUSTER vs literal steps vs CLUSTER2 on the road-like mesh: ms per decompose+quotient+estimate",
        "value": round(counts["edges"] / (t / 1e3) / 1e9, 6), "unit": "GTEPS", "n_gpus": 1, "steps": args.steps,
        "warmup": 0, "ms_per_step": t, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "u64", "data": "synthetic",
        "config": {"workload": counts["text"] + f", tau={counts['tau']}, seed={counts['seed']}",
                   "sssp_lower_bound": lb, "variants": rows},
    }


def delta0_bench(args):
    """Initial-Delta experiment (Section 5): a 2048 x 2048 mesh whose edges
    weigh 10^6 with probability 0.1 and 1 otherwise; CL-DIAM started from the
    minimum weight, from the mean weight and from about the diameter, under
    both the fixpoint growth (the default) and the literal step-synchronous
    PartialGrowth.  Only the literal form stops a growth after the step that
    covers half of the nodes, whatever the distances reached by then, so
    only it can show the paper's loss of quality for a large initial Delta."""
    import graphgen
    import oracle
    import paper_1506_03265_amd as cd
    side = args.side
    log(f"[bench] generating the bimodal mesh {side}x{side}")
    g = graphgen.bimodal_mesh(side, 1)
    dg = cd.cldiam_load_csr(g)
    lb = _sssp_lower_bound(cd, dg, oracle.sssp_source(g.n, 1))
    mean = int(dg.weight_sum // max(g.m, 1))
    rows = []
    for vname, var in (("fixpoint", cd.VARIANT_FIXPOINT), ("steps", cd.VARIANT_STEPS)):
        for label, d0 in (("min weight", 1), ("mean weight", mean), ("~diameter", lb)):
            st, est, t, td = _pipeline(cd, dg, args.tau, 1, delta0=d0, variant=var, reps=args.steps)
            rows.append({"variant": vname, "delta0": label, "value": d0, "ms": round(t * 1e3, 3),
                         "levels": st.levels, "sweeps": st.sweeps, "stages": st.stages, "delta_end": st.delta_end,
                         "clusters": st.num_clusters, "radius": st.radius, "phi_approx": est[1],
                         "ratio_to_lower_bound": round(est[1] / lb, 4)})
            if var == cd.VARIANT_STEPS:
                rows[-1].update(rounds=st.rounds, messages=st.messages, updates=st.updates)
            log(f"[bench] {vname} delta0 {label}: {rows[-1]}")
    by = {(r["variant"], r["delta0"]): r for r in rows}
    return {
        "metric": "initial-Delta experiment: approximation ratio to an SSSP lower bound and time per initial Delta",
        "value": by[("steps", "~diameter")]["ratio_to_lower_bound"], "unit": "ratio", "n_gpus": 1,
        "steps": args.steps, "warmup": 0, "ms_per_step": by[("steps", "~diameter")]["ms"],
        "higher_is_better": False, "scaling": "weak", "vs_baseline": None, "dtype": "u64", "data": "synthetic",
        "config": {"workload": f"{side}x{side} mesh, weights 10^6 w.p. 0.1 else 1, graph seed 1, tau={args.tau}; "
                               "value = literal step-synchronous variant started at about the diameter",
                   "n": g.n, "m_arcs": g.m, "sssp_lower_bound": lb,
                   "paper": "Section 5 reports about 2.5x for an initial Delta equal to the diameter against "
                            "1.0001 for the minimum weight (Spark, real weights)",
                   "runs": rows},
    }


def stepcap_bench(args):
    """Growing-step cap O(n / tau) (Section 4): the literal step-synchronous
    variant with caps of n/tau, n/(16 tau), n/(256 tau) and n/(1024 tau) steps
    per PartialGrowth call, on a mesh with skewed weights, on R-MAT and on a
    path (the deepest topology)."""
    import graphgen
    import oracle
    import paper_1506_03265_amd as cd
    out = {}
    path = graphgen.grid(1, 1 << 16, 100, 3)   # a path: growth needs as many steps as hops
    path.name = "path65536"
    for gname, g in (("bimodal512", graphgen.bimodal_mesh(512, 2)), ("rmat18", graphgen.rmat(18, seed=2)),
                     ("path65536", path)):
        dg = cd.cldiam_load_csr(g)
        lb = _sssp_lower_bound(cd, dg, oracle.sssp_source(g.n, 1))
        rows = []
        for div in (0, 1, 16, 256, 1024):
            cap = 0 if div == 0 else max(1, g.n // (args.tau * div))
            st, est, t, td = _pipeline(cd, dg, args.tau, 1, variant=cd.VARIANT_STEPS, step_cap=cap, reps=args.steps)
            rows.append({"step_cap": cap, "ms": round(t * 1e3, 3), "rounds": st.rounds, "messages": st.messages,
                         "updates": st.updates, "stages": st.stages, "levels": st.levels,
                         "clusters": st.num_clusters, "phi_approx": est[1],
                         "ratio_to_lower_bound": round(est[1] / lb, 4)})
            log(f"[bench] {gname} cap {cap}: {rows[-1]}")
        out[gname] = {"n": g.n, "m_arcs": g.m, "sssp_lower_bound": lb, "runs": rows}
    r = out["bimodal512"]["runs"][0]
    return {
        "metric": "growing-step cap: rounds, work and approximation ratio of the literal variant per cap",
        "value": r["rounds"], "unit": "rounds", "n_gpus": 1, "steps": args.steps, "warmup": 0,
        "ms_per_step": r["ms"], "higher_is_better": False, "scaling": "weak", "vs_baseline": None,
        "dtype": "u64", "data": "synthetic", "config": {"workload": f"tau={args.tau}", "graphs": out},
    }


def ceilings_bench(args):
    """Random-access ceilings of the GPU with plain PyTorch kernels: a
    streaming copy, random 8-byte gathers, and random 64-bit scatter-min
    (atomic) over a 134 MB array, the size of the road mesh's key array.
    These bound a relaxation engine whose work is one random gather per arc
    and one or two random atomics per improvement."""
    import torch
    n, ops = 1 << 24, 1 << 26
    a = torch.full((n,), 1 << 62, dtype=torch.int64, device="cuda")
    b = torch.empty_like(a)
    g = torch.Generator(device="cuda")
    g.manual_seed(1)
    idx = torch.randint(0, n, (ops,), device="cuda", generator=g)
    vals = torch.randint(0, 1 << 40, (ops,), device="cuda", dtype=torch.int64, generator=g)
    out = {}

    def timed(fn, reps=5):
        fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / reps

    t = timed(lambda: b.copy_(a))
    out["copy_GBps"] = round(2 * n * 8 / t / 1e9, 1)
    t = timed(lambda: a.index_select(0, idx))
    out["random_gather_Gops"] = round(ops / t / 1e9, 2)
    t = timed(lambda: a.scatter_reduce_(0, idx, vals, reduce="amin"))
    out["random_scatter_min_Gops"] = round(ops / t / 1e9, 2)
    srt = torch.sort(idx).values
    t = timed(lambda: a.index_select(0, srt))
    out["sorted_gather_Gops"] = round(ops / t / 1e9, 2)
    log(f"[bench] ceilings {out}")
    return {
        "metric": "random-access ceilings (streaming copy GB/s, random gathers and random 64-bit atomic min per s)",
        "value": out["random_scatter_min_Gops"], "unit": "Gatomics/s", "n_gpus": 1, "steps": 5, "warmup": 1,
        "ms_per_step": None, "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "int64",
        "data": "synthetic", "config": {"workload": f"{n} int64 array (134 MB), {ops} random indices", **out},
    }


def mesh29_bench(args):
    """The whole step on a 16384 x 32768 mesh with 1% diagonals: 2^29 nodes
    (R-MAT scale 29's node count) and 2,158M arcs, beyond 32-bit row offsets.
    No oracle run fits this size; the run checks properties that hold at any
    size: every node is labelled by a center that labels itself at D = 0, the
    labels are the quotient's nodes, for two clusters the exact distances from
    their centers (Delta-stepping SSSP) never exceed D, and Phi_approx is at
    least every such eccentricity."""
    import torch

    import graphgen
    import paper_1506_03265_amd as cd

    tau, seed = 4, 1
    rows, cols = (int(x) for x in args.mesh_shape.split("x"))
    log(f"[bench] generating the {rows} x {cols} mesh with 1% diagonals")
    t0 = time.perf_counter()
    g = graphgen.mesh64(rows, cols, 10**4, 1, 0.01)
    gen_s = time.perf_counter() - t0
    n, m = g.n, g.m
    log(f"[bench] generated n={n} m={m} arcs in {gen_s:.1f} s")
    torch.cuda.init()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    dg = cd.cldiam_load_csr(g)
    torch.cuda.synchronize()
    ingest_ms = (time.perf_counter() - t0) * 1e3
    del g
    torch.cuda.empty_cache()
    log(f"[bench] ingest {ingest_ms:.0f} ms (H2D + validation + packing)")
    job = cd.DecomposeJob([dg], [(tau, seed, 0)], driver=args.driver)
    qjob = cd.QuotientJob(dg)
    ejob = cd.EstimateJob(1, 1, dg.row_ptr.device)

    def step():
        ta = time.perf_counter()
        st = job.run()[0]
        tb = time.perf_counter()
        q = qjob.run(job.cluster[0], job.D[0])
        tc = time.perf_counter()
        est = ejob.run(q, st.radius)
        td = time.perf_counter()
        return st, q, est, (tb - ta, tc - tb, td - tc)

    for i in range(args.warmup):
        st, q, est, ph = step()
        log(f"[bench] warmup {i}: decompose {ph[0] * 1e3:.1f} ms, quotient {ph[1] * 1e3:.1f} ms, "
            f"{st.sweeps} sweeps, {st.num_clusters} clusters")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    phases = []
    for i in range(args.steps):
        st, q, est, ph = step()
        phases.append(ph)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) / args.steps * 1e3
    log(f"[bench] {args.steps} steps: {ms:.1f} ms/step")

    # properties that hold at any size
    cl = job.cluster[0]
    D = job.D[0]
    assert int(cl.min()) >= 0 and int(cl.max()) < n, "a node without a valid label"
    lab = cl.long()
    assert bool((cl[lab] == cl).all()), "a label that is not a center"
    centers = torch.nonzero(cl == torch.arange(n, device=cl.device, dtype=torch.int32)).flatten()
    assert bool((D[centers] == 0).all()), "a center with D > 0"
    assert centers.numel() == st.num_clusters == q.k, "centers, cluster count and quotient size differ"
    assert bool((q.center.long() == centers).all()), "quotient nodes are not the centers in ascending order"
    phi, approx = est
    del qjob, q
    torch.cuda.empty_cache()
    checks = []
    for v in (0, n - 1):
        c = int(cl[v])
        dist, ecc = cd.cldiam_sssp_delta_stepping(dg, c)
        mine = cl == c
        dd = dist.long() & 0xFFFFFFFF
        assert bool((dd[mine] <= D[mine]).all()), f"D below the exact distance in cluster {c}"
        assert ecc <= approx, f"Phi_approx {approx} below the eccentricity {ecc} of node {c}"
        checks.append({"center": c, "nodes": int(mine.sum()), "ecc": ecc, "max_D": int(D[mine].max())})
        del dist, dd, mine
    log(f"[bench] checks passed: {checks}")
    dec_ms = sum(p[0] for p in phases) / len(phases) * 1e3
    quot_ms = sum(p[1] for p in phases) / len(phases) * 1e3
    est_ms = sum(p[2] for p in phases) / len(phases) * 1e3
    edges = m // 2
    return {
        "metric": "decomposition GTEPS on a mesh past 32-bit row offsets",
        "value": round(edges / (ms / 1e3) / 1e9, 6), "unit": "GTEPS", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms, 3), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "u64", "data": "synthetic",
        "config": {"workload": f"{rows}x{cols} mesh, every grid edge, 1% diagonals, weights uniform in [1, 1e4], "
                               f"graph seed 1, tau={tau}, seed={seed}, step = decompose + quotient + estimate",
                   "n": n, "m_arcs": m, "edges": edges, "generate_s": round(gen_s, 1),
                   "ingest_ms": round(ingest_ms, 1), "decompose_ms": round(dec_ms, 2),
                   "quotient_ms": round(quot_ms, 2), "estimate_ms": round(est_ms, 3),
                   "clusters": st.num_clusters, "stages": st.stages, "levels": st.levels, "radius": st.radius,
                   "sweeps": st.sweeps, "arcs_relaxed": st.arcs_scanned, "phi_gc": phi, "phi_approx": approx,
                   "property_checks": checks},
        "roofline": None, "cpu_baseline": None,
    }


def sssp_bench(args):
    import torch

    import graphgen
    import paper_1506_03265_amd as cd

    counts = json.load(open(os.path.join(HERE, "tests", "golden", "road4096_counts.json")))
    log("[bench] generating road4096 for the SSSP competitor")
    g = graphgen.road_like(4096, 1)
    dg = cd.cldiam_load_csr(g)
    import oracle   # only for the source rule shared with the tests (a Philox draw) and the CPU baseline
    src = oracle.sssp_source(g.n, counts["seed"])
    widths = [int(x) for x in args.bucket_widths.split(",")] if args.bucket_widths else \
        [max(1, dg.weight_sum // max(dg.m, 1)) * f for f in (1, 4, 16, 64, 256)]
    rows = []
    best = None
    for bd in widths:
        dist, mx = cd.cldiam_sssp_delta_stepping(dg, src, bd)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            dist, mx = cd.cldiam_sssp_delta_stepping(dg, src, bd)
        torch.cuda.synchronize()
        t = (time.perf_counter() - t0) / args.steps
        rows.append({"bucket_delta": bd, "ms": round(t * 1e3, 3)})
        log(f"[bench] SSSP bucket width {bd}: {t * 1e3:.2f} ms, 2-approximation {2 * mx}")
        if best is None or t < best[0]:
            best = (t, bd, mx)
    cpu = None
    if not args.no_cpu_baseline:
        tc0 = time.perf_counter()
        rd, rmx = oracle.sssp(g, src)
        tc = time.perf_counter() - tc0
        assert rmx == best[2]
        cpu = {"value": round(counts["edges"] / tc / 1e9, 6), "unit": "GTEPS", "cores": 1, "kind": "oracle",
               "sample": f"Dijkstra from the same source on the full workload ({tc:.1f} s single-threaded)",
               "cpu_model": cpu_model()}
    t, bd, mx = best
    return {
        "metric": "Delta-stepping SSSP 2-approximation (the competitor), edges per second",
        "value": round(counts["edges"] / t / 1e9, 6), "unit": "GTEPS", "n_gpus": 1, "steps": args.steps,
        "warmup": 1, "ms_per_step": round(t * 1e3, 3), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "u32", "data": "synthetic",
        "config": {"workload": counts["text"] + f", source = Philox rule, seed {counts['seed']}",
                   "source": src, "best_bucket_delta": bd, "max_dist": mx, "two_approx": 2 * mx,
                   "cl_diam_phi_approx": counts["phi_approx"], "widths": rows},
        "cpu_baseline": cpu,
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="road4096",
                    choices=["road4096", "rmat24", "rgg256", "serve", "sssp", "variants", "delta0", "stepcap",
                             "ceilings", "mesh29"])
    ap.add_argument("--side", type=int, default=2048, help="delta0: mesh side")
    ap.add_argument("--mesh-shape", default="16384x32768", help="mesh29: rows x cols")
    ap.add_argument("--tau", type=int, default=4, help="delta0 / stepcap: tau")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--driver", type=int, default=0, help="0 auto, 1 host-driven, 2 persistent")
    ap.add_argument("--local-rounds", type=int, default=-1)
    ap.add_argument("--grid-blocks", type=int, default=0)
    ap.add_argument("--row-shift", type=int, default=0,
                    help="long-row bucket: Delta / 2^shift (0 = library default, < 0 = none)")
    ap.add_argument("--bucket-width", type=float, default=0.0,
                    help="relaxation distance bucket in mean arc weights (0 default, < 0 none)")
    ap.add_argument("--chunk-factor", type=int, default=0, help="growth chunks per workgroup (0 = default)")
    ap.add_argument("--wave-row-min", type=int, default=0, help="rows above this many arcs go to a wave (0 = default)")
    ap.add_argument("--group-row-min", type=int, default=0,
                    help="rows above this many arcs go to the workgroup (0 = default)")
    ap.add_argument("--local-queue", type=int, default=0, help="local queue tile (0 = default)")
    ap.add_argument("--local-cutoff", type=int, default=0,
                    help="percentage of finished workgroups that ends local rounds (0 = default)")
    ap.add_argument("--decompose-only", action="store_true", help="time only the decomposition (for profiles)")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="first copy a 1 GiB device buffer three times (reference kernel for HBM counters)")
    ap.add_argument("--graphs", type=int, default=256, help="rgg256: number of graphs")
    ap.add_argument("--requests", type=int, default=2000, help="serve: number of requests")
    ap.add_argument("--rate", type=float, default=200.0, help="serve: arrivals per second")
    ap.add_argument("--workers", type=int, default=4, help="serve: concurrent requests (stream pool) or "
                    "quotient/estimate threads (engine)")
    ap.add_argument("--max-graphs", type=int, default=32, help="serve: graph slots of the engine")
    ap.add_argument("--sweeps-per-step", type=int, default=4, help="serve: engine sweeps between admissions")
    ap.add_argument("--split-nodes", type=int, default=1 << 20,
                    help="serve: graphs of at least this many nodes go to a second engine server (0: one server)")
    ap.add_argument("--bucket-widths", default="", help="sssp: comma-separated bucket widths to try")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on exactly one GPU: the multi-GPU path is not built", file=sys.stderr)
        sys.exit(2)
    if args.calibrate_copy:
        import torch
        x = torch.empty(1 << 27, dtype=torch.int64, device="cuda")
        x.fill_(1)
        y = torch.empty_like(x)
        for _ in range(3):
            y.copy_(x)
        torch.cuda.synchronize()
        del x, y
    if args.workload in ("road4096", "rmat24"):
        out = step_bench(args, args.workload)
    elif args.workload == "rgg256":
        out = batched_bench(args)
    elif args.workload == "sssp":
        out = sssp_bench(args)
    elif args.workload == "variants":
        out = variants_bench(args)
    elif args.workload == "delta0":
        out = delta0_bench(args)
    elif args.workload == "stepcap":
        out = stepcap_bench(args)
    elif args.workload == "ceilings":
        out = ceilings_bench(args)
    elif args.workload == "mesh29":
        out = mesh29_bench(args)
    else:
        out = serve_bench(args)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
