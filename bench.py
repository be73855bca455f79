"""Benchmark of the CL-DIAM hot path on one MI355X.

A step is one pass of the whole path over the workload, inputs resident in
HBM: decomposition (CLUSTER, Algorithm 1), weighted quotient graph and the
diameter estimate (Section 4).  Ingest (validation + weight-sorted packing of
the CSR) runs once before the clock and is reported separately.

Workload: the road-like 4096x4096 mesh (16.8M nodes, 64.1M arcs) with tau = 4,
seed 1, initial Delta = mean arc weight.  Throughput is edges per second
(undirected input edges / step time), in GTEPS.

The roofline object covers the dominant kernel, the decomposition's sweep
kernel: algorithmic bytes of one decomposition (work counts of the sequential
oracle run, stored by tests/golden/make_workload_counts.py) divided by the
device time of the decomposition's launch loop (all its sweep and control
launches), measured by the library with HIP events on the caller's stream,
against the 8 TB/s HBM peak.  The CPU baseline times the oracle on the host on the same
workload (single thread).

Prints one JSON line.  Only one GPU is supported.
"""
import argparse
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, HERE)

HBM_PEAK_GBS = 8000.0


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--driver", type=int, default=0, help="0 auto, 1 host-driven, 2 persistent")
    ap.add_argument("--decompose-only", action="store_true", help="time only the decomposition (for profiles)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on exactly one GPU: this build has no multi-GPU path (see DESIGN.md for how it "
              "would shard)", file=sys.stderr)
        sys.exit(2)

    import torch

    import graphgen
    import paper_1506_03265_amd as cd

    counts = json.load(open(os.path.join(HERE, "tests", "golden", "road4096_counts.json")))
    log("[bench] generating road-like 4096x4096 workload")
    g = graphgen.road_like(4096, 1)
    assert g.n == counts["n"] and g.m == counts["m_arcs"], "workload differs from the stored counts"
    torch.cuda.init()
    dev = torch.device("cuda", 0)

    torch.cuda.synchronize()
    t0 = time.perf_counter()
    dg = cd.cldiam_load_csr(g, dev)
    torch.cuda.synchronize()
    ingest_ms = (time.perf_counter() - t0) * 1e3
    log(f"[bench] ingest {ingest_ms:.1f} ms (H2D + validation + packing)")

    job = cd.DecomposeJob([dg], [(counts["tau"], counts["seed"], 0)], driver=args.driver)
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

    for i in range(args.warmup):
        st, q, est, _ = step()
        log(f"[bench] warmup {i}: kernel {st.kernel_ms:.2f} ms, sweeps {st.sweeps}, iterations {st.iterations}")
    ok = (st.num_clusters == counts["num_clusters"] and st.stages == counts["stages"]
          and st.delta_end == counts["delta_end"] and st.radius == counts["radius"]
          and (args.decompose_only or (q.k == counts["quotient_k"] and est[1] == counts["phi_approx"])))
    if not ok:
        log("[bench] result differs from the stored oracle values", st, est)
        sys.exit(1)

    torch.cuda.synchronize()
    t0 = time.perf_counter()
    kms, phases = [], []
    for i in range(args.steps):
        st, q, est, ph = step()
        kms.append(st.kernel_ms)
        phases.append(ph)
    torch.cuda.synchronize()
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
        log("[bench] CPU baseline: oracle on the same workload, one thread")
        tc0 = time.perf_counter()
        rdec = oracle.decompose(g, counts["tau"], counts["seed"])
        rq = oracle.quotient(g, rdec)
        rest = oracle.estimate(rq, rdec)
        tc = time.perf_counter() - tc0
        assert rest.phi_approx == counts["phi_approx"]
        cpu = {"value": round(edges / tc / 1e9, 6), "unit": "GTEPS", "cores": 1, "kind": "oracle",
               "sample": f"the full workload once (decompose + quotient + estimate, {tc:.1f} s single-threaded, "
                         f"host {os.cpu_count()} cpus visible)"}

    out = {
        "metric": "decomposition GTEPS + % HBM roofline; p50/p99 latency served vs plain, bit-exact",
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
                   "arcs_relaxed": st.arcs_scanned, "driver": "host-driven" if st.grid_blocks == 0 else "persistent"},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 2), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 5), "traffic": None,
                     "kernel": ("k_sweep+k_control launch loop" if st.grid_blocks == 0 else "k_persistent")
                               + " (one decomposition)", "kernel_ms": round(kernel_ms, 4),
                     "algorithmic_bytes": counts["bytes_decompose"]},
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
