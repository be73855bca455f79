"""GPU parity: the HIP path through the C ABI against the CPU oracle, bit for
bit, on seeded synthetic inputs.

Everything here is integer work, so the bar is exact equality: cluster ids,
D, per-stage counts, Delta, the quotient graph (centers, CSR, weights), the
estimate and the SSSP distances.  Graphs span several waves/tiles with ragged
tails, tiny edge cases (one node, no edges, disconnected, ties), and the
full-size road-like workload in the launch configuration the benchmark uses.
"""
import functools
import sys

import numpy as np
import pytest

import graphgen
import oracle
import paper_1506_03265_amd as cd

pytestmark = pytest.mark.gpu

DRIVERS = [cd.DRIVER_HOST, cd.DRIVER_PERSISTENT]
DRIVER_IDS = ["host", "persistent"]


def _say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    cd.load_library()


def _tiny_graphs():
    rng = np.random.default_rng(777)
    out = [("grid_small", graphgen.grid_small()), ("grid13", graphgen.grid(13, 17, 3, 5))]
    for i in range(6):
        n = int(rng.integers(90, 300))
        out.append((f"er{i}", graphgen.random_small(rng, n, float(rng.choice([0.02, 0.05])),
                                                    int(rng.choice([1, 2, 50, 10000])), connected=bool(i % 2))))
    n = 200
    out.append(("path", graphgen.csr_from_edges_np(n, range(n - 1), range(1, n), [1] * (n - 1))))
    out.append(("star", graphgen.csr_from_edges_np(n, [0] * (n - 1), range(1, n), list(range(1, n)))))
    a = [(i, i + 1) for i in range(99)] + [(100 + i, 101 + i) for i in range(99)]
    out.append(("twocomp", graphgen.csr_from_edges_np(200, [x for x, _ in a], [y for _, y in a], [3] * len(a))))
    out.append(("noedges", graphgen.csr_from_edges_np(120, [], [], [])))
    out.append(("single", graphgen.csr_from_edges_np(1, [], [], [])))
    out.append(("pair", graphgen.csr_from_edges_np(2, [0], [1], [7])))
    return out


TINY = _tiny_graphs()


@functools.lru_cache(maxsize=None)
def _oracle_dec(name, tau, seed, delta0=0):
    g = _GRAPHS[name]
    return oracle.decompose(g, tau, seed, delta0=delta0)


_GRAPHS = dict(TINY)


def _check_decomposition(name, g, tau, seed, driver, delta0=0):
    _say(f"[parity] decompose {name} n={g.n} m={g.m} tau={tau} seed={seed} driver={driver}")
    dg = cd.cldiam_load_csr(g)
    cluster, D, st = cd.cldiam_decompose(dg, tau, seed, delta0=delta0, driver=driver)
    ref = _oracle_dec(name, tau, seed, delta0) if name in _GRAPHS else oracle.decompose(g, tau, seed, delta0=delta0)
    got_c = cluster.cpu().numpy()
    got_D = cd.u64(D)
    assert np.array_equal(got_c, ref.cluster), f"{name}: cluster differs at {np.nonzero(got_c != ref.cluster)[0][:10]}"
    assert np.array_equal(got_D, ref.D), f"{name}: D differs at {np.nonzero(got_D != ref.D)[0][:10]}"
    assert st.stages == ref.stages
    assert st.levels == ref.levels
    assert st.delta0 == ref.delta0 and st.delta_end == ref.delta_end
    assert st.stop == ref.stop
    assert st.num_clusters == ref.num_clusters and st.singletons == ref.singletons
    assert st.radius == ref.radius
    k = min(st.stages, cd.STAGE_LOG)
    assert st.stage_uncovered == ref.stage_uncovered[:k]
    assert st.stage_centers == ref.stage_centers[:k]
    assert st.stage_covered == ref.stage_covered[:k]
    assert st.stage_delta == ref.stage_delta[:k]
    return dg, cluster, D, st, ref


# ------------------------------------------------------------------ ingest --

@pytest.mark.parametrize("name,g", TINY[:4] + [("rmat10", graphgen.rmat(10, seed=2))], ids=lambda x: x if isinstance(x, str) else "")
def test_ingest_packs_weight_sorted_rows(name, g):
    _say(f"[parity] ingest {name}")
    dg = cd.cldiam_load_csr(g)
    arcs = cd.u64(dg.arcs)[:g.m]
    exp = (g.w.astype(np.uint64) << np.uint64(32)) | g.col.astype(np.uint64)
    for u in range(g.n):
        s, t = g.row_ptr[u], g.row_ptr[u + 1]
        assert np.array_equal(arcs[s:t], np.sort(exp[s:t])), f"row {u}"
    assert dg.weight_sum == int(g.w.astype(np.int64).sum())


def test_ingest_sorts_hub_rows():
    """Rows above the per-thread and LDS sort sizes (a star with a hub of
    degree 20000 and random weights)."""
    rng = np.random.default_rng(5)
    n = 20001
    w = rng.integers(1, 2**20, size=n - 1)
    g = graphgen.csr_from_edges_np(n, [0] * (n - 1), range(1, n), w)
    _say("[parity] ingest hub")
    dg = cd.cldiam_load_csr(g)
    arcs = cd.u64(dg.arcs)[:g.m]
    exp = (g.w.astype(np.uint64) << np.uint64(32)) | g.col.astype(np.uint64)
    assert np.array_equal(arcs[:n - 1], np.sort(exp[:n - 1]))
    assert np.array_equal(arcs[n - 1:], exp[n - 1:])


def test_ingest_sorts_many_hub_rows_together():
    """300 hub rows of 8,200 to 9,000 arcs each (more than 256 rows in one
    batch, so the stable regrouping by row takes two radix digits), weights
    drawn from a small range so that equal weights are ordered by column."""
    rng = np.random.default_rng(9)
    hubs, leaves = 300, 20000
    us, vs, ws = [], [], []
    for h in range(hubs):
        deg = int(rng.integers(8200, 9001))
        nb = rng.choice(leaves, size=deg, replace=False) + hubs
        us.append(np.full(deg, h))
        vs.append(nb)
        ws.append(rng.integers(1, 50, size=deg))
    g = graphgen.csr_from_edges_np(hubs + leaves, np.concatenate(us), np.concatenate(vs), np.concatenate(ws))
    _say(f"[parity] ingest {hubs} hub rows, m={g.m}")
    dg = cd.cldiam_load_csr(g)
    arcs = cd.u64(dg.arcs)[:g.m]
    exp = (g.w.astype(np.uint64) << np.uint64(32)) | g.col.astype(np.uint64)
    for u in range(g.n):
        s, t = g.row_ptr[u], g.row_ptr[u + 1]
        assert np.array_equal(arcs[s:t], np.sort(exp[s:t])), f"row {u}"


def test_ingest_rejects_asymmetric_csr():
    g = graphgen.grid(6, 6, 10, 1)
    w = g.w.copy()
    w[3] += 1   # breaks the weight symmetry of one edge
    bad = graphgen.Graph(g.n, g.row_ptr, g.col, w)
    with pytest.raises(cd.CldiamError) as e:
        cd.cldiam_load_csr(bad)
    assert e.value.status == cd.CLDIAM_EINVAL


def test_ingest_rejects_self_loop_and_unsorted_row():
    g = graphgen.csr_from_edges_np(3, [0, 1], [1, 2], [1, 1])
    col = g.col.copy()
    col[0] = 0   # self loop at node 0
    with pytest.raises(cd.CldiamError):
        cd.cldiam_load_csr(graphgen.Graph(3, g.row_ptr, col, g.w))


# ------------------------------------------------------------ decompose --

@pytest.mark.parametrize("driver", DRIVERS, ids=DRIVER_IDS)
@pytest.mark.parametrize("name,g", TINY, ids=[n for n, _ in TINY])
def test_decompose_tiny(name, g, driver):
    _check_decomposition(name, g, 1, 1, driver)


@pytest.mark.parametrize("driver", DRIVERS, ids=DRIVER_IDS)
@pytest.mark.parametrize("tau,seed,delta0", [(1, 7, 0), (2, 3, 0), (1, 5, 1), (3, 11, 50000)])
def test_decompose_params(tau, seed, delta0, driver):
    g = graphgen.grid_small(seed)
    _check_decomposition("grid_small_params", g, tau, seed, driver, delta0)


@pytest.mark.parametrize("driver", DRIVERS, ids=DRIVER_IDS)
def test_decompose_overflow_matches_oracle(driver):
    n = 128
    g = graphgen.csr_from_edges_np(n, range(n - 1), range(1, n), [2**31] * (n - 1))
    with pytest.raises(oracle.OracleError):
        oracle.decompose(g, 1, 1, delta0=2**31)
    dg = cd.cldiam_load_csr(g)
    with pytest.raises(cd.CldiamError) as e:
        cd.cldiam_decompose(dg, 1, 1, delta0=2**31, driver=driver)
    assert e.value.status == cd.CLDIAM_EOVERFLOW


def _hub_graph(n=30000, seed=3):
    """A hub joined to every node plus a path through the leaves: rows far
    above the per-thread size, relaxed by the whole workgroup."""
    rng = np.random.default_rng(seed)
    u = [0] * (n - 1) + list(range(1, n - 1))
    v = list(range(1, n)) + list(range(2, n))
    w = list(rng.integers(1, 10**6, size=n - 1)) + list(rng.integers(1, 1000, size=n - 2))
    return graphgen.csr_from_edges_np(n, u, v, w)


MEDIUM = [("road512", lambda: graphgen.road_like(512, 3), 2), ("rmat14", lambda: graphgen.rmat(14, seed=4), 1),
          ("grid300", lambda: graphgen.grid(300, 257, 10000, 9), 1), ("rmat17", lambda: graphgen.rmat(17, seed=5), 2),
          ("hub30k", _hub_graph, 1)]


@pytest.mark.parametrize("driver", DRIVERS, ids=DRIVER_IDS)
@pytest.mark.parametrize("name,maker,tau", MEDIUM, ids=[m[0] for m in MEDIUM])
def test_decompose_medium(name, maker, tau, driver):
    g = maker()
    _check_decomposition(name, g, tau, 1, driver)


# -------------------------------------------------- quotient + estimate --

@pytest.mark.parametrize("name,maker,tau", [("grid_small", graphgen.grid_small, 1),
                                            ("road256", lambda: graphgen.road_like(256, 2), 1),
                                            ("rmat12", lambda: graphgen.rmat(12, seed=3), 1),
                                            ("er3", lambda: _GRAPHS["er3"], 1), ("twocomp", lambda: _GRAPHS["twocomp"], 1),
                                            ("noedges", lambda: _GRAPHS["noedges"], 1), ("single", lambda: _GRAPHS["single"], 1)],
                         ids=lambda x: x if isinstance(x, str) else "")
def test_quotient_and_estimate(name, maker, tau):
    g = maker()
    dg, cluster, D, st, ref = _check_decomposition(name, g, tau, 1, cd.DRIVER_AUTO)
    _say(f"[parity] quotient {name}")
    q = cd.cldiam_build_quotient(dg, cluster, D)
    rq = oracle.quotient(g, ref)
    assert q.k == rq.k
    assert np.array_equal(q.center.cpu().numpy(), rq.center)
    rrp, rcol, rw = rq.csr()
    assert q.qm == len(rcol)
    assert np.array_equal(q.row_ptr.cpu().numpy(), rrp)
    assert np.array_equal(q.col.cpu().numpy(), rcol)
    assert np.array_equal(cd.u64(q.w), rw)
    _say(f"[parity] estimate {name}")
    phi, approx = cd.cldiam_estimate_diameter(q, st.radius)
    rest = oracle.estimate(rq, ref)
    assert (phi, approx) == (rest.phi_gc, rest.phi_approx)


def test_estimate_global_memory_path():
    """Quotient graphs larger than the LDS-resident APSP size (all
    singletons of a 4000-node graph: G_C = G)."""
    g = graphgen.grid(50, 80, 100, 4)
    lib = cd.load_library()
    dg, cluster, D, st, ref = _check_decomposition("grid50x80_tau", g, 50, 1, cd.DRIVER_AUTO)
    assert st.num_clusters == g.n
    q = cd.cldiam_build_quotient(dg, cluster, D)
    phi, approx = cd.cldiam_estimate_diameter(q, st.radius)
    rest = oracle.estimate(oracle.quotient(g, ref), ref)
    assert (phi, approx) == (rest.phi_gc, rest.phi_approx)


# ------------------------------------------------------------------ SSSP --

@pytest.mark.parametrize("name,maker,bd", [("grid_small", graphgen.grid_small, 0),
                                           ("grid_small_d1", graphgen.grid_small, 1),
                                           ("road512", lambda: graphgen.road_like(512, 3), 0),
                                           ("rmat13", lambda: graphgen.rmat(13, seed=2), 0),
                                           ("rmat13_big", lambda: graphgen.rmat(13, seed=2), 2**22),
                                           ("twocomp", lambda: _GRAPHS["twocomp"], 0), ("star", lambda: _GRAPHS["star"], 0),
                                           ("noedges", lambda: _GRAPHS["noedges"], 0)],
                         ids=lambda x: x if isinstance(x, str) else "")
def test_sssp_equals_dijkstra(name, maker, bd):
    g = maker()
    src = oracle.sssp_source(g.n, 1)
    _say(f"[parity] sssp {name} src={src} bucket={bd}")
    dg = cd.cldiam_load_csr(g)
    dist, mx = cd.cldiam_sssp_delta_stepping(dg, src, bd)
    rd, rmx = oracle.sssp(g, src)
    assert np.array_equal(cd.u32(dist), rd)
    assert mx == rmx


def test_sssp_default_width_through_the_abi():
    """bucket_delta = 0 passed straight to the C entry point runs with the
    documented default (16 x floor(mean arc weight)): same distances as an
    explicit call with that width and as Dijkstra."""
    import ctypes
    import torch
    g = graphgen.road_like(200, 4)
    dg = cd.cldiam_load_csr(g)
    lib = cd.load_library()
    src = oracle.sssp_source(g.n, 1)
    _say(f"[parity] sssp default width through the ABI, src={src}")
    out = []
    for bd in (0, 16 * (dg.weight_sum // dg.m)):
        dist = torch.empty(g.n, dtype=torch.int32, device=dg.row_ptr.device)
        wsb = lib.cldiam_sssp_workspace_size(g.n, g.m)
        ws = torch.empty(wsb, dtype=torch.uint8, device=dg.row_ptr.device)
        mx = ctypes.c_uint64()
        rc = lib.cldiam_sssp_delta_stepping(g.n, g.m, ctypes.c_void_p(dg.row_ptr.data_ptr()),
                                            ctypes.c_void_p(dg.arcs.data_ptr()), src, bd,
                                            ctypes.c_void_p(dist.data_ptr()), ctypes.byref(mx),
                                            ctypes.c_void_p(ws.data_ptr()), wsb,
                                            ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
        assert rc == cd.CLDIAM_OK, lib.cldiam_last_error()
        out.append((cd.u32(dist), mx.value))
    rd, rmx = oracle.sssp(g, src)
    for d, mx in out:
        assert np.array_equal(d, rd) and mx == rmx


# ---------------------------------------------------------------- batched --

@pytest.mark.parametrize("driver", DRIVERS, ids=DRIVER_IDS)
def test_batch_equals_single_and_oracle(driver):
    graphs = [graphgen.rgg(n, i, 1) for i, n in enumerate([1000, 3000, 500, 20000, 1200, 7000])]
    graphs += [_GRAPHS["noedges"], _GRAPHS["grid_small"], _GRAPHS["single"]]
    params = [(1 + (i % 2), 100 + i, 0) for i in range(len(graphs))]
    _say(f"[parity] batch of {len(graphs)} driver={driver}")
    dgs = [cd.cldiam_load_csr(g) for g in graphs]
    clusters, Ds, stats = cd.cldiam_decompose_batch(dgs, params, driver=driver)
    for g, dg, c, D, st, (tau, seed, d0) in zip(graphs, dgs, clusters, Ds, stats, params):
        ref = oracle.decompose(g, tau, seed, delta0=d0)
        assert np.array_equal(c.cpu().numpy(), ref.cluster)
        assert np.array_equal(cd.u64(D), ref.D)
        assert (st.stages, st.levels, st.delta_end, st.num_clusters, st.radius) == \
            (ref.stages, ref.levels, ref.delta_end, ref.num_clusters, ref.radius)
        c1, D1, _ = cd.cldiam_decompose(dg, tau, seed, delta0=d0, driver=driver)
        assert np.array_equal(c1.cpu().numpy(), c.cpu().numpy())


def test_repeat_runs_are_identical():
    g = graphgen.road_like(384, 8)
    dg = cd.cldiam_load_csr(g)
    job = cd.DecomposeJob([dg], [(1, 5, 0)])
    job.run()
    c0, d0 = job.cluster[0].clone(), job.D[0].clone()
    for _ in range(3):
        job.run()
        assert bool((job.cluster[0] == c0).all()) and bool((job.D[0] == d0).all())


@pytest.mark.parametrize("name,maker,tau", [("rmat14_singletons", lambda: graphgen.rmat(14, seed=6), 200),
                                            ("grid512_singletons", lambda: graphgen.grid(512, 512, 50, 8), 3000)],
                         ids=["rmat14", "grid512"])
def test_quotient_with_many_clusters(name, maker, tau):
    """Every node its own cluster (8 tau log2 n > n): G_C is G itself, with
    far more distinct cluster pairs per workgroup than the LDS table holds."""
    g = maker()
    dg, cluster, D, st, ref = _check_decomposition(name, g, tau, 1, cd.DRIVER_AUTO)
    assert st.num_clusters == g.n
    q = cd.cldiam_build_quotient(dg, cluster, D)
    rq = oracle.quotient(g, ref)
    rrp, rcol, rw = rq.csr()
    assert q.k == rq.k == g.n
    assert np.array_equal(q.row_ptr.cpu().numpy(), rrp)
    assert np.array_equal(q.col.cpu().numpy(), rcol)
    assert np.array_equal(cd.u64(q.w), rw)


@pytest.mark.parametrize("extra", [0, -1, 1], ids=["small", "widest_packed", "wide"])
def test_quotient_with_large_distance_bounds(extra):
    """The quotient takes any D: with the largest D one below, at, or past the
    width left beside the cluster index in the packed node word, both emission
    paths give the oracle's G_C (weights w + D_u + D_v in 64 bits)."""
    import torch
    g = graphgen.rmat(12, seed=8)
    ref = oracle.decompose(g, 2, 5)
    k = int(ref.num_clusters)
    kb = max(1, int(k - 1).bit_length())
    D = ref.D.copy()
    if extra:
        D[7] = np.uint64((1 << (64 - kb)) - 1 if extra < 0 else 1 << (64 - kb))
    _say(f"[parity] quotient large D k={k} kb={kb} D[7]={int(D[7])}")
    dec = oracle.Decomposition(ref.cluster, D, ref.stages, ref.levels, ref.delta0, ref.delta_end, ref.stop,
                               ref.num_clusters, ref.singletons, ref.radius)
    dg = cd.cldiam_load_csr(g)
    cl = torch.from_numpy(ref.cluster.astype(np.int32)).cuda()
    Dt = torch.from_numpy(D.view(np.int64)).cuda()
    q = cd.cldiam_build_quotient(dg, cl, Dt)
    rq = oracle.quotient(g, dec)
    rrp, rcol, rw = rq.csr()
    assert q.k == rq.k == k
    assert np.array_equal(q.row_ptr.cpu().numpy(), rrp)
    assert np.array_equal(q.col.cpu().numpy(), rcol)
    assert np.array_equal(cd.u64(q.w), rw)


@pytest.mark.parametrize("bad", ["out_of_range", "negative", "not_a_center"])
def test_quotient_rejects_bad_labels(bad):
    """A labelling that is not a clustering (a label out of range, or naming a
    node that is not its own center) is refused with CLDIAM_EINVAL."""
    import torch
    g = graphgen.grid_small(1)
    ref = oracle.decompose(g, 1, 1)
    cl = ref.cluster.astype(np.int32).copy()
    u, v = (int(x) for x in np.nonzero(cl != np.arange(g.n))[0][:2])   # two nodes that are not centers
    if bad == "out_of_range":
        cl[u] = g.n + 5
    elif bad == "negative":
        cl[u] = -1
    else:
        cl[u] = v   # u's label names v, which is not its own center
    _say(f"[parity] quotient bad labels {bad}")
    dg = cd.cldiam_load_csr(g)
    with pytest.raises(cd.CldiamError) as e:
        cd.cldiam_build_quotient(dg, torch.from_numpy(cl).cuda(), torch.from_numpy(ref.D.view(np.int64)).cuda())
    assert e.value.status == cd.CLDIAM_EINVAL


@pytest.mark.parametrize("bad", ["column", "offsets", "last_offset"])
def test_estimate_rejects_malformed_quotient(bad):
    """A quotient CSR with a column outside [0, k) or row offsets that do not
    run from 0 to qm without decreasing is refused with CLDIAM_EINVAL."""
    import torch
    g = graphgen.grid_small(1)
    _say(f"[parity] estimate malformed {bad}")
    dg = cd.cldiam_load_csr(g)
    c, D, st = cd.cldiam_decompose(dg, 1, 1)
    q = cd.cldiam_build_quotient(dg, c, D)
    rp, col, w = q.row_ptr.clone(), q.col.clone(), q.w.clone()
    if bad == "column":
        col[3] = q.k
    elif bad == "offsets":
        rp[1], rp[2] = rp[2].clone(), rp[1].clone()
        if int(rp[1]) == int(rp[2]):
            rp[1] += 1
    else:
        rp[-1] += 1
    fake = cd.DeviceQuotient(q.k, q.qm, q.center, rp, col, w)
    with pytest.raises(cd.CldiamError) as e:
        cd.cldiam_estimate_diameter(fake, st.radius)
    assert e.value.status == cd.CLDIAM_EINVAL
    assert cd.cldiam_estimate_diameter(q, st.radius)[0] > 0   # the untouched quotient still works
