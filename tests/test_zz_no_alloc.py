"""The estimate entry point that allocates nothing
(cldiam_estimate_diameter_noalloc, scratch in a static device array) against
the workspace entry point (cldiam_estimate_diameter) through the C ABI, on
consecutive calls whose inputs shrink, so that the second call runs on the
static array's leftovers of the first.  Quotient-shaped inputs are random
connected symmetric graphs with 64-bit weights; the smaller ones are also
checked against the oracle's all-pairs Dijkstra."""
import ctypes
import sys

import numpy as np
import pytest

import oracle
import paper_1506_03265_amd as cd

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, file=sys.stderr, flush=True)


def _quotient_like(k, extra, seed):
    """Connected symmetric CSR on k nodes (random spanning tree plus `extra`
    random edges, no self loops or parallel edges), weights in [1, 2^40]."""
    rng = np.random.default_rng(seed)
    perm = rng.permutation(k)
    a = [int(perm[i]) for i in range(1, k)]
    b = [int(perm[int(rng.integers(0, i))]) for i in range(1, k)]
    pairs = {(min(x, y), max(x, y)) for x, y in zip(a, b)}
    while len(pairs) < k - 1 + extra:
        x, y = (int(v) for v in rng.integers(0, k, 2))
        if x != y:
            pairs.add((min(x, y), max(x, y)))
    ea = np.array([p[0] for p in sorted(pairs)], dtype=np.int32)
    eb = np.array([p[1] for p in sorted(pairs)], dtype=np.int32)
    ew = rng.integers(1, 2**40, len(ea), dtype=np.uint64)
    src = np.concatenate([ea, eb]).astype(np.int64)
    dst = np.concatenate([eb, ea]).astype(np.int64)
    ww = np.concatenate([ew, ew])
    order = np.lexsort((dst, src))
    rp = np.zeros(k + 1, dtype=np.int64)
    np.add.at(rp, src + 1, 1)
    return np.cumsum(rp), dst[order].astype(np.int32), ww[order], (ea, eb, ew)


def _device(rp, col, w):
    import torch
    dev = torch.device("cuda", 0)
    return (torch.from_numpy(rp).to(dev), torch.from_numpy(col).to(dev),
            torch.from_numpy(w.view(np.int64)).to(dev))


def _both(lib, k, rp, col, w, radius):
    import torch
    qm = int(col.numel())
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    wsb = lib.cldiam_estimate_workspace_size(k, qm)
    ws = torch.empty(wsb, dtype=torch.uint8, device=rp.device)
    p1, a1 = ctypes.c_uint64(), ctypes.c_uint64()
    rc = lib.cldiam_estimate_diameter(k, qm, ctypes.c_void_p(rp.data_ptr()), ctypes.c_void_p(col.data_ptr()),
                                      ctypes.c_void_p(w.data_ptr()), radius, ctypes.byref(p1), ctypes.byref(a1),
                                      ctypes.c_void_p(ws.data_ptr()), wsb, stream)
    assert rc == cd.CLDIAM_OK, lib.cldiam_last_error()
    p2, a2 = ctypes.c_uint64(), ctypes.c_uint64()
    rc = lib.cldiam_estimate_diameter_noalloc(k, qm, ctypes.c_void_p(rp.data_ptr()),
                                              ctypes.c_void_p(col.data_ptr()), ctypes.c_void_p(w.data_ptr()),
                                              radius, ctypes.byref(p2), ctypes.byref(a2), stream)
    assert rc == cd.CLDIAM_OK, lib.cldiam_last_error()
    return (p1.value, a1.value), (p2.value, a2.value)


@pytest.fixture(scope="module")
def lib():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return cd.load_library()


def test_noalloc_equals_workspace_entry_on_shrinking_inputs(lib):
    # first call: 4500 quotient nodes (per-workgroup slices in the static
    # array); second: 900 nodes (LDS path, control words reused); third:
    # 3300 nodes (slices again, over the first call's leftovers)
    cases = [(4500, 3000, 11, 12345), (900, 700, 12, 7), (3300, 500, 13, 0)]
    for k, extra, seed, radius in cases:
        rp, col, w, edges = _quotient_like(k, extra, seed)
        _say(f"[noalloc] k={k} arcs={len(col)} seed={seed}")
        ref, got = _both(lib, k, *_device(rp, col, w), radius)
        assert got == ref, (k, got, ref)
        if k <= 1000:
            phi = oracle.diameter_edges(k, *edges)
            assert got == (phi, phi + 2 * radius)


def test_noalloc_on_a_decomposition_quotient(lib):
    """A real quotient (road-like mesh, many clusters) twice, then a smaller one."""
    import graphgen
    for side, tau in ((256, 1), (96, 1)):
        g = graphgen.road_like(side, 5)
        dg = cd.cldiam_load_csr(g)
        cluster, D, st = cd.cldiam_decompose(dg, tau, 3)
        q = cd.cldiam_build_quotient(dg, cluster, D)
        _say(f"[noalloc] road{side} k={q.k} qm={q.qm}")
        ref, got = _both(lib, q.k, q.row_ptr, q.col, q.w, st.radius)
        assert got == ref


def test_noalloc_rejects_k_above_its_maximum(lib):
    rp, col, w, _ = _quotient_like(50, 10, 3)
    drp, dcol, dw = _device(rp, col, w)
    phi, approx = ctypes.c_uint64(), ctypes.c_uint64()
    rc = lib.cldiam_estimate_diameter_noalloc(32769, int(dcol.numel()), ctypes.c_void_p(drp.data_ptr()),
                                              ctypes.c_void_p(dcol.data_ptr()), ctypes.c_void_p(dw.data_ptr()), 0,
                                              ctypes.byref(phi), ctypes.byref(approx), None)
    assert rc == cd.CLDIAM_EINVAL
    assert b"maximum" in lib.cldiam_last_error()
