"""CPU oracle for the CL-DIAM decomposition (arXiv:1506.03265), TEST
INFRASTRUCTURE ONLY.

Only the test suite, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import it.  It shares no code with the GPU library: the heavy
parts are plain sequential C (``cldiam_oracle.c`` -> ``liboracle.so``), the
brute-force checkers are pure Python (``brute.py``).

Every function cites the passage it follows; readings of the paper are listed
in the header of ``cldiam_oracle.c``.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None

OR_OK, OR_EINVAL, OR_ENOMEM, OR_EOVERFLOW, OR_ESTAGES = 0, -1, -2, -3, -4


def build_lib(force: bool = True) -> str:
    """Compile cldiam_oracle.c with gcc (no OpenMP: the oracle is sequential)."""
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-shared", "-fPIC", "-o", tmp,
                               os.path.join(_HERE, "cldiam_oracle.c"), "-lm"])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


class _Stats(ctypes.Structure):
    _fields_ = [("stages", ctypes.c_int32), ("levels", ctypes.c_int32), ("delta0", ctypes.c_uint32),
                ("delta_end", ctypes.c_uint32), ("stop", ctypes.c_int32), ("num_clusters", ctypes.c_int32),
                ("singletons", ctypes.c_int32), ("pad", ctypes.c_int32), ("radius", ctypes.c_uint64),
                ("sum_uncovered", ctypes.c_uint64), ("sum_acting", ctypes.c_uint64),
                ("sum_arcs", ctypes.c_uint64), ("sum_covered", ctypes.c_uint64)]


class _StepStats(ctypes.Structure):
    _fields_ = [("rounds", ctypes.c_uint64), ("messages", ctypes.c_uint64), ("updates", ctypes.c_uint64)]


class _Log(ctypes.Structure):
    _fields_ = [("uncovered", ctypes.POINTER(ctypes.c_int32)), ("centers", ctypes.POINTER(ctypes.c_int32)),
                ("covered", ctypes.POINTER(ctypes.c_int32)), ("delta", ctypes.POINTER(ctypes.c_uint32)),
                ("cap", ctypes.c_int32)]


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build_lib()
        lib = ctypes.CDLL(_LIB_PATH)
        P = ctypes.POINTER
        i32p, u32p, u64p, i64p = P(ctypes.c_int32), P(ctypes.c_uint32), P(ctypes.c_uint64), P(ctypes.c_int64)
        lib.or_philox.argtypes = [u32p, u32p, u32p]
        lib.or_default_delta.argtypes = [ctypes.c_int64, u32p]
        lib.or_default_delta.restype = ctypes.c_uint32
        lib.or_decompose.argtypes = [ctypes.c_int32, i64p, i32p, u32p, ctypes.c_uint32, ctypes.c_uint32,
                                     ctypes.c_uint64, i32p, u64p, P(_Stats), P(_Log)]
        lib.or_decompose_steps.argtypes = [ctypes.c_int32, i64p, i32p, u32p, ctypes.c_uint32, ctypes.c_uint32,
                                           ctypes.c_uint64, ctypes.c_uint32, i32p, u64p, P(_Stats), P(_StepStats),
                                           P(_Log)]
        lib.or_decompose_cluster2.argtypes = [ctypes.c_int32, i64p, i32p, u32p, ctypes.c_uint32, ctypes.c_uint32,
                                              ctypes.c_uint64, i32p, u64p, P(_Stats), u64p, P(_Log)]
        lib.or_quotient.argtypes = [ctypes.c_int32, i64p, i32p, u32p, i32p, u64p, i32p, P(i32p),
                                    P(ctypes.c_int64), P(i32p), P(i32p), P(u64p), P(ctypes.c_int64)]
        lib.or_free.argtypes = [ctypes.c_void_p]
        lib.or_diameter_edges.argtypes = [ctypes.c_int32, ctypes.c_int64, i32p, i32p, u64p, u64p]
        lib.or_sssp.argtypes = [ctypes.c_int32, i64p, i32p, u32p, ctypes.c_int32, u32p, u64p]
        _lib = lib
    return _lib


def _p(a, t):
    return a.ctypes.data_as(ctypes.POINTER(t))


def philox4x32_10(ctr, key):
    c = (ctypes.c_uint32 * 4)(*[int(x) & 0xFFFFFFFF for x in ctr])
    k = (ctypes.c_uint32 * 2)(*[int(x) & 0xFFFFFFFF for x in key])
    o = (ctypes.c_uint32 * 4)()
    _load().or_philox(c, k, o)
    return tuple(int(x) for x in o)


class OracleError(RuntimeError):
    def __init__(self, code, what):
        super().__init__(f"{what} failed with code {code}")
        self.code = code


@dataclass
class Decomposition:
    cluster: np.ndarray          # int32[n]: center node id of each node's cluster
    D: np.ndarray                # uint64[n]: upper bound on dist(center, node)
    stages: int
    levels: int
    delta0: int
    delta_end: int
    stop: int
    num_clusters: int
    singletons: int
    radius: int
    stage_uncovered: list = field(default_factory=list)
    stage_centers: list = field(default_factory=list)
    stage_covered: list = field(default_factory=list)
    stage_delta: list = field(default_factory=list)
    work: dict = field(default_factory=dict)


def _csr_args(g):
    """Row offsets as int64 (the oracle's offsets are 64-bit: graphs past 2^31
    arcs), columns int32, weights uint32."""
    rp = np.ascontiguousarray(g.row_ptr, dtype=np.int64)
    col = np.ascontiguousarray(g.col, dtype=np.int32)
    w = np.ascontiguousarray(g.w, dtype=np.uint32)
    return rp, col, w


def default_delta(g) -> int:
    """Initial Delta = floor(average arc weight), at least 1 (Section 5, initial
    guess equal to the average edge weight)."""
    w = np.ascontiguousarray(g.w, dtype=np.uint32)
    return int(_load().or_default_delta(len(w), _p(w, ctypes.c_uint32)))


def decompose(g, tau: int, seed: int, delta0: int = 0, log_cap: int = 256) -> Decomposition:
    """CLUSTER(G, tau) of Algorithm 1 (Section 3) with the readings stated in
    cldiam_oracle.c.  delta0 = 0 selects the average arc weight."""
    rp, col, w = _csr_args(g)
    n = g.n
    cluster = np.empty(n, dtype=np.int32)
    D = np.empty(n, dtype=np.uint64)
    st = _Stats()
    lu = np.zeros(log_cap, np.int32)
    lc = np.zeros(log_cap, np.int32)
    lv = np.zeros(log_cap, np.int32)
    ld = np.zeros(log_cap, np.uint32)
    lg = _Log(_p(lu, ctypes.c_int32), _p(lc, ctypes.c_int32), _p(lv, ctypes.c_int32), _p(ld, ctypes.c_uint32),
              log_cap)
    rc = _load().or_decompose(n, _p(rp, ctypes.c_int64), _p(col, ctypes.c_int32), _p(w, ctypes.c_uint32),
                              tau, delta0, seed, _p(cluster, ctypes.c_int32), _p(D, ctypes.c_uint64),
                              ctypes.byref(st), ctypes.byref(lg))
    if rc != OR_OK:
        raise OracleError(rc, "or_decompose")
    s = min(st.stages, log_cap)
    work = dict(sum_uncovered=int(st.sum_uncovered), sum_acting=int(st.sum_acting),
                sum_arcs=int(st.sum_arcs), sum_covered=int(st.sum_covered))
    return Decomposition(cluster, D, st.stages, st.levels, st.delta0, st.delta_end, st.stop, st.num_clusters,
                         st.singletons, int(st.radius), lu[:s].tolist(), lc[:s].tolist(), lv[:s].tolist(),
                         ld[:s].tolist(), work)


def decompose_steps(g, tau: int, seed: int, delta0: int = 0, step_cap: int = 0,
                    log_cap: int = 256) -> Decomposition:
    """CLUSTER(G, tau) with the literal PartialGrowth of Algorithm 1:
    synchronous Delta-growing steps, the strict-distance tie rule, the
    per-step half-coverage stop, Delta doubled one step at a time, and an
    optional cap on the steps of one PartialGrowth call (step_cap, 0 = none).
    work also holds rounds, messages and updates (see cldiam_oracle.c)."""
    rp, col, w = _csr_args(g)
    n = g.n
    cluster = np.empty(n, dtype=np.int32)
    D = np.empty(n, dtype=np.uint64)
    st = _Stats()
    ss = _StepStats()
    lu = np.zeros(log_cap, np.int32)
    lc = np.zeros(log_cap, np.int32)
    lv = np.zeros(log_cap, np.int32)
    ld = np.zeros(log_cap, np.uint32)
    lg = _Log(_p(lu, ctypes.c_int32), _p(lc, ctypes.c_int32), _p(lv, ctypes.c_int32), _p(ld, ctypes.c_uint32),
              log_cap)
    rc = _load().or_decompose_steps(n, _p(rp, ctypes.c_int64), _p(col, ctypes.c_int32), _p(w, ctypes.c_uint32),
                                    tau, delta0, seed, step_cap, _p(cluster, ctypes.c_int32),
                                    _p(D, ctypes.c_uint64), ctypes.byref(st), ctypes.byref(ss), ctypes.byref(lg))
    if rc != OR_OK:
        raise OracleError(rc, "or_decompose_steps")
    s = min(st.stages, log_cap)
    work = dict(sum_uncovered=int(st.sum_uncovered), sum_acting=int(st.sum_acting),
                sum_arcs=int(st.sum_arcs), sum_covered=int(st.sum_covered), rounds=int(ss.rounds),
                messages=int(ss.messages), updates=int(ss.updates))
    return Decomposition(cluster, D, st.stages, st.levels, st.delta0, st.delta_end, st.stop, st.num_clusters,
                         st.singletons, int(st.radius), lu[:s].tolist(), lc[:s].tolist(), lv[:s].tolist(),
                         ld[:s].tolist(), work)


def decompose_cluster2(g, tau: int, seed: int, delta0: int = 0, log_cap: int = 256) -> Decomposition:
    """CLUSTER2(G, tau) of Algorithm 2 (Section 4) with the readings stated in
    cldiam_oracle.c.  work['radius1'] is R_CL, the radius of the preliminary
    CLUSTER(G, tau) run; delta_end is 2 R_CL."""
    rp, col, w = _csr_args(g)
    n = g.n
    cluster = np.empty(n, dtype=np.int32)
    D = np.empty(n, dtype=np.uint64)
    st = _Stats()
    r1 = ctypes.c_uint64()
    lu = np.zeros(log_cap, np.int32)
    lc = np.zeros(log_cap, np.int32)
    lv = np.zeros(log_cap, np.int32)
    ld = np.zeros(log_cap, np.uint32)
    lg = _Log(_p(lu, ctypes.c_int32), _p(lc, ctypes.c_int32), _p(lv, ctypes.c_int32), _p(ld, ctypes.c_uint32),
              log_cap)
    rc = _load().or_decompose_cluster2(n, _p(rp, ctypes.c_int64), _p(col, ctypes.c_int32),
                                       _p(w, ctypes.c_uint32), tau, delta0, seed, _p(cluster, ctypes.c_int32),
                                       _p(D, ctypes.c_uint64), ctypes.byref(st), ctypes.byref(r1),
                                       ctypes.byref(lg))
    if rc != OR_OK:
        raise OracleError(rc, "or_decompose_cluster2")
    s = min(st.stages, log_cap)
    work = dict(sum_uncovered=int(st.sum_uncovered), sum_covered=int(st.sum_covered), radius1=int(r1.value))
    return Decomposition(cluster, D, st.stages, st.levels, st.delta0, st.delta_end, st.stop, st.num_clusters,
                         st.singletons, int(st.radius), lu[:s].tolist(), lc[:s].tolist(), lv[:s].tolist(),
                         ld[:s].tolist(), work)


@dataclass
class Quotient:
    k: int
    center: np.ndarray   # int32[k]
    ea: np.ndarray       # int32[ne], a < b, sorted by (a, b)
    eb: np.ndarray       # int32[ne]
    ew: np.ndarray       # uint64[ne]
    pairs: int           # inter-cluster undirected edges of G

    def csr(self):
        """Symmetric CSR (row_ptr int64[k+1], col int32, w uint64), rows sorted by column."""
        src = np.concatenate([self.ea, self.eb]).astype(np.int64)
        dst = np.concatenate([self.eb, self.ea]).astype(np.int64)
        ww = np.concatenate([self.ew, self.ew])
        order = np.lexsort((dst, src))
        rp = np.zeros(self.k + 1, dtype=np.int64)
        np.add.at(rp, src + 1, 1)
        return np.cumsum(rp), dst[order].astype(np.int32), ww[order].astype(np.uint64)


def quotient(g, dec: Decomposition) -> Quotient:
    """Weighted quotient graph G_C of Section 4 (minimum over parallel edges)."""
    rp, col, w = _csr_args(g)
    lib = _load()
    k = ctypes.c_int32()
    ne = ctypes.c_int64()
    P = ctypes.c_int64()
    cen, ea, eb = ctypes.POINTER(ctypes.c_int32)(), ctypes.POINTER(ctypes.c_int32)(), ctypes.POINTER(ctypes.c_int32)()
    ew = ctypes.POINTER(ctypes.c_uint64)()
    cl = np.ascontiguousarray(dec.cluster, dtype=np.int32)
    D = np.ascontiguousarray(dec.D, dtype=np.uint64)
    rc = lib.or_quotient(g.n, _p(rp, ctypes.c_int64), _p(col, ctypes.c_int32), _p(w, ctypes.c_uint32),
                         _p(cl, ctypes.c_int32), _p(D, ctypes.c_uint64), ctypes.byref(k), ctypes.byref(cen),
                         ctypes.byref(ne), ctypes.byref(ea), ctypes.byref(eb), ctypes.byref(ew), ctypes.byref(P))
    if rc != OR_OK:
        raise OracleError(rc, "or_quotient")
    kk, nn = k.value, ne.value
    out = Quotient(kk,
                   np.ctypeslib.as_array(cen, shape=(max(kk, 1),))[:kk].copy(),
                   np.ctypeslib.as_array(ea, shape=(max(nn, 1),))[:nn].copy(),
                   np.ctypeslib.as_array(eb, shape=(max(nn, 1),))[:nn].copy(),
                   np.ctypeslib.as_array(ew, shape=(max(nn, 1),))[:nn].copy(),
                   P.value)
    for p in (cen, ea, eb, ew):
        lib.or_free(ctypes.cast(p, ctypes.c_void_p))
    return out


def diameter_edges(k: int, ea, eb, ew) -> int:
    """Exact weighted diameter (max finite pairwise distance) of an edge list."""
    ea = np.ascontiguousarray(ea, dtype=np.int32)
    eb = np.ascontiguousarray(eb, dtype=np.int32)
    ew = np.ascontiguousarray(ew, dtype=np.uint64)
    phi = ctypes.c_uint64()
    rc = _load().or_diameter_edges(k, len(ea), _p(ea, ctypes.c_int32), _p(eb, ctypes.c_int32),
                                   _p(ew, ctypes.c_uint64), ctypes.byref(phi))
    if rc != OR_OK:
        raise OracleError(rc, "or_diameter_edges")
    return int(phi.value)


@dataclass
class Estimate:
    phi_gc: int
    phi_approx: int


def estimate(q: Quotient, dec: Decomposition) -> Estimate:
    """Phi_approx = Phi(G_C) + 2 max D (Section 4)."""
    phi = diameter_edges(q.k, q.ea, q.eb, q.ew)
    return Estimate(phi, phi + 2 * int(dec.radius))


def sssp(g, src: int):
    """Exact single-source distances (u32, 0xFFFFFFFF = unreachable) and the
    largest finite one; twice it is the SSSP 2-approximation of the diameter
    (Section 5)."""
    rp, col, w = _csr_args(g)
    dist = np.empty(g.n, dtype=np.uint32)
    mx = ctypes.c_uint64()
    rc = _load().or_sssp(g.n, _p(rp, ctypes.c_int64), _p(col, ctypes.c_int32), _p(w, ctypes.c_uint32), src,
                         _p(dist, ctypes.c_uint32), ctypes.byref(mx))
    if rc != OR_OK:
        raise OracleError(rc, "or_sssp")
    return dist, int(mx.value)


def sssp_source(n: int, seed: int) -> int:
    """Source node of the SSSP baseline: word 0 of Philox(counter (0,0,7,0),
    key seed) modulo n."""
    return philox4x32_10((0, 0, 7, 0), (seed & 0xFFFFFFFF, seed >> 32))[0] % n


def algorithmic_bytes(g, dec: Decomposition, q: Quotient | None = None) -> dict:
    """Bytes a work-efficient implementation must move, from this sequential
    run's work counts: per stage 8 B per uncovered node, 16 B per node whose
    row is read (row offsets + key), 16 B per arc read (packed arc + target
    key), 20 B per newly covered node (key, cluster, D); the quotient adds
    4(n+1) + 8m + 12n + 6m + 32 P + 24 E_C."""
    wk = dec.work
    decomp = 8 * wk["sum_uncovered"] + 16 * wk["sum_acting"] + 16 * wk["sum_arcs"] + 20 * wk["sum_covered"]
    out = {"decompose": decomp}
    if q is not None:
        n, m = g.n, g.m
        out["quotient"] = 4 * (n + 1) + 8 * m + 12 * n + 6 * m + 32 * q.pairs + 24 * len(q.ea)
    return out
