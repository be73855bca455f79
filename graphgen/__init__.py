"""Seeded synthetic input graphs: the one module that both the oracle and the
GPU path consume.

It holds input generation only (topology, weights, largest connected component,
canonical symmetric CSR).  None of the decomposition's arithmetic lives here.
The heavy generators are C (``gen.c``, built into ``libgraphgen.so`` next to
this file); tiny test graphs are built in numpy.

Workloads (the sizes and weight laws of the paper's experiments, which use
2D meshes and R-MAT graphs with random uniform weights, Section 5, Table 1):

* ``grid_small``   64x64 mesh, weights uniform in [1, 1000], seed 1
* ``road_like``    4096x4096 mesh, 5% of edges dropped, 1% random diagonal
                   shortcuts, largest component, weights uniform in [1, 10^4]
* ``rmat``         R-MAT(scale, 16), (a,b,c,d) = (.57,.19,.19,.05), symmetrised,
                   simple, largest component, weights uniform in [1, 2^20]
* ``rgg_batch``    random geometric graphs, sizes log-uniform in [10^3, 10^6],
                   average degree ~8, weight round(10^4 * length) + 1
* ``serving_mix``  Poisson request stream mixing meshes and R-MAT graphs
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "libgraphgen.so")
_lib = None


def build_lib(force: bool = True) -> str:
    """Compile gen.c into libgraphgen.so (gcc, OpenMP)."""
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-shared", "-fPIC", "-o", tmp,
                               os.path.join(_HERE, "gen.c"), "-lm"])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


class _CSR(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("m", ctypes.c_int64),
                ("row_ptr", ctypes.POINTER(ctypes.c_int32)), ("col", ctypes.POINTER(ctypes.c_int32)),
                ("w", ctypes.POINTER(ctypes.c_uint32)), ("row_ptr64", ctypes.POINTER(ctypes.c_int64))]


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build_lib()
        lib = ctypes.CDLL(_LIB_PATH)
        P = ctypes.POINTER
        lib.gg_grid.argtypes = [ctypes.c_int32, ctypes.c_int32, ctypes.c_uint32, ctypes.c_uint64,
                                ctypes.c_uint32, ctypes.c_uint32, P(_CSR)]
        lib.gg_rmat.argtypes = [ctypes.c_int32, ctypes.c_int32, ctypes.c_uint32, ctypes.c_uint32,
                                ctypes.c_uint32, ctypes.c_uint32, ctypes.c_uint64, P(_CSR)]
        lib.gg_rgg.argtypes = [ctypes.c_int32, ctypes.c_double, ctypes.c_double, ctypes.c_uint32,
                               ctypes.c_uint64, P(_CSR)]
        lib.gg_rgg_size.argtypes = [ctypes.c_uint32, ctypes.c_double, ctypes.c_double, ctypes.c_uint64]
        lib.gg_rgg_size.restype = ctypes.c_int32
        lib.gg_from_edges.argtypes = [ctypes.c_int64, ctypes.c_int64, P(ctypes.c_uint32), P(ctypes.c_uint32),
                                      P(ctypes.c_uint32), P(_CSR)]
        lib.gg_mesh64.argtypes = [ctypes.c_int32, ctypes.c_int32, ctypes.c_uint32, ctypes.c_uint64,
                                  ctypes.c_uint32, P(_CSR)]
        lib.gg_free.argtypes = [P(_CSR)]
        lib.gg_philox4x32_10.argtypes = [P(ctypes.c_uint32), P(ctypes.c_uint32), P(ctypes.c_uint32)]
        _lib = lib
    return _lib


@dataclass
class Graph:
    """Undirected weighted graph as a symmetric CSR (rows sorted by column)."""
    n: int
    row_ptr: np.ndarray  # int32[n+1] (int64 from mesh64)
    col: np.ndarray      # int32[m]
    w: np.ndarray        # uint32[m]
    name: str = ""

    @property
    def m(self) -> int:
        """Number of arcs (twice the number of undirected edges)."""
        return int(self.col.shape[0])

    def edges(self):
        """Undirected edge list (u < v) as three arrays."""
        src = np.repeat(np.arange(self.n, dtype=np.int64), np.diff(self.row_ptr.astype(np.int64)))
        keep = src < self.col
        return src[keep], self.col[keep].astype(np.int64), self.w[keep].astype(np.int64)


def _take(c: _CSR, name: str) -> Graph:
    n, m = int(c.n), int(c.m)
    rp = np.ctypeslib.as_array(c.row_ptr, shape=(n + 1,)).copy()
    col = np.ctypeslib.as_array(c.col, shape=(max(m, 1),))[:m].copy()
    w = np.ctypeslib.as_array(c.w, shape=(max(m, 1),))[:m].copy()
    _load().gg_free(ctypes.byref(c))
    return Graph(n, rp, col, w, name)


def _thr(p: float) -> int:
    return int(math.floor(p * 4294967296.0))


def philox4x32_10(ctr, key):
    """One Philox4x32-10 block (the C implementation in gen.c)."""
    c = (ctypes.c_uint32 * 4)(*[int(x) & 0xFFFFFFFF for x in ctr])
    k = (ctypes.c_uint32 * 2)(*[int(x) & 0xFFFFFFFF for x in key])
    o = (ctypes.c_uint32 * 4)()
    _load().gg_philox4x32_10(c, k, o)
    return tuple(int(x) for x in o)


def grid(rows: int, cols: int, wmax: int, seed: int, drop_p: float = 0.0, diag_p: float = 0.0) -> Graph:
    c = _CSR()
    rc = _load().gg_grid(rows, cols, wmax, seed, _thr(drop_p), _thr(diag_p), ctypes.byref(c))
    if rc != 0:
        raise RuntimeError("gg_grid failed")
    return _take(c, f"grid{rows}x{cols}")


def mesh64(rows: int, cols: int, wmax: int, seed: int, diag_p: float = 0.0) -> Graph:
    """Full rows x cols grid plus the diagonals of grid() (same draws and
    weights; equal to grid(rows, cols, wmax, seed, 0, diag_p)), written
    straight to a CSR with int64 row offsets: sizes past 2^31 arcs."""
    c = _CSR()
    rc = _load().gg_mesh64(rows, cols, wmax, seed, _thr(diag_p), ctypes.byref(c))
    if rc != 0:
        raise RuntimeError("gg_mesh64 failed")
    n, m = int(c.n), int(c.m)
    owner = _Owned(c)   # the arrays view the C buffers, which live as long as any of them

    def view(ptr, ctype, count, dtype):
        buf = (ctype * count).from_address(ctypes.addressof(ptr.contents))
        buf._owner = owner
        return np.frombuffer(buf, dtype=dtype)

    return Graph(n, view(c.row_ptr64, ctypes.c_int64, n + 1, np.int64), view(c.col, ctypes.c_int32, m, np.int32),
                 view(c.w, ctypes.c_uint32, m, np.uint32), f"mesh{rows}x{cols}")


class _Owned:
    """Frees a generator's C buffers when the last array viewing them goes."""

    def __init__(self, c: "_CSR"):
        self.c = c

    def __del__(self):
        _load().gg_free(ctypes.byref(self.c))


def mesh29(seed: int = 1) -> Graph:
    """16384 x 32768 mesh (2^29 nodes, the node count of R-MAT scale 29) with
    1% diagonals, weights uniform in [1, 10^4]: 2,158M arcs, past the reach of
    32-bit row offsets."""
    return mesh64(16384, 32768, 10**4, seed, 0.01)


def grid_small(seed: int = 1) -> Graph:
    """64x64 mesh, 4,096 nodes, 8,064 edges, weights uniform in [1, 1000]."""
    return grid(64, 64, 1000, seed)


def road_like(side: int = 4096, seed: int = 1) -> Graph:
    """side x side mesh with 5% of edges dropped and 1% diagonal shortcuts,
    largest component kept, weights uniform in [1, 10^4]."""
    g = grid(side, side, 10000, seed, drop_p=0.05, diag_p=0.01)
    g.name = f"road{side}"
    return g


def bimodal_mesh(side: int = 2048, seed: int = 1, heavy: int = 10**6) -> Graph:
    """side x side mesh whose edges weigh `heavy` with probability 0.1 and 1
    otherwise: the integer form (scaled by 10^6) of the mesh with weights 1
    w.p. 0.1 and 10^-6 otherwise used for the initial-Delta experiment of
    Section 5.  The weights come from the grid's uniform draws in [1, 10]:
    the top value becomes `heavy`, the others 1."""
    g = grid(side, side, 10, seed)
    g.w = np.where(g.w == 10, np.uint32(heavy), np.uint32(1)).astype(np.uint32)
    g.name = f"bimodal{side}"
    return g


def rmat(scale: int, seed: int = 1, edge_factor: int = 16, a=0.57, b=0.19, c=0.19, wbits: int = 20) -> Graph:
    """R-MAT graph, symmetrised and simple, largest component, weights in [1, 2^wbits]."""
    out = _CSR()
    rc = _load().gg_rmat(scale, edge_factor, _thr(a), _thr(b), _thr(c), 32 - wbits, seed, ctypes.byref(out))
    if rc != 0:
        raise RuntimeError("gg_rmat failed")
    return _take(out, f"rmat{scale}")


def rgg(n: int, graph_tag: int, seed: int, avg_deg: float = 8.0, wscale: float = 1.0e4) -> Graph:
    out = _CSR()
    rc = _load().gg_rgg(n, avg_deg, wscale, graph_tag, seed, ctypes.byref(out))
    if rc != 0:
        raise RuntimeError("gg_rgg failed")
    return _take(out, f"rgg{n}")


def rgg_sizes(count: int, seed: int, lo: float = 3.0, span: float = 3.0):
    lib = _load()
    return [int(lib.gg_rgg_size(g, lo, span, seed)) for g in range(count)]


def rgg_batch(count: int = 256, seed: int = 1, lo: float = 3.0, span: float = 3.0):
    """Batch of random geometric graphs with log-uniform sizes in [10^lo, 10^(lo+span)]."""
    return [rgg(nn, g, seed) for g, nn in enumerate(rgg_sizes(count, seed, lo, span))]


def from_edges(n: int, u, v, w) -> Graph:
    """Largest component of a simple undirected graph given as an edge list."""
    u = np.ascontiguousarray(u, dtype=np.uint32)
    v = np.ascontiguousarray(v, dtype=np.uint32)
    w = np.ascontiguousarray(w, dtype=np.uint32)
    out = _CSR()
    P = ctypes.POINTER(ctypes.c_uint32)
    rc = _load().gg_from_edges(n, len(u), u.ctypes.data_as(P), v.ctypes.data_as(P), w.ctypes.data_as(P),
                               ctypes.byref(out))
    if rc != 0:
        raise RuntimeError("gg_from_edges failed")
    return _take(out, "edges")


def csr_from_edges_np(n: int, u, v, w, name: str = "") -> Graph:
    """Canonical symmetric CSR of a simple edge list in numpy, keeping every
    node (no component filtering).  For tiny test graphs, including
    disconnected ones."""
    u = np.asarray(u, dtype=np.int64)
    v = np.asarray(v, dtype=np.int64)
    w = np.asarray(w, dtype=np.int64)
    src = np.concatenate([u, v])
    dst = np.concatenate([v, u])
    ww = np.concatenate([w, w])
    order = np.lexsort((dst, src))
    src, dst, ww = src[order], dst[order], ww[order]
    rp = np.zeros(n + 1, dtype=np.int64)
    np.add.at(rp, src + 1, 1)
    rp = np.cumsum(rp)
    return Graph(n, rp.astype(np.int32), dst.astype(np.int32), ww.astype(np.uint32), name)


def random_small(rng: np.random.Generator, n: int, p: float, wmax: int, connected: bool = False) -> Graph:
    """Erdos-Renyi-like tiny graph with integer weights in [1, wmax]; when
    ``connected`` a random spanning tree is added first."""
    pairs = set()
    us, vs = [], []
    if connected:
        perm = rng.permutation(n)
        for i in range(1, n):
            a, b = int(perm[i]), int(perm[rng.integers(0, i)])
            key = (min(a, b), max(a, b))
            pairs.add(key)
    for a in range(n):
        for b in range(a + 1, n):
            if rng.random() < p:
                pairs.add((a, b))
    pairs = sorted(pairs)
    us = [a for a, _ in pairs]
    vs = [b for _, b in pairs]
    ws = rng.integers(1, wmax + 1, size=len(pairs))
    return csr_from_edges_np(n, us, vs, ws, f"rand{n}")


@dataclass
class Request:
    rid: int
    arrival_s: float
    kind: str      # "grid" or "rmat"
    size: int      # grid side or R-MAT scale


def serving_mix(count: int = 2000, rate: float = 200.0, seed: int = 1,
                grid_lo: int = 256, grid_hi: int = 2048, rmat_lo: int = 12, rmat_hi: int = 22):
    """Poisson request stream (exponential gaps, mean 1/rate seconds): half
    meshes with side uniform in [grid_lo, grid_hi], half R-MAT with scale
    uniform in [rmat_lo, rmat_hi].  Random words come from Philox stream tag 6."""
    reqs = []
    t = 0.0
    for i in range(count):
        o = philox4x32_10((i, 0, 6, 0), (seed & 0xFFFFFFFF, seed >> 32))
        u = ((o[0] << 21) ^ (o[1] >> 11)) / 9007199254740992.0
        t += -math.log1p(-u) / rate
        if o[2] & 1:
            reqs.append(Request(i, t, "rmat", rmat_lo + o[3] % (rmat_hi - rmat_lo + 1)))
        else:
            reqs.append(Request(i, t, "grid", grid_lo + o[3] % (grid_hi - grid_lo + 1)))
    return reqs


def request_graph(req: Request) -> Graph:
    if req.kind == "grid":
        return grid(req.size, req.size, 10000, req.rid + 1)
    return rmat(req.size, seed=req.rid + 1)
