"""Python binding of libcldiam.so, the gfx950 implementation of the CL-DIAM
decomposition, quotient graph and diameter estimate (arXiv:1506.03265).

The functions have the names of the C entry points in include/cldiam.h and
only marshal arguments: PyTorch provides device memory and the stream, every
step of the computation runs in the library's HIP kernels.  Importing works
anywhere; calling needs the built library (``paper_1506_03265_amd/build.py``)
and a GPU, otherwise a RuntimeError is raised.  There is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libcldiam.so")

CLDIAM_OK = 0
CLDIAM_EINVAL = -1
CLDIAM_ENOMEM = -2
CLDIAM_EOVERFLOW = -3
CLDIAM_EHIP = -4
CLDIAM_ESTAGES = -5
CLDIAM_ETIMEOUT = -6
CLDIAM_NOALLOC_MAX_K = 32768   # largest quotient of cldiam_estimate_diameter_noalloc
PULL_AUTO, PULL_NEVER, PULL_ALWAYS = 0, 1, 2
STAGE_LOG = 64

DRIVER_AUTO, DRIVER_HOST, DRIVER_PERSISTENT = 0, 1, 2
VARIANT_FIXPOINT, VARIANT_STEPS, VARIANT_CLUSTER2 = 0, 1, 2

EXPORTS = [
    "cldiam_strerror", "cldiam_last_error", "cldiam_version", "cldiam_pinned_host_bytes",
    "cldiam_load_csr_workspace_size", "cldiam_load_csr",
    "cldiam_decompose_workspace_size", "cldiam_decompose_batch", "cldiam_decompose",
    "cldiam_quotient_workspace_size", "cldiam_build_quotient",
    "cldiam_estimate_workspace_size", "cldiam_estimate_diameter", "cldiam_estimate_diameter_noalloc",
    "cldiam_sssp_workspace_size", "cldiam_sssp_delta_stepping",
    "cldiam_server_workspace_size", "cldiam_server_create", "cldiam_server_destroy", "cldiam_server_submit",
    "cldiam_server_step", "cldiam_server_poll",
]


class CldiamError(RuntimeError):
    def __init__(self, status: int, what: str, detail: str):
        super().__init__(f"{what}: status {status} ({detail})")
        self.status = status


class _Csr(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("pad", ctypes.c_int32), ("m", ctypes.c_int64),
                ("d_row_ptr", ctypes.c_void_p), ("d_col", ctypes.c_void_p), ("d_w", ctypes.c_void_p)]


class _Params(ctypes.Structure):
    _fields_ = [("tau", ctypes.c_uint32), ("delta0", ctypes.c_uint32), ("seed", ctypes.c_uint64),
                ("variant", ctypes.c_uint32), ("step_cap", ctypes.c_uint32)]


class _Graph(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("pad", ctypes.c_int32), ("m", ctypes.c_int64),
                ("d_row_ptr", ctypes.c_void_p), ("d_arcs", ctypes.c_void_p), ("weight_sum", ctypes.c_uint64),
                ("params", _Params), ("d_cluster", ctypes.c_void_p), ("d_D", ctypes.c_void_p)]


class _Tuning(ctypes.Structure):
    _fields_ = [("local_rounds", ctypes.c_int32), ("grid_blocks", ctypes.c_int32), ("bucket_width", ctypes.c_float),
                ("row_bucket_shift", ctypes.c_int32), ("chunk_factor", ctypes.c_int32),
                ("wave_row_min", ctypes.c_int32), ("group_row_min", ctypes.c_int32), ("local_queue", ctypes.c_int32),
                ("local_cutoff", ctypes.c_int32), ("pull_mode", ctypes.c_int32)]


class _Stats(ctypes.Structure):
    _fields_ = [("stages", ctypes.c_int32), ("levels", ctypes.c_int32), ("delta0", ctypes.c_uint32),
                ("delta_end", ctypes.c_uint32), ("stop", ctypes.c_int32), ("num_clusters", ctypes.c_int32),
                ("singletons", ctypes.c_int32), ("sweeps", ctypes.c_int32), ("radius", ctypes.c_uint64),
                ("arcs_scanned", ctypes.c_uint64), ("status", ctypes.c_int32), ("grid_blocks", ctypes.c_int32),
                ("kernel_ms", ctypes.c_float), ("iterations", ctypes.c_int32), ("rounds", ctypes.c_uint64),
                ("messages", ctypes.c_uint64), ("updates", ctypes.c_uint64), ("radius1", ctypes.c_uint64),
                ("stage_uncovered", ctypes.c_int32 * STAGE_LOG), ("stage_centers", ctypes.c_int32 * STAGE_LOG),
                ("stage_covered", ctypes.c_int32 * STAGE_LOG), ("stage_delta", ctypes.c_uint32 * STAGE_LOG)]


_lib = None


def load_library(path: str = LIB_PATH):
    """Loads libcldiam.so and declares every exported signature."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is not built; run paper_1506_03265_amd/build.py (hipcc, gfx950)")
    lib = ctypes.CDLL(path)
    V, I32, I64, U32, U64, SZ = (ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_uint32,
                                 ctypes.c_uint64, ctypes.c_size_t)
    P = ctypes.POINTER
    lib.cldiam_strerror.argtypes, lib.cldiam_strerror.restype = [ctypes.c_int], ctypes.c_char_p
    lib.cldiam_last_error.argtypes, lib.cldiam_last_error.restype = [], ctypes.c_char_p
    lib.cldiam_version.argtypes, lib.cldiam_version.restype = [], ctypes.c_char_p
    lib.cldiam_pinned_host_bytes.argtypes, lib.cldiam_pinned_host_bytes.restype = [], I64
    lib.cldiam_load_csr_workspace_size.argtypes, lib.cldiam_load_csr_workspace_size.restype = [I32, I64], SZ
    lib.cldiam_load_csr.argtypes = [P(_Csr), V, P(U64), V, SZ, V]
    lib.cldiam_decompose_workspace_size.argtypes, lib.cldiam_decompose_workspace_size.restype = [I64, I32], SZ
    lib.cldiam_decompose_batch.argtypes = [I32, P(_Graph), P(_Stats), ctypes.c_int, P(_Tuning), V, SZ, V]
    lib.cldiam_decompose.argtypes = [P(_Graph), P(_Stats), ctypes.c_int, P(_Tuning), V, SZ, V]
    lib.cldiam_quotient_workspace_size.argtypes, lib.cldiam_quotient_workspace_size.restype = [I32, I64], SZ
    lib.cldiam_build_quotient.argtypes = [I32, I64, V, V, V, V, V, V, V, V, P(I32), P(I64), V, SZ, V]
    lib.cldiam_estimate_workspace_size.argtypes, lib.cldiam_estimate_workspace_size.restype = [I32, I64], SZ
    lib.cldiam_estimate_diameter.argtypes = [I32, I64, V, V, V, U64, P(U64), P(U64), V, SZ, V]
    lib.cldiam_estimate_diameter_noalloc.argtypes = [I32, I64, V, V, V, U64, P(U64), P(U64), V]
    lib.cldiam_sssp_workspace_size.argtypes, lib.cldiam_sssp_workspace_size.restype = [I32, I64], SZ
    lib.cldiam_sssp_delta_stepping.argtypes = [I32, I64, V, V, I32, U32, V, P(U64), V, SZ, V]
    lib.cldiam_server_workspace_size.argtypes, lib.cldiam_server_workspace_size.restype = [I64, I32], SZ
    lib.cldiam_server_create.argtypes = [P(V), I64, I32, P(_Tuning), V, SZ, V]
    lib.cldiam_server_destroy.argtypes, lib.cldiam_server_destroy.restype = [V], None
    lib.cldiam_server_submit.argtypes = [V, P(_Graph), U64]
    lib.cldiam_server_step.argtypes = [V, I32, P(I32), P(I32)]
    lib.cldiam_server_poll.argtypes = [V, P(U64), P(_Stats), I32, P(I32)]
    for name in ("cldiam_load_csr", "cldiam_decompose_batch", "cldiam_decompose", "cldiam_build_quotient",
                 "cldiam_estimate_diameter", "cldiam_estimate_diameter_noalloc", "cldiam_sssp_delta_stepping",
                 "cldiam_server_create",
                 "cldiam_server_submit", "cldiam_server_step", "cldiam_server_poll"):
        getattr(lib, name).restype = ctypes.c_int
    _lib = lib
    return lib


def _check(rc: int, what: str):
    if rc != CLDIAM_OK:
        lib = load_library()
        detail = lib.cldiam_last_error().decode(errors="replace")
        raise CldiamError(rc, what, detail)


def _torch():
    import torch
    if not torch.cuda.is_available():
        raise RuntimeError("libcldiam needs a GPU (torch.cuda.is_available() is False)")
    return torch


def _stream(stream):
    torch = _torch()
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _ws(nbytes: int, device):
    torch = _torch()
    return torch.empty(max(int(nbytes), 256), dtype=torch.uint8, device=device)


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None and t.numel() > 0 else ctypes.c_void_p(0)


# ------------------------------------------------------------------ ingest --

@dataclass
class DeviceGraph:
    """Graph resident in device memory: CSR plus weight-sorted packed arcs."""
    n: int
    m: int
    row_ptr: object      # torch int64 [n+1]
    col: object          # torch int32 [m]
    w: object            # torch int32 [m] (bit pattern of uint32)
    arcs: object         # torch int64 [m] (bit pattern of (w << 32) | col)
    weight_sum: int
    name: str = ""


def to_device(g, device="cuda"):
    """Copies a host CSR (graphgen.Graph) to device tensors (no validation)."""
    torch = _torch()
    rp = torch.from_numpy(np.ascontiguousarray(g.row_ptr, dtype=np.int64)).to(device)
    col = torch.from_numpy(np.ascontiguousarray(g.col, dtype=np.int32)).to(device)
    w = torch.from_numpy(np.ascontiguousarray(g.w, dtype=np.uint32).view(np.int32)).to(device)
    return rp, col, w


def cldiam_load_csr(g, device="cuda", stream=None) -> DeviceGraph:
    """Uploads a host CSR and runs cldiam_load_csr (validation + weight-sorted
    packed arcs)."""
    torch = _torch()
    lib = load_library()
    rp, col, w = to_device(g, device)
    n, m = int(g.n), int(len(g.col))
    arcs = torch.empty(max(m, 1), dtype=torch.int64, device=device)
    csr = _Csr(n, 0, m, rp.data_ptr(), _ptr(col).value, _ptr(w).value)
    wsb = lib.cldiam_load_csr_workspace_size(n, m)
    ws = _ws(wsb, device)
    wsum = ctypes.c_uint64()
    _check(lib.cldiam_load_csr(ctypes.byref(csr), _ptr(arcs), ctypes.byref(wsum), _ptr(ws), wsb, _stream(stream)),
           "cldiam_load_csr")
    return DeviceGraph(n, m, rp, col, w, arcs, int(wsum.value), getattr(g, "name", ""))


def cldiam_load_csr_device(n, m, rp, col, w, stream=None) -> DeviceGraph:
    """cldiam_load_csr on tensors already on the device (row offsets int64,
    columns int32, weights int32 holding uint32 bit patterns)."""
    torch = _torch()
    lib = load_library()
    if rp.dtype != torch.int64 or col.dtype != torch.int32 or w.dtype != torch.int32:
        raise TypeError("cldiam_load_csr_device: row offsets int64, columns and weights int32")
    arcs = torch.empty(max(m, 1), dtype=torch.int64, device=rp.device)
    csr = _Csr(n, 0, m, rp.data_ptr(), _ptr(col).value, _ptr(w).value)
    wsb = lib.cldiam_load_csr_workspace_size(n, m)
    ws = _ws(wsb, rp.device)
    wsum = ctypes.c_uint64()
    _check(lib.cldiam_load_csr(ctypes.byref(csr), _ptr(arcs), ctypes.byref(wsum), _ptr(ws), wsb, _stream(stream)),
           "cldiam_load_csr")
    return DeviceGraph(n, m, rp, col, w, arcs, int(wsum.value))


# ------------------------------------------------------------ decompose --

@dataclass
class Stats:
    stages: int
    levels: int
    delta0: int
    delta_end: int
    stop: int
    num_clusters: int
    singletons: int
    sweeps: int
    radius: int
    arcs_scanned: int
    status: int
    grid_blocks: int
    kernel_ms: float
    iterations: int
    rounds: int = 0
    messages: int = 0
    updates: int = 0
    radius1: int = 0
    stage_uncovered: list = field(default_factory=list)
    stage_centers: list = field(default_factory=list)
    stage_covered: list = field(default_factory=list)
    stage_delta: list = field(default_factory=list)


def _stats(s: _Stats) -> Stats:
    k = min(s.stages, STAGE_LOG)
    return Stats(s.stages, s.levels, s.delta0, s.delta_end, s.stop, s.num_clusters, s.singletons, s.sweeps,
                 int(s.radius), int(s.arcs_scanned), s.status, s.grid_blocks, float(s.kernel_ms), s.iterations,
                 int(s.rounds), int(s.messages), int(s.updates), int(s.radius1), list(s.stage_uncovered[:k]),
                 list(s.stage_centers[:k]), list(s.stage_covered[:k]), list(s.stage_delta[:k]))


class DecomposeJob:
    """Reusable decomposition launch: outputs, workspace and descriptors are
    allocated once so that repeated runs time only the device work."""

    def __init__(self, graphs, params, driver=DRIVER_AUTO, local_rounds=-1, grid_blocks=0, bucket_width=0.0,
                 row_bucket_shift=0, chunk_factor=0, wave_row_min=0, group_row_min=0, local_queue=0, local_cutoff=0,
                 pull_mode=0):
        torch = _torch()
        self.lib = load_library()
        self.graphs = list(graphs)
        dev = self.graphs[0].row_ptr.device
        self.cluster = [torch.empty(g.n, dtype=torch.int32, device=dev) for g in self.graphs]
        self.D = [torch.empty(g.n, dtype=torch.int64, device=dev) for g in self.graphs]
        G = len(self.graphs)
        self.desc = (_Graph * G)()
        for i, (g, p) in enumerate(zip(self.graphs, params)):
            tau, seed, delta0 = p[:3]
            variant, step_cap = (tuple(p[3:5]) + (0, 0))[:2]
            self.desc[i] = _Graph(g.n, 0, g.m, g.row_ptr.data_ptr(), _ptr(g.arcs).value, g.weight_sum,
                                  _Params(tau, delta0, seed, variant, step_cap), self.cluster[i].data_ptr(),
                                  self.D[i].data_ptr())
        self.stats = (_Stats * G)()
        total_n = sum(g.n for g in self.graphs)
        self.wsb = self.lib.cldiam_decompose_workspace_size(total_n, G)
        self.ws = _ws(self.wsb, dev)
        self.driver = driver
        self.tuning = _Tuning(local_rounds, grid_blocks, bucket_width, row_bucket_shift, chunk_factor, wave_row_min,
                              group_row_min, local_queue, local_cutoff, pull_mode)

    def run(self, stream=None):
        _check(self.lib.cldiam_decompose_batch(len(self.graphs), self.desc, self.stats, self.driver,
                                               ctypes.byref(self.tuning), _ptr(self.ws), self.wsb, _stream(stream)),
               "cldiam_decompose_batch")
        return [_stats(s) for s in self.stats]


def cldiam_decompose(g: DeviceGraph, tau: int, seed: int, delta0: int = 0, driver=DRIVER_AUTO, stream=None,
                     local_rounds=-1, grid_blocks=0, bucket_width=0.0, variant=0, step_cap=0, row_bucket_shift=0,
                     chunk_factor=0, wave_row_min=0, group_row_min=0, local_queue=0, local_cutoff=0, pull_mode=0):
    """CLUSTER(G, tau): returns (cluster int32 tensor, D int64 tensor holding
    uint64 bit patterns, Stats).  variant = VARIANT_STEPS runs PartialGrowth
    literally (synchronous steps, per-step stop, optional step cap)."""
    job = DecomposeJob([g], [(tau, seed, delta0, variant, step_cap)], driver, local_rounds, grid_blocks,
                       bucket_width, row_bucket_shift, chunk_factor, wave_row_min, group_row_min, local_queue,
                       local_cutoff, pull_mode)
    st = job.run(stream)
    return job.cluster[0], job.D[0], st[0]


def cldiam_decompose_batch(graphs, params, driver=DRIVER_AUTO, stream=None, local_rounds=-1, grid_blocks=0,
                           bucket_width=0.0, row_bucket_shift=0, chunk_factor=0, wave_row_min=0, group_row_min=0,
                           local_queue=0, local_cutoff=0, pull_mode=0):
    """Decomposes many graphs in one device job; params = [(tau, seed, delta0[, variant, step_cap])]."""
    job = DecomposeJob(graphs, params, driver, local_rounds, grid_blocks, bucket_width, row_bucket_shift,
                       chunk_factor, wave_row_min, group_row_min, local_queue, local_cutoff, pull_mode)
    st = job.run(stream)
    return job.cluster, job.D, st


# ---------------------------------------------------------------- server --

class Server:
    """Continuous-batching decomposition job (cldiam_server_*): submit requests
    at any time, step to advance every admitted request together, poll for
    finished ones.  Output tensors of a request are allocated at submit and
    handed back by poll."""

    def __init__(self, node_capacity: int, max_graphs: int = 64, local_rounds: int = -1, grid_blocks: int = 0,
                 bucket_width: float = 0.0, row_bucket_shift: int = 0, chunk_factor: int = 0, device="cuda",
                 stream=None, wave_row_min: int = 0, group_row_min: int = 0, local_queue: int = 0,
                 local_cutoff: int = 0, pull_mode: int = 0):
        torch = _torch()
        self.lib = load_library()
        self.device = device
        self.stream = stream if stream is not None else torch.cuda.Stream(device=device)
        self.wsb = self.lib.cldiam_server_workspace_size(node_capacity, max_graphs)
        self.ws = _ws(self.wsb, device)
        self.ptr = ctypes.c_void_p()
        _check(self.lib.cldiam_server_create(ctypes.byref(self.ptr), node_capacity, max_graphs,
                                             ctypes.byref(_Tuning(local_rounds, grid_blocks, bucket_width, row_bucket_shift,
                                                                  chunk_factor, wave_row_min, group_row_min,
                                                                  local_queue, local_cutoff, pull_mode)),
                                             _ptr(self.ws), self.wsb,
                                             ctypes.c_void_p(self.stream.cuda_stream)), "cldiam_server_create")
        self.outputs = {}
        self.max_graphs = max_graphs

    def submit(self, g: DeviceGraph, tau: int, seed: int, tag: int, delta0: int = 0, variant: int = 0,
               step_cap: int = 0):
        torch = _torch()
        cluster = torch.empty(g.n, dtype=torch.int32, device=self.device)
        D = torch.empty(g.n, dtype=torch.int64, device=self.device)
        desc = _Graph(g.n, 0, g.m, g.row_ptr.data_ptr(), _ptr(g.arcs).value, g.weight_sum,
                      _Params(tau, delta0, seed, variant, step_cap), cluster.data_ptr(), D.data_ptr())
        _check(self.lib.cldiam_server_submit(self.ptr, ctypes.byref(desc), tag), "cldiam_server_submit")
        self.outputs[tag] = (g, cluster, D)

    def step(self, max_sweeps: int = 8):
        active, queued = ctypes.c_int32(), ctypes.c_int32()
        _check(self.lib.cldiam_server_step(self.ptr, max_sweeps, ctypes.byref(active), ctypes.byref(queued)),
               "cldiam_server_step")
        return active.value, queued.value

    def poll(self):
        k = self.max_graphs
        tags = (ctypes.c_uint64 * k)()
        stats = (_Stats * k)()
        nd = ctypes.c_int32()
        _check(self.lib.cldiam_server_poll(self.ptr, tags, stats, k, ctypes.byref(nd)), "cldiam_server_poll")
        out = []
        for i in range(nd.value):
            g, cluster, D = self.outputs.pop(int(tags[i]))
            out.append((int(tags[i]), _stats(stats[i]), g, cluster, D))
        return out

    def close(self):
        if self.ptr:
            self.lib.cldiam_server_destroy(self.ptr)
            self.ptr = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ------------------------------------------------------------- quotient --

@dataclass
class DeviceQuotient:
    k: int
    qm: int
    center: object    # torch int32 [k]
    row_ptr: object   # torch int64 [k+1]
    col: object       # torch int32 [qm]
    w: object         # torch int64 [qm] (uint64 bit patterns)


class QuotientJob:
    def __init__(self, g: DeviceGraph):
        torch = _torch()
        self.lib = load_library()
        self.g = g
        dev = g.row_ptr.device
        self.center = torch.empty(max(g.n, 1), dtype=torch.int32, device=dev)
        self.row_ptr = torch.empty(g.n + 1, dtype=torch.int64, device=dev)
        self.col = torch.empty(max(g.m, 1), dtype=torch.int32, device=dev)
        self.w = torch.empty(max(g.m, 1), dtype=torch.int64, device=dev)
        self.wsb = self.lib.cldiam_quotient_workspace_size(g.n, g.m)
        self.ws = _ws(self.wsb, dev)

    def run(self, cluster, D, stream=None) -> DeviceQuotient:
        k, qm = ctypes.c_int32(), ctypes.c_int64()
        g = self.g
        _check(self.lib.cldiam_build_quotient(g.n, g.m, _ptr(g.row_ptr), _ptr(g.arcs), _ptr(cluster), _ptr(D),
                                              _ptr(self.center), _ptr(self.row_ptr), _ptr(self.col), _ptr(self.w),
                                              ctypes.byref(k), ctypes.byref(qm), _ptr(self.ws), self.wsb,
                                              _stream(stream)), "cldiam_build_quotient")
        kk, mm = int(k.value), int(qm.value)
        return DeviceQuotient(kk, mm, self.center[:kk], self.row_ptr[:kk + 1], self.col[:mm], self.w[:mm])


def cldiam_build_quotient(g: DeviceGraph, cluster, D, stream=None) -> DeviceQuotient:
    return QuotientJob(g).run(cluster, D, stream)


class EstimateJob:
    def __init__(self, max_k: int, max_qm: int, device="cuda"):
        self.lib = load_library()
        self.wsb = self.lib.cldiam_estimate_workspace_size(max(max_k, 1), max_qm)
        self.ws = _ws(self.wsb, device)

    def run(self, q: DeviceQuotient, radius: int, stream=None):
        need = self.lib.cldiam_estimate_workspace_size(max(q.k, 1), q.qm)
        if need > self.wsb:
            self.wsb = need
            self.ws = _ws(need, q.row_ptr.device)
        phi, approx = ctypes.c_uint64(), ctypes.c_uint64()
        _check(self.lib.cldiam_estimate_diameter(q.k, q.qm, _ptr(q.row_ptr), _ptr(q.col), _ptr(q.w), radius,
                                                 ctypes.byref(phi), ctypes.byref(approx), _ptr(self.ws), self.wsb,
                                                 _stream(stream)), "cldiam_estimate_diameter")
        return int(phi.value), int(approx.value)


def cldiam_estimate_diameter(q: DeviceQuotient, radius: int, stream=None):
    """(Phi(G_C), Phi(G_C) + 2 radius)."""
    return EstimateJob(q.k, q.qm, q.row_ptr.device).run(q, radius, stream)


# ----------------------------------------------------------------- SSSP --

def cldiam_sssp_delta_stepping(g: DeviceGraph, source: int, bucket_delta: int = 0, stream=None):
    """(dist int32 tensor holding uint32 bit patterns, max finite distance).
    bucket_delta = 0 lets the library pick its default width."""
    torch = _torch()
    lib = load_library()
    dist = torch.empty(g.n, dtype=torch.int32, device=g.row_ptr.device)
    wsb = lib.cldiam_sssp_workspace_size(g.n, g.m)
    ws = _ws(wsb, g.row_ptr.device)
    mx = ctypes.c_uint64()
    _check(lib.cldiam_sssp_delta_stepping(g.n, g.m, _ptr(g.row_ptr), _ptr(g.arcs), source, bucket_delta, _ptr(dist),
                                          ctypes.byref(mx), _ptr(ws), wsb, _stream(stream)),
           "cldiam_sssp_delta_stepping")
    return dist, int(mx.value)


# -------------------------------------------------------------- helpers --

def u64(t) -> np.ndarray:
    """Device int64 tensor holding uint64 bit patterns -> numpy uint64."""
    return t.detach().cpu().numpy().view(np.uint64)


def u32(t) -> np.ndarray:
    return t.detach().cpu().numpy().view(np.uint32)


def estimate(graph, tau: int, seed: int, delta0: int = 0, device="cuda"):
    """Whole CL-DIAM pipeline on a host graph: ingest, decomposition,
    quotient, estimate.  Returns a dict of host results."""
    g = cldiam_load_csr(graph, device)
    cluster, D, st = cldiam_decompose(g, tau, seed, delta0)
    q = cldiam_build_quotient(g, cluster, D)
    phi, approx = cldiam_estimate_diameter(q, st.radius)
    return dict(cluster=cluster.cpu().numpy(), D=u64(D), stats=st, k=q.k, phi_gc=phi, phi_approx=approx)
