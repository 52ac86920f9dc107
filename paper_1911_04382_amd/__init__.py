"""Python binding of libgrass.so, the gfx950 GRASS spectral sparsification
library (C ABI in include/grass.h).

The binding only marshals arguments: every step of the computation runs in the
library's HIP kernels. Tensors are torch tensors on a ROCm device; PyTorch is used
for device memory and streams only. There is no CPU fallback: if the library is
missing, loading it raises.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass, field

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libgrass.so")
HEADER = os.path.join(os.path.dirname(HERE), "include", "grass.h")

OK, NOT_CONVERGED = 0, 1
ERR_INVALID, ERR_DISCONNECTED, ERR_OOM, ERR_DEVICE, ERR_UNIMPLEMENTED, ERR_CANCELLED = -1, -2, -3, -4, -5, -6
ERR_SOLVE, ERR_NONFINITE = -7, -8
PASS_SOLVE_FAILED = 1
LAUNCH_KERNELS, LAUNCH_CAPTURED = 0, 1
STATUS_NAMES = {0: "OK", 1: "NOT_CONVERGED", -1: "ERR_INVALID", -2: "ERR_DISCONNECTED", -3: "ERR_OOM",
                -4: "ERR_DEVICE", -5: "ERR_UNIMPLEMENTED", -6: "ERR_CANCELLED", -7: "ERR_SOLVE",
                -8: "ERR_NONFINITE"}


class GrassError(RuntimeError):
    """A negative status. `result` carries what the call still returned (the
    partial SparsifyResult of ERR_SOLVE, the stats of grass_embed), else None."""

    def __init__(self, status, msg, result=None):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status
        self.result = result


class grass_graph(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("m", ctypes.c_int64), ("src", ctypes.c_void_p), ("dst", ctypes.c_void_p),
                ("w", ctypes.c_void_p)]


class grass_opts(ctypes.Structure):
    _fields_ = [
        ("sigma2", ctypes.c_double), ("k", ctypes.c_int32), ("t", ctypes.c_int32), ("seed", ctypes.c_uint64),
        ("max_iters", ctypes.c_int32), ("budget_frac", ctypes.c_double), ("sim_hops", ctypes.c_int32),
        ("lambda_steps", ctypes.c_int32), ("pcg_rtol", ctypes.c_double), ("pcg_max_iters", ctypes.c_int32),
        ("pcg_inner_rtol", ctypes.c_double), ("pcg_max_outer", ctypes.c_int32), ("precision", ctypes.c_int32),
        ("init_mask", ctypes.c_void_p),
    ]


class grass_pass_stats(ctypes.Structure):
    _fields_ = [
        ("pass_", ctypes.c_int32), ("lambda_max", ctypes.c_double), ("lambda_min", ctypes.c_double),
        ("kappa", ctypes.c_double), ("theta", ctypes.c_double), ("heat_max", ctypes.c_double),
        ("m_off", ctypes.c_int64), ("candidates", ctypes.c_int64), ("accepted", ctypes.c_int64),
        ("pcg_iters", ctypes.c_int64), ("pcg_resid64", ctypes.c_double), ("ms", ctypes.c_double),
        ("flags", ctypes.c_int32),
    ]

    def as_dict(self):
        return {f[0].rstrip("_"): getattr(self, f[0]) for f in self._fields_}


class grass_solve_info(ctypes.Structure):
    _fields_ = [
        ("iters", ctypes.c_int32), ("inner_iters", ctypes.c_int64), ("resid", ctypes.c_double),
        ("ms", ctypes.c_double), ("added_edges", ctypes.c_int64),
    ]

    def as_dict(self):
        return {f[0]: getattr(self, f[0]) for f in self._fields_}


class grass_partition_info(ctypes.Structure):
    _fields_ = [
        ("steps", ctypes.c_int32), ("outer_iters", ctypes.c_int64), ("inner_iters", ctypes.c_int64),
        ("resid", ctypes.c_double), ("ms", ctypes.c_double),
    ]

    def as_dict(self):
        return {f[0]: getattr(self, f[0]) for f in self._fields_}


class grass_summary(ctypes.Structure):
    _fields_ = [
        ("lambda_max", ctypes.c_double), ("lambda_min", ctypes.c_double), ("kappa", ctypes.c_double),
        ("pcg_resid64", ctypes.c_double), ("heat_max", ctypes.c_double), ("passes", ctypes.c_int32),
        ("tree_edges", ctypes.c_int64), ("added_edges", ctypes.c_int64), ("scored_edges", ctypes.c_int64),
        ("pcg_iters", ctypes.c_int64),
    ]

    def as_dict(self):
        return {f[0]: getattr(self, f[0]) for f in self._fields_}


class grass_kernel_stats(ctypes.Structure):
    _fields_ = [("name", ctypes.c_char_p), ("launches", ctypes.c_int64), ("total_ms", ctypes.c_double),
                ("alg_bytes", ctypes.c_double)]


class grass_launch_stats(ctypes.Structure):
    _fields_ = [("iterations", ctypes.c_int64), ("host_reads", ctypes.c_int64), ("graph_replays", ctypes.c_int64),
                ("captures", ctypes.c_int64)]


class grass_req_info(ctypes.Structure):
    _fields_ = [("state", ctypes.c_int32), ("status", ctypes.c_int), ("t_submit", ctypes.c_double),
                ("t_start", ctypes.c_double), ("t_end", ctypes.c_double), ("footprint", ctypes.c_size_t)]

    def as_dict(self):
        return {f[0]: getattr(self, f[0]) for f in self._fields_}


REQ_QUEUED, REQ_RUNNING, REQ_DONE, REQ_CANCELLED = 0, 1, 2, 3


class grass_result(ctypes.Structure):
    _fields_ = [("edge_mask", ctypes.c_void_p), ("scores", ctypes.c_void_p),
                ("summary", ctypes.POINTER(grass_summary)), ("trace", ctypes.POINTER(grass_pass_stats)),
                ("trace_cap", ctypes.c_int32)]


_lib = None


def load_library(path: str = LIB_PATH):
    """Load libgrass.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"{path} is missing: build it with `python -m paper_1911_04382_amd.build`")
    L = ctypes.CDLL(path)
    vp, i32, i64, u64, dbl = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_uint64, ctypes.c_double
    st = ctypes.c_int
    L.grass_create.argtypes = [ctypes.c_int, ctypes.POINTER(vp)]
    L.grass_create.restype = st
    L.grass_destroy.argtypes = [vp]
    L.grass_destroy.restype = None
    L.grass_last_error.argtypes = [vp]
    L.grass_last_error.restype = ctypes.c_char_p
    L.grass_opts_default.argtypes = []
    L.grass_opts_default.restype = grass_opts
    L.grass_workspace_bytes.argtypes = [i64, i64, ctypes.POINTER(grass_opts)]
    L.grass_workspace_bytes.restype = ctypes.c_size_t
    L.grass_sparsify.argtypes = [vp, ctypes.POINTER(grass_graph), ctypes.POINTER(grass_opts), vp, ctypes.c_size_t,
                                 ctypes.POINTER(grass_result), vp]
    L.grass_sparsify.restype = st
    L.grass_sparsify_static.argtypes = [vp, ctypes.POINTER(grass_graph), ctypes.POINTER(grass_opts),
                                        ctypes.POINTER(grass_result), vp]
    L.grass_sparsify_static.restype = st
    L.grass_spanning_tree.argtypes = [vp, ctypes.POINTER(grass_graph), vp, vp, ctypes.c_size_t, vp]
    L.grass_spanning_tree.restype = st
    L.grass_low_stretch_tree_workspace_bytes.argtypes = [i64, i64]
    L.grass_low_stretch_tree_workspace_bytes.restype = ctypes.c_size_t
    L.grass_low_stretch_tree.argtypes = [vp, ctypes.POINTER(grass_graph), ctypes.c_uint64, i32, vp, vp, ctypes.c_size_t,
                                         vp]
    L.grass_low_stretch_tree.restype = st
    L.grass_embed.argtypes = [vp, ctypes.POINTER(grass_graph), vp, ctypes.POINTER(grass_opts), i32, vp,
                              ctypes.POINTER(grass_pass_stats), vp, ctypes.c_size_t, vp]
    L.grass_embed.restype = st
    L.grass_select.argtypes = [vp, ctypes.POINTER(grass_graph), vp, ctypes.POINTER(grass_opts), vp, dbl, dbl,
                               ctypes.POINTER(grass_pass_stats), vp, vp, ctypes.c_size_t, vp]
    L.grass_select.restype = st
    L.grass_solve_workspace_bytes.argtypes = [i64, i64, ctypes.POINTER(grass_opts)]
    L.grass_solve_workspace_bytes.restype = ctypes.c_size_t
    L.grass_solve.argtypes = [vp, ctypes.POINTER(grass_graph), vp, ctypes.POINTER(grass_opts), vp, vp, dbl, i32,
                              ctypes.POINTER(grass_solve_info), vp, ctypes.c_size_t, vp]
    L.grass_solve.restype = st
    L.grass_partition_workspace_bytes.argtypes = [i64, i64, ctypes.POINTER(grass_opts)]
    L.grass_partition_workspace_bytes.restype = ctypes.c_size_t
    L.grass_partition.argtypes = [vp, ctypes.POINTER(grass_graph), vp, ctypes.POINTER(grass_opts), i32, dbl, vp, vp,
                                  ctypes.POINTER(grass_partition_info), vp, ctypes.c_size_t, vp]
    L.grass_partition.restype = st
    L.grass_start_vectors.argtypes = [vp, i64, i32, u64, i32, i32, vp, vp]
    L.grass_start_vectors.restype = st
    L.grass_gram.argtypes = [vp, i64, i32, i32, vp, vp, vp, vp]
    L.grass_gram.restype = st
    L.grass_profile_enable.argtypes = [vp, ctypes.c_uint32]
    L.grass_profile_enable.restype = st
    L.grass_profile_read.argtypes = [vp, ctypes.POINTER(grass_kernel_stats), i32]
    L.grass_profile_read.restype = i32
    L.grass_set_launch_mode.argtypes = [vp, i32, i32]
    L.grass_set_launch_mode.restype = st
    L.grass_launch_stats_read.argtypes = [vp, ctypes.POINTER(grass_launch_stats), i32]
    L.grass_launch_stats_read.restype = st
    L.grass_batch_workspace_bytes.argtypes = [i32, ctypes.POINTER(grass_graph), ctypes.POINTER(grass_opts), i32, i32]
    L.grass_batch_workspace_bytes.restype = ctypes.c_size_t
    L.grass_sparsify_batch.argtypes = [vp, i32, ctypes.POINTER(grass_graph), ctypes.POINTER(grass_opts), i32, i32,
                                       vp, ctypes.c_size_t, ctypes.POINTER(grass_result), ctypes.POINTER(st), vp]
    L.grass_sparsify_batch.restype = st
    L.grass_server_create.argtypes = [vp, ctypes.c_size_t, i32, ctypes.POINTER(vp)]
    L.grass_server_create.restype = st
    L.grass_server_submit.argtypes = [vp, ctypes.POINTER(grass_graph), ctypes.POINTER(grass_opts),
                                      ctypes.POINTER(grass_result), ctypes.POINTER(i64)]
    L.grass_server_submit.restype = st
    L.grass_server_poll.argtypes = [vp, i64, ctypes.POINTER(grass_req_info)]
    L.grass_server_poll.restype = st
    L.grass_server_wait.argtypes = [vp, i64]
    L.grass_server_wait.restype = st
    L.grass_server_cancel.argtypes = [vp, i64]
    L.grass_server_cancel.restype = st
    L.grass_server_error.argtypes = [vp, i64]
    L.grass_server_error.restype = ctypes.c_char_p
    L.grass_server_destroy.argtypes = [vp]
    L.grass_server_destroy.restype = None
    _lib = L
    return L


def exported_symbols_declared_in_header(header: str = HEADER):
    """Names of the functions include/grass.h declares."""
    import re

    text = open(header).read()
    return sorted(set(re.findall(r"\b(grass_[a-z_]+)\s*\(", text)))


# ------------------------------------------------------------------ context
class Context:
    """One library context on one HIP device (grass_create / grass_destroy)."""

    def __init__(self, device: int = 0):
        self.lib = load_library()
        h = ctypes.c_void_p()
        rc = self.lib.grass_create(device, ctypes.byref(h))
        if rc != OK:
            raise GrassError(rc, f"grass_create({device}) failed")
        self.h = h
        self.device = device

    def close(self):
        if getattr(self, "h", None):
            self.lib.grass_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def last_error(self) -> str:
        return self.lib.grass_last_error(self.h).decode()

    def profile(self, enable: bool = True, kinds=None):
        """Enable (and reset) per-kernel event timing (grass_profile_enable): every
        kind, or only the named ones (names as returned by profile_read)."""
        mask = 0
        if enable:
            if kinds is None:
                mask = 0xFFFFFFFF
            else:
                names = list(self.profile_read().keys())
                for k in kinds:
                    mask |= 1 << names.index(k)
        self.check(self.lib.grass_profile_enable(self.h, mask))

    def profile_read(self) -> dict:
        n = self.lib.grass_profile_read(self.h, None, 0)
        arr = (grass_kernel_stats * n)()
        got = self.lib.grass_profile_read(self.h, arr, n)
        return {arr[i].name.decode(): {"launches": arr[i].launches, "ms": arr[i].total_ms,
                                       "alg_bytes": arr[i].alg_bytes} for i in range(got)}

    def set_launch_mode(self, mode: int, chunks_per_read: int = 0):
        """grass_set_launch_mode: LAUNCH_KERNELS or LAUNCH_CAPTURED (chunks of four
        block-PCG iterations replayed chunks_per_read times between host reads; 0 lets
        the context's autotuner choose) for the batch and server paths."""
        self.check(self.lib.grass_set_launch_mode(self.h, int(mode), int(chunks_per_read)))

    def launch_stats(self, reset: bool = False) -> dict:
        """grass_launch_stats_read: iterations, host reads, graph replays, captures."""
        out = grass_launch_stats()
        self.check(self.lib.grass_launch_stats_read(self.h, ctypes.byref(out), 1 if reset else 0))
        return {f[0]: getattr(out, f[0]) for f in out._fields_}

    def check(self, rc):
        if rc < 0:
            raise GrassError(rc, self.last_error())
        return rc


# ----------------------------------------------------------------- helpers
def _torch():
    import torch

    return torch


def _stream_ptr(stream):
    torch = _torch()
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


@dataclass
class DeviceGraph:
    """A canonical graph held on the device (int32 src/dst, float64 w)."""

    n: int
    src: object
    dst: object
    w: object

    @property
    def m(self) -> int:
        return int(self.src.shape[0])

    def c(self) -> grass_graph:
        return grass_graph(self.n, self.m, self.src.data_ptr(), self.dst.data_ptr(), self.w.data_ptr())


def to_device(g, device="cuda:0") -> DeviceGraph:
    """Copy a host graph (numpy arrays n, src, dst, w) to the device."""
    torch = _torch()
    return DeviceGraph(int(g.n), torch.as_tensor(g.src, dtype=torch.int32).to(device),
                       torch.as_tensor(g.dst, dtype=torch.int32).to(device),
                       torch.as_tensor(g.w, dtype=torch.float64).to(device))


def make_opts(**kw) -> grass_opts:
    o = load_library().grass_opts_default()
    for k, v in kw.items():
        if k == "init_mask":
            o.init_mask = None if v is None else v.data_ptr()
        else:
            setattr(o, k, v)
    return o


def workspace(g: DeviceGraph, opts: grass_opts, device="cuda:0"):
    """A uint8 device tensor of grass_workspace_bytes()."""
    torch = _torch()
    nbytes = load_library().grass_workspace_bytes(g.n, g.m, ctypes.byref(opts))
    return torch.empty(int(nbytes), dtype=torch.uint8, device=device)


def _ws_args(ws):
    if ws is None:
        return None, 0
    return ctypes.c_void_p(ws.data_ptr()), int(ws.numel())


# ------------------------------------------------------- the C-ABI calls
@dataclass
class SparsifyResult:
    status: int
    mask: object
    scores: object
    summary: dict
    trace: list = field(default_factory=list)


def grass_sparsify(ctx: Context, g: DeviceGraph, opts: grass_opts, ws=None, stream=None, trace_cap=256):
    torch = _torch()
    dev = g.src.device
    mask = torch.empty(g.m, dtype=torch.uint8, device=dev)
    scores = torch.empty(g.m, dtype=torch.float64 if opts.precision == 64 else torch.float32, device=dev)
    summ = grass_summary()
    tr = (grass_pass_stats * trace_cap)()
    res = grass_result(mask.data_ptr(), scores.data_ptr(), ctypes.pointer(summ),
                       ctypes.cast(tr, ctypes.POINTER(grass_pass_stats)), trace_cap)
    gc = g.c()
    wsp, wsb = _ws_args(ws)
    rc = ctx.lib.grass_sparsify(ctx.h, ctypes.byref(gc), ctypes.byref(opts), wsp, wsb, ctypes.byref(res),
                                _stream_ptr(stream))
    if rc < 0:
        part = None
        if rc == ERR_SOLVE:  # the mask, summary and trace are still valid
            part = SparsifyResult(rc, mask, None, summ.as_dict(),
                                  [tr[i].as_dict() for i in range(min(summ.passes, trace_cap))])
        raise GrassError(rc, ctx.last_error(), part)
    trace = [tr[i].as_dict() for i in range(min(summ.passes, trace_cap))]
    return SparsifyResult(rc, mask, scores, summ.as_dict(), trace)


STATIC_SCRATCH_BYTES = 256 << 20  # GRASS_STATIC_SCRATCH_BYTES of include/grass.h


def grass_sparsify_static(ctx: Context, g: DeviceGraph, opts: grass_opts, stream=None, trace_cap=256):
    """grass_sparsify over the library's static device scratch (no device allocation
    by the library; the outputs are allocated here, by the caller)."""
    mask, scores, summ, tr, res = _result_buffers(g, opts, trace_cap)
    gc = g.c()
    rc = ctx.lib.grass_sparsify_static(ctx.h, ctypes.byref(gc), ctypes.byref(opts), ctypes.byref(res),
                                       _stream_ptr(stream))
    if rc < 0:
        raise GrassError(rc, ctx.last_error())
    trace = [tr[i].as_dict() for i in range(min(summ.passes, trace_cap))]
    return SparsifyResult(rc, mask, scores, summ.as_dict(), trace)


def _result_buffers(g: DeviceGraph, opts: grass_opts, trace_cap: int):
    torch = _torch()
    dev = g.src.device
    mask = torch.empty(g.m, dtype=torch.uint8, device=dev)
    scores = torch.empty(g.m, dtype=torch.float64 if opts.precision == 64 else torch.float32, device=dev)
    summ = grass_summary()
    tr = (grass_pass_stats * trace_cap)()
    res = grass_result(mask.data_ptr(), scores.data_ptr(), ctypes.pointer(summ),
                       ctypes.cast(tr, ctypes.POINTER(grass_pass_stats)), trace_cap)
    return mask, scores, summ, tr, res


def batch_workspace(graphs, opts, workers: int, device="cuda:0"):
    """A uint8 device tensor of grass_batch_workspace_bytes()."""
    torch = _torch()
    opts_list = opts if isinstance(opts, (list, tuple)) else [opts]
    gcs = (grass_graph * len(graphs))(*[g.c() for g in graphs])
    oc = (grass_opts * len(opts_list))(*opts_list)
    nbytes = load_library().grass_batch_workspace_bytes(len(graphs), gcs, oc, len(opts_list), workers)
    return torch.empty(int(nbytes), dtype=torch.uint8, device=device)


def grass_sparsify_batch(ctx: Context, graphs, opts, workers: int = 8, ws=None, stream=None, trace_cap=256):
    """grass_sparsify_batch: (status, one SparsifyResult per graph). opts: one
    grass_opts for every graph, or a list with one per graph. A graph that fails
    carries its own status; the call raises only when no graph ran."""
    opts_list = opts if isinstance(opts, (list, tuple)) else [opts]
    n = len(graphs)
    bufs = [_result_buffers(g, opts_list[0 if len(opts_list) == 1 else i], trace_cap) for i, g in enumerate(graphs)]
    gcs = (grass_graph * n)(*[g.c() for g in graphs])
    oc = (grass_opts * len(opts_list))(*opts_list)
    rs = (grass_result * n)(*[b[4] for b in bufs])
    sts = (ctypes.c_int * n)()
    if ws is None:
        ws = batch_workspace(graphs, opts, workers, graphs[0].src.device)
    rc = ctx.lib.grass_sparsify_batch(ctx.h, n, gcs, oc, len(opts_list), workers, ctypes.c_void_p(ws.data_ptr()),
                                      int(ws.numel()), rs, sts, _stream_ptr(stream))
    if rc < 0 and all(sts[i] >= 0 for i in range(n)):  # the call itself failed (no graph ran)
        ctx.check(rc)
    out = []
    for i, (mask, scores, summ, tr, _) in enumerate(bufs):
        trace = [tr[j].as_dict() for j in range(min(summ.passes, trace_cap))]
        out.append(SparsifyResult(sts[i], mask, scores, summ.as_dict(), trace))
    return rc, out


class Server:
    """grass_server_*: a serving queue with admission by HBM footprint."""

    def __init__(self, ctx: Context, arena_bytes: int, workers: int = 4):
        self.ctx = ctx
        self.lib = ctx.lib
        h = ctypes.c_void_p()
        ctx.check(self.lib.grass_server_create(ctx.h, int(arena_bytes), workers, ctypes.byref(h)))
        self.h = h
        self._keep = {}

    def submit(self, g: DeviceGraph, opts: grass_opts, trace_cap=64) -> int:
        mask, scores, summ, tr, res = _result_buffers(g, opts, trace_cap)
        gc = g.c()
        oc = grass_opts.from_buffer_copy(opts)
        t = ctypes.c_int64()
        self.ctx.check(self.lib.grass_server_submit(self.h, ctypes.byref(gc), ctypes.byref(oc), ctypes.byref(res),
                                                    ctypes.byref(t)))
        # everything the request points to stays alive until it is collected
        self._keep[t.value] = (g, mask, scores, summ, tr, res, gc, oc, trace_cap)
        return t.value

    def poll(self, ticket: int) -> dict:
        info = grass_req_info()
        self.ctx.check(self.lib.grass_server_poll(self.h, ticket, ctypes.byref(info)))
        return info.as_dict()

    def wait(self, ticket: int = -1):
        self.ctx.check(self.lib.grass_server_wait(self.h, ticket))

    def cancel(self, ticket: int):
        return self.lib.grass_server_cancel(self.h, ticket)

    def error(self, ticket: int) -> str:
        return self.lib.grass_server_error(self.h, ticket).decode()

    def result(self, ticket: int) -> SparsifyResult:
        """The outputs of a finished request (waits for it)."""
        self.wait(ticket)
        info = self.poll(ticket)
        g, mask, scores, summ, tr, res, gc, oc, cap = self._keep[ticket]
        trace = [tr[j].as_dict() for j in range(min(summ.passes, cap))]
        return SparsifyResult(info["status"], mask, scores, summ.as_dict(), trace)

    def close(self):
        if self.h:
            self.lib.grass_server_destroy(self.h)
            self.h = None
            self._keep.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def grass_spanning_tree(ctx: Context, g: DeviceGraph, ws=None, stream=None):
    torch = _torch()
    mask = torch.empty(g.m, dtype=torch.uint8, device=g.src.device)
    gc = g.c()
    wsp, wsb = _ws_args(ws)
    ctx.check(ctx.lib.grass_spanning_tree(ctx.h, ctypes.byref(gc), ctypes.c_void_p(mask.data_ptr()), wsp, wsb,
                                          _stream_ptr(stream)))
    return mask


def low_stretch_tree_workspace(g: DeviceGraph, device="cuda:0"):
    """A uint8 device tensor of grass_low_stretch_tree_workspace_bytes()."""
    torch = _torch()
    nbytes = load_library().grass_low_stretch_tree_workspace_bytes(g.n, g.m)
    return torch.empty(int(nbytes), dtype=torch.uint8, device=device)


def grass_low_stretch_tree(ctx: Context, g: DeviceGraph, seed=0, class_bits=2, ws=None, stream=None):
    """Low-stretch spanning tree mask (device uint8 [m]); see include/grass.h."""
    torch = _torch()
    mask = torch.empty(g.m, dtype=torch.uint8, device=g.src.device)
    gc = g.c()
    wsp, wsb = _ws_args(ws)
    ctx.check(ctx.lib.grass_low_stretch_tree(ctx.h, ctypes.byref(gc), ctypes.c_uint64(seed), int(class_bits),
                                             ctypes.c_void_p(mask.data_ptr()), wsp, wsb, _stream_ptr(stream)))
    return mask


def grass_embed(ctx: Context, g: DeviceGraph, p_mask, opts: grass_opts, pass_=0, ws=None, stream=None):
    torch = _torch()
    heat = torch.empty(g.m, dtype=torch.float64 if opts.precision == 64 else torch.float32, device=g.src.device)
    st = grass_pass_stats()
    gc = g.c()
    wsp, wsb = _ws_args(ws)
    rc = ctx.lib.grass_embed(ctx.h, ctypes.byref(gc), ctypes.c_void_p(p_mask.data_ptr()), ctypes.byref(opts), pass_,
                             ctypes.c_void_p(heat.data_ptr()), ctypes.byref(st), wsp, wsb, _stream_ptr(stream))
    if rc < 0:
        raise GrassError(rc, ctx.last_error(), st.as_dict() if rc == ERR_SOLVE else None)
    return heat, st.as_dict()


def solve_workspace(g: DeviceGraph, opts: grass_opts, device="cuda:0"):
    """A uint8 device tensor of grass_solve_workspace_bytes()."""
    torch = _torch()
    nbytes = load_library().grass_solve_workspace_bytes(g.n, g.m, ctypes.byref(opts))
    return torch.empty(int(nbytes), dtype=torch.uint8, device=device)


def grass_solve(ctx: Context, g: DeviceGraph, b, opts: grass_opts, p_mask=None, rtol=1e-3, max_iters=1000, ws=None,
                stream=None):
    """Sec. V-E: x with L_G x = b (grounded at node 0), preconditioned by L_P^+ for the
    subgraph of p_mask (None: the spanning tree). b: device n x opts.k tensor of the
    working precision. Returns (status, x, info dict)."""
    torch = _torch()
    b = b.contiguous()
    x = torch.empty_like(b)
    info = grass_solve_info()
    gc = g.c()
    wsp, wsb = _ws_args(ws)
    rc = ctx.check(ctx.lib.grass_solve(ctx.h, ctypes.byref(gc),
                                       None if p_mask is None else ctypes.c_void_p(p_mask.data_ptr()),
                                       ctypes.byref(opts), ctypes.c_void_p(b.data_ptr()), ctypes.c_void_p(x.data_ptr()),
                                       float(rtol), int(max_iters), ctypes.byref(info), wsp, wsb, _stream_ptr(stream)))
    return rc, x, info.as_dict()


def grass_partition(ctx: Context, g: DeviceGraph, opts: grass_opts, p_mask=None, steps=5, rtol=1e-3, ws=None,
                    stream=None):
    """Sec. V-F: (status, fiedler vector, side (uint8, 1 where u >= 0), info dict)."""
    torch = _torch()
    u = torch.empty(g.n, dtype=torch.float64 if opts.precision == 64 else torch.float32, device=g.src.device)
    side = torch.empty(g.n, dtype=torch.uint8, device=g.src.device)
    info = grass_partition_info()
    gc = g.c()
    wsp, wsb = _ws_args(ws)
    rc = ctx.check(ctx.lib.grass_partition(ctx.h, ctypes.byref(gc),
                                           None if p_mask is None else ctypes.c_void_p(p_mask.data_ptr()),
                                           ctypes.byref(opts), int(steps), float(rtol), ctypes.c_void_p(u.data_ptr()),
                                           ctypes.c_void_p(side.data_ptr()), ctypes.byref(info), wsp, wsb,
                                           _stream_ptr(stream)))
    return rc, u, side, info.as_dict()


def grass_select(ctx: Context, g: DeviceGraph, p_mask, opts: grass_opts, heat, lambda_max, lambda_min, ws=None,
                 stream=None, want_scores=True):
    """Filter + similarity check of one pass; p_mask is updated in place."""
    torch = _torch()
    scores = torch.empty_like(heat) if want_scores else None
    st = grass_pass_stats()
    gc = g.c()
    wsp, wsb = _ws_args(ws)
    ctx.check(ctx.lib.grass_select(ctx.h, ctypes.byref(gc), ctypes.c_void_p(p_mask.data_ptr()), ctypes.byref(opts),
                                   ctypes.c_void_p(heat.data_ptr()), float(lambda_max), float(lambda_min),
                                   ctypes.byref(st), None if scores is None else ctypes.c_void_p(scores.data_ptr()),
                                   wsp, wsb, _stream_ptr(stream)))
    return scores, st.as_dict()


def grass_start_vectors(ctx: Context, n, k, seed, pass_=0, precision=32, device="cuda:0", stream=None):
    torch = _torch()
    out = torch.empty((n, k), dtype=torch.float64 if precision == 64 else torch.float32, device=device)
    ctx.check(ctx.lib.grass_start_vectors(ctx.h, n, k, seed, pass_, precision, ctypes.c_void_p(out.data_ptr()),
                                          _stream_ptr(stream)))
    return out


def grass_gram(ctx: Context, a, b, stream=None):
    """A'B (float64, k x k) of two device n x k tensors (float32 or float64)."""
    torch = _torch()
    n, k = a.shape
    out = torch.empty((k, k), dtype=torch.float64, device=a.device)
    prec = 64 if a.dtype == torch.float64 else 32
    ctx.check(ctx.lib.grass_gram(ctx.h, n, k, prec, ctypes.c_void_p(a.data_ptr()), ctypes.c_void_p(b.data_ptr()),
                                 ctypes.c_void_p(out.data_ptr()), _stream_ptr(stream)))
    return out


def grass_workspace_bytes(n, m, opts: grass_opts) -> int:
    return int(load_library().grass_workspace_bytes(n, m, ctypes.byref(opts)))
