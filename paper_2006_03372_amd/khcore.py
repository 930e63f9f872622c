"""Python binding of libkhcore.so (ctypes): argument marshalling only.

Every computation runs in the library's HIP kernels; torch is used here for
device memory and streams.  The binding refuses to work without the built
library: there is no host fallback.
"""
from __future__ import annotations

import ctypes
import os
import weakref

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libkhcore.so")

KHC_OK = 0
KHC_EINVAL = -1
KHC_EGRAPH = -2
KHC_ENOMEM = -3
KHC_EHIP = -4
KHC_ELIMIT = -5

OPT_MAX_WIDTH = 1
OPT_SCHEDULE = 2
OPT_WORKSPACE_LIMIT = 3
OPT_VALIDATE = 4
OPT_WAVES_PER_CU = 5
OPT_PROFILE = 6
OPT_DRIVER = 7
OPT_PERSIST_WIDTH = 8
OPT_BARRIER_TIMEOUT = 9
OPT_ROUND_LIMIT = 10
OPT_PUSH_COST = 11
OPT_TUNE_REPEATS = 12
OPT_TUNE_CACHE = 13

EXPORTED = [
    "khc_create", "khc_destroy", "khc_last_error", "khc_set_option", "khc_profile_read",
    "khc_graph_create", "khc_graph_destroy", "khc_validate_csr",
    "khdeg_compute", "khdeg_compute_list", "khdeg_scanned_arcs", "khcore_decompose",
    "khc_graph_create_batched", "khcore_decompose_batched",
    "khc_mlp_create", "khc_mlp_destroy", "khc_mlp_set_params", "khc_mlp_get_params",
    "khc_mlp_forward", "khc_mlp_gradient", "khc_mlp_train", "khc_features", "khcore_decompose_approx",
    "khc_persist_profile_read", "khc_set_progress", "khc_autotune", "khc_mlp_save", "khc_mlp_load",
    "khc_mlp_get_moments", "khdeg_compute_noalloc", "khcore_decompose_sampled", "khc_gate_features",
    "khcore_decompose_gated", "khc_mlp_samples", "khc_alive_after",
]

PROGRESS_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_uint32, ctypes.c_uint64, ctypes.c_uint32)

PERSIST_PHASES = ["init", "compact", "lb_all", "keymin", "level", "collect", "clean", "select", "affected",
                  "kill", "lbd", "unmark", "bfs_reset", "bfs_seed", "bfs_level", "bfs_scatter", "done"]

N_PARAMS = 4801


TUNE_MAX = 16


class Tune(ctypes.Structure):
    _fields_ = [("width_words", ctypes.c_uint32), ("waves_per_cu", ctypes.c_uint32),
                ("persistent", ctypes.c_uint32), ("candidates", ctypes.c_uint32),
                ("cand_width", ctypes.c_uint32 * TUNE_MAX), ("cand_waves", ctypes.c_uint32 * TUNE_MAX),
                ("trial_ms", ctypes.c_double * TUNE_MAX), ("repeats", ctypes.c_uint32),
                ("cached", ctypes.c_uint32)]

    def as_dict(self):
        k = self.candidates
        return {"width_words": self.width_words, "waves_per_cu": self.waves_per_cu,
                "persistent": bool(self.persistent), "repeats": self.repeats, "cached": bool(self.cached),
                "trials": [(self.cand_width[i], self.cand_waves[i], self.trial_ms[i]) for i in range(k)]}


class KhcError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"khcore error {code}: {msg}")
        self.code = code


class CSRStruct(ctypes.Structure):
    _fields_ = [("n", ctypes.c_uint32), ("nnz", ctypes.c_uint64),
                ("row_ptr", ctypes.c_void_p), ("col", ctypes.c_void_p)]


class Profile(ctypes.Structure):
    _fields_ = [("launches", ctypes.c_uint64 * 4), ("ms", ctypes.c_double * 4),
                ("bytes", ctypes.c_double * 4)]

    CLASSES = ("clear", "level_first", "level_inner", "level_last")

    def as_dict(self):
        return {c: {"launches": int(self.launches[i]), "ms": float(self.ms[i]),
                    "bytes": float(self.bytes[i])} for i, c in enumerate(self.CLASSES)}


class Stats(ctypes.Structure):
    _fields_ = [("rounds", ctypes.c_uint64), ("h_recomputes", ctypes.c_uint64),
                ("hm1_recomputes", ctypes.c_uint64), ("bfs_batches", ctypes.c_uint64),
                ("affected_total", ctypes.c_uint64), ("max_level", ctypes.c_uint32),
                ("width_words", ctypes.c_uint32), ("wall_ms", ctypes.c_double),
                ("local_rounds", ctypes.c_uint64), ("local_sources", ctypes.c_uint64),
                ("gate_deferrals", ctypes.c_uint64)]

    def as_dict(self):
        return {name: getattr(self, name) for name, _ in self._fields_}


_lib = None


def load_library(path: str = LIB_PATH):
    """Load libkhcore.so and declare its signatures.  Raises if missing."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"{path} is not built; run __graft_entry__.build() "
                          "or python -m paper_2006_03372_amd.build")
    lib = ctypes.CDLL(path)
    P, u32, u64, i32, i64 = ctypes.c_void_p, ctypes.c_uint32, ctypes.c_uint64, ctypes.c_int, ctypes.c_int64
    PP = ctypes.POINTER(ctypes.c_void_p)
    sig = {
        "khc_create": ([PP, i32, P], i32),
        "khc_destroy": ([P], i32),
        "khc_last_error": ([P], ctypes.c_char_p),
        "khc_set_option": ([P, i32, i64], i32),
        "khc_profile_read": ([P, ctypes.POINTER(Profile), i32], i32),
        "khc_graph_create": ([P, ctypes.POINTER(CSRStruct), PP], i32),
        "khc_graph_destroy": ([P], i32),
        "khc_validate_csr": ([P, ctypes.POINTER(CSRStruct)], i32),
        "khdeg_compute": ([P, P, P, u32, P], i32),
        "khdeg_compute_noalloc": ([P, P, P, u32, P], i32),
        "khdeg_compute_list": ([P, P, P, u32, P, u32, P], i32),
        "khdeg_scanned_arcs": ([P, P, P, u32, P], i32),
        "khcore_decompose": ([P, P, u32, P, P, ctypes.POINTER(Stats)], i32),
        "khc_graph_create_batched": ([P, u32, P, P, P, u64, PP], i32),
        "khcore_decompose_batched": ([P, u32, P, P, P, u64, u32, P, P, ctypes.POINTER(Stats)], i32),
        "khc_mlp_create": ([P, u64, PP], i32),
        "khc_mlp_destroy": ([P], i32),
        "khc_mlp_set_params": ([P, P, P], i32),
        "khc_mlp_get_params": ([P, P, P, P], i32),
        "khc_mlp_forward": ([P, P, P, u32, P], i32),
        "khc_mlp_gradient": ([P, P, P, P, u32, P], i32),
        "khc_mlp_train": ([P, P, P, P, u32, u32, u32, ctypes.c_float, u64, P], i32),
        "khc_features": ([P, P, P, u32, P, P, P], i32),
        "khcore_decompose_approx": ([P, P, u32, P, P, P, ctypes.POINTER(Stats)], i32),
        "khcore_decompose_sampled": ([P, P, u32, P, P, P, ctypes.POINTER(Stats)], i32),
        "khc_gate_features": ([P, P, P, u32, P, P], i32),
        "khc_mlp_samples": ([P, P, P, u32, i32, P, P, ctypes.POINTER(u32)], i32),
        "khc_alive_after": ([P, u32, P, u32, P], i32),
        "khcore_decompose_gated": ([P, P, u32, P, ctypes.c_float, P, P, ctypes.POINTER(Stats)], i32),
        "khc_persist_profile_read": ([P, P, P, i32], i32),
        "khc_set_progress": ([P, PROGRESS_FN, P, u32], i32),
        "khc_autotune": ([P, P, u32, u32, ctypes.POINTER(Tune)], i32),
        "khc_mlp_save": ([P, P, ctypes.c_char_p], i32),
        "khc_mlp_load": ([P, P, ctypes.c_char_p], i32),
        "khc_mlp_get_moments": ([P, P, P, P, ctypes.POINTER(ctypes.c_uint64)], i32),
    }
    for name, (args, res) in sig.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = res
    _lib = lib
    return lib


def _torch():
    import torch
    return torch


def _dptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


class Context:
    """A library context bound to one device and one HIP stream."""

    def __init__(self, device: int = 0, stream=None):
        torch = _torch()
        self.lib = load_library()
        if not torch.cuda.is_available():
            raise RuntimeError("no GPU visible: the khcore library needs an MI355X")
        self.device = device
        self.stream = stream if stream is not None else torch.cuda.current_stream(device)
        h = ctypes.c_void_p()
        rc = self.lib.khc_create(ctypes.byref(h), device, ctypes.c_void_p(self.stream.cuda_stream))
        if rc:
            raise KhcError(rc, "khc_create failed")
        self.handle = h
        # graph handles refer to the context: they are released first
        self._graphs = weakref.WeakSet()

    def _check(self, rc):
        if rc:
            msg = self.lib.khc_last_error(self.handle)
            raise KhcError(rc, msg.decode() if msg else "")

    def set_option(self, option: int, value: int):
        self._check(self.lib.khc_set_option(self.handle, option, int(value)))

    def profile_read(self, reset: bool = True) -> dict:
        """Kernel timing recorded while OPT_PROFILE is on (see khc_profile)."""
        p = Profile()
        self._check(self.lib.khc_profile_read(self.handle, ctypes.byref(p), int(reset)))
        return p.as_dict()

    def set_progress(self, fn=None, interval_ms: int = 1000):
        """fn(rounds, removed, level), called from the decomposition loops at
        most every interval_ms milliseconds; None turns it off."""
        if fn is None:
            self._progress = None
            self._check(self.lib.khc_set_progress(self.handle, PROGRESS_FN(), None, interval_ms))
            return
        self._progress = PROGRESS_FN(lambda _u, r, removed, level: fn(int(r), int(removed), int(level)))
        self._check(self.lib.khc_set_progress(self.handle, self._progress, None, interval_ms))

    def autotune(self, graph: "Graph", h: int, rounds: int = 64) -> dict:
        """Time trial decompositions (cut after `rounds` rounds) over the
        width x waves-per-CU candidates, OPT_TUNE_REPEATS times each, and keep
        the smallest median on this context (or apply the choice cached for
        the graph's size class)."""
        t = Tune()
        self._check(self.lib.khc_autotune(self.handle, graph.handle, h, rounds, ctypes.byref(t)))
        return t.as_dict()

    def persist_profile_read(self, reset: bool = True) -> dict:
        """Per-phase time (ms) and counts of the persistent driver's runs made
        while OPT_PROFILE is on."""
        ms = np.zeros(len(PERSIST_PHASES), dtype=np.float64)
        cnt = np.zeros(len(PERSIST_PHASES), dtype=np.uint64)
        self._check(self.lib.khc_persist_profile_read(self.handle, ms.ctypes.data_as(ctypes.c_void_p),
                                                      cnt.ctypes.data_as(ctypes.c_void_p), int(reset)))
        return {name: (float(ms[i]), int(cnt[i])) for i, name in enumerate(PERSIST_PHASES)}

    def close(self):
        if getattr(self, "handle", None):
            for g in list(getattr(self, "_graphs", ())):
                g.close()
            self.lib.khc_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    # -------------------------------------------------------------- graph
    def graph(self, g) -> "Graph":
        """Upload a host CSR (synth.CSR) and build its row schedule."""
        return Graph(self, g)

    def batch(self, graphs) -> "BatchedGraph":
        """Pack several host CSRs (synth.CSR) into one batched graph handle."""
        return BatchedGraph(self, graphs)

    def mlp(self, seed: int = 0) -> "Mlp":
        return Mlp(self, seed)

    def features(self, graph: "Graph", h: int, alive=None):
        """(X float32 [n, 8], lb, ub) for G(alive) (device tensors)."""
        torch = _torch()
        X = torch.empty((graph.n, 8), dtype=torch.float32, device=graph.device)
        lb = torch.empty(graph.n, dtype=torch.int32, device=graph.device)
        ub = torch.empty(graph.n, dtype=torch.int32, device=graph.device)
        self._check(self.lib.khc_features(self.handle, graph.handle, _dptr(alive), h, _dptr(X),
                                          _dptr(lb), _dptr(ub)))
        return X, lb, ub

    def core_approx(self, graph: "Graph", h: int, mlp=None, with_estimate: bool = False):
        torch = _torch()
        core = torch.empty(graph.n, dtype=torch.int32, device=graph.device)
        est = torch.empty(graph.n, dtype=torch.int32, device=graph.device) if with_estimate else None
        st = Stats()
        self._check(self.lib.khcore_decompose_approx(self.handle, graph.handle, h,
                                                     None if mlp is None else mlp.handle, _dptr(core),
                                                     _dptr(est), ctypes.byref(st)))
        return core, est, st.as_dict()

    def core_sampled(self, graph: "Graph", h: int, sampled, with_estimate: bool = False):
        """Sampling-based approximate core numbers on the vertex sample
        `sampled` (device uint8 mask): (core, estimate or None, stats)."""
        torch = _torch()
        core = torch.empty(graph.n, dtype=torch.int32, device=graph.device)
        est = torch.empty(graph.n, dtype=torch.int32, device=graph.device) if with_estimate else None
        st = Stats()
        self._check(self.lib.khcore_decompose_sampled(self.handle, graph.handle, h, _dptr(sampled), _dptr(core),
                                                      _dptr(est), ctypes.byref(st)))
        return core, est, st.as_dict()

    def gate_features(self, graph: "Graph", h: int, dm, alive=None):
        """Gate features X float32 [n, 8] of G(alive) from dm, the
        (h-1)-degrees or lower bounds on them (device tensor)."""
        torch = _torch()
        X = torch.empty((graph.n, 8), dtype=torch.float32, device=graph.device)
        self._check(self.lib.khc_gate_features(self.handle, graph.handle, _dptr(alive), h, _dptr(dm), _dptr(X)))
        return X

    def mlp_samples(self, graph: "Graph", h: int, alive=None, kind: int = 0):
        """(X float32 [m, 8], target float32 [m]) of the m live vertices of
        G(alive): features (kind 0 estimating mode, 1 gate) and
        log1p(d^h) / 8, computed and compacted on the device."""
        torch = _torch()
        X = torch.empty((graph.n, 8), dtype=torch.float32, device=graph.device)
        t = torch.empty(graph.n, dtype=torch.float32, device=graph.device)
        m = ctypes.c_uint32(0)
        self._check(self.lib.khc_mlp_samples(self.handle, graph.handle, _dptr(alive), h, int(kind), _dptr(X),
                                             _dptr(t), ctypes.byref(m)))
        return X[:m.value], t[:m.value]

    def alive_after(self, rnd, r0: int):
        """uint8 mask of the vertices whose removal round (device tensor) is >= r0."""
        torch = _torch()
        out = torch.empty(rnd.numel(), dtype=torch.uint8, device=rnd.device)
        self._check(self.lib.khc_alive_after(self.handle, rnd.numel(), _dptr(rnd), int(r0), _dptr(out)))
        return out

    def core_gated(self, graph: "Graph", h: int, mlp=None, margin: float = 0.0, with_round: bool = False):
        """Bounded-schedule decomposition with the learned recompute gate:
        (core, round or None, stats); mlp None gives the exact result."""
        torch = _torch()
        core = torch.empty(graph.n, dtype=torch.int32, device=graph.device)
        rnd = torch.empty(graph.n, dtype=torch.int32, device=graph.device) if with_round else None
        st = Stats()
        self._check(self.lib.khcore_decompose_gated(self.handle, graph.handle, h,
                                                    None if mlp is None else mlp.handle, float(margin),
                                                    _dptr(core), _dptr(rnd), ctypes.byref(st)))
        return core, rnd, st.as_dict()

    def validate(self, row_ptr, col, n: int) -> int:
        """Validate a device CSR; returns the status code (0 = ok)."""
        s = CSRStruct(n, int(row_ptr[-1].item()) if row_ptr.numel() else 0,
                      _dptr(row_ptr), _dptr(col))
        return self.lib.khc_validate_csr(self.handle, ctypes.byref(s))

    # ------------------------------------------------------------ compute
    def hdeg(self, graph: "Graph", h: int, alive=None, out=None):
        torch = _torch()
        if out is None:
            out = torch.empty(graph.n, dtype=torch.int32, device=graph.device)
        self._check(self.lib.khdeg_compute(self.handle, graph.handle, _dptr(alive), h, _dptr(out)))
        return out

    def hdeg_noalloc(self, graph: "Graph", h: int, alive=None, out=None):
        """khdeg_compute_noalloc: the library allocates nothing (out, if
        given, is the caller's)."""
        torch = _torch()
        if out is None:
            out = torch.empty(graph.n, dtype=torch.int32, device=graph.device)
        self._check(self.lib.khdeg_compute_noalloc(self.handle, graph.handle, _dptr(alive), h, _dptr(out)))
        return out

    def hdeg_list(self, graph: "Graph", h: int, verts, alive=None, out=None):
        torch = _torch()
        if out is None:
            out = torch.empty(verts.numel(), dtype=torch.int32, device=graph.device)
        self._check(self.lib.khdeg_compute_list(self.handle, graph.handle, _dptr(alive), h,
                                                _dptr(verts), verts.numel(), _dptr(out)))
        return out

    def scanned_arcs(self, graph: "Graph", h: int, alive=None, out=None):
        """Arcs a scalar bounded BFS from each vertex examines (int64)."""
        torch = _torch()
        if out is None:
            out = torch.empty(graph.n, dtype=torch.int64, device=graph.device)
        self._check(self.lib.khdeg_scanned_arcs(self.handle, graph.handle, _dptr(alive), h, _dptr(out)))
        return out

    def core(self, graph: "Graph", h: int, with_round: bool = False, core=None, rnd=None):
        torch = _torch()
        if core is None:
            core = torch.empty(graph.n, dtype=torch.int32, device=graph.device)
        if with_round and rnd is None:
            rnd = torch.empty(graph.n, dtype=torch.int32, device=graph.device)
        st = Stats()
        self._check(self.lib.khcore_decompose(self.handle, graph.handle, h, _dptr(core),
                                              _dptr(rnd) if with_round else None,
                                              ctypes.byref(st)))
        return core, (rnd if with_round else None), st.as_dict()


class Graph:
    """A device CSR plus the library's graph handle."""

    def __init__(self, ctx: Context, g, validate: bool = True):
        torch = _torch()
        self.ctx = ctx
        self.n = int(g.n)
        self.nnz = int(g.row_ptr[-1]) if len(g.row_ptr) else 0
        self.device = torch.device("cuda", ctx.device)
        self.row_ptr = torch.from_numpy(np.ascontiguousarray(g.row_ptr).view(np.int64)).to(self.device)
        col = np.ascontiguousarray(g.col, dtype=np.uint32)
        if col.size == 0:
            col = np.zeros(1, dtype=np.uint32)
        self.col = torch.from_numpy(col.view(np.int32)).to(self.device)
        s = CSRStruct(self.n, self.nnz, _dptr(self.row_ptr), _dptr(self.col))
        h = ctypes.c_void_p()
        ctx._check(ctx.lib.khc_graph_create(ctx.handle, ctypes.byref(s), ctypes.byref(h)))
        self.handle = h
        ctx._graphs.add(self)

    def close(self):
        if getattr(self, "handle", None):
            if getattr(self.ctx, "handle", None):
                self.ctx.lib.khc_graph_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class BatchedGraph(Graph):
    """Several graphs packed together: concatenated rows, graph-local column
    ids, vtx_base offsets; decomposed by one persistent kernel."""

    def __init__(self, ctx: Context, graphs):
        torch = _torch()
        self.ctx = ctx
        self.device = torch.device("cuda", ctx.device)
        ns = [int(g.n) for g in graphs]
        vb = np.zeros(len(graphs) + 1, dtype=np.uint64)
        np.cumsum(ns, out=vb[1:])
        arc_off = np.zeros(len(graphs) + 1, dtype=np.uint64)
        np.cumsum([int(g.row_ptr[-1]) for g in graphs], out=arc_off[1:])
        rp = np.concatenate([np.asarray(g.row_ptr[:-1], dtype=np.uint64) + arc_off[i]
                             for i, g in enumerate(graphs)] + [arc_off[-1:]])
        col = np.concatenate([np.asarray(g.col, dtype=np.uint32) for g in graphs])
        self.n = int(vb[-1])
        self.nnz = int(arc_off[-1])
        self.vtx_base_host = vb
        self.vtx_base = torch.from_numpy(vb.view(np.int64)).to(self.device)
        self.row_ptr = torch.from_numpy(rp.view(np.int64)).to(self.device)
        if col.size == 0:
            col = np.zeros(1, dtype=np.uint32)
        col_dev = torch.from_numpy(col.view(np.int32)).to(self.device)
        h = ctypes.c_void_p()
        ctx._check(ctx.lib.khc_graph_create_batched(ctx.handle, len(graphs), _dptr(self.vtx_base),
                                                    _dptr(self.row_ptr), _dptr(col_dev), self.nnz,
                                                    ctypes.byref(h)))
        del col_dev
        self.handle = h
        ctx._graphs.add(self)


class Mlp:
    """The learned-mode network (device parameters, Adam state)."""

    def __init__(self, ctx: Context, seed: int = 0):
        self.ctx = ctx
        h = ctypes.c_void_p()
        ctx._check(ctx.lib.khc_mlp_create(ctx.handle, seed, ctypes.byref(h)))
        self.handle = h

    def close(self):
        if getattr(self, "handle", None):
            if getattr(self.ctx, "handle", None):
                self.ctx.lib.khc_mlp_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def get(self):
        p = np.zeros(N_PARAMS, dtype=np.float32)
        g = np.zeros(N_PARAMS, dtype=np.float32)
        self.ctx._check(self.ctx.lib.khc_mlp_get_params(self.ctx.handle, self.handle,
                                                         p.ctypes.data_as(ctypes.c_void_p),
                                                         g.ctypes.data_as(ctypes.c_void_p)))
        return p, g

    def moments(self):
        """(m, v, step) of the Adam state."""
        m = np.zeros(N_PARAMS, dtype=np.float32)
        v = np.zeros(N_PARAMS, dtype=np.float32)
        step = ctypes.c_uint64()
        self.ctx._check(self.ctx.lib.khc_mlp_get_moments(self.ctx.handle, self.handle,
                                                          m.ctypes.data_as(ctypes.c_void_p),
                                                          v.ctypes.data_as(ctypes.c_void_p), ctypes.byref(step)))
        return m, v, int(step.value)

    def save(self, path: str):
        self.ctx._check(self.ctx.lib.khc_mlp_save(self.ctx.handle, self.handle, os.fsencode(path)))

    def load(self, path: str):
        self.ctx._check(self.ctx.lib.khc_mlp_load(self.ctx.handle, self.handle, os.fsencode(path)))

    def set(self, params):
        p = np.ascontiguousarray(params, dtype=np.float32)
        assert p.size == N_PARAMS
        self.ctx._check(self.ctx.lib.khc_mlp_set_params(self.ctx.handle, self.handle,
                                                         p.ctypes.data_as(ctypes.c_void_p)))

    def forward(self, X):
        torch = _torch()
        y = torch.empty(X.shape[0], dtype=torch.float32, device=X.device)
        self.ctx._check(self.ctx.lib.khc_mlp_forward(self.ctx.handle, self.handle, _dptr(X), X.shape[0],
                                                      _dptr(y)))
        return y

    def gradient(self, X, t):
        loss = ctypes.c_float()
        self.ctx._check(self.ctx.lib.khc_mlp_gradient(self.ctx.handle, self.handle, _dptr(X), _dptr(t),
                                                       X.shape[0], ctypes.byref(loss)))
        return loss.value

    def train(self, X, t, epochs: int, batch: int = 4096, lr: float = 1e-3, seed: int = 0):
        losses = np.zeros(epochs, dtype=np.float32)
        self.ctx._check(self.ctx.lib.khc_mlp_train(self.ctx.handle, self.handle, _dptr(X), _dptr(t),
                                                    X.shape[0], epochs, batch, lr, seed,
                                                    losses.ctypes.data_as(ctypes.c_void_p)))
        return losses

