"""Node-aware parallel SpMV (Bienz, Gropp, Olson, arXiv 1612.08060) on one
MI355X: Python binding of ``libnapspmv.so``.

This module only marshals arguments to the C ABI declared in
``include/napspmv.h``; every step of the plan build and of the apply runs in
the library (host C++ and gfx950 HIP kernels).  PyTorch is used only to pass
device memory and HIP streams.  If the library is not built, loading fails
loudly: there is no fallback.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

__all__ = ["Plan", "Graph", "Batch", "Server", "NapspmvError", "load_library", "LIB_PATH", "MODES",
           "DTYPES", "PHASES", "SOCKET_PHASES",
           "STAGE_LOCAL", "STAGE_REMOTE", "set_device_budget", "device_bytes_in_use"]

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libnapspmv.so")
MODES = {"standard": 0, "nap": 1}
DTYPES = {"f64": 0, "f32": 1, "bf16": 2}
PHASES = ("INTER", "L0", "L1", "L2")
SOCKET_PARTS = ("on", "gather", "cross", "scatter")
SOCKET_PHASES = tuple(f"{ph}_{part}" for ph in ("L0", "L1", "L2") for part in SOCKET_PARTS)
STAGE_LOCAL, STAGE_REMOTE = 0, 1
HOST_ONLY, EXCHANGE_COPY = 0x1, 0x2
VARIANTS = {"owner_map": 0x4, "split": 0x8, "dedup": 0x10, "three_way": 0x20,
            "direct": 0x80}
PARTITION_STRIDED = 0x40
PARAMS = {"block_nnz": 0, "gather_item": 1, "window": 2, "remote_nnz": 3}
_VAL_NP = {"f64": np.float64, "f32": np.float32, "bf16": np.uint16}
_ERRNAMES = {-1: "EINVAL", -2: "ENOMEM", -3: "EHIP", -4: "EUNSUPPORTED"}


class NapspmvError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"napspmv {_ERRNAMES.get(code, code)}: {msg}")
        self.code = code


class PhaseStats(ctypes.Structure):
    _fields_ = [(k, ctypes.c_int64) for k in (
        "msgs", "elems", "max_msgs_sent", "max_elems_sent", "max_msgs_recv",
        "max_elems_recv", "max_msg_elems")]


class Stats(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("nnz", ctypes.c_int64), ("n_p", ctypes.c_int64),
                ("ppn", ctypes.c_int64), ("n_nodes", ctypes.c_int64),
                ("mode", ctypes.c_int32), ("dtype", ctypes.c_int32),
                ("value_bytes", ctypes.c_int64), ("nnz_on", ctypes.c_int64),
                ("nnz_off", ctypes.c_int64), ("ghosts", ctypes.c_int64),
                ("phase", PhaseStats * 4), ("device_bytes", ctypes.c_int64),
                ("build_seconds", ctypes.c_double), ("upload_seconds", ctypes.c_double),
                ("flags", ctypes.c_uint32)]


_lib = None
P, I64, I32, U32 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int, ctypes.c_uint32
_SIGS = {
    "napspmv_plan_create": (I32, [P, P, P, I32, I64, I64, I64, I32, P, U32, P, P]),
    "napspmv_plan_create_sockets": (I32, [P, P, P, I32, I64, I64, I64, I64, P, U32, P, P]),
    "napspmv_plan_socket_stats": (I32, [P, P, P]),
    "napspmv_apply": (I32, [P, P, P, P]),
    "napspmv_apply_stage": (I32, [P, I32, P, P, P]),
    "napspmv_plan_stats": (I32, [P, P]),
    "napspmv_plan_rows": (I32, [P, P]),
    "napspmv_plan_block_kinds": (I32, [P, P]),
    "napspmv_plan_level_stats": (I32, [P, I64, P]),
    "napspmv_plan_export": (I32, [P, I32, P, P, P, P, P, P]),
    "napspmv_plan_ghosts": (I32, [P, P, P]),
    "napspmv_plan_read_ghost_values": (I32, [P, P, P, P]),
    "napspmv_plan_workspace_bytes": (I64, [P]),
    "napspmv_apply_ws": (I32, [P, P, P, P, P]),
    "napspmv_apply_noalloc": (I32, [P, P, P, P]),
    "napspmv_noalloc_max_workspace_bytes": (I64, []),
    "napspmv_batch_create": (I32, [I32, P]),
    "napspmv_batch_apply": (I32, [P, I32, P, P, P, P, P]),
    "napspmv_batch_destroy": (I32, [P]),
    "napspmv_plan_prepare_partitions": (I32, [P]),
    "napspmv_apply_partition": (I32, [P, I64, P, P, P]),
    "napspmv_graph_create": (I32, [P, P, P, P]),
    "napspmv_graph_launch": (I32, [P, P]),
    "napspmv_graph_destroy": (I32, [P]),
    "napspmv_plan_autotune": (I32, [P, P, P, P, I32, ctypes.c_char_p, P]),
    "napspmv_server_create": (I32, [I32, I32, I64, P]),
    "napspmv_server_add_plan": (I32, [P, P, P]),
    "napspmv_server_reserve": (I32, [P, I32]),
    "napspmv_server_submit": (I32, [P, I32, P, P, P, P]),
    "napspmv_server_poll": (I64, [P]),
    "napspmv_server_wait": (I32, [P, I64]),
    "napspmv_server_request_info": (I32, [P, I64, P, P, P]),
    "napspmv_server_replay": (I32, [P, I64, P, P, P, P, P, P, P]),
    "napspmv_server_workspace_bytes": (I64, [P]),
    "napspmv_server_last_error": (ctypes.c_char_p, []),
    "napspmv_server_destroy": (I32, [P]),
    "napspmv_plan_set_param": (I32, [P, I32, I32]),
    "napspmv_plan_get_param": (I32, [P, I32]),
    "napspmv_plan_destroy": (I32, [P]),
    "napspmv_set_device_budget": (I32, [I64]),
    "napspmv_device_bytes_in_use": (I64, []),
    "napspmv_last_error": (ctypes.c_char_p, []),
    "napspmv_version": (I32, []),
}


def load_library(path: str = LIB_PATH):
    """Load libnapspmv.so (once).  Raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(path):
            raise RuntimeError(
                f"{path} is missing: build it first (python -m paper_1612_08060_amd.build "
                "or __graft_entry__.build()); there is no fallback path")
        lib = ctypes.CDLL(path)
        for name, (res, args) in _SIGS.items():
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _lib = lib
    return _lib


def _check(rc: int):
    if rc != 0:
        raise NapspmvError(rc, load_library().napspmv_last_error().decode())


def set_device_budget(nbytes: int):
    _check(load_library().napspmv_set_device_budget(int(nbytes)))


def device_bytes_in_use() -> int:
    return int(load_library().napspmv_device_bytes_in_use())


def _stream_handle(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


class Plan:
    """A communication plan plus the split matrix on the GPU.

    ``rowptr`` (int64, n+1), ``col`` (int32) and ``val`` (float64 for "f64",
    float32 for "f32", uint16 bfloat16 bits for "bf16") describe A in CSR.
    ``mode`` is "standard" or "nap".  ``host_only`` builds the plan on the
    host without touching a GPU (stats and exports only).  ``variant`` names
    NAP plan variants ("owner_map", "split", "dedup"; section 4.1): they
    change the messages, not the result; "three_way" sums each row in the
    three parts of algorithm NAPSpMV (on_process, on_node, off_node) with the
    inter-node hop overlapped with the on_node product.  ``strided`` puts
    row r on process r mod n_p (section 5); the plan, its exports and v, w
    are then in process-major order (see ``rows``).  ``sockets`` (NAP mode,
    no variant) adds a third hierarchy level of that many consecutive ranks
    per socket (napspmv_plan_create_sockets): phases "L0_on" ... "L2_scatter"
    and ``socket_stats``.
    """

    def __init__(self, rowptr, col, val, n: int, n_p: int, ppn: int, mode: str = "standard",
                 dtype: str = "f64", row_starts=None, host_only: bool = False,
                 exchange_copy: bool = False, variant=(), strided: bool = False,
                 sockets: int = 0):
        lib = load_library()
        unknown = set(variant) - set(VARIANTS)
        if unknown:
            raise ValueError(f"unknown variant(s) {sorted(unknown)}; known: {sorted(VARIANTS)}")
        if mode not in MODES:
            raise ValueError(f"mode must be one of {list(MODES)}")
        if dtype not in DTYPES:
            raise ValueError(f"dtype must be one of {list(DTYPES)}")
        self._rowptr = np.ascontiguousarray(rowptr, dtype=np.int64)
        self._col = np.ascontiguousarray(col, dtype=np.int32)
        v = np.asarray(val)
        if v.dtype != _VAL_NP[dtype]:
            raise TypeError(f"val must be {np.dtype(_VAL_NP[dtype]).name} for dtype {dtype!r} "
                            "(the library never rounds values)")
        self._val = np.ascontiguousarray(v)
        self._starts = None if row_starts is None else np.ascontiguousarray(row_starts, np.int64)
        self.n, self.n_p, self.ppn, self.mode, self.dtype = int(n), int(n_p), int(ppn), mode, dtype
        self.host_only = bool(host_only)
        flags = (HOST_ONLY if host_only else 0) | (EXCHANGE_COPY if exchange_copy else 0)
        for name in variant:
            flags |= VARIANTS[name]
        if strided:
            flags |= PARTITION_STRIDED
        self.strided = bool(strided)
        self.variant = tuple(sorted(set(variant)))
        handle = ctypes.c_void_p()
        st = Stats()
        self._h = None
        self.sockets = int(sockets)
        starts = None if self._starts is None else self._starts.ctypes.data
        if self.sockets:
            if mode != "nap":
                raise ValueError("a socket level needs mode='nap'")
            rc = lib.napspmv_plan_create_sockets(
                self._rowptr.ctypes.data, self._col.ctypes.data, self._val.ctypes.data,
                DTYPES[dtype], self.n, self.n_p, self.ppn, self.sockets, starts, flags,
                ctypes.byref(handle), ctypes.byref(st))
        else:
            rc = lib.napspmv_plan_create(
                self._rowptr.ctypes.data, self._col.ctypes.data, self._val.ctypes.data,
                DTYPES[dtype], self.n, self.n_p, self.ppn, MODES[mode], starts, flags,
                ctypes.byref(handle), ctypes.byref(st))
        _check(rc)
        self._h = handle
        # the plan has copied everything it needs
        self._rowptr = self._col = self._val = None

    # -- plan data -------------------------------------------------------
    @property
    def stats(self) -> dict:
        st = Stats()
        _check(load_library().napspmv_plan_stats(self._h, ctypes.byref(st)))
        out = {k: getattr(st, k) for k, _ in Stats._fields_ if k != "phase"}
        out["mode"] = {v: k for k, v in MODES.items()}[out["mode"]]
        out["dtype"] = {v: k for k, v in DTYPES.items()}[out["dtype"]]
        out["phases"] = {PHASES[i]: {k: getattr(st.phase[i], k) for k, _ in PhaseStats._fields_}
                         for i in range(4)}
        return out

    def export(self, phase: str):
        """(src int32, dst int32, ptr int64, idx int32) of a phase (a name of
        PHASES, or of SOCKET_PHASES for a plan with a socket level), canonical."""
        lib = load_library()
        ph = PHASES.index(phase) if phase in PHASES else 4 + SOCKET_PHASES.index(phase)
        nm, ni = ctypes.c_int64(), ctypes.c_int64()
        _check(lib.napspmv_plan_export(self._h, ph, ctypes.byref(nm), ctypes.byref(ni),
                                       None, None, None, None))
        src = np.empty(nm.value, np.int32)
        dst = np.empty(nm.value, np.int32)
        ptr = np.empty(nm.value + 1, np.int64)
        idx = np.empty(ni.value, np.int32)
        _check(lib.napspmv_plan_export(self._h, ph, None, None, src.ctypes.data,
                                       dst.ctypes.data, ptr.ctypes.data, idx.ctypes.data))
        return src, dst, ptr, idx

    def socket_stats(self) -> dict:
        """Statistics of the socket-level phases (plans built with ``sockets``)."""
        out = (PhaseStats * 12)()
        pps = ctypes.c_int64()
        _check(load_library().napspmv_plan_socket_stats(self._h, ctypes.byref(pps), out))
        return {name: {k: getattr(out[i], k) for k, _ in PhaseStats._fields_}
                for i, name in enumerate(SOCKET_PHASES)}

    def level_stats(self, procs_per_socket: int) -> dict:
        """Per phase, statistics of its on-socket and off-socket messages
        (sockets of ``procs_per_socket`` consecutive ranks)."""
        out = (PhaseStats * 8)()
        _check(load_library().napspmv_plan_level_stats(self._h, int(procs_per_socket), out))
        return {PHASES[ph]: {side: {k: getattr(out[2 * ph + i], k) for k, _ in PhaseStats._fields_}
                             for i, side in enumerate(("on_socket", "off_socket"))}
                for ph in range(4)}

    def rows(self) -> np.ndarray:
        """Original row index of every position of the plan's numbering."""
        out = np.empty(self.n, np.int64)
        _check(load_library().napspmv_plan_rows(self._h, out.ctypes.data))
        return out

    def block_kinds(self) -> dict:
        """Counts of the off-process row blocks by layout: plain, packed,
        narrow (device plans)."""
        out = np.zeros(3, np.int64)
        _check(load_library().napspmv_plan_block_kinds(self._h, out.ctypes.data))
        return {"plain": int(out[0]), "packed": int(out[1]), "narrow": int(out[2])}

    def ghosts(self):
        """(ghost_ptr int64[n_p+1], ghost_col int32[G])."""
        gp = np.empty(self.n_p + 1, np.int64)
        _check(load_library().napspmv_plan_ghosts(self._h, gp.ctypes.data, None))
        gc = np.empty(int(gp[-1]), np.int32)
        _check(load_library().napspmv_plan_ghosts(self._h, None, gc.ctypes.data))
        return gp, gc

    def set_param(self, name: str, value: int):
        """Tuning parameter (a key of PARAMS); -1 = automatic."""
        _check(load_library().napspmv_plan_set_param(self._h, PARAMS[name], int(value)))

    def get_param(self, name: str) -> int:
        r = load_library().napspmv_plan_get_param(self._h, PARAMS[name])
        if r < 0:
            _check(r)
        return r

    # -- apply -----------------------------------------------------------
    def _vec_check(self, t, name):
        import torch
        want = torch.float64 if self.dtype == "f64" else torch.float32
        if not isinstance(t, torch.Tensor) or not t.is_cuda:
            raise TypeError(f"{name} must be a CUDA (HIP) tensor")
        if t.dtype != want or t.numel() != self.n or not t.is_contiguous():
            raise ValueError(f"{name} must be a contiguous {want} tensor of {self.n} elements")
        return ctypes.c_void_p(t.data_ptr())

    def apply(self, v, w, stream=None):
        """w = A v on the GPU (asynchronous on ``stream``, default: current)."""
        _check(load_library().napspmv_apply(self._h, self._vec_check(v, "v"),
                                            self._vec_check(w, "w"), _stream_handle(stream)))
        return w

    def apply_stage(self, stage: int, v, w, stream=None):
        _check(load_library().napspmv_apply_stage(self._h, int(stage), self._vec_check(v, "v"),
                                                  self._vec_check(w, "w"),
                                                  _stream_handle(stream)))

    def read_ghosts(self, stream=None, ws=None) -> np.ndarray:
        """The ghost buffer after the last exchange (synchronizes)."""
        g = int(self.stats["ghosts"])
        out = np.empty(g, np.float64 if self.dtype == "f64" else np.float32)
        _check(load_library().napspmv_plan_read_ghost_values(
            self._h, None if ws is None else ctypes.c_void_p(ws.data_ptr()), out.ctypes.data,
            _stream_handle(stream)))
        return out

    @property
    def workspace_bytes(self) -> int:
        r = load_library().napspmv_plan_workspace_bytes(self._h)
        if r < 0:
            _check(r)
        return int(r)

    def new_workspace(self):
        """A caller-owned workspace tensor (uint8, 256-byte aligned) for apply(ws=...)."""
        import torch
        nbytes = max(self.workspace_bytes, 1)
        t = torch.empty(nbytes + 256, dtype=torch.uint8, device="cuda")
        off = (-t.data_ptr()) % 256
        return t[off:off + nbytes]

    def apply_ws(self, ws, v, w, stream=None):
        """w = A v using a caller-owned workspace (see new_workspace)."""
        _check(load_library().napspmv_apply_ws(
            self._h, ctypes.c_void_p(ws.data_ptr()), self._vec_check(v, "v"),
            self._vec_check(w, "w"), _stream_handle(stream)))
        return w

    def apply_noalloc(self, v, w, stream=None):
        """w = A v with the library's static workspace (allocates nothing;
        see napspmv_apply_noalloc)."""
        _check(load_library().napspmv_apply_noalloc(self._h, self._vec_check(v, "v"),
                                                    self._vec_check(w, "w"),
                                                    _stream_handle(stream)))
        return w

    def prepare_partitions(self):
        _check(load_library().napspmv_plan_prepare_partitions(self._h))

    def apply_partition(self, part: int, v, w, stream=None):
        """The rows of one process only (standard plans; prepare_partitions first)."""
        _check(load_library().napspmv_apply_partition(self._h, int(part), self._vec_check(v, "v"),
                                                      self._vec_check(w, "w"),
                                                      _stream_handle(stream)))

    def graph(self, v, w):
        """A replayable HIP graph of apply(v, w) (see Graph)."""
        return Graph(self, v, w)

    def autotune(self, v, w, stream=None, reps: int = 5, cache_path=None) -> float:
        """Pick the fastest tuning for this plan (see napspmv_plan_autotune)."""
        best = ctypes.c_double()
        _check(load_library().napspmv_plan_autotune(
            self._h, self._vec_check(v, "v"), self._vec_check(w, "w"), _stream_handle(stream),
            int(reps), None if cache_path is None else str(cache_path).encode(),
            ctypes.byref(best)))
        return best.value

    def close(self):
        if getattr(self, "_h", None) is not None:
            load_library().napspmv_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


class Graph:
    """A HIP graph replaying one apply of a plan on fixed vectors."""

    def __init__(self, plan: Plan, v, w):
        self.plan = plan
        self._v, self._w = v, w            # keep the vectors alive
        h = ctypes.c_void_p()
        _check(load_library().napspmv_graph_create(plan._h, plan._vec_check(v, "v"),
                                                   plan._vec_check(w, "w"), ctypes.byref(h)))
        self._h = h

    def launch(self, stream=None):
        _check(load_library().napspmv_graph_launch(self._h, _stream_handle(stream)))

    def close(self):
        if getattr(self, "_h", None) is not None:
            load_library().napspmv_graph_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Batch:
    """Batched applies over many plans in one launch sequence
    (napspmv_batch_apply); one Batch per stream."""

    def __init__(self, max_count: int):
        h = ctypes.c_void_p()
        _check(load_library().napspmv_batch_create(int(max_count), ctypes.byref(h)))
        self._h = h
        self.max_count = int(max_count)

    def apply(self, plans, vs, ws_out, workspaces=None, stream=None):
        n = len(plans)
        P_ = ctypes.c_void_p * n
        hp = P_(*[p._h.value for p in plans])
        hv = P_(*[p._vec_check(v, "v").value for p, v in zip(plans, vs)])
        hw = P_(*[p._vec_check(w, "w").value for p, w in zip(plans, ws_out)])
        hws = None
        if workspaces is not None:
            hws = P_(*[None if x is None else x.data_ptr() for x in workspaces])
        _check(load_library().napspmv_batch_apply(self._h, n, hp, hws, hv, hw,
                                                  _stream_handle(stream)))

    def close(self):
        if getattr(self, "_h", None) is not None:
            load_library().napspmv_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _scheck(rc: int):
    if rc < 0:
        raise NapspmvError(int(rc), load_library().napspmv_server_last_error().decode())


class Server:
    """The serving engine (napspmv_server_*): resident plans, slots on their
    own streams, workspace budget, continuous batching."""

    def __init__(self, slots: int = 4, max_batch: int = 16, workspace_budget: int = 0):
        h = ctypes.c_void_p()
        _scheck(load_library().napspmv_server_create(int(slots), int(max_batch),
                                                     int(workspace_budget), ctypes.byref(h)))
        self._h = h
        self.plans = []

    def add(self, plan: Plan) -> int:
        i = ctypes.c_int()
        _scheck(load_library().napspmv_server_add_plan(self._h, plan._h, ctypes.byref(i)))
        self.plans.append(plan)
        return i.value

    def reserve(self, per_plan: int):
        """Pre-allocate up to ``per_plan`` workspaces of every resident plan."""
        _scheck(load_library().napspmv_server_reserve(self._h, int(per_plan)))

    def submit(self, pid: int, v, w, stream=None) -> int:
        """Queue w = A_pid v after the work issued so far on ``stream``
        (default: the current stream); returns a ticket."""
        p = self.plans[pid]
        t = ctypes.c_int64()
        _scheck(load_library().napspmv_server_submit(self._h, int(pid), p._vec_check(v, "v"),
                                                     p._vec_check(w, "w"), _stream_handle(stream),
                                                     ctypes.byref(t)))
        return t.value

    def poll(self) -> int:
        r = load_library().napspmv_server_poll(self._h)
        _scheck(r)
        return int(r)

    def wait(self, ticket: int):
        _scheck(load_library().napspmv_server_wait(self._h, int(ticket)))

    def info(self, ticket: int):
        s, d, b = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int()
        _scheck(load_library().napspmv_server_request_info(self._h, int(ticket), ctypes.byref(s),
                                                           ctypes.byref(d), ctypes.byref(b)))
        return s.value, d.value, b.value

    def replay(self, ids, arrival_ns, vs, ws_out, stream=None):
        """Replay an arrival trace natively, after the work issued so far on
        ``stream`` (default: the current stream); returns (latency_ns,
        batch_sizes)."""
        n = len(ids)
        ids_a = np.ascontiguousarray(ids, dtype=np.int32)
        arr = np.ascontiguousarray(arrival_ns, dtype=np.int64)
        P_ = ctypes.c_void_p * n
        hv = P_(*[self.plans[i]._vec_check(v, "v").value for i, v in zip(ids, vs)])
        hw = P_(*[self.plans[i]._vec_check(w, "w").value for i, w in zip(ids, ws_out)])
        lat = np.empty(n, np.int64)
        bs = np.empty(n, np.int32)
        _scheck(load_library().napspmv_server_replay(self._h, n, ids_a.ctypes.data, arr.ctypes.data,
                                                     hv, hw, _stream_handle(stream), lat.ctypes.data,
                                                     bs.ctypes.data))
        return lat, bs

    @property
    def workspace_bytes(self) -> int:
        return int(load_library().napspmv_server_workspace_bytes(self._h))

    def close(self):
        if getattr(self, "_h", None) is not None:
            load_library().napspmv_server_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
