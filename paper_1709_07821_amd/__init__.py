"""Python binding of libroaring_gpu.so - Roaring-bitmap set operations on
MI355X (gfx950). Argument marshalling only: every step of every operation
runs in the library's HIP kernels. torch supplies device memory and streams.

The C names are kept: ``roaring_and/or/xor/andnot``, their
``_cardinality`` forms, ``roaring_jaccard`` and ``roaring_batch``, plus pool
construction (``Pool.from_sets``, ``Pool.from_dense_words``) and the pool
utilities ``rg_pool_recount/validate/digest``.

There is no CPU fallback: if the HIP library is missing, importing the
binding's entry points raises.
"""
from __future__ import annotations

import ctypes
import weakref
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libroaring_gpu.so")

RG_OK, RG_EINVAL, RG_ECAPACITY, RG_EDEVICE, RG_EFORMAT, RG_ENOTSUP = 0, -1, -2, -3, -4, -5
RG_ARRAY, RG_BITSET, RG_RUN = 1, 2, 3
RG_AND, RG_OR, RG_XOR, RG_ANDNOT = 0, 1, 2, 3
OPS = {"and": RG_AND, "or": RG_OR, "xor": RG_XOR, "andnot": RG_ANDNOT}
RG_FLAG_MATERIALIZE, RG_FLAG_CARD, RG_FLAG_JACCARD, RG_FLAG_DIGEST = 1, 2, 4, 8
RG_RULES_P1 = 1
RG_KEY_INDEX_BYTES = 10240
RG_DISPATCH_HEURISTIC, RG_DISPATCH_MLP, RG_DISPATCH_FIXED = 0, 1, 2
RG_MLP_PARAMS, RG_MLP_TABLE = 5382, 374544
VARIANTS = {"generic": 2, "merge": 3, "gallop": 4, "probe": 5, "runmerge": 6, "thread": 7}

# every symbol the C header declares
EXPORTS = ["rg_create", "rg_destroy", "rg_last_error", "rg_set_dispatch", "rg_set_thresholds", "roaring_and", "roaring_or", "roaring_xor",
           "roaring_andnot", "roaring_and_cardinality", "roaring_or_cardinality", "roaring_xor_cardinality",
           "roaring_andnot_cardinality", "roaring_jaccard", "roaring_batch", "rg_pool_measure_host",
           "rg_pool_build_host", "rg_pool_recount", "rg_pool_pack_meta", "rg_pool_validate", "rg_pool_digest",
           "rg_profile_enable",
           "rg_profile_reset", "rg_profile_read", "rg_plan_create", "rg_plan_execute", "rg_plan_capture",
           "rg_plan_tune", "rg_plan_set", "rg_plan_info", "rg_plan_destroy", "roaring_multi", "rg_serve_start",
           "rg_serve_submit", "rg_serve_poll", "rg_serve_release", "rg_serve_replay", "rg_serve_stop",
           "rg_mlp_forward", "rg_mlp_grad", "rg_mlp_adam", "rg_dispatch_sample", "rg_dispatch_train",
           "rg_dispatch_set_mlp", "rg_dispatch_table", "rg_sync", "rg_set_workspace", "rg_workspace_size",
           "roaring_jaccard_host", "rg_pool_init_dense", "roaring_batch_static",
           "roaring_contains", "roaring_to_uint32", "rg_pool_check", "rg_pool_canonicalize",
           "rg_plan_create_mat", "rg_plan_result", "rg_plan_totals", "rg_set_wave_slots",
           "rg_mpool_create", "rg_mpool_destroy", "rg_mpool_op", "rg_mpool_assign", "rg_mpool_clear",
           "rg_mpool_cards", "rg_mpool_status", "rg_mpool_export", "rg_pool_key_index", "rg_mpool_op_batch"]


class RoaringError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"status {status}: {msg}")
        self.status = status


class rg_pool(ctypes.Structure):
    _fields_ = [("n_bitmaps", ctypes.c_uint32), ("n_containers", ctypes.c_uint64),
                ("payload_bytes", ctypes.c_uint64), ("bm_begin", ctypes.c_void_p), ("keys", ctypes.c_void_p),
                ("types", ctypes.c_void_p), ("card", ctypes.c_void_p), ("size", ctypes.c_void_p),
                ("off", ctypes.c_void_p), ("payload", ctypes.c_void_p), ("bm_card", ctypes.c_void_p),
                ("bm_wbytes", ctypes.c_void_p), ("meta", ctypes.c_void_p), ("key_index", ctypes.c_void_p)]


class rg_out(ctypes.Structure):
    _fields_ = [("cap_containers", ctypes.c_uint64), ("cap_payload_bytes", ctypes.c_uint64),
                ("bm_begin", ctypes.c_void_p), ("keys", ctypes.c_void_p), ("types", ctypes.c_void_p),
                ("card", ctypes.c_void_p), ("size", ctypes.c_void_p), ("off", ctypes.c_void_p),
                ("payload", ctypes.c_void_p), ("bm_card", ctypes.c_void_p), ("bm_wbytes", ctypes.c_void_p),
                ("needed_containers", ctypes.c_uint64), ("needed_payload_bytes", ctypes.c_uint64),
                ("n_containers", ctypes.c_uint64), ("payload_used", ctypes.c_uint64)]


class rg_query(ctypes.Structure):
    _fields_ = [("op", ctypes.c_int), ("k", ctypes.c_uint32), ("ids", ctypes.POINTER(ctypes.c_uint32)),
                ("flags", ctypes.c_uint32)]


class rg_result(ctypes.Structure):
    _fields_ = [("done", ctypes.c_int), ("status", ctypes.c_int), ("card", ctypes.c_uint64),
                ("digest", ctypes.c_uint64), ("n_containers", ctypes.c_uint64), ("latency_ns", ctypes.c_uint64),
                ("view", rg_pool)]


class rg_serve_stats(ctypes.Structure):
    _fields_ = [("queries", ctypes.c_uint64), ("steps", ctypes.c_uint64), ("mean_batch", ctypes.c_double),
                ("arena_peak_bytes", ctypes.c_uint64), ("deferred", ctypes.c_uint64)]


_lib = None


def lib():
    """The loaded HIP library (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with __graft_entry__.build() "
                              "(there is no CPU fallback)")
        L = ctypes.CDLL(LIB_PATH)
        P, V, U32, U64, I = ctypes.POINTER, ctypes.c_void_p, ctypes.c_uint32, ctypes.c_uint64, ctypes.c_int
        pool_p, out_p = P(rg_pool), P(rg_out)
        L.rg_create.argtypes = [P(V), I]
        L.rg_destroy.argtypes = [V]
        L.rg_destroy.restype = None
        L.rg_last_error.argtypes = [V]
        L.rg_last_error.restype = ctypes.c_char_p
        L.rg_set_dispatch.argtypes = [V, I, I]
        L.rg_set_thresholds.argtypes = [V, U32, U32]
        for nm in ("roaring_and", "roaring_or", "roaring_xor", "roaring_andnot"):
            getattr(L, nm).argtypes = [V, pool_p, U32, pool_p, U32, out_p, V]
        for nm in ("roaring_and_cardinality", "roaring_or_cardinality", "roaring_xor_cardinality",
                   "roaring_andnot_cardinality", "roaring_jaccard"):
            getattr(L, nm).argtypes = [V, pool_p, U32, pool_p, U32, V, V]
        L.roaring_batch.argtypes = [V, I, pool_p, pool_p, V, V, U64, U32, out_p, V, V, V]
        L.rg_pool_measure_host.argtypes = [V, V, U32, P(U64), P(U64)]
        L.rg_pool_build_host.argtypes = [V, V, U32] + [V] * 9
        L.rg_pool_recount.argtypes = [V, pool_p, V]
        L.rg_pool_pack_meta.argtypes = [V, pool_p, V, V]
        L.rg_pool_validate.argtypes = [V, pool_p, P(U64), V]
        L.rg_pool_digest.argtypes = [V, pool_p, V, V]
        L.rg_profile_enable.argtypes = [V, I]
        L.rg_profile_reset.argtypes = [V]
        L.rg_profile_read.argtypes = [V, I, I, P(ctypes.c_double), P(U64), P(U64)]
        L.rg_plan_create.argtypes = [V, I, pool_p, pool_p, V, V, U64, U32, V, V, P(V), V]
        L.rg_plan_execute.argtypes = [V, V]
        L.rg_plan_capture.argtypes = [V, V]
        L.rg_plan_tune.argtypes = [V, V, I]
        L.rg_plan_set.argtypes = [V, U32, U32, U32]
        L.rg_plan_info.argtypes = [V, P(U32), P(U32), P(U32), P(U64), P(U32), P(I)]
        L.rg_plan_destroy.argtypes = [V]
        L.rg_plan_destroy.restype = None
        L.roaring_multi.argtypes = [V, I, pool_p, V, U32, U32, out_p, V, V]
        L.rg_serve_start.argtypes = [V, pool_p, U64, U32, U32, P(V)]
        L.rg_serve_submit.argtypes = [V, P(rg_query), U64, P(U64)]
        L.rg_serve_poll.argtypes = [V, U64, I, P(rg_result)]
        L.rg_serve_release.argtypes = [V, U64]
        L.rg_serve_replay.argtypes = [V, U64, P(rg_query), V, V, V, V]
        L.rg_serve_stop.argtypes = [V, P(rg_serve_stats)]
        L.rg_mlp_forward.argtypes = [V, V, V, U64, V, V]
        L.rg_mlp_grad.argtypes = [V, V, V, V, V, U64, V, V, V]
        L.rg_mlp_adam.argtypes = [V, V, V, V, V, U32, ctypes.c_float, V]
        L.rg_dispatch_sample.argtypes = [V, pool_p, pool_p, V, V, U64, I, V, V, V, U64, P(U64), V]
        L.rg_dispatch_train.argtypes = [V, V, V, V, U64, U32, U32, ctypes.c_float, U64, V, V, V]
        L.rg_dispatch_set_mlp.argtypes = [V, V, V]
        L.rg_dispatch_table.argtypes = [V, V, U64]
        L.rg_sync.argtypes = [V, V]
        L.rg_set_workspace.argtypes = [V, V, U64]
        L.rg_workspace_size.argtypes = [V, I, U32, pool_p, pool_p, U64, P(U64)]
        L.roaring_jaccard_host.argtypes = [V, pool_p, U32, pool_p, U32, P(ctypes.c_double), V]
        L.rg_pool_init_dense.argtypes = [V, pool_p, U32, V]
        L.roaring_batch_static.argtypes = [V, I, pool_p, pool_p, V, V, U64, U32, V, V, V]
        L.roaring_contains.argtypes = [V, pool_p, V, V, U64, V, V]
        L.rg_pool_check.argtypes = [V, pool_p, U32, P(U64), V]
        L.rg_pool_canonicalize.argtypes = [V, pool_p, out_p, V]
        L.rg_plan_create_mat.argtypes = [V, I, pool_p, pool_p, V, V, U64, U32, out_p, V, V, P(V), V]
        L.rg_plan_result.argtypes = [V, P(U64), P(U64), V]
        L.rg_plan_totals.argtypes = [V, P(V)]
        L.rg_set_wave_slots.argtypes = [V, U64]
        L.rg_mpool_create.argtypes = [V, U32, U32, P(V)]
        L.rg_mpool_destroy.argtypes = [V]
        L.rg_mpool_destroy.restype = None
        L.rg_mpool_op.argtypes = [V, I, U32, pool_p, U32, V]
        L.rg_mpool_op_batch.argtypes = [V, U32, V, V, pool_p, V, V]
        L.rg_mpool_assign.argtypes = [V, U32, pool_p, U32, V]
        L.rg_mpool_clear.argtypes = [V, U32, V]
        L.rg_mpool_cards.argtypes = [V, V, V]
        L.rg_mpool_status.argtypes = [V, P(U32), V]
        L.rg_mpool_export.argtypes = [V, U32, U32, out_p, V]
        L.rg_pool_key_index.argtypes = [V, pool_p, V, V]
        L.roaring_to_uint32.argtypes = [V, pool_p, U32, U32, V, V, U64, P(U64), V]
        for nm in EXPORTS:
            if nm not in ("rg_destroy", "rg_last_error", "rg_plan_destroy", "rg_mpool_destroy"):
                getattr(L, nm).restype = ctypes.c_int
        _lib = L
    return _lib


def _torch():
    import torch

    return torch


def _stream(stream=None):
    torch = _torch()
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


class Context:
    """Owns an rg_ctx (workspace, pinned staging) on one device."""

    def __init__(self, device: int = 0):
        h = ctypes.c_void_p()
        st = lib().rg_create(ctypes.byref(h), device)
        if st != RG_OK:
            raise RoaringError(st, f"rg_create failed on device {device}")
        self.h = h
        self.device = device
        self.dispatch_mode = RG_DISPATCH_HEURISTIC  # mirrors the context's variant selection
        self.servers = weakref.WeakSet()  # stopped before the context goes away

    def close(self):
        for srv in list(getattr(self, "servers", ())):
            try:
                srv.stop()
            except Exception:
                pass
        if self.h:
            lib().rg_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def check(self, st):
        if st != RG_OK:
            raise RoaringError(st, lib().rg_last_error(self.h).decode())
        return st

    def set_dispatch(self, mode: int = RG_DISPATCH_HEURISTIC, variant: int = 2):
        self.check(lib().rg_set_dispatch(self.h, mode, variant))
        self.dispatch_mode = mode

    def set_thresholds(self, gallop_ratio: int = 64, thread_max: int = 8):
        self.check(lib().rg_set_thresholds(self.h, gallop_ratio, thread_max))

    def sync(self, stream=None):
        """rg_sync: waits for the stream; raises what asynchronous calls found on the device."""
        self.check(lib().rg_sync(self.h, _stream(stream)))

    def set_wave_slots(self, n: int):
        """rg_set_wave_slots: most candidate slots per wave (results never change)."""
        self.check(lib().rg_set_wave_slots(self.h, n))

    def set_workspace(self, buf=None):
        """rg_set_workspace over a device tensor (256-byte aligned; None: the context's own).
        The context keeps a reference so the memory outlives the calls using it."""
        if buf is None:
            self.check(lib().rg_set_workspace(self.h, None, 0))
        else:
            self.check(lib().rg_set_workspace(self.h, _ptr(buf), buf.numel() * buf.element_size()))
        self.workspace = buf

    def workspace_size(self, op, flags: int, A: "Pool", B: "Pool", n_pairs: int) -> int:
        op = OPS[op] if isinstance(op, str) else op
        b = ctypes.c_uint64()
        self.check(lib().rg_workspace_size(self.h, op, flags, ctypes.byref(A.c), ctypes.byref(B.c), n_pairs,
                                           ctypes.byref(b)))
        return int(b.value)


class Pool:
    """A pool of bitmaps in device memory (torch tensors) and its rg_pool view."""

    def __init__(self, n_bitmaps, n_containers, payload_bytes, bm_begin, keys, types, card, size, off, payload,
                 bm_card, bm_wbytes):
        self.n_bitmaps = int(n_bitmaps)
        self.n_containers = int(n_containers)
        self.payload_bytes = int(payload_bytes)
        self.bm_begin, self.keys, self.types, self.card = bm_begin, keys, types, card
        self.size, self.off, self.payload, self.bm_card, self.bm_wbytes = size, off, payload, bm_card, bm_wbytes
        self._c = rg_pool(self.n_bitmaps, self.n_containers, self.payload_bytes, _ptr(bm_begin).value,
                          _ptr(keys).value, _ptr(types).value, _ptr(card).value, _ptr(size).value, _ptr(off).value,
                          _ptr(payload).value, _ptr(bm_card).value, _ptr(bm_wbytes).value)

    @property
    def c(self):
        return self._c

    def pack_meta(self, ctx: "Context", stream=None):
        """rg_pool_pack_meta into a tensor this pool keeps; sets the pool's meta.
        The pool must not change afterwards (the records mirror its arrays)."""
        torch = _torch()
        dev = self.bm_begin.device if self.bm_begin is not None else torch.device("cuda")
        self.meta = torch.empty(max(self.n_containers, 1) * 4, dtype=torch.int32, device=dev)
        ctx.check(lib().rg_pool_pack_meta(ctx.h, ctypes.byref(self._c), _ptr(self.meta), _stream(stream)))
        self._c.meta = _ptr(self.meta).value
        return self

    def key_index(self, ctx: "Context", stream=None):
        """rg_pool_key_index into a tensor this pool keeps; sets the pool's key_index."""
        torch = _torch()
        dev = self.bm_begin.device if self.bm_begin is not None else torch.device("cuda")
        self.kidx = torch.empty(max(self.n_bitmaps, 1) * RG_KEY_INDEX_BYTES, dtype=torch.uint8, device=dev)
        ctx.check(lib().rg_pool_key_index(ctx.h, ctypes.byref(self._c), _ptr(self.kidx), _stream(stream)))
        self._c.key_index = _ptr(self.kidx).value
        return self

    @staticmethod
    def from_view(view: "rg_pool") -> "Pool":
        """A Pool over device memory someone else owns (e.g. a server result view)."""
        p = Pool.__new__(Pool)
        p.n_bitmaps, p.n_containers, p.payload_bytes = view.n_bitmaps, view.n_containers, view.payload_bytes
        p.bm_begin = p.keys = p.types = p.card = p.size = p.off = p.payload = p.bm_card = p.bm_wbytes = None
        p._c = view
        return p

    @staticmethod
    def host_arrays(values, offsets):
        """rg_pool_measure_host + rg_pool_build_host: numpy arrays of the pool format."""
        values = np.ascontiguousarray(values, dtype=np.uint32)
        offsets = np.ascontiguousarray(offsets, dtype=np.uint64)
        n = len(offsets) - 1
        L = lib()
        nc, pb = ctypes.c_uint64(), ctypes.c_uint64()
        st = L.rg_pool_measure_host(values.ctypes.data, offsets.ctypes.data, n, ctypes.byref(nc), ctypes.byref(pb))
        if st != RG_OK:
            raise RoaringError(st, "rg_pool_measure_host: values must be strictly increasing per bitmap")
        nc, pb = nc.value, pb.value
        a = {"bm_begin": np.zeros(n + 1, np.uint64), "keys": np.zeros(nc, np.uint16),
             "types": np.zeros(nc, np.uint8), "card": np.zeros(nc, np.uint32), "size": np.zeros(nc, np.uint32),
             "off": np.zeros(nc, np.uint64), "payload": np.zeros(max(pb, 16), np.uint8),
             "bm_card": np.zeros(n, np.uint64), "bm_wbytes": np.zeros(n, np.uint64)}
        st = L.rg_pool_build_host(values.ctypes.data, offsets.ctypes.data, n,
                                  *[a[k].ctypes.data for k in ("bm_begin", "keys", "types", "card", "size", "off",
                                                               "payload", "bm_card", "bm_wbytes")])
        if st != RG_OK:
            raise RoaringError(st, "rg_pool_build_host failed")
        return n, nc, pb, a

    @staticmethod
    def from_sets(values, offsets, device="cuda"):
        n, nc, pb, a = Pool.host_arrays(values, offsets)
        return Pool.from_host_arrays(a, device)

    @staticmethod
    def from_host_arrays(a, device="cuda"):
        """A device pool from host arrays in the pool format (the keys of
        host_arrays' result; payload a multiple of 16 bytes)."""
        torch = _torch()

        def dev(x, dt):
            return torch.from_numpy(np.ascontiguousarray(x).view(dt)).to(device)

        n = len(a["bm_begin"]) - 1
        nc = len(a["keys"])
        return Pool(n, nc, max(len(a["payload"]), 16), dev(a["bm_begin"], np.int64), dev(a["keys"], np.int16),
                    dev(a["types"], np.uint8), dev(a["card"], np.int32), dev(a["size"], np.int32),
                    dev(a["off"], np.int64), dev(a["payload"], np.uint8), dev(a["bm_card"], np.int64),
                    dev(a["bm_wbytes"], np.int64))

    @staticmethod
    def from_dense_words(ctx: Context, words, n_bitmaps: int, n_keys: int, stream=None):
        """Pool over a device buffer of [n_bitmaps][n_keys][1024] uint64 bitset words
        (keys 0..n_keys-1 in every bitmap); cardinalities come from rg_pool_recount."""
        torch = _torch()
        dev = words.device
        nc = n_bitmaps * n_keys
        e = lambda n, dt: torch.empty(n, dtype=dt, device=dev)
        payload = words.view(torch.uint8).reshape(-1)
        p = Pool(n_bitmaps, nc, nc * 8192, e(n_bitmaps + 1, torch.int64), e(nc, torch.int16), e(nc, torch.uint8),
                 e(nc, torch.int32), e(nc, torch.int32), e(nc, torch.int64), payload, e(n_bitmaps, torch.int64),
                 e(n_bitmaps, torch.int64))
        ctx.check(lib().rg_pool_init_dense(ctx.h, ctypes.byref(p.c), n_keys, _stream(stream)))
        return p

    def to_host(self):
        """Copies of the pool arrays as numpy (for inspection and tests)."""
        f = lambda t, dt: t.detach().cpu().numpy().view(dt)
        return {"bm_begin": f(self.bm_begin, np.uint64), "keys": f(self.keys, np.uint16),
                "types": f(self.types, np.uint8), "card": f(self.card, np.uint32), "size": f(self.size, np.uint32),
                "off": f(self.off, np.uint64), "payload": f(self.payload, np.uint8),
                "bm_card": f(self.bm_card, np.uint64), "bm_wbytes": f(self.bm_wbytes, np.uint64)}


class OutArena:
    """Device buffers of an rg_out for n result bitmaps."""

    def __init__(self, n_pairs: int, cap_containers: int, cap_payload: int, device="cuda"):
        torch = _torch()
        cap_containers = max(int(cap_containers), 1)
        cap_payload = max((int(cap_payload) + 15) // 16 * 16, 16)
        self.n_pairs = n_pairs
        self.bm_begin = torch.zeros(n_pairs + 1, dtype=torch.int64, device=device)
        self.keys = torch.empty(cap_containers, dtype=torch.int16, device=device)
        self.types = torch.empty(cap_containers, dtype=torch.uint8, device=device)
        self.card = torch.empty(cap_containers, dtype=torch.int32, device=device)
        self.size = torch.empty(cap_containers, dtype=torch.int32, device=device)
        self.off = torch.empty(cap_containers, dtype=torch.int64, device=device)
        self.payload = torch.empty(cap_payload, dtype=torch.uint8, device=device)
        self.bm_card = torch.zeros(max(n_pairs, 1), dtype=torch.int64, device=device)
        self.bm_wbytes = torch.zeros(max(n_pairs, 1), dtype=torch.int64, device=device)
        self.c = rg_out(cap_containers, cap_payload, self.bm_begin.data_ptr(), self.keys.data_ptr(),
                        self.types.data_ptr(), self.card.data_ptr(), self.size.data_ptr(), self.off.data_ptr(),
                        self.payload.data_ptr(), self.bm_card.data_ptr(), self.bm_wbytes.data_ptr(), 0, 0, 0, 0)

    def as_pool(self) -> Pool:
        n = int(self.c.n_containers)
        return Pool(self.n_pairs, n, self.payload.numel(), self.bm_begin, self.keys, self.types, self.card,
                    self.size, self.off, self.payload, self.bm_card, self.bm_wbytes)


# ---------------------------------------------------------------- C names

def roaring_batch(ctx: Context, op, A: Pool, B: Pool, ia, ib, flags: int, out: OutArena | None = None,
                  cards=None, jacc=None, stream=None) -> int:
    """Thin wrapper of roaring_batch(): ia, ib are device uint32 (torch int32) tensors."""
    op = OPS[op] if isinstance(op, str) else op
    n = int(ia.numel())
    return lib().roaring_batch(ctx.h, op, ctypes.byref(A.c), ctypes.byref(B.c), _ptr(ia), _ptr(ib), n, flags,
                               ctypes.byref(out.c) if out is not None else None, _ptr(cards), _ptr(jacc),
                               _stream(stream))


RG_STATIC_SCRATCH_BYTES, RG_STATIC_MAX_PAIRS = 32 << 20, 1 << 20


def roaring_batch_static(ctx: Context, op, A: Pool, B: Pool, ia, ib, flags: int, cards=None, jacc=None,
                         stream=None, n_pairs=None) -> int:
    """Thin wrapper of roaring_batch_static() (count-only, no allocation):
    ia, ib are device uint32 (torch int32) tensors; n_pairs defaults to their length."""
    op = OPS[op] if isinstance(op, str) else op
    n = int(ia.numel()) if n_pairs is None else int(n_pairs)
    return lib().roaring_batch_static(ctx.h, op, ctypes.byref(A.c), ctypes.byref(B.c), _ptr(ia), _ptr(ib), n,
                                      flags, _ptr(cards), _ptr(jacc), _stream(stream))


def _single_mat(name):
    def f(ctx: Context, A: Pool, ia: int, B: Pool, ib: int, out: OutArena, stream=None) -> int:
        return getattr(lib(), name)(ctx.h, ctypes.byref(A.c), ia, ctypes.byref(B.c), ib, ctypes.byref(out.c),
                                    _stream(stream))
    f.__name__ = name
    return f


def _single_card(name):
    def f(ctx: Context, A: Pool, ia: int, B: Pool, ib: int, d_out, stream=None) -> int:
        return getattr(lib(), name)(ctx.h, ctypes.byref(A.c), ia, ctypes.byref(B.c), ib, _ptr(d_out),
                                    _stream(stream))
    f.__name__ = name
    return f


roaring_and = _single_mat("roaring_and")
roaring_or = _single_mat("roaring_or")
roaring_xor = _single_mat("roaring_xor")
roaring_andnot = _single_mat("roaring_andnot")
roaring_and_cardinality = _single_card("roaring_and_cardinality")
roaring_or_cardinality = _single_card("roaring_or_cardinality")
roaring_xor_cardinality = _single_card("roaring_xor_cardinality")
roaring_andnot_cardinality = _single_card("roaring_andnot_cardinality")
roaring_jaccard = _single_card("roaring_jaccard")


def roaring_jaccard_host(ctx: Context, A: Pool, ia: int, B: Pool, ib: int, stream=None) -> float:
    """roaring_jaccard_host: the Jaccard index as a Python float (synchronises)."""
    j = ctypes.c_double()
    ctx.check(lib().roaring_jaccard_host(ctx.h, ctypes.byref(A.c), ia, ctypes.byref(B.c), ib, ctypes.byref(j),
                                         _stream(stream)))
    return j.value


def roaring_contains(ctx: Context, P: Pool, ids, values, out, stream=None) -> int:
    """Thin wrapper of roaring_contains(): ids, values device uint32 (torch int32),
    out device uint8, all of one length."""
    n = int(ids.numel())
    return lib().roaring_contains(ctx.h, ctypes.byref(P.c), _ptr(ids), _ptr(values), n, _ptr(out), _stream(stream))


def contains(ctx: Context, P: Pool, ids, values, stream=None):
    """Membership of values[i] in bitmap ids[i]: a device bool tensor."""
    torch = _torch()
    out = torch.empty(max(int(ids.numel()), 1), dtype=torch.uint8, device=ids.device)
    ctx.check(roaring_contains(ctx, P, ids, values, out, stream))
    return out[:int(ids.numel())].bool()


def roaring_to_uint32(ctx: Context, P: Pool, b0: int, n: int, offsets, values, cap: int, stream=None):
    """Thin wrapper of roaring_to_uint32(): (status, needed values)."""
    need = ctypes.c_uint64()
    st = lib().roaring_to_uint32(ctx.h, ctypes.byref(P.c), b0, n, _ptr(offsets), _ptr(values), cap,
                                 ctypes.byref(need), _stream(stream))
    return st, int(need.value)


def to_uint32(ctx: Context, P: Pool, b0: int = 0, n: int | None = None, stream=None):
    """Sorted uint32 values of bitmaps b0 .. b0+n-1: (offsets int64[n+1], values
    int32 tensor viewed as uint32), sized from the library's report."""
    torch = _torch()
    n = P.n_bitmaps - b0 if n is None else n
    dev = P.bm_begin.device if P.bm_begin is not None else torch.device("cuda", ctx.device)
    offsets = torch.empty(n + 1, dtype=torch.int64, device=dev)
    # first call without room: it succeeds only when there are no values
    values = torch.empty(1, dtype=torch.int32, device=dev)
    st, need = roaring_to_uint32(ctx, P, b0, n, offsets, None, 0, stream)
    if st == RG_ECAPACITY:
        values = torch.empty(need, dtype=torch.int32, device=dev)
        st, need = roaring_to_uint32(ctx, P, b0, n, offsets, values, need, stream)
    ctx.check(st)
    return offsets, values[:need]


def rg_pool_recount(ctx: Context, pool: Pool, stream=None):
    ctx.check(lib().rg_pool_recount(ctx.h, ctypes.byref(pool.c), _stream(stream)))


def rg_pool_validate(ctx: Context, pool: Pool, stream=None) -> int:
    bad = ctypes.c_uint64()
    ctx.check(lib().rg_pool_validate(ctx.h, ctypes.byref(pool.c), ctypes.byref(bad), _stream(stream)))
    return int(bad.value)


def rg_pool_check(ctx: Context, pool: Pool, rules: int = 0, stream=None) -> int:
    """rg_pool_check: number of containers that break the rules (0: well-formed; RG_RULES_P1: also P1)."""
    n = ctypes.c_uint64()
    ctx.check(lib().rg_pool_check(ctx.h, ctypes.byref(pool.c), rules, ctypes.byref(n), _stream(stream)))
    return int(n.value)


def canonicalize(ctx: Context, pool: Pool, stream=None) -> "OutArena":
    """rg_pool_canonicalize with arena sizing: the pool's bitmaps in P1 form (an OutArena)."""
    dev = pool.bm_begin.device
    out = OutArena(pool.n_bitmaps, 0, 0, dev)
    out.c.cap_containers = 0
    out.c.cap_payload_bytes = 0
    st = lib().rg_pool_canonicalize(ctx.h, ctypes.byref(pool.c), ctypes.byref(out.c), _stream(stream))
    if st == RG_ECAPACITY:
        out = OutArena(pool.n_bitmaps, out.c.needed_containers, out.c.needed_payload_bytes, dev)
        st = lib().rg_pool_canonicalize(ctx.h, ctypes.byref(pool.c), ctypes.byref(out.c), _stream(stream))
    ctx.check(st)
    return out


def rg_pool_digest(ctx: Context, pool: Pool, stream=None):
    torch = _torch()
    dev = pool.bm_begin.device if pool.bm_begin is not None else torch.device("cuda", ctx.device)
    d = torch.zeros(max(pool.n_bitmaps, 1), dtype=torch.int64, device=dev)
    ctx.check(lib().rg_pool_digest(ctx.h, ctypes.byref(pool.c), _ptr(d), _stream(stream)))
    return d[:pool.n_bitmaps]


class Plan:
    """rg_plan: batched execution, sync-free, graph-capturable, tunable (count-only);
    materialize=True makes a materialising plan (rg_plan_create_mat) whose results
    land in self.out (an OutArena sized from the library's report).
    Keeps references to the pools, pair tensors and outputs it was made with."""

    def __init__(self, ctx: Context, op, A: Pool, B: Pool, ia, ib, card=True, jaccard=False, stream=None,
                 materialize=False):
        torch = _torch()
        dev = A.bm_begin.device
        n = int(ia.numel())
        self.n_pairs = n
        self.ctx, self.A, self.B, self.ia, self.ib = ctx, A, B, ia, ib
        self.cards = torch.zeros(n, dtype=torch.int64, device=dev) if card else None
        self.jacc = torch.zeros(n, dtype=torch.float64, device=dev) if jaccard else None
        flags = (RG_FLAG_CARD if card else 0) | (RG_FLAG_JACCARD if jaccard else 0)
        h = ctypes.c_void_p()
        op = OPS[op] if isinstance(op, str) else op
        self.out = None
        if materialize:
            flags |= RG_FLAG_MATERIALIZE
            out = OutArena(n, 0, 0, dev)
            out.c.cap_containers = 0
            out.c.cap_payload_bytes = 0
            args = lambda o: (ctx.h, op, ctypes.byref(A.c), ctypes.byref(B.c), _ptr(ia), _ptr(ib), n, flags,
                              ctypes.byref(o.c), _ptr(self.cards), _ptr(self.jacc), ctypes.byref(h), _stream(stream))
            st = lib().rg_plan_create_mat(*args(out))
            if st == RG_ECAPACITY:
                out = OutArena(n, out.c.needed_containers, out.c.needed_payload_bytes, dev)
                st = lib().rg_plan_create_mat(*args(out))
            ctx.check(st)
            self.out = out
        else:
            ctx.check(lib().rg_plan_create(ctx.h, op, ctypes.byref(A.c), ctypes.byref(B.c), _ptr(ia), _ptr(ib), n,
                                           flags, _ptr(self.cards), _ptr(self.jacc), ctypes.byref(h),
                                           _stream(stream)))
        self.h = h

    def result(self, stream=None) -> Pool:
        """rg_plan_result (synchronises): the materialised results as a Pool view of self.out."""
        nc, pu = ctypes.c_uint64(), ctypes.c_uint64()
        self.ctx.check(lib().rg_plan_result(self.h, ctypes.byref(nc), ctypes.byref(pu), _stream(stream)))
        self.out.c.n_containers = nc.value
        self.out.c.payload_used = pu.value
        return self.out.as_pool()

    def execute(self, stream=None):
        self.ctx.check(lib().rg_plan_execute(self.h, _stream(stream)))

    def capture(self, stream):
        self.ctx.check(lib().rg_plan_capture(self.h, _stream(stream)))

    def tune(self, stream=None, reps=3, cache=None, key=None):
        """rg_plan_tune. With cache (a JSON file path), a setting stored under key
        (default: the plan's pair, slot and wave counts and its dispatch mode) is
        applied with rg_plan_set instead of tuning again; a new one is stored."""
        if cache is None:
            self.ctx.check(lib().rg_plan_tune(self.h, _stream(stream), reps))
            return
        import json

        info = self.info()
        key = key or f"pairs={self.n_pairs},slots={info['slots']},waves={info['waves']},mode={self.ctx.dispatch_mode}"
        table = {}
        if os.path.exists(cache):
            with open(cache) as f:
                table = json.load(f)
        hit = table.get(key)
        if hit:
            self.set(hit["grid"], hit["gallop_ratio"], hit["thread_max"])
            return
        self.ctx.check(lib().rg_plan_tune(self.h, _stream(stream), reps))
        info = self.info()
        table[key] = {k: info[k] for k in ("grid", "gallop_ratio", "thread_max")}
        tmp = cache + ".tmp"
        with open(tmp, "w") as f:
            json.dump(table, f, indent=1, sort_keys=True)
        os.replace(tmp, cache)

    def set(self, grid: int, gallop_ratio: int, thread_max: int = 8):
        st = lib().rg_plan_set(self.h, grid, gallop_ratio, thread_max)
        if st not in (RG_OK, RG_ENOTSUP):
            self.ctx.check(st)

    def info(self):
        g, r, tm, w, gr = ctypes.c_uint32(), ctypes.c_uint32(), ctypes.c_uint32(), ctypes.c_uint32(), ctypes.c_int()
        s = ctypes.c_uint64()
        self.ctx.check(lib().rg_plan_info(self.h, ctypes.byref(g), ctypes.byref(r), ctypes.byref(tm), ctypes.byref(s),
                                          ctypes.byref(w), ctypes.byref(gr)))
        return {"grid": g.value, "gallop_ratio": r.value, "thread_max": tm.value, "slots": s.value, "waves": w.value,
                "graph": bool(gr.value)}

    def close(self):
        if self.h:
            lib().rg_plan_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# rg_profile_read classes (kernel variants; 3 in materialising form is the
# one-wave array kernel on intersections, 12 the same kernel on k-way slots,
# 13 the one-wave bitset kernel on k-way slots, 14 the one-wave fold of k-way
# unions and symmetric differences)
PROFILE_CLASSES = {0: "bb", 1: "unused", 2: "generic", 3: "merge", 4: "gallop", 5: "probe", 6: "runmerge",
                   7: "thread", 8: "bb-redo", 9: "thread-fused", 10: "count-fused", 11: "kway-eval",
                   12: "kway-small", 13: "kway-bb", 14: "kway-wave"}


def profile_enable(ctx: Context, on: bool = True):
    ctx.check(lib().rg_profile_enable(ctx.h, 1 if on else 0))


def profile_reset(ctx: Context):
    ctx.check(lib().rg_profile_reset(ctx.h))


def profile_read(ctx: Context):
    """{(class name, materialize): {"ms", "launches", "items"}} for classes that ran."""
    out = {}
    for v, name in PROFILE_CLASSES.items():
        for m in (0, 1):
            ms, n, it = ctypes.c_double(), ctypes.c_uint64(), ctypes.c_uint64()
            ctx.check(lib().rg_profile_read(ctx.h, v, m, ctypes.byref(ms), ctypes.byref(n), ctypes.byref(it)))
            if n.value or it.value:  # the fused class has items but no launches
                out[(name, bool(m))] = {"ms": ms.value, "launches": n.value, "items": it.value}
    return out


# ---------------------------------------------------------------- conveniences

def batch(ctx: Context, op, A: Pool, B: Pool, ia, ib, materialize=True, card=False, jaccard=False, out=None,
          stream=None):
    """roaring_batch with arena sizing: returns (out_arena or None, cards or None, jacc or None)."""
    torch = _torch()
    dev = A.bm_begin.device
    n = int(ia.numel())
    flags = (RG_FLAG_MATERIALIZE if materialize else 0) | (RG_FLAG_CARD if card else 0) | \
        (RG_FLAG_JACCARD if jaccard else 0)
    cards = torch.zeros(max(n, 1), dtype=torch.int64, device=dev) if card else None
    jacc = torch.zeros(max(n, 1), dtype=torch.float64, device=dev) if jaccard else None
    done = False
    if materialize and out is None:
        # first call with an empty arena: either nothing is needed, or it reports the sizes
        out = OutArena(n, 0, 0, dev)
        out.c.cap_containers = 0
        out.c.cap_payload_bytes = 0
        st = roaring_batch(ctx, op, A, B, ia, ib, flags, out, cards, jacc, stream)
        if st == RG_ECAPACITY:
            out = OutArena(n, out.c.needed_containers, out.c.needed_payload_bytes, dev)
        else:
            ctx.check(st)
            done = True
    if not done:
        ctx.check(roaring_batch(ctx, op, A, B, ia, ib, flags, out, cards, jacc, stream))
    return out, (cards[:n] if card else None), (jacc[:n] if jaccard else None)


# ---------------------------------------------------------------- mutable bitmaps

class MutablePool:
    """rg_mpool: bitmaps changed in place (op=) with maintained cardinalities."""

    def __init__(self, ctx: Context, n_bitmaps: int, n_slots: int):
        h = ctypes.c_void_p()
        ctx.check(lib().rg_mpool_create(ctx.h, n_bitmaps, n_slots, ctypes.byref(h)))
        self.ctx, self.h, self.n_bitmaps, self.n_slots = ctx, h, n_bitmaps, n_slots

    def op(self, op, b: int, P: Pool, src: int, stream=None):
        op = OPS[op] if isinstance(op, str) else op
        self.ctx.check(lib().rg_mpool_op(self.h, op, b, ctypes.byref(P.c), src, _stream(stream)))

    def op_batch(self, ops, bitmaps, P: Pool, srcs, stream=None):
        """rg_mpool_op_batch: M[bitmaps[i]] ops[i]= P[srcs[i]], the bitmaps distinct."""
        import numpy as np

        o = np.ascontiguousarray([OPS[x] if isinstance(x, str) else x for x in ops], dtype=np.int32)
        bm = np.ascontiguousarray(bitmaps, dtype=np.uint32)
        sr = np.ascontiguousarray(srcs, dtype=np.uint32)
        assert len(o) == len(bm) == len(sr)
        self.ctx.check(lib().rg_mpool_op_batch(self.h, len(o), o.ctypes.data, bm.ctypes.data, ctypes.byref(P.c),
                                               sr.ctypes.data, _stream(stream)))

    def assign(self, b: int, P: Pool, src: int, stream=None):
        self.ctx.check(lib().rg_mpool_assign(self.h, b, ctypes.byref(P.c), src, _stream(stream)))

    def clear(self, b: int, stream=None):
        self.ctx.check(lib().rg_mpool_clear(self.h, b, _stream(stream)))

    def status(self, stream=None):
        """(status code, free slots); synchronises."""
        n = ctypes.c_uint32()
        st = lib().rg_mpool_status(self.h, ctypes.byref(n), _stream(stream))
        return st, int(n.value)

    def cards(self, stream=None):
        """The maintained cardinalities (device int64 tensor of n_bitmaps, viewed from uint64)."""
        torch = _torch()
        out = torch.empty(self.n_bitmaps, dtype=torch.int64, device="cuda")
        self.ctx.check(lib().rg_mpool_cards(self.h, _ptr(out), _stream(stream)))
        return out

    def export(self, b0: int = 0, n: int | None = None, stream=None) -> OutArena:
        n = self.n_bitmaps - b0 if n is None else n
        out = OutArena(n, 0, 0)
        out.c.cap_containers = 0
        out.c.cap_payload_bytes = 0
        st = lib().rg_mpool_export(self.h, b0, n, ctypes.byref(out.c), _stream(stream))
        if st == RG_ECAPACITY:
            out = OutArena(n, out.c.needed_containers, out.c.needed_payload_bytes)
            st = lib().rg_mpool_export(self.h, b0, n, ctypes.byref(out.c), _stream(stream))
        self.ctx.check(st)
        return out

    def close(self):
        if self.h:
            lib().rg_mpool_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ---------------------------------------------------------------- k-way and serving

def roaring_multi(ctx: Context, op, pool: Pool, d_ids, flags: int, out: OutArena | None = None, d_card=None,
                  stream=None) -> int:
    op = OPS[op] if isinstance(op, str) else op
    return lib().roaring_multi(ctx.h, op, ctypes.byref(pool.c), _ptr(d_ids), int(d_ids.numel()), flags,
                               ctypes.byref(out.c) if out is not None else None, _ptr(d_card), _stream(stream))


def multi(ctx: Context, op, pool: Pool, d_ids, materialize=True, card=True, stream=None):
    """roaring_multi with arena sizing: returns (out_arena or None, card tensor or None)."""
    torch = _torch()
    dev = pool.bm_begin.device
    flags = (RG_FLAG_MATERIALIZE if materialize else 0) | (RG_FLAG_CARD if card else 0)
    d_card = torch.zeros(1, dtype=torch.int64, device=dev) if card else None
    out = None
    if materialize:
        out = OutArena(1, 0, 0, dev)
        out.c.cap_containers = 0
        out.c.cap_payload_bytes = 0
        st = roaring_multi(ctx, op, pool, d_ids, flags, out, d_card, stream)
        if st == RG_ECAPACITY:
            out = OutArena(1, out.c.needed_containers, out.c.needed_payload_bytes, dev)
            ctx.check(roaring_multi(ctx, op, pool, d_ids, flags, out, d_card, stream))
        else:
            ctx.check(st)
    else:
        ctx.check(roaring_multi(ctx, op, pool, d_ids, flags, None, d_card, stream))
    return out, d_card


class Server:
    """rg_serve_*: continuous-batching k-way query server over a device pool."""

    def __init__(self, ctx: Context, pool: Pool, arena_bytes: int = 1 << 30, max_batch: int = 64,
                 max_inflight: int = 2):
        self.ctx, self.pool = ctx, pool
        h = ctypes.c_void_p()
        ctx.check(lib().rg_serve_start(ctx.h, ctypes.byref(pool.c), arena_bytes, max_batch, max_inflight,
                                       ctypes.byref(h)))
        self.h = h
        ctx.servers.add(self)

    @staticmethod
    def _query(op, ids, materialize, digest=False):
        import numpy as np

        ids = np.ascontiguousarray(ids, dtype=np.uint32)
        q = rg_query(OPS[op] if isinstance(op, str) else op, len(ids),
                     ids.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32)),
                     (RG_FLAG_MATERIALIZE if materialize else RG_FLAG_CARD) | (RG_FLAG_DIGEST if digest else 0))
        return q, ids

    def submit(self, op, ids, materialize=False, digest=False) -> int:
        """digest: also compute the result's fingerprint (rg_result.digest)."""
        q, keep = self._query(op, ids, materialize, digest)
        t = ctypes.c_uint64()
        self.ctx.check(lib().rg_serve_submit(self.h, ctypes.byref(q), 0, ctypes.byref(t)))
        return t.value

    def poll(self, ticket: int, wait: bool = True) -> rg_result:
        r = rg_result()
        self.ctx.check(lib().rg_serve_poll(self.h, ticket, 1 if wait else 0, ctypes.byref(r)))
        return r

    def release(self, ticket: int):
        self.ctx.check(lib().rg_serve_release(self.h, ticket))

    def replay(self, queries, arrival_ns, digest=False):
        """queries: list of (op, ids, materialize); arrival_ns: offsets from the start.
        Returns (latency_ns, cards, digests) as numpy uint64 arrays (digests 0
        unless digest=True)."""
        import numpy as np

        n = len(queries)
        arr = (rg_query * max(n, 1))()
        keep = []
        for i, (op, ids, mat) in enumerate(queries):
            q, k = self._query(op, ids, mat, digest)
            arr[i] = q
            keep.append(k)
        at = np.ascontiguousarray(arrival_ns, dtype=np.uint64)
        lat = np.zeros(n, np.uint64)
        cards = np.zeros(n, np.uint64)
        dig = np.zeros(n, np.uint64)
        self.ctx.check(lib().rg_serve_replay(self.h, n, arr, at.ctypes.data, lat.ctypes.data, cards.ctypes.data,
                                             dig.ctypes.data))
        return lat, cards, dig

    def stop(self) -> dict:
        if not self.h:
            return {}
        st = rg_serve_stats()
        rc = lib().rg_serve_stop(self.h, ctypes.byref(st))
        self.h = None
        self.ctx.check(rc)
        return {"queries": st.queries, "steps": st.steps, "mean_batch": st.mean_batch,
                "arena_peak_bytes": st.arena_peak_bytes, "deferred": st.deferred}

    def __del__(self):
        try:
            self.stop()
        except Exception:
            pass


# ---------------------------------------------------------------- learned dispatcher

def mlp_forward(ctx: Context, params, x, stream=None):
    torch = _torch()
    y = torch.empty((x.shape[0], 6), dtype=torch.float32, device=x.device)
    ctx.check(lib().rg_mlp_forward(ctx.h, _ptr(params), _ptr(x), x.shape[0], _ptr(y), _stream(stream)))
    return y


def mlp_grad(ctx: Context, params, x, t, m, stream=None):
    torch = _torch()
    g = torch.empty(RG_MLP_PARAMS, dtype=torch.float32, device=x.device)
    loss = torch.zeros(1, dtype=torch.float32, device=x.device)
    ctx.check(lib().rg_mlp_grad(ctx.h, _ptr(params), _ptr(x), _ptr(t), _ptr(m), x.shape[0], _ptr(g), _ptr(loss),
                                _stream(stream)))
    return g, loss


def mlp_adam(ctx: Context, params, grad, m, v, step: int, lr: float, stream=None):
    ctx.check(lib().rg_mlp_adam(ctx.h, _ptr(params), _ptr(grad), _ptr(m), _ptr(v), step, lr, _stream(stream)))


def dispatch_samples(ctx: Context, A: Pool, B: Pool, ia, ib, stream=None):
    """Cost samples of every count variant on the pairs: (x [n, 12], t [n, 6], m [n, 6])."""
    torch = _torch()
    dev = A.bm_begin.device
    n_slots = ctypes.c_uint64()
    st = lib().rg_dispatch_sample(ctx.h, ctypes.byref(A.c), ctypes.byref(B.c), _ptr(ia), _ptr(ib), int(ia.numel()),
                                  VARIANTS["generic"], None, None, None, 0, ctypes.byref(n_slots), _stream(stream))
    if st != RG_ECAPACITY:
        ctx.check(st)
    n = max(int(n_slots.value), 1)
    x = torch.zeros((n, 12), dtype=torch.float32, device=dev)
    t = torch.zeros((n, 6), dtype=torch.float32, device=dev)
    m = torch.zeros((n, 6), dtype=torch.uint8, device=dev)
    for name in ("generic", "merge", "gallop", "probe", "runmerge", "thread"):
        ctx.check(lib().rg_dispatch_sample(ctx.h, ctypes.byref(A.c), ctypes.byref(B.c), _ptr(ia), _ptr(ib),
                                           int(ia.numel()), VARIANTS[name], _ptr(x), _ptr(t), _ptr(m), n,
                                           ctypes.byref(n_slots), _stream(stream)))
    return x, t, m


def dispatch_train(ctx: Context, x, t, m, epochs=20, batch=4096, lr=1e-3, seed=1, params=None, stream=None):
    """Trains (initialises when seed != 0); returns (params, per-epoch loss)."""
    torch = _torch()
    if params is None:
        params = torch.zeros(RG_MLP_PARAMS, dtype=torch.float32, device=x.device)
    losses = torch.zeros(max(epochs, 1), dtype=torch.float32, device=x.device)
    ctx.check(lib().rg_dispatch_train(ctx.h, _ptr(x), _ptr(t), _ptr(m), x.shape[0], epochs, batch, lr, seed,
                                      _ptr(params), _ptr(losses), _stream(stream)))
    return params, losses[:epochs]


def dispatch_set_mlp(ctx: Context, params, stream=None):
    ctx.check(lib().rg_dispatch_set_mlp(ctx.h, _ptr(params), _stream(stream)))
    ctx.dispatch_mode = RG_DISPATCH_MLP


def dispatch_table(ctx: Context):
    table = np.zeros(RG_MLP_TABLE, dtype=np.uint8)
    ctx.check(lib().rg_dispatch_table(ctx.h, table.ctypes.data, table.size))
    return table
