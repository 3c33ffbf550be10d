"""Python binding of the libbpfa serving engine (include/bpfa_serve.h): marshalling only."""
import ctypes

import numpy as np

from . import bpfa as _b

lib = _b.lib


class ServerParams(ctypes.Structure):
    _fields_ = [("ndim", ctypes.c_int32), ("patch", ctypes.c_int64 * 4),
                ("stride", ctypes.c_int64 * 4), ("K", ctypes.c_int32),
                ("a", ctypes.c_double), ("b", ctypes.c_double), ("c", ctypes.c_double),
                ("d", ctypes.c_double), ("e", ctypes.c_double), ("f", ctypes.c_double),
                ("gamma_s0", ctypes.c_double), ("gamma_eps0", ctypes.c_double),
                ("seed", ctypes.c_uint64), ("n_streams", ctypes.c_int32),
                ("sc_iters", ctypes.c_int32), ("dict_every", ctypes.c_int32),
                ("max_slots", ctypes.c_int32), ("hbm_budget", ctypes.c_uint64),
                ("device", ctypes.c_int32), ("precision", ctypes.c_int32),
                ("use_graphs", ctypes.c_int32)]


class ServeResult(ctypes.Structure):
    _fields_ = [("ticket", ctypes.c_uint64), ("stream", ctypes.c_int32),
                ("status", ctypes.c_int32), ("frame_index", ctypes.c_int64),
                ("pixels", ctypes.c_int64), ("latency_ms", ctypes.c_double),
                ("queue_ms", ctypes.c_double), ("learned", ctypes.c_int32)]


class ServeStats(ctypes.Structure):
    _fields_ = [("submitted", ctypes.c_int64), ("completed", ctypes.c_int64),
                ("failed", ctypes.c_int64), ("in_flight", ctypes.c_int64),
                ("queued", ctypes.c_int64), ("slots", ctypes.c_int64),
                ("slot_bytes", ctypes.c_int64), ("peak_slot_bytes", ctypes.c_int64),
                ("slot_creations", ctypes.c_int64), ("slot_evictions", ctypes.c_int64),
                ("graph_frames", ctypes.c_int64), ("graph_captures", ctypes.c_int64)]


EXPORTED = ["bpfa_server_params_default", "bpfa_server_create", "bpfa_server_set_dictionary",
            "bpfa_server_submit", "bpfa_server_poll", "bpfa_server_drain", "bpfa_server_stats",
            "bpfa_server_destroy"]

_P = ctypes.POINTER
_sig = {
    "bpfa_server_params_default": (None, [_P(ServerParams)]),
    "bpfa_server_create": (ctypes.c_int, [_P(ServerParams), _P(ctypes.c_void_p)]),
    "bpfa_server_set_dictionary": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p]),
    "bpfa_server_submit": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, _P(ctypes.c_int64),
                                          ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                          _P(ctypes.c_uint64)]),
    "bpfa_server_poll": (ctypes.c_int, [ctypes.c_void_p, _P(ServeResult), ctypes.c_int32,
                                        _P(ctypes.c_int32)]),
    "bpfa_server_drain": (ctypes.c_int, [ctypes.c_void_p]),
    "bpfa_server_stats": (ctypes.c_int, [ctypes.c_void_p, _P(ServeStats)]),
    "bpfa_server_destroy": (None, [ctypes.c_void_p]),
}
for _name, (_res, _args) in _sig.items():
    _fn = getattr(lib, _name)
    _fn.restype = _res
    _fn.argtypes = _args


def _check(st):
    if st != _b.OK:
        raise _b.BpfaError(st, lib.bpfa_last_error().decode() or "server call failed")


class Server:
    """Live-feed server: per-stream dictionaries resident on the GPU, frames of any size."""

    def __init__(self, patch=(10, 10), stride=None, K=128, n_streams=4, sc_iters=5, dict_every=10,
                 max_slots=4, hbm_budget=16 << 30, seed=0, device=0, precision="fp32", use_graphs=True,
                 **hyper):
        p = ServerParams()
        lib.bpfa_server_params_default(ctypes.byref(p))
        p.ndim = len(patch)
        stride = stride or (1,) * len(patch)
        for d in range(len(patch)):
            p.patch[d], p.stride[d] = int(patch[d]), int(stride[d])
        p.K, p.n_streams, p.sc_iters, p.dict_every = int(K), int(n_streams), int(sc_iters), int(dict_every)
        p.max_slots, p.hbm_budget, p.seed, p.device = int(max_slots), int(hbm_budget), int(seed), int(device)
        p.precision = _b.precision_code(precision)
        p.use_graphs = 1 if use_graphs else 0
        for k, v in hyper.items():
            setattr(p, k, float(v))
        self.params = p
        h = ctypes.c_void_p()
        _check(lib.bpfa_server_create(ctypes.byref(p), ctypes.byref(h)))
        self._h = h
        self._pending = {}      # ticket -> output array (kept alive until completion)

    def close(self):
        if getattr(self, "_h", None):
            lib.bpfa_server_destroy(self._h)
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

    def set_dictionary(self, stream, problem):
        _check(lib.bpfa_server_set_dictionary(self._h, int(stream), problem.handle))

    def submit(self, stream, image, mask):
        image = np.ascontiguousarray(image, np.float32)
        mask = np.ascontiguousarray(mask, np.uint8)
        if image.shape != mask.shape or image.ndim != self.params.ndim:
            raise ValueError("image and mask must share a shape of the server's dimension")
        out = np.empty(image.shape, np.float32)
        shape = (ctypes.c_int64 * image.ndim)(*image.shape)
        t = ctypes.c_uint64()
        _check(lib.bpfa_server_submit(self._h, int(stream), shape, image.ctypes.data,
                                      mask.ctypes.data, out.ctypes.data, ctypes.byref(t)))
        self._pending[t.value] = out
        return t.value, out

    def poll(self, max_results=1024):
        buf = (ServeResult * max_results)()
        n = ctypes.c_int32()
        _check(lib.bpfa_server_poll(self._h, buf, max_results, ctypes.byref(n)))
        res = []
        for i in range(n.value):
            r = {name: getattr(buf[i], name) for name, _ in ServeResult._fields_}
            r["out"] = self._pending.pop(r["ticket"], None)
            res.append(r)
        return res

    def drain(self):
        _check(lib.bpfa_server_drain(self._h))

    def stats(self):
        s = ServeStats()
        _check(lib.bpfa_server_stats(self._h, ctypes.byref(s)))
        return {name: getattr(s, name) for name, _ in ServeStats._fields_}
