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


class AcqPolicy(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("var_samples", ctypes.c_int32),
                ("fraction", ctypes.c_double), ("targeted_share", ctypes.c_double)]


ACQ_CALLER, ACQ_UNIFORM, ACQ_LINE_HOP, ACQ_TARGETED = 0, 1, 2, 3
_ACQ_KINDS = {"caller": ACQ_CALLER, "uniform": ACQ_UNIFORM, "line_hop": ACQ_LINE_HOP,
              "targeted": ACQ_TARGETED}


def make_policy(kind, fraction=0.1, targeted_share=0.5, var_samples=2):
    return AcqPolicy(kind=_ACQ_KINDS.get(kind, kind), var_samples=int(var_samples),
                     fraction=float(fraction), targeted_share=float(targeted_share))


EXPORTED = ["bpfa_server_params_default", "bpfa_server_create", "bpfa_server_set_dictionary",
            "bpfa_server_submit", "bpfa_server_submit_scene", "bpfa_server_set_policy",
            "bpfa_acquire_mask", "bpfa_server_poll", "bpfa_server_drain", "bpfa_server_stats",
            "bpfa_server_destroy"]

_P = ctypes.POINTER
_sig = {
    "bpfa_server_params_default": (None, [_P(ServerParams)]),
    "bpfa_server_create": (ctypes.c_int, [_P(ServerParams), _P(ctypes.c_void_p)]),
    "bpfa_server_set_dictionary": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p]),
    "bpfa_server_submit": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, _P(ctypes.c_int64),
                                          ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                          _P(ctypes.c_uint64)]),
    "bpfa_server_submit_scene": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, _P(ctypes.c_int64),
                                                ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                                _P(ctypes.c_uint64)]),
    "bpfa_server_set_policy": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, _P(AcqPolicy)]),
    "bpfa_acquire_mask": (ctypes.c_int, [_P(AcqPolicy), ctypes.c_int32, _P(ctypes.c_int64),
                                         ctypes.c_void_p, ctypes.c_uint64, ctypes.c_int32,
                                         ctypes.c_int64, ctypes.c_void_p, ctypes.c_int,
                                         ctypes.c_int32]),
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
        self._masks = {}        # ticket -> drawn mask of a scene frame

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

    def set_policy(self, stream, kind, fraction=0.1, targeted_share=0.5, var_samples=2):
        """Acquisition policy of a stream: "uniform", "line_hop", "targeted" or "caller"."""
        pol = make_policy(kind, fraction, targeted_share, var_samples)
        _check(lib.bpfa_server_set_policy(self._h, int(stream), ctypes.byref(pol)))

    def submit_scene(self, stream, scene):
        """Queue a scene: the stream's policy chooses the acquired pixels.  Returns
        (ticket, out, mask); both arrays are filled when the ticket is polled."""
        scene = np.ascontiguousarray(scene, np.float32)
        if scene.ndim != self.params.ndim:
            raise ValueError("the scene must have the server's dimension")
        out = np.empty(scene.shape, np.float32)
        mask = np.empty(scene.shape, np.uint8)
        shape = (ctypes.c_int64 * scene.ndim)(*scene.shape)
        t = ctypes.c_uint64()
        _check(lib.bpfa_server_submit_scene(self._h, int(stream), shape, scene.ctypes.data,
                                            out.ctypes.data, mask.ctypes.data, ctypes.byref(t)))
        self._pending[t.value] = out
        self._masks[t.value] = mask
        return t.value, out, mask

    def poll(self, max_results=1024):
        buf = (ServeResult * max_results)()
        n = ctypes.c_int32()
        _check(lib.bpfa_server_poll(self._h, buf, max_results, ctypes.byref(n)))
        res = []
        for i in range(n.value):
            r = {name: getattr(buf[i], name) for name, _ in ServeResult._fields_}
            r["out"] = self._pending.pop(r["ticket"], None)
            r["mask"] = self._masks.pop(r["ticket"], None)
            res.append(r)
        return res

    def drain(self):
        _check(lib.bpfa_server_drain(self._h))

    def stats(self):
        s = ServeStats()
        _check(lib.bpfa_server_stats(self._h, ctypes.byref(s)))
        return {name: getattr(s, name) for name, _ in ServeStats._fields_}


def acquire_mask(kind, shape, seed, stream, frame, fraction=0.1, targeted_share=0.5, weights=None,
                 device=0):
    """The mask a policy gives frame `frame` of stream `stream` (the server's rule,
    computed on the GPU); weights: the targeted policy's variance (host array)."""
    pol = make_policy(kind, fraction, targeted_share, 2)
    shape = tuple(int(x) for x in shape)
    mask = np.empty(shape, np.uint8)
    w = None if weights is None else np.ascontiguousarray(weights, np.float32)
    shp = (ctypes.c_int64 * len(shape))(*shape)
    _check(lib.bpfa_acquire_mask(ctypes.byref(pol), len(shape), shp,
                                 None if w is None else w.ctypes.data, int(seed), int(stream),
                                 int(frame), mask.ctypes.data, _b.HOST, int(device)))
    return mask
