"""Python binding of libbpfa (ctypes): argument marshalling only.

Every step of the Gibbs iteration runs in the HIP library; this module passes
pointers and sizes.  PyTorch supplies device memory (the workspace, device
inputs / outputs) and the HIP stream.  There is no CPU fallback: if the
library is missing the import of this module fails.
"""
import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "_lib", "libbpfa.so")

OK, EINVAL, ESHAPE, ENOMEM, EDEVICE, ESTATE, ENUMERIC, EBUSY = 0, -1, -2, -3, -4, -5, -6, -7
HOST, DEVICE = 0, 1
LEARN_DICT, SPARSE_CODE_ONLY, PRECISION_BF16 = 1, 2, 4
XFER_D, XFER_PI, XFER_GAMMAS = 1, 2, 4
FP32, BF16 = 0, 1
_NAMES = {EINVAL: "EINVAL", ESHAPE: "ESHAPE", ENOMEM: "ENOMEM", EDEVICE: "EDEVICE",
          ESTATE: "ESTATE", ENUMERIC: "ENUMERIC", EBUSY: "EBUSY"}

EXPORTED = ["bpfa_params_default", "bpfa_workspace_size", "bpfa_create", "bpfa_set_frame",
            "bpfa_reset_state", "bpfa_iterate", "bpfa_minibatch", "bpfa_reconstruct", "bpfa_mean_reset",
            "bpfa_mean_accumulate", "bpfa_mean_get", "bpfa_variance_get", "bpfa_set_precision",
            "bpfa_transfer_dictionary", "bpfa_get_state",
            "bpfa_set_state", "bpfa_set_state_noalloc", "bpfa_get_stats", "bpfa_set_timing", "bpfa_sync",
            "bpfa_get_patch_index", "bpfa_debug_philox", "bpfa_destroy", "bpfa_last_error"]


def precision_code(precision):
    codes = {"fp32": FP32, "bf16": BF16, FP32: FP32, BF16: BF16}
    if precision not in codes:
        raise ValueError("precision must be 'fp32' or 'bf16', got %r" % (precision,))
    return codes[precision]


class BpfaError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__("%s: %s" % (_NAMES.get(status, status), msg))
        self.status = status


class Params(ctypes.Structure):
    _fields_ = [("ndim", ctypes.c_int32),
                ("shape", ctypes.c_int64 * 4), ("patch", ctypes.c_int64 * 4),
                ("stride", ctypes.c_int64 * 4),
                ("K", ctypes.c_int32),
                ("a", ctypes.c_double), ("b", ctypes.c_double),
                ("c", ctypes.c_double), ("d", ctypes.c_double),
                ("e", ctypes.c_double), ("f", ctypes.c_double),
                ("gamma_s0", ctypes.c_double), ("gamma_eps0", ctypes.c_double),
                ("seed", ctypes.c_uint64), ("problem_id", ctypes.c_uint32),
                ("device", ctypes.c_int32), ("stream", ctypes.c_void_p)]


class StateView(ctypes.Structure):
    _fields_ = [("D", ctypes.c_void_p), ("W", ctypes.c_void_p), ("Z", ctypes.c_void_p),
                ("logit_pi", ctypes.c_void_p), ("gamma_s", ctypes.c_double),
                ("gamma_eps", ctypes.c_double), ("t", ctypes.c_int64), ("mem", ctypes.c_int)]


class Stats(ctypes.Structure):
    _fields_ = [("t", ctypes.c_int64), ("N", ctypes.c_int64), ("P", ctypes.c_int64),
                ("K", ctypes.c_int64), ("n_obs", ctypes.c_int64), ("sum_z", ctypes.c_int64),
                ("mean_active", ctypes.c_double), ("gamma_s", ctypes.c_double),
                ("gamma_eps", ctypes.c_double), ("pi_min", ctypes.c_double),
                ("pi_mean", ctypes.c_double), ("pi_max", ctypes.c_double),
                ("sum_w2", ctypes.c_double), ("sum_r2", ctypes.c_double),
                ("max_obs", ctypes.c_int32), ("timing", ctypes.c_int32),
                ("ms_index", ctypes.c_double), ("ms_sweep", ctypes.c_double),
                ("ms_dict", ctypes.c_double), ("ms_scalars", ctypes.c_double),
                ("ms_recon", ctypes.c_double), ("n_sweeps", ctypes.c_int64),
                ("ms_dict_stats", ctypes.c_double)]

    def as_dict(self):
        return {name: getattr(self, name) for name, _ in self._fields_}


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError("libbpfa.so is not built (%s); run __graft_entry__.build()" % LIB_PATH)
    # One HIP runtime per process.  PyTorch ships its own HIP runtime with the
    # same soname (libamdhip64.so.7) but asks for it under another name, so if
    # this library were loaded first the process would end up with two
    # runtimes (and torch's stream handles and device state would not be this
    # library's).  Importing torch first makes the library bind to torch's copy.
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    lib = ctypes.CDLL(LIB_PATH)
    vp, i32, u32, i64, u64 = (ctypes.c_void_p, ctypes.c_int32, ctypes.c_uint32, ctypes.c_int64,
                              ctypes.c_uint64)
    P = ctypes.POINTER
    sig = {
        "bpfa_params_default": (None, [P(Params)]),
        "bpfa_workspace_size": (ctypes.c_int, [P(Params), P(ctypes.c_size_t)]),
        "bpfa_create": (ctypes.c_int, [P(Params), vp, ctypes.c_size_t, vp, vp, ctypes.c_int, P(vp)]),
        "bpfa_set_frame": (ctypes.c_int, [vp, vp, vp, ctypes.c_int, ctypes.c_int]),
        "bpfa_reset_state": (ctypes.c_int, [vp]),
        "bpfa_iterate": (ctypes.c_int, [vp, i32, u32]),
        "bpfa_minibatch": (ctypes.c_int, [vp, i32, i32, u32]),
        "bpfa_reconstruct": (ctypes.c_int, [vp, vp, ctypes.c_int]),
        "bpfa_mean_reset": (ctypes.c_int, [vp]),
        "bpfa_mean_accumulate": (ctypes.c_int, [vp]),
        "bpfa_mean_get": (ctypes.c_int, [vp, vp, ctypes.c_int, P(i64)]),
        "bpfa_variance_get": (ctypes.c_int, [vp, vp, ctypes.c_int, P(i64)]),
        "bpfa_set_precision": (ctypes.c_int, [vp, u32]),
        "bpfa_transfer_dictionary": (ctypes.c_int, [vp, vp, u32]),
        "bpfa_get_state": (ctypes.c_int, [vp, P(StateView)]),
        "bpfa_set_state": (ctypes.c_int, [vp, P(StateView)]),
        "bpfa_set_state_noalloc": (ctypes.c_int, [vp, P(StateView)]),
        "bpfa_get_stats": (ctypes.c_int, [vp, P(Stats)]),
        "bpfa_set_timing": (ctypes.c_int, [vp, ctypes.c_int]),
        "bpfa_sync": (ctypes.c_int, [vp]),
        "bpfa_get_patch_index": (ctypes.c_int, [vp, vp, vp, ctypes.c_int]),
        "bpfa_debug_philox": (ctypes.c_int, [i32, u64, u32, u32, vp, u32, u32, i64, vp,
                                             ctypes.c_int]),
        "bpfa_destroy": (None, [vp]),
        "bpfa_last_error": (ctypes.c_char_p, []),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    return lib


lib = _load()


def _check(status):
    if status != OK:
        raise BpfaError(status, lib.bpfa_last_error().decode())


def default_params():
    p = Params()
    lib.bpfa_params_default(ctypes.byref(p))
    return p


def make_params(shape, patch, stride=None, K=64, a=1.0, b=1.0, c=1e-6, d=1e-6, e=1e-6, f=1e-6,
                gamma_s0=1.0, gamma_eps0=100.0, seed=0, problem_id=0, device=0, stream=None):
    p = default_params()
    nd = len(shape)
    stride = stride or (1,) * nd
    p.ndim = nd
    for i in range(nd):
        p.shape[i], p.patch[i], p.stride[i] = int(shape[i]), int(patch[i]), int(stride[i])
    p.K = int(K)
    p.a, p.b, p.c, p.d, p.e, p.f = a, b, c, d, e, f
    p.gamma_s0, p.gamma_eps0 = gamma_s0, gamma_eps0
    p.seed, p.problem_id, p.device = int(seed), int(problem_id), int(device)
    p.stream = stream
    return p


def workspace_size(params):
    n = ctypes.c_size_t()
    _check(lib.bpfa_workspace_size(ctypes.byref(params), ctypes.byref(n)))
    return n.value


def _is_torch(x):
    return type(x).__module__.startswith("torch")


def _buffer(x, dtype):
    """(pointer, kind, keep-alive) for a numpy array (host) or a torch tensor (device or host)."""
    if _is_torch(x):
        import torch
        tdt = {np.float32: torch.float32, np.uint8: torch.uint8, np.float64: torch.float64,
               np.uint32: torch.uint32, np.int32: torch.int32}[dtype]
        if x.dtype != tdt or not x.is_contiguous():
            raise TypeError("tensor must be contiguous %s" % tdt)
        return x.data_ptr(), (DEVICE if x.is_cuda else HOST), x
    arr = np.ascontiguousarray(x, dtype=dtype)
    return arr.ctypes.data, HOST, arr


class Problem:
    """One BPFA inpainting problem on one GPU (an opaque library handle).

    image / mask: numpy arrays (host) or CUDA tensors on the device (float32 /
    uint8, same shape).  The workspace is a torch uint8 tensor on the device
    when torch is importable, so the HBM it uses is visible to torch's
    allocator; the current torch stream is used unless `stream` is given.
    """

    def __init__(self, image, mask, patch, stride=None, K=64, seed=0, problem_id=0, device=0,
                 stream=None, use_torch_workspace=True, **hyper):
        shape = tuple(np.shape(image))
        if tuple(np.shape(mask)) != shape:
            raise ValueError("image and mask shapes differ")
        self.shape = shape
        self.patch = tuple(patch)
        self.stride = tuple(stride or (1,) * len(shape))
        self._ws = None
        ws_ptr, ws_bytes = None, 0
        torch = None
        try:
            import torch as _t
            torch = _t
        except ImportError:
            pass
        if stream is None and torch is not None and torch.cuda.is_available():
            stream = torch.cuda.current_stream(device).cuda_stream
        self.params = make_params(shape, patch, self.stride, K=K, seed=seed, problem_id=problem_id,
                                  device=device, stream=stream, **hyper)
        if use_torch_workspace and torch is not None and torch.cuda.is_available():
            ws_bytes = workspace_size(self.params)
            self._ws = torch.empty(ws_bytes, dtype=torch.uint8, device="cuda:%d" % device)
            ws_ptr = self._ws.data_ptr()
        ip, kind, keep_i = _buffer(image, np.float32)
        mp, kind_m, keep_m = _buffer(mask, np.uint8)
        if kind != kind_m:
            raise TypeError("image and mask must both be host or both be device memory")
        h = ctypes.c_void_p()
        _check(lib.bpfa_create(ctypes.byref(self.params), ws_ptr, ws_bytes, ip, mp, kind,
                               ctypes.byref(h)))
        self._h = h
        st = self.stats()
        self.N, self.P, self.K = int(st["N"]), int(st["P"]), int(st["K"])

    # -- lifecycle --
    def close(self):
        if getattr(self, "_h", None):
            lib.bpfa_destroy(self._h)
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

    @property
    def handle(self):
        return self._h

    # -- the hot path --
    def set_frame(self, image, mask, reset_codes=True):
        ip, kind, keep_i = _buffer(image, np.float32)
        mp, kind_m, keep_m = _buffer(mask, np.uint8)
        if kind != kind_m:
            raise TypeError("image and mask must both be host or both be device memory")
        _check(lib.bpfa_set_frame(self._h, ip, mp, kind, int(bool(reset_codes))))

    def reset_state(self):
        _check(lib.bpfa_reset_state(self._h))

    def iterate(self, n=1, flags=LEARN_DICT):
        _check(lib.bpfa_iterate(self._h, int(n), int(flags)))

    def minibatch(self, n_batches, n_steps=1, flags=LEARN_DICT):
        """n_steps mini-batch steps of a partition into n_batches batches."""
        _check(lib.bpfa_minibatch(self._h, int(n_batches), int(n_steps), int(flags)))

    def epochs(self, n_epochs, n_batches, flags=LEARN_DICT):
        """n_epochs complete epochs: n_epochs * n_batches mini-batch steps."""
        self.minibatch(n_batches, int(n_epochs) * int(n_batches), flags)

    def reconstruct(self, out=None):
        if out is None:
            out = np.empty(self.shape, np.float32)
        ptr, kind, keep = _buffer(out, np.float32)
        _check(lib.bpfa_reconstruct(self._h, ptr, kind))
        return out

    def mean_reset(self):
        """Start a new posterior mean (set_frame and reset_state do too)."""
        _check(lib.bpfa_mean_reset(self._h))

    def mean_accumulate(self):
        """Add the current sample's reconstruction to the posterior-mean sum."""
        _check(lib.bpfa_mean_accumulate(self._h))

    def posterior_mean(self, out=None):
        """Mean of the accumulated samples' reconstructions: (out, sample count)."""
        if out is None:
            out = np.empty(self.shape, np.float32)
        ptr, kind, keep = _buffer(out, np.float32)
        n = ctypes.c_int64(0)
        _check(lib.bpfa_mean_get(self._h, ptr, kind, ctypes.byref(n)))
        return out, int(n.value)

    def posterior_variance(self, out=None):
        """Unbiased per-pixel variance of the accumulated samples: (out, sample count)."""
        if out is None:
            out = np.empty(self.shape, np.float32)
        ptr, kind, keep = _buffer(out, np.float32)
        n = ctypes.c_int64(0)
        _check(lib.bpfa_variance_get(self._h, ptr, kind, ctypes.byref(n)))
        return out, int(n.value)

    def set_precision(self, precision):
        """'fp32' (binary32 contractions) or 'bf16' (BF16 matrix-core contractions with one
        binary32 correction pass)."""
        _check(lib.bpfa_set_precision(self._h, precision_code(precision)))

    def transfer_dictionary(self, src, what=XFER_D | XFER_PI | XFER_GAMMAS):
        _check(lib.bpfa_transfer_dictionary(self._h, src._h, int(what)))

    # -- state / stats --
    def get_state(self, want_codes=True):
        D = np.empty((self.K, self.P), np.float32)
        ell = np.empty(self.K, np.float64)
        W = np.empty((self.N, self.K), np.float32) if want_codes else None
        Z = np.empty((self.N, self.K), np.uint8) if want_codes else None
        v = StateView(D=D.ctypes.data, W=W.ctypes.data if want_codes else None,
                      Z=Z.ctypes.data if want_codes else None, logit_pi=ell.ctypes.data, mem=HOST)
        _check(lib.bpfa_get_state(self._h, ctypes.byref(v)))
        return dict(D=D, W=W, Z=Z, logit_pi=ell, gamma_s=v.gamma_s, gamma_eps=v.gamma_eps, t=v.t)

    def set_state(self, D=None, W=None, Z=None, logit_pi=None, gamma_s=None, gamma_eps=None,
                  t=None, noalloc=False):
        """Replace the sampler state (bpfa_set_state; noalloc=True calls
        bpfa_set_state_noalloc, which stages through the library's fixed
        device buffer instead of allocating)."""
        cur = self.stats()
        keep = []

        def ptr(x, dt):
            if x is None:
                return None
            a = np.ascontiguousarray(x, dtype=dt)
            keep.append(a)
            return a.ctypes.data

        v = StateView(D=ptr(D, np.float32), W=ptr(W, np.float32),
                      Z=ptr(None if Z is None else np.asarray(Z).astype(np.uint8), np.uint8),
                      logit_pi=ptr(logit_pi, np.float64),
                      gamma_s=float(cur["gamma_s"] if gamma_s is None else gamma_s),
                      gamma_eps=float(cur["gamma_eps"] if gamma_eps is None else gamma_eps),
                      t=int(cur["t"] if t is None else t), mem=HOST)
        fn = lib.bpfa_set_state_noalloc if noalloc else lib.bpfa_set_state
        _check(fn(self._h, ctypes.byref(v)))

    def stats(self):
        s = Stats()
        _check(lib.bpfa_get_stats(self._h, ctypes.byref(s)))
        return s.as_dict()

    def set_timing(self, on=True):
        _check(lib.bpfa_set_timing(self._h, int(bool(on))))

    def sync(self):
        _check(lib.bpfa_sync(self._h))

    def patch_index(self):
        pw = (self.P + 31) // 32
        bits = np.empty((self.N, pw), np.uint32)
        cnt = np.empty(self.N, np.int32)
        _check(lib.bpfa_get_patch_index(self._h, bits.ctypes.data, cnt.ctypes.data, HOST))
        return bits, cnt


def debug_philox(seed, problem_id, tag, c0, c1, t, device=0):
    c0 = np.ascontiguousarray(c0, dtype=np.uint32)
    out = np.empty((c0.size, 4), np.uint32)
    _check(lib.bpfa_debug_philox(int(device), int(seed), int(problem_id), int(tag),
                                 c0.ctypes.data, int(c1), int(t), int(c0.size), out.ctypes.data,
                                 HOST))
    return out
