"""Python binding of libfastcpd, the gfx950 Fast Coherent Point Drift library.

Argument marshalling only: every numerical step runs in the HIP kernels of
libfastcpd.so.  PyTorch supplies device memory (tensors) and the HIP stream.
The functions keep the names of the C ABI declared in include/fastcpd.h;
``Registration`` bundles one handle with its workspace.

The library is built in-tree by ``paper_2006_06281_amd.build.build()``.
Importing this package when it is missing raises at once: there is no
fallback implementation.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libfastcpd.so")

CPD_ABI_VERSION = 1

CPD_OK, CPD_NOT_CONVERGED = 0, 1
CPD_E_ARG, CPD_E_STATE, CPD_E_WORKSPACE = -1, -2, -3
CPD_E_DEVICE, CPD_E_NUMERIC, CPD_E_UNSUPPORTED = -4, -5, -6

CPD_METHOD_ORIGINAL, CPD_METHOD_FAST, CPD_METHOD_ORIGINAL_LOWRANK = 0, 1, 2
CPD_PREC_FP64, CPD_PREC_FP32, CPD_PREC_BF16X = 0, 1, 2
CPD_EIG_FULL, CPD_EIG_TOPK, CPD_EIG_IMPORT = 0, 1, 2
CPD_FLAG_NO_SORT, CPD_FLAG_NO_CULL = 1, 2
CPDNET_BF16, CPDNET_FP32 = 0, 1
CPDNET_SHAPE_SPHERE, CPDNET_SHAPE_BUMPS = 0, 1
SHAPES = {"sphere": CPDNET_SHAPE_SPHERE, "bumps": CPDNET_SHAPE_BUMPS}
NET_PRECISIONS = {"bf16": CPDNET_BF16, "fp32": CPDNET_FP32}

METHODS = {"original": CPD_METHOD_ORIGINAL, "fast": CPD_METHOD_FAST,
           "cpdl": CPD_METHOD_ORIGINAL_LOWRANK}
PRECISIONS = {"fp64": CPD_PREC_FP64, "fp32": CPD_PREC_FP32, "bf16x": CPD_PREC_BF16X}
EIG_MODES = {"full": CPD_EIG_FULL, "topk": CPD_EIG_TOPK, "import": CPD_EIG_IMPORT}

EXPORTED = [
    "cpd_workspace_size", "cpd_init", "cpd_eig_prepare", "cpd_eig_count",
    "cpd_eig_export", "cpd_step", "cpd_register", "cpd_set_state",
    "cpd_get_state", "cpd_estep", "cpd_destroy", "cpd_status_str",
    "cpd_last_error", "cpd_abi_version", "cpd_build_info", "cpd_time_kernels",
    "cpd_matches", "cpd_solve_matches",
    "cpd_batch_workspace_size", "cpd_batch_init", "cpd_batch_prepare", "cpd_batch_register",
    "cpd_batch_info", "cpd_batch_destroy",
    "cpdnet_param_count", "cpdnet_init", "cpdnet_workspace_size", "cpdnet_forward",
    "cpdnet_forward_noalloc", "cpdnet_loss_grad", "cpdnet_adam", "cpdnet_synth",
]


class cpd_params(ctypes.Structure):
    _fields_ = [
        ("abi_version", ctypes.c_int32), ("M", ctypes.c_int32), ("N", ctypes.c_int32),
        ("D", ctypes.c_int32), ("beta", ctypes.c_double), ("lambda_", ctypes.c_double),
        ("w", ctypes.c_double), ("sigma2_init", ctypes.c_double),
        ("method", ctypes.c_int32), ("precision", ctypes.c_int32),
        ("eig_mode", ctypes.c_int32), ("K", ctypes.c_int32),
        ("oversample", ctypes.c_int32), ("power_iters", ctypes.c_int32),
        ("seed", ctypes.c_uint64), ("tol", ctypes.c_double),
        ("max_iter", ctypes.c_int32), ("flags", ctypes.c_int32),
    ]


class cpd_step_info(ctypes.Structure):
    _fields_ = [("iter", ctypes.c_int32), ("converged", ctypes.c_int32),
                ("sigma2", ctypes.c_double), ("dsigma2", ctypes.c_double),
                ("loglik", ctypes.c_double)]


class cpd_result(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int32), ("converged", ctypes.c_int32),
                ("sigma2", ctypes.c_double), ("t_c", ctypes.c_double),
                ("t_eig", ctypes.c_double), ("t_iter", ctypes.c_double),
                ("t_o", ctypes.c_double)]


class FastCPDError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{status_name(status)}: {msg}")
        self.status = status


_lib = None


def load_library(path: str = LIB_PATH):
    """Load libfastcpd.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(
            f"{path} is missing: build it with `python -m paper_2006_06281_amd.build`")
    lib = ctypes.CDLL(path)
    vp, sz = ctypes.c_void_p, ctypes.c_size_t
    P = ctypes.POINTER
    sig = {
        "cpd_workspace_size": ([P(cpd_params), P(sz)], ctypes.c_int),
        "cpd_init": ([P(vp), P(cpd_params), vp, vp, vp, sz, vp], ctypes.c_int),
        "cpd_eig_prepare": ([vp, vp, vp, vp], ctypes.c_int),
        "cpd_eig_count": ([vp, P(ctypes.c_int32)], ctypes.c_int),
        "cpd_eig_export": ([vp, vp, vp], ctypes.c_int),
        "cpd_step": ([vp, P(cpd_step_info)], ctypes.c_int),
        "cpd_register": ([vp, vp, vp, vp, P(cpd_result)], ctypes.c_int),
        "cpd_set_state": ([vp, vp, ctypes.c_double], ctypes.c_int),
        "cpd_get_state": ([vp, vp, vp, P(ctypes.c_double)], ctypes.c_int),
        "cpd_estep": ([vp, vp, vp, vp, vp], ctypes.c_int),
        "cpd_destroy": ([vp], ctypes.c_int),
        "cpd_time_kernels": ([vp, ctypes.c_int32, P(ctypes.c_double)], ctypes.c_int),
        "cpd_matches": ([vp, ctypes.c_int32, vp], ctypes.c_int),
        "cpd_solve_matches": ([vp, vp, ctypes.c_double, vp, vp], ctypes.c_int),
        "cpd_batch_workspace_size": ([ctypes.c_int32, P(cpd_params), P(sz)], ctypes.c_int),
        "cpd_batch_init": ([P(vp), ctypes.c_int32, P(cpd_params), vp, vp, P(ctypes.c_int64),
                            P(ctypes.c_int64), vp, sz, vp], ctypes.c_int),
        "cpd_batch_prepare": ([vp, ctypes.c_int32], ctypes.c_int),
        "cpd_batch_register": ([vp, vp, vp, vp, P(cpd_result)], ctypes.c_int),
        "cpd_batch_info": ([vp, P(ctypes.c_int32), P(ctypes.c_int32), P(ctypes.c_double),
                            P(ctypes.c_int32)], ctypes.c_int),
        "cpd_batch_destroy": ([vp], ctypes.c_int),
        "cpdnet_param_count": ([P(sz)], ctypes.c_int),
        "cpdnet_init": ([vp, ctypes.c_uint64, ctypes.c_float, vp], ctypes.c_int),
        "cpdnet_workspace_size": ([ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                   P(sz)], ctypes.c_int),
        "cpdnet_forward": ([vp, vp, vp, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                            ctypes.c_int32, vp, vp, sz, vp], ctypes.c_int),
        "cpdnet_forward_noalloc": ([vp, vp, vp, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                    ctypes.c_int32, vp, vp], ctypes.c_int),
        "cpdnet_loss_grad": ([vp, vp, vp, vp, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                              ctypes.c_int32, ctypes.c_double, vp, P(ctypes.c_double), vp, sz,
                              vp], ctypes.c_int),
        "cpdnet_adam": ([vp, vp, vp, vp, ctypes.c_int32, ctypes.c_float, vp], ctypes.c_int),
        "cpdnet_synth": ([vp, vp, vp, vp, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                          ctypes.c_double, ctypes.c_double, ctypes.c_double, ctypes.c_double,
                          ctypes.c_uint64, vp], ctypes.c_int),
        "cpd_status_str": ([ctypes.c_int], ctypes.c_char_p),
        "cpd_last_error": ([vp], ctypes.c_char_p),
        "cpd_abi_version": ([], ctypes.c_int32),
        "cpd_build_info": ([], ctypes.c_char_p),
    }
    for name, (args, res) in sig.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = res
    if lib.cpd_abi_version() != CPD_ABI_VERSION:
        raise ImportError("libfastcpd ABI version mismatch")
    _lib = lib
    return lib


def status_name(s: int) -> str:
    try:
        return load_library().cpd_status_str(s).decode()
    except ImportError:
        return str(s)


def last_error(h=None) -> str:
    return load_library().cpd_last_error(h).decode()


def _check(status: int, h=None, ok=(CPD_OK,)):
    if status not in ok:
        raise FastCPDError(status, last_error(h))
    return status


def require_device():
    """Raise unless the library is built and a HIP device is visible."""
    import torch
    load_library()
    if not torch.cuda.is_available():
        raise RuntimeError("no HIP device visible to torch")


def make_params(M, N, D=3, beta=2.0, lam=3.0, w=0.1, sigma2_init=0.0, method="fast",
                precision="fp32", eig_mode="full", K=0, oversample=20, power_iters=2,
                seed=0, tol=1e-8, max_iter=1000, sort=True, cull=True) -> cpd_params:
    """cpd_params; sort / cull map to the CPD_FLAG_NO_SORT / CPD_FLAG_NO_CULL
    bits (spatial order of the points inside the library, far-tile culling)."""
    flags = (0 if sort else CPD_FLAG_NO_SORT) | (0 if cull else CPD_FLAG_NO_CULL)
    return cpd_params(CPD_ABI_VERSION, int(M), int(N), int(D), float(beta), float(lam),
                      float(w), float(sigma2_init), METHODS.get(method, method),
                      PRECISIONS.get(precision, precision), EIG_MODES.get(eig_mode, eig_mode),
                      int(K), int(oversample), int(power_iters), int(seed), float(tol),
                      int(max_iter), flags)


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream_ptr(stream=None):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


# ----------------------------------------------------------- C ABI, 1:1
def cpd_workspace_size(p: cpd_params) -> int:
    out = ctypes.c_size_t(0)
    _check(load_library().cpd_workspace_size(ctypes.byref(p), ctypes.byref(out)))
    return out.value


def cpd_init(p: cpd_params, X, Y, workspace, stream=None):
    h = ctypes.c_void_p()
    nbytes = workspace.numel() * workspace.element_size()
    _check(load_library().cpd_init(ctypes.byref(h), ctypes.byref(p), _ptr(X), _ptr(Y),
                                   _ptr(workspace), nbytes, _stream_ptr(stream)))
    return h


def cpd_eig_prepare(h, U=None, lam=None, omega=None) -> int:
    """CPD_OK, or CPD_NOT_CONVERGED for a FULL decomposition cut at its cap."""
    return _check(load_library().cpd_eig_prepare(h, _ptr(U), _ptr(lam), _ptr(omega)), h,
                  ok=(CPD_OK, CPD_NOT_CONVERGED))


def cpd_eig_count(h) -> int:
    k = ctypes.c_int32(0)
    _check(load_library().cpd_eig_count(h, ctypes.byref(k)), h)
    return k.value


def cpd_eig_export(h, U_out, lam_out):
    _check(load_library().cpd_eig_export(h, _ptr(U_out), _ptr(lam_out)), h)


def cpd_step(h, want_info=True):
    info = cpd_step_info()
    _check(load_library().cpd_step(h, ctypes.byref(info) if want_info else None), h)
    return info if want_info else None


def cpd_register(h, W0=None, X_out=None, W_out=None):
    res = cpd_result()
    st = _check(load_library().cpd_register(h, _ptr(W0), _ptr(X_out), _ptr(W_out),
                                            ctypes.byref(res)), h,
                ok=(CPD_OK, CPD_NOT_CONVERGED))
    return res, st


def cpd_set_state(h, Xt, sigma2):
    _check(load_library().cpd_set_state(h, _ptr(Xt), float(sigma2)), h)


def cpd_get_state(h, Xt_out=None, W_out=None) -> float:
    s2 = ctypes.c_double(0)
    _check(load_library().cpd_get_state(h, _ptr(Xt_out), _ptr(W_out), ctypes.byref(s2)), h)
    return s2.value


def cpd_estep(h, logd=None, P1=None, Yt=None, tbar=None):
    _check(load_library().cpd_estep(h, _ptr(logd), _ptr(P1), _ptr(Yt), _ptr(tbar)), h)


KERNEL_STAGES = ("passA", "passA_merge", "passB", "passB_merge", "mstep", "sigma2",
                 "prescale", "iteration")


def cpd_time_kernels(h, reps=10) -> dict:
    out = (ctypes.c_double * 8)()
    _check(load_library().cpd_time_kernels(h, int(reps), out), h)
    return dict(zip(KERNEL_STAGES, list(out)))


def cpd_destroy(h):
    if h:
        load_library().cpd_destroy(h)


# ------------------------------------------------------------------ batch
def cpd_batch_workspace_size(params) -> int:
    arr = (cpd_params * len(params))(*params)
    out = ctypes.c_size_t(0)
    _check(load_library().cpd_batch_workspace_size(len(params), arr, ctypes.byref(out)))
    return out.value


class BatchRegistration:
    """Many independent Fast CPD registrations advanced together (FP32, D=3).

    Xs, Ys: lists of CUDA float32 tensors (M_i x 3, N_i x 3); per-instance
    keyword lists (beta, lam, w, ...) or scalars shared by all instances."""

    def __init__(self, Xs, Ys, stream=None, **kw):
        import torch
        B = len(Xs)
        self.B = B
        per = []
        for i in range(B):
            a = {k: (v[i] if isinstance(v, (list, tuple)) else v) for k, v in kw.items()}
            a.setdefault("precision", "fp32")
            per.append(make_params(Xs[i].shape[0], Ys[i].shape[0], 3, **a))
        self.params = per
        self.Xp = torch.cat([x.float().reshape(-1, 3) for x in Xs]).contiguous()
        self.Yp = torch.cat([y.float().reshape(-1, 3) for y in Ys]).contiguous()
        xo = [0]
        yo = [0]
        for x, y in zip(Xs, Ys):
            xo.append(xo[-1] + x.shape[0])
            yo.append(yo[-1] + y.shape[0])
        self.x_off = (ctypes.c_int64 * (B + 1))(*xo)
        self.y_off = (ctypes.c_int64 * (B + 1))(*yo)
        self._xo = xo
        arr = (cpd_params * B)(*per)
        self._arr = arr
        n = cpd_batch_workspace_size(per)
        self.workspace = torch.empty(max(n, 256), dtype=torch.uint8, device=self.Xp.device)
        self.h = ctypes.c_void_p()
        _check(load_library().cpd_batch_init(
            ctypes.byref(self.h), B, arr, _ptr(self.Xp), _ptr(self.Yp), self.x_off, self.y_off,
            _ptr(self.workspace), self.workspace.numel(), _stream_ptr(stream)))

    CHUNKS = (1024, 2048, 512, 4096)
    TILES = (1024, 512)

    def prepare(self, tune=True, candidate=None, cache=None):
        """tune: time every (split length, tile) candidate and keep the
        fastest; candidate: force one (index into candidates()) untimed.
        cache: a TuneCache or a JSON path; with tune, a stored plan for this
        batch's key is forced untimed, and a newly timed choice is stored
        (the environment variable FASTCPD_TUNE_CACHE names a default path)."""
        from . import tune_cache as tc
        if cache is None and os.environ.get("FASTCPD_TUNE_CACHE"):
            cache = os.environ["FASTCPD_TUNE_CACHE"]
        if isinstance(cache, str):
            cache = tc.TuneCache(cache)
        key = None
        if candidate is None and tune and cache is not None:
            key = self.tune_key()
            hit = cache.get(key)
            if hit is not None and 0 <= int(hit.get("candidate", -1)) < 8:
                candidate = int(hit["candidate"])
        code = 2 + int(candidate) if candidate is not None else int(bool(tune))
        _check(load_library().cpd_batch_prepare(self.h, code))
        if code == 1 and key is not None:
            inf = self.info()
            c = self.candidates().index((inf["chunk"], inf["tile"]))
            cache.put(key, {"candidate": c, "chunk": inf["chunk"], "tile": inf["tile"],
                            "tune_ms": [inf["tune_ms"][cd] for cd in self.candidates()]})
        return self

    def tune_key(self):
        """The autotune cache key of this batch (device arch, mean set sizes,
        instance count, D, precision)."""
        import torch
        from . import tune_cache as tc
        arch = torch.cuda.get_device_properties(self.Xp.device).gcnArchName
        return tc.batch_key(arch, [p.M for p in self.params], [p.N for p in self.params],
                            3, "fp32")

    @classmethod
    def candidates(cls):
        return [(cls.CHUNKS[c // 2], cls.TILES[c % 2]) for c in range(8)]

    def info(self):
        """dict: chunk, tile, tune_ms {(chunk, tile): ms per iteration}, K per instance."""
        c, t = ctypes.c_int32(0), ctypes.c_int32(0)
        ms = (ctypes.c_double * 8)()
        K = (ctypes.c_int32 * self.B)()
        _check(load_library().cpd_batch_info(self.h, ctypes.byref(c), ctypes.byref(t), ms, K))
        return {"chunk": c.value, "tile": t.value,
                "tune_ms": dict(zip(self.candidates(), list(ms))), "K": list(K)}

    def register(self, W0=None, sigma2=None):
        """W0: optional packed (sum M_i x 3) float32 CUDA tensor of warm-start
        coefficients; sigma2: optional per-instance starting sigma^2 (values
        <= 0 keep the default start)."""
        import torch
        out = torch.empty_like(self.Xp)
        res = (cpd_result * self.B)()
        s2 = None if sigma2 is None else (ctypes.c_double * self.B)(*[float(v) for v in sigma2])
        _check(load_library().cpd_batch_register(self.h, _ptr(W0), s2, _ptr(out), res),
               ok=(CPD_OK, CPD_NOT_CONVERGED))
        Xt = [out[self._xo[i]:self._xo[i + 1]] for i in range(self.B)]
        return Xt, list(res)

    def close(self):
        """Destroy the handle and release the workspace and packed inputs."""
        if getattr(self, "h", None):
            load_library().cpd_batch_destroy(self.h)
            self.h = None
        self.workspace = self.Xp = self.Yp = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ------------------------------------------------------------ warm start
class WarmStartNet:
    """The warm-start point-set network: fp32 master parameters, Adam state
    and a workspace sized for (batch, M, N).  precision "bf16" (default) or
    "fp32" selects the storage of activations and weight copies."""

    def __init__(self, seed=0, out_scale=1e-3, device="cuda", precision="bf16"):
        import torch
        self.precision = NET_PRECISIONS[precision]
        n = ctypes.c_size_t(0)
        _check(load_library().cpdnet_param_count(ctypes.byref(n)))
        self.count = n.value
        self.params = torch.empty(self.count, dtype=torch.float32, device=device)
        self.m = torch.zeros_like(self.params)
        self.v = torch.zeros_like(self.params)
        self.grad = torch.zeros_like(self.params)
        self.step_no = 0
        self.device = device
        self._ws = None
        self._ws_key = None
        _check(load_library().cpdnet_init(_ptr(self.params), int(seed), float(out_scale),
                                          _stream_ptr()))

    def _workspace(self, batch, M, N):
        import torch
        key = (batch, M, N, self.precision)
        if self._ws_key != key:
            n = ctypes.c_size_t(0)
            _check(load_library().cpdnet_workspace_size(batch, M, N, self.precision,
                                                        ctypes.byref(n)))
            self._ws = torch.empty(max(n.value, 256), dtype=torch.uint8, device=self.device)
            self._ws_key = key
        return self._ws

    def forward(self, X, Y):
        """X: (batch, M, 3), Y: (batch, N, 3) float32 -> W0 (batch, M, 3)."""
        import torch
        B, M, N = X.shape[0], X.shape[1], Y.shape[1]
        W0 = torch.empty(B, M, 3, dtype=torch.float32, device=X.device)
        ws = self._workspace(B, M, N)
        _check(load_library().cpdnet_forward(_ptr(self.params), _ptr(X), _ptr(Y), B, M, N,
                                             self.precision, _ptr(W0), _ptr(ws), ws.numel(),
                                             _stream_ptr()))
        return W0

    def forward_noalloc(self, X, Y):
        """forward() through cpdnet_forward_noalloc: the library's static
        device scratch replaces the workspace (no allocation in the call)."""
        import torch
        B, M, N = X.shape[0], X.shape[1], Y.shape[1]
        W0 = torch.empty(B, M, 3, dtype=torch.float32, device=X.device)
        _check(load_library().cpdnet_forward_noalloc(_ptr(self.params), _ptr(X), _ptr(Y), B, M,
                                                     N, self.precision, _ptr(W0),
                                                     _stream_ptr()))
        return W0

    def loss_grad(self, X, Y, V, beta, want_loss=True):
        """Gradient into self.grad; the loss (a host scalar, which waits for
        the stream) when want_loss, else None."""
        B, M, N = X.shape[0], X.shape[1], Y.shape[1]
        ws = self._workspace(B, M, N)
        loss = ctypes.c_double(0)
        _check(load_library().cpdnet_loss_grad(_ptr(self.params), _ptr(X), _ptr(Y), _ptr(V), B,
                                               M, N, self.precision, float(beta), _ptr(self.grad),
                                               ctypes.byref(loss) if want_loss else None,
                                               _ptr(ws), ws.numel(), _stream_ptr()))
        return loss.value if want_loss else None

    def train_step(self, X, Y, V, beta, lr=1e-3, want_loss=True):
        loss = self.loss_grad(X, Y, V, beta, want_loss)
        self.step_no += 1
        _check(load_library().cpdnet_adam(_ptr(self.params), _ptr(self.m), _ptr(self.v),
                                          _ptr(self.grad), self.step_no, float(lr),
                                          _stream_ptr()))
        return loss


def synth_pairs(batch, M, beta=2.0, coef=0.15, jitter=0.01, outlier_frac=0.10, seed0=0,
                device="cuda", shape="sphere"):
    """Training pairs drawn on the device (see cpdnet_synth): X, Y, V (batch, M, 3);
    shape "sphere" or "bumps"."""
    import torch
    X = torch.empty(batch, M, 3, dtype=torch.float32, device=device)
    Y = torch.empty_like(X)
    V = torch.empty_like(X)
    W = torch.empty_like(X)
    _check(load_library().cpdnet_synth(_ptr(X), _ptr(Y), _ptr(V), _ptr(W), batch, M,
                                       SHAPES[shape], float(beta),
                                       float(coef), float(jitter), float(outlier_frac),
                                       int(seed0), _stream_ptr()))
    return X, Y, V


# ------------------------------------------------------------- convenience
@dataclass
class RegistrationResult:
    Xt: object
    W: object
    iters: int
    converged: bool
    sigma2: float
    t_c: float
    t_eig: float
    t_iter: float
    t_o: float


class Registration:
    """One handle plus its workspace.  X, Y: CUDA tensors (M x D, N x D) of
    the working precision (float64 for 'fp64', float32 otherwise)."""

    def __init__(self, X, Y, stream=None, **kw):
        import torch
        self.params = make_params(X.shape[0], Y.shape[0], X.shape[1], **kw)
        self.dtype = torch.float64 if self.params.precision == CPD_PREC_FP64 else torch.float32
        for t in (X, Y):
            if not t.is_cuda or t.dtype != self.dtype or not t.is_contiguous():
                raise ValueError(f"X, Y must be contiguous {self.dtype} CUDA tensors")
        nbytes = cpd_workspace_size(self.params)
        self.workspace = torch.empty(max(nbytes, 256), dtype=torch.uint8, device=X.device)
        self.stream = stream
        self.h = cpd_init(self.params, X, Y, self.workspace, stream)
        self.M, self.N, self.D = X.shape[0], Y.shape[0], X.shape[1]
        self.device = X.device

    def prepare(self, U=None, lam=None, omega=None):
        """Eigen-prep.  A FULL decomposition cut at its width cap (status
        CPD_NOT_CONVERGED) sets eig_truncated and eig_message and warns."""
        st = cpd_eig_prepare(self.h, U, lam, omega)
        self.eig_truncated = st == CPD_NOT_CONVERGED
        self.eig_message = last_error(self.h) if self.eig_truncated else ""
        if self.eig_truncated:
            import warnings
            warnings.warn(self.eig_message)
        return self

    @property
    def K(self) -> int:
        return cpd_eig_count(self.h)

    def export_eig(self):
        import torch
        K = self.K
        U = torch.empty(self.M, K, dtype=torch.float64, device=self.device)
        lam = torch.empty(K, dtype=torch.float64, device=self.device)
        cpd_eig_export(self.h, U, lam)
        return U, lam

    def step(self):
        return cpd_step(self.h)

    def estep(self):
        import torch
        o = dict(logd=torch.empty(self.N, dtype=self.dtype, device=self.device),
                 P1=torch.empty(self.M, dtype=self.dtype, device=self.device),
                 Yt=torch.empty(self.M, self.D, dtype=self.dtype, device=self.device),
                 tbar=torch.empty(self.M, dtype=self.dtype, device=self.device))
        cpd_estep(self.h, **o)
        return o

    def time_kernels(self, reps=10) -> dict:
        return cpd_time_kernels(self.h, reps)

    def set_state(self, Xt, sigma2):
        cpd_set_state(self.h, Xt, sigma2)

    def state(self):
        import torch
        Xt = torch.empty(self.M, self.D, dtype=self.dtype, device=self.device)
        W = torch.empty_like(Xt)
        s2 = cpd_get_state(self.h, Xt, W)
        return Xt, W, s2

    def matches(self, mutual_only=True):
        """For every scene point the nearest transformed model point (caller's
        rows), -1 for pairs that are not mutual nearest neighbours."""
        import torch
        out = torch.empty(self.N, dtype=torch.int32, device=self.device)
        _check(load_library().cpd_matches(self.h, int(bool(mutual_only)), _ptr(out)), self.h)
        return out

    def solve_matches(self, match, sigma2):
        """The model's transformation from one-to-one correspondences (match:
        M int32 CUDA tensor, scene row or -1): (Xt, W)."""
        import torch
        Xt = torch.empty(self.M, self.D, dtype=self.dtype, device=self.device)
        W = torch.empty_like(Xt)
        _check(load_library().cpd_solve_matches(self.h, _ptr(match), float(sigma2), _ptr(Xt),
                                                _ptr(W)), self.h)
        return Xt, W

    def register(self, W0=None) -> RegistrationResult:
        import torch
        Xt = torch.empty(self.M, self.D, dtype=self.dtype, device=self.device)
        W = torch.empty_like(Xt)
        res, st = cpd_register(self.h, W0, Xt, W)
        return RegistrationResult(Xt, W, res.iters, bool(res.converged), res.sigma2,
                                  res.t_c, res.t_eig, res.t_iter, res.t_o)

    def close(self):
        """Destroy the handle and release its workspace."""
        if getattr(self, "h", None):
            cpd_destroy(self.h)
            self.h = None
        if hasattr(self, "workspace"):
            self.workspace = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def register_two_way(X, Y, stream=None, **kw):
    """Two-way registration for a scene with missing points (Section IV-A):
    register Y onto X, take the mutual-nearest one-to-one correspondences,
    then solve X's transformation from them with sigma^2 from the first
    stage.  kw: Registration parameters (method FAST or CPD-L).  Returns
    (Xt, W, match, first-stage RegistrationResult)."""
    rev = Registration(Y, X, stream=stream, **kw)
    try:
        rev.prepare()
        first = rev.register()
        match = rev.matches(mutual_only=True)
    finally:
        rev.close()
    fwd = Registration(X, Y, stream=stream, **kw)
    try:
        fwd.prepare()
        Xt, W = fwd.solve_matches(match, first.sigma2)
    finally:
        fwd.close()
    return Xt, W, match, first
