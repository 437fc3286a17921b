"""Thin ctypes binding of libmlct.so (include/mlct.h).

Argument marshalling only: every step of the estimator runs in the library's
HIP kernels.  Device buffers are torch tensors on a ROCm device (PyTorch is
used for device memory and streams); their ``data_ptr()`` is passed through.
If the library has not been built this module raises on first use; there is
no fallback implementation.
"""
from __future__ import annotations

import ctypes as C
import os
import weakref

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libmlct.so")

# ---- enumerations (same values as include/mlct.h) -------------------------
MLCT_OK, MLCT_EINVAL, MLCT_ENOMEM, MLCT_EDEVICE = 0, 1, 2, 3
MLCT_ESPECTRUM, MLCT_ERANGE, MLCT_EUNSUPPORTED = 4, 5, 6
STATUS_NAMES = {0: "MLCT_OK", 1: "MLCT_EINVAL", 2: "MLCT_ENOMEM", 3: "MLCT_EDEVICE",
                4: "MLCT_ESPECTRUM", 5: "MLCT_ERANGE", 6: "MLCT_EUNSUPPORTED"}
MLCT_LOG, MLCT_SQRT, MLCT_EXP, MLCT_CUBE, MLCT_INV, MLCT_POW = 0, 1, 2, 3, 4, 5
MLCT_FP64, MLCT_FP32, MLCT_BF16X3 = 0, 1, 2
MLCT_DIRECT, MLCT_DOUBLING = 0, 1
MLCT_LEVEL_INTERP = 0x10
MLCT_DT_F32, MLCT_DT_F64, MLCT_DT_PATTERN = 0, 1, 2
MLCT_PROBE_RADEMACHER, MLCT_PROBE_EXPLICIT = 0, 1
MLCT_MAX_LEVELS = 32
MLCT_EXACT_LOW = 0x20
MLCT_BATCH_PERSISTENT = 0x40
MLCT_BATCH_LOCKSTEP = 0x80
MLCT_FLAG_FEW_SAMPLES, MLCT_FLAG_OVERFLOW, MLCT_FLAG_BF16 = 0x1, 0x2, 0x4
MLCT_KERNEL_CSR_STEP, MLCT_KERNEL_DENSE_STEP, MLCT_KERNEL_TRI_STEP, MLCT_KERNEL_GRAM = 0, 1, 2, 3
MLCT_KERNEL_BATCH_STEP, MLCT_KERNEL_GRAM_CSR_STEP = 4, 5
MLCT_KERNEL_SLQ_SPMM, MLCT_KERNEL_SLQ_UPDATE = 6, 7
MLCT_KERNEL_CALLBACK_STEP = 8
MLCT_KERNEL_CSR_STEP2 = 9
MLCT_OPT_TWO_STEP = 1
MLCT_OPT_WAIT_LIMIT_US = 2
MLCT_OPT_TWO_STEP_LAG = 3
MLCT_OPT_TWO_STEP_ROWS = 4
MLCT_OPT_TWO_STEP_WGS = 5
MLCT_OPT_BATCH_SOLO_ROWS = 6


class mlct_func(C.Structure):
    _fields_ = [("kind", C.c_int32), ("power", C.c_double)]


class mlct_probes(C.Structure):
    _fields_ = [("kind", C.c_int32), ("seed", C.c_uint64), ("first_id", C.c_int64),
                ("m", C.c_int64), ("entries_dev", C.c_void_p), ("ld_entries", C.c_int64)]


class mlct_levels(C.Structure):
    _fields_ = [("L", C.c_int32), ("degree", C.POINTER(C.c_int32)),
                ("m", C.POINTER(C.c_int64))]


class mlct_result(C.Structure):
    _fields_ = [("estimate", C.c_double), ("value", C.c_double), ("log_scale", C.c_double),
                ("est_var", C.c_double),
                ("level_mean", C.c_double * MLCT_MAX_LEVELS),
                ("level_var", C.c_double * MLCT_MAX_LEVELS),
                ("matvecs", C.c_int64), ("probe_degrees", C.c_int64),
                ("max_moment_ratio", C.c_double), ("interval_a", C.c_double),
                ("interval_b", C.c_double), ("flags", C.c_uint32)]


class mlct_tri_result(C.Structure):
    _fields_ = [("sum_w3", C.c_int64), ("estimate", C.c_double), ("estimate_cv", C.c_double),
                ("a1", C.c_double), ("a2", C.c_double)]


class MlctError(RuntimeError):
    def __init__(self, status: int, message: str):
        self.status = status
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {message}")


_lib_handle = None


def lib() -> C.CDLL:
    """The loaded library; raises if it has not been built."""
    global _lib_handle
    if _lib_handle is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(
                f"{LIB_PATH} is missing: build it with `python -m paper_2103_10516_amd.build`"
                " (there is no fallback implementation)")
        h = C.CDLL(LIB_PATH)
        P, I32, I64, U64, D = C.c_void_p, C.c_int32, C.c_int64, C.c_uint64, C.c_double
        sig = {
            "mlct_create": [C.c_int, P, C.c_char_p, C.POINTER(P)],
            "mlct_destroy": [P],
            "mlct_set_workspace_limit": [P, U64],
            "mlct_op_csr": [P, I64, I64, P, P, P, I32, C.POINTER(P)],
            "mlct_op_dense": [P, I64, P, I64, I32, C.POINTER(P)],
            "mlct_op_gram": [P, I64, I64, P, I64, I32, I32, C.POINTER(P)],
            "mlct_op_destroy": [P],
            "mlct_op_read_dense": [P, P, P],
            "mlct_cheb_coeffs": [P, mlct_func, D, D, I32, P, C.POINTER(D)],
            "mlct_moments": [P, P, D, D, I32, C.POINTER(mlct_probes), I32, I32, P],
            "mlct_bounds": [P, P, I32, U64, D, C.POINTER(D), C.POINTER(D)],
            "mlct_lanczos": [P, P, I32, U64, D, P, P, C.POINTER(I32), P],
            "mlct_estimate": [P, P, mlct_func, D, D, C.POINTER(mlct_levels), U64, I32, I32,
                              C.POINTER(mlct_result)],
            "mlct_triangles": [P, P, I64, U64, P, C.POINTER(mlct_tri_result)],
            "mlct_timing": [P, I32],
            "mlct_timing_read": [P, I32, C.POINTER(I64), C.POINTER(D)],
        }
        for name, args in sig.items():
            fn = getattr(h, name)
            fn.argtypes = args
            fn.restype = C.c_int
        h.mlct_last_error.argtypes = [P]
        h.mlct_last_error.restype = C.c_char_p
        _lib_handle = h
    return _lib_handle


def _check(ctx, status: int):
    if status != MLCT_OK:
        msg = lib().mlct_last_error(ctx.handle if ctx is not None else None)
        raise MlctError(status, msg.decode() if msg else "")


def _ptr(t) -> int | None:
    return None if t is None else int(t.data_ptr())


class Context:
    """Owns an mlct_ctx bound to a device and a HIP stream."""

    def __init__(self, device: int = 0, stream=None, tune_cache=None):
        import torch

        if stream is None:
            stream = torch.cuda.current_stream(device)
        self.device = device
        self.stream = stream
        h = C.c_void_p()
        st = lib().mlct_create(device, C.c_void_p(stream.cuda_stream),
                               None if tune_cache is None else str(tune_cache).encode(),
                               C.byref(h))
        if st != MLCT_OK:
            raise MlctError(st, "mlct_create failed")
        self.handle = h
        self._ops = weakref.WeakSet()

    def close(self):
        """Destroy the context; operators created on it are destroyed first."""
        if self.handle:
            for op in list(self._ops):
                op.close()
            lib().mlct_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Op:
    """Operator handle; keeps the tensors it borrows alive."""

    def __init__(self, ctx: Context, handle, keep, d: int):
        self.ctx, self.handle, self._keep, self.d = ctx, handle, keep, d
        ctx._ops.add(self)

    def close(self):
        if self.handle:
            lib().mlct_op_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ---- entry points, same names as the C ABI --------------------------------
def mlct_create(device: int = 0, stream=None, tune_cache=None) -> Context:
    return Context(device, stream, tune_cache)


def mlct_timing(ctx: Context, enable: bool):
    _check(ctx, lib().mlct_timing(ctx.handle, 1 if enable else 0))


def mlct_timing_read(ctx: Context, kernel: int):
    """(launches, total_ms) of one kernel family since timing was enabled."""
    n = C.c_int64()
    ms = C.c_double()
    _check(ctx, lib().mlct_timing_read(ctx.handle, kernel, C.byref(n), C.byref(ms)))
    return n.value, ms.value


def mlct_set_workspace_limit(ctx: Context, nbytes: int):
    _check(ctx, lib().mlct_set_workspace_limit(ctx.handle, int(nbytes)))


def mlct_set_option(ctx: Context, option: int, value: int):
    h = lib()
    h.mlct_set_option.argtypes = [C.c_void_p, C.c_int32, C.c_int64]
    h.mlct_set_option.restype = C.c_int
    _check(ctx, h.mlct_set_option(ctx.handle, option, int(value)))


def mlct_op_csr(ctx: Context, rowptr, col, val=None) -> Op:
    """rowptr int32[d+1], col int32[nnz], val float32[nnz] or None (pattern),
    all device tensors."""
    d = rowptr.numel() - 1
    nnz = col.numel()
    h = C.c_void_p()
    dt = MLCT_DT_PATTERN if val is None else MLCT_DT_F32
    _check(ctx, lib().mlct_op_csr(ctx.handle, d, nnz, _ptr(rowptr), _ptr(col), _ptr(val), dt,
                                  C.byref(h)))
    return Op(ctx, h, (rowptr, col, val), d)


def mlct_cheb_coeffs(ctx: Context, kind: int, a: float, b: float, n: int, power: float = 1.0):
    c = np.empty(n + 1, dtype=np.float64)
    ls = C.c_double()
    _check(ctx, lib().mlct_cheb_coeffs(ctx.handle, mlct_func(kind, power), a, b, n,
                                       c.ctypes.data, C.byref(ls)))
    return c, ls.value


def rademacher_probes(seed: int, m: int, first_id: int = 0) -> mlct_probes:
    return mlct_probes(MLCT_PROBE_RADEMACHER, seed & ((1 << 64) - 1), first_id, m, None, 0)


def explicit_probes(entries, m: int | None = None, first_id: int = 0) -> mlct_probes:
    """entries: device int8 tensor [d, ld] (probe index fastest)."""
    ld = entries.shape[1]
    m = ld - first_id if m is None else m
    p = mlct_probes(MLCT_PROBE_EXPLICIT, 0, first_id, m, _ptr(entries), ld)
    p._keep = entries
    return p


def mlct_moments(ctx: Context, op: Op, a: float, b: float, n: int, probes: mlct_probes,
                 prec: int = MLCT_FP32, mode: int = MLCT_DIRECT) -> np.ndarray:
    mu = np.empty((probes.m, n + 1), dtype=np.float64)
    _check(ctx, lib().mlct_moments(ctx.handle, op.handle, a, b, n, C.byref(probes), prec, mode,
                                   mu.ctypes.data))
    return mu


def mlct_estimate(ctx: Context, op: Op, kind: int, a: float, b: float, degrees, m, seed: int,
                  prec: int = MLCT_FP32, mode: int = MLCT_DIRECT, power: float = 1.0) -> dict:
    L = len(degrees)
    deg = (C.c_int32 * L)(*[int(x) for x in degrees])
    mm = (C.c_int64 * L)(*[int(x) for x in m])
    lv = mlct_levels(L, deg, mm)
    r = mlct_result()
    _check(ctx, lib().mlct_estimate(ctx.handle, op.handle, mlct_func(kind, power), a, b,
                                    C.byref(lv), seed & ((1 << 64) - 1), prec, mode, C.byref(r)))
    return {
        "estimate": r.estimate, "value": r.value, "log_scale": r.log_scale,
        "est_var": r.est_var, "level_mean": np.array(r.level_mean[:L]),
        "level_var": np.array(r.level_var[:L]), "matvecs": r.matvecs,
        "probe_degrees": r.probe_degrees, "max_moment_ratio": r.max_moment_ratio,
        "interval": (r.interval_a, r.interval_b), "flags": r.flags,
    }


def mlct_triangles(ctx: Context, op: Op, m: int, seed: int, want_w: bool = True):
    """Triangle-count estimate over a pattern CSR operator.  Returns
    (result dict, w int64 [m, 3] or None)."""
    r = mlct_tri_result()
    w = np.empty((m, 3), dtype=np.int64) if want_w else None
    _check(ctx, lib().mlct_triangles(ctx.handle, op.handle, m, seed & ((1 << 64) - 1),
                                     None if w is None else w.ctypes.data, C.byref(r)))
    return {"sum_w3": r.sum_w3, "estimate": r.estimate, "estimate_cv": r.estimate_cv,
            "a1": r.a1, "a2": r.a2}, w


def mlct_op_dense(ctx: Context, A) -> Op:
    """Dense symmetric A: device tensor [d, lda >= d] float32 or float64."""
    import torch

    d = A.shape[0]
    dt = MLCT_DT_F64 if A.dtype == torch.float64 else MLCT_DT_F32
    h = C.c_void_p()
    _check(ctx, lib().mlct_op_dense(ctx.handle, d, _ptr(A), A.stride(0), dt, C.byref(h)))
    return Op(ctx, h, (A,), d)


def mlct_op_gram(ctx: Context, X, prec: int = MLCT_FP32) -> Op:
    """A = X^T X for a device float32 tensor X [rows, cols] (formed on the device)."""
    rows, cols = X.shape
    h = C.c_void_p()
    _check(ctx, lib().mlct_op_gram(ctx.handle, rows, cols, _ptr(X), X.stride(0), MLCT_DT_F32,
                                   prec, C.byref(h)))
    return Op(ctx, h, (X,), cols)


def mlct_op_read_dense(ctx: Context, op: Op) -> np.ndarray:
    out = np.empty((op.d, op.d), dtype=np.float64)
    _check(ctx, lib().mlct_op_read_dense(ctx.handle, op.handle, out.ctypes.data))
    return out


def mlct_bounds(ctx: Context, op: Op, steps: int = 64, seed: int = 0, rel_margin: float = 0.01):
    a, b = C.c_double(), C.c_double()
    _check(ctx, lib().mlct_bounds(ctx.handle, op.handle, steps, seed & ((1 << 64) - 1),
                                  rel_margin, C.byref(a), C.byref(b)))
    return a.value, b.value


def mlct_lanczos(ctx: Context, op: Op, steps: int = 64, seed: int = 0, rel_margin: float = 0.01):
    """(alpha[k], beta[k], info dict) of the Lanczos run behind mlct_bounds."""
    al = np.zeros(steps)
    be = np.zeros(steps)
    k = C.c_int32()
    info = np.zeros(6)
    _check(ctx, lib().mlct_lanczos(ctx.handle, op.handle, steps, seed & ((1 << 64) - 1),
                                   rel_margin, al.ctypes.data, be.ctypes.data, C.byref(k),
                                   info.ctypes.data))
    n = k.value
    return al[:n], be[:n], {"theta_min": info[0], "theta_max": info[1], "r_min": info[2],
                            "r_max": info[3], "a": info[4], "b": info[5]}


# ---- learned control-variate level ------------------------------------------
class mlct_mlp_cfg(C.Structure):
    _fields_ = [("epochs", C.c_int32), ("lr", C.c_float), ("train_fraction", C.c_double),
                ("init_seed", C.c_uint64)]


class mlct_mlp_info(C.Structure):
    _fields_ = [("var_q", C.c_double), ("var_resid", C.c_double), ("mean_resid", C.c_double),
                ("var_g", C.c_double), ("ybar", C.c_double), ("ysd", C.c_double), ("final_loss", C.c_double),
                ("fallback", C.c_int32), ("n_features", C.c_int32), ("n_cheap", C.c_int32),
                ("n_fine", C.c_int32), ("ntrain", C.c_int64), ("nval", C.c_int64),
                ("nparams", C.c_int64), ("x_mean", C.c_double * 16), ("x_sd", C.c_double * 16),
                ("lin", C.c_double * 16)]


MLCT_FLAG_LEARNED_FALLBACK = 0x8

_MLP_SIGS = {
    "mlct_learned_fit": [C.c_void_p, C.c_void_p, mlct_func, C.c_double, C.c_double, C.c_int32,
                         C.c_int32, C.c_int64, C.c_uint64, C.c_int32, C.POINTER(mlct_mlp_cfg),
                         C.POINTER(C.c_void_p)],
    "mlct_estimate_learned": [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int64, C.c_int64,
                              C.c_uint64, C.POINTER(mlct_result)],
    "mlct_mlp_info_get": [C.c_void_p, C.POINTER(mlct_mlp_info)],
    "mlct_mlp_loss_history": [C.c_void_p, C.c_void_p, C.c_int32, C.POINTER(C.c_int32)],
    "mlct_mlp_weights": [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p],
    "mlct_mlp_grad": [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_int32, C.c_void_p,
                      C.POINTER(C.c_float)],
    "mlct_mlp_destroy": [C.c_void_p],
}


def _mlp_lib():
    h = lib()
    if not getattr(h, "_mlp_sigs_set", False):
        for name, args in _MLP_SIGS.items():
            fn = getattr(h, name)
            fn.argtypes = args
            fn.restype = C.c_int
        h._mlp_sigs_set = True
    return h


class Mlp:
    """Trained learned level (owns an mlct_mlp)."""

    def __init__(self, ctx: Context, handle):
        self.ctx, self.handle = ctx, handle
        ctx._ops.add(self)

    def close(self):
        if self.handle:
            _mlp_lib().mlct_mlp_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def mlct_learned_fit(ctx: Context, op: Op, kind: int, a: float, b: float, n_fine: int = 256,
                     n_cheap: int = 8, m_pilot: int = 2048, seed: int = 1,
                     prec: int = MLCT_FP32, epochs: int = 2000, lr: float = 1e-3,
                     train_fraction: float = 0.75, init_seed: int = 0,
                     power: float = 1.0) -> Mlp:
    cfg = mlct_mlp_cfg(epochs, lr, train_fraction, init_seed & ((1 << 64) - 1))
    h = C.c_void_p()
    _check(ctx, _mlp_lib().mlct_learned_fit(ctx.handle, op.handle, mlct_func(kind, power), a, b,
                                            n_fine, n_cheap, m_pilot, seed & ((1 << 64) - 1),
                                            prec, C.byref(cfg), C.byref(h)))
    return Mlp(ctx, h)


def mlct_estimate_learned(ctx: Context, op: Op, mlp: Mlp, M0: int, M1: int, seed: int) -> dict:
    r = mlct_result()
    _check(ctx, _mlp_lib().mlct_estimate_learned(ctx.handle, op.handle, mlp.handle, M0, M1,
                                                 seed & ((1 << 64) - 1), C.byref(r)))
    return _result_dict(r, 2)


def mlct_mlp_info_get(mlp: Mlp) -> dict:
    i = mlct_mlp_info()
    st = _mlp_lib().mlct_mlp_info_get(mlp.handle, C.byref(i))
    if st != MLCT_OK:
        raise MlctError(st, "mlct_mlp_info_get failed")
    return {k: (np.array(getattr(i, k)) if k in ("x_mean", "x_sd", "lin") else getattr(i, k))
            for k, _ in mlct_mlp_info._fields_}


def mlct_mlp_loss_history(mlp: Mlp) -> np.ndarray:
    n = C.c_int32()
    _mlp_lib().mlct_mlp_loss_history(mlp.handle, None, 0, C.byref(n))
    out = np.empty(n.value, dtype=np.float32)
    _mlp_lib().mlct_mlp_loss_history(mlp.handle, out.ctypes.data, n.value, None)
    return out


def mlct_mlp_weights(ctx: Context, mlp: Mlp, set_to=None) -> np.ndarray:
    P = mlct_mlp_info_get(mlp)["nparams"]
    out = np.empty(P, dtype=np.float32)
    src = None
    if set_to is not None:
        src = np.ascontiguousarray(set_to, dtype=np.float32)
        assert src.size == P
    _check(ctx, _mlp_lib().mlct_mlp_weights(ctx.handle, mlp.handle, out.ctypes.data,
                                            None if src is None else src.ctypes.data))
    return out


def mlct_mlp_grad(ctx: Context, mlp: Mlp, X, y):
    X = np.ascontiguousarray(X, dtype=np.float32)
    y = np.ascontiguousarray(y, dtype=np.float32)
    P = mlct_mlp_info_get(mlp)["nparams"]
    g = np.empty(P, dtype=np.float32)
    loss = C.c_float()
    _check(ctx, _mlp_lib().mlct_mlp_grad(ctx.handle, mlp.handle, X.ctypes.data, y.ctypes.data,
                                         X.shape[0], g.ctypes.data, C.byref(loss)))
    return g, loss.value


# ---- batched estimates --------------------------------------------------------
class mlct_batch_item(C.Structure):
    _fields_ = [("op", C.c_void_p), ("f", mlct_func), ("a", C.c_double), ("b", C.c_double),
                ("levels", mlct_levels), ("seed", C.c_uint64)]


def _batch_items(items):
    n = len(items)
    arr = (mlct_batch_item * n)()
    keep = []
    for i, it in enumerate(items):
        L = len(it["degrees"])
        deg = (C.c_int32 * L)(*[int(x) for x in it["degrees"]])
        mm = (C.c_int64 * L)(*[int(x) for x in it["m"]])
        keep += [deg, mm]
        arr[i] = mlct_batch_item(it["op"].handle, mlct_func(it["kind"], it.get("power", 1.0)),
                                 it["a"], it["b"], mlct_levels(L, deg, mm),
                                 it["seed"] & ((1 << 64) - 1))
    return arr, keep


def mlct_autotune_batch(ctx: Context, items, prec: int = MLCT_FP32,
                        mode: int = MLCT_DOUBLING) -> int:
    """Times both batch launch forms on these items; returns 1 if the
    persistent launch was faster (the context then uses it by default)."""
    h = lib()
    h.mlct_autotune_batch.argtypes = [C.c_void_p, C.c_int32, C.POINTER(mlct_batch_item),
                                      C.c_int32, C.c_int32, C.POINTER(C.c_int32)]
    h.mlct_autotune_batch.restype = C.c_int
    arr, keep = _batch_items(items)
    ch = C.c_int32()
    _check(ctx, h.mlct_autotune_batch(ctx.handle, len(items), arr, prec, mode, C.byref(ch)))
    return ch.value


def mlct_estimate_batch(ctx: Context, items, prec: int = MLCT_FP32, mode: int = MLCT_DOUBLING):
    """items: list of dicts with keys op, kind, a, b, degrees, m, seed (power
    optional).  Returns one result dict per item."""
    h = lib()
    if not getattr(h, "_batch_sig", False):
        h.mlct_estimate_batch.argtypes = [C.c_void_p, C.c_int32, C.POINTER(mlct_batch_item),
                                          C.c_int32, C.c_int32, C.POINTER(mlct_result)]
        h.mlct_estimate_batch.restype = C.c_int
        h._batch_sig = True
    n = len(items)
    arr = (mlct_batch_item * n)()
    keep = []
    for i, it in enumerate(items):
        L = len(it["degrees"])
        deg = (C.c_int32 * L)(*[int(x) for x in it["degrees"]])
        mm = (C.c_int64 * L)(*[int(x) for x in it["m"]])
        keep += [deg, mm]
        arr[i] = mlct_batch_item(it["op"].handle, mlct_func(it["kind"], it.get("power", 1.0)),
                                 it["a"], it["b"], mlct_levels(L, deg, mm),
                                 it["seed"] & ((1 << 64) - 1))
    outs = (mlct_result * n)()
    _check(ctx, h.mlct_estimate_batch(ctx.handle, n, arr, prec, mode, outs))
    res = []
    for i, it in enumerate(items):
        r = outs[i]
        L = len(it["degrees"])
        res.append({"estimate": r.estimate, "value": r.value, "log_scale": r.log_scale,
                    "est_var": r.est_var, "level_mean": np.array(r.level_mean[:L]),
                    "level_var": np.array(r.level_var[:L]), "matvecs": r.matvecs,
                    "probe_degrees": r.probe_degrees, "flags": r.flags})
    return res


def mlct_autotune(ctx: Context, op: Op, B_max: int = 64, prec: int = MLCT_FP32) -> int:
    h = lib()
    h.mlct_autotune.argtypes = [C.c_void_p, C.c_void_p, C.c_int32, C.c_int32, C.POINTER(C.c_int32)]
    h.mlct_autotune.restype = C.c_int
    c = C.c_int32()
    _check(ctx, h.mlct_autotune(ctx.handle, op.handle, B_max, prec, C.byref(c)))
    return c.value


# ---- automatic level selection ------------------------------------------------
MLCT_TARGET_VARIANCE = 0
MLCT_TARGET_BUDGET = 1
MLCT_MAX_PLAN_DEGREE = 1024


class mlct_level_plan(C.Structure):
    _fields_ = [("L", C.c_int32), ("degree", C.c_int32 * MLCT_MAX_LEVELS),
                ("m", C.c_int64 * MLCT_MAX_LEVELS), ("var", C.c_double * MLCT_MAX_LEVELS),
                ("cost", C.c_double * MLCT_MAX_LEVELS), ("m_real", C.c_double * MLCT_MAX_LEVELS),
                ("opt_total", C.c_double), ("single_total", C.c_double),
                ("predicted_var", C.c_double), ("predicted_cost", C.c_double)]


def _plan_dict(p: mlct_level_plan) -> dict:
    L = p.L
    return {"L": L, "degrees": list(p.degree[:L]), "m": list(p.m[:L]),
            "var": np.array(p.var[:L]), "cost": np.array(p.cost[:L]),
            "m_real": np.array(p.m_real[:L]), "opt_total": p.opt_total,
            "single_total": p.single_total, "predicted_var": p.predicted_var,
            "predicted_cost": p.predicted_cost}


def mlct_plan_levels(ctx: Context, terms: np.ndarray, mode: int, target: float,
                     target_kind: int = MLCT_TARGET_VARIANCE, min_top: int = 0) -> dict:
    """terms: host FP64 array m_pilot x (n+1)."""
    t = np.ascontiguousarray(terms, dtype=np.float64)
    m, n1 = t.shape
    h = lib()
    h.mlct_plan_levels.argtypes = [C.c_void_p, C.c_void_p, C.c_int64, C.c_int32, C.c_int32,
                                   C.c_double, C.c_int32, C.c_int64, C.POINTER(mlct_level_plan)]
    h.mlct_plan_levels.restype = C.c_int
    p = mlct_level_plan()
    _check(ctx, h.mlct_plan_levels(ctx.handle, t.ctypes.data, m, n1 - 1, mode, target,
                                   target_kind, min_top, C.byref(p)))
    return _plan_dict(p)


def mlct_select_levels(ctx: Context, op: Op, kind: int, a: float, b: float, n: int,
                       m_pilot: int, seed: int, prec: int = MLCT_FP32,
                       mode: int = MLCT_DOUBLING, target: float = 1.0,
                       target_kind: int = MLCT_TARGET_VARIANCE, power: float = 1.0,
                       return_moments: bool = False):
    h = lib()
    h.mlct_select_levels.argtypes = [C.c_void_p, C.c_void_p, mlct_func, C.c_double, C.c_double,
                                     C.c_int32, C.c_int64, C.c_uint64, C.c_int32, C.c_int32,
                                     C.c_double, C.c_int32, C.POINTER(mlct_level_plan),
                                     C.c_void_p]
    h.mlct_select_levels.restype = C.c_int
    p = mlct_level_plan()
    mu = np.empty((m_pilot, n + 1), dtype=np.float64) if return_moments else None
    _check(ctx, h.mlct_select_levels(ctx.handle, op.handle, mlct_func(kind, power), a, b, n,
                                     m_pilot, seed & ((1 << 64) - 1), prec, mode, target,
                                     target_kind, C.byref(p),
                                     mu.ctypes.data if mu is not None else None))
    d = _plan_dict(p)
    return (d, mu) if return_moments else d


def mlct_estimate_auto(ctx: Context, op: Op, kind: int, a: float, b: float, n: int, m_pilot: int,
                       seed: int, prec: int = MLCT_FP32, mode: int = MLCT_DOUBLING,
                       target: float = 1.0, target_kind: int = MLCT_TARGET_VARIANCE,
                       power: float = 1.0):
    """(result dict, plan dict)."""
    h = lib()
    h.mlct_estimate_auto.argtypes = [C.c_void_p, C.c_void_p, mlct_func, C.c_double, C.c_double,
                                     C.c_int32, C.c_int64, C.c_uint64, C.c_int32, C.c_int32,
                                     C.c_double, C.c_int32, C.POINTER(mlct_level_plan),
                                     C.POINTER(mlct_result)]
    h.mlct_estimate_auto.restype = C.c_int
    p = mlct_level_plan()
    r = mlct_result()
    _check(ctx, h.mlct_estimate_auto(ctx.handle, op.handle, mlct_func(kind, power), a, b, n,
                                     m_pilot, seed & ((1 << 64) - 1), prec, mode, target,
                                     target_kind, C.byref(p), C.byref(r)))
    L = p.L
    res = {"estimate": r.estimate, "value": r.value, "log_scale": r.log_scale,
           "est_var": r.est_var, "level_mean": np.array(r.level_mean[:L]),
           "level_var": np.array(r.level_var[:L]), "matvecs": r.matvecs,
           "probe_degrees": r.probe_degrees, "max_moment_ratio": r.max_moment_ratio,
           "interval": (r.interval_a, r.interval_b), "flags": r.flags}
    return res, _plan_dict(p)


def mlct_op_gram_csr(ctx: Context, rowptr, col, val, cols: int, lam: float = 0.0) -> Op:
    """A = X^T X + lam I for X a device CSR (rowptr int32[rows+1], col
    int32[nnz] in [0, cols), val float32[nnz] or None for a pattern)."""
    rows = rowptr.numel() - 1
    nnz = col.numel()
    h = lib()
    h.mlct_op_gram_csr.argtypes = [C.c_void_p, C.c_int64, C.c_int64, C.c_int64, C.c_void_p,
                                   C.c_void_p, C.c_void_p, C.c_double, C.POINTER(C.c_void_p)]
    h.mlct_op_gram_csr.restype = C.c_int
    hd = C.c_void_p()
    _check(ctx, h.mlct_op_gram_csr(ctx.handle, rows, cols, nnz, _ptr(rowptr), _ptr(col),
                                   _ptr(val), lam, C.byref(hd)))
    return Op(ctx, hd, (rowptr, col, val), cols)


# ---- stochastic Lanczos quadrature ------------------------------------------------
def mlct_slq_quadforms(ctx: Context, op: Op, kind: int, k: int, probes: mlct_probes,
                       power: float = 1.0) -> np.ndarray:
    h = lib()
    h.mlct_slq_quadforms.argtypes = [C.c_void_p, C.c_void_p, mlct_func, C.c_int32,
                                     C.POINTER(mlct_probes), C.c_void_p]
    h.mlct_slq_quadforms.restype = C.c_int
    q = np.empty(probes.m, dtype=np.float64)
    _check(ctx, h.mlct_slq_quadforms(ctx.handle, op.handle, mlct_func(kind, power), k,
                                     C.byref(probes), q.ctypes.data))
    return q


def mlct_estimate_slq(ctx: Context, op: Op, kind: int, a: float, b: float, cheb_degree: int,
                      m0: int, k: int, m1: int, seed: int, prec: int = MLCT_FP64,
                      mode: int = MLCT_DOUBLING, power: float = 1.0) -> dict:
    h = lib()
    h.mlct_estimate_slq.argtypes = [C.c_void_p, C.c_void_p, mlct_func, C.c_double, C.c_double,
                                    C.c_int32, C.c_int64, C.c_int32, C.c_int64, C.c_uint64,
                                    C.c_int32, C.c_int32, C.POINTER(mlct_result)]
    h.mlct_estimate_slq.restype = C.c_int
    r = mlct_result()
    _check(ctx, h.mlct_estimate_slq(ctx.handle, op.handle, mlct_func(kind, power), a, b,
                                    cheb_degree, m0, k, m1, seed & ((1 << 64) - 1), prec, mode,
                                    C.byref(r)))
    return {"estimate": r.estimate, "value": r.value, "log_scale": r.log_scale,
            "est_var": r.est_var, "level_mean": np.array(r.level_mean[:2]),
            "level_var": np.array(r.level_var[:2]), "matvecs": r.matvecs,
            "probe_degrees": r.probe_degrees, "interval": (r.interval_a, r.interval_b),
            "flags": r.flags}


def _result_dict(r: mlct_result, L: int) -> dict:
    return {"estimate": r.estimate, "value": r.value, "log_scale": r.log_scale,
            "est_var": r.est_var, "level_mean": np.array(r.level_mean[:L]),
            "level_var": np.array(r.level_var[:L]), "matvecs": r.matvecs,
            "probe_degrees": r.probe_degrees, "max_moment_ratio": r.max_moment_ratio,
            "interval": (r.interval_a, r.interval_b), "flags": r.flags}


def mlct_learned_eval(ctx: Context, op: Op, mlp: Mlp, probes: mlct_probes, fine: bool = False):
    """Per-probe g (and, with fine=True, q = z^T p_n z) of the learned level.
    Returns (g, q) with q None unless fine."""
    h = _mlp_lib()
    h.mlct_learned_eval.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p, C.POINTER(mlct_probes),
                                    C.c_int32, C.c_void_p, C.c_void_p]
    h.mlct_learned_eval.restype = C.c_int
    g = np.empty(probes.m, dtype=np.float64)
    q = np.empty(probes.m, dtype=np.float64) if fine else None
    _check(ctx, h.mlct_learned_eval(ctx.handle, op.handle, mlp.handle, C.byref(probes),
                                    1 if fine else 0, g.ctypes.data,
                                    q.ctypes.data if fine else None))
    return g, q


def mlct_estimate_learned_ml(ctx: Context, op: Op, mlp: Mlp, degrees, m, seed: int) -> dict:
    """Multilevel estimate with the learned level g at degree n_cheap in the
    chain (see include/mlct.h)."""
    h = _mlp_lib()
    h.mlct_estimate_learned_ml.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p,
                                           C.POINTER(mlct_levels), C.c_uint64,
                                           C.POINTER(mlct_result)]
    h.mlct_estimate_learned_ml.restype = C.c_int
    L = len(degrees)
    deg = (C.c_int32 * L)(*[int(x) for x in degrees])
    mm = (C.c_int64 * L)(*[int(x) for x in m])
    lv = mlct_levels(L, deg, mm)
    r = mlct_result()
    _check(ctx, h.mlct_estimate_learned_ml(ctx.handle, op.handle, mlp.handle, C.byref(lv),
                                           seed & ((1 << 64) - 1), C.byref(r)))
    return _result_dict(r, L)


def mlct_learned_plan(ctx: Context, mlp: Mlp, target: float,
                      target_kind: int = MLCT_TARGET_VARIANCE) -> dict:
    """Levels and sample sizes for mlct_estimate_learned_ml from the fit's
    held-out pilot probes."""
    h = _mlp_lib()
    h.mlct_learned_plan.argtypes = [C.c_void_p, C.c_void_p, C.c_double, C.c_int32,
                                    C.POINTER(mlct_level_plan)]
    h.mlct_learned_plan.restype = C.c_int
    p = mlct_level_plan()
    _check(ctx, h.mlct_learned_plan(ctx.handle, mlp.handle, target, target_kind, C.byref(p)))
    return _plan_dict(p)


def mlct_moments_noalloc(ctx: Context, op: Op, a: float, b: float, n: int, probes: mlct_probes,
                         prec: int = MLCT_FP32, mode: int = MLCT_DIRECT, out=None):
    """mlct_moments into a device tensor (m x (n+1) float64) without any
    allocation inside the library; ``out`` may be given (then nothing at all
    is allocated here either).  The work is enqueued on the context stream."""
    import torch

    h = lib()
    h.mlct_moments_noalloc.argtypes = [C.c_void_p, C.c_void_p, C.c_double, C.c_double, C.c_int32,
                                       C.POINTER(mlct_probes), C.c_int32, C.c_int32, C.c_void_p]
    h.mlct_moments_noalloc.restype = C.c_int
    if out is None:
        out = torch.empty((probes.m, n + 1), dtype=torch.float64, device=f"cuda:{ctx.device}")
    if out.dtype != torch.float64 or not out.is_cuda or not out.is_contiguous() or \
            out.numel() < probes.m * (n + 1):
        raise ValueError("out must be a contiguous float64 device tensor of m x (n+1)")
    _check(ctx, h.mlct_moments_noalloc(ctx.handle, op.handle, a, b, n, C.byref(probes), prec, mode,
                                       out.data_ptr()))
    return out


# int32 apply(void* user, const float* V, float* AV, int64 B, void* hip_stream)
MLCT_APPLY_FN = C.CFUNCTYPE(C.c_int32, C.c_void_p, C.c_void_p, C.c_void_p, C.c_int64, C.c_void_p)


class _DeviceArray:
    """A borrowed device buffer presented to torch.as_tensor (no copy)."""

    def __init__(self, ptr: int, shape, typestr: str):
        self.__cuda_array_interface__ = {"shape": tuple(shape), "typestr": typestr,
                                         "data": (int(ptr), False), "version": 2,
                                         "strides": None}


def mlct_op_callback(ctx: Context, d: int, apply) -> Op:
    """Matrix-free operator.  ``apply(V, AV)`` receives two float32 device
    tensors of shape (d, B) that view the library's buffers (valid during
    the call only) and must write A @ V into AV on the current stream (the
    context's stream).  Any exception fails the library call."""
    import torch

    def tramp(user, v_ptr, av_ptr, B, stream):
        try:
            V = torch.as_tensor(_DeviceArray(v_ptr, (d, B), "<f4"), device=f"cuda:{ctx.device}")
            AV = torch.as_tensor(_DeviceArray(av_ptr, (d, B), "<f4"), device=f"cuda:{ctx.device}")
            apply(V, AV)
            return 0
        except Exception:  # reported as MLCT_EDEVICE by the library
            import traceback

            traceback.print_exc()
            return 1

    fn = MLCT_APPLY_FN(tramp)
    h = lib()
    h.mlct_op_callback.argtypes = [C.c_void_p, C.c_int64, MLCT_APPLY_FN, C.c_void_p,
                                   C.POINTER(C.c_void_p)]
    h.mlct_op_callback.restype = C.c_int
    out = C.c_void_p()
    _check(ctx, h.mlct_op_callback(ctx.handle, d, fn, None, C.byref(out)))
    return Op(ctx, out, (fn, apply), d)
