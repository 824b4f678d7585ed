"""ctypes binding of libqs (include/qs.h): argument marshalling only.

Every function keeps the C name and forwards to the library; every step of the gate path runs in the HIP
kernels behind it. PyTorch supplies device memory and streams (``torch.cuda``); it does no state arithmetic.
The binding fails loudly (ImportError / QSError) when libqs.so is missing: there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence

import numpy as np

PKG = os.path.dirname(os.path.abspath(__file__))
# QS_LIBQS selects another build of the same library (the sanitizer build of build.py --sanitize)
LIB_PATH = os.environ.get("QS_LIBQS") or os.path.join(PKG, "libqs.so")

QS_OK, QS_EINVAL, QS_ENOMEM, QS_EDEVICE, QS_EUNSUPPORTED = 0, -1, -2, -3, -4
QS_C128, QS_C64 = 0, 1
QS_MAX_K, QS_MAX_DIAG_K, QS_MAX_CONTROLS, QS_MAX_QUBITS = 6, 12, 16, 40
QS_PLAN_BLOCK, QS_PLAN_FUSE, QS_PLAN_REMAP = 0, 1, 2
QS_RUN_SCALE_FIRST, QS_RUN_NORM_LAST = 1, 2
QS_PLAN_NFEAT = 48


class qs_plan_opts(ctypes.Structure):
    _fields_ = [("mode", ctypes.c_int), ("block_bits", ctypes.c_int), ("low_bits", ctypes.c_int),
                ("dtype", ctypes.c_int)]


class qs_plan_model(ctypes.Structure):
    _fields_ = [("model", ctypes.c_void_p), ("mean", ctypes.POINTER(ctypes.c_float)),
                ("std", ctypes.POINTER(ctypes.c_float)), ("nshapes", ctypes.c_int),
                ("shape_bits", ctypes.POINTER(ctypes.c_int)), ("shape_low", ctypes.POINTER(ctypes.c_int)),
                ("per_shape", ctypes.c_int), ("gate_slack", ctypes.c_int), ("lookahead", ctypes.c_int)]


_lib = None


class QSError(RuntimeError):
    def __init__(self, code: int, fn: str, msg: str):
        super().__init__(f"{fn} -> {code}: {msg}")
        self.code = code


_P = ctypes.c_void_p
_I = ctypes.c_int
_IP = ctypes.POINTER(ctypes.c_int)
_DP = ctypes.POINTER(ctypes.c_double)

# name -> argtypes (all return int unless listed in _RESTYPES)
SIGNATURES = {
    "qs_alloc": [ctypes.POINTER(_P), _I, _I, _P, _P],
    "qs_free": [_P],
    "qs_apply_gate": [_P, _IP, _I, _DP],
    "qs_apply_diag": [_P, _IP, _I, _DP],
    "qs_apply_controlled": [_P, _IP, _I, _IP, _I, _DP],
    "qs_fused_swap": [_P, _I, _I, _I],
    "qs_probs": [_P, _P, _DP],
    "qs_probs_noalloc": [_P, _I, _I, _P, _P, _P],
    "qs_init_zero": [_P],
    "qs_copy_in": [_P, _P],
    "qs_copy_out": [_P, _P],
    "qs_sync": [_P],
    "qs_scale": [_P, ctypes.c_double],
    "qs_norm": [_P, _DP],
    "qs_renormalize": [_P, _DP],
    "qs_get_info": [_P, _IP, _IP, ctypes.POINTER(_P), ctypes.POINTER(_P)],
    "qs_last_error": [],
    "qs_probe_copy": [_P, _P, ctypes.c_size_t, _P],
    "qs_probe_rmw": [_P, ctypes.c_size_t, _P],
    "qs_set_tunable": [ctypes.c_char_p, ctypes.c_int64],
    "qs_get_tunable": [ctypes.c_char_p, ctypes.POINTER(ctypes.c_int64)],
    "qs_circuit_create": [ctypes.POINTER(_P), _I],
    "qs_circuit_free": [_P],
    "qs_circuit_add_gate": [_P, _IP, _I, _DP],
    "qs_circuit_add_diag": [_P, _IP, _I, _DP],
    "qs_circuit_add_controlled": [_P, _IP, _I, _IP, _I, _DP],
    "qs_circuit_add_fused_swap": [_P, _I, _I, _I],
    "qs_circuit_size": [_P, _IP],
    "qs_circuit_run": [_P, _P],
    "qs_plan_create": [ctypes.POINTER(_P), _P, _P],
    "qs_plan_create_learned": [ctypes.POINTER(_P), _P, _P, _P],
    "qs_plan_run": [_P, _P],
    "qs_plan_run_range": [_P, _P, _I, _I],
    "qs_plan_run_renorm": [_P, _P, _I],
    "qs_plan_run_range_renorm": [_P, _P, _I, _I, _I],
    "qs_renormalize_pending": [_P, _DP],
    "qs_plan_info": [_P, _IP, _IP, _IP, _IP, _IP],
    "qs_plan_pass_info": [_P, _I, _IP, _IP, ctypes.POINTER(ctypes.c_int64), _IP, _IP],
    "qs_plan_pass_gates": [_P, _I, _IP, _I, _IP],
    "qs_plan_free": [_P],
    "qs_plan_features": [_P, _I, ctypes.POINTER(ctypes.c_float)],
    "qs_batch_create": [ctypes.POINTER(_P), _I, _I, _I, _I, _P],
    "qs_batch_add": [_P, _P],
    "qs_batch_finalize": [_P],
    "qs_batch_run": [_P, _I],
    "qs_batch_info": [_P, _IP, ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int64), _IP, _IP],
    "qs_batch_probs": [_P, _I, ctypes.POINTER(_P), _DP],
    "qs_batch_free": [_P],
    "qs_measure": [_P, _I, ctypes.c_double, _IP, _DP],
    "qs_reset": [_P, _I, ctypes.c_double, _IP],
    "qs_sample": [_P, ctypes.c_int64, _DP, ctypes.POINTER(ctypes.c_int64)],
    "qs_batch_set_launch": [_P, _I],
    "qs_mlp_create": [ctypes.POINTER(_P), _I, _I, _P],
    "qs_mlp_free": [_P],
    "qs_mlp_num_params": [_P, _IP],
    "qs_mlp_set_params": [_P, ctypes.POINTER(ctypes.c_float)],
    "qs_mlp_get_params": [_P, ctypes.POINTER(ctypes.c_float)],
    "qs_mlp_predict": [_P, ctypes.POINTER(ctypes.c_float), _I, ctypes.POINTER(ctypes.c_float)],
    "qs_mlp_grad": [_P, ctypes.POINTER(ctypes.c_float), ctypes.POINTER(ctypes.c_float), _I,
                    ctypes.POINTER(ctypes.c_float), ctypes.POINTER(ctypes.c_float)],
    "qs_mlp_train_step": [_P, ctypes.POINTER(ctypes.c_float), ctypes.POINTER(ctypes.c_float), _I, ctypes.c_float,
                          ctypes.POINTER(ctypes.c_float)],
}
_RESTYPES = {"qs_last_error": ctypes.c_char_p}


def lib():
    """Load libqs.so (raises ImportError if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"libqs.so not found at {LIB_PATH}; run __graft_entry__.build() "
                              "(python paper_2203_16044_amd/build.py) first")
        L = ctypes.CDLL(LIB_PATH)
        for name, args in SIGNATURES.items():
            fn = getattr(L, name)
            fn.argtypes = args
            fn.restype = _RESTYPES.get(name, ctypes.c_int)
        _lib = L
    return _lib


def _check(rc: int, fn: str) -> int:
    if rc != QS_OK:
        raise QSError(rc, fn, lib().qs_last_error().decode())
    return rc


def _ints(v: Sequence[int]):
    v = [int(x) for x in v]
    return (ctypes.c_int * max(1, len(v)))(*v)


def _mat(m, k: int, diag: bool = False) -> np.ndarray:
    """The matrix (or diagonal) as contiguous complex128, checked against the target count: the C ABI
    reads exactly 2^k x 2^k (or 2^k) entries from the pointer it is given."""
    a = np.ascontiguousarray(np.asarray(m, dtype=np.complex128))
    want = (1 << k,) if diag else (1 << k, 1 << k)
    if a.shape != want:
        raise ValueError(f"matrix shape {a.shape} does not match {k} target(s): expected {want}")
    return a


def _dptr(a: np.ndarray):
    return a.ctypes.data_as(_DP)


# ------------------------------------------------------------------------------------------------ C names

def qs_alloc(n: int, dtype: int = QS_C128, dev_buf: Optional[int] = None, hip_stream: Optional[int] = None) -> int:
    h = _P()
    _check(lib().qs_alloc(ctypes.byref(h), int(n), int(dtype), dev_buf, hip_stream), "qs_alloc")
    return h.value


def qs_free(h: int) -> None:
    _check(lib().qs_free(h), "qs_free")


def qs_apply_gate(h: int, targets: Sequence[int], U) -> None:
    U = _mat(U, len(targets))
    _check(lib().qs_apply_gate(h, _ints(targets), len(targets), _dptr(U.view(np.float64))), "qs_apply_gate")


def qs_apply_diag(h: int, targets: Sequence[int], d) -> None:
    d = _mat(d, len(targets), diag=True)
    _check(lib().qs_apply_diag(h, _ints(targets), len(targets), _dptr(d.view(np.float64))), "qs_apply_diag")


def qs_apply_controlled(h: int, controls: Sequence[int], targets: Sequence[int], U) -> None:
    U = _mat(U, len(targets))
    _check(lib().qs_apply_controlled(h, _ints(controls), len(controls), _ints(targets), len(targets),
                                     _dptr(U.view(np.float64))), "qs_apply_controlled")


def qs_fused_swap(h: int, p: int, q: int, s: int) -> None:
    _check(lib().qs_fused_swap(h, int(p), int(q), int(s)), "qs_fused_swap")


def qs_measure(h: int, qubit: int, u: float):
    """Returns (outcome, P(outcome 1) before the collapse)."""
    o, p1 = ctypes.c_int(), ctypes.c_double()
    _check(lib().qs_measure(h, int(qubit), float(u), ctypes.byref(o), ctypes.byref(p1)), "qs_measure")
    return o.value, p1.value


def qs_reset(h: int, qubit: int, u: float) -> int:
    o = ctypes.c_int()
    _check(lib().qs_reset(h, int(qubit), float(u), ctypes.byref(o)), "qs_reset")
    return o.value


def qs_sample(h: int, u) -> np.ndarray:
    u = np.ascontiguousarray(np.asarray(u, dtype=np.float64).reshape(-1))
    out = np.empty(u.size, dtype=np.int64)
    _check(lib().qs_sample(h, ctypes.c_int64(u.size), _dptr(u),
                           out.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))), "qs_sample")
    return out


def qs_probs(h: int, out_dev: Optional[int] = None, want_norm: bool = False) -> Optional[float]:
    nrm = ctypes.c_double(0.0)
    _check(lib().qs_probs(h, out_dev, ctypes.byref(nrm) if want_norm else None), "qs_probs")
    return nrm.value if want_norm else None


def qs_probs_noalloc(psi_dev: int, n: int, dtype: int, out_dev: Optional[int], norm_dev: Optional[int],
                     hip_stream: Optional[int] = None) -> None:
    """Probabilities and norm of a raw amplitude buffer, without allocating (device pointers in and out)."""
    _check(lib().qs_probs_noalloc(psi_dev, int(n), int(dtype), out_dev, norm_dev, hip_stream), "qs_probs_noalloc")


def qs_init_zero(h: int) -> None:
    _check(lib().qs_init_zero(h), "qs_init_zero")


def qs_copy_in(h: int, host: np.ndarray) -> None:
    host = np.ascontiguousarray(host)
    _check(lib().qs_copy_in(h, host.ctypes.data), "qs_copy_in")


def qs_copy_out(h: int, host: np.ndarray) -> None:
    if not host.flags.c_contiguous:
        raise ValueError("qs_copy_out needs a C-contiguous array")
    _check(lib().qs_copy_out(h, host.ctypes.data), "qs_copy_out")


def qs_sync(h: int) -> None:
    _check(lib().qs_sync(h), "qs_sync")


def qs_scale(h: int, f: float) -> None:
    _check(lib().qs_scale(h, float(f)), "qs_scale")


def qs_norm(h: int) -> float:
    v = ctypes.c_double(0.0)
    _check(lib().qs_norm(h, ctypes.byref(v)), "qs_norm")
    return v.value


def qs_renormalize(h: int, want_norm: bool = False) -> Optional[float]:
    v = ctypes.c_double(0.0)
    _check(lib().qs_renormalize(h, ctypes.byref(v) if want_norm else None), "qs_renormalize")
    return v.value if want_norm else None


def qs_get_info(h: int):
    n, dt, p, s = ctypes.c_int(), ctypes.c_int(), _P(), _P()
    _check(lib().qs_get_info(h, ctypes.byref(n), ctypes.byref(dt), ctypes.byref(p), ctypes.byref(s)), "qs_get_info")
    return n.value, dt.value, p.value, s.value


def qs_last_error() -> str:
    return lib().qs_last_error().decode()


def qs_probe_copy(dst: int, src: int, nbytes: int, hip_stream: Optional[int] = None) -> None:
    _check(lib().qs_probe_copy(dst, src, int(nbytes), hip_stream), "qs_probe_copy")


def qs_probe_rmw(buf: int, nbytes: int, hip_stream: Optional[int] = None) -> None:
    _check(lib().qs_probe_rmw(buf, int(nbytes), hip_stream), "qs_probe_rmw")


def qs_set_tunable(name: str, value: int) -> None:
    _check(lib().qs_set_tunable(name.encode(), int(value)), "qs_set_tunable")


def qs_get_tunable(name: str) -> int:
    v = ctypes.c_int64(0)
    _check(lib().qs_get_tunable(name.encode(), ctypes.byref(v)), "qs_get_tunable")
    return int(v.value)


# ------------------------------------------------------------------------------------------------ circuits, plans

def qs_circuit_create(n: int) -> int:
    h = _P()
    _check(lib().qs_circuit_create(ctypes.byref(h), int(n)), "qs_circuit_create")
    return h.value


def qs_circuit_free(c: int) -> None:
    _check(lib().qs_circuit_free(c), "qs_circuit_free")


def qs_circuit_add_gate(c: int, targets, U) -> None:
    U = _mat(U, len(targets))
    _check(lib().qs_circuit_add_gate(c, _ints(targets), len(targets), _dptr(U.view(np.float64))),
           "qs_circuit_add_gate")


def qs_circuit_add_diag(c: int, targets, d) -> None:
    d = _mat(d, len(targets), diag=True)
    _check(lib().qs_circuit_add_diag(c, _ints(targets), len(targets), _dptr(d.view(np.float64))),
           "qs_circuit_add_diag")


def qs_circuit_add_controlled(c: int, controls, targets, U) -> None:
    U = _mat(U, len(targets))
    _check(lib().qs_circuit_add_controlled(c, _ints(controls), len(controls), _ints(targets), len(targets),
                                           _dptr(U.view(np.float64))), "qs_circuit_add_controlled")


def qs_circuit_add_fused_swap(c: int, p: int, q: int, s: int) -> None:
    _check(lib().qs_circuit_add_fused_swap(c, int(p), int(q), int(s)), "qs_circuit_add_fused_swap")


def qs_circuit_size(c: int) -> int:
    v = ctypes.c_int()
    _check(lib().qs_circuit_size(c, ctypes.byref(v)), "qs_circuit_size")
    return v.value


def qs_circuit_run(h: int, c: int) -> None:
    _check(lib().qs_circuit_run(h, c), "qs_circuit_run")


def qs_plan_create(c: int, mode: int, block_bits: int, low_bits: int = 0, dtype: int = QS_C128) -> int:
    o = qs_plan_opts(int(mode), int(block_bits), int(low_bits), int(dtype))
    h = _P()
    _check(lib().qs_plan_create(ctypes.byref(h), c, ctypes.byref(o)), "qs_plan_create")
    return h.value


def qs_plan_create_learned(c: int, dtype: int, model: int, mean, std, shapes, per_shape: int,
                           gate_slack: int = 0, lookahead: int = 0) -> int:
    """shapes: sequence of (block_bits, low_bits); mean / std: QS_PLAN_NFEAT floats each."""
    mean = np.ascontiguousarray(mean, dtype=np.float32)
    std = np.ascontiguousarray(std, dtype=np.float32)
    if mean.size != QS_PLAN_NFEAT or std.size != QS_PLAN_NFEAT:
        raise ValueError(f"mean and std must hold {QS_PLAN_NFEAT} floats")
    bits = (ctypes.c_int * len(shapes))(*[int(b) for b, _ in shapes])
    low = (ctypes.c_int * len(shapes))(*[int(w) for _, w in shapes])
    fp = ctypes.POINTER(ctypes.c_float)
    m = qs_plan_model(model, mean.ctypes.data_as(fp), std.ctypes.data_as(fp), len(shapes), bits, low, int(per_shape),
                      int(gate_slack), int(lookahead))
    o = qs_plan_opts(QS_PLAN_BLOCK, 0, 0, int(dtype))
    h = _P()
    _check(lib().qs_plan_create_learned(ctypes.byref(h), c, ctypes.byref(o), ctypes.byref(m)),
           "qs_plan_create_learned")
    return h.value


def qs_plan_run(h: int, p: int) -> None:
    _check(lib().qs_plan_run(h, p), "qs_plan_run")


def qs_plan_run_range(h: int, p: int, begin: int, end: int) -> None:
    _check(lib().qs_plan_run_range(h, p, int(begin), int(end)), "qs_plan_run_range")


def qs_plan_run_renorm(h: int, p: int, flags: int) -> None:
    _check(lib().qs_plan_run_renorm(h, p, int(flags)), "qs_plan_run_renorm")


def qs_plan_run_range_renorm(h: int, p: int, begin: int, end: int, flags: int) -> None:
    _check(lib().qs_plan_run_range_renorm(h, p, int(begin), int(end), int(flags)), "qs_plan_run_range_renorm")


def qs_renormalize_pending(h: int, want_norm: bool = False) -> Optional[float]:
    v = ctypes.c_double(0.0)
    _check(lib().qs_renormalize_pending(h, ctypes.byref(v) if want_norm else None), "qs_renormalize_pending")
    return v.value if want_norm else None


def qs_plan_info(p: int):
    v = [ctypes.c_int() for _ in range(5)]
    _check(lib().qs_plan_info(p, *[ctypes.byref(x) for x in v]), "qs_plan_info")
    return {"passes": v[0].value, "block": v[1].value, "dense": v[2].value, "other": v[3].value,
            "fused_ops": v[4].value}


def qs_plan_pass_info(p: int, i: int):
    t, nq, no, ng = ctypes.c_int(), ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
    m = ctypes.c_int64()
    _check(lib().qs_plan_pass_info(p, int(i), ctypes.byref(t), ctypes.byref(nq), ctypes.byref(m), ctypes.byref(no),
                                   ctypes.byref(ng)), "qs_plan_pass_info")
    return {"type": t.value, "nqubits": nq.value, "qmask": m.value, "nops": no.value, "ngates": ng.value}


def qs_plan_pass_gates(p: int, i: int) -> list:
    cnt = ctypes.c_int()
    _check(lib().qs_plan_pass_gates(p, int(i), None, 0, ctypes.byref(cnt)), "qs_plan_pass_gates")
    buf = (ctypes.c_int * max(cnt.value, 1))()
    _check(lib().qs_plan_pass_gates(p, int(i), buf, cnt.value, ctypes.byref(cnt)), "qs_plan_pass_gates")
    return list(buf[:cnt.value])


def qs_plan_free(p: int) -> None:
    _check(lib().qs_plan_free(p), "qs_plan_free")


# ------------------------------------------------------------------------------------------------ cost model

_FP = ctypes.POINTER(ctypes.c_float)


def _f32(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.float32))


def qs_plan_features(p: int, i: int) -> np.ndarray:
    out = np.empty(QS_PLAN_NFEAT, dtype=np.float32)
    _check(lib().qs_plan_features(p, int(i), out.ctypes.data_as(_FP)), "qs_plan_features")
    return out


def qs_mlp_create(nin: int, hidden: int, hip_stream: Optional[int] = None) -> int:
    h = _P()
    _check(lib().qs_mlp_create(ctypes.byref(h), int(nin), int(hidden), hip_stream), "qs_mlp_create")
    return h.value


def qs_mlp_free(m: int) -> None:
    _check(lib().qs_mlp_free(m), "qs_mlp_free")


def qs_mlp_num_params(m: int) -> int:
    v = ctypes.c_int()
    _check(lib().qs_mlp_num_params(m, ctypes.byref(v)), "qs_mlp_num_params")
    return v.value


def qs_mlp_set_params(m: int, params) -> None:
    p = _f32(params)
    if p.size != qs_mlp_num_params(m):
        raise ValueError("parameter vector has the wrong size")
    _check(lib().qs_mlp_set_params(m, p.ctypes.data_as(_FP)), "qs_mlp_set_params")


def qs_mlp_get_params(m: int) -> np.ndarray:
    out = np.empty(qs_mlp_num_params(m), dtype=np.float32)
    _check(lib().qs_mlp_get_params(m, out.ctypes.data_as(_FP)), "qs_mlp_get_params")
    return out


def qs_mlp_predict(m: int, X) -> np.ndarray:
    X = _f32(X)
    out = np.empty(X.shape[0], dtype=np.float32)
    _check(lib().qs_mlp_predict(m, X.ctypes.data_as(_FP), X.shape[0], out.ctypes.data_as(_FP)), "qs_mlp_predict")
    return out


def qs_mlp_grad(m: int, X, T):
    X, T = _f32(X), _f32(T)
    g = np.empty(qs_mlp_num_params(m), dtype=np.float32)
    loss = ctypes.c_float()
    _check(lib().qs_mlp_grad(m, X.ctypes.data_as(_FP), T.ctypes.data_as(_FP), X.shape[0], g.ctypes.data_as(_FP),
                             ctypes.byref(loss)), "qs_mlp_grad")
    return g, loss.value


def qs_mlp_train_step(m: int, X, T, lr: float) -> float:
    X, T = _f32(X), _f32(T)
    loss = ctypes.c_float()
    _check(lib().qs_mlp_train_step(m, X.ctypes.data_as(_FP), T.ctypes.data_as(_FP), X.shape[0], float(lr),
                                   ctypes.byref(loss)), "qs_mlp_train_step")
    return loss.value


# ------------------------------------------------------------------------------------------------ batches

def qs_batch_create(dtype: int = QS_C128, block_bits: int = 12, low_bits: int = 4, wg_per_cu: int = 2,
                    hip_stream: Optional[int] = None) -> int:
    h = _P()
    _check(lib().qs_batch_create(ctypes.byref(h), int(dtype), int(block_bits), int(low_bits), int(wg_per_cu),
                                 hip_stream), "qs_batch_create")
    return h.value


def qs_batch_set_launch(b: int, wg_per_cu: int) -> None:
    _check(lib().qs_batch_set_launch(b, int(wg_per_cu)), "qs_batch_set_launch")


def qs_batch_add(b: int, c: int) -> None:
    _check(lib().qs_batch_add(b, c), "qs_batch_add")


def qs_batch_finalize(b: int) -> None:
    _check(lib().qs_batch_finalize(b), "qs_batch_finalize")


def qs_batch_run(b: int, use_graph: bool = False) -> None:
    _check(lib().qs_batch_run(b, 1 if use_graph else 0), "qs_batch_run")


def qs_batch_info(b: int):
    n, sb, pc, npass, nlev = ctypes.c_int(), ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int(), ctypes.c_int()
    _check(lib().qs_batch_info(b, ctypes.byref(n), ctypes.byref(sb), ctypes.byref(pc), ctypes.byref(npass),
                               ctypes.byref(nlev)), "qs_batch_info")
    return {"circuits": n.value, "state_bytes": sb.value, "prob_count": pc.value, "passes": npass.value,
            "levels": nlev.value}


def qs_batch_probs(b: int, i: int, n: Optional[int] = None):
    """Device pointer of circuit i's probabilities; with n given, also a host copy of its 2^n values."""
    p = _P()
    out = None
    if n is not None:
        out = np.empty(1 << int(n), dtype=np.float64)
    _check(lib().qs_batch_probs(b, int(i), ctypes.byref(p), _dptr(out) if out is not None else None),
           "qs_batch_probs")
    return p.value, out


def qs_batch_free(b: int) -> None:
    _check(lib().qs_batch_free(b), "qs_batch_free")
