"""Python access to the oracle of the guess network (oracle/cnn_oracle.c).

TEST INFRASTRUCTURE ONLY, like the rest of oracle/.  Arrays are float64;
a batch of single-channel fields has shape (batch, nz, ny, nx), a batch of
network inputs with C = 3 channels (batch, 3, nz, ny, nx).
"""
from __future__ import annotations

import ctypes as C

import numpy as np

from . import lib as _oracle_lib

LAYERS = 4
TAPS = 27
CIN = (1, 16, 16, 16)     # the one-input network; cin(inputs, l) in general
COUT = (16, 16, 16, 1)

_DP = C.POINTER(C.c_double)


class Dims(C.Structure):
    _fields_ = [("batch", C.c_int32), ("nz", C.c_int32), ("ny", C.c_int32), ("nx", C.c_int32),
                ("periodic", C.c_int32), ("bf16", C.c_int32), ("inputs", C.c_int32),
                ("reserved", C.c_int32), ("alpha", C.c_double)]


_ready = False


def lib():
    global _ready
    L = _oracle_lib()
    if not _ready:
        dp = C.POINTER(Dims)
        for f in ("ocnn_cin", "ocnn_weight_offset", "ocnn_bias_offset"):
            getattr(L, f).argtypes = [C.c_int, C.c_int]
            getattr(L, f).restype = C.c_int
        L.ocnn_cout.argtypes = [C.c_int]
        L.ocnn_cout.restype = C.c_int
        L.ocnn_param_count.argtypes = [C.c_int]
        L.ocnn_param_count.restype = C.c_int
        L.ocnn_bf16.argtypes = [C.c_double]
        L.ocnn_bf16.restype = C.c_double
        L.ocnn_forward.argtypes = [dp, _DP, _DP, _DP, C.POINTER(_DP), C.POINTER(_DP)]
        L.ocnn_backward.argtypes = [dp, _DP, C.POINTER(_DP), C.POINTER(_DP), _DP, _DP]
        L.ocnn_loss.argtypes = [C.c_int32] * 4 + [C.c_double] * 3 + [_DP, _DP, _DP, _DP]
        L.ocnn_adam.argtypes = [C.c_int32, _DP, _DP, _DP, _DP, C.c_int32] + [C.c_double] * 4
        _ready = True
    return L


def param_count(inputs: int = 1) -> int:
    return lib().ocnn_param_count(inputs)


def cin(l: int, inputs: int = 1) -> int:
    return lib().ocnn_cin(inputs, l)


def weight_offset(l: int, inputs: int = 1) -> int:
    return lib().ocnn_weight_offset(inputs, l)


def bias_offset(l: int, inputs: int = 1) -> int:
    return lib().ocnn_bias_offset(inputs, l)


def bf16(a):
    """bfloat16 round-to-nearest-even of each element (as float64)."""
    L = lib()
    a = np.asarray(a, dtype=np.float64)
    return np.vectorize(L.ocnn_bf16, otypes=[np.float64])(a) if a.size else a.copy()


def _p(a):
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(_DP)


def _inputs(x):
    """Input channel count of x: (batch, nz, ny, nx) is one channel,
    (batch, C, nz, ny, nx) C."""
    return 1 if x.ndim == 4 else x.shape[1]


def _dims(x, periodic, alpha, bf16_):
    b, nz, ny, nx = x.shape[0], x.shape[-3], x.shape[-2], x.shape[-1]
    return Dims(b, nz, ny, nx, 1 if periodic else 0, 1 if bf16_ else 0, _inputs(x), 0,
                float(alpha))


def layer_size(ny, nx, l, periodic):
    t = 0 if periodic else 2 * l
    return ny - t, nx - t


def forward(params, x, periodic=False, alpha=0.1, bf16=True):
    """Returns (out (batch, nz, ny_out, nx_out), acts, pre) with acts[l] the
    rounded input of layer l and pre[l] the pre-activation of layer l < 3."""
    params = np.ascontiguousarray(params, dtype=np.float64)
    x = np.ascontiguousarray(x, dtype=np.float64)
    assert x.ndim in (4, 5) and params.size == param_count(_inputs(x))
    d = _dims(x, periodic, alpha, bf16)
    b, nz, ny, nx = d.batch, d.nz, d.ny, d.nx
    acts, pre = [], []
    for l in range(LAYERS):
        yi, xi = layer_size(ny, nx, l, periodic)
        acts.append(np.zeros((b, cin(l, d.inputs), nz, yi, xi)))
        if l < LAYERS - 1:
            yo, xo = layer_size(ny, nx, l + 1, periodic)
            pre.append(np.zeros((b, COUT[l], nz, yo, xo)))
    yo, xo = layer_size(ny, nx, LAYERS, periodic)
    out = np.zeros((b, nz, yo, xo))
    ap = (_DP * LAYERS)(*[_p(a) for a in acts])
    pp = (_DP * LAYERS)(*([_p(a) for a in pre] + [None]))
    rc = lib().ocnn_forward(C.byref(d), _p(params), _p(x), _p(out), ap, pp)
    if rc:
        raise ValueError(f"ocnn_forward failed ({rc})")
    return out, acts, pre


def backward(params, x, acts, pre, gout, periodic=False, alpha=0.1, bf16=True):
    """Gradient of the loss with respect to the parameter vector."""
    params = np.ascontiguousarray(params, dtype=np.float64)
    x = np.ascontiguousarray(x, dtype=np.float64)
    gout = np.ascontiguousarray(gout, dtype=np.float64)
    d = _dims(x, periodic, alpha, bf16)
    grad = np.zeros(param_count(d.inputs))
    ap = (_DP * LAYERS)(*[_p(a) for a in acts])
    pp = (_DP * LAYERS)(*([_p(a) for a in pre] + [None]))
    rc = lib().ocnn_backward(C.byref(d), _p(params), ap, pp, _p(gout), _p(grad))
    if rc:
        raise ValueError(f"ocnn_backward failed ({rc})")
    return grad


def loss(y, t, dx, dy, dz):
    """(loss, dloss/dy) of the residual loss on (batch, nz, ny, nx) crops."""
    y = np.ascontiguousarray(y, dtype=np.float64)
    t = np.ascontiguousarray(t, dtype=np.float64)
    b, nz, ny, nx = y.shape
    out = C.c_double()
    gy = np.zeros_like(y)
    rc = lib().ocnn_loss(b, nz, ny, nx, dx, dy, dz, _p(y), _p(t), C.byref(out), _p(gy))
    if rc:
        raise ValueError(f"ocnn_loss failed ({rc})")
    return out.value, gy


def adam(params, grad, m, v, step, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam step in place on float64 arrays."""
    for a in (params, grad, m, v):
        assert a.dtype == np.float64 and a.flags.c_contiguous
    rc = lib().ocnn_adam(params.size, _p(params), _p(grad), _p(m), _p(v), step, lr, beta1, beta2,
                         eps)
    if rc:
        raise ValueError(f"ocnn_adam failed ({rc})")
