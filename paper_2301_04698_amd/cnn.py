"""ctypes binding of the guess network ABI (include/les_cnn.h).

Argument marshalling only: every computation runs in the HIP kernels of
liblesmi.so.  Tensors are torch CUDA tensors; calls are ordered on the
current torch stream.  A batch of single-channel fields is a float32
tensor of shape (batch, nz, ny, nx); a batch of three-input network inputs
(batch, 3, nz, ny, nx).  The network's input count follows from those
shapes and from the length of a parameter vector.
"""
from __future__ import annotations

import ctypes as C
import os

from . import les

EXPORTS = ("les_cnn_param_count", "les_cnn_work_bytes", "les_cnn_pack", "les_cnn_forward",
           "les_cnn_loss", "les_cnn_backward", "les_cnn_stored_input", "les_cnn_adam",
           "les_cnn_train_step",
           "les_cnn_pair_scratch_bytes", "les_cnn_pair", "les_cnn_pair_noalloc",
           "les_cnn_pair3", "les_cnn_gather", "les_bind_cnn",
           "les_cnn_guess")

LAYERS = 4
CIN = (1, 16, 16, 16)     # the one-input network; cin(l, inputs) in general
COUT = (16, 16, 16, 1)


def cin(l: int, inputs: int = 1) -> int:
    return inputs if l == 0 else 16


class CnnDims(C.Structure):
    _fields_ = [("batch", C.c_int32), ("nz", C.c_int32), ("ny", C.c_int32), ("nx", C.c_int32),
                ("periodic", C.c_int32), ("inputs", C.c_int32), ("alpha", C.c_double)]


_ready = False
_vp = C.c_void_p
_dp = C.POINTER(CnnDims)


def lib():
    global _ready
    L = les.load()
    if not _ready:
        L.les_cnn_param_count.argtypes = [C.c_int32]
        L.les_cnn_param_count.restype = C.c_int32
        L.les_cnn_work_bytes.argtypes = [_dp]
        L.les_cnn_work_bytes.restype = C.c_size_t
        L.les_cnn_pack.argtypes = [C.c_int32, _vp, _vp, _vp]
        L.les_cnn_forward.argtypes = [_dp, _vp, _vp, _vp, _vp, _vp, _vp]
        L.les_cnn_loss.argtypes = [_dp, C.c_double, C.c_double, C.c_double, _vp, _vp, _vp, _vp,
                                   C.POINTER(C.c_double), _vp]
        L.les_cnn_backward.argtypes = [_dp, _vp, _vp, _vp, _vp, _vp]
        L.les_cnn_stored_input.argtypes = [_dp, _vp, C.c_int32, _vp, _vp]
        L.les_cnn_adam.argtypes = [C.c_int32, _vp, _vp, _vp, _vp, C.c_int32, C.c_double,
                                   C.c_double, C.c_double, C.c_double, _vp]
        L.les_cnn_train_step.argtypes = [_dp, C.c_double, C.c_double, C.c_double, _vp, _vp, _vp,
                                         _vp, C.c_int32, C.c_double, C.c_double, C.c_double,
                                         C.c_double, _vp, _vp, _vp, _vp, C.POINTER(C.c_double),
                                         _vp]
        L.les_cnn_pair_scratch_bytes.argtypes = [C.POINTER(les.LesConfig)]
        L.les_cnn_pair_scratch_bytes.restype = C.c_size_t
        L.les_cnn_pair.argtypes = [C.POINTER(les.LesConfig), _vp, _vp, _vp, _vp, _vp, _vp,
                                   C.POINTER(C.c_double), _vp]
        L.les_cnn_pair_noalloc.argtypes = [C.POINTER(les.LesConfig), _vp, _vp, _vp, _vp, _vp,
                                           C.POINTER(C.c_double), _vp]
        L.les_cnn_pair3.argtypes = [C.POINTER(les.LesConfig), _vp, _vp, _vp, _vp, _vp, _vp,
                                    C.POINTER(C.c_double), _vp]
        L.les_cnn_gather.argtypes = [C.c_int32, _vp, _vp, C.c_int32, C.c_int32, C.c_int32,
                                     C.c_int32, _vp, C.c_int32, C.c_int32, C.c_int32, _vp, _vp,
                                     _vp]
        L.les_bind_cnn.argtypes = [_vp, _vp, C.c_double]
        L.les_cnn_guess.argtypes = [_vp, _vp, _vp, _vp, C.POINTER(C.c_double)]
        _ready = True
    return L


def _stream():
    import torch
    return _vp(torch.cuda.current_stream().cuda_stream)


def _ptr(t):
    return _vp(t.data_ptr()) if t is not None else None


def param_count(inputs: int = 1) -> int:
    n = int(lib().les_cnn_param_count(int(inputs)))
    if n < 0:
        raise les.LesError(n, les.last_error())
    return n


def inputs_of(params) -> int:
    """Input count of a parameter vector, from its length."""
    n = params.numel() if hasattr(params, "numel") else len(params)
    for c in (1, 3):
        if n == param_count(c):
            return c
    raise ValueError(f"{n} parameters fit no guess network")


def weight_offset(l: int, inputs: int = 1) -> int:
    off = 0
    for q in range(l):
        off += 27 * cin(q, inputs) * COUT[q] + COUT[q]
    return off


def bias_offset(l: int, inputs: int = 1) -> int:
    return weight_offset(l, inputs) + 27 * cin(l, inputs) * COUT[l]


def dims(shape, periodic=False, alpha=0.1) -> CnnDims:
    """Dims of a batch of shape (batch, nz, ny, nx) (one input) or (batch,
    C, nz, ny, nx)."""
    inputs = 1 if len(shape) == 4 else shape[1]
    b, nz, ny, nx = shape[0], shape[-3], shape[-2], shape[-1]
    return CnnDims(b, nz, ny, nx, 1 if periodic else 0, inputs, float(alpha))


def out_shape(d: CnnDims):
    t = 0 if d.periodic else 8
    return (d.batch, d.nz, d.ny - t, d.nx - t)


def work_bytes(d: CnnDims) -> int:
    n = int(lib().les_cnn_work_bytes(C.byref(d)))
    if n == 0:
        raise les.LesError(les.LES_ERR_ARG, les.last_error())
    return n


def _f32(t):
    import torch
    assert t.is_cuda and t.dtype == torch.float32 and t.is_contiguous()
    return t


WEIGHTS = os.path.join(os.path.dirname(os.path.abspath(__file__)), "weights",
                       "guess_256x256x128.npy")
WEIGHTS3 = os.path.join(os.path.dirname(os.path.abspath(__file__)), "weights",
                        "guess3_256x256x128.npy")


def load_weights(path=WEIGHTS):
    """Shipped network parameters (float32 numpy) and their metadata (the
    JSON file beside them: training command, alpha, ...)."""
    import json
    import numpy as np
    prm = np.load(path).astype(np.float32)
    meta = {"alpha": 0.1}
    side = os.path.splitext(path)[0] + ".json"
    if os.path.exists(side):
        with open(side) as f:
            meta.update(json.load(f))
    return prm, meta


def pack(params):
    import torch
    inputs = inputs_of(params)
    packed = torch.empty(param_count(inputs), dtype=torch.int16, device=params.device)
    les.check(lib().les_cnn_pack(inputs, _ptr(_f32(params)), _ptr(packed), _stream()))
    return packed


def empty_work(d: CnnDims, device="cuda"):
    import torch
    return torch.empty(work_bytes(d), dtype=torch.uint8, device=device)


def forward(params, packed, x, periodic=False, alpha=0.1, work=None):
    """Returns (out, work); work keeps the layer inputs for backward()."""
    import torch
    d = dims(x.shape, periodic, alpha)
    if work is None:
        work = empty_work(d, x.device)
    out = torch.empty(out_shape(d), dtype=torch.float32, device=x.device)
    les.check(lib().les_cnn_forward(C.byref(d), _ptr(_f32(params)), _ptr(packed),
                                    _ptr(_f32(x)), _ptr(work), _ptr(out), _stream()))
    return out, work


def loss(x_shape, out, target, dx, dy, dz, work, alpha=0.1):
    """(loss, gout) of a forward() output on valid crops."""
    import torch
    d = dims(x_shape, False, alpha)
    gout = torch.empty_like(out)
    val = C.c_double()
    les.check(lib().les_cnn_loss(C.byref(d), dx, dy, dz, _ptr(_f32(out)), _ptr(_f32(target)),
                                 _ptr(work), _ptr(gout), C.byref(val), _stream()))
    return val.value, gout


def backward(x_shape, packed, work, gout, alpha=0.1):
    import torch
    d = dims(x_shape, False, alpha)
    grad = torch.empty(param_count(d.inputs), dtype=torch.float32, device=gout.device)
    les.check(lib().les_cnn_backward(C.byref(d), _ptr(packed), _ptr(work), _ptr(_f32(gout)),
                                     _ptr(grad), _stream()))
    return grad


def stored_input(x_shape, work, layer, periodic=False, alpha=0.1):
    """Layer `layer`'s input kept in work by the last forward, as a float32
    tensor (batch, channels, nz, ny_l, nx_l)."""
    import torch
    d = dims(x_shape, periodic=periodic, alpha=alpha)
    b, nz, ny, nx = d.batch, d.nz, d.ny, d.nx
    t = 0 if periodic else 2 * layer
    out = torch.empty((b, cin(layer, d.inputs), nz, ny - t, nx - t), dtype=torch.float32,
                      device=work.device)
    les.check(lib().les_cnn_stored_input(C.byref(d), _ptr(work), int(layer), _ptr(out), _stream()))
    return out


def adam(params, grad, m, v, step, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
    les.check(lib().les_cnn_adam(params.numel(), _ptr(_f32(params)), _ptr(_f32(grad)),
                                 _ptr(_f32(m)), _ptr(_f32(v)), int(step), lr, beta1, beta2, eps,
                                 _stream()))


class Trainer:
    """FP32 master parameters, Adam moments and the buffers of one training
    batch shape; step() runs les_cnn_train_step."""

    def __init__(self, params, batch, nz, cy, cx, dx, dy, dz, alpha=0.1, lr=1e-3,
                 beta1=0.9, beta2=0.999, eps=1e-8, device="cuda"):
        import torch
        self.params = _f32(params.to(device=device, dtype=torch.float32).contiguous().clone())
        self.packed = pack(self.params)
        self.m = torch.zeros_like(self.params)
        self.v = torch.zeros_like(self.params)
        self.grad = torch.zeros_like(self.params)
        inputs = inputs_of(self.params)
        shape = (batch, nz, cy + 8, cx + 8) if inputs == 1 else (batch, inputs, nz, cy + 8, cx + 8)
        self.d = dims(shape, False, alpha)
        self.work = empty_work(self.d, device)
        self.spacing = (dx, dy, dz)
        self.hyper = (lr, beta1, beta2, eps)
        self.t = 0

    def step(self, x, target, want_loss=False):
        self.t += 1
        val = C.c_double()
        lr, b1, b2, eps = self.hyper
        les.check(lib().les_cnn_train_step(
            C.byref(self.d), *self.spacing, _ptr(self.params), _ptr(self.packed), _ptr(self.m),
            _ptr(self.v), self.t, lr, b1, b2, eps, _ptr(_f32(x)), _ptr(_f32(target)),
            _ptr(self.work), _ptr(self.grad), C.byref(val) if want_loss else None, _stream()))
        return val.value if want_loss else None


def pair(sim, rhs, base, phi, x, target, scratch=None):
    """Training pair of one solve of `sim`'s grid into float32 fields x,
    target (shape (nz, ny, nx)); returns s = RMS of the base's residual."""
    import torch
    L = lib()
    if scratch is None:
        scratch = torch.empty(int(L.les_cnn_pair_scratch_bytes(C.byref(sim.cfg))),
                              dtype=torch.uint8, device=rhs.device)
    for t in (rhs, phi) + ((base,) if base is not None else ()):
        assert t.dtype == sim.dtype and t.is_contiguous() and t.numel() == sim._n()
    s = C.c_double()
    les.check(L.les_cnn_pair(C.byref(sim.cfg), _ptr(rhs), _ptr(base), _ptr(phi), _ptr(_f32(x)),
                             _ptr(_f32(target)), _ptr(scratch), C.byref(s), _stream()))
    return s.value


def pair_noalloc(sim, rhs, base, phi, x, target):
    """As pair() through the entry point that allocates nothing (its scratch
    is a fixed device array of the library)."""
    L = lib()
    for t in (rhs, phi) + ((base,) if base is not None else ()):
        assert t.dtype == sim.dtype and t.is_contiguous() and t.numel() == sim._n()
    s = C.c_double()
    les.check(L.les_cnn_pair_noalloc(C.byref(sim.cfg), _ptr(rhs), _ptr(base), _ptr(phi),
                                     _ptr(_f32(x)), _ptr(_f32(target)), C.byref(s), _stream()))
    return s.value


def pair3(sim, rhs, base, phi, x, target, scratch=None):
    """Training pair of the three-input network from one solve of `sim`'s
    grid: x (3, nz, ny, nx), target (nz, ny, nx) float32 (phi and target
    None: the inputs only); returns s."""
    import torch
    L = lib()
    if scratch is None:
        scratch = torch.empty(int(L.les_cnn_pair_scratch_bytes(C.byref(sim.cfg))),
                              dtype=torch.uint8, device=rhs.device)
    for t in (rhs, base) + ((phi,) if phi is not None else ()):
        assert t.dtype == sim.dtype and t.is_contiguous() and t.numel() == sim._n()
    assert x.numel() == 3 * sim._n()
    s = C.c_double()
    les.check(L.les_cnn_pair3(C.byref(sim.cfg), _ptr(rhs), _ptr(base), _ptr(phi), _ptr(_f32(x)),
                              _ptr(_f32(target)) if target is not None else None, _ptr(scratch),
                              C.byref(s), _stream()))
    return s.value


def gather(X, T, crops, cy, cx, xb=None, tb=None):
    """Crops (pair, j0, i0) of stored pairs: X of shape (npairs, nz, ny, nx)
    (one input) or (npairs, C, nz, ny, nx), T (npairs, nz, ny, nx)."""
    import torch
    inputs = 1 if X.dim() == 4 else X.shape[1]
    npairs, nz, ny, nx = X.shape[0], X.shape[-3], X.shape[-2], X.shape[-1]
    assert T.shape == (npairs, nz, ny, nx)
    crops = crops.to(device=X.device, dtype=torch.int32).contiguous()
    batch = crops.numel() // 3
    xshape = (batch, nz, cy + 8, cx + 8) if inputs == 1 else (batch, inputs, nz, cy + 8, cx + 8)
    if xb is None:
        xb = torch.empty(xshape, dtype=torch.float32, device=X.device)
    if tb is None:
        tb = torch.empty((batch, nz, cy, cx), dtype=torch.float32, device=X.device)
    les.check(lib().les_cnn_gather(inputs, _ptr(_f32(X)), _ptr(_f32(T)), npairs, nz, ny, nx,
                                   _ptr(crops), batch, cy, cx, _ptr(xb), _ptr(tb), _stream()))
    return xb, tb


def bind(sim, params, alpha=0.1):
    """Bind the network of a LES handle created with guess='learned' (one
    input) or 'learned3' (three inputs)."""
    import torch
    p = params.to(device=sim.device, dtype=torch.float32).contiguous()
    les.check(lib().les_bind_cnn(sim.handle, _ptr(p), float(alpha)))


def guess(sim, rhs, base):
    """(guess, s) of the bound network for one solve of `sim`'s grid."""
    import torch
    g = torch.empty_like(base)
    s = C.c_double()
    les.check(lib().les_cnn_guess(sim.handle, _ptr(rhs.contiguous()), _ptr(base.contiguous()),
                                  _ptr(g), C.byref(s)))
    return g, s.value
