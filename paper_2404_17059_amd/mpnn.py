"""Binding of the learned spread estimator (C ABI in include/imsim_mpnn.h).

Argument marshalling only: the forward pass, backward pass and Adam step run
in libimsim.so's HIP kernels on caller-owned torch tensors.
"""
from __future__ import annotations

import ctypes

import numpy as np
import torch

from . import _check, _lib, _np_ptr, _stream_handle, pack_sets

_P = ctypes.c_void_p
_i64, _u64, _u32, _int, _f32 = ctypes.c_int64, ctypes.c_uint64, ctypes.c_uint32, ctypes.c_int, ctypes.c_float


def _sig(name, res, *args):
    f = getattr(_lib, name)
    f.restype = res
    f.argtypes = list(args)
    return f


_sig("ims_mpnn_create", _int, _i64, _i64, _P, _P, _P, _u32, ctypes.POINTER(_P))
_sig("ims_mpnn_destroy", _int, _P)
_sig("ims_mpnn_init_params", _int, _u64, _P)
_sig("ims_mpnn_forward", _int, _P, _P, _P, _P, _u32, _P, _P)
_sig("ims_mpnn_backward", _int, _P, _P, _P, _P, _P, _P)
_sig("ims_mpnn_adam_step", _int, _P, _P, _P, _P, _i64, _f32, _f32, _f32, _f32, _u32, _P)
_sig("ims_mpnn_fetch", _int, _P, _int, _P, _i64, ctypes.POINTER(_i64), _P)

HIDDEN = 64
IN = 16
MAX_BATCH = 256
NPARAMS = 18689
OFF = {"W0": 0, "b0": 2048, "W1": 2112, "b1": 10304, "W2": 10368, "b2": 18560, "wo": 18624, "bo": 18688}
T = {"X0": 0, "M0": 1, "H1": 2, "M1": 3, "H2": 4, "M2": 5, "H3": 6, "YHAT": 7, "DZ3": 8, "DH2": 9, "DM2": 10,
     "DZ2": 11, "DH1": 12, "DM1": 13, "DZ1": 14}
_WIDTH = {"X0": IN, "M0": IN, "YHAT": 1}


def _dptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def init_params(seed: int) -> np.ndarray:
    out = np.zeros(NPARAMS, dtype=np.float32)
    _check(_lib.ims_mpnn_init_params(int(seed) & ((1 << 64) - 1), _np_ptr(out)), "ims_mpnn_init_params")
    return out


class Surrogate:
    """Plan of the estimator on one graph (out-CSR + per-arc weights a_uv)."""

    def __init__(self, n: int, offsets, indices, arc_weight, max_batch: int = 32):
        self.n = int(n)
        offsets = np.ascontiguousarray(offsets, dtype=np.int64)
        indices = np.ascontiguousarray(indices, dtype=np.uint32)
        a = np.ascontiguousarray(arc_weight, dtype=np.float32)
        self.max_batch = int(max_batch)
        h = ctypes.c_void_p()
        _check(_lib.ims_mpnn_create(self.n, indices.shape[0], _np_ptr(offsets), _np_ptr(indices), _np_ptr(a),
                                    self.max_batch, ctypes.byref(h)), "ims_mpnn_create")
        self._h = h
        self.last_B = 0

    def close(self):
        if getattr(self, "_h", None) and self._h.value:
            _lib.ims_mpnn_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def forward_packed(self, params, offs: np.ndarray, nodes: np.ndarray, pred=None, stream=None):
        B = int(offs.shape[0]) - 1
        if pred is None:
            pred = torch.empty(B, dtype=torch.float32, device=params.device)
        _check(_lib.ims_mpnn_forward(self._h, _dptr(params), _np_ptr(offs), _np_ptr(nodes) if nodes.size else None, B,
                                     _dptr(pred), _stream_handle(stream)), "ims_mpnn_forward")
        self.last_B = B
        return pred

    def forward(self, params, sets, pred=None, stream=None):
        """pred[b] = estimated sigma(sets[b]) (device float32)."""
        offs, nodes = pack_sets(sets)
        return self.forward_packed(params, offs, nodes, pred, stream)

    def backward(self, params, target, grads=None, loss=None, stream=None):
        """Gradient of the last forward's loss against `target` (device float32)."""
        if grads is None:
            grads = torch.empty(NPARAMS, dtype=torch.float32, device=params.device)
        _check(_lib.ims_mpnn_backward(self._h, _dptr(params), _dptr(target), _dptr(grads), _dptr(loss),
                                      _stream_handle(stream)), "ims_mpnn_backward")
        return grads

    def fetch(self, name: str, nodes=None, stream=None) -> np.ndarray:
        """Internal tensor of the last forward/backward: float64 [n, B, width]
        (YHAT: [n, B]), or only the rows of `nodes`; bf16 values are widened
        exactly."""
        B = self.last_B
        width = _WIDTH.get(name, HIDDEN)
        if name == "YHAT":
            out = np.zeros(self.n * B, dtype=np.float32)
        else:
            out = np.zeros(self.n * B * width, dtype=np.uint16)
        written = ctypes.c_int64()
        _check(_lib.ims_mpnn_fetch(self._h, T[name], _np_ptr(out), out.nbytes, ctypes.byref(written),
                                   _stream_handle(stream)), "ims_mpnn_fetch")
        if name == "YHAT":
            y = out.reshape(self.n, B)
            return (y if nodes is None else y[nodes]).astype(np.float64)
        raw = out.reshape(self.n, B, width)
        if nodes is not None:
            raw = raw[nodes]
        return (raw.astype(np.uint32) << 16).view(np.float32).astype(np.float64)


def adam_step(params, grads, m, v, lr: float, step: int, beta1: float = 0.9, beta2: float = 0.999, eps: float = 1e-8,
              stream=None) -> None:
    _check(_lib.ims_mpnn_adam_step(_dptr(params), _dptr(grads), _dptr(m), _dptr(v), params.numel(), float(lr),
                                   float(beta1), float(beta2), float(eps), int(step), _stream_handle(stream)),
           "ims_mpnn_adam_step")
