"""CPU oracle for the IC/LT Monte Carlo simulator.

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the benchmark's
CPU-baseline leg are the only callers.  The product path never imports this
package.  The arithmetic lives in imsim_oracle.c (plain C, written from the
model definitions of the paper's Section 2); this module only builds and
marshals it.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "imsim_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

IC, LT = 0, 1
OK, E_ARG, E_GRAPH, E_WSUM, E_SEED, E_OOM = 0, -1, -2, -3, -4, -5


def build() -> str:
    """Compile the oracle with the host C compiler (-O2, OpenMP)."""
    tmp = _LIB + ".tmp"
    subprocess.check_call(["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared",
                           "-Wall", "-Wextra", "-o", tmp, _SRC, "-lm"])
    os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib() -> ctypes.CDLL:
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build()
        L = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        i64, u64, u32, ci = ctypes.c_int64, ctypes.c_uint64, ctypes.c_uint32, ctypes.c_int
        L.orc_philox4x64_10.argtypes = [P, P, P]
        L.orc_philox4x64_10.restype = None
        L.orc_hash32.argtypes = [u64, u64, u64, u64]
        L.orc_hash32.restype = u32
        L.orc_encode_p.argtypes = [P, i64, P]
        L.orc_encode_p.restype = ci
        L.orc_encode_w.argtypes = [P, i64, P]
        L.orc_encode_w.restype = ci
        L.orc_validate.argtypes = [ci, i64, P, P, P]
        L.orc_validate.restype = ci
        L.orc_simulate.argtypes = [ci, i64, P, P, P, P, i64, i64, i64, u64, ci, P, P, P, P, P]
        L.orc_simulate.restype = ci
        L.orc_max_threads.argtypes = []
        L.orc_max_threads.restype = ci
        _lib = L
    return _lib


def _ptr(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


class OracleError(RuntimeError):
    def __init__(self, code: int):
        super().__init__(f"oracle error {code}")
        self.code = code


def philox4x64_10(ctr, key) -> np.ndarray:
    c = np.ascontiguousarray(ctr, dtype=np.uint64)
    k = np.ascontiguousarray(key, dtype=np.uint64)
    out = np.zeros(4, dtype=np.uint64)
    lib().orc_philox4x64_10(_ptr(c), _ptr(k), _ptr(out))
    return out


def hash32(rng_seed: int, domain: int, trial: int, ident: int) -> int:
    return int(lib().orc_hash32(rng_seed, domain, trial, ident))


def encode_p(p) -> np.ndarray:
    p = np.ascontiguousarray(p, dtype=np.float64)
    thr = np.zeros(p.shape[0], dtype=np.uint32)
    rc = lib().orc_encode_p(_ptr(p), p.shape[0], _ptr(thr))
    if rc:
        raise OracleError(rc)
    return thr


def encode_w(w) -> np.ndarray:
    w = np.ascontiguousarray(w, dtype=np.float64)
    out = np.zeros(w.shape[0], dtype=np.uint64)
    rc = lib().orc_encode_w(_ptr(w), w.shape[0], _ptr(out))
    if rc:
        raise OracleError(rc)
    return out


def encode(model: str, real_param) -> np.ndarray:
    return encode_p(real_param) if model == "ic" else encode_w(real_param)


def validate(model: str, n: int, offsets, indices, param=None) -> int:
    offsets = np.ascontiguousarray(offsets, dtype=np.int64)
    indices = np.ascontiguousarray(indices, dtype=np.uint32)
    w = None if model == "ic" else np.ascontiguousarray(param, dtype=np.uint64)
    return int(lib().orc_validate(IC if model == "ic" else LT, n, _ptr(offsets), _ptr(indices), _ptr(w)))


def simulate(model: str, n: int, offsets, indices, param, seeds, n_trials: int, rng_seed: int,
             t_begin: int = 0, threads: int = 1, want_bits: bool = True,
             want_levels: bool = False, want_node_counts: bool = True) -> dict:
    """Run trials [t_begin, t_begin + n_trials).  `param` is the encoded
    per-arc parameter (uint32 thresholds for IC, uint64 weights for LT)."""
    offsets = np.ascontiguousarray(offsets, dtype=np.int64)
    indices = np.ascontiguousarray(indices, dtype=np.uint32)
    param = np.ascontiguousarray(param, dtype=np.uint32 if model == "ic" else np.uint64)
    seeds = np.ascontiguousarray(seeds, dtype=np.uint32)
    T = int(n_trials)
    W = (T + 63) // 64
    counts = np.zeros(T, dtype=np.uint32)
    exams = np.zeros(T, dtype=np.uint64)
    node_counts = np.zeros(n, dtype=np.uint32) if want_node_counts else None
    bits = np.zeros((W, n), dtype=np.uint64) if want_bits else None
    levels = np.zeros((T, n), dtype=np.int32) if want_levels else None
    rc = lib().orc_simulate(IC if model == "ic" else LT, n, _ptr(offsets), _ptr(indices), _ptr(param),
                            _ptr(seeds), seeds.shape[0], t_begin, t_begin + T, rng_seed, threads,
                            _ptr(counts), _ptr(exams), _ptr(node_counts), _ptr(bits), _ptr(levels))
    if rc:
        raise OracleError(rc)
    total = int(counts.astype(np.uint64).sum())
    return {"trial_counts": counts, "exams": exams, "node_counts": node_counts,
            "active_bits": bits, "levels": levels, "total": total,
            "mean": total / T if T else float("nan")}


def max_threads() -> int:
    return int(lib().orc_max_threads())
