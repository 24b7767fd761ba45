"""imsim: Monte Carlo IC / LT diffusion on one gfx950 GPU.

A thin ctypes binding over libimsim.so (C ABI declared in include/imsim.h).
PyTorch provides device memory and the stream; every step of the simulation
runs in the library's HIP kernels.  There is no CPU fallback: importing this
package without the built library raises.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np
# torch ships its own HIP runtime with the same SONAME as /opt/rocm's; loading
# it first makes libimsim.so bind to that one copy, so both share devices,
# streams and memory.
import torch  # noqa: F401

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libimsim.so")

IC, LT = 0, 1
ERRORS = {0: "IMS_OK", -1: "IMS_E_INVALID_ARG", -2: "IMS_E_INVALID_GRAPH", -3: "IMS_E_WEIGHT_SUM",
          -4: "IMS_E_SEED_RANGE", -5: "IMS_E_OOM", -6: "IMS_E_HIP", -7: "IMS_E_LEVEL_CAP",
          -8: "IMS_E_UNSUPPORTED"}

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_2404_17059_amd.build` "
                      "(this package has no CPU fallback)")

_lib = ctypes.CDLL(LIB_PATH)
_P = ctypes.c_void_p
_i64, _u64, _u32, _int = ctypes.c_int64, ctypes.c_uint64, ctypes.c_uint32, ctypes.c_int


class Opts(ctypes.Structure):
    _fields_ = [("shape", ctypes.c_int), ("blocks_per_cu", ctypes.c_int32), ("alpha", ctypes.c_double),
                ("profile", ctypes.c_int32), ("test_flags", ctypes.c_int32), ("ic_alpha", ctypes.c_double),
                ("ic_beta", ctypes.c_double), ("ic_direction", ctypes.c_int32)]


class BatchItem(ctypes.Structure):
    _fields_ = [("graph", ctypes.c_void_p), ("seeds", ctypes.c_void_p), ("n_seeds", ctypes.c_uint32),
                ("n_trials", ctypes.c_uint32), ("rng_seed", ctypes.c_uint64), ("trial_counts", ctypes.c_void_p),
                ("node_counts", ctypes.c_void_p), ("total", ctypes.c_void_p)]


class Tuning(ctypes.Structure):
    _fields_ = [("blocks_per_cu", ctypes.c_int32), ("order", ctypes.c_int32), ("split", ctypes.c_int32),
                ("ic_alpha", ctypes.c_double), ("ic_beta", ctypes.c_double)]


def _sig(name, res, *args):
    f = getattr(_lib, name)
    f.restype = res
    f.argtypes = list(args)
    return f


_sig("ims_last_error", ctypes.c_char_p)
_sig("ims_version", ctypes.c_char_p)
_sig("ims_encode_p", _int, _P, _i64, _P)
_sig("ims_encode_w", _int, _P, _i64, _P)
_sig("ims_validate_csr", _int, _i64, _i64, _P, _P)
_sig("ims_graph_create", _int, _i64, _i64, _P, _P, _int, _P, ctypes.POINTER(_P))
_sig("ims_graph_destroy", _int, _P)
_sig("ims_graph_info", _int, _P, ctypes.POINTER(_i64), ctypes.POINTER(_i64), ctypes.POINTER(_int))
_sig("ims_simulate", _int, _P, _P, _u32, _u32, _u64, ctypes.POINTER(Opts), _P, _P, _P, _P, _P)
_sig("ims_graph_last_status", _int, _P, _P, _P)
_sig("ims_batch_create", _int, ctypes.POINTER(BatchItem), _u32, ctypes.POINTER(Tuning), ctypes.POINTER(_P))
_sig("ims_batch_autotune", _int, _P, _int, _P, ctypes.POINTER(Tuning))
_sig("ims_batch_launch", _int, _P, _P)
_sig("ims_batch_destroy", _int, _P)
_sig("ims_batch_task_timing", _int, _P, _int)
_sig("ims_batch_task_times", _int, _P, _u32, _P, _P, ctypes.POINTER(_u32), _P)
_sig("ims_simulate_sets", _int, _P, _P, _P, _u32, _u32, _u64, ctypes.POINTER(Opts), _P, _P, _P)
_sig("ims_simulate_levels", _int, _P, _P, _u32, _u32, _u64, _u32, _P, _P, _P, _P)
_sig("ims_simulate_sets_from", _int, _P, _P, _P, _P, _u32, _u32, _u64, ctypes.POINTER(Opts), _P, _P, _P)
_sig("ims_graph_profile", _int, _P, _int, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(_u32))
_sig("ims_graph_level_directions", _int, _P, _u32, _P, ctypes.POINTER(_u32), _P)
_sig("ims_graph_last_counters", _int, _P, _P, _P)
_sig("ims_debug_hash", _int, _u64, _u64, _P, _P, _P, _i64, _P)
_sig("ims_simulate_noalloc", _int, _P, _P, _u32, _u32, _u64, _P, _P, _P, _P)

NOALLOC_SCRATCH_BYTES = 64 << 20  # IMS_NOALLOC_SCRATCH_BYTES of include/imsim.h


class ImsError(RuntimeError):
    def __init__(self, code: int, where: str, msg: str | None = None):
        if msg is None:
            msg = _lib.ims_last_error().decode(errors="replace")
        super().__init__(f"{where}: {ERRORS.get(code, code)}: {msg}")
        self.code = code


def _check(code: int, where: str) -> None:
    if code != 0:
        raise ImsError(code, where)


def _np_ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def version() -> str:
    return _lib.ims_version().decode()


def encode_p(p) -> np.ndarray:
    p = np.ascontiguousarray(p, dtype=np.float64)
    out = np.zeros(p.shape[0], dtype=np.uint32)
    _check(_lib.ims_encode_p(_np_ptr(p), p.shape[0], _np_ptr(out)), "ims_encode_p")
    return out


def encode_w(w) -> np.ndarray:
    w = np.ascontiguousarray(w, dtype=np.float64)
    out = np.zeros(w.shape[0], dtype=np.uint64)
    _check(_lib.ims_encode_w(_np_ptr(w), w.shape[0], _np_ptr(out)), "ims_encode_w")
    return out


def validate_csr(n: int, offsets, indices) -> None:
    offsets = np.ascontiguousarray(offsets, dtype=np.int64)
    indices = np.ascontiguousarray(indices, dtype=np.uint32)
    _check(_lib.ims_validate_csr(n, indices.shape[0], _np_ptr(offsets), _np_ptr(indices)), "ims_validate_csr")


def _torch():
    import torch
    return torch


def _stream_handle(stream):
    torch = _torch()
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


class Graph:
    """Device graph plan.  `param` is the real-valued per-arc parameter in
    out-CSR order (IC probability or LT weight), encoded by the library, or an
    already encoded array (uint32 thresholds / uint64 weights)."""

    def __init__(self, n: int, offsets, indices, model: str, param):
        self.n = int(n)
        self.model = model
        offsets = np.ascontiguousarray(offsets, dtype=np.int64)
        indices = np.ascontiguousarray(indices, dtype=np.uint32)
        self.m = int(indices.shape[0])
        param = np.asarray(param)
        if model == "ic":
            enc = param if param.dtype == np.uint32 else encode_p(param)
            enc = np.ascontiguousarray(enc, dtype=np.uint32)
        elif model == "lt":
            enc = param if param.dtype == np.uint64 else encode_w(param)
            enc = np.ascontiguousarray(enc, dtype=np.uint64)
        else:
            raise ValueError(f"unknown model {model!r}")
        self.encoded = enc
        self.outdeg = np.diff(offsets)
        h = ctypes.c_void_p()
        _check(_lib.ims_graph_create(self.n, self.m, _np_ptr(offsets), _np_ptr(indices),
                                     IC if model == "ic" else LT, _np_ptr(enc), ctypes.byref(h)),
               "ims_graph_create")
        self._h = h

    def close(self):
        if getattr(self, "_h", None) and self._h.value:
            _lib.ims_graph_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def handle(self):
        return self._h

    def profile(self, reset: bool = True) -> tuple[float, int]:
        """(summed kernel ms, number of runs) of runs made with Opts.profile."""
        ms = ctypes.c_double()
        cnt = ctypes.c_uint32()
        _check(_lib.ims_graph_profile(self._h, int(reset), ctypes.byref(ms), ctypes.byref(cnt)), "ims_graph_profile")
        return float(ms.value), int(cnt.value)

    def level_directions(self, max_levels: int = 4096, stream=None) -> np.ndarray:
        """Per level of the last IC grid-shape run: 1 = push, 2 = pull."""
        out = np.zeros(max(int(max_levels), 1), dtype=np.uint32)
        cnt = ctypes.c_uint32()
        _check(_lib.ims_graph_level_directions(self._h, int(max_levels), _np_ptr(out), ctypes.byref(cnt),
                                               _stream_handle(stream)), "ims_graph_level_directions")
        return out[:cnt.value]

    def last_counters(self, stream=None) -> np.ndarray:
        """The last run's four status words: steps, guard, tasks taken, hand-overs refused."""
        out = np.zeros(4, dtype=np.uint32)
        _check(_lib.ims_graph_last_counters(self._h, _stream_handle(stream), _np_ptr(out)), "ims_graph_last_counters")
        return out

    def last_status(self, stream=None) -> tuple[int, int]:
        out = np.zeros(2, dtype=np.uint32)
        _check(_lib.ims_graph_last_status(self._h, _stream_handle(stream), _np_ptr(out)), "ims_graph_last_status")
        return int(out[0]), int(out[1])


def _dev_ptr(t, where: str, name: str, itemsize: int, numel: int, required: bool = True):
    """Device address of an output tensor after checking that the library can
    write `numel` items of `itemsize` bytes there: a CUDA tensor on the
    current device, contiguous, of that item size, large enough.  The check
    runs before any device work, so a wrong buffer is an error, not a write
    out of bounds."""
    if t is None:
        if required:
            raise ImsError(-1, where, f"{name} is required")
        return None
    torch = _torch()
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise ImsError(-1, where, f"{name} must be a CUDA tensor")
    if t.device.index != torch.cuda.current_device():
        raise ImsError(-1, where, f"{name} is on {t.device}, not the current device")
    if not t.is_contiguous():
        raise ImsError(-1, where, f"{name} must be contiguous")
    if t.element_size() != itemsize or t.is_floating_point() or t.is_complex():
        raise ImsError(-1, where, f"{name} must hold {itemsize}-byte integers, not {t.dtype}")
    if t.numel() < numel:
        raise ImsError(-1, where, f"{name} holds {t.numel()} items, needs {numel}")
    return ctypes.c_void_p(t.data_ptr())


def simulate_into(graph: Graph, seeds, n_trials: int, rng_seed: int, trial_counts, total,
                  node_counts=None, active_bits=None, stream=None, opts: Opts | None = None) -> None:
    """Enqueue one simulation on `stream` writing into caller tensors."""
    seeds = np.ascontiguousarray(seeds, dtype=np.uint32)
    T = int(n_trials)
    W = (T + 63) // 64
    where = "ims_simulate"
    tc = _dev_ptr(trial_counts, where, "trial_counts", 4, T)
    tot = _dev_ptr(total, where, "total", 8, 1)
    nc = _dev_ptr(node_counts, where, "node_counts", 4, graph.n, required=False)
    bits = _dev_ptr(active_bits, where, "active_bits", 8, W * graph.n, required=False)
    _check(_lib.ims_simulate(graph.handle, _np_ptr(seeds) if seeds.size else None, seeds.shape[0],
                             T, int(rng_seed) & ((1 << 64) - 1),
                             ctypes.byref(opts) if opts is not None else None,
                             tc, nc, tot, bits, _stream_handle(stream)), where)


def simulate_noalloc_into(graph: Graph, seeds, n_trials: int, rng_seed: int, trial_counts, total,
                          node_counts=None, stream=None) -> None:
    """Enqueue one counts-only simulation through the allocation-free entry
    point (its device state lives in the library's fixed per-GPU array;
    overlapping calls on one GPU race)."""
    seeds = np.ascontiguousarray(seeds, dtype=np.uint32)
    T = int(n_trials)
    where = "ims_simulate_noalloc"
    tc = _dev_ptr(trial_counts, where, "trial_counts", 4, T)
    tot = _dev_ptr(total, where, "total", 8, 1)
    nc = _dev_ptr(node_counts, where, "node_counts", 4, graph.n, required=False)
    _check(_lib.ims_simulate_noalloc(graph.handle, _np_ptr(seeds) if seeds.size else None, seeds.shape[0],
                                     T, int(rng_seed) & ((1 << 64) - 1), tc, nc, tot, _stream_handle(stream)), where)


def simulate(graph: Graph, seeds, n_trials: int, rng_seed: int, want_bits: bool = False,
             want_node_counts: bool = True, stream=None, opts: Opts | None = None) -> dict:
    """Run trials 0..n_trials-1; returns device tensors and the mean spread."""
    torch = _torch()
    dev = torch.device("cuda", torch.cuda.current_device())
    T = int(n_trials)
    W = (T + 63) // 64
    tc = torch.empty(T, dtype=torch.int32, device=dev)
    tot = torch.empty(1, dtype=torch.int64, device=dev)
    nc = torch.empty(graph.n, dtype=torch.int32, device=dev) if want_node_counts else None
    bits = torch.empty((W, graph.n), dtype=torch.int64, device=dev) if want_bits else None
    simulate_into(graph, seeds, T, rng_seed, tc, tot, nc, bits, stream, opts)
    steps, guard = graph.last_status(stream)
    if guard:
        raise ImsError(-7, "ims_simulate")
    total = int(tot.item())
    return {"trial_counts": tc, "total": total, "mean": total / T, "node_counts": nc,
            "active_bits": bits, "steps": steps}


def simulate_levels(graph: Graph, seeds, n_trials: int, rng_seed: int, max_levels: int = 256, stream=None) -> dict:
    """Per-trial counts of nodes first activated at each level (level 0 =
    seeds; LT runs synchronous steps here); returns host arrays level_counts
    [levels, T] (trimmed to the levels reached), trial_counts, and the mean
    spread."""
    torch = _torch()
    dev = torch.device("cuda", torch.cuda.current_device())
    seeds = np.ascontiguousarray(seeds, dtype=np.uint32)
    T = int(n_trials)
    lc = torch.empty((int(max_levels), T), dtype=torch.int32, device=dev)
    tc = torch.empty(T, dtype=torch.int32, device=dev)
    tot = torch.empty(1, dtype=torch.int64, device=dev)
    _check(_lib.ims_simulate_levels(graph.handle, _np_ptr(seeds) if seeds.size else None, seeds.shape[0], T,
                                    int(rng_seed) & ((1 << 64) - 1), int(max_levels), ctypes.c_void_p(lc.data_ptr()),
                                    ctypes.c_void_p(tc.data_ptr()), ctypes.c_void_p(tot.data_ptr()),
                                    _stream_handle(stream)), "ims_simulate_levels")
    steps, guard = graph.last_status(stream)
    if guard:
        raise ImsError(-7, "ims_simulate_levels")
    counts = lc.cpu().numpy().view(np.uint32)
    used = min(int(max_levels), steps + 1)
    total = int(tot.item())
    return {"level_counts": counts[:used], "levels_processed": steps, "truncated": steps + 1 > int(max_levels),
            "trial_counts": tc.cpu().numpy().view(np.uint32), "total": total, "mean": total / T}


def pack_sets(sets) -> tuple[np.ndarray, np.ndarray]:
    """Concatenate seed sets into (offsets uint32[k+1], nodes uint32)."""
    offs = np.zeros(len(sets) + 1, dtype=np.uint32)
    parts = []
    for i, st in enumerate(sets):
        a = np.ascontiguousarray(st, dtype=np.uint32).ravel()
        parts.append(a)
        offs[i + 1] = offs[i] + a.shape[0]
    nodes = np.concatenate(parts) if parts else np.zeros(0, dtype=np.uint32)
    return offs, np.ascontiguousarray(nodes, dtype=np.uint32)


def simulate_sets_into(graph: Graph, offsets: np.ndarray, nodes: np.ndarray, n_trials: int, rng_seed: int,
                       totals, node_counts=None, stream=None, opts: Opts | None = None) -> None:
    """Enqueue the simulation of many seed sets (common random numbers)."""
    n_sets = int(offsets.shape[0]) - 1
    where = "ims_simulate_sets"
    tot = _dev_ptr(totals, where, "totals", 8, n_sets)
    nc = _dev_ptr(node_counts, where, "node_counts", 4, n_sets * graph.n, required=False)
    _check(_lib.ims_simulate_sets(graph.handle, _np_ptr(offsets), _np_ptr(nodes) if nodes.size else None, n_sets,
                                  int(n_trials), int(rng_seed) & ((1 << 64) - 1),
                                  ctypes.byref(opts) if opts is not None else None,
                                  tot, nc, _stream_handle(stream)), where)


def simulate_sets(graph: Graph, sets, n_trials: int, rng_seed: int, want_node_counts: bool = False,
                  stream=None, opts: Opts | None = None) -> dict:
    """sigma of every seed set in `sets` under the same trials (common random
    numbers); returns host arrays."""
    torch = _torch()
    offs, nodes = pack_sets(sets)
    n_sets = len(sets)
    dev = torch.device("cuda", torch.cuda.current_device())
    tot = torch.empty(max(n_sets, 1), dtype=torch.int64, device=dev)
    nc = torch.empty((max(n_sets, 1), graph.n), dtype=torch.int32, device=dev) if want_node_counts else None
    simulate_sets_into(graph, offs, nodes, n_trials, rng_seed, tot, nc, stream, opts)
    totals = tot.cpu().numpy()[:n_sets]
    out = {"totals": totals, "sigma": totals / float(n_trials)}
    if want_node_counts:
        out["node_counts"] = nc.cpu().numpy().view(np.uint32)[:n_sets]
    return out


def simulate_sets_from_into(graph: Graph, base_bits, offsets: np.ndarray, nodes: np.ndarray, n_trials: int, rng_seed: int,
                            totals, node_counts=None, stream=None, opts: Opts | None = None) -> None:
    """Enqueue marginal simulations of many sets on top of the state
    base_bits ([W, n] active bits of a run with the same n_trials and
    rng_seed); totals receive the new activations only."""
    n_sets = int(offsets.shape[0]) - 1
    where = "ims_simulate_sets_from"
    W = (int(n_trials) + 63) // 64
    base = _dev_ptr(base_bits, where, "base_bits", 8, W * graph.n)
    tot = _dev_ptr(totals, where, "totals", 8, n_sets)
    nc = _dev_ptr(node_counts, where, "node_counts", 4, n_sets * graph.n, required=False)
    _check(_lib.ims_simulate_sets_from(graph.handle, base, _np_ptr(offsets), _np_ptr(nodes) if nodes.size else None,
                                       n_sets, int(n_trials), int(rng_seed) & ((1 << 64) - 1),
                                       ctypes.byref(opts) if opts is not None else None, tot, nc,
                                       _stream_handle(stream)), where)


def simulate_sets_from(graph: Graph, base_bits, sets, n_trials: int, rng_seed: int, want_node_counts: bool = False,
                       stream=None, opts: Opts | None = None) -> dict:
    """New activations of each set in `sets` added to the seed set whose run
    produced base_bits (common random numbers); returns host arrays."""
    torch = _torch()
    offs, nodes = pack_sets(sets)
    n_sets = len(sets)
    dev = torch.device("cuda", torch.cuda.current_device())
    tot = torch.empty(max(n_sets, 1), dtype=torch.int64, device=dev)
    nc = torch.empty((max(n_sets, 1), graph.n), dtype=torch.int32, device=dev) if want_node_counts else None
    simulate_sets_from_into(graph, base_bits, offs, nodes, n_trials, rng_seed, tot, nc, stream, opts)
    out = {"new_totals": tot.cpu().numpy()[:n_sets]}
    if want_node_counts:
        out["node_counts"] = nc.cpu().numpy().view(np.uint32)[:n_sets]
    return out


class Batch:
    """Several simulations (IC and LT, graphs of any size) run by one
    persistent launch; the first launch captures a HIP graph that later
    launches replay.  items: (Graph, seeds, n_trials, rng_seed) tuples."""

    def __init__(self, items, tuning: tuple | None = None, want_node_counts: bool = True):
        torch = _torch()
        dev = torch.device("cuda", torch.cuda.current_device())
        self.graphs = [it[0] for it in items]
        self.outputs = []
        arr = (BatchItem * max(len(items), 1))()
        keep = []
        for i, (g, seeds, T, rs) in enumerate(items):
            sd = np.ascontiguousarray(seeds, dtype=np.uint32)
            keep.append(sd)
            tc = torch.empty(int(T), dtype=torch.int32, device=dev)
            nc = torch.empty(g.n, dtype=torch.int32, device=dev) if want_node_counts else None
            tot = torch.empty(1, dtype=torch.int64, device=dev)
            self.outputs.append((tc, nc, tot, int(T)))
            arr[i] = BatchItem(g.handle.value, sd.ctypes.data if sd.size else None, sd.shape[0], int(T),
                               int(rs) & ((1 << 64) - 1), tc.data_ptr(), nc.data_ptr() if nc is not None else None,
                               tot.data_ptr())
        tun = Tuning(*tuning) if tuning is not None else None
        h = ctypes.c_void_p()
        _check(_lib.ims_batch_create(arr, len(items), ctypes.byref(tun) if tun is not None else None, ctypes.byref(h)),
               "ims_batch_create")
        self._h = h

    def autotune(self, repeats: int = 2, stream=None) -> tuple:
        """Returns the chosen (blocks_per_cu, order, split, ic_alpha, ic_beta)."""
        t = Tuning()
        _check(_lib.ims_batch_autotune(self._h, int(repeats), _stream_handle(stream), ctypes.byref(t)), "ims_batch_autotune")
        return int(t.blocks_per_cu), int(t.order), int(t.split), float(t.ic_alpha), float(t.ic_beta)

    def launch(self, stream=None) -> None:
        _check(_lib.ims_batch_launch(self._h, _stream_handle(stream)), "ims_batch_launch")

    def task_timing(self, enable: bool = True) -> None:
        """Record every task's start, end (device wall clock) and slot at later launches."""
        _check(_lib.ims_batch_task_timing(self._h, int(bool(enable))), "ims_batch_task_timing")

    def task_times(self, max_tasks: int = 1 << 22, stream=None) -> tuple[np.ndarray, np.ndarray]:
        """(task codes uint64[k], times uint64[k, 3] = start, end, slot) of the last launch."""
        codes = np.zeros(max(int(max_tasks), 1), dtype=np.uint64)
        times = np.zeros((max(int(max_tasks), 1), 3), dtype=np.uint64)
        cnt = ctypes.c_uint32()
        _check(_lib.ims_batch_task_times(self._h, int(max_tasks), _np_ptr(codes), _np_ptr(times), ctypes.byref(cnt),
                                         _stream_handle(stream)), "ims_batch_task_times")
        return codes[:cnt.value], times[:cnt.value]

    def results(self) -> list[dict]:
        out = []
        for tc, nc, tot, T in self.outputs:
            total = int(tot.item())
            out.append({"trial_counts": tc.cpu().numpy().view(np.uint32),
                        "node_counts": None if nc is None else nc.cpu().numpy().view(np.uint32),
                        "total": total, "mean": total / T})
        return out

    def close(self):
        if getattr(self, "_h", None) and self._h.value:
            _lib.ims_batch_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def debug_hash(rng_seed: int, domain: int, trials, ids) -> np.ndarray:
    torch = _torch()
    # uint64 counters pass as their bit patterns
    t = torch.as_tensor(np.ascontiguousarray(np.asarray(trials).astype(np.uint64)).view(np.int64)).cuda()
    i = torch.as_tensor(np.ascontiguousarray(np.asarray(ids).astype(np.uint64)).view(np.int64)).cuda()
    out = torch.empty(t.shape[0], dtype=torch.int32, device=t.device)
    _check(_lib.ims_debug_hash(int(rng_seed), int(domain), ctypes.c_void_p(t.data_ptr()),
                               ctypes.c_void_p(i.data_ptr()), ctypes.c_void_p(out.data_ptr()), t.shape[0],
                               _stream_handle(None)), "ims_debug_hash")
    return out.cpu().numpy().view(np.uint32)
