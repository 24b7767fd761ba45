"""Host-side checks of the C-ABI library that need no GPU: it loads, exports
every function the headers under include/ declare, and its encoders and validation
behave as the header states."""
import ctypes
import os
import re

import numpy as np
import pytest

import oracle
import paper_2404_17059_amd as ims

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    text = "".join(open(os.path.join(ROOT, "include", h)).read()
                   for h in sorted(os.listdir(os.path.join(ROOT, "include"))) if h.endswith(".h"))
    return sorted(set(re.findall(r"^\s*(?:const\s+)?[\w\s\*]+?\b(ims_\w+)\s*\(", text, flags=re.M)))


def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(ims.LIB_PATH)
    names = declared_functions()
    assert len(names) >= 10, names
    for name in names:
        assert hasattr(lib, name), name


def test_version():
    assert "gfx950" in ims.version()


def test_encode_p_closed_forms_and_agrees_with_oracle():
    p = np.array([0.0, 2.0**-33, 0.01, 0.1, 0.5, 1 - 2.0**-33, 1.0, 2.0**-32])
    assert ims.encode_p(p).tolist() == [0, 0, 0x028F5C28, 0x19999999, 0x80000000, 0xFFFFFFFF, 0xFFFFFFFF, 1]
    r = np.random.default_rng(0).random(10000)
    assert (ims.encode_p(r) == oracle.encode_p(r)).all()


def test_encode_w_closed_forms_and_agrees_with_oracle():
    d = np.arange(1, 500)
    assert ims.encode_w(1.0 / d).tolist() == [(1 << 32) // int(k) for k in d]
    r = np.random.default_rng(1).random(10000)
    assert (ims.encode_w(r) == oracle.encode_w(r)).all()


@pytest.mark.parametrize("bad", [float("nan"), -0.5, 1.5])
def test_encoders_reject(bad):
    with pytest.raises(ims.ImsError) as e:
        ims.encode_p([0.2, bad])
    assert e.value.code == -1
    with pytest.raises(ims.ImsError):
        ims.encode_w([bad])


def test_validate_csr_errors():
    ims.validate_csr(3, [0, 2, 3, 3], [1, 2, 0])
    for off, idx in [([1, 2, 3, 3], [1, 2, 0]), ([0, 2, 1, 3], [1, 2, 0]), ([0, 2, 3, 3], [1, 2, 3]),
                     ([0, 2, 3, 4], [1, 2, 0])]:
        with pytest.raises(ims.ImsError) as e:
            ims.validate_csr(3, off, idx)
        assert e.value.code == -2


def test_graph_create_rejects_before_touching_the_device():
    off = np.array([0, 2, 3, 3], dtype=np.int64)
    idx = np.array([2, 2, 2], dtype=np.uint32)
    with pytest.raises(ims.ImsError) as e:
        ims.Graph(3, off, idx, "lt", np.array([1 << 31, 1 << 31, 1], dtype=np.uint64))
    assert e.value.code == -3
    with pytest.raises(ims.ImsError) as e:
        ims.Graph(3, off, np.array([2, 2, 7], dtype=np.uint32), "ic", np.zeros(3))
    assert e.value.code == -2
    with pytest.raises(ims.ImsError) as e:
        ims.Graph(3, off, idx, "ic", np.array([0.1, 2.0, 0.1]))
    assert e.value.code == -1


def test_output_buffers_checked_before_any_device_call():
    """The binding rejects outputs the library could not write safely (host
    tensors, wrong item size, too small, not contiguous, missing) before it
    touches the device; a stand-in graph object is enough since nothing
    reaches the library."""
    import types

    import torch
    g = types.SimpleNamespace(n=10, handle=None)
    cases = [
        dict(trial_counts=torch.zeros(5, dtype=torch.int32), total=torch.zeros(1, dtype=torch.int64)),
        dict(trial_counts=None, total=torch.zeros(1, dtype=torch.int64)),
    ]
    for kw in cases:
        for fn in (ims.simulate_into, ims.simulate_noalloc_into):
            with pytest.raises(ims.ImsError) as e:
                fn(g, [0], 5, 1, **kw)
            assert e.value.code == -1
    with pytest.raises(ims.ImsError):
        ims.simulate_sets_into(g, np.array([0, 1], dtype=np.uint32), np.array([0], dtype=np.uint32), 5, 1,
                               torch.zeros(1, dtype=torch.int64))
    with pytest.raises(ims.ImsError):
        ims.simulate_sets_from_into(g, torch.zeros(10, dtype=torch.int64), np.array([0, 1], dtype=np.uint32),
                                    np.array([0], dtype=np.uint32), 5, 1, torch.zeros(1, dtype=torch.int64))
    # the checks themselves, without a GPU (only the host-tensor rule applies here)
    with pytest.raises(ims.ImsError, match="CUDA tensor"):
        ims._dev_ptr(torch.zeros(4, dtype=torch.int32), "w", "x", 4, 4)
    with pytest.raises(ims.ImsError, match="required"):
        ims._dev_ptr(None, "w", "x", 4, 4)
    assert ims._dev_ptr(None, "w", "x", 4, 4, required=False) is None
