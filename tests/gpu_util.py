"""Helpers for the GPU parity tests (no arithmetic of the method here)."""
import numpy as np
import pytest

try:
    import torch
except Exception:  # pragma: no cover
    torch = None

TOL = 1e-5  # relative L2 against the FP64 oracle, per image / per signal


def need_gpu():
    if torch is None or not torch.cuda.is_available():
        pytest.skip("no GPU")


def announce(msg):
    print("[gpu case] %s" % msg, flush=True)


def to_dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def to_host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def rel_l2(got, ref, nd):
    """max over leading entries of ||got - ref|| / ||ref|| over the last nd axes."""
    got = np.asarray(got, dtype=np.complex128)
    ref = np.asarray(ref, dtype=np.complex128)
    assert got.shape == ref.shape, (got.shape, ref.shape)
    lead = int(np.prod(got.shape[:got.ndim - nd])) if got.ndim > nd else 1
    g = got.reshape(lead, -1)
    r = ref.reshape(lead, -1)
    num = np.linalg.norm(g - r, axis=1)
    den = np.maximum(np.linalg.norm(r, axis=1), 1e-300)
    return float(np.max(num / den))
