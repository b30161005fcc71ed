"""Helpers shared by the GPU parity tests (comparison metrics, device transfer)."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")


def dev():
    return torch.device("cuda:0")


def to_dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(dev())


def normwise(got, ref):
    """max_k |got_k - ref_k| / max_k |ref_k| -- the per-fit gate for coefficient vectors."""
    got = np.asarray(got, float)
    ref = np.asarray(ref, float)
    return float(np.max(np.abs(got - ref)) / np.max(np.abs(ref)))


def per_coef(got, ref):
    got = np.asarray(got, float)
    ref = np.asarray(ref, float)
    return np.abs(got - ref) / np.abs(ref)


def announce(msg):
    print(msg, flush=True)
