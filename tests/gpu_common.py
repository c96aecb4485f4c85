"""Helpers of the GPU parity tests (device buffers, oracle references)."""

import json
import os

import numpy as np
import pytest

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def torch_cuda():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def workload_params():
    with open(os.path.join(GOLDEN, "workload_params.json")) as f:
        return json.load(f)


def rel_err(got, ref, floor_frac=1e-10):
    """max and median relative error over entries above floor_frac * max|ref|."""
    ref = np.asarray(ref)
    got = np.asarray(got)
    scale = np.max(np.abs(ref))
    sel = np.abs(ref) > floor_frac * scale
    if not np.any(sel):
        return 0.0, 0.0, float(np.max(np.abs(got - ref)))
    r = np.abs(got[sel] - ref[sel]) / np.abs(ref[sel])
    absmax = float(np.max(np.abs(got[~sel] - ref[~sel]))) if np.any(~sel) else 0.0
    return float(np.max(r)), float(np.median(r)), absmax
