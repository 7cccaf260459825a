"""Helpers for the GPU parity tests (comparison only; no expected values come from here)."""

import sys

import numpy as np

from oracle import ptebd_oracle as po


def say(*args):
    print(*args, flush=True)
    sys.stdout.flush()


def to_oracle(mps_gpu, s=0) -> po.VidalMPS:
    """The GPU state exported to host complex128 arrays, wrapped for comparisons."""
    g, l = mps_gpu.export(s)
    return po.VidalMPS(g, l)


def lambda_diff(a: po.VidalMPS, b: po.VidalMPS) -> float:
    assert a.bond_dims() == b.bond_dims(), (a.bond_dims(), b.bond_dims())
    return max(float(np.max(np.abs(x - y))) for x, y in zip(a.lam, b.lam))
