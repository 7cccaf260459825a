"""Helpers for the GPU parity tests (comparison only; no expected values come from here)."""

import sys

import numpy as np

from oracle import ptebd_oracle as po


# The FP32 path drops sigma <= max(cutoff, 2^-19) sigma_1 (documented in include/ptebd.h);
# the oracle is run with the same effective cutoff when it checks that path.
FP32_CUTOFF_FLOOR = 2.0 ** -19


def oracle_cutoff(cutoff: float, precision: str) -> float:
    return max(cutoff, FP32_CUTOFF_FLOOR) if precision == "fp32" else cutoff


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
