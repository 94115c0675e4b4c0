"""Shared helpers for the GPU parity tests: seeded inputs and error measures."""
import math

import numpy as np

from paper_1406_0359_amd import synth

DEV = "cuda:0"


def rel_l2(a, b):
    a = np.asarray(a)
    b = np.asarray(b)
    return float(np.linalg.norm((a - b).ravel()) / np.linalg.norm(b.ravel()))


def max_rel(a, b):
    """max_j |a_j - b_j| / max_j |b_j| (element-wise, scaled by the largest reference value)."""
    a = np.asarray(a).ravel()
    b = np.asarray(b).ravel()
    return float(np.max(np.abs(a - b)) / np.max(np.abs(b)))


def uv_case(M, n, seed, uniform_frac=0.0):
    return synth.uv_coverage(M, 2 * n, np.random.default_rng(seed), uniform_frac)


def rand_complex(shape, seed):
    rng = np.random.default_rng(seed)
    return rng.standard_normal(shape) + 1j * rng.standard_normal(shape)


def to_np(t):
    return t.detach().cpu().numpy()
