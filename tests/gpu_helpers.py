"""Helpers for the GPU parity tests (no method arithmetic here)."""
import sys

import numpy as np


def say(*a):
    """Progress line, flushed before a GPU step so a crash names its case."""
    print(*a, flush=True)
    sys.stdout.flush()


def normwise(got, ref):
    """max |got - ref| / max |ref| (normwise relative error)."""
    got = np.asarray(got, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    den = np.max(np.abs(ref))
    return float(np.max(np.abs(got - ref)) / (den if den > 0 else 1.0))


def sample_pixels(N, count, seed):
    """Pixel indices k2*N + k1: the four corners, the centre and a seeded
    uniform sample."""
    rng = np.random.default_rng(seed)
    fixed = [0, N - 1, N * (N - 1), N * N - 1, (N // 2) * N + N // 2]
    rnd = rng.integers(0, N * N, size=count)
    return np.unique(np.concatenate([fixed, rnd])).astype(np.int32)


def sample_taps(N, count, seed):
    rng = np.random.default_rng(seed)
    fixed = [(0, 0), (N - 1, N - 1), (-(N - 1), N - 1), (1, 0), (0, 1), (3, -2)]
    rnd = rng.integers(-(N - 1), N, size=(count, 2))
    return np.unique(np.concatenate([np.array(fixed), rnd]), axis=0).astype(np.int32)
