"""Seeded synthetic inputs shared by the oracle-based tests, smoke() and bench.py.

This module holds random draws only; it contains none of the method's
arithmetic (no basis functions, no index maps, no operators).  All draws use
numpy's PCG64 generator seeded explicitly, so both sides of every parity
check consume the same numbers.
"""
import numpy as np


def rng(seed):
    return np.random.Generator(np.random.PCG64(seed))


def uniform(count, seed, low=-1.0, high=1.0):
    """float64 array of ``count`` draws from U[low, high)."""
    return rng(seed).uniform(low, high, size=int(count))


def integer_valued(count, seed, low=-8, high=8):
    """float64 array of small integers, for sums that must be exact in floating point."""
    return rng(seed).integers(low, high + 1, size=int(count)).astype(np.float64)


def coefficient_modes(seed, max_mode=2):
    """Random Fourier data for a smooth scalar field.

    Returns (modes, amplitudes, phases): modes is an (M, 3) integer array
    covering every m with max|m_a| <= max_mode, amplitudes ~ U[-1, 1],
    phases ~ U[0, 2 pi).
    """
    r = np.arange(-max_mode, max_mode + 1)
    mz, my, mx = np.meshgrid(r, r, r, indexing="ij")
    modes = np.stack([mx.ravel(), my.ravel(), mz.ravel()], axis=1).astype(np.int64)
    g = rng(seed)
    amps = g.uniform(-1.0, 1.0, size=len(modes))
    phases = g.uniform(0.0, 2.0 * np.pi, size=len(modes))
    return modes, amps, phases
