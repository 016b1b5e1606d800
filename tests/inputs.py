"""Seeded synthetic inputs shared by the oracle side and the HIP side of tests.

Only random arrays and their shapes live here: no step of the method.
"""
import numpy as np


def rng(seed):
    return np.random.default_rng(seed)


def random_spinors(seed, shape, scale=1.0):
    """Complex Gaussian array of the given shape (FP64)."""
    g = rng(seed)
    return scale * (g.standard_normal(shape) + 1j * g.standard_normal(shape))


def random_field(seed, shape, background=1.0, noise=0.3):
    """Field [S, 3, ...] = polar background on the middle component plus noise."""
    psi = random_spinors(seed, shape, noise)
    psi[:, 1] += background
    return psi


def uniform_unit(seed, shape):
    return rng(seed).uniform(-1.0, 1.0, size=shape)
