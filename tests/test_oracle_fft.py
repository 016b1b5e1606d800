"""Pins of the oracle's own FFT: brute-force DFT, numpy.fft, closed forms."""
import numpy as np
import pytest

from oracle.fft import dft_axis, fft_axis, fftn_last
from tests.inputs import random_spinors


@pytest.mark.parametrize("n", [1, 2, 4, 8, 16])
@pytest.mark.parametrize("ndim", [1, 2, 3])
def test_fft_equals_naive_dft(n, ndim):
    a = random_spinors(10 + n + ndim, (2,) + (n,) * ndim)
    ref = fftn_last(a, ndim, transform=dft_axis)
    got = fftn_last(a, ndim)
    assert np.max(np.abs(got - ref)) <= 1e-14 * max(1.0, np.max(np.abs(ref)))
    back = fftn_last(got, ndim, inverse=True)
    assert np.max(np.abs(back - a)) <= 1e-14 * np.max(np.abs(a))


@pytest.mark.parametrize("n", [256, 512, 4096])
def test_fft_equals_numpy(n):
    a = random_spinors(n, (3, n))
    got = fft_axis(a, axis=-1)
    ref = np.fft.fft(a, axis=-1)
    assert np.linalg.norm(got - ref) / np.linalg.norm(ref) < 1e-14
    inv = fft_axis(a, axis=-1, inverse=True)
    assert np.linalg.norm(inv - np.fft.ifft(a, axis=-1)) / np.linalg.norm(inv) < 1e-14


def test_fft_axis_argument_and_2d():
    a = random_spinors(7, (4, 32, 64))
    got = fftn_last(a, 2)
    ref = np.fft.fft2(a)
    assert np.linalg.norm(got - ref) / np.linalg.norm(ref) < 1e-14
    got0 = fft_axis(a, axis=1)
    assert np.allclose(got0, np.fft.fft(a, axis=1), rtol=0, atol=1e-12)


def test_fft_closed_forms():
    n = 64
    delta = np.zeros(n, complex)
    delta[0] = 1.0
    assert np.allclose(fft_axis(delta), np.ones(n), atol=1e-15)
    k0 = 5
    wave = np.exp(2j * np.pi * k0 * np.arange(n) / n)
    spec = fft_axis(wave)
    expect = np.zeros(n, complex)
    expect[k0] = n
    assert np.max(np.abs(spec - expect)) < 1e-12
    a = random_spinors(3, (n,))
    assert abs(np.sum(np.abs(fft_axis(a)) ** 2) / n - np.sum(np.abs(a) ** 2)) < 1e-12 * n


def test_fft_rejects_non_power_of_two():
    with pytest.raises(ValueError):
        fft_axis(np.zeros(12, complex))
