"""Own discrete Fourier transforms for the oracle (no vendor FFT).

TEST INFRASTRUCTURE ONLY (see the package docstring).

The kinetic sub-step of the split-step method, Eq. (3), is a forward Fourier
transform, a phase multiply and an inverse transform.  The paper does not fix
a sign or normalisation convention; here the forward transform is
X[k] = sum_j x[j] exp(-2 pi i j k / N) (unnormalised) and the inverse carries
the 1/N.

``fft_axis`` is an iterative radix-2 decimation-in-time transform along one
axis (bit-reversal permutation, then log2 N butterfly levels), vectorised
over all other axes.  ``dft_axis`` is the O(N^2) definition, for tiny N.
"""
import numpy as np


def _bitrev(n):
    bits = n.bit_length() - 1
    idx = np.arange(n)
    rev = np.zeros(n, dtype=np.int64)
    for b in range(bits):
        rev |= ((idx >> b) & 1) << (bits - 1 - b)
    return rev


def fft_axis(a, axis=-1, inverse=False):
    """Radix-2 FFT of ``a`` along ``axis`` (length must be a power of two)."""
    a = np.moveaxis(np.asarray(a, dtype=np.complex128), axis, -1)
    n = a.shape[-1]
    if n & (n - 1) or n < 1:
        raise ValueError("fft_axis needs a power-of-two length, got %d" % n)
    lead = a.shape[:-1]
    x = a[..., _bitrev(n)].copy()
    sign = 1.0 if inverse else -1.0
    m = 1
    while m < n:
        # blocks of length 2m: first half = DFT of evens, second = DFT of odds
        w = np.exp(sign * 1j * np.pi * np.arange(m) / m)
        x = x.reshape(lead + (n // (2 * m), 2, m))
        even = x[..., 0, :]
        odd = x[..., 1, :] * w
        x = np.stack([even + odd, even - odd], axis=-2).reshape(lead + (n,))
        m *= 2
    if inverse:
        x = x / n
    return np.moveaxis(x, -1, axis)


def dft_axis(a, axis=-1, inverse=False):
    """O(N^2) discrete Fourier transform along ``axis`` (the definition)."""
    a = np.moveaxis(np.asarray(a, dtype=np.complex128), axis, -1)
    n = a.shape[-1]
    jk = np.outer(np.arange(n), np.arange(n)) % n
    sign = 1.0 if inverse else -1.0
    mat = np.exp(sign * 2j * np.pi * jk / n)
    out = a @ mat
    if inverse:
        out = out / n
    return np.moveaxis(out, -1, axis)


def fftn_last(a, ndim, inverse=False, transform=fft_axis):
    """Transform over the last ``ndim`` axes, one axis at a time."""
    out = np.asarray(a, dtype=np.complex128)
    for ax in range(1, ndim + 1):
        out = transform(out, axis=-ax, inverse=inverse)
    return out
