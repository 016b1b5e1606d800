"""Differentiable FP64 reference of the split-step map (torch on the CPU).

TEST INFRASTRUCTURE ONLY (see the package docstring).

The same symmetric step as ``oracle.spin1.strang_step`` (readings there),
written with torch complex128 CPU operations so that torch autograd gives an
independent gradient of a structure-factor loss with respect to the initial
field, q and c1:

  * R(tau): per-site exp(-i tau (c0 n + c1 F.f)) by ``torch.linalg.matrix_exp``
    of the Hermitian site matrix (n and F taken from the field it acts on);
  * K Q(dt): own radix-2 FFT along each axis (bit reversal + butterflies,
    twiddles from ``torch.exp``), phase exp(-i(|k|^2/2 + q m^2) dt), inverse;
  * loss: L = sum over shells b with k_b < k_cut of (S_b - T_b)^2, S_b the
    sample mean of the per-sample shell means of |DFT F_perp|^2 / N_sites.

Torch's gradient of a real loss with respect to a complex tensor is
dL/dRe + i dL/dIm; the library's adjoint returns the same convention.
"""
import math

import numpy as np
import torch

from . import spin1 as O

SQRT2 = math.sqrt(2.0)


def _spin_matrices():
    fx, fy, fz = O.spin_matrices()
    return [torch.tensor(f, dtype=torch.complex128) for f in (fx, fy, fz)]


def _bitrev(n):
    bits = n.bit_length() - 1
    idx = np.arange(n)
    rev = np.zeros(n, dtype=np.int64)
    for b in range(bits):
        rev |= ((idx >> b) & 1) << (bits - 1 - b)
    return torch.tensor(rev)


def fft_last(x, inverse=False):
    """Radix-2 transform along the last axis (unnormalised forward; inverse /N)."""
    n = x.shape[-1]
    lead = x.shape[:-1]
    y = x[..., _bitrev(n)]
    sign = 1.0 if inverse else -1.0
    m = 1
    while m < n:
        w = torch.exp(sign * 1j * math.pi * torch.arange(m, dtype=torch.float64) / m)
        y = y.reshape(lead + (n // (2 * m), 2, m))
        even = y[..., 0, :]
        odd = y[..., 1, :] * w
        y = torch.stack([even + odd, even - odd], dim=-2).reshape(lead + (n,))
        m *= 2
    return y / n if inverse else y


def fftn(x, ndim, inverse=False):
    for ax in range(1, ndim + 1):
        x = torch.movedim(fft_last(torch.movedim(x, -ax, -1), inverse), -1, -ax)
    return x


def local_flow(psi, tau, c0, c1):
    """exp(-i tau (c0 n + c1 F.f)) at every site; psi [S, 3, ...]."""
    fm = _spin_matrices()
    sv = torch.movedim(psi, 1, -1)                       # [S, ..., 3]
    n = (sv.conj() * sv).real.sum(-1)
    h = c0 * n[..., None, None] * torch.eye(3, dtype=torch.complex128)
    for f in fm:
        fa = torch.einsum("...i,ij,...j->...", sv.conj(), f, sv).real
        h = h + c1 * fa[..., None, None] * f
    u = torch.linalg.matrix_exp(-1j * tau * h)
    out = torch.einsum("...ij,...j->...i", u, sv)
    return torch.movedim(out, -1, 1)


def kinetic_zeeman(psi, dt, q, grid):
    k2 = torch.tensor(O.k_squared(grid), dtype=torch.float64)
    outs = []
    for c, m in enumerate((1.0, 0.0, -1.0)):
        phase = torch.exp(-1j * (0.5 * k2 + q * m * m) * dt)
        outs.append(fftn(fftn(psi[:, c], grid.dim) * phase, grid.dim, inverse=True))
    return torch.stack(outs, dim=1)


def strang_step(psi, dt, c0, c1, q, grid):
    psi = local_flow(psi, 0.5 * dt, c0, c1)
    psi = kinetic_zeeman(psi, dt, q, grid)
    return local_flow(psi, 0.5 * dt, c0, c1)


def shell_means(psi, grid):
    """Per-sample shell means of |DFT F_perp|^2 / N_sites, [S, n_bins]."""
    p1, p0, pm = psi[:, 0], psi[:, 1], psi[:, 2]
    fp = SQRT2 * (p1.conj() * p0 + p0.conj() * pm)
    power = (fftn(fp, grid.dim).abs() ** 2) / grid.sites
    b = torch.tensor(O.bin_index(grid).ravel())
    counts = torch.bincount(b).to(torch.float64)
    out = torch.zeros((grid.samples, counts.numel()), dtype=torch.float64)
    out = out.index_add(1, b, power.reshape(grid.samples, -1))
    return out / counts


def loss(psi0, q, c1, c0, target, k_cut, nsteps, dt, grid):
    """L(psi0, q, c1) of the structure factor after nsteps steps."""
    psi = psi0
    for _ in range(nsteps):
        psi = strang_step(psi, dt, c0, c1, q, grid)
    s = shell_means(psi, grid).mean(0)
    kb = torch.tensor(O.bin_k(grid))
    mask = kb < k_cut
    return ((s - target) ** 2 * mask).sum()


def gradients(psi0, q, c1, c0, target, k_cut, nsteps, dt, grid):
    """(L, dL/dpsi0 [complex, dL/dRe + i dL/dIm], dL/dq, dL/dc1) by autograd."""
    p = torch.tensor(psi0, dtype=torch.complex128, requires_grad=True)
    tq = torch.tensor(float(q), dtype=torch.float64, requires_grad=True)
    tc1 = torch.tensor(float(c1), dtype=torch.float64, requires_grad=True)
    tgt = torch.tensor(np.asarray(target), dtype=torch.float64)
    L = loss(p, tq, tc1, float(c0), tgt, k_cut, nsteps, dt, grid)
    L.backward()
    return float(L.detach()), p.grad.numpy(), float(tq.grad), float(tc1.grad)
