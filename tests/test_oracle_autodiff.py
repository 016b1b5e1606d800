"""Pins of the differentiable oracle: same forward map as the numpy oracle,
gradients equal to central finite differences of the numpy oracle's loss."""
import numpy as np
import pytest
import torch

from oracle import autodiff as A
from oracle import spin1 as O
from tests.inputs import random_field, uniform_unit


def np_loss(psi0, q, c1, c0, target, k_cut, nsteps, dt, grid):
    p = O.Params(c0, c1, q)
    psi = O.evolve(psi0, nsteps, dt, p, grid)
    s = O.structure_factor(psi, grid).mean(0)
    mask = O.bin_k(grid) < k_cut
    return float(np.sum((s - target) ** 2 * mask))


def test_torch_step_equals_numpy_oracle():
    g = O.Grid(2, (16, 8), 0.5, 2)
    psi = random_field(31, g.shape, noise=0.5)
    got = A.strang_step(torch.tensor(psi), 0.05, 1.0, -0.3, 0.2, g).numpy()
    ref = O.strang_step(psi, 0.05, O.Params(1.0, -0.3, 0.2), g)
    assert np.max(np.abs(got - ref)) < 1e-13
    sm = A.shell_means(torch.tensor(psi), g).numpy()
    assert np.max(np.abs(sm - O.structure_factor(psi, g))) < 1e-12


@pytest.mark.parametrize("grid", [O.Grid(1, (32,), 0.5, 2), O.Grid(2, (8, 16), 0.5, 2)])
def test_gradients_match_finite_differences(grid):
    psi0 = random_field(32, grid.shape, noise=0.4)
    nb = O.num_bins(grid)
    target = 8.0 * (1.0 + 0.1 * uniform_unit(33, (nb,)))
    args = dict(c0=1.0, target=target, k_cut=3.0, nsteps=4, dt=0.05, grid=grid)
    q, c1 = 0.09, -0.3
    L, gpsi, gq, gc1 = A.gradients(psi0, q, c1, **args)
    assert abs(L - np_loss(psi0, q, c1, **args)) < 1e-12 * max(1.0, L)
    h = 1e-5
    fq = (np_loss(psi0, q + h, c1, **args) - np_loss(psi0, q - h, c1, **args)) / (2 * h)
    fc = (np_loss(psi0, q, c1 + h, **args) - np_loss(psi0, q, c1 - h, **args)) / (2 * h)
    assert abs(gq - fq) < 1e-7 * max(1.0, abs(fq))
    assert abs(gc1 - fc) < 1e-7 * max(1.0, abs(fc))
    rng = np.random.default_rng(34)
    for _ in range(3):
        v = rng.standard_normal(grid.shape) + 1j * rng.standard_normal(grid.shape)
        fd = (np_loss(psi0 + h * v, q, c1, **args) - np_loss(psi0 - h * v, q, c1, **args)) / (2 * h)
        an = float(np.sum(np.real(np.conj(gpsi) * v)))
        assert abs(an - fd) < 1e-7 * max(1.0, abs(fd))
