"""Pins of the oracle's trap potential V(x) (the V_m of Eq. (4), the same for
the three components) against closed forms, an ODE solver and invariants."""
import numpy as np
import pytest
import scipy.integrate

from oracle import spin1 as O
from tests.inputs import random_field, random_spinors


def rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


def harmonic(grid, omega, centre):
    """V = omega^2 |x - centre|^2 / 2 on the grid (spatial shape)."""
    axes = [np.arange(grid.n[a]) * grid.dx - centre[a] for a in range(grid.dim)]
    mesh = np.meshgrid(*reversed(axes), indexing="ij")  # [.., y, x]
    return 0.5 * omega ** 2 * sum(m ** 2 for m in mesh)


def test_energy_with_trap_is_generator_of_eq2_with_trap():
    """i d_t psi = dE/dpsi^* / dx^d with V n in the energy and V in the bracket."""
    g = O.Grid(1, (16,), 0.5, 1)
    psi = random_field(31, g.shape, noise=0.5)
    p = O.Params(c0=0.8, c1=-0.3, q=0.4)
    V = np.random.default_rng(5).uniform(-2.0, 3.0, size=g.spatial)
    rhs = O.gpe_rhs_printed(psi, p, g, V=V)
    rhs0 = O.gpe_rhs_printed(psi, p, g)
    assert np.allclose(rhs - rhs0, V[None, None] * psi, atol=1e-13)
    h = 1e-6
    for (c, j) in [(0, 3), (1, 0), (2, 11), (1, 7)]:
        grad = 0.0
        for unit, fac in ((1.0, 0.5), (1j, 0.5j)):
            e = np.zeros_like(psi)
            e[0, c, j] = unit * h
            dplus = O.observables(psi + e, p, g, V=V)[0, 2]
            dminus = O.observables(psi - e, p, g, V=V)[0, 2]
            grad += fac * (dplus - dminus) / (2 * h)
        assert abs(grad / g.cell - rhs[0, c, j]) < 1e-6 * max(1.0, abs(rhs[0, c, j]))


def test_local_flow_with_trap_solves_local_ode():
    """R(tau) with V equals the ODE flow of i d_t psi = (V + c0 n + c1 F.f) psi."""
    p = O.Params(c0=0.9, c1=-0.45, q=0.0)
    psi0 = random_spinors(41, (1, 3, 8))
    psi0[0, :, 0] = [1e-7, 1.0, 2e-7]  # nearly polar: |F| ~ 1e-7
    V = np.array([0.0, 1.3, -2.1, 0.4, 5.0, -0.7, 2.2, 0.9])
    g = O.Grid(1, (8,), 1.0, 1)

    def f(t, y):
        y = y.reshape(psi0.shape)
        full = O.gpe_rhs_printed(y, p, g, V=V)
        lap = np.fft.ifft(0.5 * O.k_squared(g) * np.fft.fft(y, axis=-1), axis=-1)
        return (-1j * (full - lap)).ravel()

    for tau in (0.07, 1.3):
        sol = scipy.integrate.solve_ivp(f, (0, tau), psi0.ravel(), method="DOP853", rtol=1e-12, atol=1e-14)
        ref = sol.y[:, -1].reshape(psi0.shape)
        got = O.local_flow(psi0, tau, p.c0, p.c1, V=V)
        assert rel(got, ref) < 1e-10


@pytest.mark.parametrize("step", [O.strang_step, O.paper_step])
def test_constant_potential_is_a_global_phase(step):
    """V = V0 everywhere multiplies the state by exp(-i V0 t), for any dt."""
    g = O.Grid(2, (16, 8), 0.5, 2)
    psi = random_field(43, g.shape, noise=0.6)
    p = O.Params(c0=1.1, c1=-0.3, q=0.25)
    V0 = 0.83
    dt, n = 0.3, 7
    with_v = O.evolve(psi, n, dt, p, g, step=step, V=np.full(g.spatial, V0))
    without = O.evolve(psi, n, dt, p, g, step=step)
    assert rel(with_v, np.exp(-1j * V0 * n * dt) * without) < 1e-12


def test_harmonic_ground_state_is_stationary_second_order():
    """Linear case c0 = c1 = q = 0: the ground state of V = w^2 (x - xc)^2 / 2,
    (w/pi)^(1/4) exp(-w (x - xc)^2 / 2), only acquires exp(-i w t / 2); the
    split-step error is second order in dt."""
    g = O.Grid(1, (128,), 0.25, 1)
    w, xc = 0.5, 16.0
    x = np.arange(128) * 0.25
    gs = (w / np.pi) ** 0.25 * np.exp(-0.5 * w * (x - xc) ** 2)
    psi = np.zeros(g.shape, complex)
    for c in range(3):
        psi[0, c] = gs * (1.0 + 0.5j * c)
    V = harmonic(g, w, (xc,))
    p = O.Params(c0=0.0, c1=0.0, q=0.0)
    t = 2.0
    ref = np.exp(-0.5j * w * t) * psi
    errs = [rel(O.evolve(psi, m, t / m, p, g, V=V), ref) for m in (20, 40, 80)]
    assert errs[-1] < 2e-4
    assert 3.6 < errs[0] / errs[1] < 4.4 and 3.6 < errs[1] / errs[2] < 4.4


def test_harmonic_centre_of_mass_oscillates():
    """Linear case: a displaced ground state keeps its shape and its centre
    follows x0 cos(w t) about the trap centre (Ehrenfest, exact for a
    harmonic trap); the split-step error is second order in dt."""
    g = O.Grid(1, (128,), 0.25, 1)
    w, xc, x0 = 0.5, 16.0, 2.0
    x = np.arange(128) * 0.25
    psi = np.zeros(g.shape, complex)
    psi[0, 1] = (w / np.pi) ** 0.25 * np.exp(-0.5 * w * (x - xc - x0) ** 2)
    V = harmonic(g, w, (xc,))
    p = O.Params(c0=0.0, c1=0.0, q=0.0)
    t = 3.0

    def centre(f):
        d = np.abs(f[0, 1]) ** 2
        return np.sum(d * (x - xc)) / np.sum(d)

    errs = [abs(centre(O.evolve(psi, m, t / m, p, g, V=V)) - x0 * np.cos(w * t)) for m in (30, 60, 120)]
    assert errs[-1] < 1e-3
    assert 3.5 < errs[0] / errs[1] < 4.5 and 3.5 < errs[1] / errs[2] < 4.5


def test_trap_norm_fz_conserved_energy_second_order():
    """With a trap and interactions, N and F_z stay exact and E (with V n)
    oscillates with an amplitude proportional to dt^2."""
    g = O.Grid(1, (64,), 0.5, 2)
    psi = random_field(47, g.shape, noise=0.3)
    V = harmonic(g, 0.2, (16.0,))
    p = O.Params(c0=1.0, c1=-0.1, q=0.09)
    o0 = O.observables(psi, p, g, V=V)
    drift = []
    for dt, nst in ((0.04, 50), (0.02, 100)):
        cur = psi.copy()
        worst = 0.0
        for _ in range(nst):
            cur = O.strang_step(cur, dt, p, g, V=V)
            o = O.observables(cur, p, g, V=V)
            assert np.allclose(o[:, 0], o0[:, 0], rtol=1e-13)
            assert np.allclose(o[:, 1], o0[:, 1], rtol=0, atol=1e-12 * abs(o0[:, 0]).max())
            worst = max(worst, np.max(np.abs(o[:, 2] - o0[:, 2])))
        drift.append(worst)
    assert 3.0 < drift[0] / drift[1] < 5.0


def test_paper_scheme_with_trap_first_order_same_limit():
    """The Lie scheme with V in Eq. (4) converges (first order) to the Strang flow with V."""
    g = O.Grid(1, (16,), 0.5, 1)
    x = np.arange(16) * 0.5
    psi = np.zeros(g.shape, complex)
    coef = random_spinors(49, (3, 2), 0.3)
    for c in range(3):
        psi[0, c] = coef[c, 0] + coef[c, 1] * np.exp(2j * np.pi * x / 8.0)
    psi[0, 1] += 1.0
    V = 0.6 * np.cos(2 * np.pi * x / 8.0)
    p = O.Params(c0=1.0, c1=-0.4, q=0.2)
    t = 0.5
    ref = O.evolve(psi, 200, t / 200, p, g, V=V)
    e = [rel(O.evolve(psi, m, t / m, p, g, step=O.paper_step, V=V), ref) for m in (20, 40, 80)]
    r1, r2 = e[0] / e[1], e[1] / e[2]
    assert 1.6 < r1 < 2.6 and 1.6 < r2 < 2.6
