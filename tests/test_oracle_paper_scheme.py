"""Pins of the sub-steps of the paper's own scheme in the oracle (Sec. 2.2,
Eqs. (3)-(5)), each taken alone.

* The generators of the kinetic, diagonal (Eq. (4)) and off-diagonal
  (Eq. (5)) sub-steps add up to the right-hand side of Eq. (2) as printed, so
  a wrong sign, component index or coupling in f_m, a or b fails.
* The diagonal sub-step is the exact flow of its own equation for any dt: the
  phases keep every |psi_m|^2, so the rates f_m stay constant along it.
* The off-diagonal sub-step with the predictor-averaged couplings is a
  second-order approximation of the flow of i d_t psi = c1 S(a(psi), b(psi)) psi:
  its local error falls as dt^3.  A predictor taken over dt instead of
  c1 dt (planted below, on the CPU) leaves an O(dt^2) local error, and the
  same test tells the two apart.
"""
import numpy as np
import scipy.integrate

from oracle import spin1 as O
from tests.inputs import random_field, random_spinors, uniform_unit

P = O.Params(c0=1.0, c1=-0.45, q=0.3)


def rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


def kinetic_rhs(psi, grid):
    """-Lap/2 psi of every component, spectrally with numpy.fft."""
    axes = tuple(range(-grid.dim, 0))
    k2 = O.k_squared(grid)
    return np.stack([np.fft.ifftn(0.5 * k2 * np.fft.fftn(psi[:, c], axes=axes), axes=axes) for c in range(3)],
                    axis=1)


def offdiag_rhs(psi, c1):
    """c1 S(a(psi), b(psi)) psi at every site."""
    a, b = O.paper_couplings(psi)
    s = O.offdiag_matrix(a, b)
    sv = np.moveaxis(psi, 1, -1)
    return np.moveaxis(c1 * np.einsum("...ij,...j->...i", s, sv), -1, 1)


def test_sub_step_generators_add_up_to_printed_eq2():
    g = O.Grid(2, (16, 8), 0.5, 2)
    psi = random_field(31, g.shape, background=0.8, noise=0.6)
    V = 2.0 * uniform_unit(32, g.spatial)
    for v in (None, V):
        total = kinetic_rhs(psi, g) + O.paper_diagonal_rates(psi, P, v) * psi + offdiag_rhs(psi, P.c1)
        assert rel(total, O.gpe_rhs_printed(psi, P, g, V=v)) < 1e-13
    # each part on its own: the off-diagonal part has no diagonal entries, and
    # the rates are real and carry q on m = +1, -1 only
    a, b = O.paper_couplings(psi)
    s = O.offdiag_matrix(a, b)
    assert np.all(s[..., 0, 0] == 0) and np.all(s[..., 1, 1] == 0) and np.all(s[..., 2, 2] == 0)
    r0 = O.paper_diagonal_rates(psi, O.Params(P.c0, P.c1, 0.0))
    r1 = O.paper_diagonal_rates(psi, P)
    assert np.allclose(r1 - r0, np.array([P.q, 0.0, P.q])[None, :, None, None], atol=1e-15)
    # negative control: f_{+1} and f_{-1} taking their own density instead of
    # the other component's (a plausible index mistake, planted in a copy) no
    # longer add up
    d = np.abs(psi) ** 2
    swapped = O.paper_diagonal_rates(psi, P).copy()
    swapped[:, 0] += 2.0 * P.c1 * (d[:, 2] - d[:, 0])
    swapped[:, 2] += 2.0 * P.c1 * (d[:, 0] - d[:, 2])
    total = kinetic_rhs(psi, g) + swapped * psi + offdiag_rhs(psi, P.c1)
    assert rel(total, O.gpe_rhs_printed(psi, P, g)) > 1e-3


def test_paper_kinetic_is_the_free_flow():
    """Eq. (3) alone: a plane wave e^{i k0 x} in every component gets e^{-i k0^2 dt / 2}, no q."""
    g = O.Grid(1, (32,), 0.5, 1)
    k0 = 2 * np.pi * 3 / (32 * 0.5)
    x = np.arange(32) * 0.5
    psi = np.zeros(g.shape, complex)
    coef = random_spinors(33, (3,))
    for c in range(3):
        psi[0, c] = coef[c] * np.exp(1j * k0 * x)
    for dt in (0.01, 0.7):
        out = O.paper_kinetic(psi, dt, g)
        assert rel(out, psi * np.exp(-0.5j * k0 ** 2 * dt)) < 1e-13


def ode_flow(rhs, psi, t):
    """Flow of i d_t psi = rhs(psi) over t by DOP853 (rtol 1e-13)."""
    shape = psi.shape

    def f(_, y):
        z = y[: y.size // 2] + 1j * y[y.size // 2:]
        d = -1j * rhs(z.reshape(shape)).ravel()
        return np.concatenate([d.real, d.imag])

    y0 = np.concatenate([psi.ravel().real, psi.ravel().imag])
    sol = scipy.integrate.solve_ivp(f, (0.0, t), y0, method="DOP853", rtol=1e-13, atol=1e-15)
    z = sol.y[: y0.size // 2, -1] + 1j * sol.y[y0.size // 2:, -1]
    return z.reshape(shape)


def test_paper_diagonal_is_exact_flow_of_its_rates():
    """Eq. (4) with the densities of the field it multiplies is the exact flow
    of i d_t psi_m = f_m(|psi|^2) psi_m (the |psi_m|^2 are constants of it), for
    small and large steps, with and without the potential."""
    g = O.Grid(1, (8,), 0.5, 2)
    psi = random_field(34, g.shape, background=1.0, noise=0.7)
    V = uniform_unit(35, g.spatial)
    for v in (None, V):
        for dt in (0.05, 1.3):
            ref = ode_flow(lambda z: O.paper_diagonal_rates(z, P, v) * z, psi, dt)
            assert rel(O.paper_diagonal(psi, dt, P, v), ref) < 1e-11


def offdiag_local_errors(step, psi, c1, dts):
    return [rel(step(psi, dt, c1), ode_flow(lambda z: offdiag_rhs(z, c1), psi, dt)) for dt in dts]


def wrong_predictor_step(psi, dt, c1):
    """Eq. (5) with the predictor taken over dt instead of c1 dt: a plausible
    mistake planted in a copy of the oracle's sub-step (negative control)."""
    a0, b0 = O.paper_couplings(psi)
    sv = np.moveaxis(psi, 1, -1)
    pred = sv - 1j * dt * np.einsum("...ij,...j->...i", O.offdiag_matrix(a0, b0), sv)
    a = 0.5 * (a0 + np.conj(pred[..., 2]) * pred[..., 1])
    b = 0.5 * (b0 + np.conj(pred[..., 1]) * pred[..., 0])
    return np.moveaxis(np.einsum("...ij,...j->...i", O.eq5_matrix(a, b, c1 * dt), sv), -1, 1)


def test_paper_offdiagonal_local_error_is_third_order():
    """Eq. (5) with couplings averaged over psi and the predictor approximates
    the flow of i d_t psi = c1 S(a(psi), b(psi)) psi with an O(dt^3) local error
    (the averaged couplings are the trapezoidal mean of a(t), b(t) to O(dt^2)).
    The planted predictor over dt instead of c1 dt only reaches O(dt^2)."""
    g = O.Grid(1, (8,), 0.5, 3)
    psi = random_field(36, g.shape, background=1.0, noise=0.8)
    dts = (0.1, 0.05, 0.025, 0.0125)
    e = offdiag_local_errors(O.paper_offdiagonal, psi, P.c1, dts)
    ratios = [e[i] / e[i + 1] for i in range(len(e) - 1)]
    assert all(7.0 < r < 9.0 for r in ratios), ratios
    w = offdiag_local_errors(wrong_predictor_step, psi, P.c1, dts)
    wr = [w[i] / w[i + 1] for i in range(len(w) - 1)]
    assert all(3.0 < r < 5.0 for r in wr), wr
    assert not all(7.0 < r < 9.0 for r in wr)
    # the off-diagonal flow keeps |psi|^2 at every site; so does the sub-step
    out = O.paper_offdiagonal(psi, 0.2, P.c1)
    assert np.allclose(O.density(out), O.density(psi), rtol=1e-13)


def test_paper_step_composes_its_sub_steps():
    g = O.Grid(2, (8, 16), 0.5, 1)
    psi = random_field(37, g.shape)
    V = uniform_unit(38, g.spatial)
    manual = O.paper_offdiagonal(O.paper_diagonal(O.paper_kinetic(psi, 0.03, g), 0.03, P, V), 0.03, P.c1)
    assert np.array_equal(O.paper_step(psi, 0.03, P, g, V=V), manual)
