"""Pins of the oracle's split-step method against the paper and mathematics.

Each test ties one part of ``oracle.spin1`` to something other than itself:
Eq. (2) as printed, an ODE solver, a closed-form solution, an invariant, a
symmetry, or a statistical closed form.
"""
import numpy as np
import pytest
import scipy.integrate
import scipy.linalg

from oracle import spin1 as O
from tests.inputs import random_field, random_spinors

P1 = O.Params(c0=1.0, c1=-0.1, q=0.09)


def grid1(n=32, s=2, dx=0.5):
    return O.Grid(1, (n,), dx, s)


def rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


def local_rhs_printed(psi, p):
    """Eq. (2) as printed without the Laplacian (the kinetic part is then
    zero only for uniform fields, so it is removed explicitly here)."""
    g = O.Grid(1, (psi.shape[-1],), 1.0, psi.shape[0])
    full = O.gpe_rhs_printed(psi, p, g)
    k2 = O.k_squared(g)
    lap = np.fft.ifft(0.5 * k2 * np.fft.fft(psi, axis=-1), axis=-1)
    return full - lap


# ---------------------------------------------------------------- Eq. (2)
def test_generator_form_equals_printed_eq2():
    """[-Lap/2 + q f_z^2 + c0 n + c1 F.f] psi equals the printed Eq. (2)."""
    g = O.Grid(2, (16, 8), 0.5, 2)
    psi = random_field(1, g.shape, noise=0.7)
    p = O.Params(c0=1.3, c1=-0.37, q=0.21)
    printed = O.gpe_rhs_printed(psi, p, g)
    h = O.local_hamiltonian(psi, p.c0, p.c1)
    loc = np.einsum("s...ij,sj...->si...", h, psi)
    zee = p.q * psi * (O.M_VALUES ** 2)[None, :, None, None]
    k2 = O.k_squared(g)
    kin = np.fft.ifftn(0.5 * k2 * np.fft.fftn(psi, axes=(-2, -1)), axes=(-2, -1))
    assert rel(kin + zee + loc, printed) < 1e-13


def test_spin_vector_components():
    """F_+ = sqrt2 (psi_1^* psi_0 + psi_0^* psi_-1), F_z = |psi_1|^2 - |psi_-1|^2."""
    psi = random_spinors(2, (3, 3, 10))
    fx, fy, fz = O.spin_vector(psi)
    fp = np.sqrt(2) * (np.conj(psi[:, 0]) * psi[:, 1] + np.conj(psi[:, 1]) * psi[:, 2])
    assert np.allclose(fx + 1j * fy, fp, atol=1e-13)
    assert np.allclose(fz, np.abs(psi[:, 0]) ** 2 - np.abs(psi[:, 2]) ** 2, atol=1e-13)


def test_energy_is_generator_of_eq2():
    """i d_t psi = dE/dpsi^* / dx^d, with dE/dpsi^* from central differences."""
    g = O.Grid(1, (16,), 0.5, 1)
    psi = random_field(3, g.shape, noise=0.5)
    p = O.Params(c0=0.8, c1=-0.3, q=0.4)
    rhs = O.gpe_rhs_printed(psi, p, g)
    h = 1e-6
    for (c, j) in [(0, 3), (1, 0), (2, 11), (1, 7)]:
        grad = 0.0
        for unit, fac in ((1.0, 0.5), (1j, 0.5j)):
            e = np.zeros_like(psi)
            e[0, c, j] = unit * h
            dplus = O.observables(psi + e, p, g)[0, 2]
            dminus = O.observables(psi - e, p, g)[0, 2]
            grad += fac * (dplus - dminus) / (2 * h)
        assert abs(grad / g.cell - rhs[0, c, j]) < 1e-6 * max(1.0, abs(rhs[0, c, j]))


# ---------------------------------------------------------------- R (local)
def test_local_flow_solves_printed_local_eq2():
    """R(tau) equals the ODE flow of Eq. (2)'s local part (q = 0), any tau."""
    p = O.Params(c0=0.9, c1=-0.45, q=0.0)
    psi0 = random_spinors(4, (1, 3, 8))
    psi0[0, :, 0] = [1e-7, 1.0, 2e-7]          # nearly polar: |F| ~ 1e-7
    psi0[0, :, 1] = [1.5, 0.1 + 0.2j, -0.7]    # large |F|
    for tau in (0.05, 1.7):
        def f(t, y):
            return (-1j * local_rhs_printed(y.reshape(psi0.shape), p)).ravel()
        sol = scipy.integrate.solve_ivp(f, (0, tau), psi0.ravel(), method="DOP853",
                                        rtol=1e-12, atol=1e-14)
        ref = sol.y[:, -1].reshape(psi0.shape)
        got = O.local_flow(psi0, tau, p.c0, p.c1)
        assert rel(got, ref) < 1e-10


def test_local_flow_equals_expm():
    psi = random_spinors(5, (2, 3, 4), 1.3)
    psi[1, :, 2] = [0.0, 0.7, 0.0]
    tau, c0, c1 = 0.37, 1.1, -0.6
    h = O.local_hamiltonian(psi, c0, c1)
    got = O.local_flow(psi, tau, c0, c1)
    for s in range(2):
        for j in range(4):
            u = scipy.linalg.expm(-1j * tau * h[s, j])
            assert np.allclose(got[s, :, j], u @ psi[s, :, j], atol=1e-13)


def test_local_flow_conserves_n_and_F_pointwise():
    psi = random_spinors(6, (2, 3, 16), 0.8)
    out = O.local_flow(psi, 2.3, 1.0, -0.7)
    assert np.allclose(O.density(out), O.density(psi), atol=1e-13)
    for a, b in zip(O.spin_vector(out), O.spin_vector(psi)):
        assert np.allclose(a, b, atol=1e-13)


def test_local_flow_group_and_inverse():
    psi = random_spinors(7, (1, 3, 16))
    c0, c1 = 1.0, -0.5
    a = O.local_flow(O.local_flow(psi, 0.3, c0, c1), 0.45, c0, c1)
    b = O.local_flow(psi, 0.75, c0, c1)
    assert rel(a, b) < 1e-13
    back = O.local_flow(O.local_flow(psi, 0.9, c0, c1), -0.9, c0, c1)
    assert rel(back, psi) < 1e-13


def test_uniform_polar_phase():
    """Uniform polar state: psi_0 = sqrt(n) exp(-i c0 n t), psi_{+-1} = 0."""
    g = grid1(16, 1)
    n = 1.7
    psi = np.zeros(g.shape, complex)
    psi[:, 1] = np.sqrt(n)
    p = O.Params(c0=1.0, c1=-0.1, q=0.3)
    t, dt = 2.0, 0.13
    out = O.evolve(psi, int(round(t / dt)), dt, p, g)
    tt = dt * int(round(t / dt))
    assert np.allclose(out[:, 1], np.sqrt(n) * np.exp(-1j * p.c0 * n * tt), atol=1e-13)
    assert np.max(np.abs(out[:, [0, 2]])) < 1e-14


def test_uniform_ferromagnet_exact_any_dt():
    """psi_1 = sqrt(n) uniform: exp(-i (q + (c0 + c1) n) t) for any dt."""
    g = grid1(8, 1)
    n = 0.8
    psi = np.zeros(g.shape, complex)
    psi[:, 0] = np.sqrt(n)
    p = O.Params(c0=1.2, c1=-0.4, q=0.7)
    for dt in (0.05, 0.5):
        out = O.evolve(psi, 6, dt, p, g)
        ph = np.exp(-1j * (p.q + (p.c0 + p.c1) * n) * 6 * dt)
        assert np.allclose(out[:, 0], np.sqrt(n) * ph, atol=1e-13)
        assert np.max(np.abs(out[:, 1:])) < 1e-14


def test_uniform_spinor_order2_against_ode():
    """Uniform spinor with q != 0: the split step converges at O(dt^2) to the
    ODE flow of Eq. (2) as printed."""
    p = O.Params(c0=1.0, c1=-0.6, q=0.5)
    g = O.Grid(1, (4,), 1.0, 1)
    v = random_spinors(8, (3,))
    psi0 = np.repeat(v[None, :, None], 4, axis=2)
    t = 1.0

    def f(_, y):
        return (-1j * O.gpe_rhs_printed(y.reshape(psi0.shape), p, g)).ravel()
    ref = scipy.integrate.solve_ivp(f, (0, t), psi0.ravel(), method="DOP853",
                                    rtol=1e-12, atol=1e-14).y[:, -1].reshape(psi0.shape)
    errs = [rel(O.evolve(psi0, m, t / m, p, g), ref) for m in (10, 20, 40)]
    assert 3.5 < errs[0] / errs[1] < 4.5 and 3.5 < errs[1] / errs[2] < 4.5


def test_uniform_spinor_q0_exact():
    """At q = 0 and k = 0 only R acts: exact for any dt."""
    p = O.Params(c0=1.0, c1=-0.6, q=0.0)
    g = O.Grid(1, (4,), 1.0, 1)
    v = random_spinors(9, (3,))
    psi0 = np.repeat(v[None, :, None], 4, axis=2)
    a = O.evolve(psi0, 2, 0.5, p, g)
    b = O.local_flow(psi0, 1.0, p.c0, p.c1)
    assert rel(a, b) < 1e-13


# ---------------------------------------------------------------- K (kinetic)
def free_gaussian(x, t, x0, s0):
    z = 1.0 + 1j * t / s0 ** 2
    return (np.pi * s0 ** 2) ** -0.25 * z ** -0.5 * np.exp(-(x - x0) ** 2 / (2 * s0 ** 2 * z))


@pytest.mark.parametrize("dt", [0.05, 0.5])
def test_free_gaussian_spreading_1d(dt):
    g = O.Grid(1, (256,), 0.5, 1)
    x = np.arange(256) * 0.5
    p = O.Params(c0=0.0, c1=0.0, q=0.0)
    psi = np.zeros(g.shape, complex)
    for c in range(3):
        psi[0, c] = free_gaussian(x, 0.0, 64.0, 3.0)
    nsteps = int(round(5.0 / dt))
    out = O.evolve(psi, nsteps, dt, p, g)
    ref = free_gaussian(x, nsteps * dt, 64.0, 3.0)
    for c in range(3):
        assert np.max(np.abs(out[0, c] - ref)) < 1e-12


def test_free_gaussian_spreading_2d_product():
    g = O.Grid(2, (128, 64), 0.5, 1)
    x = np.arange(128) * 0.5
    y = np.arange(64) * 0.5
    p = O.Params(c0=0.0, c1=0.0, q=0.0)
    psi = np.zeros(g.shape, complex)
    psi[0, 1] = free_gaussian(y, 0, 16.0, 1.5)[:, None] * free_gaussian(x, 0, 32.0, 2.0)[None, :]
    out = O.evolve(psi, 4, 0.25, p, g)
    ref = free_gaussian(y, 1.0, 16.0, 1.5)[:, None] * free_gaussian(x, 1.0, 32.0, 2.0)[None, :]
    assert np.max(np.abs(out[0, 1] - ref)) < 1e-12


def test_plane_wave_and_zeeman_phases():
    """e^{i k0 x} gets exp(-i (k0^2/2 + q m^2) t) (c0 = c1 = 0)."""
    g = O.Grid(3, (8, 8, 16), 0.5, 1)
    p = O.Params(c0=0.0, c1=0.0, q=0.37)
    x = np.arange(8) * 0.5
    z = np.arange(16) * 0.5
    kx, kz = 2 * np.pi * 3 / (8 * 0.5), 2 * np.pi * (-2) / (16 * 0.5)
    wave = np.exp(1j * kx * x)[None, None, :] * np.exp(1j * kz * z)[:, None, None] * np.ones((16, 8, 8))
    psi = np.stack([wave, 2 * wave, -wave])[None]
    t = 0.9
    out = O.evolve(psi, 3, t / 3, p, g)
    for c, m in enumerate((1, 0, -1)):
        ph = np.exp(-1j * (0.5 * (kx ** 2 + kz ** 2) + p.q * m * m) * t)
        assert np.max(np.abs(out[0, c] - psi[0, c] * ph)) < 1e-12


# ---------------------------------------------------------------- full step
def test_time_reversal():
    g = O.Grid(2, (16, 16), 0.5, 2)
    psi = random_field(10, g.shape, noise=0.3)
    fwd = O.evolve(psi, 20, 0.02, P1, g)
    back = O.evolve(fwd, 20, -0.02, P1, g)
    assert rel(back, psi) < 1e-12


def test_strang_second_order():
    g = O.Grid(1, (32,), 0.5, 1)
    # smooth field: low modes only
    x = np.arange(32) * 0.5
    psi = np.zeros(g.shape, complex)
    L = 16.0
    coef = random_spinors(11, (3, 3), 0.3)
    for c in range(3):
        for m in range(3):
            psi[0, c] += coef[c, m] * np.exp(2j * np.pi * (m - 1) * x / L)
    psi[0, 1] += 1.0
    p = O.Params(c0=1.0, c1=-0.5, q=0.3)
    t = 0.8
    ref = O.evolve(psi, 256, t / 256, p, g)
    e = [rel(O.evolve(psi, m, t / m, p, g), ref) for m in (8, 16, 32)]
    assert 3.6 < e[0] / e[1] < 4.4 and 3.6 < e[1] / e[2] < 4.4


def test_norm_and_fz_conserved_energy_second_order():
    g = O.Grid(1, (64,), 0.5, 2)
    psi = random_field(12, g.shape, noise=0.3)
    o0 = O.observables(psi, P1, g)
    drift = []
    for dt, nst in ((0.04, 50), (0.02, 100)):
        cur = psi.copy()
        worst = 0.0
        for _ in range(nst):
            cur = O.strang_step(cur, dt, P1, g)
            o = O.observables(cur, P1, g)
            assert np.allclose(o[:, 0], o0[:, 0], rtol=1e-13)
            assert np.allclose(o[:, 1], o0[:, 1], rtol=0, atol=1e-12 * abs(o0[:, 0]).max())
            worst = max(worst, np.max(np.abs(o[:, 2] - o0[:, 2])))
        drift.append(worst)
    assert 3.0 < drift[0] / drift[1] < 5.0


def spin_rotation(alpha, beta, gamma):
    fx, fy, fz = O.spin_matrices()
    return (scipy.linalg.expm(-1j * alpha * fz) @ scipy.linalg.expm(-1j * beta * fy)
            @ scipy.linalg.expm(-1j * gamma * fz))


def test_spin_rotation_covariance_q0():
    g = O.Grid(1, (32,), 0.5, 1)
    psi = random_field(13, g.shape)
    p = O.Params(c0=1.0, c1=-0.3, q=0.0)
    d = spin_rotation(0.4, 1.1, -0.8)
    rot = lambda f: np.einsum("ij,sj...->si...", d, f)
    a = rot(O.evolve(psi, 5, 0.05, p, g))
    b = O.evolve(rot(psi), 5, 0.05, p, g)
    assert rel(a, b) < 1e-12


def test_z_rotation_covariance_any_q():
    g = O.Grid(1, (32,), 0.5, 1)
    psi = random_field(14, g.shape)
    d = spin_rotation(0.9, 0.0, 0.0)
    rot = lambda f: np.einsum("ij,sj...->si...", d, f)
    a = rot(O.evolve(psi, 5, 0.05, P1, g))
    b = O.evolve(rot(psi), 5, 0.05, P1, g)
    assert rel(a, b) < 1e-12
    # a general rotation does not commute once q != 0
    d2 = spin_rotation(0.0, 1.0, 0.0)
    rot2 = lambda f: np.einsum("ij,sj...->si...", d2, f)
    assert rel(rot2(O.evolve(psi, 5, 0.05, P1, g)), O.evolve(rot2(psi), 5, 0.05, P1, g)) > 1e-4


def test_translation_covariance():
    g = O.Grid(2, (16, 8), 0.5, 1)
    psi = random_field(15, g.shape)
    sh = lambda f: np.roll(f, (3, -5), axis=(-2, -1))
    a = sh(O.evolve(psi, 4, 0.03, P1, g))
    b = O.evolve(sh(psi), 4, 0.03, P1, g)
    assert rel(a, b) < 1e-13


def test_bogoliubov_growth():
    """Polar state + small plane-wave seed in psi_{+1}: the seed grows as
    eps |cosh(G t) - i (A/G) sinh(G t)|, A = k0^2/2 + q + c1 n, G^2 = (c1 n)^2 - A^2."""
    n_sites, dx = 256, 0.5
    g = O.Grid(1, (n_sites,), dx, 1)
    p = O.Params(c0=1.0, c1=-0.1, q=0.09)
    x = np.arange(n_sites) * dx
    j0 = 3
    k0 = 2 * np.pi * j0 / (n_sites * dx)
    eps = 1e-6
    psi = np.zeros(g.shape, complex)
    psi[0, 1] = 1.0
    psi[0, 0] = eps * np.exp(1j * k0 * x)
    t, dt = 10.0, 0.01
    out = O.evolve(psi, int(round(t / dt)), dt, p, g)
    amp = abs(np.fft.fft(out[0, 0])[j0]) / n_sites
    a = 0.5 * k0 ** 2 + p.q + p.c1
    gam = np.sqrt(p.c1 ** 2 - a ** 2)
    expect = eps * abs(np.cosh(gam * t) - 1j * a / gam * np.sinh(gam * t))
    assert abs(amp / expect - 1) < 1e-5
    assert amp / eps > 1.5  # the mode really grew (cosh(1) ~ 1.54)


# ---------------------------------------------------------------- Eq. (5)
def test_eq5_is_exponential_of_offdiagonal_part():
    a = random_spinors(16, (5,))
    b = random_spinors(17, (5,))
    a[0], b[0] = 1e-9, 2e-9j
    theta = -0.7
    m = O.eq5_matrix(a, b, theta)
    for i in range(5):
        ref = scipy.linalg.expm(-1j * theta * O.offdiag_matrix(a[i], b[i]))
        assert np.allclose(m[i], ref, atol=1e-13)


def test_paper_scheme_first_order_same_limit():
    """The literal Lie scheme converges (first order) to the same flow."""
    g = O.Grid(1, (16,), 0.5, 1)
    x = np.arange(16) * 0.5
    psi = np.zeros(g.shape, complex)
    coef = random_spinors(18, (3, 2), 0.3)
    for c in range(3):
        psi[0, c] = coef[c, 0] + coef[c, 1] * np.exp(2j * np.pi * x / 8.0)
    psi[0, 1] += 1.0
    p = O.Params(c0=1.0, c1=-0.4, q=0.2)
    t = 0.5
    ref = O.evolve(psi, 200, t / 200, p, g)
    e = [rel(O.evolve(psi, m, t / m, p, g, step=O.paper_step), ref) for m in (20, 40, 80)]
    r1, r2 = e[0] / e[1], e[1] / e[2]
    assert 1.6 < r1 < 2.6 and 1.6 < r2 < 2.6


# ---------------------------------------------------------------- S(k)
def test_bin_layout_matches_rounding_and_counts():
    for dim, n in ((1, 256), (1, 4096), (2, 256), (2, 512), (2, 1024), (3, 256)):
        g = O.Grid(dim, (n,) * dim, 0.5, 1)
        nb = O.num_bins(g)
        assert nb == {(1, 256): 129, (1, 4096): 2049, (2, 256): 182, (2, 512): 363,
                      (2, 1024): 725, (3, 256): 223}[(dim, n)]
        if dim == 3:
            continue  # index array of 16.7M modes: covered by the small 3D case below
        b = O.bin_index(g)
        jj = sum(O.signed_index(n).reshape([-1 if i == a else 1 for i in range(dim)]) ** 2
                 for a in range(dim))
        assert np.array_equal(b, np.rint(np.sqrt(jj)).astype(np.int64))
        counts = O.bin_counts(g)
        assert counts.sum() == g.sites and np.all(counts > 0)
    g = O.Grid(3, (16, 8, 32), 0.5, 1)
    b = O.bin_index(g)
    zz, yy, xx = np.meshgrid(O.signed_index(32) * 1, O.signed_index(8) * 4, O.signed_index(16) * 2,
                             indexing="ij")
    assert np.array_equal(b, np.rint(np.sqrt(xx ** 2 + yy ** 2 + zz ** 2)).astype(np.int64))


def test_structure_factor_single_plane_wave():
    g = O.Grid(2, (32, 16), 0.5, 1)
    x = np.arange(32) * 0.5
    psi = np.zeros(g.shape, complex)
    psi[0, 1] = 1.0
    eps = 0.01
    jx = 5
    psi[0, 0] = eps * np.exp(-2j * np.pi * jx * x / 16.0)[None, :] * np.ones((16, 1))
    sf = O.structure_factor(psi, g)
    nz = np.nonzero(sf[0] > 1e-20)[0]
    assert list(nz) == [jx]
    # F_perp = sqrt2 eps exp(+i k x): |DFT|^2 / N = 2 eps^2 N at one mode
    count = O.bin_counts(g)[jx]
    assert abs(sf[0, jx] - 2 * eps ** 2 * g.sites / count) < 1e-15


@pytest.mark.parametrize("dim,n,expect", [(1, 256, 8.0), (2, 32, 24.0)])
def test_structure_factor_initial_closed_form(dim, n, expect):
    """At t = 0 with Wigner noise: S(k) = 4 s^2 (n0 + s^2), s^2 = w / dx^d."""
    g = O.Grid(dim, (n,) * dim, 0.5, 64)
    psi = O.init_wigner(1234, g, P1)
    sf = O.structure_factor(psi, g)
    w = O.bin_counts(g)
    grand = np.sum(sf * w[None]) / (g.samples * g.sites)
    se = expect / np.sqrt(g.samples * g.sites)
    assert abs(grand - expect) < 4 * se
    assert expect == 4 * (0.5 / g.cell) * (1 + 0.5 / g.cell)


def test_init_wigner_moments_and_determinism():
    g = O.Grid(2, (32, 32), 0.5, 8)
    p = O.Params(c0=1, c1=-0.1, q=0.09, n0=2.0, wigner_var=0.5)
    psi = O.init_wigner(77, g, p)
    nvals = psi.size // 3
    var = 0.5 / g.cell
    assert abs(psi[:, 1].mean() - np.sqrt(2.0)) < 5 * np.sqrt(var / nvals)
    for c in range(3):
        d = psi[:, c] - (np.sqrt(2.0) if c == 1 else 0.0)
        assert abs(np.mean(np.abs(d) ** 2) - var) < 5 * var / np.sqrt(nvals)
    again = O.init_wigner(77, g, p)
    assert np.array_equal(psi, again)
    other = O.init_wigner(77, g, p, group=1)
    assert not np.allclose(psi, other)
    # samples are independent streams: sample s of an 8-sample draw equals
    # the same counters evaluated on their own
    g1 = O.Grid(2, (32, 32), 0.5, 1)
    assert np.array_equal(O.init_wigner(77, g1, p)[0], psi[0])


def test_observables_uniform_closed_form():
    g = O.Grid(2, (8, 8), 0.5, 1)
    psi = np.zeros(g.shape, complex)
    v = np.array([0.3 + 0.1j, 0.9, -0.2j])
    psi[0] = v[:, None, None]
    p = O.Params(c0=1.1, c1=-0.4, q=0.25)
    o = O.observables(psi, p, g)[0]
    n = np.sum(np.abs(v) ** 2)
    fp = np.sqrt(2) * (np.conj(v[0]) * v[1] + np.conj(v[1]) * v[2])
    fz = abs(v[0]) ** 2 - abs(v[2]) ** 2
    vol = g.sites * g.cell
    assert abs(o[0] - n * vol) < 1e-13
    assert abs(o[1] - fz * vol) < 1e-13
    e = 0.5 * p.c0 * n * n + 0.5 * p.c1 * (abs(fp) ** 2 + fz ** 2) + p.q * (abs(v[0]) ** 2 + abs(v[2]) ** 2)
    assert abs(o[2] - e * vol) < 1e-13


# ------------------------------------------------------------------ real-space spin texture (Fig. 1)
@pytest.mark.parametrize("dim,n", [(1, (64,)), (2, (32, 8)), (3, (16, 4, 2))])
@pytest.mark.parametrize("w", [-3, 0, 1, 5])
def test_spin_texture_of_helix_is_integer_winding(dim, n, w):
    """A helix turning w times along x has F_perp = n0 e^{i phi} (|F_perp| = n0)
    and winds w times on every x-row."""
    g = O.Grid(dim, n, 0.5, 2)
    psi = O.spin_helix(g, w, n0=1.7)
    fp = O.f_perp(psi)
    phi = 2 * np.pi * w * np.arange(n[0]) / n[0]
    assert np.allclose(fp, 1.7 * np.exp(1j * phi), atol=1e-14)
    tex = O.spin_texture(psi, g)
    rows = g.sites // n[0]
    assert np.allclose(tex[:, 0], 1.7, rtol=1e-14)
    assert np.allclose(tex[:, 1], 1.7 ** 2, rtol=1e-14)
    assert np.allclose(tex[:, 2], w * rows, atol=1e-12)


def test_spin_texture_winding_by_hand():
    """Four sites with Larmor phases 0, pi/2, pi, 3pi/2 wind once; the
    reversed order winds -1; a jump by more than pi counts the short way."""
    g = O.Grid(1, (4,), 1.0, 1)
    for phases, expect in (([0, 0.5, 1.0, 1.5], 1), ([0, 1.5, 1.0, 0.5], -1), ([0, 1.2, 1.2, 1.2], 0)):
        fp = np.exp(1j * np.pi * np.array(phases))
        # a transversely polarised spinor per site with this F_perp
        psi = np.empty((1, 3, 4), dtype=np.complex128)
        psi[0, 0] = 0.5 * np.conj(fp)
        psi[0, 1] = 1 / np.sqrt(2)
        psi[0, 2] = 0.5 * fp
        assert abs(O.spin_texture(psi, g)[0, 2] - expect) < 1e-12


def test_spin_texture_invariances_and_parseval():
    """A spin rotation about z moves phi_L uniformly (Q_w and |F_perp| fixed);
    the mean |F_perp|^2 equals the shell sum of S(k) (Parseval)."""
    g = O.Grid(2, (16, 8), 0.5, 3)
    psi = random_field(41, g.shape, noise=0.6)
    tex = O.spin_texture(psi, g)
    alpha = 0.77
    rot = psi * np.exp(-1j * alpha * np.array([1.0, 0.0, -1.0]))[None, :, None, None]
    assert np.allclose(O.spin_texture(rot, g), tex, atol=1e-12)
    bins = O.structure_factor(psi, g)
    assert np.allclose((bins * O.bin_counts(g)).sum(1) / g.sites, tex[:, 1], rtol=1e-12)


def test_init_wigner_sample_subset():
    """Generating selected samples gives exactly those rows of the full set
    (the counter carries the sample index)."""
    g = O.Grid(2, (16, 8), 0.5, 4)
    p = O.Params(1.0, -0.1, 0.09, 1.0, 0.5)
    full = O.init_wigner(77, g, p, group=1)
    part = O.init_wigner(77, g, p, group=1, samples=[3, 0])
    assert np.array_equal(part, full[[3, 0]])
