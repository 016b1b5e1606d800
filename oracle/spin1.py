"""FP64 oracle of the spin-1 split-step method (arXiv:2310.03636, Sec. 2.2).

TEST INFRASTRUCTURE ONLY (see the package docstring).  Plain, slow and
direct: every step is written out in the order the method states it, with
library primitives (``numpy.linalg.eigh``, the own FFT of ``oracle.fft``)
as building blocks and no blocking, fusion or merging of sub-steps.

Conventions (readings of the paper where it is silent or ambiguous):
  * hbar = m = 1 (the kinetic phase of Eq. (3) is exp(-i dt |k|^2 / 2)).
  * Components are ordered (psi_{+1}, psi_0, psi_{-1}) as in Eq. (2);
    array axis 1 holds them, index c = 0, 1, 2 <-> m = +1, 0, -1.
  * Field arrays are [S, 3, (Nz), (Ny), Nx] with x fastest.
  * Forward DFT with exp(-i k x), unnormalised; k = 2 pi j' / (N dx),
    j' the signed index.
  * Eq. (2) equals i d_t psi = [-Lap/2 + q f_z^2 + c0 n + c1 F.f] psi with the
    spin-1 matrices f and F_a = psi^dag f_a psi; the tests pin this against
    Eq. (2) as printed.
  * The local (c0, c1) part conserves n and F at every site, so its exact
    flow over tau is exp(-i tau (c0 n + c1 F.f)); the oracle takes that
    exponential by Hermitian eigendecomposition.
  * Hot-path step (symmetric split of the operator in Eq. (2)):
        psi <- R(dt/2) psi;  psi_m <- IFFT[exp(-i(|k|^2/2 + q m^2) dt) FFT psi_m];
        psi <- R(dt/2) psi.
  * ``paper_step`` is the literal Lie-order scheme of Eqs. (3)-(5).
  * Optional trap potential V(x) (the V_m of Eq. (4), a diagonal term of the
    operator in Eq. (2)), taken the same for the three components: an array
    of the spatial shape, or None.  Being a multiple of the identity at each
    site, it joins the exact local flow: R(tau) = exp(-i tau (V + c0 n + c1 F.f)).
"""
from dataclasses import dataclass
import numpy as np

from .fft import fft_axis, fftn_last
from .philox import gaussian_pair

SQRT2 = np.sqrt(2.0)
M_VALUES = np.array([1.0, 0.0, -1.0])  # magnetic quantum numbers of axis 1


@dataclass(frozen=True)
class Grid:
    """Periodic lattice: ``n`` = (Nx[, Ny[, Nz]]), spacing ``dx``, ``samples`` runs."""

    dim: int
    n: tuple
    dx: float
    samples: int

    @property
    def spatial(self):
        return tuple(reversed(tuple(self.n[: self.dim])))

    @property
    def shape(self):
        return (self.samples, 3) + self.spatial

    @property
    def sites(self):
        return int(np.prod(self.n[: self.dim]))

    @property
    def cell(self):
        return self.dx ** self.dim


@dataclass(frozen=True)
class Params:
    """Couplings of Eq. (2) in units hbar = m = 1, plus the initial state."""

    c0: float
    c1: float
    q: float
    n0: float = 1.0
    wigner_var: float = 0.5


# --------------------------------------------------------------------------
# spin-1 algebra (Eq. (2) and the spin vector F of Sec. 2.1)
# --------------------------------------------------------------------------
def spin_matrices():
    """Spin-1 matrices f_x, f_y, f_z in the basis (m=+1, 0, -1)."""
    s = 1.0 / SQRT2
    fx = np.array([[0, s, 0], [s, 0, s], [0, s, 0]], dtype=np.complex128)
    fy = np.array([[0, -1j * s, 0], [1j * s, 0, -1j * s], [0, 1j * s, 0]], dtype=np.complex128)
    fz = np.diag([1.0, 0.0, -1.0]).astype(np.complex128)
    return fx, fy, fz


def density(psi):
    """rho = sum_m |psi_m|^2 (Sec. 2.2, after Eq. (2))."""
    return np.sum(np.abs(psi) ** 2, axis=1)


def spin_vector(psi):
    """(F_x, F_y, F_z) with F_a = psi^dag f_a psi, each of shape [S, spatial]."""
    out = []
    for f in spin_matrices():
        fpsi = np.einsum("ij,sj...->si...", f, psi)
        out.append(np.real(np.sum(np.conj(psi) * fpsi, axis=1)))
    return out


def f_perp(psi):
    """Transverse spin F_perp = F_x + i F_y (Sec. 2.1, the paragraph after Fig. 1)."""
    fx, fy, _ = spin_vector(psi)
    return fx + 1j * fy


def spin_texture(psi, grid):
    """Real-space transverse-spin diagnostics per sample, array [S, 3]:
    (mean |F_perp|, mean |F_perp|^2, Q_w), means over the lattice sites.

    F_perp = |F_perp| exp(i phi_L) (Fig. 1 caption, Sec. 2.1).  Q_w is the
    winding of the Larmor phase along x, the lattice form of the integral of
    d phi_L / dx over the periodic line in units of 2 pi: the phase steps
    phi_L(x_{j+1}) - phi_L(x_j), each taken in [-pi, pi), summed around every
    x-row and over the rows (in 1D, the paper's Q_w).  phi_L = 0 where
    F_perp = 0.
    """
    fp = f_perp(psi)
    axes = tuple(range(1, 1 + grid.dim))
    mag = np.abs(fp)
    phi = np.angle(fp)
    step = np.roll(phi, -1, axis=-1) - phi
    step = step - 2.0 * np.pi * np.floor((step + np.pi) / (2.0 * np.pi))
    out = np.empty((grid.samples, 3))
    out[:, 0] = np.mean(mag, axis=axes)
    out[:, 1] = np.mean(mag ** 2, axis=axes)
    out[:, 2] = np.sum(step, axis=axes) / (2.0 * np.pi)
    return out


def spin_helix(grid, winding, n0=1.0):
    """Transversely polarised state whose spin turns `winding` times along x:
    the spin-1 state of spin n0 along (cos phi, sin phi, 0) with
    phi = 2 pi winding x / L, i.e. psi = sqrt(n0) (e^{-i phi}/2, 1/sqrt2, e^{i phi}/2);
    F_perp = n0 e^{i phi}.  Array [S, 3, spatial]."""
    nx = grid.n[0]
    phi = 2.0 * np.pi * winding * np.arange(nx) / nx
    shape = grid.spatial
    phi = np.broadcast_to(phi, shape)
    psi = np.empty((grid.samples, 3) + shape, dtype=np.complex128)
    psi[:, 0] = 0.5 * np.exp(-1j * phi)
    psi[:, 1] = 1.0 / np.sqrt(2.0)
    psi[:, 2] = 0.5 * np.exp(1j * phi)
    return np.sqrt(n0) * psi


# --------------------------------------------------------------------------
# lattice and momentum grid (Eq. (3), Laplacian of Sec. 2.2)
# --------------------------------------------------------------------------
def signed_index(n):
    j = np.arange(n)
    return np.where(j < n // 2, j, j - n)


def wavenumbers(grid):
    """Per-axis k arrays shaped to broadcast over the spatial axes (x last)."""
    ks = []
    for a in range(grid.dim):
        n = grid.n[a]
        k = 2.0 * np.pi * signed_index(n) / (n * grid.dx)
        shape = [1] * grid.dim
        shape[grid.dim - 1 - a] = n
        ks.append(k.reshape(shape))
    return ks


def k_squared(grid):
    return sum(k ** 2 for k in wavenumbers(grid))


# --------------------------------------------------------------------------
# initial state: polar condensate plus Wigner noise (Sec. 2.1 and Sec. 2.2)
# --------------------------------------------------------------------------
def init_wigner(seed, grid, p, group=0, samples=None):
    """psi_m(x_j) = sqrt(n0) delta_{m0} + delta psi_{m,j}.

    The paper starts each run from a weakly fluctuating state with vanishing
    mean spin (Sec. 2.1) and averages over many such runs to include quantum
    fluctuations (Sec. 2.2).  delta psi is complex Gaussian with
    <|delta psi|^2> = w / dx^d per site and component (half a quantum per mode
    for w = 1/2).  Each number comes from one Philox4x64-10 block with
    counter (site, component, sample, group) and key (seed, 0); words 0 and 1
    feed Box-Muller.  samples: optional list of sample indices to generate
    (rows of the result in that order); all samples by default.
    """
    spatial = grid.spatial
    nsite = grid.sites
    site = np.arange(nsite, dtype=np.uint64).reshape(spatial)
    which = list(range(grid.samples)) if samples is None else list(samples)
    psi = np.empty((len(which), 3) + spatial, dtype=np.complex128)
    amp = np.sqrt(p.wigner_var / (2.0 * grid.cell))
    for i, s in enumerate(which):
        for c in range(3):
            ctr = (site, np.uint64(c), np.uint64(s), np.uint64(group))
            g_re, g_im = gaussian_pair(ctr, (np.uint64(seed), np.uint64(0)))
            psi[i, c] = amp * (g_re + 1j * g_im)
        psi[i, 1] += np.sqrt(p.n0)
    return psi


# --------------------------------------------------------------------------
# sub-steps
# --------------------------------------------------------------------------
def local_hamiltonian(psi, c0, c1, V=None):
    """Per-site 3x3 matrix V + c0 n + c1 F.f; shape [S, spatial..., 3, 3]."""
    fmats = spin_matrices()
    n = density(psi)
    fvec = spin_vector(psi)
    diag = c0 * n if V is None else c0 * n + np.asarray(V, dtype=np.float64)
    h = diag[..., None, None] * np.eye(3)
    for fa, f in zip(fvec, fmats):
        h = h + c1 * fa[..., None, None] * f
    return h


def local_flow(psi, tau, c0, c1, chunk=1 << 18, V=None):
    """Exact flow R(tau) of i d_t psi = (V + c0 n + c1 F.f) psi at every site.

    n and F are constants of this local motion, so the flow is the matrix
    exponential exp(-i tau H) of the site matrix H; it is taken from the
    eigendecomposition H = V diag(w) V^dag.  This covers the diagonal
    (Eq. (4), c0 and c1 parts) and off-diagonal (Eq. (5)) interaction
    sub-steps in one exact update.
    """
    psi = np.asarray(psi, dtype=np.complex128)
    h = local_hamiltonian(psi, c0, c1, V)
    sv = np.moveaxis(psi, 1, -1)  # [S, spatial..., 3]
    flat_h = h.reshape(-1, 3, 3)
    flat_v = sv.reshape(-1, 3)
    out = np.empty_like(flat_v)
    for lo in range(0, flat_v.shape[0], chunk):
        hi = min(lo + chunk, flat_v.shape[0])
        w, v = np.linalg.eigh(flat_h[lo:hi])
        coeff = np.einsum("nji,nj->ni", np.conj(v), flat_v[lo:hi])
        coeff = coeff * np.exp(-1j * tau * w)
        out[lo:hi] = np.einsum("nij,nj->ni", v, coeff)
    return np.moveaxis(out.reshape(sv.shape), -1, 1)


def kinetic_zeeman(psi, dt, q, grid):
    """Kinetic sub-step Eq. (3) together with the quadratic Zeeman phase.

    psi_m <- IFFT[exp(-i (|k|^2/2 + q m^2) dt) FFT psi_m].  The q term is the
    uniform diagonal "+q" of Eq. (2) acting on m = +1 and m = -1 only (the
    -q/c1 entry cancels it for m = 0); it commutes with the kinetic operator.
    """
    k2 = k_squared(grid)
    out = np.empty_like(psi, dtype=np.complex128)
    for c in range(3):
        m = M_VALUES[c]
        phase = np.exp(-1j * (0.5 * k2 + q * m * m) * dt)
        spec = fftn_last(psi[:, c], grid.dim)
        out[:, c] = fftn_last(spec * phase, grid.dim, inverse=True)
    return out


def strang_step(psi, dt, p, grid, V=None):
    """One step of the symmetric split R(dt/2) [K Q](dt) R(dt/2)."""
    psi = local_flow(psi, 0.5 * dt, p.c0, p.c1, V=V)
    psi = kinetic_zeeman(psi, dt, p.q, grid)
    psi = local_flow(psi, 0.5 * dt, p.c0, p.c1, V=V)
    return psi


def evolve(psi, nsteps, dt, p, grid, step=None, V=None):
    step = strang_step if step is None else step
    for _ in range(nsteps):
        psi = step(psi, dt, p, grid) if V is None else step(psi, dt, p, grid, V=V)
    return psi


# --------------------------------------------------------------------------
# the paper's literal scheme, Eqs. (3)-(5), Lie order
# --------------------------------------------------------------------------
def eq5_matrix(a, b, theta):
    """The 3x3 matrix of Eq. (5) for couplings a, b and angle theta = c1 dt.

    Entries (0,2) and (2,0) are read as a b (cos - 1) and a* b* (cos - 1).
    For lambda -> 0 the limit (identity) is taken via sinc forms.
    """
    a = np.asarray(a, dtype=np.complex128)
    b = np.asarray(b, dtype=np.complex128)
    lam2 = np.abs(a) ** 2 + np.abs(b) ** 2
    lam = np.sqrt(lam2)
    x = lam * theta
    cs = np.cos(x)
    # sin(x)/lam and (cos(x) - 1)/lam^2 written without division by lam
    s_over = theta * np.sinc(x / np.pi)
    cm1_over = -0.5 * theta ** 2 * np.sinc(x / (2.0 * np.pi)) ** 2
    # (|a|^2 cos + |b|^2)/lam^2 = 1 + |a|^2 (cos - 1)/lam^2
    m = np.empty(a.shape + (3, 3), dtype=np.complex128)
    m[..., 0, 0] = 1.0 + np.abs(a) ** 2 * cm1_over
    m[..., 0, 1] = -1j * a * s_over
    m[..., 0, 2] = a * b * cm1_over
    m[..., 1, 0] = -1j * np.conj(a) * s_over
    m[..., 1, 1] = cs
    m[..., 1, 2] = -1j * b * s_over
    m[..., 2, 0] = np.conj(a) * np.conj(b) * cm1_over
    m[..., 2, 1] = -1j * np.conj(b) * s_over
    m[..., 2, 2] = 1.0 + np.abs(b) ** 2 * cm1_over
    return m


def offdiag_matrix(a, b):
    """S(a, b): the off-diagonal part of the matrix in Eq. (2)."""
    a = np.asarray(a, dtype=np.complex128)
    s = np.zeros(a.shape + (3, 3), dtype=np.complex128)
    s[..., 0, 1] = a
    s[..., 1, 0] = np.conj(a)
    s[..., 1, 2] = b
    s[..., 2, 1] = np.conj(b)
    return s


def paper_step(psi, dt, p, grid, V=None):
    """One step of the literal Lie-order scheme of Eqs. (3)-(5): the kinetic
    phase of Eq. (3) (``paper_kinetic``), then the diagonal phases of Eq. (4)
    with the densities of the field they act on (``paper_diagonal``), then the
    off-diagonal mixing of Eq. (5) with predictor-averaged couplings
    (``paper_offdiagonal``)."""
    psi1 = paper_kinetic(psi, dt, grid)
    psi2 = paper_diagonal(psi1, dt, p, V)
    return paper_offdiagonal(psi2, dt, p.c1)


def paper_kinetic(psi, dt, grid):
    """Eq. (3): every component goes to IFFT[exp(-i dt |k|^2 / 2) FFT psi_m].
    No q here: the paper's scheme keeps q in the diagonal phases of Eq. (4)."""
    k2 = k_squared(grid)
    out = np.empty_like(psi, dtype=np.complex128)
    for c in range(3):
        spec = fftn_last(psi[:, c], grid.dim)
        out[:, c] = fftn_last(spec * np.exp(-1j * 0.5 * k2 * dt), grid.dim, inverse=True)
    return out


def paper_diagonal_rates(psi, p, V=None):
    """The rates f_m of Eq. (4), evaluated with the densities of ``psi``:
    the diagonal of the bracket of Eq. (2) without the kinetic term,
        f_{+1} = q + (c0 + c1) rho - 2 c1 |psi_{-1}|^2,
        f_0    =     (c0 + c1) rho -   c1 |psi_0|^2,
        f_{-1} = q + (c0 + c1) rho - 2 c1 |psi_{+1}|^2,
    plus V_m(x_j) (the same for every m).  Real array of the field's shape."""
    c0, c1, q = p.c0, p.c1, p.q
    dens = np.abs(psi) ** 2
    rho = np.sum(dens, axis=1)
    f_p = q + (c0 + c1) * rho - 2.0 * c1 * dens[:, 2]
    f_0 = (c0 + c1) * rho - c1 * dens[:, 1]
    f_m = q + (c0 + c1) * rho - 2.0 * c1 * dens[:, 0]
    diag = np.stack([f_p, f_0, f_m], axis=1)
    if V is not None:  # V_m(x_j) of Eq. (4), the same for every m
        diag = diag + np.asarray(V, dtype=np.float64)[None, None]
    return diag


def paper_diagonal(psi, dt, p, V=None):
    """Eq. (4): psi_m -> exp(-i f_m dt) psi_m with f_m = paper_diagonal_rates(psi)
    (the densities of the field being multiplied)."""
    return psi * np.exp(-1j * paper_diagonal_rates(psi, p, V) * dt)


def paper_couplings(psi):
    """Couplings of the off-diagonal part S(a, b) of Eq. (2)'s matrix at every
    site (Eq. (5) and the definitions below it): a = psi_{-1}^* psi_0 and
    b = psi_0^* psi_{+1}."""
    return np.conj(psi[:, 2]) * psi[:, 1], np.conj(psi[:, 1]) * psi[:, 0]


def paper_offdiagonal(psi, dt, c1):
    """Eq. (5): psi -> M(a, b) psi, with M the matrix of Eq. (5) at angle
    theta = c1 dt and couplings averaged over the field and a one-step
    predictor: a0, b0 = paper_couplings(psi), tpsi = psi - i c1 dt S(a0, b0) psi,
    a = [a0 + tpsi_{-1}^* tpsi_0] / 2, b = [b0 + tpsi_0^* tpsi_{+1}] / 2."""
    a0, b0 = paper_couplings(psi)
    sv = np.moveaxis(psi, 1, -1)
    pred = sv - 1j * c1 * dt * np.einsum("...ij,...j->...i", offdiag_matrix(a0, b0), sv)
    a = 0.5 * (a0 + np.conj(pred[..., 2]) * pred[..., 1])
    b = 0.5 * (b0 + np.conj(pred[..., 1]) * pred[..., 0])
    out = np.einsum("...ij,...j->...i", eq5_matrix(a, b, c1 * dt), sv)
    return np.moveaxis(out, -1, 1)


# --------------------------------------------------------------------------
# observables (energy functional whose Wirtinger derivative is Eq. (2))
# --------------------------------------------------------------------------
def observables(psi, p, grid, V=None):
    """Per sample (N, F_z, E) in FP64, array [S, 3].

    N = dx^d sum n;  F_z = dx^d sum (|psi_1|^2 - |psi_-1|^2);
    E = dx^d sum [V n + c0 n^2/2 + c1 |F|^2/2 + q (|psi_1|^2 + |psi_-1|^2)]
        + (dx^d / N_sites) sum_m sum_k |k|^2/2 |FFT psi_m (k)|^2.
    """
    sp_axes = tuple(range(1, 1 + grid.dim))
    n = density(psi)
    fx, fy, fz = spin_vector(psi)
    d1 = np.abs(psi[:, 0]) ** 2
    dm = np.abs(psi[:, 2]) ** 2
    e_loc = 0.5 * p.c0 * n ** 2 + 0.5 * p.c1 * (fx ** 2 + fy ** 2 + fz ** 2) + p.q * (d1 + dm)
    if V is not None:
        e_loc = e_loc + np.asarray(V, dtype=np.float64)[None] * n
    k2 = k_squared(grid)
    e_kin = np.zeros(grid.samples)
    for c in range(3):
        spec = fftn_last(psi[:, c], grid.dim)
        e_kin += np.sum(0.5 * k2 * np.abs(spec) ** 2, axis=sp_axes) / grid.sites
    out = np.empty((grid.samples, 3))
    out[:, 0] = grid.cell * np.sum(n, axis=sp_axes)
    out[:, 1] = grid.cell * np.sum(d1 - dm, axis=sp_axes)
    out[:, 2] = grid.cell * (np.sum(e_loc, axis=sp_axes) + e_kin)
    return out


# --------------------------------------------------------------------------
# structure factor S(t, k) = < F_perp(k)^* F_perp(k) > (Sec. 2.1, Fig. 2)
# --------------------------------------------------------------------------
def bin_index(grid):
    """Radial shell of every mode, integer-exact.

    With J = |j'|^2 in units of the smallest grid step (j'_a scaled by
    Nmax / N_a), the shell is the integer b >= 0 with 4J < (2b+1)^2 and, for
    b >= 1, (2b-1)^2 <= 4J: |j'| rounded to the nearest integer (no ties, since
    4J is even and (2b+-1)^2 odd).
    """
    nmax = max(grid.n[: grid.dim])
    jj = np.zeros(grid.spatial, dtype=np.int64)
    for a in range(grid.dim):
        n = grid.n[a]
        j = signed_index(n).astype(np.int64) * (nmax // n)
        shape = [1] * grid.dim
        shape[grid.dim - 1 - a] = n
        jj = jj + (j ** 2).reshape(shape)
    b0 = np.floor(np.sqrt(jj.astype(np.float64))).astype(np.int64)
    out = np.full(jj.shape, -1, dtype=np.int64)
    for cand in (b0 - 1, b0, b0 + 1):
        lower = np.where(cand >= 1, (2 * cand - 1) ** 2, 0)
        ok = (lower <= 4 * jj) & (4 * jj < (2 * cand + 1) ** 2) & (cand >= 0)
        if np.any(ok & (out >= 0)):
            raise AssertionError("mode falls in two shells")
        out = np.where(ok, cand, out)
    if np.any(out < 0):
        raise AssertionError("mode falls in no shell")
    return out


def num_bins(grid):
    return int(bin_index(grid).max()) + 1


def bin_counts(grid):
    return np.bincount(bin_index(grid).ravel(), minlength=num_bins(grid))


def bin_k(grid):
    """|k| at the centre of each shell: b * 2 pi / (Nmax dx)."""
    nmax = max(grid.n[: grid.dim])
    return np.arange(num_bins(grid)) * 2.0 * np.pi / (nmax * grid.dx)


def structure_factor(psi, grid):
    """Per-sample shell means of |DFT F_perp|^2 / N_sites, array [S, n_bins]."""
    fp = f_perp(psi)
    spec = fftn_last(fp, grid.dim)
    power = np.abs(spec) ** 2 / grid.sites
    b = bin_index(grid).ravel()
    nb = int(b.max()) + 1
    counts = np.bincount(b, minlength=nb).astype(np.float64)
    out = np.zeros((grid.samples, nb))
    filled = counts > 0  # a shell without modes reports 0
    for s in range(grid.samples):
        sums = np.bincount(b, weights=power[s].ravel(), minlength=nb)
        out[s, filled] = sums[filled] / counts[filled]
    return out


def sample_mean_se(bins):
    """Mean over samples and its standard error std / sqrt(S)."""
    s = bins.shape[0]
    mean = bins.mean(axis=0)
    se = bins.std(axis=0, ddof=1) / np.sqrt(s) if s > 1 else np.zeros_like(mean)
    return mean, se


# --------------------------------------------------------------------------
# right-hand side of Eq. (2) exactly as printed (for pinning only)
# --------------------------------------------------------------------------
def gpe_rhs_printed(psi, p, grid, V=None):
    """i d_t psi from Eq. (2) with the printed matrix, hbar = m = 1, plus the
    diagonal potential V (the V_m of Eq. (4)) when given.

    The Laplacian is applied spectrally with ``fft_axis``.
    """
    c0, c1, q = p.c0, p.c1, p.q
    p1, p0, pm = psi[:, 0], psi[:, 1], psi[:, 2]
    rho = density(psi)
    k2 = k_squared(grid)
    lap = np.empty_like(psi, dtype=np.complex128)
    for c in range(3):
        lap[:, c] = fftn_last(0.5 * k2 * fftn_last(psi[:, c], grid.dim), grid.dim, inverse=True)
    diag = q + (c0 + c1) * rho
    if V is not None:
        diag = diag + np.asarray(V, dtype=np.float64)[None]
    out = np.empty_like(psi, dtype=np.complex128)
    out[:, 0] = lap[:, 0] + diag * p1 + c1 * (-2 * np.abs(pm) ** 2 * p1 + np.conj(pm) * p0 * p0)
    # the printed entry c1 (-|psi_0|^2 - q/c1) is expanded so that c1 = 0 is allowed
    out[:, 1] = (lap[:, 1] + diag * p0
                 + c1 * (pm * np.conj(p0) * p1 - np.abs(p0) ** 2 * p0 + np.conj(p0) * p1 * pm) - q * p0)
    out[:, 2] = lap[:, 2] + diag * pm + c1 * (p0 * np.conj(p1) * p0 - 2 * np.abs(p1) ** 2 * pm)
    return out


def fft_field(psi, grid):
    """d-dimensional forward DFT of every component (own FFT)."""
    return fftn_last(psi, grid.dim)


__all__ = [
    "Grid", "Params", "spin_matrices", "density", "spin_vector", "f_perp",
    "wavenumbers", "k_squared", "init_wigner", "local_hamiltonian", "local_flow",
    "kinetic_zeeman", "strang_step", "evolve", "eq5_matrix", "offdiag_matrix",
    "paper_step", "paper_kinetic", "paper_diagonal_rates", "paper_diagonal", "paper_couplings",
    "paper_offdiagonal", "observables", "bin_index", "num_bins", "bin_counts", "bin_k",
    "structure_factor", "sample_mean_se", "gpe_rhs_printed", "fft_field", "fft_axis",
]
