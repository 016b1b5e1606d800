"""GPU parity of the trap potential V(x) (the V_m of Eq. (4), the same for the
three components) against the FP64 oracle, through the C ABI."""
import numpy as np
import pytest

from oracle import spin1 as O
from tests.inputs import random_field

pytestmark = pytest.mark.gpu

P1 = dict(c0=1.0, c1=-0.1, q=0.09, n0=1.0, wigner_var=0.5)


def oparams(p):
    return O.Params(p["c0"], p["c1"], p["q"], p["n0"], p["wigner_var"])


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def trap(og, seed, edge=4.0, rough=0.5):
    """A harmonic trap about the box centre rising to `edge` at the box faces,
    plus seeded site-to-site roughness, so that every site carries its own
    value (a wrong site index shows)."""
    axes = [(np.arange(og.n[a]) - 0.5 * og.n[a]) / (0.5 * og.n[a]) for a in range(og.dim)]
    mesh = np.meshgrid(*reversed(axes), indexing="ij")
    v = edge * sum(m ** 2 for m in mesh)
    return v + rough * np.random.default_rng(seed).uniform(-1.0, 1.0, size=og.spatial)


def ogrid(g):
    return O.Grid(g[0], g[1], g[2], g[3])


GRIDS = [(1, (256,), 0.5, 3), (1, (4096,), 0.5, 2), (2, (64, 32), 0.5, 2), (2, (2048, 16), 0.5, 1),
         (3, (16, 8, 16), 0.5, 2)]


@pytest.mark.parametrize("grid", GRIDS)
def test_trap_steps_match_oracle(lib, grid):
    """Strang steps with a trap (streaming x-pass for Nx <= 1024, the other
    x-pass kernel above; 1D without the multi-step kernel) against the oracle."""
    og = ogrid(grid)
    V = trap(og, 3)
    psi0 = random_field(31, og.shape, noise=0.5)
    n, dt = 30, 0.01
    ref = O.evolve(psi0, n, dt, oparams(P1), og, V=V)
    for dtype, tol in (("c128", 1e-11), ("c64", 2e-5)):
        sim = lib.Sim([grid], P1, dtype=dtype)
        sim.set_fields([psi0])
        sim.set_potential(0, V)
        sim.step(n - 10, dt)
        sim.step(10, dt)
        assert rel(sim.fields()[0], ref) < tol, dtype
        sim.close()


@pytest.mark.parametrize("grid", [(1, (128,), 0.5, 2), (2, (32, 64), 0.5, 2), (3, (16, 16, 8), 0.5, 1)])
def test_trap_paper_scheme_matches_oracle(lib, grid):
    og = ogrid(grid)
    V = trap(og, 5)
    psi0 = random_field(33, og.shape, noise=0.5)
    ref = O.evolve(psi0, 12, 0.01, oparams(P1), og, step=O.paper_step, V=V)
    sim = lib.Sim([grid], P1, dtype="c128")
    sim.set_option(lib.OPT_SCHEME, lib.SCHEME_PAPER)
    sim.set_fields([psi0])
    sim.set_potential(0, V)
    sim.step(12, 0.01)
    assert rel(sim.fields()[0], ref) < 1e-11


@pytest.mark.parametrize("grid", [(1, (256,), 0.5, 3), (2, (64, 32), 0.5, 2), (3, (16, 8, 16), 0.5, 2)])
def test_trap_energy_and_step_log_match_oracle(lib, grid):
    """The energy gains dx^d sum V n, in spin1_observables and in the per-step log."""
    og = ogrid(grid)
    V = trap(og, 7)
    p, dt, n = oparams(P1), 0.02, 5
    psi0 = random_field(35, og.shape, noise=0.5)
    ref_obs = O.observables(psi0, p, og, V=V)
    ref_log, cur = [], psi0
    for _ in range(n):
        ref_log.append(O.observables(O.local_flow(cur, 0.5 * dt, p.c0, p.c1, V=V), p, og, V=V))
        cur = O.strang_step(cur, dt, p, og, V=V)
    ref_log = np.array(ref_log)
    for dtype, tol in (("c128", 1e-12), ("c64", 2e-6)):
        sim = lib.Sim([grid], P1, dtype=dtype)
        sim.set_fields([psi0])
        sim.set_potential(0, V)
        got = sim.observables()
        assert np.allclose(got, ref_obs, rtol=tol, atol=tol * np.abs(ref_obs).max()), dtype
        log = sim.step_observed(n, dt)
        assert np.allclose(log, ref_log, rtol=tol, atol=tol * np.abs(ref_log).max()), dtype
        assert rel(sim.fields()[0], cur) < (1e-12 if dtype == "c128" else 1e-5), dtype
        sim.close()


def test_trap_in_uneven_batch_with_grouped_and_multi_step_groups(lib):
    """Groups with a trap leave the grouped x-pass and the 1D multi-step
    kernel; the other groups keep them; every group matches the oracle."""
    grids = [(1, (256,), 0.5, 2), (1, (512,), 0.5, 2), (2, (32, 32), 0.5, 2), (2, (64, 16), 0.5, 1),
             (2, (16, 64), 0.5, 2)]
    pots = {0: trap(ogrid(grids[0]), 11), 2: trap(ogrid(grids[2]), 12)}
    sim = lib.Sim(grids, P1, dtype="c128")
    sim.init_wigner(17)
    for g, v in pots.items():
        sim.set_potential(g, v)
    f0 = sim.fields()
    sim.step(9, 0.02)
    f = sim.fields()
    for gi, g in enumerate(grids):
        ref = O.evolve(f0[gi], 9, 0.02, oparams(P1), ogrid(g), V=pots.get(gi))
        assert rel(f[gi], ref) < 1e-11, gi


def test_trap_set_remove_graphs_and_rebind(lib):
    """Setting or removing the potential retires captured graphs; init_wigner
    keeps the potential of the Python object; removal restores plain steps."""
    grid = (2, (32, 32), 0.5, 2)
    og = ogrid(grid)
    V = trap(og, 13)
    p = oparams(P1)
    sim = lib.Sim([grid], P1, dtype="c128")
    sim.init_wigner(19)
    f0 = sim.fields()[0]
    sim.step(5, 0.02)  # captured without the potential
    sim.set_potential(0, V)
    sim.step(5, 0.02)  # same (n, dt): must not replay the old graph
    ref = O.evolve(O.evolve(f0, 5, 0.02, p, og), 5, 0.02, p, og, V=V)
    assert rel(sim.fields()[0], ref) < 1e-11
    sim.set_potential(0, None)
    sim.step(5, 0.02)
    ref = O.evolve(ref, 5, 0.02, p, og)
    assert rel(sim.fields()[0], ref) < 1e-11
    sim.set_potential(0, V)
    sim.init_wigner(19)  # rebinds; the object sets the potential again
    sim.step(5, 0.02)
    assert rel(sim.fields()[0], O.evolve(f0, 5, 0.02, p, og, V=V)) < 1e-11


def test_deep_trap_single_precision_phase(lib):
    """A trap whose phase per step runs to hundreds of radians: the angle is
    reduced in FP64 before single precision takes it, so the complex64 local
    update stays at its usual accuracy."""
    grid = (1, (1024,), 0.5, 2)
    og = ogrid(grid)
    V = trap(og, 29, edge=3.0e4)
    psi0 = random_field(39, og.shape, noise=0.5)
    sim = lib.Sim([grid], P1, dtype="c64")
    sim.set_fields([psi0])
    sim.set_potential(0, V)
    sim.local_update(0.01)
    ref = O.local_flow(psi0, 0.01, P1["c0"], P1["c1"], V=V)
    assert rel(sim.fields()[0], ref) < 1e-6


def test_trap_local_update_and_errors(lib):
    grid = (2, (32, 16), 0.5, 2)
    og = ogrid(grid)
    V = trap(og, 23)
    psi0 = random_field(37, og.shape, noise=0.5)
    sim = lib.Sim([grid], P1, dtype="c128")
    sim.set_fields([psi0])
    sim.set_potential(0, V)
    sim.local_update(0.3)
    ref = O.local_flow(psi0, 0.3, P1["c0"], P1["c1"], V=V)
    assert rel(sim.fields()[0], ref) < 1e-13
    import torch
    buf = torch.zeros(og.sites + 1, dtype=torch.float64, device=sim.device)
    with pytest.raises(lib.Spin1Error):
        lib.set_potential(sim.ctx, 1, buf.data_ptr())  # no group 1
    with pytest.raises(lib.Spin1Error):
        lib.set_potential(sim.ctx, 0, buf.data_ptr() + 4)  # misaligned
    # reverse mode takes no potential
    with pytest.raises(lib.Spin1Error) as err:
        sim.forward_ckpt(4, 0.02, 2)
    assert err.value.code == lib.EUNSUPPORTED
    sim.close()
    fresh = lib.create(lib.C128)
    with pytest.raises(lib.Spin1Error) as err:
        lib.set_potential(fresh, 0, buf.data_ptr())  # not bound
    assert err.value.code == lib.ESTATE
    lib.destroy(fresh)
