"""GPU parity: the HIP path through the C ABI against the FP64 oracle.

Tolerances (relative L2 over all samples, components and sites, from
identical initial fields): complex128 <= 1e-10 after 100 steps; complex64
<= 1e-4 after 100 steps, and within FLOOR_FACTOR of the single-precision
floor of the dynamics.  The floor is the oracle run in FP64 with its state
rounded to complex64 after every step: no single-precision code can beat it,
and chaotic configurations (the 3D one amplifies a 1e-8 change of the
initial state ~7000-fold in 100 steps) put it above 1e-4, so the 3D case
misses 1e-4 (an expected failure).  Single steps and transforms are held
tighter.
"""
import numpy as np
import pytest

from oracle import spin1 as O
from tests.inputs import random_field

pytestmark = pytest.mark.gpu

P1 = dict(c0=1.0, c1=-0.1, q=0.09, n0=1.0, wigner_var=0.5)
P3 = dict(c0=1.0, c1=-0.05, q=0.025, n0=1.0, wigner_var=0.5)


def oparams(p):
    return O.Params(p["c0"], p["c1"], p["q"], p["n0"], p["wigner_var"])


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def run_gpu(lib, grid, p, dtype, psi0=None, seed=None, nsteps=0, dt=0.01):
    sim = lib.Sim([grid], p, dtype=dtype)
    if seed is not None:
        sim.init_wigner(seed)
    else:
        sim.set_fields([psi0])
    if nsteps:
        sim.step(nsteps, dt)
    return sim


# ------------------------------------------------------------------ init
@pytest.mark.parametrize("grid", [(1, (256,), 0.5, 4), (2, (32, 16), 0.5, 3), (3, (16, 8, 8), 0.5, 2)])
def test_init_wigner_matches_oracle(lib, grid):
    og = O.Grid(grid[0], grid[1], grid[2], grid[3])
    ref = O.init_wigner(1001, og, oparams(P1))
    sim = run_gpu(lib, grid, P1, "c128", seed=1001)
    got = sim.fields()[0]
    assert rel(got, ref) < 1e-14
    sim32 = run_gpu(lib, grid, P1, "c64", seed=1001)
    assert rel(sim32.fields()[0], ref) < 1e-7


def test_init_wigner_groups_use_group_counter(lib):
    grids = [(1, (64,), 0.5, 2), (2, (16, 16), 0.5, 2)]
    sim = lib.Sim(grids, P1, dtype="c128")
    sim.init_wigner(7)
    f = sim.fields()
    for gi, g in enumerate(grids):
        og = O.Grid(g[0], g[1], g[2], g[3])
        assert rel(f[gi], O.init_wigner(7, og, oparams(P1), group=gi)) < 1e-14


# ------------------------------------------------------------------ one step, every size
@pytest.mark.parametrize("per_launch", [1, 64])
@pytest.mark.parametrize("n", [8, 16, 32, 64, 128, 256, 512, 1024, 2048, 4096])
def test_one_step_1d_all_sizes(lib, n, per_launch):
    """per_launch 1: the x-pass kernel; 64: the 1D multi-step kernel."""
    grid = (1, (n,), 0.5, 5)
    og = O.Grid(1, (n,), 0.5, 5)
    psi0 = random_field(n, og.shape, noise=0.4)
    ref = O.strang_step(psi0, 0.01, oparams(P1), og)
    for dtype, tol in (("c128", 1e-13), ("c64", 2e-6)):
        sim = lib.Sim([grid], P1, dtype=dtype)
        sim.set_option(lib.OPT_STEPS_PER_LAUNCH_1D, per_launch)
        sim.set_fields([psi0])
        sim.step(1, 0.01)
        assert rel(sim.fields()[0], ref) < tol, dtype


@pytest.mark.parametrize("n,samples", [(2048, 300), (4096, 300), (2048, 40), (4096, 40)])
def test_long_pencils_both_table_forms(lib, n, samples):
    """Pencils of 2048 and 4096 points: up to one workgroup per CU the x-pass
    stages its twiddles in LDS, beyond that it reads them from global memory;
    both forms, in every mode a step and the observables use, against the
    oracle."""
    grid = (1, (n,), 0.5, samples)
    og = O.Grid(1, (n,), 0.5, samples)
    psi0 = random_field(n + 7, og.shape, noise=0.4)
    ref = O.evolve(psi0, 2, 0.01, oparams(P1), og)
    for dtype, tol in (("c128", 1e-12), ("c64", 5e-6)):
        sim = lib.Sim([grid], P1, dtype=dtype)
        sim.set_option(lib.OPT_STEPS_PER_LAUNCH_1D, 1)
        sim.set_fields([psi0])
        sim.step(2, 0.01)
        assert rel(sim.fields()[0], ref) < tol, dtype
        obs = sim.observables()
        ref_obs = O.observables(ref, oparams(P1), og)
        rt = 1e-10 if dtype == "c128" else 1e-5
        assert np.allclose(obs[:, 0::2], ref_obs[:, 0::2], rtol=rt), dtype  # N, E
        assert np.abs(obs[:, 1] - ref_obs[:, 1]).max() < rt * ref_obs[:, 0].max(), dtype  # F_z, a difference
        _, _, _, _, per = sim.structure_factor()
        ref_sk = O.structure_factor(ref, og)
        assert rel(per, ref_sk) < (1e-10 if dtype == "c128" else 2e-5), dtype
        sim.close()


@pytest.mark.parametrize("n", [8, 16, 64, 256, 512, 1024, 2048, 4096])
def test_multi_step_1d_chunks_match_oracle(lib, n):
    """23 steps as launches of 7, 7, 7 and 2 steps (first opens, last closes
    with a half step), in both multi-step kernels, against the oracle and
    against one launch per step."""
    grid = (1, (n,), 0.5, 3)
    og = O.Grid(1, (n,), 0.5, 3)
    psi0 = random_field(n + 1, og.shape, noise=0.4)
    ref = O.evolve(psi0, 23, 0.01, oparams(P1), og)
    for dtype, tol, tol_pair in (("c128", 1e-12, 1e-13), ("c64", 1e-5, 5e-6)):
        out = {}
        for per_launch, kern in ((1, 0), (7, 1), (7, 2)):
            sim = lib.Sim([grid], P1, dtype=dtype)
            sim.set_option(lib.OPT_STEPS_PER_LAUNCH_1D, per_launch)
            sim.set_option(lib.OPT_1D_KERNEL, kern)
            sim.set_fields([psi0])
            sim.step(23, 0.01)
            out[kern] = sim.fields()[0]
            assert rel(out[kern], ref) < tol, (dtype, per_launch, kern)
        assert rel(out[1], out[0]) < tol_pair and rel(out[2], out[0]) < tol_pair, dtype


def test_multi_step_1d_graph_and_option(lib):
    """Changing the steps per launch retires captured graphs; replays of the
    multi-step launches equal direct launches."""
    grid = (1, (512,), 0.5, 6)
    a = lib.Sim([grid], P1, dtype="c64")
    b = lib.Sim([grid], P1, dtype="c64")
    b.set_option(lib.OPT_GRAPHS, 0)
    a.init_wigner(12)
    b.init_wigner(12)
    for rep in range(3):
        a.step(40, 0.02)
        b.step(40, 0.02)
        assert np.array_equal(a.fields()[0], b.fields()[0]), rep
    a.set_option(lib.OPT_STEPS_PER_LAUNCH_1D, 1)
    b.set_option(lib.OPT_STEPS_PER_LAUNCH_1D, 1)
    a.step(40, 0.02)
    b.step(40, 0.02)
    assert np.array_equal(a.fields()[0], b.fields()[0])
    a.set_option(lib.OPT_STEPS_PER_LAUNCH_1D, 0)  # automatic
    b.set_option(lib.OPT_STEPS_PER_LAUNCH_1D, 0)
    a.step(40, 0.02)
    b.step(40, 0.02)
    assert np.array_equal(a.fields()[0], b.fields()[0])
    for bad in (-1, 1025):
        with pytest.raises(lib.Spin1Error):
            a.set_option(lib.OPT_STEPS_PER_LAUNCH_1D, bad)


@pytest.mark.parametrize("ny", [8, 16, 32, 64, 128, 256, 512, 1024])
def test_one_step_2d_all_strided_sizes(lib, ny):
    nx = 16
    grid = (2, (nx, ny), 0.5, 2)
    og = O.Grid(2, (nx, ny), 0.5, 2)
    psi0 = random_field(ny + 1, og.shape, noise=0.4)
    ref = O.strang_step(psi0, 0.02, oparams(P1), og)
    got = run_gpu(lib, grid, P1, "c128", psi0=psi0, nsteps=1, dt=0.02).fields()[0]
    assert rel(got, ref) < 1e-13
    got32 = run_gpu(lib, grid, P1, "c64", psi0=psi0, nsteps=1, dt=0.02).fields()[0]
    assert rel(got32, ref) < 2e-6


@pytest.mark.parametrize("n", [(16, 1024, 8), (16, 8, 1024), (64, 8, 8)])
def test_one_step_3d_longest_strided_axes(lib, n):
    """3D grids with the longest y or z axis (1024 points) and a short one."""
    grid = (3, n, 0.5, 2)
    og = O.Grid(3, n, 0.5, 2)
    psi0 = random_field(n[1] + 7 * n[2], og.shape, noise=0.4)
    ref = O.strang_step(psi0, 0.02, oparams(P3), og)
    for dtype, tol in (("c128", 1e-13), ("c64", 2e-6)):
        got = run_gpu(lib, grid, P3, dtype, psi0=psi0, nsteps=1, dt=0.02).fields()[0]
        assert rel(got, ref) < tol, dtype


def test_one_step_3d_non_cubic(lib):
    grid = (3, (32, 16, 8), 0.5, 2)
    og = O.Grid(3, (32, 16, 8), 0.5, 2)
    psi0 = random_field(3, og.shape, noise=0.4)
    ref = O.strang_step(psi0, 0.02, oparams(P3), og)
    got = run_gpu(lib, grid, P3, "c128", psi0=psi0, nsteps=1, dt=0.02).fields()[0]
    assert rel(got, ref) < 1e-13


# ------------------------------------------------------------------ 100 steps
HUNDRED = [
    ((1, (256,), 0.5, 4), P1, 0.01),         # the 1D L=256 FP64 configuration
    ((2, (64, 32), 0.5, 3), P1, 0.02),       # several tiles, ragged pencil count
    ((3, (16, 16, 16), 0.5, 2), P3, 0.02),
]
# the complex64 error over the single-precision floor of the dynamics (below):
# measured 5.0 (1D), 5.7 (2D) and 5.2 (3D); the bound leaves 20% on the largest
FLOOR_FACTOR = 7.0
_hundred_cache = {}


def hundred_step_case(lib, grid, p, dt):
    """(complex128 error, complex64 error, floor) after 100 steps against the oracle."""
    key = (grid, dt)
    if key not in _hundred_cache:
        og = O.Grid(grid[0], grid[1], grid[2], grid[3])
        psi0 = O.init_wigner(1001, og, oparams(p))
        ref = O.evolve(psi0, 100, dt, oparams(p), og)
        got = run_gpu(lib, grid, p, "c128", seed=1001, nsteps=100, dt=dt).fields()[0]
        # complex64 starts from the rounded FP64 initial state
        got32 = run_gpu(lib, grid, p, "c64", seed=1001, nsteps=100, dt=dt).fields()[0]
        floor = single_precision_floor(psi0, 100, dt, p, og, ref)
        _hundred_cache[key] = (rel(got, ref), rel(got32, ref), floor)
    return _hundred_cache[key]


@pytest.mark.parametrize("grid,p,dt", HUNDRED)
def test_hundred_steps(lib, grid, p, dt):
    e128, e64, floor = hundred_step_case(lib, grid, p, dt)
    print("%dD %s: complex128 %.2e; complex64 %.2e = %.2f x the floor %.2e"
          % (grid[0], grid[1], e128, e64, e64 / floor, floor))
    assert e128 < 1e-10
    assert e64 < FLOOR_FACTOR * floor


@pytest.mark.parametrize("grid,p,dt", [
    HUNDRED[0], HUNDRED[1],
    pytest.param(*HUNDRED[2], marks=pytest.mark.xfail(
        strict=True, reason="the 3D parameters amplify rounding ~7000-fold in 100 steps: the single-precision "
                            "floor of the dynamics itself (5e-4) is above 1e-4, so complex64 misses the target")),
])
def test_hundred_steps_single_precision_target(lib, grid, p, dt):
    """The stated complex64 tolerance, 1e-4 relative L2 after 100 steps."""
    assert hundred_step_case(lib, grid, p, dt)[1] < 1e-4


def single_precision_floor(psi0, nsteps, dt, p, og, ref):
    """Error of the oracle itself when its state is rounded to complex64
    after every step (FP64 arithmetic otherwise)."""
    cur = psi0.astype(np.complex64).astype(np.complex128)
    for _ in range(nsteps):
        cur = O.strang_step(cur, dt, oparams(p), og).astype(np.complex64).astype(np.complex128)
    return rel(cur, ref)


def test_step_calls_compose(lib):
    """n steps in one call equal the same steps split over several calls."""
    grid = (2, (32, 32), 0.5, 2)
    og = O.Grid(2, (32, 32), 0.5, 2)
    psi0 = random_field(5, og.shape)
    a = run_gpu(lib, grid, P1, "c128", psi0=psi0, nsteps=10, dt=0.02).fields()[0]
    sim = run_gpu(lib, grid, P1, "c128", psi0=psi0)
    for k in (3, 1, 6):
        sim.step(k, 0.02)
    assert rel(sim.fields()[0], a) < 1e-13


def test_time_reversal_on_gpu(lib):
    grid = (2, (64, 64), 0.5, 2)
    og = O.Grid(2, (64, 64), 0.5, 2)
    psi0 = random_field(6, og.shape)
    sim = run_gpu(lib, grid, P1, "c128", psi0=psi0, nsteps=50, dt=0.02)
    sim.step(50, -0.02)
    assert rel(sim.fields()[0], psi0) < 1e-12


def test_zero_steps_is_identity(lib):
    grid = (1, (64,), 0.5, 2)
    og = O.Grid(1, (64,), 0.5, 2)
    psi0 = random_field(8, og.shape)
    sim = run_gpu(lib, grid, P1, "c128", psi0=psi0)
    sim.step(0, 0.01)
    assert np.array_equal(sim.fields()[0], psi0)


def test_sync_field_leaves_the_synchronized_field_alone(lib):
    """Step calls end at a synchronized time, so spin1_sync_field has nothing
    to apply: it rejects an unbound context and leaves a stepped field bit for
    bit as it was."""
    fresh = lib.create(lib.C128)
    with pytest.raises(lib.Spin1Error) as err:
        lib.sync_field(fresh)
    assert err.value.code == lib.ESTATE
    lib.destroy(fresh)
    grid = (2, (32, 16), 0.5, 2)
    og = O.Grid(2, (32, 16), 0.5, 2)
    psi0 = random_field(10, og.shape)
    sim = run_gpu(lib, grid, P1, "c128", psi0=psi0, nsteps=3, dt=0.01)
    before = sim.fields()[0]
    lib.sync_field(sim.ctx)
    sim.synchronize()
    assert np.array_equal(sim.fields()[0], before)
    ref = O.evolve(psi0, 3, 0.01, oparams(P1), og)
    assert rel(before, ref) < 1e-12


def test_long_run_single_precision_ensemble_statistics(lib):
    """Past the chaotic horizon the complex64 and complex128 trajectories of
    one seed part ways (measured: relative difference sqrt(2), that of
    unrelated fields, from step 500 on), so what has to agree after 10^4
    steps of 0.02 is the ensemble: the sample-mean S(k) of every shell within
    four combined standard errors (measured rms z 0.96 over 92 shells), and
    each sample's N and F_z, which the step conserves (measured drift 5e-7 in
    complex64, 3e-12 in complex128)."""
    grid = (2, (128, 128), 0.5, 64)
    out = {}
    for dtype in ("c128", "c64"):
        sim = lib.Sim([grid], P1, dtype=dtype)
        sim.init_wigner(1007)
        obs0 = sim.observables()
        sim.step(10000, 0.02)
        _, mean, se, _, _ = sim.structure_factor()
        obs1 = sim.observables()
        out[dtype] = (mean, se)
        sim.close()
        assert np.allclose(obs1[:, 0], obs0[:, 0], rtol=1e-5 if dtype == "c64" else 1e-11), dtype
        assert np.allclose(obs1[:, 1], obs0[:, 1], atol=(1e-5 if dtype == "c64" else 1e-11) * obs0[:, 0].max()), dtype
    (m64, s64), (m128, s128) = out["c64"], out["c128"]
    z = np.abs(m64 - m128) / np.sqrt(s64**2 + s128**2)
    assert z.max() < 4.0, (int(z.argmax()), float(z.max()))


@pytest.mark.timeout(300)
def test_long_run_ensemble_matches_oracle_ensemble(lib):
    """1D 64 sites x 64 samples, 1000 steps of 0.05 (t = 50) in complex128 on
    the GPU and in the oracle from the same seed.  Rounding differences grow
    by about e^1.1 per unit of time here (measured: 7e-2 relative at t = 30),
    so by the end the fields are unrelated (measured: 1.3 relative) and the
    comparison is between ensembles (measured: rms z 0.87 over 33 shells): the
    sample-mean S(k) of every shell within four combined standard errors, and
    N and F_z of every sample (conserved by both) to 1e-10."""
    grid = (1, (64,), 0.5, 64)
    sim = lib.Sim([grid], P1, dtype="c128")
    sim.init_wigner(1008)
    sim.step(1000, 0.05)
    _, m_gpu, se_gpu, _, _ = sim.structure_factor()
    obs = sim.observables()
    psi_gpu = sim.fields()[0]
    sim.close()
    og = O.Grid(1, (64,), 0.5, 64)
    p = oparams(P1)
    psi = O.evolve(O.init_wigner(1008, og, p), 1000, 0.05, p, og)
    m_ora, se_ora = O.sample_mean_se(O.structure_factor(psi, og))
    z = np.abs(m_gpu - m_ora) / np.sqrt(se_gpu**2 + se_ora**2)
    print("field rel diff %.3e, z rms %.2f max %.2f" % (rel(psi_gpu, psi), np.sqrt((z**2).mean()), z.max()))
    assert z.max() < 4.0, (int(z.argmax()), float(z.max()))
    ref = O.observables(psi, p, og)
    assert np.allclose(obs[:, 0], ref[:, 0], rtol=1e-10)
    assert np.allclose(obs[:, 1], ref[:, 1], atol=1e-10 * ref[:, 0].max())


def test_quench_set_params(lib):
    grid = (1, (128,), 0.5, 2)
    og = O.Grid(1, (128,), 0.5, 2)
    psi0 = random_field(9, og.shape)
    p2 = dict(P1, q=0.3)
    ref = O.evolve(O.evolve(psi0, 5, 0.01, oparams(P1), og), 5, 0.01, oparams(p2), og)
    sim = run_gpu(lib, grid, P1, "c128", psi0=psi0, nsteps=5)
    sim.set_params(p2)
    sim.step(5, 0.01)
    assert rel(sim.fields()[0], ref) < 1e-12


def test_local_update_matches_oracle(lib):
    grid = (2, (16, 8), 0.5, 2)
    og = O.Grid(2, (16, 8), 0.5, 2)
    psi0 = random_field(10, og.shape, noise=1.0)
    sim = run_gpu(lib, grid, P1, "c128", psi0=psi0)
    sim.local_update(0.7)
    assert rel(sim.fields()[0], O.local_flow(psi0, 0.7, P1["c0"], P1["c1"])) < 1e-13


# ------------------------------------------------------------------ multiple groups
def test_uneven_groups_step(lib):
    grids = [(1, (4096,), 0.5, 3), (2, (32, 32), 0.5, 2), (2, (64, 16), 0.5, 1)]
    sim = lib.Sim(grids, P1, dtype="c128")
    sim.init_wigner(11)
    sim.step(20, 0.02)
    f = sim.fields()
    for gi, g in enumerate(grids):
        og = O.Grid(g[0], g[1], g[2], g[3])
        ref = O.evolve(O.init_wigner(11, og, oparams(P1), group=gi), 20, 0.02, oparams(P1), og)
        assert rel(f[gi], ref) < 1e-11


@pytest.mark.parametrize("dtype,tol", [("c128", 1e-11), ("c64", 2e-5)])
def test_grouped_x_pass_matches_oracle(lib, dtype, tol):
    """Groups of different pencil lengths share one x-pass launch per step
    (a 1D group stepped one launch per step among them, with its closing half
    step); results equal the oracle and the per-group launches."""
    grids = [(2, (64, 32), 0.5, 2), (1, (256,), 0.5, 3), (3, (16, 16, 8), 0.5, 1), (2, (1024, 16), 0.5, 1),
             (2, (16, 64), 0.5, 3)]
    out = {}
    for grouped in (1, 0):
        sim = lib.Sim(grids, P1, dtype=dtype)
        sim.set_option(lib.OPT_STEPS_PER_LAUNCH_1D, 1)
        sim.set_option(lib.OPT_GROUPED_X, grouped)
        sim.init_wigner(16)
        sim.step(7, 0.02)
        sim.step(3, 0.02)
        out[grouped] = sim.fields()
    for gi, g in enumerate(grids):
        og = O.Grid(g[0], g[1], g[2], g[3])
        ref = O.evolve(O.init_wigner(16, og, oparams(P1), group=gi), 10, 0.02, oparams(P1), og)
        assert rel(out[1][gi], ref) < tol, gi
        assert rel(out[1][gi], out[0][gi]) < tol / 10, gi


@pytest.mark.parametrize("grouped", [1, 0])
def test_more_groups_than_one_grouped_launch_takes(lib, grouped):
    """Nine eligible groups.  Grouped: eight share the grouped x-pass, the
    ninth runs its own launches on a side stream.  Not grouped: nine
    sequences on four streams, round robin.  All match the oracle."""
    sizes = [(16, 16), (32, 16), (16, 32), (64, 16), (16, 64), (32, 32), (128, 16), (16, 128), (64, 32)]
    grids = [(2, n, 0.5, 1) for n in sizes]
    sim = lib.Sim(grids, P1, dtype="c128")
    sim.set_option(lib.OPT_GROUPED_X, grouped)
    sim.init_wigner(25)
    sim.step(6, 0.02)
    f = sim.fields()
    for gi, g in enumerate(grids):
        og = O.Grid(g[0], g[1], g[2], g[3])
        ref = O.evolve(O.init_wigner(25, og, oparams(P1), group=gi), 6, 0.02, oparams(P1), og)
        assert rel(f[gi], ref) < 1e-12, gi


@pytest.mark.parametrize("grouped", [0, 1])
def test_concurrent_groups_match_one_stream(lib, grouped):
    """Independent group sequences on streams of their own (forked and joined
    inside each call, captured into the graph; with the grouped x-pass, the
    grouped set is one sequence): bit-identical to one stream, over replays
    with eager work in between."""
    grids = [(1, (4096,), 0.5, 3), (2, (64, 32), 0.5, 2), (1, (512,), 0.5, 2), (2, (128, 16), 0.5, 2),
             (3, (16, 16, 16), 0.5, 1)]
    sims = []
    for conc in (1, 0):
        s = lib.Sim(grids, P1, dtype="c64")
        s.set_option(lib.OPT_CONCURRENT_GROUPS, conc)
        s.set_option(lib.OPT_GROUPED_X, grouped)
        s.init_wigner(24)
        sims.append(s)
    for rep in range(3):
        for s in sims:
            s.step(9, 0.02)
        fa, fb = sims[0].fields(), sims[1].fields()
        for gi in range(len(grids)):
            assert np.array_equal(fa[gi], fb[gi]), (rep, gi)
        sims[0].observables(1)


@pytest.mark.parametrize("grid", [(1, (256,), 0.5, 3), (2, (64, 32), 0.5, 2), (3, (16, 8, 16), 0.5, 2)])
def test_paper_scheme_matches_oracle(lib, grid):
    """The paper's Lie scheme (kinetic, Eq. (4) phases, Eq. (5) mixing with the
    predictor) against the oracle's literal step, split over two calls."""
    og = O.Grid(grid[0], grid[1], grid[2], grid[3])
    p, dt = oparams(P1), 0.02
    psi0 = random_field(17, og.shape, noise=0.5)
    ref = psi0
    for _ in range(7):
        ref = O.paper_step(ref, dt, p, og)
    for dtype, tol in (("c128", 1e-12), ("c64", 2e-5)):
        sim = lib.Sim([grid], P1, dtype=dtype)
        sim.set_option(lib.OPT_SCHEME, lib.SCHEME_PAPER)
        sim.set_fields([psi0])
        sim.step(4, dt)
        sim.step(3, dt)
        assert rel(sim.fields()[0], ref) < tol, dtype


def test_paper_scheme_first_order_and_limits(lib):
    """First-order convergence to the same flow as the symmetric split, on the
    GPU; the scheme is rejected where only the symmetric split is supported."""
    grid = (2, (32, 32), 0.5, 2)
    og = O.Grid(2, (32, 32), 0.5, 2)
    psi0 = random_field(18, og.shape, noise=0.3)
    t_end = 0.32

    def run(scheme, m):
        sim = lib.Sim([grid], P1, dtype="c128")
        sim.set_option(lib.OPT_SCHEME, scheme)
        sim.set_fields([psi0])
        sim.step(m, t_end / m)
        return sim.fields()[0]

    ref = run(lib.SCHEME_STRANG, 256)
    e = [rel(run(lib.SCHEME_PAPER, m), ref) for m in (16, 32, 64)]
    assert 1.7 < e[0] / e[1] < 2.3 and 1.7 < e[1] / e[2] < 2.3, e
    sim = lib.Sim([grid], P1, dtype="c128")
    sim.init_wigner(3)
    sim.set_option(lib.OPT_SCHEME, lib.SCHEME_PAPER)
    with pytest.raises(lib.Spin1Error):
        sim.step_observed(2, 0.02)
    with pytest.raises(lib.Spin1Error):
        sim.forward_ckpt(4, 0.02, 2)
    with pytest.raises(lib.Spin1Error):
        sim.set_option(lib.OPT_SCHEME, 7)


# ------------------------------------------------------------------ real-space spin texture
@pytest.mark.parametrize("grid", [(1, (256,), 0.5, 3), (2, (64, 32), 0.5, 2), (3, (16, 8, 16), 0.5, 2)])
def test_spin_texture_matches_oracle(lib, grid):
    og = O.Grid(grid[0], grid[1], grid[2], grid[3])
    psi0 = random_field(19, og.shape, noise=0.8)
    ref_fp = O.f_perp(psi0)
    ref = O.spin_texture(psi0, og)
    for dtype, tol in (("c128", 1e-13), ("c64", 2e-6)):
        sim = run_gpu(lib, grid, P1, dtype, psi0=psi0)
        fp_dev = sim.transverse_spin()
        sim.synchronize()
        fp = fp_dev.cpu().numpy()
        assert rel(fp, ref_fp) < tol, dtype
        tex = sim.spin_texture()
        assert np.allclose(tex[:, :2], ref[:, :2], rtol=tol), dtype
        if dtype == "c128":
            assert np.allclose(tex[:, 2], ref[:, 2], atol=1e-9)
        # the winding of a periodic row is an integer
        assert np.allclose(tex[:, 2], np.round(tex[:, 2]), atol=1e-6 if dtype == "c64" else 1e-9)


@pytest.mark.parametrize("w", [-2, 3])
def test_spin_texture_of_helix_and_after_steps(lib, w):
    grid = (1, (512,), 0.5, 2)
    og = O.Grid(1, (512,), 0.5, 2)
    psi = O.spin_helix(og, w)
    for dtype in ("c128", "c64"):
        sim = run_gpu(lib, grid, P1, dtype, psi0=psi)
        tex = sim.spin_texture()
        assert np.allclose(tex[:, 2], w, atol=1e-6) and np.allclose(tex[:, 0], 1.0, rtol=1e-6)
    # a Wigner run keeps integer windings
    sim = run_gpu(lib, grid, P1, "c128", seed=20, nsteps=200, dt=0.02)
    q = sim.spin_texture()[:, 2]
    assert np.allclose(q, np.round(q), atol=1e-9)
    og2 = O.Grid(1, (512,), 0.5, 2)
    assert np.allclose(q, O.spin_texture(sim.fields()[0], og2)[:, 2], atol=1e-9)


# ------------------------------------------------------------------ structure factor
@pytest.mark.parametrize("grid", [(1, (256,), 0.5, 4), (2, (32, 64), 0.5, 3), (3, (16, 16, 8), 0.5, 2),
                                  (1, (4096,), 0.5, 2), (2, (256, 256), 0.5, 1)])
def test_structure_factor_matches_oracle(lib, grid):
    og = O.Grid(grid[0], grid[1], grid[2], grid[3])
    psi0 = random_field(12, og.shape, noise=0.5)
    ref = O.structure_factor(psi0, og)
    sim = run_gpu(lib, grid, P1, "c128", psi0=psi0)
    got = sim.structure_factor_samples()
    assert got.shape == ref.shape
    assert np.max(np.abs(got - ref)) <= 1e-12 * np.max(np.abs(ref))
    sim32 = run_gpu(lib, grid, P1, "c64", psi0=psi0)
    got32 = sim32.structure_factor_samples()
    assert np.max(np.abs(got32 - ref)) <= 1e-5 * np.max(np.abs(ref))


def test_structure_factor_deterministic(lib):
    grid = (2, (64, 64), 0.5, 4)
    sim = run_gpu(lib, grid, P1, "c64", seed=3)
    a = sim.structure_factor_samples()
    b = sim.structure_factor_samples()
    assert np.array_equal(a, b)


# ------------------------------------------------------------------ observables
@pytest.mark.parametrize("grid", [(1, (256,), 0.5, 3), (2, (64, 32), 0.5, 2), (3, (16, 8, 16), 0.5, 2),
                                  (1, (2048,), 0.5, 2)])
def test_observables_match_oracle(lib, grid):
    og = O.Grid(grid[0], grid[1], grid[2], grid[3])
    psi0 = random_field(13, og.shape, noise=0.5)
    ref = O.observables(psi0, oparams(P1), og)
    got = run_gpu(lib, grid, P1, "c128", psi0=psi0).observables()
    assert np.allclose(got, ref, rtol=1e-12, atol=1e-12 * np.abs(ref).max())
    got32 = run_gpu(lib, grid, P1, "c64", psi0=psi0).observables()
    assert np.allclose(got32, ref, rtol=2e-6, atol=2e-6 * np.abs(ref).max())


@pytest.mark.parametrize("grid", [(1, (256,), 0.5, 3), (2, (64, 32), 0.5, 2), (3, (16, 8, 16), 0.5, 2)])
def test_step_observed_matches_oracle(lib, grid):
    """Per-step logged (N, F_z, E) of R(dt/2) psi(t_i) against the oracle, and
    the stepped field against plain spin1_step."""
    og = O.Grid(grid[0], grid[1], grid[2], grid[3])
    p, dt, n = oparams(P1), 0.02, 6
    psi0 = random_field(14, og.shape, noise=0.5)
    ref, cur = [], psi0
    for i in range(n):
        ref.append(O.observables(O.local_flow(cur, 0.5 * dt, p.c0, p.c1), p, og))
        cur = O.strang_step(cur, dt, p, og)
    ref = np.array(ref)
    for dtype, tol in (("c128", 1e-12), ("c64", 2e-6)):
        sim = run_gpu(lib, grid, P1, dtype, psi0=psi0)
        obs = sim.step_observed(n, dt)
        assert obs.shape == (n, og.samples, 3)
        assert np.allclose(obs, ref, rtol=tol, atol=tol * np.abs(ref).max()), dtype
        plain = run_gpu(lib, grid, P1, dtype, psi0=psi0, nsteps=n, dt=dt).fields()[0]
        assert rel(sim.fields()[0], plain) < (1e-13 if dtype == "c128" else 1e-6), dtype
        # N and F_z are those of psi(t_i) itself (R conserves them); F_z, a
        # difference of two densities, carries the rounding of N
        o0 = O.observables(psi0, p, og)
        assert np.allclose(obs[0, :, :2], o0[:, :2], rtol=tol, atol=tol * np.abs(o0[:, 0]).max())


def test_step_observed_groups_and_errors(lib):
    grids = [(2, (32, 32), 0.5, 2), (1, (128,), 0.5, 3)]
    sim = lib.Sim(grids, P1, dtype="c128")
    sim.init_wigner(15)
    f0 = sim.fields()
    obs = sim.step_observed(4, 0.02, group=1)
    assert obs.shape == (4, 3, 3)
    f = sim.fields()
    for gi, g in enumerate(grids):
        og = O.Grid(g[0], g[1], g[2], g[3])
        assert rel(f[gi], O.evolve(f0[gi], 4, 0.02, oparams(P1), og)) < 1e-12
    import torch
    buf = torch.zeros(64, dtype=torch.float64, device=sim.device)
    with pytest.raises(lib.Spin1Error):
        lib.step_observed(sim.ctx, 2, 0.02, 2, buf.data_ptr())  # no group 2
    with pytest.raises(lib.Spin1Error):
        lib.step_observed(sim.ctx, 2, 0.02, 0, 0)  # NULL log
    assert sim.step_observed(0, 0.02).shape == (0, 2, 3)


def test_norm_and_fz_conserved_on_gpu(lib):
    grid = (2, (128, 128), 0.5, 4)
    sim = run_gpu(lib, grid, P1, "c64", seed=21)
    o0 = sim.observables()
    sim.step(200, 0.02)
    o1 = sim.observables()
    assert np.allclose(o1[:, 0], o0[:, 0], rtol=1e-5)
    assert np.allclose(o1[:, 1], o0[:, 1], rtol=0, atol=1e-5 * o0[:, 0].max())


# ------------------------------------------------------------------ graph replay
def test_profiling_times_each_pass_by_its_own_launch(lib):
    """The profiling mode times every step pass by the kernel's own begin and
    end, and a scope with several launches by events around it: counts per
    kind, positive times, and the same field as unprofiled direct launches;
    the sum of the per-kernel times stays below the wall time of the calls."""
    import torch

    grid = (2, (64, 32), 0.5, 3)
    a = lib.Sim([grid], P1, dtype="c64")
    b = lib.Sim([grid], P1, dtype="c64")
    a.init_wigner(5)
    b.init_wigner(5)
    b.set_option(lib.OPT_GRAPHS, 0)
    lib.profile_read(a.ctx)
    lib.profile_enable(a.ctx, True)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(a.stream)
    a.step(7, 0.02)
    a.observables()
    e1.record(a.stream)
    b.step(7, 0.02)
    prof = lib.profile_read(a.ctx)
    lib.profile_enable(a.ctx, False)
    wall = e0.elapsed_time(e1)
    assert np.array_equal(a.fields()[0], b.fields()[0])
    assert prof["xpass"][1] == 7 and prof["ypass"][1] == 7 and prof["local"][1] == 1, prof
    assert prof["observables"][1] == 1, prof  # x-pass, y-pass and finish under one scope
    for k in ("xpass", "ypass", "local", "observables"):
        assert prof[k][0] > 0, (k, prof)
    assert sum(v[0] for v in prof.values()) < wall, (prof, wall)
    a.close()
    b.close()


def test_graph_replays_match_direct_launches(lib):
    """Captured step sequences replay bit-identically to direct launches, with
    eager work and synchronisation between the replays."""
    grid = (2, (64, 32), 0.5, 3)
    a = lib.Sim([grid], P1, dtype="c64")
    b = lib.Sim([grid], P1, dtype="c64")
    b.set_option(lib.OPT_GRAPHS, 0)
    a.init_wigner(5)
    b.init_wigner(5)
    for rep in range(4):
        a.step(10, 0.02)
        b.step(10, 0.02)
        fa, fb = a.fields()[0], b.fields()[0]
        assert np.array_equal(fa, fb), "replay %d differs" % rep
        # eager work between replays
        assert np.array_equal(a.structure_factor_samples(), b.structure_factor_samples())
        a.observables()
    # a new dt and new couplings retire the old graphs
    a.step(7, 0.01)
    b.step(7, 0.01)
    p2 = dict(P1, q=0.2)
    a.set_params(p2)
    b.set_params(p2)
    a.step(10, 0.02)
    b.step(10, 0.02)
    assert np.array_equal(a.fields()[0], b.fields()[0])


def test_graph_chunking_matches_split_calls(lib):
    grid = (1, (256,), 0.5, 4)
    a = lib.Sim([grid], P1, dtype="c128")
    a.set_option(lib.OPT_GRAPH_MAX_STEPS, 4)
    b = lib.Sim([grid], P1, dtype="c128")
    b.set_option(lib.OPT_GRAPHS, 0)
    a.init_wigner(6)
    b.init_wigner(6)
    a.step(10, 0.01)
    for k in (4, 4, 2):
        b.step(k, 0.01)
    assert np.array_equal(a.fields()[0], b.fields()[0])


def test_graph_option_validation(lib):
    sim = lib.Sim([(1, (64,), 0.5, 1)], P1)
    with pytest.raises(lib.Spin1Error):
        sim.set_option(lib.OPT_GRAPH_MAX_STEPS, 0)
    with pytest.raises(lib.Spin1Error):
        sim.set_option(99, 1)
    with pytest.raises(lib.Spin1Error):
        sim.set_option(lib.OPT_STREAMING_STORES, 3)


@pytest.mark.parametrize("grid,p", [((2, (64, 256), 0.5, 3), P1), ((3, (32, 16, 256), 0.5, 2), P3)])
@pytest.mark.parametrize("dtype", ["c64", "c128"])
def test_streaming_stores_give_the_same_fields(lib, grid, p, dtype):
    """The non-temporal and the ordinary field stores of the step passes give
    the same fields bit for bit (every variant of the strided pass, graphs on),
    and both match the oracle step."""
    og = O.Grid(grid[0], grid[1], grid[2], grid[3])
    psi0 = random_field(41, og.shape, noise=0.4)
    ref = O.strang_step(psi0, 0.02, oparams(p), og)
    for v in range(lib.num_variants()):
        out = []
        for form in (lib.STORES_CACHED, lib.STORES_STREAMING, lib.STORES_AUTO):
            sim = lib.Sim([grid], p, dtype=dtype)
            sim.set_option(lib.OPT_STREAMING_STORES, form)
            for a in range(1, grid[0]):
                lib.set_variant(sim.ctx, 1, grid[1][a], v)
            sim.set_fields([psi0])
            sim.step(1, 0.02)
            out.append(sim.fields()[0])
            sim.step(5, 0.02)
            out.append(sim.fields()[0])
            sim.close()
        assert np.array_equal(out[0], out[2]) and np.array_equal(out[1], out[3]), (dtype, v)
        assert np.array_equal(out[0], out[4]) and np.array_equal(out[1], out[5]), (dtype, v)
        assert rel(out[2], ref) < (1e-13 if dtype == "c128" else 2e-6), (dtype, v)


# ------------------------------------------------------------------ step-pass variants and autotuning
@pytest.mark.parametrize("nx,ny", [(16, 8), (64, 128), (512, 512), (16, 512), (256, 1024), (1024, 64), (4096, 16),
                                   (64, 256), (16, 256)])
def test_every_step_variant_matches_oracle(lib, nx, ny):
    # (64, 256): two 32-column tiles of variant 1 on 256-point columns;
    # (16, 256): rows narrower than that tile, where variant 1 runs the default
    grid = (2, (nx, ny), 0.5, 2)
    og = O.Grid(2, (nx, ny), 0.5, 2)
    psi0 = random_field(nx + ny, og.shape, noise=0.4)
    ref = O.strang_step(psi0, 0.02, oparams(P1), og)
    for dtype, tol in (("c128", 1e-13), ("c64", 2e-6)):
        for v in range(lib.num_variants()):
            sim = lib.Sim([grid], P1, dtype=dtype)
            lib.set_variant(sim.ctx, 0, nx, v)
            lib.set_variant(sim.ctx, 1, ny, v)
            sim.set_fields([psi0])
            sim.step(1, 0.02)
            assert rel(sim.fields()[0], ref) < tol, (dtype, v)
            sim.close()


@pytest.mark.parametrize("n", [(32, 256, 16), (16, 32, 256)])
def test_every_strided_variant_3d(lib, n):
    """Every strided-pass variant on a 256-point y or z axis of a 3D grid (one
    32-column tile across 32 rows of x, and 16 tiles across the 16 x 32 plane)."""
    grid = (3, n, 0.5, 2)
    og = O.Grid(3, n, 0.5, 2)
    psi0 = random_field(n[1] + 3 * n[2], og.shape, noise=0.4)
    ref = O.strang_step(psi0, 0.02, oparams(P3), og)
    for dtype, tol in (("c128", 1e-13), ("c64", 2e-6)):
        for v in range(lib.num_variants()):
            sim = lib.Sim([grid], P3, dtype=dtype)
            for a in (1, 2):
                lib.set_variant(sim.ctx, 1, n[a], v)
            sim.set_fields([psi0])
            sim.step(1, 0.02)
            assert rel(sim.fields()[0], ref) < tol, (dtype, v)
            sim.close()


@pytest.mark.parametrize("mode", ["dithered", "compensated"])
def test_fp32_table_options(lib, mode):
    """Both FP32 table forms of the streaming passes: every variant matches the
    oracle step to single precision, and over 100 steps neither adds a
    rounding that grows step after step (dithered: 2.1e-5, compensated 2.1e-5
    here; a once-rounded table measured 9.3e-5)."""
    opt = lib.TWIDDLES_DITHERED if mode == "dithered" else lib.TWIDDLES_COMPENSATED
    grid = (2, (512, 256), 0.5, 2)
    og = O.Grid(2, (512, 256), 0.5, 2)
    psi0 = random_field(23, og.shape, noise=0.4)
    ref = O.strang_step(psi0, 0.02, oparams(P1), og)
    for v in range(lib.num_variants()):
        sim = lib.Sim([grid], P1, dtype="c64")
        sim.set_option(lib.OPT_FP32_TWIDDLES, opt)
        lib.set_variant(sim.ctx, 0, 512, v)
        lib.set_variant(sim.ctx, 1, 256, v)
        sim.set_fields([psi0])
        sim.step(1, 0.02)
        assert rel(sim.fields()[0], ref) < 3e-6, v
        sim.close()
    g2 = (2, (64, 32), 0.5, 3)
    og2 = O.Grid(2, (64, 32), 0.5, 3)
    psi = O.init_wigner(1001, og2, oparams(P1))
    ref100 = O.evolve(psi, 100, 0.02, oparams(P1), og2)
    for calls in (1, 10):  # the dithering restarts with every call
        sim = lib.Sim([g2], P1, dtype="c64")
        sim.set_option(lib.OPT_FP32_TWIDDLES, opt)
        sim.init_wigner(1001)
        for _ in range(calls):
            sim.step(100 // calls, 0.02)
        assert rel(sim.fields()[0], ref100) < 4e-5, calls
        sim.close()
    with pytest.raises(lib.Spin1Error):
        lib.Sim([g2], P1, dtype="c64").set_option(lib.OPT_FP32_TWIDDLES, 2)


def test_dithered_tables_keep_the_norm_over_long_runs(lib):
    """Over 5000 steps the per-sample norm of the complex64 field drifts much
    less with dithered tables (their rounding does not repeat step after
    step) than with compensated ones (measured 2.2e-7 against 7.4e-7)."""
    grid = (2, (128, 128), 0.5, 4)
    drift = {}
    for opt in (lib.TWIDDLES_DITHERED, lib.TWIDDLES_COMPENSATED):
        sim = lib.Sim([grid], P1, dtype="c64")
        sim.set_option(lib.OPT_FP32_TWIDDLES, opt)
        sim.init_wigner(5)
        n0 = sim.observables()[:, 0]
        for _ in range(5):
            sim.step(1000, 0.02)
        drift[opt] = float(np.max(np.abs(sim.observables()[:, 0] / n0 - 1)))
        sim.close()
    assert drift[lib.TWIDDLES_DITHERED] < 5e-7
    assert drift[lib.TWIDDLES_DITHERED] < 0.6 * drift[lib.TWIDDLES_COMPENSATED]


def test_autotune_choices_and_cache(lib, tmp_path):
    grids = [(2, (128, 64), 0.5, 4), (1, (1024,), 0.5, 8)]
    sim = lib.Sim(grids, P1, dtype="c64")
    sim.init_wigner(3)
    before = sim.fields()
    cache = tmp_path / "tune.json"
    chosen = sim.autotune(reps=2, cache_path=str(cache))
    assert set(chosen) and all(0 <= v < lib.num_variants() for v in chosen.values())
    after = sim.fields()
    for a, b in zip(before, after):
        assert np.array_equal(a, b)  # the bound fields are not touched
    # a second object restores the same choices from the cache without timing
    sim2 = lib.Sim(grids, P1, dtype="c64")
    sim2.init_wigner(3)
    again = sim2.autotune(cache_path=str(cache))
    assert again == chosen
    for (p, n) in sim2.pass_sizes():
        key = [k for k in chosen if k.endswith("/%d/%d" % (p, n))][0]
        assert lib.get_variant(sim2.ctx, p, n) == chosen[key]
    # tuned stepping still matches the oracle
    sim2.step(5, 0.02)
    for gi, g in enumerate(grids):
        og = O.Grid(g[0], g[1], g[2], g[3])
        ref = O.evolve(O.init_wigner(3, og, oparams(P1), group=gi), 5, 0.02, oparams(P1), og)
        assert rel(sim2.fields()[gi], ref) < 2e-5
    with pytest.raises(lib.Spin1Error):
        lib.set_variant(sim.ctx, 0, 512, 7)
    with pytest.raises(lib.Spin1Error):
        lib.set_variant(sim.ctx, 1, 4096, 0)


# ------------------------------------------------------------------ degenerate cases with closed forms
def _free_gaussian(x, t, x0, s0):
    """Free Schroedinger evolution of a normalised Gaussian (hbar = m = 1)."""
    a = 1.0 + 1j * t / s0 ** 2
    return (np.pi * s0 ** 2) ** -0.25 * a ** -0.5 * np.exp(-((x - x0) ** 2) / (2 * s0 ** 2 * a))


@pytest.mark.parametrize("dtype,tol", [("c128", 1e-11), ("c64", 2e-5)])
def test_free_gaussian_on_gpu(lib, dtype, tol):
    """c0 = c1 = q = 0: every component spreads as the free Gaussian, in 1D and
    as a product in 2D, for any dt (the kinetic step is exact)."""
    p0 = dict(c0=0.0, c1=0.0, q=0.0, n0=1.0, wigner_var=0.5)
    x = np.arange(256) * 0.5
    psi = np.zeros((1, 3, 256), complex)
    for c in range(3):
        psi[0, c] = _free_gaussian(x, 0.0, 64.0, 3.0)
    sim = run_gpu(lib, (1, (256,), 0.5, 1), p0, dtype, psi0=psi, nsteps=40, dt=0.125)
    ref = _free_gaussian(x, 5.0, 64.0, 3.0)
    out = sim.fields()[0]
    for c in range(3):
        assert np.max(np.abs(out[0, c] - ref)) < tol * 10
    y = np.arange(128) * 0.5  # box of 64: the tails at the edges stay below 1e-30
    g2 = np.zeros((1, 3, 128, 256), complex)
    for c in range(3):
        g2[0, c] = _free_gaussian(y, 0.0, 32.0, 2.5)[:, None] * _free_gaussian(x, 0.0, 64.0, 3.0)[None, :]
    sim = run_gpu(lib, (2, (256, 128), 0.5, 1), p0, dtype, psi0=g2, nsteps=20, dt=0.1)
    ref2 = _free_gaussian(y, 2.0, 32.0, 2.5)[:, None] * _free_gaussian(x, 2.0, 64.0, 3.0)[None, :]
    out2 = sim.fields()[0]
    for c in range(3):
        assert np.max(np.abs(out2[0, c] - ref2)) < tol * 10


@pytest.mark.parametrize("dtype,tol", [("c128", 1e-12), ("c64", 2e-6)])
def test_uniform_polar_and_ferromagnet_on_gpu(lib, dtype, tol):
    """Uniform polar state: psi_0 = sqrt(n) e^{-i c0 n t}; uniform ferromagnet
    psi_1 = sqrt(n) e^{-i (q + (c0 + c1) n) t}; exact for any dt."""
    p = dict(c0=1.0, c1=-0.1, q=0.3, n0=1.0, wigner_var=0.5)
    n = 1.7
    pol = np.zeros((2, 3, 32, 16), complex)
    pol[:, 1] = np.sqrt(n)
    sim = run_gpu(lib, (2, (16, 32), 0.5, 2), p, dtype, psi0=pol, nsteps=15, dt=0.13)
    out = sim.fields()[0]
    t = 15 * 0.13
    assert np.max(np.abs(out[:, 1] - np.sqrt(n) * np.exp(-1j * p["c0"] * n * t))) < tol * 10
    assert np.max(np.abs(out[:, [0, 2]])) < tol
    fer = np.zeros((1, 3, 64), complex)
    fer[:, 0] = np.sqrt(0.8)
    p2 = dict(c0=1.2, c1=-0.4, q=0.7, n0=1.0, wigner_var=0.5)
    sim = run_gpu(lib, (1, (64,), 0.5, 1), p2, dtype, psi0=fer, nsteps=6, dt=0.5)
    ph = np.exp(-1j * (p2["q"] + (p2["c0"] + p2["c1"]) * 0.8) * 3.0)
    out = sim.fields()[0]
    assert np.max(np.abs(out[:, 0] - np.sqrt(0.8) * ph)) < tol * 10
    assert np.max(np.abs(out[:, 1:])) < tol


@pytest.mark.parametrize("dtype", ["c128", "c64"])
@pytest.mark.parametrize("grid", [(1, (4096,), 0.5, 3), (2, (512, 64), 0.5, 2), (3, (32, 16, 64), 0.5, 2)])
def test_vacuum_stays_empty(lib, grid, dtype):
    """The empty field (no condensate, no noise) is a fixed point of every
    sub-step: after steps in every kernel form it is exactly zero, and so are
    its observables and structure factor (no NaN from the local update's
    0/0 limits at n = |F| = 0)."""
    og = O.Grid(grid[0], grid[1], grid[2], grid[3])
    zero = np.zeros(og.shape, complex)
    for per_launch in (1, 64):
        sim = lib.Sim([grid], P1, dtype=dtype)
        sim.set_option(lib.OPT_STEPS_PER_LAUNCH_1D, per_launch)
        sim.set_fields([zero])
        sim.step(9, 0.02)
        assert np.array_equal(sim.fields()[0], zero), per_launch
        assert np.array_equal(sim.observables(), np.zeros((grid[3], 3)))
        _, mean, _, _, per = sim.structure_factor()
        assert np.array_equal(per, np.zeros_like(per)) and np.all(mean == 0)
        sim.close()


@pytest.mark.parametrize("dtype,tol", [("c128", 1e-13), ("c64", 1e-6)])
@pytest.mark.parametrize("grid", [(1, (4096,), 0.5, 3), (2, (512, 64), 0.5, 2), (3, (32, 16, 64), 0.5, 2)])
def test_zero_time_step_is_the_identity(lib, grid, dtype, tol):
    """dt = 0: every phase is 1, so a step returns the field up to the
    rounding of a forward and an inverse transform per axis."""
    og = O.Grid(grid[0], grid[1], grid[2], grid[3])
    psi0 = random_field(29, og.shape, noise=0.4)
    sim = lib.Sim([grid], P1, dtype=dtype)
    sim.set_fields([psi0])
    sim.step(3, 0.0)
    assert rel(sim.fields()[0], psi0) < tol
    sim.close()


@pytest.mark.parametrize("dtype,tol", [("c128", 1e-13), ("c64", 2e-6)])
def test_out_of_line_sincos_under_divergence(lib, dtype, tol):
    """A sample with one site of huge density shares a wavefront with a normal
    sample (1D, 256 points: two pencils per wavefront).  That site's local
    update takes the out-of-line sine/cosine (the angle c0 n tau is 1e6)
    while the other lanes do not; the samples sharing wavefronts with it must
    still match the oracle step (values held in the lanes that sit out a call
    must survive it)."""
    grid = (1, (256,), 0.5, 4)
    og = O.Grid(1, (256,), 0.5, 4)
    psi0 = random_field(61, og.shape, noise=0.4)
    psi0[1, 1, 100] = 1.0e4  # n = 1e8 at one site of sample 1
    ref = O.strang_step(psi0, 0.01, oparams(P1), og)
    sim = lib.Sim([grid], P1, dtype=dtype)
    sim.set_option(lib.OPT_STEPS_PER_LAUNCH_1D, 1)  # the streaming x-pass, two pencils per wavefront
    sim.set_fields([psi0])
    sim.step(1, 0.01)
    got = sim.fields()[0]
    for s in (0, 2, 3):
        assert rel(got[s], ref[s]) < tol, s
    assert np.all(np.isfinite(got))
