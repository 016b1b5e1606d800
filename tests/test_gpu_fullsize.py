"""The benchmark workloads at their full sizes, in the launch configuration
the benchmark times (autotuned variants, captured step graphs): sampled Wigner
runs against the oracle run on those samples alone (the runs are independent),
and properties that hold at any size where the oracle would take minutes.

Tolerances: after 100 split steps, relative L2 per checked sample, 1e-10 for
complex128 and 1e-4 for complex64 (the stated tolerances); after two split
steps, complex64 within 1e-5 (one step holds 2e-6 in the small-size tests)."""
import numpy as np
import pytest

from oracle import spin1 as O
from tests import oracle_jobs

pytestmark = pytest.mark.gpu

P2 = dict(c0=1.0, c1=-0.1, q=0.09, n0=1.0, wigner_var=0.5)


def oparams(p):
    return O.Params(p["c0"], p["c1"], p["q"], p["n0"], p["wigner_var"])


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def oracle_samples(seed, g, p, group, which, nsteps, dt):
    og = O.Grid(g[0], g[1], g[2], g[3])
    psi = O.init_wigner(seed, og, oparams(p), group=group, samples=which)
    sub = O.Grid(g[0], g[1], g[2], len(which))
    return O.evolve(psi, nsteps, dt, oparams(p), sub)


def test_2d_512_64_samples_full_size(lib):
    g = (2, (512, 512), 0.5, 64)
    sim = lib.Sim([g], P2, dtype="c64")
    sim.init_wigner(1002)
    sim.autotune(reps=1)
    sim.step(2, 0.02)
    which = [0, 37, 63]
    got = sim.field_tensor(0)[which].cpu().numpy().astype(np.complex128)
    ref = oracle_samples(1002, g, P2, 0, which, 2, 0.02)
    for i, s in enumerate(which):
        assert rel(got[i], ref[i]) < 1e-5, s


def test_uneven_batch_full_size(lib):
    """The four groups of the uneven workload in one plan (grouped x-pass,
    1D group on the second stream): first and last sample of every group."""
    groups = [(1, (4096,), 0.5, 128), (2, (256, 256), 0.5, 32), (2, (512, 512), 0.5, 16),
              (2, (1024, 1024), 0.5, 4)]
    sim = lib.Sim(groups, P2, dtype="c64")
    sim.init_wigner(1004)
    sim.autotune(reps=1)
    sim.step(2, 0.02)
    for gi, g in enumerate(groups):
        which = [0, g[3] - 1]
        got = sim.field_tensor(gi)[which].cpu().numpy().astype(np.complex128)
        ref = oracle_samples(1004, g, P2, gi, which, 2, 0.02)
        for i, s in enumerate(which):
            assert rel(got[i], ref[i]) < 1e-5, (gi, s)


def test_3d_256_8_samples_full_size_invariants(lib):
    """256^3 x 8 (3 GiB of complex64): one oracle step takes minutes per
    sample, so the full-size check is by properties: norm and F_z per sample
    conserved, and 10 steps forward then 10 back return the initial state
    (the map is time-reversible)."""
    p3 = dict(c0=1.0, c1=-0.05, q=0.025, n0=1.0, wigner_var=0.5)
    g = (3, (256, 256, 256), 0.5, 8)
    sim = lib.Sim([g], p3, dtype="c64")
    sim.init_wigner(1003)
    sim.autotune(reps=1)
    psi0 = sim.field_tensor(0).clone()
    obs0 = sim.observables()
    sim.step(10, 0.02)
    obs1 = sim.observables()
    assert np.allclose(obs1[:, 0], obs0[:, 0], rtol=1e-5)
    assert np.allclose(obs1[:, 1], obs0[:, 1], atol=1e-5 * obs0[:, 0].max())
    sim.step(10, -0.02)
    import torch
    err = (torch.linalg.vector_norm(sim.field_tensor(0) - psi0) / torch.linalg.vector_norm(psi0)).item()
    assert err < 1e-4, err


def test_2d_512_384_samples_full_size(lib):
    """The 2.4 GB batch of 384 samples of 512^2 (beyond the last-level cache:
    non-temporal field stores) in the benchmark's launch configuration, two
    split steps; its first and last samples against the oracle run on them."""
    g = (2, (512, 512), 0.5, 384)
    sim = lib.Sim([g], P2, dtype="c64")
    sim.init_wigner(1002)
    sim.autotune(reps=1)
    sim.step(2, 0.02)
    f = sim.field_tensor(0)
    got = [f[s].cpu().numpy().astype(np.complex128) for s in (0, 383)]
    sim.close()
    ref = oracle_samples(1002, g, P2, 0, [0, 383], 2, 0.02)
    for k in range(2):
        assert rel(got[k], ref[k]) < 1e-5, k


@pytest.mark.timeout(600)
def test_3d_256_8_samples_full_size_last_sample_against_oracle(lib):
    """One split step of the full 256^3 x 8 batch in the benchmark's launch
    configuration (autotuned variants, captured graph); its last sample
    against the oracle run on that sample alone (16.8M sites, about a minute
    of CPU)."""
    p3 = dict(c0=1.0, c1=-0.05, q=0.025, n0=1.0, wigner_var=0.5)
    g = (3, (256, 256, 256), 0.5, 8)
    sim = lib.Sim([g], p3, dtype="c64")
    sim.init_wigner(1003)
    sim.autotune(reps=1)
    sim.step(1, 0.02)
    got = sim.field_tensor(0)[7].cpu().numpy().astype(np.complex128)
    sim.close()
    ref = oracle_samples(1003, g, p3, 0, [7], 1, 0.02)[0]
    assert rel(got, ref) < 1e-5


def test_1d_4096_250_runs_fp64_full_size(lib):
    """The paper's production shape: 250 runs of 1D L = 4096 in double precision."""
    g = (1, (4096,), 0.5, 250)
    sim = lib.Sim([g], P2, dtype="c128")
    sim.init_wigner(1006)
    sim.step(3, 0.01)
    which = [0, 123, 249]
    got = sim.field_tensor(0)[which].cpu().numpy()
    ref = oracle_samples(1006, g, P2, 0, which, 3, 0.01)
    for i, s in enumerate(which):
        assert rel(got[i], ref[i]) < 1e-12, s


@pytest.mark.timeout(600)
def test_paper_scheme_2d_512_64_samples_full_size(lib):
    """The paper's own Lie scheme (Eqs. (3)-(5)) on the 512^2 x 64 batch in the
    benchmark's launch configuration for that scheme (autotuned variants,
    captured graph): 5 steps of dt = 0.02 in one call, the first and last
    sample against the oracle's literal steps run on those samples alone."""
    import torch

    g = (2, (512, 512), 0.5, 64)
    which = [0, 63]
    og = O.Grid(2, (512, 512), 0.5, 64)
    psi = O.init_wigner(1002, og, oparams(P2), group=0, samples=which)
    sub = O.Grid(2, (512, 512), 0.5, len(which))
    ref = O.evolve(psi, 5, 0.02, oparams(P2), sub, step=O.paper_step)
    for dtype, tol in (("c128", 1e-12), ("c64", 2e-5)):
        sim = lib.Sim([g], P2, dtype=dtype)
        sim.init_wigner(1002)
        sim.autotune(reps=1)
        sim.set_option(lib.OPT_SCHEME, lib.SCHEME_PAPER)
        sim.step(5, 0.02)
        got = sim.field_tensor(0)[which].to(torch.complex128).cpu().numpy()
        sim.close()
        for i, s in enumerate(which):
            assert rel(got[i], ref[i]) < tol, (dtype, s)


@pytest.mark.timeout(600)
def test_1d_4096_250_runs_100_steps_against_oracle(lib):
    """The paper's 1D production shape in the benchmark's launch
    configuration (up to 64 steps per launch with the samples on chip,
    captured graph): 100 split steps of dt = 0.01, first, middle and last
    sample against the oracle run on those samples alone, complex128 within
    1e-10 and complex64 within 1e-4."""
    import torch

    g = (1, (4096,), 0.5, 250)
    which = [0, 123, 249]
    ref = oracle_samples(1006, g, P2, 0, which, 100, 0.01)
    for dtype, tol in (("c128", 1e-10), ("c64", 1e-4)):
        sim = lib.Sim([g], P2, dtype=dtype)
        sim.init_wigner(1006)
        sim.autotune(reps=1)
        sim.step(100, 0.01)
        got = sim.field_tensor(0)[which].to(torch.complex128).cpu().numpy()
        sim.close()
        errs = [rel(got[i], ref[i]) for i in range(len(which))]
        print("1D 4096 x 250, 100 steps, %s: %s" % (dtype, ", ".join("%.2e" % e for e in errs)))
        assert max(errs) < tol, (dtype, errs)


@pytest.mark.timeout(900)
def test_2d_512_64_samples_100_steps_against_oracle(lib):
    """The headline workload (512^2 x 64) in the benchmark's launch
    configuration, 100 split steps of dt = 0.02 in one call (autotuned
    variants, captured graph), complex128 and complex64 from the same Wigner
    state: the last sample against the oracle run on that sample alone."""
    import torch

    g = (2, (512, 512), 0.5, 64)
    with oracle_jobs.pool(1) as ex:
        job = ex.submit(oracle_jobs.evolve_samples, 1002, g, P2, 0, [63], 100, 0.02)
        got = {}
        for dtype in ("c128", "c64"):
            sim = lib.Sim([g], P2, dtype=dtype)
            sim.init_wigner(1002)
            sim.autotune(reps=1)
            sim.step(100, 0.02)
            got[dtype] = sim.field_tensor(0)[63].to(torch.complex128).cpu().numpy()
            sim.close()
            del sim
            torch.cuda.empty_cache()
        ref = job.result()[0]
    e128, e64 = rel(got["c128"], ref), rel(got["c64"], ref)
    print("512^2 x 64, sample 63, 100 steps: complex128 %.2e, complex64 %.2e" % (e128, e64))
    assert e128 < 1e-10
    assert e64 < 1e-4


@pytest.mark.timeout(900)
def test_uneven_batch_against_oracle_long(lib):
    """The uneven four-group workload in one plan, complex64, the benchmark's
    launch configuration: the first sample of the 1D 4096 and 2D 256^2 groups
    after 100 split steps, and of the 1024^2 group after 20 (its oracle steps
    cost seconds each), against the oracle run on those samples alone."""
    import torch

    groups = [(1, (4096,), 0.5, 128), (2, (256, 256), 0.5, 32), (2, (512, 512), 0.5, 16),
              (2, (1024, 1024), 0.5, 4)]
    checks = {0: 100, 1: 100, 3: 20}
    with oracle_jobs.pool(len(checks)) as ex:
        jobs = {gi: ex.submit(oracle_jobs.evolve_samples, 1004, groups[gi], P2, gi, [0], n, 0.02)
                for gi, n in checks.items()}
        got = {}
        for nsteps in sorted(set(checks.values())):
            sim = lib.Sim(groups, P2, dtype="c64")
            sim.init_wigner(1004)
            sim.autotune(reps=1)
            sim.step(nsteps, 0.02)
            for gi, n in checks.items():
                if n == nsteps:
                    got[gi] = sim.field_tensor(gi)[0].to(torch.complex128).cpu().numpy()
            sim.close()
            del sim
            torch.cuda.empty_cache()
        errs = {gi: rel(got[gi], jobs[gi].result()[0]) for gi in checks}
    print("uneven batch, complex64, first samples: %s" % ", ".join(
        "group %d (%d steps) %.2e" % (gi, checks[gi], e) for gi, e in errs.items()))
    for gi, e in errs.items():
        assert e < 1e-4, (gi, e)
