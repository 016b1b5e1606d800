"""Throughput of the spin-1 split-step hot path on one MI355X.

Workload: 2D 512 x 512 periodic grid, 64 truncated-Wigner samples, complex64
bulk with FP64 reductions, c0 = 1, c1 = -0.1, q = 0.09 (quench into the
easy-plane phase), dt = 0.02.  One bench step = 100 split steps of every
sample plus one structure-factor snapshot (the snapshot cadence of the
workload), so the default 100 steps are the full 10^4-step run.  The initial
Wigner state is drawn once before the timed region.

Prints one JSON line: site-steps/s (whole job), the roofline entry of the
dominant kernel (algorithmic bytes / live HIP-event time), the complex128
rate and speedup, the FP32-vs-FP64 error after 100 steps, and the oracle's
rate on the host cores.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBPS = 8000.0
WORKLOAD = dict(dim=2, n=(512, 512), dx=0.5, samples=64, dt=0.02, split_steps=100,
                params=dict(c0=1.0, c1=-0.1, q=0.09, n0=1.0, wigner_var=0.5), seed=1002)


def algorithmic_bytes(kind, grid, cbytes):
    """Bytes one launch of a pass kind must move: the 3-component field read
    and written once (48 B per site in complex64, 96 B in complex128)."""
    dim, n, samples = grid
    sites = 1
    for v in n:
        sites *= v
    if kind in ("xpass", "ypass", "zpass", "local"):
        return 2 * 3 * cbytes * sites * samples
    return None


def run_gpu(dtype, steps, warmup, profile):
    import torch
    from paper_2310_03636_amd import spin1

    w = WORKLOAD
    grid = (w["dim"], w["n"], w["dx"], w["samples"])
    sim = spin1.Sim([grid], w["params"], dtype=dtype)
    sim.init_wigner(w["seed"])
    # the library's own autotuner picks the radix / tile variant of each pass
    # (timed on a scratch copy; the bound field is untouched)
    sim.variants = sim.autotune(reps=2)
    torch.cuda.synchronize()

    def bench_step():
        sim.step(w["split_steps"], w["dt"])
        sim.structure_factor_device()

    for _ in range(warmup):
        bench_step()
    torch.cuda.synchronize()
    if profile:
        spin1.profile_read(sim.ctx)  # clear
        spin1.profile_enable(sim.ctx, True)
    # events on the library's stream (the Sim's own stream)
    start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    start.record(sim.stream)
    for _ in range(steps):
        bench_step()
    stop.record(sim.stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    prof = spin1.profile_read(sim.ctx) if profile else None
    if profile:
        spin1.profile_enable(sim.ctx, False)
    ev_ms = start.elapsed_time(stop)
    return sim, wall, ev_ms, prof


def fp32_vs_fp64_error():
    """Error of every complex64 result against the complex128 path (which the
    tests hold to the FP64 oracle within 1e-10) after 100 split steps from the
    same Wigner state, whole workload: the field (relative L2), N, F_z and E
    per sample, and the structure factor (per-sample shell means and their
    sample mean)."""
    import numpy as np
    import torch
    from paper_2310_03636_amd import spin1

    w = WORKLOAD
    grid = (w["dim"], w["n"], w["dx"], w["samples"])
    fields, obs, bins = [], [], []
    for dt in ("c64", "c128"):
        sim = spin1.Sim([grid], w["params"], dtype=dt)
        sim.init_wigner(w["seed"])
        sim.step(w["split_steps"], w["dt"])
        fields.append(sim.field_tensor(0).to(torch.complex128))
        obs.append(sim.observables())
        bins.append(sim.structure_factor_samples())
        sim.close()
    psi = (torch.linalg.vector_norm(fields[0] - fields[1]) / torch.linalg.vector_norm(fields[1])).item()
    del fields
    torch.cuda.empty_cache()
    o32, o64 = obs
    b32, b64 = bins
    m32, m64 = b32.mean(0), b64.mean(0)
    return {
        "psi_rel_l2": psi,
        "N_max_rel": float(np.max(np.abs(o32[:, 0] - o64[:, 0]) / np.abs(o64[:, 0]))),
        "Fz_max_abs_over_N": float(np.max(np.abs(o32[:, 1] - o64[:, 1]) / np.abs(o64[:, 0]))),
        "E_max_rel": float(np.max(np.abs(o32[:, 2] - o64[:, 2]) / np.abs(o64[:, 2]))),
        "S_k_per_sample_rel_l2": float(np.linalg.norm(b32 - b64) / np.linalg.norm(b64)),
        "S_k_mean_max_rel": float(np.max(np.abs(m32 - m64) / np.abs(m64))),
    }


def compensated_tables_run(steps):
    """The main workload with the compensated (hi+lo) FP32 tables in the
    streaming passes instead of the default dithered ones (the precision
    option of the library): rate from the captured graph, per-pass times, and
    the field error against the FP64 path after 100 split steps."""
    import torch
    from paper_2310_03636_amd import spin1

    w = WORKLOAD
    grid = (w["dim"], w["n"], w["dx"], w["samples"])
    ref = spin1.Sim([grid], w["params"], dtype="c128")
    ref.init_wigner(w["seed"])
    ref.step(w["split_steps"], w["dt"])
    ref.synchronize()
    r = ref.psi[0].clone()
    ref.close()
    sim = spin1.Sim([grid], w["params"], dtype="c64")
    sim.set_option(spin1.OPT_FP32_TWIDDLES, spin1.TWIDDLES_COMPENSATED)
    sim.init_wigner(w["seed"])
    variants = sim.autotune(reps=2)
    sim.step(w["split_steps"], w["dt"])
    sim.synchronize()
    err = (torch.linalg.vector_norm(sim.psi[0].to(torch.complex128) - r) / torch.linalg.vector_norm(r)).item()
    del r
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(sim.stream)
    for _ in range(steps):
        sim.step(w["split_steps"], w["dt"])
    e1.record(sim.stream)
    sim.synchronize()
    ms = e0.elapsed_time(e1)
    spin1.profile_read(sim.ctx)
    spin1.profile_enable(sim.ctx, True)
    sim.step(w["split_steps"], w["dt"])
    sim.synchronize()
    prof = spin1.profile_read(sim.ctx)
    spin1.profile_enable(sim.ctx, False)
    sim.close()
    torch.cuda.empty_cache()
    sites = w["n"][0] * w["n"][1] * w["samples"]
    return {"value": sites * w["split_steps"] * steps / (ms / 1e3), "unit": "site-steps/s",
            "err_fp32_vs_fp64_rel_l2_100_split_steps": err, "variants": variants,
            "avg_ms": {k: v[0] / v[1] for k, v in prof.items() if v[1] and k in ("xpass", "ypass")}}


ADJOINT = dict(n=(256, 256), samples=16, steps=500, dt=0.02, every=23, k_cut=1.0,
               params=dict(c0=1.0, c1=-0.1, q=0.09, n0=1.0, wigner_var=0.5), seed=1005)


def adjoint_timing():
    """Reverse mode on the 2D 256 x 256, 16-sample, 500-step workload
    (complex64, checkpoints every 23 steps): forward + backward time over the
    plain forward time."""
    import numpy as np
    import torch
    from paper_2310_03636_amd import spin1

    a = ADJOINT
    grid = (2, a["n"], 0.5, a["samples"])
    sim = spin1.Sim([grid], a["params"], dtype="c64")
    sim.init_wigner(a["seed"])
    psi0 = sim.field_tensor(0).clone()
    sim.step(a["steps"], a["dt"])  # warm up (graphs, tables)
    sim.synchronize()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
    sim.set_fields([psi0])
    ev[0].record(sim.stream)
    sim.step(a["steps"], a["dt"])
    sim.structure_factor_device()
    ev[1].record(sim.stream)
    sim.set_fields([psi0])
    ev[2].record(sim.stream)
    ckpt = sim.forward_ckpt(a["steps"], a["dt"], a["every"])
    bins = sim.structure_factor_samples()
    nb = bins.shape[1]
    kb = np.arange(nb) * 2 * np.pi / (a["n"][0] * 0.5)
    target = bins.mean(0) * 1.05
    dl = np.tile(2 * (bins.mean(0) - target) * (kb < a["k_cut"]) / bins.shape[0], (bins.shape[0], 1))
    grad, gqc = sim.adjoint(a["steps"], a["dt"], a["every"], ckpt, dl)
    ev[3].record(sim.stream)
    sim.synchronize()
    fwd = ev[0].elapsed_time(ev[1])
    tot = ev[2].elapsed_time(ev[3])
    sim.close()
    del ckpt, grad
    torch.cuda.empty_cache()
    return {"workload": "2D 256x256, 16 samples, 500 steps, complex64, checkpoints every 23",
            "forward_ms": fwd, "forward_backward_ms": tot, "ratio": tot / fwd,
            "dL_dq": float(gqc[0]), "dL_dc1": float(gqc[1])}


OTHER_CONFIGS = {
    "1d_256_s4_c128": dict(groups=[(1, (256,), 0.5, 4)], dtype="c128", dt=0.01, steps=1000,
                           params=dict(c0=1.0, c1=-0.1, q=0.09), seed=1001),
    # the paper's production runs: 1D L = 4096 in double precision, 250 runs per GPU
    # (Sec. 2.2; the runs are independent, so they are one batch here)
    "1d_4096_s250_c128": dict(groups=[(1, (4096,), 0.5, 250)], dtype="c128", dt=0.01, steps=200,
                              params=dict(c0=1.0, c1=-0.1, q=0.09), seed=1006),
    "3d_256_s8_c64": dict(groups=[(3, (256, 256, 256), 0.5, 8)], dtype="c64", dt=0.02, steps=20,
                          params=dict(c0=1.0, c1=-0.05, q=0.025), seed=1003, log=True, roofline="3d256_s8"),
    # the paper's own Lie scheme (Eqs. (3)-(5) in its order) on the main workload
    "2d_512_s64_c64_paper_scheme": dict(groups=[(2, (512, 512), 0.5, 64)], dtype="c64", dt=0.02, steps=20,
                                        params=dict(c0=1.0, c1=-0.1, q=0.09), seed=1002, scheme=1),
    # six times the main batch (2.4 GB of field, beyond the 256 MB last-level cache)
    "2d_512_s384_c64": dict(groups=[(2, (512, 512), 0.5, 384)], dtype="c64", dt=0.02, steps=20,
                            params=dict(c0=1.0, c1=-0.1, q=0.09), seed=1002, roofline="2d512_s384"),
    # the main workload in a harmonic trap V(x) (the V_m of Eq. (4)) rising to 4 at the box faces
    "2d_512_s64_c64_trap": dict(groups=[(2, (512, 512), 0.5, 64)], dtype="c64", dt=0.02, steps=20,
                                params=dict(c0=1.0, c1=-0.1, q=0.09), seed=1002, trap=4.0),
    "uneven_c64": dict(groups=[(1, (4096,), 0.5, 128), (2, (256, 256), 0.5, 32), (2, (512, 512), 0.5, 16),
                               (2, (1024, 1024), 0.5, 4)], dtype="c64", dt=0.02, steps=100,
                       params=dict(c0=1.0, c1=-0.1, q=0.09), seed=1004),
}


def other_configs():
    """Site-steps/s of the other workloads (graph replay, autotuned passes):
    three calls of `steps` split steps each, timed together after one call
    that captures the graph."""
    import torch
    from paper_2310_03636_amd import spin1

    out = {}
    for name, c in OTHER_CONFIGS.items():
        sim = spin1.Sim(c["groups"], c["params"], dtype=c["dtype"])
        sim.init_wigner(c["seed"])
        tuned = sim.autotune(reps=2)
        if c.get("scheme"):
            sim.set_option(spin1.OPT_SCHEME, c["scheme"])
        if c.get("trap"):
            import numpy as np
            g = c["groups"][0]
            axes = [(np.arange(n) - 0.5 * n) / (0.5 * n) for n in reversed(g[1])]
            mesh = np.meshgrid(*axes, indexing="ij")
            sim.set_potential(0, c["trap"] * sum(m ** 2 for m in mesh))
        sim.step(c["steps"], c["dt"])  # capture and warm up
        sim.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        reps = 3
        e0.record(sim.stream)
        for _ in range(reps):
            sim.step(c["steps"], c["dt"])
        e1.record(sim.stream)
        sim.synchronize()
        ms = e0.elapsed_time(e1) / reps
        sites = sum(g[3] * int(__import__("math").prod(g[1])) for g in c["groups"])
        obs = sim.observables(0)
        out[name] = {"value": sites * c["steps"] / (ms / 1e3), "unit": "site-steps/s", "steps": c["steps"], "calls": reps,
                     "ms_per_split_step": ms / c["steps"], "dtype": c["dtype"], "variants": tuned,
                     "norm_sample0": float(obs[0, 0])}
        if name == MAIN_2D_NAME:
            out[name]["spin_texture"] = spin_texture_timing(sim)
        if c.get("roofline"):
            # the step passes of the same call timed one by one (direct
            # launches, HIP events on the library's stream)
            spin1.profile_read(sim.ctx)
            spin1.profile_enable(sim.ctx, True)
            sim.step(c["steps"], c["dt"])
            prof = spin1.profile_read(sim.ctx)
            spin1.profile_enable(sim.ctx, False)
            out[name]["whole_step"] = whole_step_entry(out[name]["value"], c["groups"], c["dtype"])
            out[name]["rooflines"] = pass_rooflines(prof, c["groups"], c["dtype"], c["roofline"], tuned)
        if c.get("log"):
            # the same steps with the per-step FP64 (N, F_z, E) log of group 0
            e0.record(sim.stream)
            log = sim.step_observed(c["steps"], c["dt"])
            e1.record(sim.stream)
            sim.synchronize()
            ms_log = e0.elapsed_time(e1)
            n_, fz_, en_ = log[:, :, 0], log[:, :, 1], log[:, :, 2]
            out[name]["logged"] = {
                "value": sites * c["steps"] / (ms_log / 1e3), "unit": "site-steps/s",
                "max_rel_norm_change": float(abs(n_ / n_[0] - 1).max()),
                "max_abs_fz_change_per_norm": float((abs(fz_ - fz_[0]) / n_[0]).max()),
                "max_rel_energy_change": float((abs(en_ / en_[0] - 1)).max())}
        sim.close()
        del sim
        torch.cuda.empty_cache()
    return out


MAIN_2D_NAME = "2d_512_s384_c64"


def spin_texture_timing(sim):
    """Real-space diagnostics of Fig. 1 on a bound group: spin1_spin_texture
    (F_perp, per-row FP64 sums, winding) timed over 10 calls; it reads 24 B
    per site."""
    import torch
    from paper_2310_03636_amd import spin1

    g = sim.grids[0]
    sites = g.samples * g.n[0] * max(g.n[1], 1) * max(g.n[2], 1)
    with torch.cuda.stream(sim.stream):
        out = torch.empty((g.samples, 3), dtype=torch.float64, device=sim.device)
    spin1.spin_texture(sim.ctx, 0, out.data_ptr())
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(sim.stream)
    for _ in range(10):
        spin1.spin_texture(sim.ctx, 0, out.data_ptr())
    e1.record(sim.stream)
    sim.synchronize()
    ms = e0.elapsed_time(e1) / 10
    return {"ms": ms, "GBps_read": sites * 24 / (ms / 1e3) / 1e9}


def full_run():
    """The 2D workload as specified end to end: 10^4 split steps of the
    512 x 512 x 64 batch with the radially binned F_perp structure factor every
    100 steps (101 snapshots, per-sample shell means kept on the device)."""
    import torch
    from paper_2310_03636_amd import spin1

    w = WORKLOAD
    grid = (w["dim"], w["n"], w["dx"], w["samples"])
    sim = spin1.Sim([grid], w["params"], dtype="c64")
    sim.init_wigner(w["seed"])
    sim.autotune(reps=2)
    sim.step(100, w["dt"])  # capture the 100-step graph
    sim.init_wigner(w["seed"])
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(sim.stream)
    snaps = [sim.structure_factor_device()]
    for _ in range(100):
        sim.step(100, w["dt"])
        snaps.append(sim.structure_factor_device())
    e1.record(sim.stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    sites = w["n"][0] * w["n"][1] * w["samples"]
    first, last = snaps[0].mean(0), snaps[-1].mean(0)
    out = {"workload": "2D 512x512, 64 samples, complex64, dt=0.02, 10^4 split steps, S(k) every 100 steps",
           "wall_ms": ms, "value": sites * 10000 / (ms / 1e3), "unit": "site-steps/s",
           "snapshots": len(snaps), "S_k1_first_last": [float(first[1]), float(last[1])]}
    sim.close()
    del snaps
    torch.cuda.empty_cache()
    return out


def oracle_run(job):
    """One oracle run on one host thread (a worker process): sample `which` of
    a workload, Strang steps until `budget_s` seconds have passed or `max_steps`
    are done.  Returns (site-steps, seconds, steps)."""
    dim, n, dx, samples, params, dt, seed, which, budget_s, max_steps = job
    import numpy as np
    from oracle import spin1 as O

    g = O.Grid(dim, n, dx, samples)
    p = O.Params(**params)
    psi = O.init_wigner(seed, g, p, samples=which)
    sub = O.Grid(dim, n, dx, len(which))
    t0 = time.perf_counter()
    k = 0
    while k < max_steps:
        psi = O.strang_step(psi, dt, p, sub)
        k += 1
        if time.perf_counter() - t0 >= budget_s:
            break
    el = time.perf_counter() - t0
    assert np.isfinite(psi).all()
    return sub.sites * len(which) * k, el, k


def host_workers():
    """Worker processes for the oracle baseline: the cores this process may
    run on, at most 16 (the host share of one GPU on the benchmark machines)."""
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(n, 16))


UNEVEN_GROUPS = [(1, (4096,), 0.5, 128), (2, (256, 256), 0.5, 32), (2, (512, 512), 0.5, 16), (2, (1024, 1024), 0.5, 4)]


def oracle_baseline(budget_s=12.0, with_3d=False):
    """The FP64 oracle as it stands, on the host cores, in worker processes of
    one thread each (spawned, with the BLAS/OpenMP thread counts set to 1):
    (a) the main workload, one 512 x 512 sample per worker, steps until
    budget_s; the rate is the sum of the workers' own rates (their timed loops
    overlap); (b) the same sample on one thread alone; (c) the 1D 256 x 4
    double-precision workload in full (1000 steps) on one thread; (d) one
    sample of each group of the uneven batch, one worker each, steps until a
    third of budget_s (at least one step); (e) with with_3d, one 256^3 sample
    for one step (minutes of CPU time, so not in the default run)."""
    import multiprocessing
    from concurrent.futures import ProcessPoolExecutor

    w = WORKLOAD
    workers = host_workers()
    saved = {k: os.environ.get(k) for k in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS")}
    for k in saved:
        os.environ[k] = "1"
    try:
        ctx = multiprocessing.get_context("spawn")
        main_job = lambda s, budget: (w["dim"], w["n"], w["dx"], w["samples"], w["params"], w["dt"], w["seed"], [s],
                                      budget, 10 ** 9)
        with ProcessPoolExecutor(max_workers=workers, mp_context=ctx) as ex:
            res = list(ex.map(oracle_run, [main_job(s % w["samples"], budget_s) for s in range(workers)]))
        with ProcessPoolExecutor(max_workers=1, mp_context=ctx) as ex:
            one = ex.submit(oracle_run, main_job(0, budget_s)).result()
            c1 = ex.submit(oracle_run, (1, (256,), 0.5, 4, dict(c0=1.0, c1=-0.1, q=0.09), 0.01, 1001,
                                        [0, 1, 2, 3], 10 ** 9, 1000)).result()
        uneven_params = dict(c0=1.0, c1=-0.1, q=0.09)
        with ProcessPoolExecutor(max_workers=min(workers, len(UNEVEN_GROUPS)), mp_context=ctx) as ex:
            c4 = list(ex.map(oracle_run, [(g[0], g[1], g[2], g[3], uneven_params, 0.02, 1004, [0], budget_s / 3,
                                           10 ** 9) for g in UNEVEN_GROUPS]))
        c3 = None
        if with_3d:
            with ProcessPoolExecutor(max_workers=1, mp_context=ctx) as ex:
                c3 = ex.submit(oracle_run, (3, (256, 256, 256), 0.5, 8, dict(c0=1.0, c1=-0.05, q=0.025), 0.02, 1003,
                                            [0], 0.0, 1)).result()
    finally:
        for k, v in saved.items():
            if v is None:
                os.environ.pop(k, None)
            else:
                os.environ[k] = v
    rate = sum(r[0] / r[1] for r in res)
    return {"value": rate, "unit": "site-steps/s", "cores": workers, "kind": "oracle",
            "sample": "FP64 numpy oracle on the 512x512 workload: %d worker processes of one thread, one Wigner "
                      "sample each, %d-%d Strang steps in about %.0f s each; rate = sum of the workers' rates"
                      % (workers, min(r[2] for r in res), max(r[2] for r in res), budget_s),
            "single_thread": {"value": one[0] / one[1], "unit": "site-steps/s", "steps": one[2],
                              "seconds": one[1]},
            "config_1d_256_s4_c128_full": {"value": c1[0] / c1[1], "unit": "site-steps/s", "steps": c1[2],
                                            "seconds": c1[1], "threads": 1},
            # the whole batch's site-steps over the core-seconds one sample of
            # each group takes, per sample-step in proportion to its group
            "config_uneven_one_sample_per_group": {
                "value": sum(g[3] * r[0] / r[2] for g, r in zip(UNEVEN_GROUPS, c4))
                / sum(g[3] * r[1] / r[2] for g, r in zip(UNEVEN_GROUPS, c4)),
                "unit": "site-steps/s per core", "groups": [
                    {"grid": list(g[1]), "steps": r[2], "seconds": r[1], "value": r[0] / r[1]}
                    for g, r in zip(UNEVEN_GROUPS, c4)]},
            "config_3d_256_s8_one_sample_one_step": (
                {"value": c3[0] / c3[1], "unit": "site-steps/s", "steps": c3[2], "seconds": c3[1], "threads": 1}
                if c3 else "not run by default (one oracle step of a 256^3 sample takes minutes); --cpu-3d runs it")}


PROFILE_WORKLOADS = {
    "2d512_s64": ([(2, (512, 512), 0.5, 64)], dict(c0=1.0, c1=-0.1, q=0.09), 0.02),
    "2d512_s384": ([(2, (512, 512), 0.5, 384)], dict(c0=1.0, c1=-0.1, q=0.09), 0.02),
    "3d256_s8": ([(3, (256, 256, 256), 0.5, 8)], dict(c0=1.0, c1=-0.05, q=0.025), 0.02),
    "uneven": ([(1, (4096,), 0.5, 128), (2, (256, 256), 0.5, 32), (2, (512, 512), 0.5, 16),
                (2, (1024, 1024), 0.5, 4)], dict(c0=1.0, c1=-0.1, q=0.09), 0.02),
    "1d4096_s250": ([(1, (4096,), 0.5, 250)], dict(c0=1.0, c1=-0.1, q=0.09), 0.01),
    "2d512_s64_c128": ([(2, (512, 512), 0.5, 64)], dict(c0=1.0, c1=-0.1, q=0.09), 0.02),
}
PROFILE_DTYPE = {"1d4096_s250": "c128", "2d512_s64_c128": "c128"}


def profile_pass(workload="2d512_s64"):
    """Short run for hardware-counter passes: a few split steps of a workload
    (direct launches, variants chosen by the autotuner as in the timed run),
    then a plain device copy of 402.65 MB (read and written once) as the
    calibration kernel of known traffic.  A small fill kernel before the
    steps and the fill of the copy's source after them bracket the steps in
    a kernel trace."""
    import torch
    from paper_2310_03636_amd import spin1

    groups, params, dt = PROFILE_WORKLOADS[workload]
    sim = spin1.Sim(groups, dict(params, n0=1.0, wigner_var=0.5), dtype=PROFILE_DTYPE.get(workload, "c64"))
    sim.init_wigner(1002)
    variants = sim.autotune(reps=2)  # the same choice as the timed run
    sim.set_option(spin1.OPT_GRAPHS, 0)
    torch.zeros(16, device="cuda")  # a fill kernel that marks the start of the steps in a trace
    torch.cuda.synchronize()
    sim.step(3, dt)
    sim.synchronize()
    sim.close()
    print("profile pass variants: %s" % json.dumps(variants), flush=True)
    n = 64 * 512 * 512 * 3  # complex64 values of one field: 402.65 MB
    src = torch.ones(n, dtype=torch.complex64, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    print("profile pass done: copy of %d bytes" % (n * 8), flush=True)


def pass_bytes(groups, dtype):
    """Algorithmic bytes of one step pass over every group: the 3-component
    field read and written once."""
    import math
    cb = 16 if dtype == "c128" else 8
    return 2 * 3 * cb * sum(g[3] * math.prod(g[1]) for g in groups)


def whole_step_entry(value, groups, dtype):
    """The whole split step against the HBM roofline: site-steps/s times the
    pass-model bytes of a site-step (one field read + write per axis pass)."""
    import math
    cb = 16 if dtype == "c128" else 8
    sites = sum(g[3] * math.prod(g[1]) for g in groups)
    bytes_per_site_step = sum(g[3] * math.prod(g[1]) * g[0] for g in groups) * 2 * 3 * cb / sites
    achieved = value * bytes_per_site_step / 1e9
    return {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBPS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBPS, "bytes_per_site_step": bytes_per_site_step}


def copy_reference(nbytes, reps=10):
    """Two plain streaming kernels that read and write `nbytes` in all, the
    practical ceilings beside the published peak: a device copy (torch's
    copy_) between two buffers of half of `nbytes` each, and an in-place
    scaling (torch's mul_) of one such buffer, which reads and writes the same
    addresses as the step passes do.  Timed with HIP events on a stream of
    its own (default priority) after three untimed launches each; `achieved`
    is the faster of the two."""
    import torch

    n = nbytes // 2 // 8  # complex64 elements of each buffer
    src = torch.ones(n, dtype=torch.complex64, device="cuda")
    dst = torch.empty_like(src)
    st = torch.cuda.Stream()

    def timed(fn):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        with torch.cuda.stream(st):
            for _ in range(3):
                fn()
            e0.record(st)
            for _ in range(reps):
                fn()
            e1.record(st)
        st.synchronize()
        return e0.elapsed_time(e1) / reps

    ms_copy = timed(lambda: dst.copy_(src))
    ms_inplace = timed(lambda: src.mul_(1.0000001))
    del src, dst
    torch.cuda.empty_cache()
    ms = min(ms_copy, ms_inplace)
    return {"kernel": "device copy (torch copy_) and in-place scaling (torch mul_) of a buffer the size of the field",
            "bytes_per_launch": nbytes, "avg_launch_ms": ms, "achieved": nbytes / (ms / 1e3) / 1e9, "unit": "GB/s",
            "copy_GBps": nbytes / (ms_copy / 1e3) / 1e9, "inplace_GBps": nbytes / (ms_inplace / 1e3) / 1e9,
            "launches": reps}


def pass_rooflines(prof, groups, dtype, workload, variants=None):
    """Roofline entry of every step pass kind of a one-group workload:
    algorithmic bytes per launch over the live average launch time, and the
    same bytes moved by a plain device copy for comparison."""
    out = {}
    nbytes = pass_bytes(groups, dtype)
    cref = copy_reference(nbytes)
    for kind in ("xpass", "ypass", "zpass"):
        total, n = prof.get(kind, (0.0, 0))
        if not n:
            continue
        avg = total / n
        achieved = nbytes / (avg / 1e3) / 1e9
        out[kind] = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBPS, "avg_launch_ms": avg, "launches": n,
                     "algorithmic_bytes_per_launch": nbytes,
                     "traffic": measured_traffic(kind, workload, variant_of(kind, groups, variants, dtype)),
                     "frac_of_copy": achieved / cref["achieved"]}
    out["copy_reference"] = cref
    return out


def kernel_source_hash():
    import hashlib
    h = hashlib.sha256()
    for f in ("kernels_xstream.hip", "kernels_sstream.hip", "pass_common.hpp", "device_math.hpp"):
        with open(os.path.join(ROOT, "paper_2310_03636_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


TRAFFIC_FILES = {"2d512_s64": "traffic_xpass_ypass_2d512_s64.md",
                 "2d512_s64_c128": "traffic_xpass_ypass_2d512_s64_c128.md",
                 "2d512_s384": "traffic_xpass_ypass_2d512_s384.md",
                 "3d256_s8": "traffic_xpass_ypass_zpass_3d256_s8.md"}


def variant_of(kind, groups, variants, dtype="c64"):
    """The autotuned variant of a pass kind on the first group (None if unknown)."""
    axis = {"xpass": 0, "ypass": 1, "zpass": 2}[kind]
    g = groups[0]
    if axis >= len(g[1]):
        return None
    return (variants or {}).get("gfx950/%s/%d/%d" % (dtype, 0 if axis == 0 else 1, g[1][axis]))


def summary_lines(path, tag):
    """{(kind, variant): fields} of the machine-readable `tag:` lines of a
    committed profile summary."""
    rec = {}
    if os.path.isfile(path):
        for line in open(path):
            if line.startswith(tag + ":"):
                parts = dict(kv.split("=") for kv in line.split()[1:])
                rec[(parts["kind"], int(parts.get("variant", -1)))] = parts
    return rec


def measured_traffic(kernel, workload="2d512_s64", variant=None):
    """HBM bytes per launch of `kernel` (of the given autotuned variant) on
    `workload` from the committed counter summary, or None when the summary
    has no such line or the kernel sources changed since the counters were
    taken."""
    rec = summary_lines(os.path.join(ROOT, "profiles", TRAFFIC_FILES.get(workload, "")), "traffic")
    r = rec.get((kernel, variant if variant is not None else 0))
    if not r or r.get("source") != kernel_source_hash():
        return None
    return float(r["bytes"])


VALU_PEAK = 256 * 4 * 2.4e9 / 4  # wave64 FP32 VALU instructions per second (non-packed)


def measured_valu(kernel, variant=None):
    """VALU wavefront instructions per launch of `kernel` (of the given
    autotuned variant) from the committed counter summary, or None when the
    summary has no such line or the kernel sources changed since."""
    rec = summary_lines(os.path.join(ROOT, "profiles", "valu_xpass_ypass_2d512_s64.md"), "valu")
    r = rec.get((kernel, variant if variant is not None else 0))
    if not r or r.get("source") != kernel_source_hash():
        return None
    return float(r["instr"])


def valu_entry(kernel, avg_ms, variant=None):
    """The issue side of the same launch: counted VALU instructions per launch
    over the live launch time, against the non-packed FP32 issue ceiling."""
    instr = measured_valu(kernel, variant)
    if instr is None:
        return None
    achieved = instr / (avg_ms / 1e3)
    return {"instructions_per_launch": instr, "achieved": achieved, "peak": VALU_PEAK, "unit": "wave-instr/s",
            "frac": achieved / VALU_PEAK}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--fp64-steps", type=int, default=10)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-budget", type=float, default=12.0)
    ap.add_argument("--cpu-3d", action="store_true",
                    help="also time one oracle step of one 256^3 sample (minutes of CPU time)")
    ap.add_argument("--profile-pass", nargs="?", const="2d512_s64", default=None,
                    choices=sorted(PROFILE_WORKLOADS),
                    help="short run of a workload for rocprofv3 counter passes (no JSON line)")
    args = ap.parse_args()
    if args.profile_pass:
        profile_pass(args.profile_pass)
        return
    if args.gpus != 1:
        print("bench.py measures one GPU: the Wigner samples are independent, so N GPUs would each run "
              "this same single-GPU workload on their own share; --gpus %d is not run."
              % args.gpus, file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2310_03636_amd import spin1
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    spin1.load()

    w = WORKLOAD
    sites = w["n"][0] * w["n"][1]
    per_step_site_steps = w["samples"] * sites * w["split_steps"]
    grid = (w["dim"], w["n"], w["samples"])
    grid4 = (w["dim"], w["n"], w["dx"], w["samples"])

    # the timed region as the library runs it by default: each call's launches
    # replayed from a captured HIP graph
    simg, wall, evg_ms, _ = run_gpu("c64", args.steps, args.warmup, profile=False)
    value = per_step_site_steps * args.steps / (evg_ms / 1e3)
    variants = simg.variants
    simg.close()
    del simg
    torch.cuda.empty_cache()
    # the same steps as direct launches, each kernel timed by its own begin and
    # end (the library's profiling mode): the per-kernel times of the rooflines
    sim, wall_direct, ev_ms, prof = run_gpu("c64", args.steps, args.warmup, profile=True)
    value_direct = per_step_site_steps * args.steps / (ev_ms / 1e3)
    sim.close()
    del sim
    torch.cuda.empty_cache()

    # dominant kernel and its live average duration
    kinds = {k: v for k, v in prof.items() if v[1] > 0}
    dom = max(kinds, key=lambda k: kinds[k][0])
    dom_ms, dom_n = kinds[dom]
    dom_avg_ms = dom_ms / dom_n
    dom_bytes = algorithmic_bytes(dom, grid, 8)
    achieved = dom_bytes / (dom_avg_ms / 1e3) / 1e9 if dom_bytes else None
    cref = copy_reference(dom_bytes) if dom_bytes else None

    sim64, wall64, ev64, _ = run_gpu("c128", args.fp64_steps, 1, profile=False)
    value64 = per_step_site_steps * args.fp64_steps / (ev64 / 1e3)
    variants64 = sim64.variants
    sim64.close()
    del sim64
    torch.cuda.empty_cache()
    # the double-precision passes timed one by one (two profiled steps)
    simp, _, _, prof64 = run_gpu("c128", 2, 0, profile=True)
    simp.close()
    del simp
    torch.cuda.empty_cache()
    rooflines64 = pass_rooflines(prof64, [grid4], "c128", "2d512_s64_c128", variants64)

    err = fp32_vs_fp64_error()
    compensated = compensated_tables_run(args.steps)
    adj = adjoint_timing()
    others = other_configs()
    full = full_run()

    cpu = None
    if not args.no_cpu_baseline:
        cpu = oracle_baseline(args.cpu_budget, with_3d=args.cpu_3d)

    line = {
        "metric": "site-steps/s, spin-1 split-step (FP32 vs FP64 at stated err); HBM GB/s",
        "value": value,
        "unit": "site-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": evg_ms / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic: seeded truncated-Wigner polar state (Philox4x64-10), no dataset",
        "config": {"workload": "2D 512x512 periodic spin-1 GPE, 64 Wigner samples, complex64 bulk + FP64 "
                               "reductions, dt=0.02; step = 100 split steps + 1 structure-factor snapshot",
                   "grid": list(w["n"]), "samples": w["samples"], "split_steps_per_step": w["split_steps"],
                   "dt": w["dt"], "params": w["params"]},
        "roofline": {"bound": "hbm", "kernel": dom, "scope": "the dominant kernel alone, each launch timed by its own begin and end in a profiled run of the same steps",
                     "achieved": achieved, "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBPS if achieved else None,
                     "traffic": measured_traffic(dom, "2d512_s64", variant_of(dom, [grid4], variants)),
                     "avg_launch_ms": dom_avg_ms, "algorithmic_bytes_per_launch": dom_bytes,
                     "valu": valu_entry(dom, dom_avg_ms, variant_of(dom, [grid4], variants)), "copy_reference": cref,
                     "frac_of_copy": achieved / cref["achieved"] if cref else None},
        # the whole split step of the timed region, and of the profiled direct launches
        "roofline_whole_step": dict(whole_step_entry(value, [grid4], "c64"),
                                    frac_direct_launches=whole_step_entry(value_direct, [grid4], "c64")["frac"]),
        # working sets beyond the 256 MB last-level cache: every pass of the
        # 2.4 GB 2D batch and of the 3 GiB 3D batch
        "rooflines_cache_cold": {
            "2d512_s384": {"whole_step": others["2d_512_s384_c64"]["whole_step"],
                           "passes": others["2d_512_s384_c64"]["rooflines"]},
            "3d256_s8": {"whole_step": others["3d_256_s8_c64"]["whole_step"],
                         "passes": others["3d_256_s8_c64"]["rooflines"]}},
        "autotuned_variants": variants,
        "kernels_ms": {k: {"total_ms": v[0], "launches": v[1], "avg_ms": v[0] / v[1]} for k, v in kinds.items()},
        "direct_launches_profiled": {"value": value_direct, "unit": "site-steps/s", "ms_per_step": ev_ms / args.steps},
        "fp64": {"value": value64, "unit": "site-steps/s", "steps": args.fp64_steps,
                 "ms_per_step": ev64 / args.fp64_steps, "variants": variants64,
                 "whole_step": whole_step_entry(value64, [grid4], "c128"), "rooflines": rooflines64},
        "speedup_fp32_vs_fp64": value / value64,
        "adjoint": adj,
        "other_configs": others,
        "full_run": full,
        "err_fp32_vs_fp64_rel_l2_100_split_steps": err["psi_rel_l2"],
        "fp32_errors_vs_fp64_100_split_steps": err,
        "fp32_compensated_tables": compensated,
        "wall_s": wall,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line))


if __name__ == "__main__":
    main()
