"""spin1_observables_noalloc (partial sums in the library's static device
scratch, no allocation) against spin1_observables (partial sums in the bound
workspace) through the C ABI: two calls in a row, the second on a smaller
input, so that the second call runs over what the first left in the shared
scratch; and a group beyond the scratch's limit is rejected."""
import numpy as np
import pytest
import torch

pytestmark = pytest.mark.gpu

P = dict(c0=1.0, c1=-0.1, q=0.09)


def both(lib, sim, group):
    """(spin1_observables, spin1_observables_noalloc) of one group, [S, 3] each."""
    S = sim.grids[group].samples
    with torch.cuda.stream(sim.stream):
        a = torch.full((S, 3), float("nan"), dtype=torch.float64, device=sim.device)
        b = torch.full((S, 3), float("nan"), dtype=torch.float64, device=sim.device)
    lib.observables(sim.ctx, group, a.data_ptr())
    lib.observables_noalloc(sim.ctx, group, b.data_ptr())
    sim.synchronize()
    return a.cpu().numpy(), b.cpu().numpy()


@pytest.mark.parametrize("dtype", ["c64", "c128"])
def test_noalloc_observables_match_workspace_form(lib, dtype):
    cases = [
        [(3, (32, 16, 64), 0.5, 6)],                       # larger input first
        [(2, (64, 32), 0.5, 3), (1, (128,), 0.5, 2)],      # then smaller ones
    ]
    for groups in cases:
        sim = lib.Sim(groups, P, dtype=dtype)
        sim.init_wigner(77)
        sim.step(3, 0.02)
        for g in range(len(groups)):
            ref, got = both(lib, sim, g)
            assert np.all(np.isfinite(ref))
            # the same kernels in the same order: equal to the last bit
            assert np.array_equal(got, ref), (groups[g], np.max(np.abs(got - ref)))
        sim.close()


def test_noalloc_observables_reject_beyond_scratch(lib):
    # 1024 samples of 16 x 1024: 1M x-pencils of 4 partial sums fill the 32 MiB
    # on their own, the y-pass partials exceed it
    sim = lib.Sim([(2, (16, 1024), 0.5, 1024)], P, dtype="c64")
    sim.init_wigner(5)
    out = torch.empty((1024, 3), dtype=torch.float64, device=sim.device)
    with pytest.raises(lib.Spin1Error) as ei:
        lib.observables_noalloc(sim.ctx, 0, out.data_ptr())
    assert ei.value.code == lib.EUNSUPPORTED
    assert "static scratch" in str(ei.value)
    sim.close()
