"""Oracle runs of selected Wigner samples, importable by worker processes
(no GPU imports here): the full-size tests compute their FP64 references in
a few CPU processes while the GPU side runs."""
import multiprocessing
from concurrent.futures import ProcessPoolExecutor

from oracle import spin1 as O


def evolve_samples(seed, grid, params, group, which, nsteps, dt):
    """The oracle's init_wigner of samples `which` of group `group` of the
    grid tuple (dim, n, dx, S), advanced nsteps of dt; array [len(which), 3, ...]."""
    og = O.Grid(grid[0], grid[1], grid[2], grid[3])
    p = O.Params(params["c0"], params["c1"], params["q"], params.get("n0", 1.0), params.get("wigner_var", 0.5))
    psi = O.init_wigner(seed, og, p, group=group, samples=which)
    sub = O.Grid(grid[0], grid[1], grid[2], len(which))
    return O.evolve(psi, nsteps, dt, p, sub)


def pool(workers):
    """A process pool that starts its workers fresh (spawn): they never share
    the GPU state of the test process."""
    return ProcessPoolExecutor(max_workers=workers, mp_context=multiprocessing.get_context("spawn"))
