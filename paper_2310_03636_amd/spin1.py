"""Python binding of the spin-1 split-step C ABI (include/spin1.h).

Argument marshalling only: every step of the method runs in the HIP kernels of
``libspin1.so``.  The functions below carry the C names without the
``spin1_`` prefix and raise ``Spin1Error`` on a negative status.  ``Sim``
bundles the device buffers (torch tensors used purely as device memory and a
stream) for the common case.

There is no CPU fallback: if the library is missing, loading fails loudly.
"""
import ctypes
import math
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libspin1.so")

C64, C128 = 0, 1
OK, EINVAL, EUNSUPPORTED, EHIP, ESTATE, ENOMEM = 0, -1, -2, -3, -4, -5

FUNCTIONS = [
    "spin1_create", "spin1_destroy", "spin1_check_grid", "spin1_field_bytes",
    "spin1_workspace_bytes", "spin1_num_bins", "spin1_bin_counts", "spin1_bind",
    "spin1_init_wigner", "spin1_init_wigner_shard", "spin1_set_params", "spin1_set_potential", "spin1_step", "spin1_sync_field",
    "spin1_structure_factor",
    "spin1_observables", "spin1_observables_noalloc", "spin1_step_observed", "spin1_transverse_spin", "spin1_spin_texture",
    "spin1_local_update", "spin1_set_option", "spin1_profile_enable",
    "spin1_profile_read", "spin1_adjoint_workspace_bytes", "spin1_forward_ckpt", "spin1_adjoint",
    "spin1_num_variants", "spin1_autotune", "spin1_get_variant", "spin1_set_variant", "spin1_last_error",
]

OPT_GRAPHS, OPT_GRAPH_MAX_STEPS, OPT_STEPS_PER_LAUNCH_1D, OPT_GROUPED_X, OPT_SCHEME = 0, 1, 2, 3, 4
SCHEME_STRANG, SCHEME_PAPER = 0, 1
OPT_FP32_TWIDDLES = 5
OPT_CONCURRENT_GROUPS = 6
OPT_1D_KERNEL = 7
OPT_STREAMING_STORES = 8
STORES_AUTO, STORES_CACHED, STORES_STREAMING = 0, 1, 2
TWIDDLES_COMPENSATED, TWIDDLES_DITHERED = 0, 1

KERNEL_KINDS = ["xpass", "ypass", "zpass", "local", "spectrum", "shells", "observables", "other"]


class Grid(ctypes.Structure):
    _fields_ = [("dim", ctypes.c_int32), ("n", ctypes.c_int32 * 3), ("dx", ctypes.c_double),
                ("samples", ctypes.c_int32)]


class Params(ctypes.Structure):
    _fields_ = [("c0", ctypes.c_double), ("c1", ctypes.c_double), ("q", ctypes.c_double),
                ("n0", ctypes.c_double), ("wigner_var", ctypes.c_double)]


class Spin1Error(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("spin1 error %d: %s" % (code, msg))
        self.code = code


_lib = None


def load():
    """Load libspin1.so (built by ``__graft_entry__.build()``)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError("libspin1.so not found at %s: build it first (python -c "
                          "'import __graft_entry__; __graft_entry__.build()')" % LIB_PATH)
    lib = ctypes.CDLL(LIB_PATH)
    vp, i32, i64, f64, sz = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double, ctypes.c_size_t
    gp, pp = ctypes.POINTER(Grid), ctypes.POINTER(Params)
    sig = {
        "spin1_create": (ctypes.c_int, [ctypes.POINTER(vp), i32, vp]),
        "spin1_destroy": (ctypes.c_int, [vp]),
        "spin1_check_grid": (ctypes.c_int, [gp, i32]),
        "spin1_field_bytes": (sz, [gp, i32]),
        "spin1_workspace_bytes": (sz, [gp, i32, i32]),
        "spin1_num_bins": (i32, [gp]),
        "spin1_bin_counts": (ctypes.c_int, [gp, ctypes.POINTER(i64)]),
        "spin1_bind": (ctypes.c_int, [vp, gp, i32, pp, ctypes.POINTER(vp), vp]),
        "spin1_init_wigner": (ctypes.c_int, [vp, ctypes.c_uint64, gp, i32, pp, ctypes.POINTER(vp), vp]),
        "spin1_init_wigner_shard": (ctypes.c_int, [vp, ctypes.c_uint64, gp, i32, ctypes.POINTER(i64), pp,
                                                   ctypes.POINTER(vp), vp]),
        "spin1_set_params": (ctypes.c_int, [vp, pp]),
        "spin1_set_potential": (ctypes.c_int, [vp, i32, vp]),
        "spin1_step": (ctypes.c_int, [vp, i64, f64]),
        "spin1_sync_field": (ctypes.c_int, [vp]),
        "spin1_structure_factor": (ctypes.c_int, [vp, i32, vp]),
        "spin1_observables": (ctypes.c_int, [vp, i32, vp]),
        "spin1_observables_noalloc": (ctypes.c_int, [vp, i32, vp]),
        "spin1_step_observed": (ctypes.c_int, [vp, i64, f64, i32, vp]),
        "spin1_transverse_spin": (ctypes.c_int, [vp, i32, vp]),
        "spin1_spin_texture": (ctypes.c_int, [vp, i32, vp]),
        "spin1_local_update": (ctypes.c_int, [vp, f64]),
        "spin1_set_option": (ctypes.c_int, [vp, i32, i64]),
        "spin1_adjoint_workspace_bytes": (sz, [gp, i32, i64]),
        "spin1_num_variants": (i32, []),
        "spin1_autotune": (ctypes.c_int, [vp, vp, sz, i32]),
        "spin1_get_variant": (ctypes.c_int, [vp, i32, i32, ctypes.POINTER(i32)]),
        "spin1_set_variant": (ctypes.c_int, [vp, i32, i32, i32]),
        "spin1_forward_ckpt": (ctypes.c_int, [vp, i64, f64, i64, vp]),
        "spin1_adjoint": (ctypes.c_int, [vp, i64, f64, i64, vp, vp, vp, vp, vp]),
        "spin1_profile_enable": (ctypes.c_int, [vp, i32]),
        "spin1_profile_read": (ctypes.c_int, [vp, ctypes.POINTER(f64), ctypes.POINTER(i64), i32]),
        "spin1_last_error": (ctypes.c_char_p, []),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def last_error():
    return load().spin1_last_error().decode()


def _check(rc):
    if rc != OK:
        raise Spin1Error(rc, last_error())
    return rc


def make_grid(dim, n, dx, samples):
    """Grid(dim, (Nx[, Ny[, Nz]]), dx, samples); missing axes are 1."""
    n = tuple(int(v) for v in n) + (1,) * (3 - len(n))
    return Grid(int(dim), (ctypes.c_int32 * 3)(*n[:3]), float(dx), int(samples))


def make_params(c0, c1, q, n0=1.0, wigner_var=0.5):
    return Params(float(c0), float(c1), float(q), float(n0), float(wigner_var))


def _grid_array(grids):
    grids = list(grids)
    arr = (Grid * len(grids))(*grids)
    return arr, len(grids)


def _ptr_array(ptrs):
    return (ctypes.c_void_p * len(ptrs))(*[ctypes.c_void_p(int(p)) for p in ptrs])


# ---- thin wrappers with the C names -------------------------------------
def create(dtype, stream=0):
    h = ctypes.c_void_p()
    _check(load().spin1_create(ctypes.byref(h), int(dtype), ctypes.c_void_p(int(stream) if stream else None)))
    return h


def destroy(ctx):
    _check(load().spin1_destroy(ctx))


def check_grid(grid, dtype):
    _check(load().spin1_check_grid(ctypes.byref(grid), int(dtype)))


def field_bytes(grid, dtype):
    v = load().spin1_field_bytes(ctypes.byref(grid), int(dtype))
    if v == 0:
        raise Spin1Error(EINVAL, last_error())
    return int(v)


def workspace_bytes(grids, dtype):
    arr, n = _grid_array(grids)
    v = load().spin1_workspace_bytes(arr, n, int(dtype))
    if v == 0:
        raise Spin1Error(EINVAL, last_error())
    return int(v)


def num_bins(grid):
    v = load().spin1_num_bins(ctypes.byref(grid))
    if v < 0:
        raise Spin1Error(v, last_error())
    return int(v)


def bin_counts(grid):
    out = np.zeros(num_bins(grid), dtype=np.int64)
    _check(load().spin1_bin_counts(ctypes.byref(grid), out.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))))
    return out


def bind(ctx, grids, params, psi_ptrs, workspace_ptr):
    arr, n = _grid_array(grids)
    _check(load().spin1_bind(ctx, arr, n, ctypes.byref(params), _ptr_array(psi_ptrs),
                             ctypes.c_void_p(int(workspace_ptr))))


def init_wigner(ctx, seed, grids, params, psi_ptrs, workspace_ptr):
    arr, n = _grid_array(grids)
    _check(load().spin1_init_wigner(ctx, ctypes.c_uint64(int(seed)), arr, n, ctypes.byref(params),
                                    _ptr_array(psi_ptrs), ctypes.c_void_p(int(workspace_ptr))))


def init_wigner_shard(ctx, seed, grids, first_samples, params, psi_ptrs, workspace_ptr):
    """init_wigner with sample s of group i numbered first_samples[i] + s in the
    generator's counter (first_samples None: all zeros)."""
    arr, n = _grid_array(grids)
    offs = None
    if first_samples is not None:
        offs = (ctypes.c_int64 * n)(*[int(v) for v in first_samples])
    _check(load().spin1_init_wigner_shard(ctx, ctypes.c_uint64(int(seed)), arr, n, offs, ctypes.byref(params),
                                          _ptr_array(psi_ptrs), ctypes.c_void_p(int(workspace_ptr))))


def set_params(ctx, params):
    _check(load().spin1_set_params(ctx, ctypes.byref(params)))


def set_potential(ctx, group, v_ptr):
    """v_ptr: device address of sites FP64 values, or 0 to remove the potential."""
    _check(load().spin1_set_potential(ctx, int(group), ctypes.c_void_p(int(v_ptr)) if v_ptr else None))


def step(ctx, n, dt):
    _check(load().spin1_step(ctx, int(n), float(dt)))


def sync_field(ctx):
    _check(load().spin1_sync_field(ctx))


def structure_factor(ctx, group, bins_ptr):
    _check(load().spin1_structure_factor(ctx, int(group), ctypes.c_void_p(int(bins_ptr))))


def observables(ctx, group, obs_ptr):
    _check(load().spin1_observables(ctx, int(group), ctypes.c_void_p(int(obs_ptr))))


def observables_noalloc(ctx, group, obs_ptr):
    _check(load().spin1_observables_noalloc(ctx, int(group), ctypes.c_void_p(int(obs_ptr))))


def step_observed(ctx, n, dt, group, obs_ptr):
    _check(load().spin1_step_observed(ctx, int(n), float(dt), int(group), ctypes.c_void_p(int(obs_ptr))))


def transverse_spin(ctx, group, out_ptr):
    _check(load().spin1_transverse_spin(ctx, int(group), ctypes.c_void_p(int(out_ptr))))


def spin_texture(ctx, group, out_ptr):
    _check(load().spin1_spin_texture(ctx, int(group), ctypes.c_void_p(int(out_ptr))))


def local_update(ctx, tau):
    _check(load().spin1_local_update(ctx, float(tau)))


def set_option(ctx, option, value):
    _check(load().spin1_set_option(ctx, int(option), int(value)))


def profile_enable(ctx, enable=True):
    _check(load().spin1_profile_enable(ctx, 1 if enable else 0))


def profile_read(ctx):
    """{kind: (total_ms, launches)} since the last read (synchronises the stream)."""
    k = len(KERNEL_KINDS)
    ms = (ctypes.c_double * k)()
    cnt = (ctypes.c_int64 * k)()
    _check(load().spin1_profile_read(ctx, ms, cnt, k))
    return {name: (float(ms[i]), int(cnt[i])) for i, name in enumerate(KERNEL_KINDS)}


def num_variants():
    return int(load().spin1_num_variants())


def autotune(ctx, scratch_ptr, scratch_bytes, reps=3):
    _check(load().spin1_autotune(ctx, ctypes.c_void_p(int(scratch_ptr)), int(scratch_bytes), int(reps)))


def get_variant(ctx, pass_, n):
    v = ctypes.c_int32()
    _check(load().spin1_get_variant(ctx, int(pass_), int(n), ctypes.byref(v)))
    return int(v.value)


def set_variant(ctx, pass_, n, variant):
    _check(load().spin1_set_variant(ctx, int(pass_), int(n), int(variant)))


def adjoint_workspace_bytes(grid, dtype, every):
    v = load().spin1_adjoint_workspace_bytes(ctypes.byref(grid), int(dtype), int(every))
    if v == 0:
        raise Spin1Error(EINVAL, last_error())
    return int(v)


def forward_ckpt(ctx, n, dt, every, ckpt_ptr):
    _check(load().spin1_forward_ckpt(ctx, int(n), float(dt), int(every), ctypes.c_void_p(int(ckpt_ptr))))


def adjoint(ctx, n, dt, every, ckpt_ptr, dl_dbins_ptr, ws_ptr, grad_psi0_ptr, grad_qc1_ptr):
    vp = ctypes.c_void_p
    _check(load().spin1_adjoint(ctx, int(n), float(dt), int(every), vp(int(ckpt_ptr)), vp(int(dl_dbins_ptr)),
                                vp(int(ws_ptr)), vp(int(grad_psi0_ptr)), vp(int(grad_qc1_ptr))))


# ---- convenience owner of device buffers ---------------------------------
def _spatial(grid):
    return tuple(reversed([grid.n[a] for a in range(grid.dim)]))


class Sim:
    """Fields, workspace and a context for a list of groups on one GPU.

    groups: list of (dim, (Nx, ...), dx, samples) tuples or Grid objects.
    dtype: "c64" or "c128".  Torch supplies the device memory and a stream
    of its own (default priority); every torch operation of this object runs
    on that stream, so the library's work and torch's copies stay ordered.
    Ordering against the caller: every method first makes this object's
    stream wait for the caller's current stream (so device tensors the caller
    produced there, and the caller's own work on ``psi``, are complete before
    the library reads them), tensors of the caller read here are marked as in
    use on this object's stream, and device tensors handed back without
    synchronising are ordered the other way round (the caller's current
    stream waits for this object's stream).  Methods that return host arrays
    synchronise.  ``psi`` holds the device tensors themselves.
    """

    def __init__(self, groups, params, dtype="c64", device="cuda:0"):
        import torch

        self.torch = torch
        self.device = torch.device(device)
        self.dtype_code = C64 if dtype in ("c64", C64, torch.complex64) else C128
        self.cdtype = torch.complex64 if self.dtype_code == C64 else torch.complex128
        self.grids = [g if isinstance(g, Grid) else make_grid(*g) for g in groups]
        for g in self.grids:
            check_grid(g, self.dtype_code)
        self.params = params if isinstance(params, Params) else make_params(**params)
        self.stream = torch.cuda.Stream(device=self.device)
        with torch.cuda.device(self.device), torch.cuda.stream(self.stream):
            self.psi = [torch.zeros((g.samples, 3) + _spatial(g), dtype=self.cdtype, device=self.device)
                        for g in self.grids]
            self.ws = torch.empty(workspace_bytes(self.grids, self.dtype_code), dtype=torch.uint8,
                                  device=self.device)
        self.ctx = create(self.dtype_code, self.stream.cuda_stream)
        self.nbins = [num_bins(g) for g in self.grids]
        self.bound = False
        self.potentials = {}  # group -> FP64 device tensor (the library borrows it)

    def close(self):
        if getattr(self, "ctx", None) is not None:
            self.stream.synchronize()
            destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _ptrs(self):
        return [p.data_ptr() for p in self.psi]

    def _follow_caller(self):
        """This object's stream waits for the caller's current stream."""
        self.stream.wait_stream(self.torch.cuda.current_stream(self.device))

    def _borrow(self, t):
        """A caller's device tensor that work on this object's stream reads:
        keep its memory from being reused before that work is done."""
        if isinstance(t, self.torch.Tensor) and t.is_cuda:
            t.record_stream(self.stream)

    def _hand_back(self, t):
        """A device tensor produced on this object's stream and returned
        without synchronising: the caller's current stream waits for it."""
        cur = self.torch.cuda.current_stream(self.device)
        if cur != self.stream:
            cur.wait_stream(self.stream)
            t.record_stream(cur)
        return t

    def synchronize(self):
        self.stream.synchronize()

    def _rebind_potentials(self):
        for group, v in self.potentials.items():
            set_potential(self.ctx, group, v.data_ptr())

    def init_wigner(self, seed, first_samples=None):
        """Wigner initial state; first_samples (one offset per group, or None)
        numbers this object's samples within a larger ensemble
        (spin1_init_wigner_shard)."""
        self._follow_caller()
        if first_samples is None:
            init_wigner(self.ctx, seed, self.grids, self.params, self._ptrs(), self.ws.data_ptr())
        else:
            init_wigner_shard(self.ctx, seed, self.grids, first_samples, self.params, self._ptrs(),
                              self.ws.data_ptr())
        self.bound = True
        self._rebind_potentials()

    def set_potential(self, group, V):
        """Trap potential V(x) of a group (array of the spatial shape, the same
        for every component and sample), or None to remove it.  Applies from
        the next step; kept across init_wigner / set_fields."""
        torch = self.torch
        if V is None:
            self.potentials.pop(group, None)
            if self.bound:
                set_potential(self.ctx, group, 0)
            return
        shape = _spatial(self.grids[group])
        self._follow_caller()
        self._borrow(V)
        with torch.cuda.stream(self.stream):
            v = torch.as_tensor(np.asarray(V, dtype=np.float64) if not isinstance(V, torch.Tensor) else V)
            v = v.to(device=self.device, dtype=torch.float64).reshape(shape).contiguous()
        self.potentials[group] = v
        if self.bound:
            set_potential(self.ctx, group, v.data_ptr())

    def set_fields(self, fields):
        """Copy host or device arrays into the fields and bind them."""
        torch = self.torch
        self._follow_caller()
        with torch.cuda.stream(self.stream):
            for dst, src in zip(self.psi, fields):
                self._borrow(src)
                src_t = torch.as_tensor(np.asarray(src) if not isinstance(src, torch.Tensor) else src)
                dst.copy_(src_t.to(self.cdtype).reshape(dst.shape))
        bind(self.ctx, self.grids, self.params, self._ptrs(), self.ws.data_ptr())
        self.bound = True
        self._rebind_potentials()

    def set_params(self, params):
        self.params = params if isinstance(params, Params) else make_params(**params)
        set_params(self.ctx, self.params)

    def set_option(self, option, value):
        set_option(self.ctx, option, value)

    def step(self, n, dt):
        self._follow_caller()
        step(self.ctx, n, dt)

    def local_update(self, tau):
        self._follow_caller()
        local_update(self.ctx, tau)

    def field_tensor(self, group=0):
        """The device tensor of a group's field once this object's stream has
        finished its queued work (synchronises)."""
        self.stream.synchronize()
        return self.psi[group]

    def fields(self):
        """The fields as numpy complex128 arrays (synchronises)."""
        self._follow_caller()
        with self.torch.cuda.stream(self.stream):
            out = [p.cpu().numpy().astype(np.complex128) for p in self.psi]
        return out

    def structure_factor_device(self, group=0):
        """Per-sample shell means [S, n_bins] (FP64) on the device, enqueued on
        this object's stream and returned without synchronising (the caller's
        current stream waits for it)."""
        self._follow_caller()
        with self.torch.cuda.stream(self.stream):
            out = self.torch.empty((self.grids[group].samples, self.nbins[group]), dtype=self.torch.float64,
                                   device=self.device)
        structure_factor(self.ctx, group, out.data_ptr())
        return self._hand_back(out)

    def structure_factor_samples(self, group=0):
        """Per-sample shell means [S, n_bins] as a numpy array."""
        self._follow_caller()
        with self.torch.cuda.stream(self.stream):
            out = self.torch.empty((self.grids[group].samples, self.nbins[group]), dtype=self.torch.float64,
                                   device=self.device)
        structure_factor(self.ctx, group, out.data_ptr())
        with self.torch.cuda.stream(self.stream):
            return out.cpu().numpy()

    def structure_factor(self, group=0):
        """(k_b, mean, se, counts, per-sample bins) for one group."""
        per = self.structure_factor_samples(group)
        g = self.grids[group]
        s = per.shape[0]
        mean = per.mean(axis=0)
        se = per.std(axis=0, ddof=1) / math.sqrt(s) if s > 1 else np.zeros_like(mean)
        nmax = max(g.n[a] for a in range(g.dim))
        kb = np.arange(per.shape[1]) * 2.0 * math.pi / (nmax * g.dx)
        return kb, mean, se, bin_counts(g), per

    # ---- autotuning ----
    def pass_sizes(self):
        """(pass, n) pairs of the step passes the bound groups use."""
        out = set()
        for g in self.grids:
            out.add((0, g.n[0]))
            for a in range(1, g.dim):
                out.add((1, g.n[a]))
        return sorted(out)

    def autotune(self, reps=3, cache_path=None):
        """Pick the fastest step-pass variants; with cache_path, reuse and
        extend a JSON cache keyed by (arch, dtype, pass, n)."""
        import json
        import os

        torch = self.torch
        arch = torch.cuda.get_device_properties(self.device).gcnArchName.split(":")[0]
        dname = "c64" if self.dtype_code == C64 else "c128"
        cache = {}
        if cache_path and os.path.exists(cache_path):
            with open(cache_path) as fh:
                cache = json.load(fh)
        keys = {(p, n): "%s/%s/%d/%d" % (arch, dname, p, n) for p, n in self.pass_sizes()}
        self._follow_caller()
        if all(k in cache for k in keys.values()):
            for (p, n), k in keys.items():
                set_variant(self.ctx, p, n, cache[k])
            return {k: cache[k] for k in keys.values()}
        with torch.cuda.stream(self.stream):
            nbytes = max(p.numel() * p.element_size() for p in self.psi)
            scratch = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        autotune(self.ctx, scratch.data_ptr(), nbytes, reps)
        self.stream.synchronize()
        chosen = {k: get_variant(self.ctx, p, n) for (p, n), k in keys.items()}
        if cache_path:
            cache.update(chosen)
            with open(cache_path, "w") as fh:
                json.dump(cache, fh, indent=1, sort_keys=True)
        return chosen

    # ---- reverse mode (one group) ----
    def forward_ckpt(self, n, dt, every):
        """Advance n steps, keeping a checkpoint every `every` steps (device tensor)."""
        torch = self.torch
        nck = (int(n) + int(every) - 1) // int(every) if int(every) > 0 and int(n) > 0 else 1
        self._follow_caller()
        with torch.cuda.stream(self.stream):
            ckpt = torch.empty((nck,) + tuple(self.psi[0].shape), dtype=self.cdtype, device=self.device)
        forward_ckpt(self.ctx, n, dt, every, ckpt.data_ptr())
        return ckpt

    def adjoint(self, n, dt, every, ckpt, dl_dbins):
        """(dL/dpsi0 field, tensor [dL/dq, dL/dc1]) for dL/dS_{s,b} = dl_dbins [S, n_bins]."""
        torch = self.torch
        self._follow_caller()
        self._borrow(dl_dbins)
        self._borrow(ckpt)
        with torch.cuda.stream(self.stream):
            dl = torch.as_tensor(dl_dbins, dtype=torch.float64).to(self.device).contiguous()
            ws = torch.empty(adjoint_workspace_bytes(self.grids[0], self.dtype_code, every), dtype=torch.uint8,
                             device=self.device)
            grad = torch.empty_like(self.psi[0])
            gqc = torch.empty(2, dtype=torch.float64, device=self.device)
        adjoint(self.ctx, n, dt, every, ckpt.data_ptr(), dl.data_ptr(), ws.data_ptr(), grad.data_ptr(), gqc.data_ptr())
        self.stream.synchronize()
        return grad, gqc

    def observables(self, group=0):
        """Per-sample (N, F_z, E) [S, 3] as a numpy array."""
        self._follow_caller()
        with self.torch.cuda.stream(self.stream):
            out = self.torch.empty((self.grids[group].samples, 3), dtype=self.torch.float64, device=self.device)
        observables(self.ctx, group, out.data_ptr())
        with self.torch.cuda.stream(self.stream):
            return out.cpu().numpy()


    def transverse_spin(self, group=0):
        """F_perp per site of `group` as a device tensor [S, spatial...],
        enqueued on this object's stream and returned without synchronising
        (the caller's current stream waits for it)."""
        g = self.grids[group]
        self._follow_caller()
        with self.torch.cuda.stream(self.stream):
            out = self.torch.empty((g.samples,) + _spatial(g), dtype=self.psi[group].dtype, device=self.device)
        transverse_spin(self.ctx, group, out.data_ptr())
        return self._hand_back(out)

    def spin_texture(self, group=0):
        """Per-sample (mean |F_perp|, mean |F_perp|^2, Q_w) [S, 3] as numpy."""
        self._follow_caller()
        with self.torch.cuda.stream(self.stream):
            out = self.torch.empty((self.grids[group].samples, 3), dtype=self.torch.float64, device=self.device)
        spin_texture(self.ctx, group, out.data_ptr())
        with self.torch.cuda.stream(self.stream):
            return out.cpu().numpy()

    def step_observed(self, n, dt, group=0):
        """n steps, returning the per-step FP64 (N, F_z, E) of `group` as a
        numpy array [n, S, 3] (row i: the state R(dt/2) psi(t + i dt))."""
        self._follow_caller()
        with self.torch.cuda.stream(self.stream):
            out = self.torch.empty((max(int(n), 1), self.grids[group].samples, 3), dtype=self.torch.float64,
                                   device=self.device)
        step_observed(self.ctx, n, dt, group, out.data_ptr())
        with self.torch.cuda.stream(self.stream):
            return out[: int(n)].cpu().numpy()


def _loss_from_bins(bins, target, mask):
    sbar = bins.mean(0)
    return ((sbar - target) ** 2 * mask).sum(), sbar


def make_split_step_loss():
    """torch.autograd.Function for L = sum_{k_b < k_cut} (S_b(t_T) - T_b)^2, S_b the
    sample mean of the shell means of |DFT F_perp|^2 / N_sites after `steps` steps
    from psi0; differentiable in psi0 (complex), q and c1 through the library's
    reverse mode (checkpoints every `every` steps)."""
    import torch

    class SplitStepLoss(torch.autograd.Function):
        @staticmethod
        def forward(fctx, psi0, q, c1, target, k_cut, steps, dt, every, grid, c0=1.0, dtype="c64"):
            params = make_params(c0, float(c1), float(q))
            sim = Sim([grid], params, dtype=dtype, device=psi0.device)
            sim.set_fields([psi0.detach()])
            ckpt = sim.forward_ckpt(steps, dt, every)
            bins = sim.structure_factor_device()
            with torch.cuda.stream(sim.stream):
                g = sim.grids[0]
                nmax = max(g.n[a] for a in range(g.dim))
                kb = torch.arange(bins.shape[1], dtype=torch.float64, device=bins.device) * 2 * math.pi / (nmax * g.dx)
                mask = (kb < k_cut).to(torch.float64)
                tgt = torch.as_tensor(target, dtype=torch.float64).to(bins.device)
                L, sbar = _loss_from_bins(bins, tgt, mask)
                L = L.detach()
            sim.stream.synchronize()
            fctx.sim, fctx.ckpt, fctx.steps, fctx.dt, fctx.every = sim, ckpt, steps, dt, every
            fctx.psi_dtype = psi0.dtype
            fctx.dl = (2.0 * (sbar - tgt) * mask / bins.shape[0]).expand_as(bins).contiguous()
            return L.to(psi0.device)

        @staticmethod
        def backward(fctx, gl):
            sim = fctx.sim
            grad, gqc = sim.adjoint(fctx.steps, fctx.dt, fctx.every, fctx.ckpt, fctx.dl)
            gl = gl.to(torch.float64)
            gpsi = grad.to(fctx.psi_dtype) * gl.to(fctx.psi_dtype)
            sim.close()
            return (gpsi, gqc[0] * gl, gqc[1] * gl) + (None,) * 8

    return SplitStepLoss
