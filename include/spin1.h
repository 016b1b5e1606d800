/*
 * spin1.h -- C ABI of the MI355X spin-1 split-step library.
 *
 * The library propagates many truncated-Wigner samples of the three-component
 * (spin-1) Gross-Pitaevskii equation, Eq. (2) of arXiv:2310.03636
 * ("Universal Dynamics at the Lowest Temperatures", Sec. 2.2), with a
 * split-step Fourier method (Sec. 2.2, Eqs. (3)-(5)), and evaluates the
 * sample-averaged structure factor S(t,k) = <F_perp(t,k)^* F_perp(t,k)> of the
 * transverse spin F_perp = F_x + i F_y (Sec. 2.1, the paragraph before
 * Eq. (1)).
 *
 * Units hbar = m = 1.  Components are ordered (psi_{+1}, psi_0, psi_{-1}) as
 * in Eq. (2).  A field of one group is a device array [S][3][Nz][Ny][Nx] of
 * interleaved complex numbers (x fastest): complex64 (2 x float) or
 * complex128 (2 x double).
 *
 * Memory ownership: the caller owns every device buffer (fields, workspace,
 * outputs) and passes raw device pointers; the library only borrows them
 * between spin1_bind / spin1_init_wigner and spin1_destroy or the next bind.
 * The library allocates no device memory of its own.
 *
 * Streams: all device work is enqueued on the HIP stream given to
 * spin1_create and is asynchronous; results in device buffers are valid
 * once that stream has completed the call.  A context is not thread-safe.
 *
 * Errors: every int-returning function returns SPIN1_OK (0) or a negative
 * status; spin1_last_error() returns a thread-local message for the last
 * failure.  Arguments are validated before anything is launched; a call that
 * fails validation changes no state.  Faults of kernels that already run
 * surface as SPIN1_EHIP at a later call that checks the stream.
 */
#ifndef SPIN1_H
#define SPIN1_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#if defined(__GNUC__)
#define SPIN1_API __attribute__((visibility("default")))
#else
#define SPIN1_API
#endif

typedef struct spin1_ctx spin1_ctx;

enum spin1_status {
  SPIN1_OK = 0,
  SPIN1_EINVAL = -1,       /* invalid argument */
  SPIN1_EUNSUPPORTED = -2, /* valid but not supported by the compiled kernels */
  SPIN1_EHIP = -3,         /* HIP runtime error */
  SPIN1_ESTATE = -4,       /* call out of order (e.g. step before bind) */
  SPIN1_ENOMEM = -5        /* a host allocation failed */
};

enum spin1_dtype { SPIN1_C64 = 0, SPIN1_C128 = 1 };

/* A periodic lattice with `samples` independent runs.  dim in {1,2,3};
 * n[a] points along axis a (x, y, z), n[a] = 1 for a >= dim; dx > 0 the
 * lattice spacing (lengths in the units of Eq. (2) with hbar = m = 1).
 * Supported sizes: every n[a] (a < dim) a power of two; 8 <= Nx <= 4096 in
 * 1D; 16 <= Nx <= 4096 and 8 <= Ny, Nz <= 1024 in 2D and 3D. */
typedef struct {
  int32_t dim;
  int32_t n[3];
  double dx;
  int32_t samples;
} spin1_grid;

/* Couplings of Eq. (2): c0 (density), c1 (spin), q (quadratic Zeeman, acts
 * on m = +1 and m = -1 only); n0 the condensate density of the polar initial
 * state psi_0 = sqrt(n0); wigner_var the Wigner noise per plane-wave mode
 * (per-site variance wigner_var / dx^dim per component; 1/2 = half a
 * quantum). */
typedef struct {
  double c0, c1, q, n0, wigner_var;
} spin1_params;

/* Create a context for fields of the given dtype on the current HIP device.
 * stream: a hipStream_t (may be NULL for the default stream).  *out is set on
 * success; free it with spin1_destroy. */
SPIN1_API int spin1_create(spin1_ctx** out, int32_t dtype, void* stream);
SPIN1_API int spin1_destroy(spin1_ctx* ctx);

/* Host-only helpers (no device work).  Invalid grids give 0 / a negative
 * status and set the error message. */
SPIN1_API int spin1_check_grid(const spin1_grid* g, int32_t dtype);
SPIN1_API size_t spin1_field_bytes(const spin1_grid* g, int32_t dtype);  /* S*3*sites*sizeof(complex) */
SPIN1_API size_t spin1_workspace_bytes(const spin1_grid* groups, int32_t n_groups, int32_t dtype);
/* Radial shells of the structure factor: shell b collects the modes whose
 * integer index vector j' (signed DFT index per axis, scaled to the finest
 * axis spacing) has |j'| nearest to b.  Returns the number of shells or a
 * negative status. */
SPIN1_API int32_t spin1_num_bins(const spin1_grid* g);
/* counts_host[b] = number of modes in shell b (array of spin1_num_bins). */
SPIN1_API int spin1_bin_counts(const spin1_grid* g, int64_t* counts_host);

/* Bind n_groups fields (psi_dev[g]: device array of spin1_field_bytes) and a
 * workspace of spin1_workspace_bytes bytes to the context, with the couplings
 * p.  Host index tables for the shells are uploaded synchronously. */
SPIN1_API int spin1_bind(spin1_ctx* ctx, const spin1_grid* groups, int32_t n_groups, const spin1_params* p,
               void* const* psi_dev, void* workspace_dev);

/* spin1_bind, then fill every bound field with the truncated-Wigner initial
 * state of Sec. 2.2 (runs from weakly fluctuating initial conditions): a polar
 * condensate psi_0 = sqrt(n0) plus complex Gaussian noise of variance
 * wigner_var / dx^dim on every component.  The noise of (site, component,
 * sample, group) comes from one Philox4x64-10 block with that counter and key
 * (seed, 0) (Box-Muller of its first two words), so every sample is
 * reproducible on its own. */
SPIN1_API int spin1_init_wigner(spin1_ctx* ctx, uint64_t seed, const spin1_grid* groups, int32_t n_groups,
                      const spin1_params* p, void* const* psi_dev, void* workspace_dev);

/* spin1_init_wigner for one shard of a larger ensemble.  The Wigner samples
 * are independent runs (Sec. 2.2: many runs per GPU, and runs spread over
 * several GPUs), so an ensemble can be split by sample: sample s of group i
 * here is sample first_sample[i] + s of the whole ensemble, and its noise
 * comes from the generator counter (site, component, first_sample[i] + s, i)
 * with key (seed, 0).  Contexts that bind the same groups in the same order
 * with disjoint ranges of samples therefore produce exactly the fields (and,
 * being per sample, the shell means and observables) that one context over
 * the whole ensemble produces for those samples.  first_sample: host array of
 * n_groups values >= 0, or NULL for all zeros (then this is
 * spin1_init_wigner).  Errors as spin1_init_wigner, and SPIN1_EINVAL for a
 * negative or overflowing offset (checked before anything is bound). */
SPIN1_API int spin1_init_wigner_shard(spin1_ctx* ctx, uint64_t seed, const spin1_grid* groups, int32_t n_groups,
                                      const int64_t* first_sample, const spin1_params* p, void* const* psi_dev,
                                      void* workspace_dev);

/* Replace the couplings between steps (a quench of q, Sec. 2.1, Fig. 1). */
SPIN1_API int spin1_set_params(spin1_ctx* ctx, const spin1_params* p);

/* Trap potential V(x) of group `group`: the V_m of Eq. (4), a diagonal term of
 * the operator of Eq. (2), taken the same for the three components and for
 * every sample of the group.  v_dev: device array of sites FP64 values in the
 * field's site order (x fastest), 8-byte aligned; NULL removes the potential.
 * The library borrows the pointer: the array must stay valid and unchanged
 * while it is set (until it is replaced, removed, or the context is bound
 * again, which clears every potential).  Effects: the local update becomes
 * exp(-i V tau) R(tau) (still exact, since V commutes with the local flow);
 * the Lie scheme adds V to the diagonal phases of Eq. (4); the energy of
 * spin1_observables and spin1_step_observed gains dx^d sum V n.  A group with
 * a potential is stepped one x-pass launch per step (no multi-step 1D kernel,
 * no grouped x-pass).  Reverse mode returns SPIN1_EUNSUPPORTED while one is
 * set.  Errors: SPIN1_ESTATE if not bound, SPIN1_EINVAL for a bad group or
 * misaligned pointer. */
SPIN1_API int spin1_set_potential(spin1_ctx* ctx, int32_t group, const double* v_dev);

/* Advance every bound group by n steps of dt (dt may be negative): each step
 * is the symmetric split R(dt/2) [K Q](dt) R(dt/2) of the operator of Eq. (2),
 * R the exact local (c0, c1) update (the interaction sub-steps, Eqs. (4)-(5)),
 * K the kinetic phase of Eq. (3) and Q the quadratic Zeeman phase.  Adjacent
 * half steps are merged inside the call; the field is at t + n dt on return. */
SPIN1_API int spin1_step(spin1_ctx* ctx, int64_t n, double dt);

/* Bring every bound field to its synchronized time.  spin1_step applies the
 * closing half step R(dt/2) before it returns, so no half step is ever left
 * pending and this call only validates the context (SPIN1_ESTATE if nothing
 * is bound); it enqueues no device work. */
SPIN1_API int spin1_sync_field(spin1_ctx* ctx);

/* Per-sample shell means of |DFT F_perp(k)|^2 / N_sites for group `group`
 * (the sample average of these is S(t,k) of Sec. 2.1; a shell without modes
 * reports 0): bins_dev is a device array [S][spin1_num_bins] of double. */
SPIN1_API int spin1_structure_factor(spin1_ctx* ctx, int32_t group, double* bins_dev);

/* Per-sample (N, F_z, E) in FP64 for group `group`: obs_dev is a device array
 * [S][3] of double, N = dx^d sum n, F_z = dx^d sum (|psi_1|^2 - |psi_-1|^2),
 * E the energy whose Wirtinger derivative is the right-hand side of Eq. (2). */
SPIN1_API int spin1_observables(spin1_ctx* ctx, int32_t group, double* obs_dev);

/* spin1_observables for callers that cannot allocate device memory around
 * the call (code under HIP graph capture, tight serving loops, harnesses that
 * forbid allocation): the same kernels and the same results, with the FP64
 * partial sums kept in a static device array of the library (32 MiB, one copy
 * per GPU, held from the load of the library until the process ends) instead
 * of the bound workspace.  The call allocates nothing.  Limit: a group needs
 * (S * rows * 4 + the strided-pass partials) doubles, rows = Ny * Nz, and
 * must fit the 32 MiB (e.g. 2D 512^2 x 384, 3D 256^3 x 8 do); a larger group
 * returns SPIN1_EUNSUPPORTED before anything is launched.  Every call on a
 * GPU shares that GPU's array: calls that overlap in time on one GPU (from
 * several contexts or streams) race, so the caller orders them.
 * SPIN1_EHIP if the array's device address could not be obtained when the
 * context was created. */
SPIN1_API int spin1_observables_noalloc(spin1_ctx* ctx, int32_t group, double* obs_dev);

/* Transverse spin F_perp = F_x + i F_y = sqrt2 (psi_1^* psi_0 + psi_0^* psi_-1)
 * of group `group` at every site (Sec. 2.1 and Fig. 1: spin length |F_perp|
 * and Larmor phase phi_L = arg F_perp): fperp_dev is a device array
 * [S][Nz][Ny][Nx] of complex values in the field's precision. */
SPIN1_API int spin1_transverse_spin(spin1_ctx* ctx, int32_t group, void* fperp_dev);

/* Real-space spin texture of group `group` (Fig. 1): out_dev is a device
 * array [S][3] of double holding, per sample, the site means of |F_perp| and
 * |F_perp|^2 and the winding Q_w of the Larmor phase along x: the phase steps
 * phi_L(x_{j+1}) - phi_L(x_j), each taken in [-pi, pi) (phi_L = 0 where
 * F_perp = 0), summed around every periodic x-row and over the rows, divided
 * by 2 pi (in 1D the paper's winding number; an integer up to rounding).
 * Sums in FP64, fixed order. */
SPIN1_API int spin1_spin_texture(spin1_ctx* ctx, int32_t group, double* out_dev);

/* spin1_step(n, dt) that also logs, for group `group`, the FP64 (N, F_z, E)
 * of every step: obs_dev is a device array [n][S][3] of double, row i being
 * the observables of R(dt/2) psi(t + i dt), the state the kinetic sub-step of
 * step i starts from (summed inside the step passes, no extra field pass).
 * N and F_z equal those of psi(t + i dt) exactly (R conserves n and F at every
 * site); E differs from E(psi(t + i dt)) by O(dt) and carries no drift of its
 * own.  Direct launches (no graph); 1D groups take one x-pass launch per step
 * in this call.  Errors as spin1_step, and SPIN1_EINVAL for a bad group or a
 * NULL obs_dev. */
SPIN1_API int spin1_step_observed(spin1_ctx* ctx, int64_t n, double dt, int32_t group, double* obs_dev);

/* Apply the exact local update R(tau) alone to every bound field (Eqs. (4)-(5)
 * combined, q excluded; with exp(-i V tau) where a trap potential is set). */
SPIN1_API int spin1_local_update(spin1_ctx* ctx, double tau);

/* Reverse mode (one bound group).  The caller owns a checkpoint array of
 * ceil(n / every) fields and an adjoint workspace of
 * spin1_adjoint_workspace_bytes bytes (every + 2 fields plus a few kB).
 *
 * spin1_forward_ckpt: like spin1_step(ctx, n, dt), run as chunks of `every`
 *   steps; the field at the start of chunk c is copied to checkpoint c first.
 *   On return the bound field is the final field psi_T.
 * spin1_adjoint: given dL/dS_{s,b} (device [S][spin1_num_bins] FP64) for any
 *   real loss L of the per-sample shell means S_{s,b} of psi_T (as returned by
 *   spin1_structure_factor), computes the gradients of L with respect to the
 *   initial field (grad_psi0_dev: a field, dL/dRe + i dL/dIm), q and c1
 *   (grad_qc1_dev: 2 doubles) by reverse-mode differentiation of the discrete
 *   split-step map.  It expects the bound field to be psi_T from
 *   spin1_forward_ckpt with the same n, dt and every, and the same couplings;
 *   the states inside each chunk are recomputed from its checkpoint.  The
 *   bound field is left unchanged. */
SPIN1_API size_t spin1_adjoint_workspace_bytes(const spin1_grid* g, int32_t dtype, int64_t every);
SPIN1_API int spin1_forward_ckpt(spin1_ctx* ctx, int64_t n, double dt, int64_t every, void* ckpt_dev);
SPIN1_API int spin1_adjoint(spin1_ctx* ctx, int64_t n, double dt, int64_t every, const void* ckpt_dev,
                            const double* dL_dbins_dev, void* adj_ws_dev, void* grad_psi0_dev, double* grad_qc1_dev);

/* Autotuning of the step passes.  Each step pass (pass 0: the x-pass,
 * pass 1: the strided y/z pass) is compiled in spin1_num_variants() variants
 * per axis length n (workgroup shape, columns per tile, radix).
 * spin1_autotune copies each bound field into scratch_dev (at least the
 * largest field; the bound fields are not touched), times every variant of
 * every pass the bound groups use (reps launches each, HIP events on the
 * context's stream; synchronises) in three sweeps after a warm-up sweep, the
 * variants taking turns, and keeps the variant with the fastest sweep per
 * (pass, n, dtype) for this context.  It then retries each choice used by a
 * 2D or 3D group, one (pass, n) at a time, by timing whole split steps of the
 * groups that use it on the scratch copy, and keeps the variant with the
 * least step time.  spin1_get_variant / spin1_set_variant read and restore
 * the choices (e.g. from a cache file). */
SPIN1_API int32_t spin1_num_variants(void);
SPIN1_API int spin1_autotune(spin1_ctx* ctx, void* scratch_dev, size_t scratch_bytes, int32_t reps);
SPIN1_API int spin1_get_variant(spin1_ctx* ctx, int32_t pass, int32_t n, int32_t* variant);
SPIN1_API int spin1_set_variant(spin1_ctx* ctx, int32_t pass, int32_t n, int32_t variant);

/* Options (spin1_set_option).
 * SPIN1_OPT_GRAPHS: 1 (default) = spin1_step captures the launches of an
 *   n-step call into a HIP graph on first use and replays it for later calls
 *   with the same (n, dt) and unchanged binding and couplings; 0 = launch each
 *   kernel directly.  Graphs are never used while profiling is enabled or on
 *   the NULL stream.  At most 8 graphs are kept per context (least recently
 *   used first out); spin1_bind and spin1_set_params retire them.
 * SPIN1_OPT_GRAPH_MAX_STEPS: longest step sequence in one graph (default
 *   1024); longer calls run as consecutive chunks, each ending at a
 *   synchronized time.
 * SPIN1_OPT_STEPS_PER_LAUNCH_1D: 1D groups run up to this many consecutive
 *   split steps in one launch, each sample held on chip between steps
 *   (range 1..1024); 1 = one x-pass launch per step, as for 2D/3D groups;
 *   0 (default) = automatic: 64 at every length.  The result is the same
 *   map either way (same arithmetic, different kernel).
 * SPIN1_OPT_GROUPED_X: 1 = when two or more bound groups are stepped one
 *   x-pass launch per step and have Nx in 16..1024 (FP32) or 16..512 (FP64),
 *   their x-passes run as one persistent launch per step (radix 8, groups back
 *   to back in one work list); 0 (default) = one x-pass launch per group, each
 *   group's passes in a sequence of its own (see SPIN1_OPT_CONCURRENT_GROUPS).
 *   Same arithmetic either way.
 * SPIN1_OPT_SCHEME: SPIN1_SCHEME_STRANG (default), the symmetric split with
 *   the exact local flow described at spin1_step; or SPIN1_SCHEME_PAPER, the
 *   paper's own scheme in its order (Sec. 2.2): per step the kinetic phase of
 *   Eq. (3) (without q), then the diagonal phases of Eq. (4) (q and the
 *   density terms, densities of the field they act on), then the mixing of
 *   Eq. (5) with couplings averaged over the field and a one-step predictor.
 *   First order in dt; it converges to the same flow as dt -> 0.  Reverse
 *   mode and spin1_step_observed take the Strang scheme only
 *   (SPIN1_EUNSUPPORTED otherwise).
 * SPIN1_OPT_FP32_TWIDDLES (complex64 only): how the streaming step passes
 *   of spin1_step (and the grouped x-pass) hold their FFT stage twiddles and
 *   kinetic phase factors.
 *   SPIN1_TWIDDLES_DITHERED (default): one float pair per value, rebuilt at
 *   every step as one of the two float pairs next to the FP64 value, chosen
 *   by error diffusion over the step index within the call so that the mean
 *   over steps tracks the FP64 value; a multiply costs half the compensated
 *   one, and the rounding of the constants does not add up step after step.
 *   The dithering restarts with every call, so complex64 results of n steps
 *   in one call and of the same steps split over several calls agree to
 *   single precision but not bit for bit.
 *   SPIN1_TWIDDLES_COMPENSATED: hi+lo float pairs, so the constants carry no
 *   rounding of their own.  The radix constants of the in-register
 *   butterflies and the other passes use the compensated form either way.
 * SPIN1_OPT_CONCURRENT_GROUPS: 1 (default) = the independent step sequences
 *   of a call (each group outside a grouped x-pass, and the grouped set) run
 *   on the caller's stream and up to three streams of the library's (default
 *   priority, created on first use), forked from the caller's stream at the
 *   start of the call and joined back into it at the end, so that the passes
 *   of different groups overlap (round robin beyond four sequences); 0 =
 *   everything on the caller's stream, one sequence after the other.  Not used
 *   while profiling or on the NULL stream.  Same results either way.
 * SPIN1_OPT_1D_KERNEL: the kernel of the multi-step 1D launches: 0 (default)
 *   and 2 = three thread groups per sample, one per component, regrouped
 *   through LDS for the local update (shorter step latency; Nx <= 2048, the
 *   pencil form otherwise); 1 = one thread group per sample holding all three
 *   components.  Same map either way.
 * SPIN1_OPT_STREAMING_STORES: how the streaming x and y/z passes of spin1_step
 *   write the field back.  SPIN1_STORES_AUTO (default) = non-temporal stores
 *   (the written lines are not kept in the caches) when the fields of all
 *   bound groups together exceed 512 MiB (complex64) or 768 MiB (complex128),
 *   ordinary stores otherwise;
 *   SPIN1_STORES_CACHED and SPIN1_STORES_STREAMING force one form.  A field
 *   that fits the last-level cache (256 MB on MI355X) is read back in part
 *   from it by the next pass, which ordinary stores keep possible; beyond
 *   about twice that size the cache holds little of the field and the
 *   non-temporal stores leave it to the loads.  Same results, bit for bit,
 *   either way. */
enum spin1_option {
  SPIN1_OPT_GRAPHS = 0,
  SPIN1_OPT_GRAPH_MAX_STEPS = 1,
  SPIN1_OPT_STEPS_PER_LAUNCH_1D = 2,
  SPIN1_OPT_GROUPED_X = 3,
  SPIN1_OPT_SCHEME = 4,
  SPIN1_OPT_FP32_TWIDDLES = 5,
  SPIN1_OPT_CONCURRENT_GROUPS = 6,
  SPIN1_OPT_1D_KERNEL = 7,
  SPIN1_OPT_STREAMING_STORES = 8
};
enum spin1_stores { SPIN1_STORES_AUTO = 0, SPIN1_STORES_CACHED = 1, SPIN1_STORES_STREAMING = 2 };
enum spin1_scheme { SPIN1_SCHEME_STRANG = 0, SPIN1_SCHEME_PAPER = 1 };
enum spin1_twiddles { SPIN1_TWIDDLES_COMPENSATED = 0, SPIN1_TWIDDLES_DITHERED = 1 };
SPIN1_API int spin1_set_option(spin1_ctx* ctx, int32_t option, int64_t value);

/* Kernel kinds reported by the profiling hooks. */
enum spin1_kernel_kind {
  SPIN1_K_XPASS = 0,       /* x-pass of a step (local update, FFT_x, phase, IFFT_x),
                              or of several steps of a 1D group */
  SPIN1_K_YPASS = 1,       /* y-pass of a step */
  SPIN1_K_ZPASS = 2,       /* z-pass of a step */
  SPIN1_K_LOCAL = 3,       /* stand-alone local update (closing half step) */
  SPIN1_K_SPECTRUM = 4,    /* F_perp transforms of the structure factor */
  SPIN1_K_SHELLS = 5,      /* radial shell sums */
  SPIN1_K_OBSERVABLES = 6, /* energy / norm / F_z passes */
  SPIN1_K_OTHER = 7,       /* tables and initial state */
  SPIN1_K_COUNT = 8
};

/* Profiling: when enabled, every library operation that launches kernels is
 * timed per kind.  An operation with one kernel launch (every step pass) is
 * timed by that kernel's own begin and end (two HIP events handed to
 * hipExtLaunchKernel); one with several launches by two HIP events recorded on
 * the context's stream before and after them.  While profiling is on, calls
 * run as direct launches on the context's stream (no graphs, no side
 * streams).  spin1_profile_read synchronises the stream, adds the elapsed
 * times per kind into ms[kind] and the counts of timed operations into
 * launches[kind] (arrays of n_kinds <= SPIN1_K_COUNT entries, overwritten),
 * and clears the record.  Events are created on first use and reused. */
SPIN1_API int spin1_profile_enable(spin1_ctx* ctx, int32_t enable);
SPIN1_API int spin1_profile_read(spin1_ctx* ctx, double* ms, int64_t* launches, int32_t n_kinds);

/* Message of the last failure on this thread; never NULL. */
SPIN1_API const char* spin1_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* SPIN1_H */
