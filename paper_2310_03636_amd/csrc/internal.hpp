// Internal interface between the C ABI (api.hip) and the kernel units (kernels*.hip).
#pragma once
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include <tuple>
#include <utility>

namespace spin1 {

// Every kernel launch of the library goes through launch_kernel.  While
// profiling is on, the bracket around a launch (api.hip) hands the thread's
// next launch a start and a stop event: that launch then goes through
// hipExtLaunchKernel, which stamps the kernel's own begin and end into them,
// so the measured time leaves out the dispatch gap that events recorded on
// the stream around the launch would include.  The arguments are converted
// to the kernel's parameter types before their addresses are handed over.
struct LaunchTiming {
  hipEvent_t start = nullptr, stop = nullptr;
  int64_t launches = 0;  // launches made by this thread so far
};
LaunchTiming& launch_timing();  // the calling thread's

template <typename... P, typename... A>
hipError_t launch_kernel(void (*kernel)(P...), dim3 grid, dim3 block, uint32_t shmem, hipStream_t st, A&&... args) {
  static_assert(sizeof...(P) == sizeof...(A), "kernel argument count");
  std::tuple<P...> values(std::forward<A>(args)...);
  void* ptrs[sizeof...(P) > 0 ? sizeof...(P) : 1] = {};
  std::apply([&ptrs](auto&... v) {
    int i = 0;
    ((ptrs[i++] = static_cast<void*>(&v)), ...);
  }, values);
  const void* fn = reinterpret_cast<const void*>(kernel);
  LaunchTiming& lt = launch_timing();
  lt.launches++;
  if (lt.start) {
    hipEvent_t a = lt.start, b = lt.stop;
    lt.start = lt.stop = nullptr;
    return hipExtLaunchKernel(fn, grid, block, ptrs, shmem, st, a, b, 0);
  }
  return hipLaunchKernel(fn, grid, block, ptrs, shmem, st);
}

// Geometry of one group: S samples of a dim-dimensional periodic grid,
// field layout [S][3][Nz][Ny][Nx] (x fastest), n[a] = 1 for a >= dim.
struct Geom {
  int dim;
  int n[3];
  double dx;
  int S;
  int64_t sites;  // Nx * Ny * Nz
  int64_t rows;   // sites / Nx: x-pencils per component and sample
};

// Number of strided-pass workgroups per (field, outer) and their column
// width for axis length N (shared by host layout and launches).
int spass_tx(int n, bool dbl);

// Kernel modes
// MODE_STEP_LOG: a step pass that also writes the FP64 partial sums of
// MODE_MEASURE for the state its kinetic sub-step starts from
// MODE_PAPER: x-pass of the paper's Lie scheme: [D, O of the previous step
// (tau_pre = dt)] K_x(dt) without q [D, O (tau_post = dt, 1D)]
enum PassMode { MODE_STEP = 0, MODE_MEASURE = 1, MODE_SF = 2, MODE_SF_POWER = 3, MODE_STEP_LOG = 4, MODE_PAPER = 5 };

struct XPassArgs {
  void* psi;        // field base [S][3][rows][Nx] (STEP, MEASURE, SF*)
  const void* src;  // STEP: when non-null the field is read from here and written to psi
  const double* pot;  // trap potential V [rows][Nx] of the group (same for every sample), or null
  void* out;        // SF: complex [S][rows][Nx]; SF_POWER: real [S][rows][Nx]
  double* part;     // MEASURE: [S*rows][4] = (sum n, sum Fz, sum e_loc, sum e_kin_x)
  const void* tw;   // exp(-2 pi i m / Nx)
  const void* ph;   // [3][Nx] exp(-i (k^2/2 + q m^2) dt) / Nx
  int64_t rows, sites;
  int S;
  double tau_pre, tau_post;  // local update before / after the kinetic step (0 = none)
  double c0, c1, q;
  double kscale;    // 2 pi / (Nx dx)
  double power_scale;  // SF_POWER: 1 / N_sites
  int lg_rows;      // log2(rows), set by the launcher
  int reverse;      // STEP (streaming kernel): walk the work items from the last one
  int nt;           // STEP (streaming kernel): non-temporal stores of the field
  int64_t tick;     // STEP: index of the step in the call (dithered single-precision tables)
};

// One x-pass launch over the step passes of several groups (pencil lengths
// 16..kGroupedMaxN, radix 8, 256 threads per workgroup).  Group g owns the
// work items [item_begin[g], item_begin[g + 1]) of P_g = 2048 / n_g pencils each.
constexpr int kMaxGroupedX = 8;
struct XGroupEntry {
  void* psi;
  const void* tw;
  const void* ph;
  int64_t rows, sites, pencils;  // pencils = S * rows
  int64_t item_begin;
  double tau_post;
  int n, lg_rows;
};
struct XGroupArgs {
  XGroupEntry g[kMaxGroupedX];
  int64_t item_end;  // item_begin of a virtual group past the last
  int ngroups;
  double tau_pre, c0, c1;
  int dither;        // FP32: dithered plain tables for step `tick`
  int64_t tick;
};

struct SPassArgs {
  void* psi;        // field base
  void* out;        // SF_POWER: real power array, same layout as psi (1 component)
  double* part;     // MEASURE: one double per workgroup
  const void* tw;   // exp(-2 pi i m / N)
  const void* ph;   // [N] exp(-i k^2 dt / 2) / N
  int64_t sa;       // element stride along the axis
  int64_t inner;    // contiguous pencils per (field, outer)
  int64_t outer;
  int64_t outer_stride;
  int64_t nfield;   // 3*S (STEP, MEASURE) or S (SF)
  int64_t field_stride;
  double kscale;
  double power_scale;
  int lg_tiles, lg_outer;  // log2 of (inner / TX) and of outer, set by the launcher
  int reverse;      // STEP (streaming kernel): walk the work items from the last one
  int nt;           // STEP (streaming kernel): non-temporal stores of the field
  int64_t tick;     // STEP: index of the step in the call (dithered single-precision tables)
};

hipError_t launch_tables(hipStream_t st, bool dbl, void* ph, void* tw, int n, int ncomp, double dt, double q,
                         double dx);
// first_sample: index of the field's sample 0 in the whole ensemble (the
// generator's sample counter is first_sample + s)
hipError_t launch_init(hipStream_t st, bool dbl, void* psi, const Geom& g, uint64_t seed, uint64_t group,
                       uint64_t first_sample, double n0, double wigner_var);
// variant: step-pass variant index (0 = default), ignored by the other modes
// step-pass variant offset selecting the dithered plain FP32 tables (twiddles and phases)
constexpr int kPlainTwiddles = 3;
hipError_t launch_xpass(hipStream_t st, bool dbl, int mode, int n, const XPassArgs& a, int variant = 0);
hipError_t launch_spass(hipStream_t st, bool dbl, int mode, int n, const SPassArgs& a, int variant = 0);
int step_variants();
// largest pencil length the grouped x-pass takes
int grouped_x_max_n(bool dbl);
// work items of a group in the grouped x-pass
int64_t grouped_x_items(int n, int64_t pencils);
hipError_t launch_xpass_grouped(hipStream_t st, bool dbl, const XGroupArgs& a);
// 1D: K split steps of one pencil per workgroup in one launch (open_half: the
// first step opens with R(dt/2) instead of R(dt); close_half: closing R(dt/2))
// split: the latency form (three component groups per sample) instead of one
// thread group holding all three components
hipError_t launch_x1d_multi(hipStream_t st, bool dbl, int n, const XPassArgs& a, int K, double dt, bool open_half,
                            bool close_half, bool split);
// pot: trap potential [sites] or null
hipError_t launch_local(hipStream_t st, bool dbl, void* psi, int S, int64_t sites, double tau, double c0, double c1,
                        const double* pot);
// F_perp per site [S][sites] (field precision)
hipError_t launch_f_perp(hipStream_t st, bool dbl, const void* psi, int S, int64_t sites, void* out);
// per sample (mean |F_perp|, mean |F_perp|^2, Larmor-phase winding along x); part: S*rows*3 doubles
hipError_t launch_texture(hipStream_t st, bool dbl, const void* psi, int S, int64_t rows, int64_t sites, int n,
                          double* part, double* out);
// the paper's local sub-steps (4)-(5) over dt at every site
hipError_t launch_paper_local(hipStream_t st, bool dbl, void* psi, int S, int64_t sites, double dt, double c0,
                              double c1, double q, const double* pot);
hipError_t launch_bin(hipStream_t st, bool dbl, const void* power, int S, int64_t sites, const int32_t* perm,
                      const int32_t* offs, int nbins, double* out);
hipError_t launch_obs_finish(hipStream_t st, int S, const double* part_x, int64_t rows, const double* part_y,
                             int64_t ny_blocks, const double* part_z, int64_t nz_blocks, double cell, double* obs);

// reverse mode
hipError_t launch_fft1_x(hipStream_t st, bool dbl, int n, void* f, const void* tw, int64_t pencils);
int adj_local_blocks(int S, int64_t sites);
// which local-update VJPs k_adj_local applies at the state it is given
enum AdjLocalKind { ADJ_OPEN = 0, ADJ_CLOSE = 1, ADJ_OPEN_CLOSE = 2 };
hipError_t launch_adj_local(hipStream_t st, bool dbl, int kind, const void* state, void* h, int S, int64_t sites,
                            double tau, double c0, double c1, double dt, double* part);
hipError_t launch_adj_accum(hipStream_t st, const double* part, int nblocks, double* acc);
hipError_t launch_adj_spectrum(hipStream_t st, bool dbl, void* f, const Geom& g, const int32_t* offs, int nbins,
                               const double* dl_dbins);
hipError_t launch_adj_seed(hipStream_t st, bool dbl, const void* psi, const void* hf, void* h, int S, int64_t sites);
hipError_t launch_conj(hipStream_t st, bool dbl, const void* in, void* out, int64_t n);

// x-pass pencils per workgroup for axis length n (host copy of the kernel config)
int xpass_pencils(int n, bool dbl);

}  // namespace spin1
