// Elementwise and reduction kernels of the spin-1 library (local updates,
// tables, initial state, shells, observables, spin texture) and the kernels
// of reverse mode, with their launchers.
#include "pass_common.hpp"

namespace spin1 {

// --------------------------------------------------------------------------
// local update alone (closing half step of multi-dimensional grids); pot: the
// trap potential [sites] or null
// --------------------------------------------------------------------------
template <typename Real>
__global__ __launch_bounds__(256) void k_local(Cx<Real>* psi, int S, int64_t sites, Real tau, Real c0, Real c1,
                                               const double* pot, double tau_d) {
  const int64_t total = int64_t(S) * sites;
  for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < total; i += int64_t(gridDim.x) * blockDim.x) {
    const int64_t s = i / sites, x = i - s * sites;
    Cx<Real>* b = psi + s * 3 * sites + x;
    Cx<Real> site[3] = {b[0], b[sites], b[2 * sites]};
    local_update(site, tau, c0, c1);
    if (pot) potential_phase(site, pot_angle<Real>(pot[x], tau_d));
    b[0] = site[0];
    b[sites] = site[1];
    b[2 * sites] = site[2];
  }
}

// --------------------------------------------------------------------------
// Real-space transverse spin (Fig. 1): F_perp = sqrt2 (psi_1^* psi_0 + psi_0^* psi_-1)
// per site, and per x-row the FP64 sums of |F_perp|, |F_perp|^2 and of the
// Larmor-phase steps phi_L(x+1) - phi_L(x) taken in [-pi, pi) (periodic in x).
// --------------------------------------------------------------------------
template <typename Real>
__device__ __forceinline__ Cx<Real> f_perp_at(const Cx<Real>* psi, int64_t sites, int64_t i) {
  const Cx<Real> p1 = psi[i], p0 = psi[sites + i], pm = psi[2 * sites + i];
  return scale(cmulc(p1, p0) + cmulc(p0, pm), Real(1.41421356237309504880));
}

template <typename Real>
__global__ __launch_bounds__(256) void k_f_perp(const Cx<Real>* psi, int S, int64_t sites, Cx<Real>* out) {
  const int64_t total = int64_t(S) * sites;
  for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < total; i += int64_t(gridDim.x) * blockDim.x) {
    const int64_t s = i / sites, x = i - s * sites;
    out[i] = f_perp_at(psi + s * 3 * sites, sites, x);
  }
}

// one workgroup per x-row of N sites: part[row] = (sum |F|, sum |F|^2, sum of phase steps)
template <typename Real>
__global__ __launch_bounds__(256) void k_texture_rows(const Cx<Real>* psi, int64_t rows, int64_t sites, int n,
                                                      double* part) {
  __shared__ double scratch[8];
  const int64_t row = blockIdx.x;
  const int64_t s = row / rows, r = row - s * rows;
  const Cx<Real>* base = psi + s * 3 * sites;
  const int64_t x0 = r * n;
  constexpr double kTwoPi = 6.28318530717958647693;
  double a[3] = {0.0, 0.0, 0.0};
  for (int j = threadIdx.x; j < n; j += blockDim.x) {
    const Cx<Real> z = f_perp_at(base, sites, x0 + j);
    const Cx<Real> zn = f_perp_at(base, sites, x0 + (j + 1 == n ? 0 : j + 1));
    const double zr = double(z.re), zi = double(z.im);
    const double m2 = zr * zr + zi * zi;
    a[0] += sqrt(m2);
    a[1] += m2;
    double d = atan2(double(zn.im), double(zn.re)) - atan2(zi, zr);
    d -= kTwoPi * floor((d + 0.5 * kTwoPi) / kTwoPi);
    a[2] += d;
  }
  double tot[3];
  for (int i = 0; i < 3; ++i) tot[i] = block_sum(a[i], scratch);
  if (threadIdx.x == 0)
    for (int i = 0; i < 3; ++i) part[row * 3 + i] = tot[i];
}

// per sample, rows summed in order: (mean |F|, mean |F|^2, winding)
__global__ __launch_bounds__(256) void k_texture_finish(const double* part, int64_t rows, int64_t sites, double* out) {
  __shared__ double scratch[8];
  const int64_t s = blockIdx.x;
  double a[3] = {0.0, 0.0, 0.0};
  for (int64_t r = threadIdx.x; r < rows; r += blockDim.x)
    for (int i = 0; i < 3; ++i) a[i] += part[(s * rows + r) * 3 + i];
  double tot[3];
  for (int i = 0; i < 3; ++i) tot[i] = block_sum(a[i], scratch);
  if (threadIdx.x == 0) {
    out[s * 3 + 0] = tot[0] / double(sites);
    out[s * 3 + 1] = tot[1] / double(sites);
    out[s * 3 + 2] = tot[2] / 6.28318530717958647693;
  }
}

template <typename Real>
__global__ __launch_bounds__(256) void k_paper_local(Cx<Real>* psi, int S, int64_t sites, Real dt, Real c0, Real c1,
                                                     Real q, const double* pot, double dt_d) {
  const int64_t total = int64_t(S) * sites;
  for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < total; i += int64_t(gridDim.x) * blockDim.x) {
    const int64_t s = i / sites, x = i - s * sites;
    Cx<Real>* b = psi + s * 3 * sites + x;
    Cx<Real> site[3] = {b[0], b[sites], b[2 * sites]};
    paper_local_update(site, dt, c0, c1, q, pot ? pot_angle<Real>(pot[x], dt_d) : Real(0));
    b[0] = site[0];
    b[sites] = site[1];
    b[2 * sites] = site[2];
  }
}

// --------------------------------------------------------------------------
// phase and twiddle tables, computed in FP64 (hi + lo floats in single precision)
// ph[m][k] = exp(-i (k^2/2 + q m^2) dt) / N (m = +1, 0, -1 when ncomp = 3)
// tw[k]    = exp(-2 pi i k / N)
// --------------------------------------------------------------------------
template <typename Real>
__global__ void k_tables(TabEntry<Real>* ph, TabEntry<Real>* tw, int n, int ncomp, double dt, double q, double dx) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  const int js = k < n / 2 ? k : k - n;
  const double kk = 2.0 * M_PI * double(js) / (double(n) * dx);
  const double inv = 1.0 / double(n);
  for (int c = 0; c < ncomp; ++c) {
    const double m = ncomp == 3 ? double(1 - c) : 0.0;
    const double ang = (0.5 * kk * kk + q * m * m) * dt;
    double sn, cs;
    sincos(ang, &sn, &cs);
    store_tab(ph + c * n + k, cs * inv, -sn * inv);
  }
  double sn, cs;
  sincospi(-2.0 * double(k) / double(n), &sn, &cs);
  store_tab(tw + k, cs, sn);
}

// --------------------------------------------------------------------------
// Wigner initial state: psi_m = sqrt(n0) delta_{m0} + sqrt(w / (2 dx^d)) (g_re + i g_im),
// (g_re, g_im) by Box-Muller from Philox4x64-10(counter = (site, m, sample, group), key = (seed, 0))
// --------------------------------------------------------------------------
template <typename Real>
__global__ __launch_bounds__(256) void k_init(Cx<Real>* psi, int S, int64_t sites, uint64_t seed, uint64_t group,
                                              uint64_t first_sample, double amp, double sqrt_n0) {
  const int64_t total = int64_t(S) * 3 * sites;
  for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < total; i += int64_t(gridDim.x) * blockDim.x) {
    const int64_t x = i % sites;
    const int64_t sc = i / sites;
    const int64_t c = sc % 3, s = sc / 3;
    U64x4 ctr;
    ctr.v[0] = uint64_t(x);
    ctr.v[1] = uint64_t(c);
    ctr.v[2] = uint64_t(s) + first_sample;  // the sample's index in the whole ensemble
    ctr.v[3] = group;
    const U64x4 r = philox4x64_10(ctr, seed, 0ull);
    const double u1 = open_unit(r.v[0]), u2 = open_unit(r.v[1]);
    const double rad = sqrt(-2.0 * log(u1));
    double sn, cs;
    sincospi(2.0 * u2, &sn, &cs);
    double re = amp * rad * cs, im = amp * rad * sn;
    if (c == 1) re += sqrt_n0;
    psi[i] = Cx<Real>{Real(re), Real(im)};
  }
}

// --------------------------------------------------------------------------
// radial shells: one wavefront per (sample, shell), FP64 sum over the shell's
// modes (listed in perm[offs[b] .. offs[b+1])), fixed order -> deterministic
// --------------------------------------------------------------------------
template <typename Real>
__global__ __launch_bounds__(256) void k_bin(const Real* power, int64_t sites, const int32_t* perm,
                                             const int32_t* offs, int nbins, double* out) {
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int b = blockIdx.x * 4 + wave;
  const int64_t s = blockIdx.y;
  double acc = 0.0;
  int lo = 0, hi = 0;
  if (b < nbins) {
    lo = offs[b];
    hi = offs[b + 1];
    const Real* ps = power + s * sites;
    for (int i = lo + lane; i < hi; i += 64) acc += double(ps[perm[i]]);
  }
  acc = lane_group_sum<64>(acc);
  if (b < nbins && lane == 0) out[s * nbins + b] = hi > lo ? acc / double(hi - lo) : 0.0;
}

// --------------------------------------------------------------------------
// observables: per sample (N, Fz, E) from the per-pencil / per-workgroup partials
// --------------------------------------------------------------------------
// One workgroup of 1024 threads per sample (the sums of a 256^3 sample run over
// 10^5 partials; 256 threads took 166 us for eight samples, latency-bound).
__global__ __launch_bounds__(1024) void k_obs_finish(const double* part_x, int64_t rows, const double* part_y,
                                                     int64_t ny_blocks, const double* part_z, int64_t nz_blocks,
                                                     double cell, double* obs) {
  __shared__ double scratch[16];
  const int64_t s = blockIdx.x;
  double a[4] = {0.0, 0.0, 0.0, 0.0};
  for (int64_t r = threadIdx.x; r < rows; r += blockDim.x)
    for (int i = 0; i < 4; ++i) a[i] += part_x[(s * rows + r) * 4 + i];
  double ek = 0.0;
  if (part_y)
    for (int64_t r = threadIdx.x; r < ny_blocks; r += blockDim.x) ek += part_y[s * ny_blocks + r];
  if (part_z)
    for (int64_t r = threadIdx.x; r < nz_blocks; r += blockDim.x) ek += part_z[s * nz_blocks + r];
  double tot[5];
  for (int i = 0; i < 4; ++i) tot[i] = block_sum(a[i], scratch);
  tot[4] = block_sum(ek, scratch);
  if (threadIdx.x == 0) {
    obs[s * 3 + 0] = cell * tot[0];
    obs[s * 3 + 1] = cell * tot[1];
    obs[s * 3 + 2] = cell * (tot[2] + tot[3] + tot[4]);
  }
}

// --------------------------------------------------------------------------
// Reverse mode.  The backward sweep carries H = conj(G), G = dL/dRe + i dL/dIm:
// in this form the adjoint of the kinetic + Zeeman step K Q(dt) is K Q(dt)
// itself (the phase exp(-i(|k|^2/2 + q m^2) dt) is even in k, so
// (K Q(dt))^H G = conj(K Q(dt) conj(G))), and the forward pass kernels serve
// unchanged.  Only the local update needs its own VJP kernel.
// --------------------------------------------------------------------------
// One forward transform along x of a one-component field [S][rows][Nx].
template <typename Real, int N>
__global__ __launch_bounds__((XCfg<N, Real>::THREADS)) void k_fft1_x(Cx<Real>* f, const TabEntry<Real>* tw,
                                                                   int64_t pencils) {
  using C = Cx<Real>;
  constexpr int R = XCfg<N, Real>::R, T = XCfg<N, Real>::T, P = XCfg<N, Real>::P;
  __shared__ C lds[P * RowPad<N, T>::ROW];
  const int t = threadIdx.x % T;
  const int p = threadIdx.x / T;
  const int64_t pid = int64_t(blockIdx.x) * P + p;
  const bool active = pid < pencils;
  RowLds<Real, N, T, (T <= 64)> L{lds + p * RowPad<N, T>::ROW};
  C* base = f + (active ? pid : 0) * N + t;
  C v[R];
#pragma unroll
  for (int e = 0; e < R; ++e) v[e] = active ? base[e * T] : C{Real(0), Real(0)};
  fft_pencil<Real, N, R>(v, t, L, tw);
  if (active) {
#pragma unroll
    for (int e = 0; e < R; ++e) base[e * T] = v[e];
  }
}

// Local-update VJP over a whole field (tau = dt/2).
//  CLOSE (backward of a step's closing half): state = psi_{n+1} = R(tau) psi_b;
//    H in = conj(G) at psi_{n+1}, H out = conj(G) at psi_b; adds
//    tau Im<G, M psi_{n+1}> to dL/dc1 and dt sum_{m=+-1} Im<G_b, psi_b> to dL/dq.
//  OPEN (backward of a step's opening half): state = psi_n, psi_a = R(tau) psi_n;
//    H in = conj(G) at psi_a, H out = conj(G) at psi_n; adds tau Im<G, M psi_a>.
//  OPEN_CLOSE: the OPEN of step n followed by the CLOSE of step n - 1, both at
//    state = psi_n (the two halves meet there), in one read and write of H.
// Per-block FP64 partials (dL/dq, dL/dc1) go to part[2 * blockIdx.x + {0, 1}].
template <typename Real>
__device__ __forceinline__ void adj_half(const Cx<Real>* pin, const Cx<Real>* pout, const Cx<Real>* gout,
                                         Cx<Real>* gin, Real tau, Real c0, Real c1, double* dc1) {
  // dL/dc1 += tau Im<G_out, M psi_out>   (M is the same at input and output)
  const Cx<Real> g = cmulc(pout[0], pout[1]) + cmulc(pout[1], pout[2]);
  const Real fz = norm2(pout[0]) - norm2(pout[2]);
  Cx<Real> mp[3];
  apply_M(pout, mp, g, fz);
  double acc = 0.0;
#pragma unroll
  for (int m = 0; m < 3; ++m) acc += double(cmulc(gout[m], mp[m]).im);
  *dc1 += double(tau) * acc;
  local_update_vjp(pin, pout, gout, gin, tau, c0, c1);
}

template <typename Real, int KIND>
__global__ __launch_bounds__(256) void k_adj_local(const Cx<Real>* __restrict__ state, Cx<Real>* __restrict__ h,
                                                   int S, int64_t sites, Real tau, Real c0, Real c1, double dt,
                                                   double* part) {
  using C = Cx<Real>;
  __shared__ double scratch[8];
  const int64_t total = int64_t(S) * sites;
  double dq = 0.0, dc1 = 0.0;
  for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < total; i += int64_t(gridDim.x) * blockDim.x) {
    const int64_t s = i / sites, x = i - s * sites;
    const int64_t o = s * 3 * sites + x;
    const C st[3] = {state[o], state[o + sites], state[o + 2 * sites]};
    C g[3] = {conj(h[o]), conj(h[o + sites]), conj(h[o + 2 * sites])};
    if constexpr (KIND != ADJ_CLOSE) {
      // opening half: psi_a = R(tau) psi_n
      C pout[3] = {st[0], st[1], st[2]}, gin[3];
      local_update(pout, tau, c0, c1);
      adj_half(st, pout, g, gin, tau, c0, c1, &dc1);
#pragma unroll
      for (int m = 0; m < 3; ++m) g[m] = gin[m];
    }
    if constexpr (KIND != ADJ_OPEN) {
      // closing half: psi_b = R(-tau) psi_{n+1}
      C pin[3] = {st[0], st[1], st[2]}, gin[3];
      local_update(pin, -tau, c0, c1);
      adj_half(pin, st, g, gin, tau, c0, c1, &dc1);
      // q enters through exp(-i q m^2 dt) on m = +-1 in the step before: dt Im<G_b, psi_b>
      dq += dt * (double(cmulc(gin[0], pin[0]).im) + double(cmulc(gin[2], pin[2]).im));
#pragma unroll
      for (int m = 0; m < 3; ++m) g[m] = gin[m];
    }
    h[o] = conj(g[0]);
    h[o + sites] = conj(g[1]);
    h[o + 2 * sites] = conj(g[2]);
  }
  const double tq = block_sum(dq, scratch);
  const double tc = block_sum(dc1, scratch);
  if (threadIdx.x == 0) {
    part[2 * blockIdx.x] = tq;
    part[2 * blockIdx.x + 1] = tc;
  }
}

// acc[i] += sum_b part[2 b + i] (fixed order)
__global__ __launch_bounds__(256) void k_adj_accum(const double* part, int nblocks, double* acc) {
  __shared__ double scratch[8];
  double a0 = 0.0, a1 = 0.0;
  for (int b = threadIdx.x; b < nblocks; b += blockDim.x) {
    a0 += part[2 * b];
    a1 += part[2 * b + 1];
  }
  const double t0 = block_sum(a0, scratch);
  const double t1 = block_sum(a1, scratch);
  if (threadIdx.x == 0) {
    acc[0] += t0;
    acc[1] += t1;
  }
}

// shell of a mode (same rule as the host tables): b = floor((isqrt(4J) + 1) / 2)
__device__ __forceinline__ int mode_shell(int64_t site, int dim, int n0, int n1, int n2) {
  const int n[3] = {n0, n1, n2};
  int nm = n0;
  if (dim > 1 && n1 > nm) nm = n1;
  if (dim > 2 && n2 > nm) nm = n2;
  int64_t J = 0, rest = site;
  for (int a = 0; a < dim; ++a) {
    const int64_t j = rest % n[a];
    rest /= n[a];
    const int64_t js = (j < n[a] / 2 ? j : j - n[a]) * (nm / n[a]);
    J += js * js;
  }
  int64_t r = int64_t(sqrt(double(4 * J)));
  while (r > 0 && r * r > 4 * J) --r;
  while ((r + 1) * (r + 1) <= 4 * J) ++r;
  return int((r + 1) / 2);
}

// Seed of the backward sweep in spectral space: with P_s(k) = |Fhat_s(k)|^2 / N
// and S_{s,b} the mean of P_s over shell b, H(Fhat) = 2 (dL/dS_{s,b} / count_b) conj(Fhat) / N.
template <typename Real>
__global__ __launch_bounds__(256) void k_adj_spectrum(Cx<Real>* f, int S, int64_t sites, int dim, int n0, int n1,
                                                      int n2, const int32_t* offs, int nbins, const double* dl_dbins) {
  const int64_t total = int64_t(S) * sites;
  for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < total; i += int64_t(gridDim.x) * blockDim.x) {
    const int64_t s = i / sites, x = i - s * sites;
    const int b = mode_shell(x, dim, n0, n1, n2);
    const double cnt = double(offs[b + 1] - offs[b]);
    const double w = 2.0 * dl_dbins[s * nbins + b] / (cnt * double(sites));
    f[i] = scale(conj(f[i]), Real(w));
  }
}

// H(psi) from H(F_perp) (both conj of real gradients): F_perp = sqrt2 (psi_1^* psi_0 + psi_0^* psi_-1)
//   H_1 = sqrt2 conj(H_F psi_0),  H_0 = sqrt2 (H_F conj(psi_1) + conj(H_F psi_-1)),  H_-1 = sqrt2 H_F conj(psi_0)
template <typename Real>
__global__ __launch_bounds__(256) void k_adj_seed(const Cx<Real>* __restrict__ psi, const Cx<Real>* __restrict__ hf,
                                                  Cx<Real>* __restrict__ h, int S, int64_t sites) {
  const int64_t total = int64_t(S) * sites;
  const Real r2 = Real(1.41421356237309504880);
  for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < total; i += int64_t(gridDim.x) * blockDim.x) {
    const int64_t s = i / sites, x = i - s * sites;
    const int64_t o = s * 3 * sites + x;
    const Cx<Real> p1 = psi[o], p0 = psi[o + sites], pm = psi[o + 2 * sites];
    const Cx<Real> H = hf[i];
    h[o] = scale(conj(H * p0), r2);
    h[o + sites] = scale(H * conj(p1) + conj(H * pm), r2);
    h[o + 2 * sites] = scale(H * conj(p0), r2);
  }
}

// out = conj(in), elementwise over n complex values
template <typename Real>
__global__ __launch_bounds__(256) void k_conj(const Cx<Real>* in, Cx<Real>* out, int64_t n) {
  for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += int64_t(gridDim.x) * blockDim.x)
    out[i] = conj(in[i]);
}

// --------------------------------------------------------------------------
// launchers
// --------------------------------------------------------------------------
hipError_t launch_tables(hipStream_t st, bool dbl, void* ph, void* tw, int n, int ncomp, double dt, double q,
                         double dx) {
  const unsigned blocks = unsigned((n + 255) / 256);
  if (dbl)
    (void)launch_kernel(k_tables<double>, dim3(blocks), dim3(256), 0, st, static_cast<TabEntry<double>*>(ph),
                       static_cast<TabEntry<double>*>(tw), n, ncomp, dt, q, dx);
  else
    (void)launch_kernel(k_tables<float>, dim3(blocks), dim3(256), 0, st, static_cast<TabEntry<float>*>(ph),
                       static_cast<TabEntry<float>*>(tw), n, ncomp, dt, q, dx);
  return hipGetLastError();
}

hipError_t launch_init(hipStream_t st, bool dbl, void* psi, const Geom& g, uint64_t seed, uint64_t group,
                       uint64_t first_sample, double n0, double wigner_var) {
  const double cell = g.dim == 1 ? g.dx : (g.dim == 2 ? g.dx * g.dx : g.dx * g.dx * g.dx);
  const double amp = sqrt(wigner_var / (2.0 * cell));
  const unsigned blocks = grid_for(int64_t(g.S) * 3 * g.sites, 256);
  if (dbl)
    (void)launch_kernel(k_init<double>, dim3(blocks), dim3(256), 0, st, static_cast<Cx<double>*>(psi), g.S, g.sites,
                       seed, group, first_sample, amp, sqrt(n0));
  else
    (void)launch_kernel(k_init<float>, dim3(blocks), dim3(256), 0, st, static_cast<Cx<float>*>(psi), g.S, g.sites,
                       seed, group, first_sample, amp, sqrt(n0));
  return hipGetLastError();
}

hipError_t launch_local(hipStream_t st, bool dbl, void* psi, int S, int64_t sites, double tau, double c0, double c1,
                        const double* pot) {
  const unsigned blocks = grid_for(int64_t(S) * sites, 256);
  if (dbl)
    (void)launch_kernel(k_local<double>, dim3(blocks), dim3(256), 0, st, static_cast<Cx<double>*>(psi), S, sites, tau,
                       c0, c1, pot, tau);
  else
    (void)launch_kernel(k_local<float>, dim3(blocks), dim3(256), 0, st, static_cast<Cx<float>*>(psi), S, sites,
                       float(tau), float(c0), float(c1), pot, tau);
  return hipGetLastError();
}

hipError_t launch_paper_local(hipStream_t st, bool dbl, void* psi, int S, int64_t sites, double dt, double c0,
                              double c1, double q, const double* pot) {
  const unsigned blocks = grid_for(int64_t(S) * sites, 256);
  if (dbl)
    (void)launch_kernel(k_paper_local<double>, dim3(blocks), dim3(256), 0, st, static_cast<Cx<double>*>(psi), S, sites,
                       dt, c0, c1, q, pot, dt);
  else
    (void)launch_kernel(k_paper_local<float>, dim3(blocks), dim3(256), 0, st, static_cast<Cx<float>*>(psi), S, sites,
                       float(dt), float(c0), float(c1), float(q), pot, dt);
  return hipGetLastError();
}

hipError_t launch_f_perp(hipStream_t st, bool dbl, const void* psi, int S, int64_t sites, void* out) {
  const unsigned blocks = grid_for(int64_t(S) * sites, 256);
  if (dbl)
    (void)launch_kernel(k_f_perp<double>, dim3(blocks), dim3(256), 0, st, static_cast<const Cx<double>*>(psi), S,
                       sites, static_cast<Cx<double>*>(out));
  else
    (void)launch_kernel(k_f_perp<float>, dim3(blocks), dim3(256), 0, st, static_cast<const Cx<float>*>(psi), S, sites,
                       static_cast<Cx<float>*>(out));
  return hipGetLastError();
}

hipError_t launch_texture(hipStream_t st, bool dbl, const void* psi, int S, int64_t rows, int64_t sites, int n,
                          double* part, double* out) {
  const unsigned blocks = unsigned(int64_t(S) * rows);
  if (dbl)
    (void)launch_kernel(k_texture_rows<double>, dim3(blocks), dim3(256), 0, st, static_cast<const Cx<double>*>(psi),
                       rows, sites, n, part);
  else
    (void)launch_kernel(k_texture_rows<float>, dim3(blocks), dim3(256), 0, st, static_cast<const Cx<float>*>(psi),
                       rows, sites, n, part);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  (void)launch_kernel(k_texture_finish, dim3(unsigned(S)), dim3(256), 0, st, part, rows, sites, out);
  return hipGetLastError();
}

hipError_t launch_bin(hipStream_t st, bool dbl, const void* power, int S, int64_t sites, const int32_t* perm,
                      const int32_t* offs, int nbins, double* out) {
  const dim3 grid(unsigned((nbins + 3) / 4), unsigned(S));
  if (dbl)
    (void)launch_kernel(k_bin<double>, grid, dim3(256), 0, st, static_cast<const double*>(power), sites, perm, offs,
                       nbins, out);
  else
    (void)launch_kernel(k_bin<float>, grid, dim3(256), 0, st, static_cast<const float*>(power), sites, perm, offs,
                       nbins, out);
  return hipGetLastError();
}

hipError_t launch_obs_finish(hipStream_t st, int S, const double* part_x, int64_t rows, const double* part_y,
                             int64_t ny_blocks, const double* part_z, int64_t nz_blocks, double cell, double* obs) {
  (void)launch_kernel(k_obs_finish, dim3(unsigned(S)), dim3(1024), 0, st, part_x, rows, part_y, ny_blocks, part_z,
                     nz_blocks, cell, obs);
  return hipGetLastError();
}


template <typename Real, int N>
static hipError_t fft1_n(hipStream_t st, void* f, const void* tw, int64_t pencils) {
  constexpr int P = XCfg<N, Real>::P;
  const int64_t blocks = (pencils + P - 1) / P;
  (void)launch_kernel((k_fft1_x<Real, N>), dim3(unsigned(blocks)), dim3(XCfg<N, Real>::THREADS), 0, st,
                     static_cast<Cx<Real>*>(f), static_cast<const TabEntry<Real>*>(tw), pencils);
  return hipGetLastError();
}

template <typename Real>
static hipError_t fft1_t(hipStream_t st, int n, void* f, const void* tw, int64_t pencils) {
  switch (n) {
    case 8: return fft1_n<Real, 8>(st, f, tw, pencils);
    case 16: return fft1_n<Real, 16>(st, f, tw, pencils);
    case 32: return fft1_n<Real, 32>(st, f, tw, pencils);
    case 64: return fft1_n<Real, 64>(st, f, tw, pencils);
    case 128: return fft1_n<Real, 128>(st, f, tw, pencils);
    case 256: return fft1_n<Real, 256>(st, f, tw, pencils);
    case 512: return fft1_n<Real, 512>(st, f, tw, pencils);
    case 1024: return fft1_n<Real, 1024>(st, f, tw, pencils);
    case 2048: return fft1_n<Real, 2048>(st, f, tw, pencils);
    case 4096: return fft1_n<Real, 4096>(st, f, tw, pencils);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_fft1_x(hipStream_t st, bool dbl, int n, void* f, const void* tw, int64_t pencils) {
  return dbl ? fft1_t<double>(st, n, f, tw, pencils) : fft1_t<float>(st, n, f, tw, pencils);
}

int adj_local_blocks(int S, int64_t sites) { return int(grid_for(int64_t(S) * sites, 256)); }

template <typename Real, int KIND>
static void adj_local_t(hipStream_t st, unsigned blocks, const void* state, void* h, int S, int64_t sites, double tau,
                        double c0, double c1, double dt, double* part) {
  (void)launch_kernel((k_adj_local<Real, KIND>), dim3(blocks), dim3(256), 0, st, static_cast<const Cx<Real>*>(state),
                     static_cast<Cx<Real>*>(h), S, sites, Real(tau), Real(c0), Real(c1), dt, part);
}

hipError_t launch_adj_local(hipStream_t st, bool dbl, int kind, const void* state, void* h, int S, int64_t sites,
                            double tau, double c0, double c1, double dt, double* part) {
  const unsigned blocks = grid_for(int64_t(S) * sites, 256);
  if (kind != ADJ_OPEN && kind != ADJ_CLOSE && kind != ADJ_OPEN_CLOSE) return hipErrorInvalidValue;
  auto run = [&](auto tag) {
    using Real = decltype(tag);
    if (kind == ADJ_OPEN)
      adj_local_t<Real, ADJ_OPEN>(st, blocks, state, h, S, sites, tau, c0, c1, dt, part);
    else if (kind == ADJ_CLOSE)
      adj_local_t<Real, ADJ_CLOSE>(st, blocks, state, h, S, sites, tau, c0, c1, dt, part);
    else
      adj_local_t<Real, ADJ_OPEN_CLOSE>(st, blocks, state, h, S, sites, tau, c0, c1, dt, part);
  };
  if (dbl)
    run(double{});
  else
    run(float{});
  return hipGetLastError();
}

hipError_t launch_adj_accum(hipStream_t st, const double* part, int nblocks, double* acc) {
  (void)launch_kernel(k_adj_accum, dim3(1), dim3(256), 0, st, part, nblocks, acc);
  return hipGetLastError();
}

hipError_t launch_adj_spectrum(hipStream_t st, bool dbl, void* f, const Geom& g, const int32_t* offs, int nbins,
                               const double* dl_dbins) {
  const unsigned blocks = grid_for(int64_t(g.S) * g.sites, 256);
  if (dbl)
    (void)launch_kernel(k_adj_spectrum<double>, dim3(blocks), dim3(256), 0, st, static_cast<Cx<double>*>(f), g.S,
                       g.sites, g.dim, g.n[0], g.n[1], g.n[2], offs, nbins, dl_dbins);
  else
    (void)launch_kernel(k_adj_spectrum<float>, dim3(blocks), dim3(256), 0, st, static_cast<Cx<float>*>(f), g.S,
                       g.sites, g.dim, g.n[0], g.n[1], g.n[2], offs, nbins, dl_dbins);
  return hipGetLastError();
}

hipError_t launch_adj_seed(hipStream_t st, bool dbl, const void* psi, const void* hf, void* h, int S, int64_t sites) {
  const unsigned blocks = grid_for(int64_t(S) * sites, 256);
  if (dbl)
    (void)launch_kernel(k_adj_seed<double>, dim3(blocks), dim3(256), 0, st, static_cast<const Cx<double>*>(psi),
                       static_cast<const Cx<double>*>(hf), static_cast<Cx<double>*>(h), S, sites);
  else
    (void)launch_kernel(k_adj_seed<float>, dim3(blocks), dim3(256), 0, st, static_cast<const Cx<float>*>(psi),
                       static_cast<const Cx<float>*>(hf), static_cast<Cx<float>*>(h), S, sites);
  return hipGetLastError();
}

hipError_t launch_conj(hipStream_t st, bool dbl, const void* in, void* out, int64_t n) {
  const unsigned blocks = grid_for(n, 256);
  if (dbl)
    (void)launch_kernel(k_conj<double>, dim3(blocks), dim3(256), 0, st, static_cast<const Cx<double>*>(in),
                       static_cast<Cx<double>*>(out), n);
  else
    (void)launch_kernel(k_conj<float>, dim3(blocks), dim3(256), 0, st, static_cast<const Cx<float>*>(in),
                       static_cast<Cx<float>*>(out), n);
  return hipGetLastError();
}

}  // namespace spin1
