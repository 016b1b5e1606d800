// HIP kernels of the spin-1 split-step library for gfx950 (MI355X).
//
// One time step of the symmetric split R(dt/2) [K Q](dt) R(dt/2) is a
// sequence of streaming passes over the field [S][3][Nz][Ny][Nx]:
//   x-pass  (contiguous pencils, all three components of a site in one
//            thread): local update R(tau) -> FFT_x -> x-phase table (kinetic
//            x part, quadratic Zeeman q m^2, 1/Nx) -> inverse FFT_x;
//   y-, z-pass (strided pencils, one component per workgroup, a tile of TX
//            adjacent columns so every row of the tile is one contiguous
//            global segment): FFT -> axis phase table -> inverse FFT.
// The kinetic operator factorises exactly over axes (the Laplacian is a sum
// of per-axis second derivatives and the per-axis phases commute), so these
// passes reproduce the d-dimensional Eq. (3) step.
// The same pass skeletons also run forward-only transforms for the energy
// (MODE_MEASURE) and for the transverse-spin spectrum (MODE_SF*).
// This unit holds the non-streaming x-pass (every mode) and its dispatch;
// kernels_smodes.hip the strided counterpart, kernels_xstream.hip and
// kernels_sstream.hip the streaming step kernels, kernels_step.hip the grouped
// and multi-step kernels, kernels_aux.hip the rest.
#include "pass_common.hpp"

namespace spin1 {

int xpass_pencils(int n, bool dbl) {
  switch (n) {
    case 8: return dbl ? XCfg<8, double>::P : XCfg<8, float>::P;
    case 16: return dbl ? XCfg<16, double>::P : XCfg<16, float>::P;
    case 32: return dbl ? XCfg<32, double>::P : XCfg<32, float>::P;
    case 64: return dbl ? XCfg<64, double>::P : XCfg<64, float>::P;
    case 128: return dbl ? XCfg<128, double>::P : XCfg<128, float>::P;
    case 256: return dbl ? XCfg<256, double>::P : XCfg<256, float>::P;
    case 512: return dbl ? XCfg<512, double>::P : XCfg<512, float>::P;
    case 1024: return dbl ? XCfg<1024, double>::P : XCfg<1024, float>::P;
    case 2048: return dbl ? XCfg<2048, double>::P : XCfg<2048, float>::P;
    case 4096: return dbl ? XCfg<4096, double>::P : XCfg<4096, float>::P;
  }
  return 0;
}

template <typename Real>
static int spass_tx_t(int n) {
  switch (n) {
    case 8: return SCfg<8, Real>::TX;
    case 16: return SCfg<16, Real>::TX;
    case 32: return SCfg<32, Real>::TX;
    case 64: return SCfg<64, Real>::TX;
    case 128: return SCfg<128, Real>::TX;
    case 256: return SCfg<256, Real>::TX;
    case 512: return SCfg<512, Real>::TX;
    case 1024: return SCfg<1024, Real>::TX;
  }
  return 0;
}

int spass_tx(int n, bool dbl) { return dbl ? spass_tx_t<double>(n) : spass_tx_t<float>(n); }

// --------------------------------------------------------------------------
// x-pass: contiguous pencils, all 3 components of each site in one thread
// --------------------------------------------------------------------------
template <typename Real, int N, int MODE, bool STAGE_TW = false>
__global__ __launch_bounds__((XCfg<N, Real>::THREADS)) void k_xpass(XPassArgs a) {
  using C = Cx<Real>;
  constexpr int R = XCfg<N, Real>::R, T = XCfg<N, Real>::T, P = XCfg<N, Real>::P;
  __shared__ C lds[P * RowPad<N, T>::ROW];
  const int t = threadIdx.x % T;
  const int p = threadIdx.x / T;
  const int64_t pid = int64_t(blockIdx.x) * P + p;
  const bool active = pid < int64_t(a.S) * a.rows;
  const int64_t s = active ? pid / a.rows : 0;
  const int64_t row = active ? pid - s * a.rows : 0;
  RowLds<Real, N, T, (T <= 64)> L{lds + p * RowPad<N, T>::ROW};
  const TabEntry<Real>* tw = static_cast<const TabEntry<Real>*>(a.tw);
  // STAGE_TW: the twiddles are staged in LDS in stage order first.  Read from
  // global memory, every stage of every transform waits for its twiddle loads.
  // Taken for long pencils when there is at most one workgroup per CU
  // (nothing else covers those waits; with more workgroups the larger LDS
  // footprint costs more than it saves) and for the step-log pass at every
  // length (measured 22% faster on 256^3).
  using STW = StagedTwiddles<Real, N, R>;
  __shared__ TabEntry<Real> stw[STAGE_TW ? STW::SIZE : 1];
  if constexpr (STAGE_TW) {
    for (int i = threadIdx.x; i < STW::SIZE; i += blockDim.x) stw[i] = tw[STW::exponent(i)];
    __syncthreads();
  }
  const auto twa = [&] {
    if constexpr (STAGE_TW)
      return STW{stw};
    else
      return tw;
  }();
  const int64_t off = s * 3 * a.sites + row * N + t;
  C* base = static_cast<C*>(a.psi) + off;
  const C* in = (MODE == MODE_STEP && a.src) ? static_cast<const C*>(a.src) + off : base;

  C v[3][R];
#pragma unroll
  for (int m = 0; m < 3; ++m)
#pragma unroll
    for (int e = 0; e < R; ++e) v[m][e] = active ? in[m * a.sites + e * T] : C{Real(0), Real(0)};

  // trap potential of this pencil's row (x = t + e*T), or null
  const double* prow = a.pot ? a.pot + row * N : nullptr;
  if constexpr (MODE == MODE_STEP || MODE == MODE_STEP_LOG) {
    const Real c0 = Real(a.c0), c1 = Real(a.c1);
    if (a.tau_pre != 0.0) local_update_sites<Real, R, T, POT_IF_SET>(v, t, Real(a.tau_pre), c0, c1, prow, a.tau_pre);
    const TabEntry<Real>* ph = static_cast<const TabEntry<Real>*>(a.ph);
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    if constexpr (MODE == MODE_STEP_LOG) {
#pragma unroll
      for (int e = 0; e < R; ++e)
        site_sums(v[0][e], v[1][e], v[2][e], a.c0, a.c1, a.q, acc, prow ? prow[t + e * T] : 0.0);
#pragma unroll
      for (int m = 0; m < 3; ++m) {
        fft_pencil<Real, N, R>(v[m], t, L, twa);
#pragma unroll
        for (int e = 0; e < R; ++e) {
          const double kk = a.kscale * double(signed_k<N>(t + e * T));
          acc[3] += 0.5 * kk * kk * double(norm2(v[m][e]));
          v[m][e] = conj(mul_tab(v[m][e], ph[m * N + t + e * T]));
        }
        fft_pencil<Real, N, R>(v[m], t, L, twa);
#pragma unroll
        for (int e = 0; e < R; ++e) v[m][e] = conj(v[m][e]);
      }
      acc[3] *= 1.0 / double(N);
    } else {
#pragma unroll
      for (int m = 0; m < 3; ++m) fft_phase_ifft<Real, N, R>(v[m], t, L, twa, ph + m * N);
    }
    if (a.tau_post != 0.0) local_update_sites<Real, R, T, POT_IF_SET>(v, t, Real(a.tau_post), c0, c1, prow, a.tau_post);
    if (active) {
#pragma unroll
      for (int m = 0; m < 3; ++m)
#pragma unroll
        for (int e = 0; e < R; ++e) base[m * a.sites + e * T] = v[m][e];
    }
    if constexpr (MODE == MODE_STEP_LOG) pencil_sums_out<T>(acc, lds, p, t, active, a.part + pid * 4);
  } else if constexpr (MODE == MODE_PAPER) {
    const Real c0 = Real(a.c0), c1 = Real(a.c1), q = Real(a.q);
    auto local_all = [&](double dt) {
#pragma unroll
      for (int e = 0; e < R; ++e) {
        C site[3] = {v[0][e], v[1][e], v[2][e]};
        paper_local_update(site, Real(dt), c0, c1, q, prow ? pot_angle<Real>(prow[t + e * T], dt) : Real(0));
        v[0][e] = site[0];
        v[1][e] = site[1];
        v[2][e] = site[2];
      }
    };
    if (a.tau_pre != 0.0) local_all(a.tau_pre);
    // kinetic phase alone (the m = 0 row of the x table; q sits in D)
    const TabEntry<Real>* ph0 = static_cast<const TabEntry<Real>*>(a.ph) + N;
#pragma unroll
    for (int m = 0; m < 3; ++m) fft_phase_ifft<Real, N, R>(v[m], t, L, twa, ph0);
    if (a.tau_post != 0.0) local_all(a.tau_post);
    if (active) {
#pragma unroll
      for (int m = 0; m < 3; ++m)
#pragma unroll
        for (int e = 0; e < R; ++e) base[m * a.sites + e * T] = v[m][e];
    }
  } else if constexpr (MODE == MODE_MEASURE) {
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int e = 0; e < R; ++e)
      site_sums(v[0][e], v[1][e], v[2][e], a.c0, a.c1, a.q, acc, prow ? prow[t + e * T] : 0.0);
#pragma unroll
    for (int m = 0; m < 3; ++m) {
      fft_pencil<Real, N, R>(v[m], t, L, twa);
#pragma unroll
      for (int e = 0; e < R; ++e) {
        const double kk = a.kscale * double(signed_k<N>(t + e * T));
        acc[3] += 0.5 * kk * kk * double(norm2(v[m][e]));
      }
    }
    acc[3] *= 1.0 / double(N);
    pencil_sums_out<T>(acc, lds, p, t, active, a.part + pid * 4);
  } else {
    // transverse spin F_perp = sqrt2 (psi_1^* psi_0 + psi_0^* psi_-1), forward FFT along x
    const Real r2 = Real(1.41421356237309504880);
    C f[R];
#pragma unroll
    for (int e = 0; e < R; ++e) f[e] = scale(cmulc(v[0][e], v[1][e]) + cmulc(v[1][e], v[2][e]), r2);
    fft_pencil<Real, N, R>(f, t, L, twa);
    if (active) {
      const int64_t o = (s * a.rows + row) * N + t;
      if constexpr (MODE == MODE_SF) {
        C* out = static_cast<C*>(a.out) + o;
#pragma unroll
        for (int e = 0; e < R; ++e) out[e * T] = f[e];
      } else {
        Real* out = static_cast<Real*>(a.out) + o;
        const Real ps = Real(a.power_scale);
#pragma unroll
        for (int e = 0; e < R; ++e) out[e * T] = norm2(f[e]) * ps;
      }
    }
  }
}

// --------------------------------------------------------------------------
// launchers
// --------------------------------------------------------------------------
// variant: 0..2 the step-pass variant; + kPlainTwiddles for the dithered plain FP32 tables
template <typename Real, int N, int MODE>
static hipError_t xpass_n(hipStream_t st, const XPassArgs& a, int variant) {
  if constexpr (MODE == MODE_STEP && XCfg<N, Real>::STREAM) {
    return launch_xpass_stream(st, sizeof(Real) == 8, N, a, variant);
  } else {
    constexpr int P = XCfg<N, Real>::P;
    const int64_t blocks = (int64_t(a.S) * a.rows + P - 1) / P;
    if constexpr (N >= 2048 || (MODE == MODE_STEP_LOG && N > XCfg<N, Real>::R)) {
      if (MODE == MODE_STEP_LOG || blocks <= device_cus()) {
        (void)launch_kernel((k_xpass<Real, N, MODE, true>), dim3(unsigned(blocks)), dim3(XCfg<N, Real>::THREADS), 0,
                           st, a);
        return hipGetLastError();
      }
    }
    (void)launch_kernel((k_xpass<Real, N, MODE>), dim3(unsigned(blocks)), dim3(XCfg<N, Real>::THREADS), 0, st, a);
    return hipGetLastError();
  }
}

template <typename Real, int MODE>
static hipError_t xpass_mode(hipStream_t st, int n, const XPassArgs& a, int v) {
  switch (n) {
    case 8: return xpass_n<Real, 8, MODE>(st, a, v);
    case 16: return xpass_n<Real, 16, MODE>(st, a, v);
    case 32: return xpass_n<Real, 32, MODE>(st, a, v);
    case 64: return xpass_n<Real, 64, MODE>(st, a, v);
    case 128: return xpass_n<Real, 128, MODE>(st, a, v);
    case 256: return xpass_n<Real, 256, MODE>(st, a, v);
    case 512: return xpass_n<Real, 512, MODE>(st, a, v);
    case 1024: return xpass_n<Real, 1024, MODE>(st, a, v);
    case 2048: return xpass_n<Real, 2048, MODE>(st, a, v);
    case 4096: return xpass_n<Real, 4096, MODE>(st, a, v);
  }
  return hipErrorInvalidValue;
}

template <typename Real>
static hipError_t xpass_t(hipStream_t st, int mode, int n, const XPassArgs& a, int v) {
  switch (mode) {
    case MODE_STEP: return xpass_mode<Real, MODE_STEP>(st, n, a, v);
    case MODE_MEASURE: return xpass_mode<Real, MODE_MEASURE>(st, n, a, v);
    case MODE_SF: return xpass_mode<Real, MODE_SF>(st, n, a, v);
    case MODE_SF_POWER: return xpass_mode<Real, MODE_SF_POWER>(st, n, a, v);
    case MODE_STEP_LOG: return xpass_mode<Real, MODE_STEP_LOG>(st, n, a, v);
    case MODE_PAPER: return xpass_mode<Real, MODE_PAPER>(st, n, a, v);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_xpass(hipStream_t st, bool dbl, int mode, int n, const XPassArgs& a, int variant) {
  return dbl ? xpass_t<double>(st, mode, n, a, variant) : xpass_t<float>(st, mode, n, a, variant);
}

}  // namespace spin1
