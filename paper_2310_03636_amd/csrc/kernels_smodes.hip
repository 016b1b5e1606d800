// Non-streaming strided (y/z) pass of the spin-1 library (every mode) and its dispatch.
#include "pass_common.hpp"

namespace spin1 {

// --------------------------------------------------------------------------
// strided pass: TX adjacent pencils of one component, stride sa between
// consecutive pencil elements
// --------------------------------------------------------------------------
template <typename Real, int N, int MODE>
__global__ __launch_bounds__((SCfg<N, Real>::THREADS)) void k_spass(SPassArgs a) {
  using C = Cx<Real>;
  constexpr int R = SCfg<N, Real>::R, T = SCfg<N, Real>::T, TX = SCfg<N, Real>::TX;
  __shared__ C lds[N * (TX + 1)];
  const int c = threadIdx.x % TX;
  const int t = threadIdx.x / TX;
  const int64_t tiles = a.inner / TX;
  int64_t wg = blockIdx.x;
  const int64_t tile = wg % tiles;
  wg /= tiles;
  const int64_t o = wg % a.outer;
  const int64_t f = wg / a.outer;
  const int64_t off = f * a.field_stride + o * a.outer_stride + tile * TX + c;
  C* base = static_cast<C*>(a.psi) + off;
  ColLds<Real, TX> L{lds + c};
  const TabEntry<Real>* tw = static_cast<const TabEntry<Real>*>(a.tw);
  // the step-log pass stages its twiddles in LDS in stage order (read from
  // global memory, every stage waits for its twiddle loads)
  constexpr bool STAGE_TW = MODE == MODE_STEP_LOG && N > R;
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

  C v[R];
#pragma unroll
  for (int e = 0; e < R; ++e) v[e] = base[int64_t(t + e * T) * a.sa];

  if constexpr (MODE == MODE_STEP) {
    fft_phase_ifft<Real, N, R>(v, t, L, twa, static_cast<const TabEntry<Real>*>(a.ph));
#pragma unroll
    for (int e = 0; e < R; ++e) base[int64_t(t + e * T) * a.sa] = v[e];
  } else if constexpr (MODE == MODE_STEP_LOG) {
    const TabEntry<Real>* ph = static_cast<const TabEntry<Real>*>(a.ph);
    fft_pencil<Real, N, R>(v, t, L, twa);
    double acc = 0.0;
#pragma unroll
    for (int e = 0; e < R; ++e) {
      const double kk = a.kscale * double(signed_k<N>(t + e * T));
      acc += 0.5 * kk * kk * double(norm2(v[e]));
      v[e] = conj(mul_tab(v[e], ph[t + e * T]));
    }
    fft_pencil<Real, N, R>(v, t, L, twa);
#pragma unroll
    for (int e = 0; e < R; ++e) base[int64_t(t + e * T) * a.sa] = conj(v[e]);
    acc *= 1.0 / double(N);
    const double tot = block_sum(acc, reinterpret_cast<double*>(lds));
    if (threadIdx.x == 0) a.part[blockIdx.x] = tot;
  } else if constexpr (MODE == MODE_MEASURE) {
    fft_pencil<Real, N, R>(v, t, L, twa);
    double acc = 0.0;
#pragma unroll
    for (int e = 0; e < R; ++e) {
      const double kk = a.kscale * double(signed_k<N>(t + e * T));
      acc += 0.5 * kk * kk * double(norm2(v[e]));
    }
    acc *= 1.0 / double(N);
    const double tot = block_sum(acc, reinterpret_cast<double*>(lds));
    if (threadIdx.x == 0) a.part[blockIdx.x] = tot;
  } else if constexpr (MODE == MODE_SF) {
    fft_pencil<Real, N, R>(v, t, L, twa);
#pragma unroll
    for (int e = 0; e < R; ++e) base[int64_t(t + e * T) * a.sa] = v[e];
  } else {
    fft_pencil<Real, N, R>(v, t, L, twa);
    Real* out = static_cast<Real*>(a.out) + off;
    const Real ps = Real(a.power_scale);
#pragma unroll
    for (int e = 0; e < R; ++e) out[int64_t(t + e * T) * a.sa] = norm2(v[e]) * ps;
  }
}

// --------------------------------------------------------------------------
// launchers
// --------------------------------------------------------------------------
template <typename Real, int N, int MODE>
static hipError_t spass_n(hipStream_t st, const SPassArgs& a, int variant) {
  if constexpr (MODE == MODE_STEP && SCfg<N, Real>::STREAM) {
    return launch_spass_stream(st, sizeof(Real) == 8, N, a, variant);
  } else {
    constexpr int TX = SCfg<N, Real>::TX;
    if (a.inner % TX != 0) return hipErrorInvalidValue;
    const int64_t blocks = a.nfield * a.outer * (a.inner / TX);
    (void)launch_kernel((k_spass<Real, N, MODE>), dim3(unsigned(blocks)), dim3(SCfg<N, Real>::THREADS), 0, st, a);
    return hipGetLastError();
  }
}

template <typename Real, int MODE>
static hipError_t spass_mode(hipStream_t st, int n, const SPassArgs& a, int v) {
  switch (n) {
    case 8: return spass_n<Real, 8, MODE>(st, a, v);
    case 16: return spass_n<Real, 16, MODE>(st, a, v);
    case 32: return spass_n<Real, 32, MODE>(st, a, v);
    case 64: return spass_n<Real, 64, MODE>(st, a, v);
    case 128: return spass_n<Real, 128, MODE>(st, a, v);
    case 256: return spass_n<Real, 256, MODE>(st, a, v);
    case 512: return spass_n<Real, 512, MODE>(st, a, v);
    case 1024: return spass_n<Real, 1024, MODE>(st, a, v);
  }
  return hipErrorInvalidValue;
}

template <typename Real>
static hipError_t spass_t(hipStream_t st, int mode, int n, const SPassArgs& a, int v) {
  switch (mode) {
    case MODE_STEP: return spass_mode<Real, MODE_STEP>(st, n, a, v);
    case MODE_MEASURE: return spass_mode<Real, MODE_MEASURE>(st, n, a, v);
    case MODE_SF: return spass_mode<Real, MODE_SF>(st, n, a, v);
    case MODE_SF_POWER: return spass_mode<Real, MODE_SF_POWER>(st, n, a, v);
    case MODE_STEP_LOG: return spass_mode<Real, MODE_STEP_LOG>(st, n, a, v);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_spass(hipStream_t st, bool dbl, int mode, int n, const SPassArgs& a, int variant) {
  return dbl ? spass_t<double>(st, mode, n, a, variant) : spass_t<float>(st, mode, n, a, variant);
}

}  // namespace spin1
