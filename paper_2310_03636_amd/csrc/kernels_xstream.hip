// Streaming x-pass of the spin-1 step (gfx950) and its launcher.
#include "pass_common.hpp"

namespace spin1 {

// --------------------------------------------------------------------------
// Streaming (persistent) variants of the step passes.  A grid of about
// (CUs x resident workgroups) walks the work items with a stride of gridDim.x.
// The strided pass prefetches: while item i is transformed, the global loads
// of item i + gridDim.x are already in flight, so HBM traffic overlaps the FFT
// arithmetic even at one or two resident workgroups per CU.  Every item is
// owned by exactly one workgroup, so reading the next item early sees the
// pre-pass state.  The x-pass does not: without the second register set it
// fits three wavefronts per SIMD instead of two, and the other wavefronts
// cover its loads (measured 4-6% faster on 256- and 512-point pencils).
// Consecutive passes walk the items in opposite directions (the host sets
// `reverse` on every other pass), so each pass starts on the data the one
// before it wrote last, which the last-level cache still holds.
// --------------------------------------------------------------------------
// The twiddle and phase tables are staged in LDS once per workgroup: a global
// load issued after the prefetch could only be consumed once the whole
// prefetch had arrived (the vector-memory counter retires in order).
// PLAIN: the stage twiddles and phase factors held as plain complex values
// (FP32 only), rebuilt per launch as the dithered rounding of the FP64 value
// for the step index `tick` (dither_round): half the multiply cost and LDS of
// the hi+lo form, and no rounding that repeats identically in every step
// POT: the group has a trap potential (a separate instantiation, so that the
// common case keeps its register budget)
// Wavefronts per SIMD the register allocation must allow: three for the
// single-precision dithered-table form up to 1024 points (168 VGPRs; at 1024
// points one register is reloaded once per item, and the 128-thread variant 1
// cannot reach three), else whatever the allocation gives.
template <typename Real, int N, int V, bool PLAIN, bool POT>
constexpr int xstream_waves() {
  return (PLAIN && !POT && sizeof(Real) == 4 && (N <= 512 || (N == 1024 && V != 1))) ? 3 : 1;
}

template <typename Real, int N, int V, bool PLAIN, bool POT = false, bool ENABLED = XCfg<N, Real, V>::STREAM>
__global__ __launch_bounds__((XCfg<N, Real, V>::THREADS)) __attribute__((
    amdgpu_waves_per_eu(xstream_waves<Real, N, V, PLAIN, POT>()))) void k_xpass_stream(XPassArgs a, int64_t groups) {
 if constexpr (ENABLED) {
  using C = Cx<Real>;
  constexpr int R = XCfg<N, Real, V>::R, T = XCfg<N, Real, V>::T, P = XCfg<N, Real, V>::P;
  __shared__ C lds[P * RowPad<N, T>::ROW];
  using TW = StagedTwiddles<Real, N, R>;
  using TE = std::conditional_t<PLAIN, Cx<Real>, TabEntry<Real>>;
  using TWA = std::conditional_t<PLAIN, StagedTwiddlesPlain<Real, N, R>, TW>;
  __shared__ TE stw[TW::SIZE > 0 ? TW::SIZE : 1];
  // phase tables of m = +1 (equal to m = -1, q enters as q m^2) and m = 0
  using PE = std::conditional_t<PLAIN, Cx<Real>, TabEntry<Real>>;
  __shared__ PE ph[2 * N];
  const int t = threadIdx.x % T;
  // a pencil of a whole number of wavefronts has a wave-uniform index: held
  // in a scalar register, it makes the pencil's addresses scalar bases
  int p = threadIdx.x / T;
  if constexpr (T % 64 == 0) p = __builtin_amdgcn_readfirstlane(p);
  RowLds<Real, N, T, (T <= 64)> L{lds + p * RowPad<N, T>::ROW};
  {
    const TabEntry<Real>* gtw = static_cast<const TabEntry<Real>*>(a.tw);
    const TabEntry<Real>* gph = static_cast<const TabEntry<Real>*>(a.ph);
    for (int i = threadIdx.x; i < TW::SIZE; i += blockDim.x) {
      const TabEntry<Real> w = gtw[TW::exponent(i)];
      if constexpr (PLAIN)
        stw[i] = C{dither_round(w.hr, w.lr, a.tick, dither_salt(2 * i)),
                   dither_round(w.hi, w.li, a.tick, dither_salt(2 * i + 1))};
      else
        stw[i] = w;
    }
    for (int i = threadIdx.x; i < 2 * N; i += blockDim.x) {
      if constexpr (PLAIN)
        ph[i] = C{dither_round(gph[i].hr, gph[i].lr, a.tick, dither_salt(2 * (i + N))),
                  dither_round(gph[i].hi, gph[i].li, a.tick, dither_salt(2 * (i + N) + 1))};
      else
        ph[i] = gph[i];
    }
    __syncthreads();
  }
  C* psi = static_cast<C*>(a.psi);
  // out of place when a source field of the same layout is given
  const C* in = a.src ? static_cast<const C*>(a.src) : psi;
  const int64_t npen = int64_t(a.S) * a.rows;
  const Real c0 = Real(a.c0), c1 = Real(a.c1);
  // pencil pid: component m starts at ((s*3 + m) * sites + row * N); rows is a power of two
  auto comp_off = [&](int64_t pid, int m) -> int64_t {
    const int64_t s = pid >> a.lg_rows;
    return (s * 3 + m) * a.sites + (pid & (a.rows - 1)) * N;
  };
  auto load3 = [&](C (&dst)[3][R], int64_t pid) {
#pragma unroll
    for (int m = 0; m < 3; ++m) {
      const C* src = in + comp_off(pid, m);
#pragma unroll
      for (int e = 0; e < R; ++e) dst[m][e] = src[uint32_t(t + e * T)];
    }
  };
  int64_t g = blockIdx.x;
  if (g >= groups) return;
  for (; g < groups; g += gridDim.x) {
    int64_t pid = (a.reverse ? groups - 1 - g : g) * P + p;
    if constexpr (T % 64 == 0) pid = wave_uniform(pid);
    const bool active = pid < npen;
    C v[3][R];
    if (active) {
      // the loads of the item are issued at a raised wavefront priority, so
      // that they go out ahead of the other wavefronts' FFT arithmetic
      // (512^2 x 64: 155.7 -> 152.6 us per launch)
      __builtin_amdgcn_s_setprio(2);
      load3(v, pid);
      __builtin_amdgcn_s_setprio(0);
    } else {  // a pencil past the end: defined values, never stored
#pragma unroll
      for (int m = 0; m < 3; ++m)
#pragma unroll
        for (int e = 0; e < R; ++e) v[m][e] = C{Real(0), Real(0)};
    }
    const double* prow = POT ? a.pot + (pid & (a.rows - 1)) * N : nullptr;
    if (a.tau_pre != 0.0) local_update_sites<Real, R, T, POT ? POT_ALWAYS : POT_NEVER>(v, t, Real(a.tau_pre), c0, c1, prow, a.tau_pre);
#pragma unroll
    for (int m = 0; m < 3; ++m) fft_phase_ifft<Real, N, R>(v[m], t, L, TWA{stw}, ph + (m == 1 ? N : 0));
    if (a.tau_post != 0.0) local_update_sites<Real, R, T, POT ? POT_ALWAYS : POT_NEVER>(v, t, Real(a.tau_post), c0, c1, prow,
                                                                           a.tau_post);
    if (active) {
      if (a.nt) {
#pragma unroll
        for (int m = 0; m < 3; ++m) {
          C* dst = psi + comp_off(pid, m);
#pragma unroll
          for (int e = 0; e < R; ++e) put<true>(&dst[uint32_t(t + e * T)], v[m][e]);
        }
      } else {
#pragma unroll
        for (int m = 0; m < 3; ++m) {
          C* dst = psi + comp_off(pid, m);
#pragma unroll
          for (int e = 0; e < R; ++e) put<false>(&dst[uint32_t(t + e * T)], v[m][e]);
        }
      }
    }
  }
}
 }

// --------------------------------------------------------------------------
// launchers
// --------------------------------------------------------------------------
template <typename Real, int N, int V, bool PLAIN, bool POT = false>
static hipError_t xpass_stream_v(hipStream_t st, const XPassArgs& a) {
  constexpr int P = XCfg<N, Real, V>::P;
  const int64_t blocks = (int64_t(a.S) * a.rows + P - 1) / P;
  XPassArgs b = a;
  b.lg_rows = ilog2(a.rows);
  const int64_t grid = stream_grid(k_xpass_stream<Real, N, V, PLAIN, POT>, XCfg<N, Real, V>::THREADS, blocks);
  (void)launch_kernel((k_xpass_stream<Real, N, V, PLAIN, POT>), dim3(unsigned(grid)), dim3(XCfg<N, Real, V>::THREADS),
                     0, st, b, blocks);
  return hipGetLastError();
}

template <typename Real, int N, bool PLAIN>
static hipError_t xpass_stream_p(hipStream_t st, const XPassArgs& a, int v) {
  // variants whose tables no longer fit in LDS fall back to the default one
  if (v == 1 && XCfg<N, Real, 1>::STREAM) return xpass_stream_v<Real, N, 1, PLAIN>(st, a);
  if (v == 2 && XCfg<N, Real, 2>::STREAM) return xpass_stream_v<Real, N, 2, PLAIN>(st, a);
  return xpass_stream_v<Real, N, 0, PLAIN>(st, a);
}


template <typename Real, int N>
static hipError_t xstream_n(hipStream_t st, const XPassArgs& a, int variant) {
  if constexpr (XCfg<N, Real>::STREAM) {
    // a group with a trap potential runs the default variant, with the table
    // form the variant index asks for
    if (a.pot) {
      if constexpr (sizeof(Real) == 4)
        if (variant >= kPlainTwiddles) return xpass_stream_v<Real, N, 0, true, true>(st, a);
      return xpass_stream_v<Real, N, 0, false, true>(st, a);
    }
    if constexpr (sizeof(Real) == 4)
      if (variant >= kPlainTwiddles) return xpass_stream_p<Real, N, true>(st, a, variant - kPlainTwiddles);
    return xpass_stream_p<Real, N, false>(st, a, variant % kPlainTwiddles);
  } else {
    return hipErrorInvalidValue;
  }
}

template <typename Real>
static hipError_t xstream_t(hipStream_t st, int n, const XPassArgs& a, int v) {
  switch (n) {
    case 8: return xstream_n<Real, 8>(st, a, v);
    case 16: return xstream_n<Real, 16>(st, a, v);
    case 32: return xstream_n<Real, 32>(st, a, v);
    case 64: return xstream_n<Real, 64>(st, a, v);
    case 128: return xstream_n<Real, 128>(st, a, v);
    case 256: return xstream_n<Real, 256>(st, a, v);
    case 512: return xstream_n<Real, 512>(st, a, v);
    case 1024: return xstream_n<Real, 1024>(st, a, v);
    case 2048: return xstream_n<Real, 2048>(st, a, v);
    case 4096: return xstream_n<Real, 4096>(st, a, v);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_xpass_stream(hipStream_t st, bool dbl, int n, const XPassArgs& a, int variant) {
  return dbl ? xstream_t<double>(st, n, a, variant) : xstream_t<float>(st, n, a, variant);
}

}  // namespace spin1
