// Streaming strided (y/z) pass of the spin-1 step (gfx950) and its launcher.
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
// PLAIN: plain complex twiddles and phase factors, dithered per step (FP32).
// NT: non-temporal stores of the field (a template parameter: a branch on the
// store form inside the kernel costs the wide tiles up to 90 registers).
template <typename Real, int N, int V, bool PLAIN, bool NT>
__global__ __launch_bounds__((SCfg<N, Real, V>::THREADS)) void k_spass_stream(SPassArgs a, int64_t items) {
  using C = Cx<Real>;
  constexpr int R = SCfg<N, Real, V>::R, T = SCfg<N, Real, V>::T, TX = SCfg<N, Real, V>::TX;
  constexpr int PITCH = SCfg<N, Real, V>::PITCH;
  __shared__ C lds[N * PITCH];
  using TE = std::conditional_t<PLAIN, Cx<Real>, TabEntry<Real>>;
  __shared__ TE tw[N];
  using PE = std::conditional_t<PLAIN, Cx<Real>, TabEntry<Real>>;
  __shared__ PE ph[N / 2 + 1];  // the phase is even in k
  const int c = threadIdx.x % TX;
  const int t = threadIdx.x / TX;
  const int64_t tiles = a.inner / TX;
  ColLds<Real, TX, PITCH> L{lds + c};
  {
    const TabEntry<Real>* gtw = static_cast<const TabEntry<Real>*>(a.tw);
    const TabEntry<Real>* gph = static_cast<const TabEntry<Real>*>(a.ph);
    for (int i = threadIdx.x; i < N; i += blockDim.x) {
      if constexpr (PLAIN)
        tw[i] = C{dither_round(gtw[i].hr, gtw[i].lr, a.tick, dither_salt(2 * i)),
                  dither_round(gtw[i].hi, gtw[i].li, a.tick, dither_salt(2 * i + 1))};
      else
        tw[i] = gtw[i];
    }
    for (int i = threadIdx.x; i <= N / 2; i += blockDim.x) {
      if constexpr (PLAIN)
        ph[i] = C{dither_round(gph[i].hr, gph[i].lr, a.tick, dither_salt(2 * (i + N))),
                  dither_round(gph[i].hi, gph[i].li, a.tick, dither_salt(2 * (i + N) + 1))};
      else
        ph[i] = gph[i];
    }
    __syncthreads();
  }
  // item -> (field f, outer o, tile): shifts, all three extents are powers of two
  char* psi = static_cast<char*>(a.psi);
  const uint32_t lane_off = uint32_t((c + int64_t(t) * a.sa) * int64_t(sizeof(C)));
  const uint32_t step_e = uint32_t(int64_t(T) * a.sa * int64_t(sizeof(C)));
  auto tile_base = [&](int64_t item) -> char* {
    if (a.reverse) item = items - 1 - item;
    const int64_t tile = item & (tiles - 1);
    const int64_t rest = item >> a.lg_tiles;
    const int64_t o = rest & (a.outer - 1), f = rest >> a.lg_outer;
    return psi + (f * a.field_stride + o * a.outer_stride + tile * TX) * int64_t(sizeof(C));
  };
  int64_t item = blockIdx.x;
  if (item >= items) return;
  C nxt[R];
  {
    const char* src = tile_base(item);
#pragma unroll
    for (int e = 0; e < R; ++e) nxt[e] = *reinterpret_cast<const C*>(src + (lane_off + uint32_t(e) * step_e));
  }
  for (; item < items; item += gridDim.x) {
    C v[R];
#pragma unroll
    for (int e = 0; e < R; ++e) v[e] = nxt[e];
    char* dst = tile_base(item);
    const int64_t next = item + gridDim.x;
    if (next < items) {
      const char* src = tile_base(next);
      if constexpr (SCfg<N, Real, V>::PRIO) __builtin_amdgcn_s_setprio(2);
#pragma unroll
      for (int e = 0; e < R; ++e) nxt[e] = *reinterpret_cast<const C*>(src + (lane_off + uint32_t(e) * step_e));
      if constexpr (SCfg<N, Real, V>::PRIO) __builtin_amdgcn_s_setprio(0);
    }
    fft_halfphase_ifft<Real, N, R>(v, t, L, static_cast<const TE*>(tw), static_cast<const PE*>(ph),
                                   static_cast<const PE*>(nullptr));
#pragma unroll
    for (int e = 0; e < R; ++e) put<NT>(reinterpret_cast<C*>(dst + (lane_off + uint32_t(e) * step_e)), v[e]);
  }
}

// --------------------------------------------------------------------------
// launchers
// --------------------------------------------------------------------------
template <typename Real, int N, int V, bool PLAIN>
static hipError_t spass_stream_v(hipStream_t st, const SPassArgs& a) {
  constexpr int TX = SCfg<N, Real, V>::TX;
  if (a.inner % TX != 0) return hipErrorInvalidValue;
  const int64_t blocks = a.nfield * a.outer * (a.inner / TX);
  SPassArgs b = a;
  b.lg_tiles = ilog2(a.inner / TX);
  b.lg_outer = ilog2(a.outer);
  if (a.nt) {
    const int64_t grid = stream_grid(k_spass_stream<Real, N, V, PLAIN, true>, SCfg<N, Real, V>::THREADS, blocks);
    (void)launch_kernel((k_spass_stream<Real, N, V, PLAIN, true>), dim3(unsigned(grid)),
                        dim3(SCfg<N, Real, V>::THREADS), 0, st, b, blocks);
  } else {
    const int64_t grid = stream_grid(k_spass_stream<Real, N, V, PLAIN, false>, SCfg<N, Real, V>::THREADS, blocks);
    (void)launch_kernel((k_spass_stream<Real, N, V, PLAIN, false>), dim3(unsigned(grid)),
                        dim3(SCfg<N, Real, V>::THREADS), 0, st, b, blocks);
  }
  return hipGetLastError();
}

template <typename Real, int N, bool PLAIN>
static hipError_t spass_stream_p(hipStream_t st, const SPassArgs& a, int v) {
  // a variant whose column tile does not divide the rows runs the default one
  if (v == 1 && a.inner % SCfg<N, Real, 1>::TX == 0) return spass_stream_v<Real, N, 1, PLAIN>(st, a);
  if (v == 2) return spass_stream_v<Real, N, 2, PLAIN>(st, a);
  return spass_stream_v<Real, N, 0, PLAIN>(st, a);
}


template <typename Real, int N>
static hipError_t sstream_n(hipStream_t st, const SPassArgs& a, int variant) {
  if constexpr (sizeof(Real) == 4)
    if (variant >= kPlainTwiddles) return spass_stream_p<Real, N, true>(st, a, variant - kPlainTwiddles);
  return spass_stream_p<Real, N, false>(st, a, variant % kPlainTwiddles);
}

template <typename Real>
static hipError_t sstream_t(hipStream_t st, int n, const SPassArgs& a, int v) {
  switch (n) {
    case 8: return sstream_n<Real, 8>(st, a, v);
    case 16: return sstream_n<Real, 16>(st, a, v);
    case 32: return sstream_n<Real, 32>(st, a, v);
    case 64: return sstream_n<Real, 64>(st, a, v);
    case 128: return sstream_n<Real, 128>(st, a, v);
    case 256: return sstream_n<Real, 256>(st, a, v);
    case 512: return sstream_n<Real, 512>(st, a, v);
    case 1024: return sstream_n<Real, 1024>(st, a, v);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_spass_stream(hipStream_t st, bool dbl, int n, const SPassArgs& a, int variant) {
  return dbl ? sstream_t<double>(st, n, a, variant) : sstream_t<float>(st, n, a, variant);
}

}  // namespace spin1
