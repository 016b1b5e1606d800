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
#include "device_math.hpp"
#include "internal.hpp"

namespace spin1 {

// --------------------------------------------------------------------------
// launch configurations
// --------------------------------------------------------------------------
// x-pass: radix R, N/R threads per pencil, P pencils per workgroup; STREAM
// selects the persistent streaming kernel for the step pass.  V picks one of
// the step-pass variants the autotuner times: workgroups of about 256 (V = 0),
// 128 (V = 1) or 512 (V = 2) threads.
template <int N, typename Real, int V = 0>
struct XCfg {
  // radix 16 only where 3 x 16 single-precision values per thread still fit
  static constexpr int R = N <= 8 ? N : ((N <= 1024 || sizeof(Real) == 8) ? 8 : 16);
  static constexpr int T = N / R;
  static constexpr int TARGET = V == 1 ? 128 : (V == 2 ? 512 : 256);
  static constexpr int P = T >= TARGET ? 1 : TARGET / T;
  static constexpr int THREADS = T * P;
  // the streaming kernel keeps twiddles and two phase tables in LDS
  static constexpr int STREAM_LDS = P * (N + N / 16) * int(sizeof(Cx<Real>)) + 3 * N * 16;
  static constexpr bool STREAM = STREAM_LDS <= 96 * 1024;
};

// strided pass: radix R, TX adjacent columns per workgroup (TX x N/R threads).
// Step-pass variants: V = 0 the default, V = 1 half the columns (radix 16 on 512
// and radix 32 on 1024 for FP32), V = 2 radix 8.
template <int N, typename Real, int V = 0>
struct SCfg {
  static constexpr int R0 = N <= 8 ? N : (N <= 128 ? 8 : 16);
  // FP32 columns of 512: radix 32 by default (two stages, one LDS exchange per
  // transform), variant 1 is radix 16 on the full 16-column tile
  // and variant 1 of FP32 columns of 1024 is radix 32 on a 16-column tile
  static constexpr bool C512 = N == 512 && sizeof(Real) == 4;
  static constexpr bool C1024 = N == 1024 && sizeof(Real) == 4;
  static constexpr bool R32 = (V == 0 && C512) || (V == 1 && C1024);
  static constexpr int R = (V == 2 && N >= 64) ? 8 : (R32 ? 32 : R0);
  static constexpr int T = N / R;
  static constexpr int CB = int(sizeof(Cx<Real>));
  static constexpr int TXRAW = 65536 / (N * CB);
  static constexpr int TX0 = TXRAW >= 16 ? 16 : (TXRAW >= 8 ? 8 : 4);
  static constexpr int TX1 = (V == 1 && C1024) ? 16 : ((V == 1 && TX0 > 4 && !C512) ? TX0 / 2 : TX0);
  // keep workgroups within 1024 threads
  static constexpr int TX = TX1 * T > 1024 ? 1024 / T : TX1;
  static constexpr int THREADS = TX * T;
  static constexpr bool STREAM = true;
};

constexpr int kStepVariants = 3;
static_assert(kPlainTwiddles == kStepVariants, "plain-twiddle variants follow the compensated ones");

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
// LDS views used by the FFT stages
// --------------------------------------------------------------------------
// One pencil per row with one padding element after every 16 (measured best
// on gfx950 for the radix-8 exchanges: it breaks up the power-of-two strides
// of the early stages across LDS banks).
template <int N, int T>
struct RowPad {
  static constexpr int ROW = N + N / 16;
  __device__ static __forceinline__ int at(int i) { return i + (i >> 4); }
};

// LDS ordering among the lanes of one wavefront: LDS instructions of a wave
// execute in issue order, so the exchange only needs the compiler to keep the
// stores before the loads (fences at wavefront scope around a wave barrier).
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// WAVE: every pencil lies inside one wavefront (N/R <= 64), so its exchanges
// synchronise only that wavefront; otherwise the whole workgroup.
template <typename Real, int N, int T, bool WAVE>
struct RowLds {
  Cx<Real>* row;
  __device__ __forceinline__ void store(int i, Cx<Real> v) { row[RowPad<N, T>::at(i)] = v; }
  __device__ __forceinline__ Cx<Real> load(int i) const { return row[RowPad<N, T>::at(i)]; }
  __device__ __forceinline__ void sync() {
    if constexpr (WAVE)
      wave_sync();
    else
      __syncthreads();
  }
};

// Column tiles: element i of column c at i * (TX + 1) + c; the odd row pitch
// spreads rows that differ by a power of two over different banks.
template <typename Real, int TX>
struct ColLds {
  static constexpr int PITCH = TX >= 16 ? TX : TX + 1;
  Cx<Real>* col;
  __device__ __forceinline__ void store(int i, Cx<Real> v) { col[i * PITCH] = v; }
  __device__ __forceinline__ Cx<Real> load(int i) const { return col[i * PITCH]; }
  __device__ __forceinline__ void sync() { __syncthreads(); }
};

// signed wavenumber index of DFT bin k
template <int N>
__device__ __forceinline__ int signed_k(int k) {
  return k < N / 2 ? k : k - N;
}

// sum over the T consecutive lanes of a pencil (T a power of two <= 64)
template <int T>
__device__ __forceinline__ double lane_group_sum(double v) {
#pragma unroll
  for (int off = T / 2; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// workgroup sum, fixed order; scratch must hold blockDim/64 doubles and may
// alias LDS that is no longer in use.  Result valid in thread 0.  Workgroups
// smaller than a wavefront shuffle only among their own lanes.
__device__ __forceinline__ double block_sum(double v, double* scratch) {
  const int width = blockDim.x < 64 ? int(blockDim.x) : 64;
  for (int off = width / 2; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int nw = (blockDim.x + 63) >> 6;
  __syncthreads();
  if (lane == 0) scratch[wave] = v;
  __syncthreads();
  double s = 0.0;
  if (threadIdx.x == 0)
    for (int w = 0; w < nw; ++w) s += scratch[w];
  return s;
}

// FP64 site sums of the observables: n, F_z and the local energy density
// c0/2 n^2 + c1/2 |F|^2 + q (|psi_1|^2 + |psi_-1|^2) (acc[0..2])
template <typename Real>
__device__ __forceinline__ void site_sums(Cx<Real> p1, Cx<Real> p0, Cx<Real> pm, double c0, double c1, double q,
                                          double* acc) {
  const double d1 = double(norm2(p1)), d0 = double(norm2(p0)), dm = double(norm2(pm));
  const Cx<Real> g = cmulc(p1, p0) + cmulc(p0, pm);
  const double gre = double(g.re), gim = double(g.im);
  const double n = d1 + d0 + dm, fz = d1 - dm;
  const double f2 = 2.0 * (gre * gre + gim * gim) + fz * fz;
  acc[0] += n;
  acc[1] += fz;
  acc[2] += 0.5 * c0 * n * n + 0.5 * c1 * f2 + q * (d1 + dm);
}

// Sum acc[0..3] over the T threads of pencil p and write the four totals to
// out (thread t = 0 of an active pencil).  Every thread of the workgroup
// calls it (it may synchronise the workgroup and reuse the pencil LDS).
template <int T, typename Real>
__device__ __forceinline__ void pencil_sums_out(const double* acc, Cx<Real>* lds, int p, int t, bool active,
                                                double* out) {
  double tot[4];
  if constexpr (T <= 64) {
#pragma unroll
    for (int i = 0; i < 4; ++i) tot[i] = lane_group_sum<T>(acc[i]);
  } else {
    constexpr int NW = T / 64;
    double* scratch = reinterpret_cast<double*>(lds);
    __syncthreads();
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const double w = lane_group_sum<64>(acc[i]);
      if ((t & 63) == 0) scratch[(p * NW + (t >> 6)) * 4 + i] = w;
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      double sacc = 0.0;
      for (int w = 0; w < NW; ++w) sacc += scratch[(p * NW + w) * 4 + i];
      tot[i] = sacc;
    }
  }
  if (active && t == 0) {
#pragma unroll
    for (int i = 0; i < 4; ++i) out[i] = tot[i];
  }
}

// --------------------------------------------------------------------------
// x-pass: contiguous pencils, all 3 components of each site in one thread
// --------------------------------------------------------------------------
template <typename Real, int N, int MODE>
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
  C* base = static_cast<C*>(a.psi) + s * 3 * a.sites + row * N + t;

  C v[3][R];
#pragma unroll
  for (int m = 0; m < 3; ++m)
#pragma unroll
    for (int e = 0; e < R; ++e) v[m][e] = active ? base[m * a.sites + e * T] : C{Real(0), Real(0)};

  if constexpr (MODE == MODE_STEP || MODE == MODE_STEP_LOG) {
    const Real c0 = Real(a.c0), c1 = Real(a.c1);
    if (a.tau_pre != 0.0) {
      const Real tau = Real(a.tau_pre);
#pragma unroll
      for (int e = 0; e < R; ++e) {
        C site[3] = {v[0][e], v[1][e], v[2][e]};
        local_update(site, tau, c0, c1);
        v[0][e] = site[0];
        v[1][e] = site[1];
        v[2][e] = site[2];
      }
    }
    const TabEntry<Real>* ph = static_cast<const TabEntry<Real>*>(a.ph);
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    if constexpr (MODE == MODE_STEP_LOG) {
#pragma unroll
      for (int e = 0; e < R; ++e) site_sums(v[0][e], v[1][e], v[2][e], a.c0, a.c1, a.q, acc);
#pragma unroll
      for (int m = 0; m < 3; ++m) {
        fft_pencil<Real, N, R>(v[m], t, L, tw);
#pragma unroll
        for (int e = 0; e < R; ++e) {
          const double kk = a.kscale * double(signed_k<N>(t + e * T));
          acc[3] += 0.5 * kk * kk * double(norm2(v[m][e]));
          v[m][e] = conj(mul_tab(v[m][e], ph[m * N + t + e * T]));
        }
        fft_pencil<Real, N, R>(v[m], t, L, tw);
#pragma unroll
        for (int e = 0; e < R; ++e) v[m][e] = conj(v[m][e]);
      }
      acc[3] *= 1.0 / double(N);
    } else {
#pragma unroll
      for (int m = 0; m < 3; ++m) fft_phase_ifft<Real, N, R>(v[m], t, L, tw, ph + m * N);
    }
    if (a.tau_post != 0.0) {
      const Real tau = Real(a.tau_post);
#pragma unroll
      for (int e = 0; e < R; ++e) {
        C site[3] = {v[0][e], v[1][e], v[2][e]};
        local_update(site, tau, c0, c1);
        v[0][e] = site[0];
        v[1][e] = site[1];
        v[2][e] = site[2];
      }
    }
    if (active) {
#pragma unroll
      for (int m = 0; m < 3; ++m)
#pragma unroll
        for (int e = 0; e < R; ++e) base[m * a.sites + e * T] = v[m][e];
    }
    if constexpr (MODE == MODE_STEP_LOG) pencil_sums_out<T>(acc, lds, p, t, active, a.part + pid * 4);
  } else if constexpr (MODE == MODE_PAPER) {
    const Real c0 = Real(a.c0), c1 = Real(a.c1), q = Real(a.q);
    auto local_all = [&](Real dt) {
#pragma unroll
      for (int e = 0; e < R; ++e) {
        C site[3] = {v[0][e], v[1][e], v[2][e]};
        paper_local_update(site, dt, c0, c1, q);
        v[0][e] = site[0];
        v[1][e] = site[1];
        v[2][e] = site[2];
      }
    };
    if (a.tau_pre != 0.0) local_all(Real(a.tau_pre));
    // kinetic phase alone (the m = 0 row of the x table; q sits in D)
    const TabEntry<Real>* ph0 = static_cast<const TabEntry<Real>*>(a.ph) + N;
#pragma unroll
    for (int m = 0; m < 3; ++m) fft_phase_ifft<Real, N, R>(v[m], t, L, tw, ph0);
    if (a.tau_post != 0.0) local_all(Real(a.tau_post));
    if (active) {
#pragma unroll
      for (int m = 0; m < 3; ++m)
#pragma unroll
        for (int e = 0; e < R; ++e) base[m * a.sites + e * T] = v[m][e];
    }
  } else if constexpr (MODE == MODE_MEASURE) {
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int e = 0; e < R; ++e) site_sums(v[0][e], v[1][e], v[2][e], a.c0, a.c1, a.q, acc);
#pragma unroll
    for (int m = 0; m < 3; ++m) {
      fft_pencil<Real, N, R>(v[m], t, L, tw);
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
    fft_pencil<Real, N, R>(f, t, L, tw);
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

  C v[R];
#pragma unroll
  for (int e = 0; e < R; ++e) v[e] = base[int64_t(t + e * T) * a.sa];

  if constexpr (MODE == MODE_STEP) {
    fft_phase_ifft<Real, N, R>(v, t, L, tw, static_cast<const TabEntry<Real>*>(a.ph));
#pragma unroll
    for (int e = 0; e < R; ++e) base[int64_t(t + e * T) * a.sa] = v[e];
  } else if constexpr (MODE == MODE_STEP_LOG) {
    const TabEntry<Real>* ph = static_cast<const TabEntry<Real>*>(a.ph);
    fft_pencil<Real, N, R>(v, t, L, tw);
    double acc = 0.0;
#pragma unroll
    for (int e = 0; e < R; ++e) {
      const double kk = a.kscale * double(signed_k<N>(t + e * T));
      acc += 0.5 * kk * kk * double(norm2(v[e]));
      v[e] = conj(mul_tab(v[e], ph[t + e * T]));
    }
    fft_pencil<Real, N, R>(v, t, L, tw);
#pragma unroll
    for (int e = 0; e < R; ++e) base[int64_t(t + e * T) * a.sa] = conj(v[e]);
    acc *= 1.0 / double(N);
    const double tot = block_sum(acc, reinterpret_cast<double*>(lds));
    if (threadIdx.x == 0) a.part[blockIdx.x] = tot;
  } else if constexpr (MODE == MODE_MEASURE) {
    fft_pencil<Real, N, R>(v, t, L, tw);
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
    fft_pencil<Real, N, R>(v, t, L, tw);
#pragma unroll
    for (int e = 0; e < R; ++e) base[int64_t(t + e * T) * a.sa] = v[e];
  } else {
    fft_pencil<Real, N, R>(v, t, L, tw);
    Real* out = static_cast<Real*>(a.out) + off;
    const Real ps = Real(a.power_scale);
#pragma unroll
    for (int e = 0; e < R; ++e) out[int64_t(t + e * T) * a.sa] = norm2(v[e]) * ps;
  }
}

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
// --------------------------------------------------------------------------
// The twiddle and phase tables are staged in LDS once per workgroup: a global
// load issued after the prefetch could only be consumed once the whole
// prefetch had arrived (the vector-memory counter retires in order).
template <typename Real, int N, int V, bool PLAIN>
__global__ __launch_bounds__((SCfg<N, Real, V>::THREADS)) void k_spass_stream(SPassArgs a, int64_t items) {
  using C = Cx<Real>;
  constexpr int R = SCfg<N, Real, V>::R, T = SCfg<N, Real, V>::T, TX = SCfg<N, Real, V>::TX;
  __shared__ C lds[N * ColLds<Real, TX>::PITCH];
  using TE = std::conditional_t<PLAIN, Cx<Real>, TabEntry<Real>>;
  __shared__ TE tw[N];
  __shared__ TabEntry<Real> ph[N / 2 + 1];  // the phase is even in k
  const int c = threadIdx.x % TX;
  const int t = threadIdx.x / TX;
  const int64_t tiles = a.inner / TX;
  ColLds<Real, TX> L{lds + c};
  {
    const TabEntry<Real>* gtw = static_cast<const TabEntry<Real>*>(a.tw);
    const TabEntry<Real>* gph = static_cast<const TabEntry<Real>*>(a.ph);
    for (int i = threadIdx.x; i < N; i += blockDim.x) {
      if constexpr (PLAIN)
        tw[i] = C{gtw[i].hr, gtw[i].hi};
      else
        tw[i] = gtw[i];
    }
    for (int i = threadIdx.x; i <= N / 2; i += blockDim.x) ph[i] = gph[i];
    __syncthreads();
  }
  // item -> (field f, outer o, tile): shifts, all three extents are powers of two
  char* psi = static_cast<char*>(a.psi);
  const uint32_t lane_off = uint32_t((c + int64_t(t) * a.sa) * int64_t(sizeof(C)));
  const uint32_t step_e = uint32_t(int64_t(T) * a.sa * int64_t(sizeof(C)));
  auto tile_base = [&](int64_t item) -> char* {
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
#pragma unroll
      for (int e = 0; e < R; ++e) nxt[e] = *reinterpret_cast<const C*>(src + (lane_off + uint32_t(e) * step_e));
    }
    fft_halfphase_ifft<Real, N, R>(v, t, L, static_cast<const TE*>(tw), ph,
                                   static_cast<const TabEntry<Real>*>(nullptr));
#pragma unroll
    for (int e = 0; e < R; ++e) *reinterpret_cast<C*>(dst + (lane_off + uint32_t(e) * step_e)) = v[e];
  }
}

// PLAIN: the stage twiddles rounded once to plain complex values (FP32 only):
// half the multiply cost and LDS of the hi+lo form, at a larger systematic
// rounding of the transform (see the precision option in spin1.h)
template <typename Real, int N, int V, bool PLAIN, bool ENABLED = XCfg<N, Real, V>::STREAM>
__global__ __launch_bounds__((XCfg<N, Real, V>::THREADS)) void k_xpass_stream(XPassArgs a, int64_t groups) {
 if constexpr (ENABLED) {
  using C = Cx<Real>;
  constexpr int R = XCfg<N, Real, V>::R, T = XCfg<N, Real, V>::T, P = XCfg<N, Real, V>::P;
  __shared__ C lds[P * RowPad<N, T>::ROW];
  using TW = StagedTwiddles<Real, N, R>;
  using TE = std::conditional_t<PLAIN, Cx<Real>, TabEntry<Real>>;
  using TWA = std::conditional_t<PLAIN, StagedTwiddlesPlain<Real, N, R>, TW>;
  __shared__ TE stw[TW::SIZE > 0 ? TW::SIZE : 1];
  // phase tables of m = +1 (equal to m = -1, q enters as q m^2) and m = 0
  __shared__ TabEntry<Real> ph[2 * N];
  const int t = threadIdx.x % T;
  const int p = threadIdx.x / T;
  RowLds<Real, N, T, (T <= 64)> L{lds + p * RowPad<N, T>::ROW};
  {
    const TabEntry<Real>* gtw = static_cast<const TabEntry<Real>*>(a.tw);
    const TabEntry<Real>* gph = static_cast<const TabEntry<Real>*>(a.ph);
    for (int i = threadIdx.x; i < TW::SIZE; i += blockDim.x) {
      const TabEntry<Real> w = gtw[TW::exponent(i)];
      if constexpr (PLAIN)
        stw[i] = C{w.hr, w.hi};
      else
        stw[i] = w;
    }
    for (int i = threadIdx.x; i < 2 * N; i += blockDim.x) ph[i] = gph[i];
    __syncthreads();
  }
  C* psi = static_cast<C*>(a.psi);
  const int64_t npen = int64_t(a.S) * a.rows;
  const Real c0 = Real(a.c0), c1 = Real(a.c1);
  // pencil pid: component m starts at ((s*3 + m) * sites + row * N); rows is a power of two
  auto comp_base = [&](int64_t pid, int m) -> C* {
    const int64_t s = pid >> a.lg_rows;
    return psi + (s * 3 + m) * a.sites + (pid & (a.rows - 1)) * N;
  };
  auto load3 = [&](C (&dst)[3][R], int64_t pid) {
#pragma unroll
    for (int m = 0; m < 3; ++m) {
      const C* src = comp_base(pid, m);
#pragma unroll
      for (int e = 0; e < R; ++e) dst[m][e] = src[uint32_t(t + e * T)];
    }
  };
  int64_t g = blockIdx.x;
  if (g >= groups) return;
  for (; g < groups; g += gridDim.x) {
    const int64_t pid = g * P + p;
    const bool active = pid < npen;
    C v[3][R];
    if (active) load3(v, pid);
    if (a.tau_pre != 0.0) {
      const Real tau = Real(a.tau_pre);
#pragma unroll
      for (int e = 0; e < R; ++e) {
        C site[3] = {v[0][e], v[1][e], v[2][e]};
        local_update(site, tau, c0, c1);
        v[0][e] = site[0];
        v[1][e] = site[1];
        v[2][e] = site[2];
      }
    }
#pragma unroll
    for (int m = 0; m < 3; ++m) fft_phase_ifft<Real, N, R>(v[m], t, L, TWA{stw}, ph + (m == 1 ? N : 0));
    if (a.tau_post != 0.0) {
      const Real tau = Real(a.tau_post);
#pragma unroll
      for (int e = 0; e < R; ++e) {
        C site[3] = {v[0][e], v[1][e], v[2][e]};
        local_update(site, tau, c0, c1);
        v[0][e] = site[0];
        v[1][e] = site[1];
        v[2][e] = site[2];
      }
    }
    if (active) {
#pragma unroll
      for (int m = 0; m < 3; ++m) {
        C* dst = comp_base(pid, m);
#pragma unroll
        for (int e = 0; e < R; ++e) dst[uint32_t(t + e * T)] = v[m][e];
      }
    }
  }
}
 }

// --------------------------------------------------------------------------
// Grouped x-pass: the step x-passes of several groups (different pencil
// lengths N) in one persistent launch.  Radix 8 for every N, so each thread
// holds the same 3 x 8 values whatever the group; a workgroup of 256 threads
// runs P = 2048 / N pencils of N / 8 threads.  The workgroup walks the
// concatenated item list with a stride of gridDim.x; items of one group are
// contiguous, so it reloads the group's tables (staged twiddles, phases) into
// LDS at most once per group.  The next item is prefetched into registers
// whatever its group.
// --------------------------------------------------------------------------
template <typename Real>
struct GroupedX {
  static constexpr int R = 8, THREADS = 256;
  static constexpr int NMAX = sizeof(Real) == 4 ? 1024 : 512;
  static constexpr int ROWS_LDS = (THREADS * R / 16) * 17;  // P (N + N/16) for every N >= 16
  // FP32: two workgroups per CU, as the single-group kernel gets
  static constexpr int WAVES_PER_EU = sizeof(Real) == 4 ? 2 : 1;
};

template <typename Real, int N>
__device__ __forceinline__ void grouped_x_body(Cx<Real> (&v)[3][8], int tid, Cx<Real>* lds,
                                               const TabEntry<Real>* stw, const TabEntry<Real>* ph) {
  constexpr int R = 8, T = N / R;
  const int t = tid % T, p = tid / T;
  RowLds<Real, N, T, (T <= 64)> L{lds + p * RowPad<N, T>::ROW};
#pragma unroll
  for (int m = 0; m < 3; ++m)
    fft_phase_ifft<Real, N, R>(v[m], t, L, StagedTwiddles<Real, N, R>{stw}, ph + (m == 1 ? N : 0));
}

template <typename Real>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(GroupedX<Real>::WAVES_PER_EU))) void
k_xpass_grouped(XGroupArgs a) {
  using C = Cx<Real>;
  using G = GroupedX<Real>;
  constexpr int R = G::R, NMAX = G::NMAX;
  __shared__ C lds[G::ROWS_LDS];
  __shared__ TabEntry<Real> stw[NMAX - R];
  __shared__ TabEntry<Real> ph[2 * NMAX];
  const int tid = threadIdx.x;
  auto group_of = [&](int64_t item) {
    int g = 0;
    while (g + 1 < a.ngroups && item >= a.g[g + 1].item_begin) ++g;
    return g;
  };
  // thread's pencil and lane in group g, item `item`; false if past the group's pencils
  auto place = [&](int g, int64_t item, int64_t* pid, int* t) {
    const int T = a.g[g].n / R, P = G::THREADS / T;
    *t = tid % T;
    *pid = (item - a.g[g].item_begin) * P + tid / T;
    return *pid < a.g[g].pencils;
  };
  auto comp_base = [&](int g, int64_t pid, int m) -> C* {
    const XGroupEntry& e = a.g[g];
    const int64_t s = pid >> e.lg_rows;
    return static_cast<C*>(e.psi) + (s * 3 + m) * e.sites + (pid & (e.rows - 1)) * e.n;
  };
  auto load3 = [&](C (&dst)[3][R], int g, int64_t item) {
    int64_t pid;
    int t;
    if (!place(g, item, &pid, &t)) return;
    const int T = a.g[g].n / R;
#pragma unroll
    for (int m = 0; m < 3; ++m) {
      const C* src = comp_base(g, pid, m);
#pragma unroll
      for (int e = 0; e < R; ++e) dst[m][e] = src[uint32_t(t + e * T)];
    }
  };
  int64_t item = blockIdx.x;
  if (item >= a.item_end) return;
  int cur = -1;
  C nxt[3][R];
  load3(nxt, group_of(item), item);
  const Real c0 = Real(a.c0), c1 = Real(a.c1);
  for (; item < a.item_end; item += gridDim.x) {
    const int g = group_of(item);
    if (g != cur) {  // uniform over the workgroup: every thread has the same item
      __syncthreads();
      const int n = a.g[g].n;
      const TabEntry<Real>* gtw = static_cast<const TabEntry<Real>*>(a.g[g].tw);
      const TabEntry<Real>* gph = static_cast<const TabEntry<Real>*>(a.g[g].ph);
      switch (n) {
        case 16: for (int i = tid; i < 16 - R; i += G::THREADS) stw[i] = gtw[StagedTwiddles<Real, 16, R>::exponent(i)]; break;
        case 32: for (int i = tid; i < 32 - R; i += G::THREADS) stw[i] = gtw[StagedTwiddles<Real, 32, R>::exponent(i)]; break;
        case 64: for (int i = tid; i < 64 - R; i += G::THREADS) stw[i] = gtw[StagedTwiddles<Real, 64, R>::exponent(i)]; break;
        case 128: for (int i = tid; i < 128 - R; i += G::THREADS) stw[i] = gtw[StagedTwiddles<Real, 128, R>::exponent(i)]; break;
        case 256: for (int i = tid; i < 256 - R; i += G::THREADS) stw[i] = gtw[StagedTwiddles<Real, 256, R>::exponent(i)]; break;
        case 512: for (int i = tid; i < 512 - R; i += G::THREADS) stw[i] = gtw[StagedTwiddles<Real, 512, R>::exponent(i)]; break;
        default:
          if constexpr (NMAX >= 1024)
            for (int i = tid; i < 1024 - R; i += G::THREADS) stw[i] = gtw[StagedTwiddles<Real, 1024, R>::exponent(i)];
          break;
      }
      for (int i = tid; i < 2 * n; i += G::THREADS) ph[i] = gph[i];
      __syncthreads();
      cur = g;
    }
    C v[3][R];
#pragma unroll
    for (int m = 0; m < 3; ++m)
#pragma unroll
      for (int e = 0; e < R; ++e) v[m][e] = nxt[m][e];
    const int64_t next = item + gridDim.x;
    if (next < a.item_end) load3(nxt, group_of(next), next);
    int64_t pid;
    int t;
    const bool active = place(g, item, &pid, &t);
    if (a.tau_pre != 0.0) {
      const Real tau = Real(a.tau_pre);
#pragma unroll
      for (int e = 0; e < R; ++e) {
        C site[3] = {v[0][e], v[1][e], v[2][e]};
        local_update(site, tau, c0, c1);
        v[0][e] = site[0];
        v[1][e] = site[1];
        v[2][e] = site[2];
      }
    }
    switch (a.g[g].n) {
      case 16: grouped_x_body<Real, 16>(v, tid, lds, stw, ph); break;
      case 32: grouped_x_body<Real, 32>(v, tid, lds, stw, ph); break;
      case 64: grouped_x_body<Real, 64>(v, tid, lds, stw, ph); break;
      case 128: grouped_x_body<Real, 128>(v, tid, lds, stw, ph); break;
      case 256: grouped_x_body<Real, 256>(v, tid, lds, stw, ph); break;
      case 512: grouped_x_body<Real, 512>(v, tid, lds, stw, ph); break;
      default:
        if constexpr (NMAX >= 1024) grouped_x_body<Real, 1024>(v, tid, lds, stw, ph);
        break;
    }
    if (a.g[g].tau_post != 0.0) {
      const Real tau = Real(a.g[g].tau_post);
#pragma unroll
      for (int e = 0; e < R; ++e) {
        C site[3] = {v[0][e], v[1][e], v[2][e]};
        local_update(site, tau, c0, c1);
        v[0][e] = site[0];
        v[1][e] = site[1];
        v[2][e] = site[2];
      }
    }
    if (active) {
      const int T = a.g[g].n / R;
#pragma unroll
      for (int m = 0; m < 3; ++m) {
        C* dst = comp_base(g, pid, m);
#pragma unroll
        for (int e = 0; e < R; ++e) dst[uint32_t(t + e * T)] = v[m][e];
      }
    }
  }
}

__device__ __forceinline__ void store_tab(TabEntry<float>* p, double re, double im) {
  const float hr = float(re), hi = float(im);
  *p = TabEntry<float>{hr, hi, float(re - double(hr)), float(im - double(hi))};
}
__device__ __forceinline__ void store_tab(TabEntry<double>* p, double re, double im) { *p = TabEntry<double>{re, im}; }


// --------------------------------------------------------------------------
// 1D: several steps per launch.  A 1D sample is one pencil, so a workgroup
// can keep it in registers for K consecutive split steps with no HBM traffic
// in between: load, K x [R(tau) -> FFT -> phase -> inverse FFT], optional
// closing R(dt/2), store.  One pencil per workgroup (the sample count is the
// parallelism); tables in LDS: twiddles (half table for N = 4096) and the
// kinetic phase for k <= N/2 (it is even in k), the Zeeman factor
// exp(-i q dt) applied separately to m = +-1.
// --------------------------------------------------------------------------
template <int N, typename Real>
struct MultiCfg {
  static constexpr int R = XCfg<N, Real>::R;
  static constexpr int T = N / R;
  static constexpr bool HALF_TW = N >= 4096;
  static constexpr int TW_N = HALF_TW ? N / 2 + 1 : N;
};

template <typename Real, int N>
__global__ __launch_bounds__((MultiCfg<N, Real>::T)) void k_x1d_multi(XPassArgs a, int K, double dt, int open_half,
                                                                       int close_half) {
  using C = Cx<Real>;
  using Cfg = MultiCfg<N, Real>;
  constexpr int R = Cfg::R, T = Cfg::T;
  __shared__ C lds[RowPad<N, T>::ROW];
  __shared__ TabEntry<Real> stw[Cfg::TW_N];
  __shared__ TabEntry<Real> ph0[N / 2 + 1];
  __shared__ TabEntry<Real> zq;
  const int t = threadIdx.x;
  {
    const TabEntry<Real>* gtw = static_cast<const TabEntry<Real>*>(a.tw);
    const TabEntry<Real>* gph = static_cast<const TabEntry<Real>*>(a.ph) + N;  // m = 0 row
    for (int i = t; i < Cfg::TW_N; i += T) stw[i] = gtw[i];
    for (int i = t; i <= N / 2; i += T) ph0[i] = gph[i];
    if (t == 0) {
      double sn, cs;
      sincos(a.q * dt, &sn, &cs);
      store_tab(&zq, cs, -sn);
    }
    __syncthreads();
  }
  RowLds<Real, N, T, (T <= 64)> L{lds};
  C* psi = static_cast<C*>(a.psi) + int64_t(blockIdx.x) * 3 * a.sites + t;
  C v[3][R];
#pragma unroll
  for (int m = 0; m < 3; ++m)
#pragma unroll
    for (int e = 0; e < R; ++e) v[m][e] = psi[m * a.sites + e * T];
  const Real c0 = Real(a.c0), c1 = Real(a.c1);
  auto local_all = [&](Real tau) {
#pragma unroll
    for (int e = 0; e < R; ++e) {
      C site[3] = {v[0][e], v[1][e], v[2][e]};
      local_update(site, tau, c0, c1);
      v[0][e] = site[0];
      v[1][e] = site[1];
      v[2][e] = site[2];
    }
  };
  for (int k = 0; k < K; ++k) {
    local_all(Real((k == 0 && open_half) ? 0.5 * dt : dt));
    if constexpr (Cfg::HALF_TW) {
      const HalfTwiddles<Real, N> tw{stw};
      fft_halfphase_ifft<Real, N, R>(v[0], t, L, tw, ph0, &zq);
      fft_halfphase_ifft<Real, N, R>(v[1], t, L, tw, ph0, static_cast<const TabEntry<Real>*>(nullptr));
      fft_halfphase_ifft<Real, N, R>(v[2], t, L, tw, ph0, &zq);
    } else {
      const TabEntry<Real>* tw = stw;
      fft_halfphase_ifft<Real, N, R>(v[0], t, L, tw, ph0, &zq);
      fft_halfphase_ifft<Real, N, R>(v[1], t, L, tw, ph0, static_cast<const TabEntry<Real>*>(nullptr));
      fft_halfphase_ifft<Real, N, R>(v[2], t, L, tw, ph0, &zq);
    }
  }
  if (close_half) local_all(Real(0.5 * dt));
#pragma unroll
  for (int m = 0; m < 3; ++m)
#pragma unroll
    for (int e = 0; e < R; ++e) psi[m * a.sites + e * T] = v[m][e];
}

// --------------------------------------------------------------------------
// local update alone (closing half step of multi-dimensional grids)
// --------------------------------------------------------------------------
template <typename Real>
__global__ __launch_bounds__(256) void k_local(Cx<Real>* psi, int S, int64_t sites, Real tau, Real c0, Real c1) {
  const int64_t total = int64_t(S) * sites;
  for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < total; i += int64_t(gridDim.x) * blockDim.x) {
    const int64_t s = i / sites, x = i - s * sites;
    Cx<Real>* b = psi + s * 3 * sites + x;
    Cx<Real> site[3] = {b[0], b[sites], b[2 * sites]};
    local_update(site, tau, c0, c1);
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
                                                     Real q) {
  const int64_t total = int64_t(S) * sites;
  for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < total; i += int64_t(gridDim.x) * blockDim.x) {
    const int64_t s = i / sites, x = i - s * sites;
    Cx<Real>* b = psi + s * 3 * sites + x;
    Cx<Real> site[3] = {b[0], b[sites], b[2 * sites]};
    paper_local_update(site, dt, c0, c1, q);
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
                                              double amp, double sqrt_n0) {
  const int64_t total = int64_t(S) * 3 * sites;
  for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < total; i += int64_t(gridDim.x) * blockDim.x) {
    const int64_t x = i % sites;
    const int64_t sc = i / sites;
    const int64_t c = sc % 3, s = sc / 3;
    U64x4 ctr;
    ctr.v[0] = uint64_t(x);
    ctr.v[1] = uint64_t(c);
    ctr.v[2] = uint64_t(s);
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
__global__ __launch_bounds__(256) void k_obs_finish(const double* part_x, int64_t rows, const double* part_y,
                                                    int64_t ny_blocks, const double* part_z, int64_t nz_blocks,
                                                    double cell, double* obs) {
  __shared__ double scratch[8];
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

// Local-update VJP over a whole field.
//  CLOSE (backward of a step's closing half): state = psi_{n+1} = R(tau) psi_b;
//    H in = conj(G) at psi_{n+1}, H out = conj(G) at psi_b; adds
//    tau Im<G, M psi_{n+1}> to dL/dc1 and dt sum_{m=+-1} Im<G_b, psi_b> to dL/dq.
//  OPEN (backward of a step's opening half): state = psi_n, psi_a = R(tau) psi_n;
//    H in = conj(G) at psi_a, H out = conj(G) at psi_n; adds tau Im<G, M psi_a>.
// Per-block FP64 partials (dL/dq, dL/dc1) go to part[2 * blockIdx.x + {0, 1}].
template <typename Real, bool CLOSE>
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
    C st[3] = {state[o], state[o + sites], state[o + 2 * sites]};
    C gout[3] = {conj(h[o]), conj(h[o + sites]), conj(h[o + 2 * sites])};
    C pin[3], pout[3];
    if constexpr (CLOSE) {
      // psi_b = R(-tau) psi_{n+1}
#pragma unroll
      for (int m = 0; m < 3; ++m) {
        pin[m] = st[m];
        pout[m] = st[m];
      }
      local_update(pin, -tau, c0, c1);
    } else {
#pragma unroll
      for (int m = 0; m < 3; ++m) {
        pin[m] = st[m];
        pout[m] = st[m];
      }
      local_update(pout, tau, c0, c1);
    }
    // dL/dc1 += tau Im<G_out, M psi_out>   (M is the same at input and output)
    {
      const Cx<Real> g = cmulc(pout[0], pout[1]) + cmulc(pout[1], pout[2]);
      const Real fz = norm2(pout[0]) - norm2(pout[2]);
      C mp[3];
      apply_M(pout, mp, g, fz);
      double acc = 0.0;
#pragma unroll
      for (int m = 0; m < 3; ++m) acc += double(cmulc(gout[m], mp[m]).im);
      dc1 += double(tau) * acc;
    }
    C gin[3];
    local_update_vjp(pin, pout, gout, gin, tau, c0, c1);
    if constexpr (CLOSE) {
      // q enters through exp(-i q m^2 dt) on m = +-1 in the step before: dt Im<G_b, psi_b>
      dq += dt * (double(cmulc(gin[0], pin[0]).im) + double(cmulc(gin[2], pin[2]).im));
    }
    h[o] = conj(gin[0]);
    h[o + sites] = conj(gin[1]);
    h[o + 2 * sites] = conj(gin[2]);
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
// host launchers
// --------------------------------------------------------------------------
[[maybe_unused]] static int ilog2(int64_t v) {
  int r = 0;
  while ((int64_t(1) << (r + 1)) <= v) ++r;
  return r;
}

// Number of compute units of the current device (cached per device).
[[maybe_unused]] static int device_cus() {
  static int cached[64] = {0};
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 256;
  if (!cached[dev]) {
    int n = 0;
    if (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || n <= 0) n = 256;
    cached[dev] = n;
  }
  return cached[dev];
}

// Grid of a streaming kernel: resident workgroups per CU x CUs, capped by the work.
template <class K>
static int64_t stream_grid(K kernel, int threads, int64_t items) {
  int per_cu = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, threads, 0) != hipSuccess || per_cu < 1)
    per_cu = 1;
  const int64_t g = int64_t(per_cu) * device_cus();
  return items < g ? items : g;
}

template <typename Real, int N, int V, bool PLAIN>
static hipError_t xpass_stream_v(hipStream_t st, const XPassArgs& a) {
  constexpr int P = XCfg<N, Real, V>::P;
  const int64_t blocks = (int64_t(a.S) * a.rows + P - 1) / P;
  XPassArgs b = a;
  b.lg_rows = ilog2(a.rows);
  const int64_t grid = stream_grid(k_xpass_stream<Real, N, V, PLAIN>, XCfg<N, Real, V>::THREADS, blocks);
  hipLaunchKernelGGL((k_xpass_stream<Real, N, V, PLAIN>), dim3(unsigned(grid)), dim3(XCfg<N, Real, V>::THREADS), 0,
                     st, b, blocks);
  return hipGetLastError();
}

template <typename Real, int N, bool PLAIN>
static hipError_t xpass_stream_p(hipStream_t st, const XPassArgs& a, int v) {
  // variants whose tables no longer fit in LDS fall back to the default one
  if (v == 1 && XCfg<N, Real, 1>::STREAM) return xpass_stream_v<Real, N, 1, PLAIN>(st, a);
  if (v == 2 && XCfg<N, Real, 2>::STREAM) return xpass_stream_v<Real, N, 2, PLAIN>(st, a);
  return xpass_stream_v<Real, N, 0, PLAIN>(st, a);
}

// variant: 0..2 the step-pass variant; + kPlainTwiddles for plain FP32 twiddles
template <typename Real, int N, int MODE>
static hipError_t xpass_n(hipStream_t st, const XPassArgs& a, int variant) {
  if constexpr (MODE == MODE_STEP && XCfg<N, Real>::STREAM) {
    if constexpr (sizeof(Real) == 4)
      if (variant >= kPlainTwiddles) return xpass_stream_p<Real, N, true>(st, a, variant - kPlainTwiddles);
    return xpass_stream_p<Real, N, false>(st, a, variant % kPlainTwiddles);
  } else {
    constexpr int P = XCfg<N, Real>::P;
    const int64_t blocks = (int64_t(a.S) * a.rows + P - 1) / P;
    hipLaunchKernelGGL((k_xpass<Real, N, MODE>), dim3(unsigned(blocks)), dim3(XCfg<N, Real>::THREADS), 0, st, a);
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

template <typename Real, int N, int V, bool PLAIN>
static hipError_t spass_stream_v(hipStream_t st, const SPassArgs& a) {
  constexpr int TX = SCfg<N, Real, V>::TX;
  if (a.inner % TX != 0) return hipErrorInvalidValue;
  const int64_t blocks = a.nfield * a.outer * (a.inner / TX);
  SPassArgs b = a;
  b.lg_tiles = ilog2(a.inner / TX);
  b.lg_outer = ilog2(a.outer);
  const int64_t grid = stream_grid(k_spass_stream<Real, N, V, PLAIN>, SCfg<N, Real, V>::THREADS, blocks);
  hipLaunchKernelGGL((k_spass_stream<Real, N, V, PLAIN>), dim3(unsigned(grid)), dim3(SCfg<N, Real, V>::THREADS), 0,
                     st, b, blocks);
  return hipGetLastError();
}

template <typename Real, int N, bool PLAIN>
static hipError_t spass_stream_p(hipStream_t st, const SPassArgs& a, int v) {
  if (v == 1) return spass_stream_v<Real, N, 1, PLAIN>(st, a);
  if (v == 2) return spass_stream_v<Real, N, 2, PLAIN>(st, a);
  return spass_stream_v<Real, N, 0, PLAIN>(st, a);
}

template <typename Real, int N, int MODE>
static hipError_t spass_n(hipStream_t st, const SPassArgs& a, int variant) {
  if constexpr (MODE == MODE_STEP && SCfg<N, Real>::STREAM) {
    if constexpr (sizeof(Real) == 4)
      if (variant >= kPlainTwiddles) return spass_stream_p<Real, N, true>(st, a, variant - kPlainTwiddles);
    return spass_stream_p<Real, N, false>(st, a, variant % kPlainTwiddles);
  } else {
    constexpr int TX = SCfg<N, Real>::TX;
    if (a.inner % TX != 0) return hipErrorInvalidValue;
    const int64_t blocks = a.nfield * a.outer * (a.inner / TX);
    hipLaunchKernelGGL((k_spass<Real, N, MODE>), dim3(unsigned(blocks)), dim3(SCfg<N, Real>::THREADS), 0, st, a);
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

int step_variants() { return kStepVariants; }

int grouped_x_max_n(bool dbl) { return dbl ? GroupedX<double>::NMAX : GroupedX<float>::NMAX; }

int64_t grouped_x_items(int n, int64_t pencils) {
  const int P = GroupedX<float>::THREADS * GroupedX<float>::R / n;
  return (pencils + P - 1) / P;
}

template <typename Real>
static hipError_t xpass_grouped_t(hipStream_t st, const XGroupArgs& a) {
  if (a.ngroups < 1 || a.ngroups > kMaxGroupedX) return hipErrorInvalidValue;
  for (int g = 0; g < a.ngroups; ++g) {
    const XGroupEntry& e = a.g[g];
    if (e.n < 16 || e.n > GroupedX<Real>::NMAX || (e.n & (e.n - 1)) != 0) return hipErrorInvalidValue;
    const int64_t end = g + 1 < a.ngroups ? a.g[g + 1].item_begin : a.item_end;
    if (end - e.item_begin != grouped_x_items(e.n, e.pencils)) return hipErrorInvalidValue;
    if ((e.rows & (e.rows - 1)) != 0 || (int64_t(1) << e.lg_rows) != e.rows) return hipErrorInvalidValue;
  }
  if (a.g[0].item_begin != 0 || a.item_end < 1) return hipErrorInvalidValue;
  const int64_t grid = stream_grid(k_xpass_grouped<Real>, GroupedX<Real>::THREADS, a.item_end);
  hipLaunchKernelGGL(k_xpass_grouped<Real>, dim3(unsigned(grid)), dim3(GroupedX<Real>::THREADS), 0, st, a);
  return hipGetLastError();
}

hipError_t launch_xpass_grouped(hipStream_t st, bool dbl, const XGroupArgs& a) {
  return dbl ? xpass_grouped_t<double>(st, a) : xpass_grouped_t<float>(st, a);
}

template <typename Real, int N>
static hipError_t x1d_multi_n(hipStream_t st, const XPassArgs& a, int K, double dt, bool open_half, bool close_half) {
  hipLaunchKernelGGL((k_x1d_multi<Real, N>), dim3(unsigned(a.S)), dim3(MultiCfg<N, Real>::T), 0, st, a, K, dt,
                     int(open_half), int(close_half));
  return hipGetLastError();
}

template <typename Real>
static hipError_t x1d_multi_t(hipStream_t st, int n, const XPassArgs& a, int K, double dt, bool oh, bool ch) {
  switch (n) {
    case 8: return x1d_multi_n<Real, 8>(st, a, K, dt, oh, ch);
    case 16: return x1d_multi_n<Real, 16>(st, a, K, dt, oh, ch);
    case 32: return x1d_multi_n<Real, 32>(st, a, K, dt, oh, ch);
    case 64: return x1d_multi_n<Real, 64>(st, a, K, dt, oh, ch);
    case 128: return x1d_multi_n<Real, 128>(st, a, K, dt, oh, ch);
    case 256: return x1d_multi_n<Real, 256>(st, a, K, dt, oh, ch);
    case 512: return x1d_multi_n<Real, 512>(st, a, K, dt, oh, ch);
    case 1024: return x1d_multi_n<Real, 1024>(st, a, K, dt, oh, ch);
    case 2048: return x1d_multi_n<Real, 2048>(st, a, K, dt, oh, ch);
    case 4096: return x1d_multi_n<Real, 4096>(st, a, K, dt, oh, ch);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_x1d_multi(hipStream_t st, bool dbl, int n, const XPassArgs& a, int K, double dt, bool open_half,
                            bool close_half) {
  return dbl ? x1d_multi_t<double>(st, n, a, K, dt, open_half, close_half)
             : x1d_multi_t<float>(st, n, a, K, dt, open_half, close_half);
}

static unsigned grid_for(int64_t work, int threads) {
  int64_t b = (work + threads - 1) / threads;
  if (b > 65536) b = 65536;
  if (b < 1) b = 1;
  return unsigned(b);
}

hipError_t launch_tables(hipStream_t st, bool dbl, void* ph, void* tw, int n, int ncomp, double dt, double q,
                         double dx) {
  const unsigned blocks = unsigned((n + 255) / 256);
  if (dbl)
    hipLaunchKernelGGL(k_tables<double>, dim3(blocks), dim3(256), 0, st, static_cast<TabEntry<double>*>(ph),
                       static_cast<TabEntry<double>*>(tw), n, ncomp, dt, q, dx);
  else
    hipLaunchKernelGGL(k_tables<float>, dim3(blocks), dim3(256), 0, st, static_cast<TabEntry<float>*>(ph),
                       static_cast<TabEntry<float>*>(tw), n, ncomp, dt, q, dx);
  return hipGetLastError();
}

hipError_t launch_init(hipStream_t st, bool dbl, void* psi, const Geom& g, uint64_t seed, uint64_t group, double n0,
                       double wigner_var) {
  const double cell = g.dim == 1 ? g.dx : (g.dim == 2 ? g.dx * g.dx : g.dx * g.dx * g.dx);
  const double amp = sqrt(wigner_var / (2.0 * cell));
  const unsigned blocks = grid_for(int64_t(g.S) * 3 * g.sites, 256);
  if (dbl)
    hipLaunchKernelGGL(k_init<double>, dim3(blocks), dim3(256), 0, st, static_cast<Cx<double>*>(psi), g.S, g.sites,
                       seed, group, amp, sqrt(n0));
  else
    hipLaunchKernelGGL(k_init<float>, dim3(blocks), dim3(256), 0, st, static_cast<Cx<float>*>(psi), g.S, g.sites,
                       seed, group, amp, sqrt(n0));
  return hipGetLastError();
}

hipError_t launch_local(hipStream_t st, bool dbl, void* psi, int S, int64_t sites, double tau, double c0, double c1) {
  const unsigned blocks = grid_for(int64_t(S) * sites, 256);
  if (dbl)
    hipLaunchKernelGGL(k_local<double>, dim3(blocks), dim3(256), 0, st, static_cast<Cx<double>*>(psi), S, sites, tau,
                       c0, c1);
  else
    hipLaunchKernelGGL(k_local<float>, dim3(blocks), dim3(256), 0, st, static_cast<Cx<float>*>(psi), S, sites,
                       float(tau), float(c0), float(c1));
  return hipGetLastError();
}

hipError_t launch_paper_local(hipStream_t st, bool dbl, void* psi, int S, int64_t sites, double dt, double c0,
                              double c1, double q) {
  const unsigned blocks = grid_for(int64_t(S) * sites, 256);
  if (dbl)
    hipLaunchKernelGGL(k_paper_local<double>, dim3(blocks), dim3(256), 0, st, static_cast<Cx<double>*>(psi), S, sites,
                       dt, c0, c1, q);
  else
    hipLaunchKernelGGL(k_paper_local<float>, dim3(blocks), dim3(256), 0, st, static_cast<Cx<float>*>(psi), S, sites,
                       float(dt), float(c0), float(c1), float(q));
  return hipGetLastError();
}

hipError_t launch_f_perp(hipStream_t st, bool dbl, const void* psi, int S, int64_t sites, void* out) {
  const unsigned blocks = grid_for(int64_t(S) * sites, 256);
  if (dbl)
    hipLaunchKernelGGL(k_f_perp<double>, dim3(blocks), dim3(256), 0, st, static_cast<const Cx<double>*>(psi), S,
                       sites, static_cast<Cx<double>*>(out));
  else
    hipLaunchKernelGGL(k_f_perp<float>, dim3(blocks), dim3(256), 0, st, static_cast<const Cx<float>*>(psi), S, sites,
                       static_cast<Cx<float>*>(out));
  return hipGetLastError();
}

hipError_t launch_texture(hipStream_t st, bool dbl, const void* psi, int S, int64_t rows, int64_t sites, int n,
                          double* part, double* out) {
  const unsigned blocks = unsigned(int64_t(S) * rows);
  if (dbl)
    hipLaunchKernelGGL(k_texture_rows<double>, dim3(blocks), dim3(256), 0, st, static_cast<const Cx<double>*>(psi),
                       rows, sites, n, part);
  else
    hipLaunchKernelGGL(k_texture_rows<float>, dim3(blocks), dim3(256), 0, st, static_cast<const Cx<float>*>(psi),
                       rows, sites, n, part);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_texture_finish, dim3(unsigned(S)), dim3(256), 0, st, part, rows, sites, out);
  return hipGetLastError();
}

hipError_t launch_bin(hipStream_t st, bool dbl, const void* power, int S, int64_t sites, const int32_t* perm,
                      const int32_t* offs, int nbins, double* out) {
  const dim3 grid(unsigned((nbins + 3) / 4), unsigned(S));
  if (dbl)
    hipLaunchKernelGGL(k_bin<double>, grid, dim3(256), 0, st, static_cast<const double*>(power), sites, perm, offs,
                       nbins, out);
  else
    hipLaunchKernelGGL(k_bin<float>, grid, dim3(256), 0, st, static_cast<const float*>(power), sites, perm, offs,
                       nbins, out);
  return hipGetLastError();
}

hipError_t launch_obs_finish(hipStream_t st, int S, const double* part_x, int64_t rows, const double* part_y,
                             int64_t ny_blocks, const double* part_z, int64_t nz_blocks, double cell, double* obs) {
  hipLaunchKernelGGL(k_obs_finish, dim3(unsigned(S)), dim3(256), 0, st, part_x, rows, part_y, ny_blocks, part_z,
                     nz_blocks, cell, obs);
  return hipGetLastError();
}


template <typename Real, int N>
static hipError_t fft1_n(hipStream_t st, void* f, const void* tw, int64_t pencils) {
  constexpr int P = XCfg<N, Real>::P;
  const int64_t blocks = (pencils + P - 1) / P;
  hipLaunchKernelGGL((k_fft1_x<Real, N>), dim3(unsigned(blocks)), dim3(XCfg<N, Real>::THREADS), 0, st,
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

hipError_t launch_adj_local(hipStream_t st, bool dbl, bool close, const void* state, void* h, int S, int64_t sites,
                            double tau, double c0, double c1, double dt, double* part) {
  const unsigned blocks = grid_for(int64_t(S) * sites, 256);
  if (dbl) {
    if (close)
      hipLaunchKernelGGL((k_adj_local<double, true>), dim3(blocks), dim3(256), 0, st,
                         static_cast<const Cx<double>*>(state), static_cast<Cx<double>*>(h), S, sites, tau, c0, c1, dt,
                         part);
    else
      hipLaunchKernelGGL((k_adj_local<double, false>), dim3(blocks), dim3(256), 0, st,
                         static_cast<const Cx<double>*>(state), static_cast<Cx<double>*>(h), S, sites, tau, c0, c1, dt,
                         part);
  } else {
    if (close)
      hipLaunchKernelGGL((k_adj_local<float, true>), dim3(blocks), dim3(256), 0, st,
                         static_cast<const Cx<float>*>(state), static_cast<Cx<float>*>(h), S, sites, float(tau),
                         float(c0), float(c1), dt, part);
    else
      hipLaunchKernelGGL((k_adj_local<float, false>), dim3(blocks), dim3(256), 0, st,
                         static_cast<const Cx<float>*>(state), static_cast<Cx<float>*>(h), S, sites, float(tau),
                         float(c0), float(c1), dt, part);
  }
  return hipGetLastError();
}

hipError_t launch_adj_accum(hipStream_t st, const double* part, int nblocks, double* acc) {
  hipLaunchKernelGGL(k_adj_accum, dim3(1), dim3(256), 0, st, part, nblocks, acc);
  return hipGetLastError();
}

hipError_t launch_adj_spectrum(hipStream_t st, bool dbl, void* f, const Geom& g, const int32_t* offs, int nbins,
                               const double* dl_dbins) {
  const unsigned blocks = grid_for(int64_t(g.S) * g.sites, 256);
  if (dbl)
    hipLaunchKernelGGL(k_adj_spectrum<double>, dim3(blocks), dim3(256), 0, st, static_cast<Cx<double>*>(f), g.S,
                       g.sites, g.dim, g.n[0], g.n[1], g.n[2], offs, nbins, dl_dbins);
  else
    hipLaunchKernelGGL(k_adj_spectrum<float>, dim3(blocks), dim3(256), 0, st, static_cast<Cx<float>*>(f), g.S,
                       g.sites, g.dim, g.n[0], g.n[1], g.n[2], offs, nbins, dl_dbins);
  return hipGetLastError();
}

hipError_t launch_adj_seed(hipStream_t st, bool dbl, const void* psi, const void* hf, void* h, int S, int64_t sites) {
  const unsigned blocks = grid_for(int64_t(S) * sites, 256);
  if (dbl)
    hipLaunchKernelGGL(k_adj_seed<double>, dim3(blocks), dim3(256), 0, st, static_cast<const Cx<double>*>(psi),
                       static_cast<const Cx<double>*>(hf), static_cast<Cx<double>*>(h), S, sites);
  else
    hipLaunchKernelGGL(k_adj_seed<float>, dim3(blocks), dim3(256), 0, st, static_cast<const Cx<float>*>(psi),
                       static_cast<const Cx<float>*>(hf), static_cast<Cx<float>*>(h), S, sites);
  return hipGetLastError();
}

hipError_t launch_conj(hipStream_t st, bool dbl, const void* in, void* out, int64_t n) {
  const unsigned blocks = grid_for(n, 256);
  if (dbl)
    hipLaunchKernelGGL(k_conj<double>, dim3(blocks), dim3(256), 0, st, static_cast<const Cx<double>*>(in),
                       static_cast<Cx<double>*>(out), n);
  else
    hipLaunchKernelGGL(k_conj<float>, dim3(blocks), dim3(256), 0, st, static_cast<const Cx<float>*>(in),
                       static_cast<Cx<float>*>(out), n);
  return hipGetLastError();
}

}  // namespace spin1
