// Shared pieces of the HIP translation units of the spin-1 library: launch
// configurations of the passes, LDS exchange views, FP64 reductions and the
// host-side grid helpers.
#pragma once
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
// and radix 32 on 1024 for FP32; twice the columns on FP32 columns of 256),
// V = 2 radix 8.
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
  // variant 1 of FP32 columns of 256: 32 columns (256-byte row segments, 64 KB
  // of LDS, two workgroups per CU)
  static constexpr bool W256 = V == 1 && N == 256 && sizeof(Real) == 4;
  static constexpr int TX1 =
      W256 ? 32 : ((V == 1 && C1024) ? 16 : ((V == 1 && TX0 > 4 && !C512) ? TX0 / 2 : TX0));
  // keep workgroups within 1024 threads
  static constexpr int TX = TX1 * T > 1024 ? 1024 / T : TX1;
  static constexpr int THREADS = TX * T;
  static constexpr bool STREAM = true;
  // the prefetch loads go out at a raised wavefront priority in workgroups of
  // up to 256 threads (measured faster there: 512-point FP32 columns -2 to -6%
  // per step, FP64 -1%; slower by 1% with the 512-thread tiles)
  static constexpr bool PRIO = THREADS <= 256;
  // FP64 columns of 512 on 8-column tiles: rows unpadded, so that two
  // workgroups fit in LDS (77.8 instead of 86 KB each)
  static constexpr int PITCH = (sizeof(Real) == 8 && N == 512 && TX == 8) ? TX : (TX >= 16 ? TX : TX + 1);
};

constexpr int kStepVariants = 3;
static_assert(kPlainTwiddles == kStepVariants, "the dithered-table variants follow the compensated ones");

// --------------------------------------------------------------------------
// LDS views used by the FFT stages
// --------------------------------------------------------------------------
// One pencil per row with one padding element after every 16 (measured best
// on gfx950 for the radix-8 exchanges: it breaks up the power-of-two strides
// of the early stages across LDS banks).
// SH: one padding element after every 2^SH.
template <int N, int T, int SH = 4>
struct RowPad {
  static constexpr int ROW = N + (N >> SH);
  __device__ static __forceinline__ int at(int i) { return i + (i >> SH); }
};

// LDS ordering among the lanes of one wavefront: LDS instructions of a wave
// execute in issue order, so the exchange only needs the compiler to keep the
// stores before the loads (fences at wavefront scope around a wave barrier).
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// A value the caller knows to be the same in every lane of the wavefront,
// moved to scalar registers (the compiler cannot always prove it uniform).
__device__ __forceinline__ int64_t wave_uniform(int64_t v) {
  const uint32_t lo = __builtin_amdgcn_readfirstlane(uint32_t(uint64_t(v)));
  const uint32_t hi = __builtin_amdgcn_readfirstlane(uint32_t(uint64_t(v) >> 32));
  return int64_t((uint64_t(hi) << 32) | lo);
}
__device__ __forceinline__ double wave_uniform(double v) {
  return __builtin_bit_cast(double, wave_uniform(__builtin_bit_cast(int64_t, v)));
}

// WAVE: every pencil lies inside one wavefront (N/R <= 64), so its exchanges
// synchronise only that wavefront; otherwise the whole workgroup.
template <typename Real, int N, int T, bool WAVE, int SH = 4>
struct RowLds {
  Cx<Real>* row;
  __device__ __forceinline__ void store(int i, Cx<Real> v) { row[RowPad<N, T, SH>::at(i)] = v; }
  __device__ __forceinline__ Cx<Real> load(int i) const { return row[RowPad<N, T, SH>::at(i)]; }
  // Slot of index i, and the slot step of a compile-time index step k: in the
  // exchanges of the FFT stages (index base + k with k a multiple of the
  // stage's sub-transform size, or t + e N/R) the low four bits of base and k
  // never carry, so slot(base + k) = slot(base) + off(k), and one per-lane
  // slot per stage serves every element through immediate offsets.
  __device__ static __forceinline__ int slot(int i) { return RowPad<N, T, SH>::at(i); }
  __device__ static constexpr int off(int k) { return k + (k >> SH); }
  __device__ __forceinline__ void store_slot(int s, Cx<Real> v) { row[s] = v; }
  __device__ __forceinline__ Cx<Real> load_slot(int s) const { return row[s]; }
  __device__ __forceinline__ void sync() {
    if constexpr (WAVE)
      wave_sync();
    else
      __syncthreads();
  }
};

// Column tiles: element i of column c at i * (TX + 1) + c; the odd row pitch
// spreads rows that differ by a power of two over different banks.
template <typename Real, int TX, int PITCH_ = (TX >= 16 ? TX : TX + 1)>
struct ColLds {
  static constexpr int PITCH = PITCH_;
  Cx<Real>* col;
  __device__ __forceinline__ void store(int i, Cx<Real> v) { col[i * PITCH] = v; }
  __device__ __forceinline__ Cx<Real> load(int i) const { return col[i * PITCH]; }
  __device__ static __forceinline__ int slot(int i) { return i * PITCH; }
  __device__ static constexpr int off(int k) { return k * PITCH; }
  __device__ __forceinline__ void store_slot(int s, Cx<Real> v) { col[s] = v; }
  __device__ __forceinline__ Cx<Real> load_slot(int s) const { return col[s]; }
  __device__ __forceinline__ void sync() { __syncthreads(); }
};

// signed wavenumber index of DFT bin k
template <int N>
__device__ __forceinline__ int signed_k(int k) {
  return k < N / 2 ? k : k - N;
}

// Local update R(tau) of the R sites held by thread t of a pencil (element e
// at x = t + e*T), followed by exp(-i V tau) with V from prow, the trap
// potential of the pencil's row: POT_NEVER, POT_ALWAYS (prow valid), or
// POT_IF_SET (when prow is not null).
enum { POT_NEVER = 0, POT_ALWAYS = 1, POT_IF_SET = 2 };
template <typename Real, int R, int T, int POT = POT_NEVER>
__device__ __forceinline__ void local_update_sites(Cx<Real> (&v)[3][R], int t, Real tau, Real c0, Real c1,
                                                   const double* prow = nullptr, double tau_d = 0.0) {
#pragma unroll
  for (int e = 0; e < R; ++e) {
    Cx<Real> site[3] = {v[0][e], v[1][e], v[2][e]};
    local_update(site, tau, c0, c1);
    if constexpr (POT == POT_ALWAYS) potential_phase(site, pot_angle<Real>(prow[t + e * T], tau_d));
    if constexpr (POT == POT_IF_SET)
      if (prow) potential_phase(site, pot_angle<Real>(prow[t + e * T], tau_d));
    v[0][e] = site[0];
    v[1][e] = site[1];
    v[2][e] = site[2];
  }
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
// V n + c0/2 n^2 + c1/2 |F|^2 + q (|psi_1|^2 + |psi_-1|^2) (acc[0..2]), V the trap
// potential at the site (0 without one)
template <typename Real>
__device__ __forceinline__ void site_sums(Cx<Real> p1, Cx<Real> p0, Cx<Real> pm, double c0, double c1, double q,
                                          double* acc, double v = 0.0) {
  const double d1 = double(norm2(p1)), d0 = double(norm2(p0)), dm = double(norm2(pm));
  const Cx<Real> g = cmulc(p1, p0) + cmulc(p0, pm);
  const double gre = double(g.re), gim = double(g.im);
  const double n = d1 + d0 + dm, fz = d1 - dm;
  const double f2 = 2.0 * (gre * gre + gim * gim) + fz * fz;
  acc[0] += n;
  acc[1] += fz;
  acc[2] += v * n + 0.5 * c0 * n * n + 0.5 * c1 * f2 + q * (d1 + dm);
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

__device__ __forceinline__ void store_tab(TabEntry<float>* p, double re, double im) {
  const float hr = float(re), hi = float(im);
  *p = TabEntry<float>{hr, hi, float(re - double(hr)), float(im - double(hi))};
}
__device__ __forceinline__ void store_tab(TabEntry<double>* p, double re, double im) { *p = TabEntry<double>{re, im}; }


// --------------------------------------------------------------------------
// host launchers
// --------------------------------------------------------------------------
[[maybe_unused]] static inline int ilog2(int64_t v) {
  int r = 0;
  while ((int64_t(1) << (r + 1)) <= v) ++r;
  return r;
}

// Number of compute units of the current device (cached per device).
[[maybe_unused]] static inline int device_cus() {
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
[[maybe_unused]] static int64_t stream_grid(K kernel, int threads, int64_t items) {
  int per_cu = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, threads, 0) != hipSuccess || per_cu < 1)
    per_cu = 1;
  const int64_t g = int64_t(per_cu) * device_cus();
  return items < g ? items : g;
}

[[maybe_unused]] static inline unsigned grid_for(int64_t work, int threads) {
  int64_t b = (work + threads - 1) / threads;
  if (b > 65536) b = 65536;
  if (b < 1) b = 1;
  return unsigned(b);
}

// streaming step passes (kernels_xstream.hip, kernels_sstream.hip); variant as
// for launch_xpass
hipError_t launch_xpass_stream(hipStream_t st, bool dbl, int n, const XPassArgs& a, int variant);
hipError_t launch_spass_stream(hipStream_t st, bool dbl, int n, const SPassArgs& a, int variant);

}  // namespace spin1
