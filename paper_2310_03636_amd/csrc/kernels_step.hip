// The grouped x-pass over several groups and the 1D multi-step kernel of the
// spin-1 step (gfx950), with their launchers.
#include "pass_common.hpp"

namespace spin1 {

// --------------------------------------------------------------------------
// Grouped x-pass: the step x-passes of several groups (different pencil
// lengths N) in one persistent launch.  Radix 8 for every N, so each thread
// holds the same 3 x 8 values whatever the group; a workgroup of 256 threads
// runs P = 2048 / N pencils of N / 8 threads.  The workgroup walks the
// concatenated item list with a stride of gridDim.x; items of one group are
// contiguous, so it reloads the group's tables (staged twiddles, the halves
// k <= N/2 of the two phase rows, the phase being even in k) into LDS at most
// once per group.  It does not prefetch the next item: on the uneven batch
// (1D 4096 x 128, 256^2 x 32, 512^2 x 16, 1024^2 x 4) the launch took 178 us
// with a prefetch register set and 160 us without one, both at two
// wavefronts per SIMD.
// --------------------------------------------------------------------------
template <typename Real>
struct GroupedX {
  static constexpr int R = 8, THREADS = 256;
  static constexpr int NMAX = sizeof(Real) == 4 ? 1024 : 512;
  static constexpr int ROWS_LDS = (THREADS * R / 16) * 17;  // P (N + N/16) for every N >= 16
  static constexpr int PH_HALF = NMAX / 2 + 1;                // entries of one half phase row
  // FP32: two wavefronts per SIMD (at three the kernel spills, and measured slower)
  static constexpr int WAVES_PER_EU = sizeof(Real) == 4 ? 2 : 1;
};

// DITHER: plain complex tables, dithered per step
template <typename Real, int N, bool DITHER, class TE>
__device__ __forceinline__ void grouped_x_body(Cx<Real> (&v)[3][8], int tid, Cx<Real>* lds, const TE* stw,
                                               const TE* ph) {
  constexpr int R = 8, T = N / R;
  const int t = tid % T, p = tid / T;
  RowLds<Real, N, T, (T <= 64)> L{lds + p * RowPad<N, T>::ROW};
  // ph: the half rows k <= N/2 of m = +1 (also m = -1) and m = 0, one after the other
#pragma unroll
  for (int m = 0; m < 3; ++m) {
    if constexpr (DITHER)
      fft_halfphase_ifft<Real, N, R>(v[m], t, L, StagedTwiddlesPlain<Real, N, R>{stw}, ph + (m == 1 ? N / 2 + 1 : 0),
                                     static_cast<const TE*>(nullptr));
    else
      fft_halfphase_ifft<Real, N, R>(v[m], t, L, StagedTwiddles<Real, N, R>{stw}, ph + (m == 1 ? N / 2 + 1 : 0),
                                     static_cast<const TE*>(nullptr));
  }
}

template <typename Real, bool DITHER>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(GroupedX<Real>::WAVES_PER_EU))) void
k_xpass_grouped(XGroupArgs a) {
  using C = Cx<Real>;
  using G = GroupedX<Real>;
  using TE = std::conditional_t<DITHER, C, TabEntry<Real>>;
  constexpr int R = G::R, NMAX = G::NMAX;
  __shared__ C lds[G::ROWS_LDS];
  __shared__ TE stw[NMAX - R];
  __shared__ TE ph[2 * G::PH_HALF];
  // a table entry in the kernel's form: hi+lo, or the dithered float pair
  auto entry = [&](const TabEntry<Real>& w, uint32_t i) -> TE {
    if constexpr (DITHER)
      return C{dither_round(w.hr, w.lr, a.tick, dither_salt(2 * i)),
               dither_round(w.hi, w.li, a.tick, dither_salt(2 * i + 1))};
    else
      return w;
  };
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
    if (!place(g, item, &pid, &t)) {  // a pencil past the group's end: defined values, never stored
#pragma unroll
      for (int m = 0; m < 3; ++m)
#pragma unroll
        for (int e = 0; e < R; ++e) dst[m][e] = C{Real(0), Real(0)};
      return;
    }
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
  const Real c0 = Real(a.c0), c1 = Real(a.c1);
  for (; item < a.item_end; item += gridDim.x) {
    const int g = group_of(item);
    if (g != cur) {  // uniform over the workgroup: every thread has the same item
      __syncthreads();
      const int n = a.g[g].n;
      const TabEntry<Real>* gtw = static_cast<const TabEntry<Real>*>(a.g[g].tw);
      const TabEntry<Real>* gph = static_cast<const TabEntry<Real>*>(a.g[g].ph);
      switch (n) {
        case 16: for (int i = tid; i < 16 - R; i += G::THREADS) stw[i] = entry(gtw[StagedTwiddles<Real, 16, R>::exponent(i)], i); break;
        case 32: for (int i = tid; i < 32 - R; i += G::THREADS) stw[i] = entry(gtw[StagedTwiddles<Real, 32, R>::exponent(i)], i); break;
        case 64: for (int i = tid; i < 64 - R; i += G::THREADS) stw[i] = entry(gtw[StagedTwiddles<Real, 64, R>::exponent(i)], i); break;
        case 128: for (int i = tid; i < 128 - R; i += G::THREADS) stw[i] = entry(gtw[StagedTwiddles<Real, 128, R>::exponent(i)], i); break;
        case 256: for (int i = tid; i < 256 - R; i += G::THREADS) stw[i] = entry(gtw[StagedTwiddles<Real, 256, R>::exponent(i)], i); break;
        case 512: for (int i = tid; i < 512 - R; i += G::THREADS) stw[i] = entry(gtw[StagedTwiddles<Real, 512, R>::exponent(i)], i); break;
        default:
          if constexpr (NMAX >= 1024)
            for (int i = tid; i < 1024 - R; i += G::THREADS)
              stw[i] = entry(gtw[StagedTwiddles<Real, 1024, R>::exponent(i)], i);
          break;
      }
      const int h = n / 2 + 1;
      for (int i = tid; i < 2 * h; i += G::THREADS) ph[i] = entry(gph[i < h ? i : n + (i - h)], i + 4096);
      __syncthreads();
      cur = g;
    }
    C v[3][R];
    load3(v, g, item);
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
      case 16: grouped_x_body<Real, 16, DITHER>(v, tid, lds, stw, ph); break;
      case 32: grouped_x_body<Real, 32, DITHER>(v, tid, lds, stw, ph); break;
      case 64: grouped_x_body<Real, 64, DITHER>(v, tid, lds, stw, ph); break;
      case 128: grouped_x_body<Real, 128, DITHER>(v, tid, lds, stw, ph); break;
      case 256: grouped_x_body<Real, 256, DITHER>(v, tid, lds, stw, ph); break;
      case 512: grouped_x_body<Real, 512, DITHER>(v, tid, lds, stw, ph); break;
      default:
        if constexpr (NMAX >= 1024) grouped_x_body<Real, 1024, DITHER>(v, tid, lds, stw, ph);
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

// --------------------------------------------------------------------------
// 1D: several steps per launch.  A 1D sample is one pencil, so a workgroup
// can keep it in registers for K consecutive split steps with no HBM traffic
// in between: load, K x [R(tau) -> FFT -> phase -> inverse FFT], optional
// closing R(dt/2), store.  One pencil per workgroup (the sample count is the
// parallelism), radix 8, N/8 threads each holding the same eight sites of the
// three components, so the local update needs no exchange.  The kinetic phase
// of the thread's own wavenumbers (even in k) is loaded once into registers,
// and the Zeeman factor exp(-i q dt) of m = +-1 is a uniform value.
//
// LDS holds the exchange rows and the twiddles.  Where N is a power of the
// radix and two rows fit, the exchanges use the two rows in turn, which
// halves the workgroup barriers (see fft_stages_2row).  In double precision
// the twiddles are then held as two base values per butterfly and stage (see
// BaseTwiddles), 18 KB at N = 4096 instead of 64 KB for every power, which is
// what makes room for the second 68 KB row.  The twiddles are re-read from
// LDS in every step: kept in registers across steps (the compiler would hoist
// them out of the step loop) they would spill.
// --------------------------------------------------------------------------

// Double precision: the twiddles of the stage with sub-transform size Ns as
// two base values per butterfly, w^j and w^(2j) (w = exp(-2 pi i / (Ns R))),
// the stages Ns = R, R^2, ..., N/R one after another from butterfly entry
// (Ns - R)/(R - 1).  The other powers w^(j r) are formed in registers by
// products of depth at most two (a few units of FP64 rounding, against one
// for a table of every power, in a quarter of its space).
template <int N, int R>
struct BaseTwiddles {
  static_assert(R == 8, "powers formed for radix 8");
  const Cx<double>* t;
  static constexpr int BUTTERFLIES = (N - R) / (R - 1);
  static constexpr int SIZE = 2 * BUTTERFLIES;
  // exponent m of entry i in exp(-2 pi i m / N) (table construction)
  __device__ static __forceinline__ int exponent(int i) {
    int j = i >> 1, ns = R;
    while (j >= ns) {
      j -= ns;
      ns *= R;
    }
    return ((i & 1) + 1) * j * (N / (ns * R));
  }
};

__device__ __forceinline__ void twiddle_powers(Cx<double> (&p)[8], Cx<double> w1, Cx<double> w2) {
  p[1] = w1;
  p[2] = w2;
  p[3] = w2 * w1;
  p[4] = w2 * w2;
  p[5] = p[4] * w1;
  p[6] = p[4] * w2;
  p[7] = p[4] * p[3];
}

template <int N, int Ns, int R, typename Real>
__device__ __forceinline__ void apply_twiddles(Cx<Real> (&w)[R], const StagedTwiddles<Real, N, R>& tw, int j) {
#pragma unroll
  for (int r = 1; r < R; ++r) w[r] = mul_tab(w[r], tw_at<N, Ns, R>(tw, j, r));
}
template <int N, int Ns, int R>
__device__ __forceinline__ void apply_twiddles(Cx<double> (&w)[R], const BaseTwiddles<N, R>& tw, int j) {
  Cx<double> p[R];
  const Cx<double>* e = tw.t + 2 * ((Ns - R) / (R - 1) + j);
  twiddle_powers(p, e[0], e[1]);
#pragma unroll
  for (int r = 1; r < R; ++r) w[r] = w[r] * p[r];
}

// The stages of fft_stages for N a power of R (one butterfly per thread, the
// same index maps), with two exchange rows ROW elements apart used in turn.
// An exchange writes the row at offset buf, waits at a barrier and reads it
// back; the next exchange writes the other row, which every thread finished
// reading before that barrier, so the barrier after the reads is not needed.
// buf (0 or ROW) carries the turn from one transform to the next.
template <typename Real, int N, int R, int ROW, int Ns, class Lds, class TW>
__device__ __forceinline__ void fft_stages_2row(Cx<Real>* v, int t, Lds& lds, int& buf, const TW& tw) {
  if constexpr (Ns < N) {
    constexpr int T = N / R;
    static_assert(StageRadix<N, R, Ns>::value == R, "N must be a power of R");
    const int j = t & (Ns - 1);
    Cx<Real> w[R];
#pragma unroll
    for (int r = 0; r < R; ++r) w[r] = v[r];
    if constexpr (Ns > 1) apply_twiddles<N, Ns, R>(w, tw, j);
    dft<Real, R>(w);
    if constexpr (Ns * R == N) {
#pragma unroll
      for (int r = 0; r < R; ++r) v[r] = w[r];
    } else {
      const int sb = lds.slot((t / Ns) * Ns * R + j) + buf;
#pragma unroll
      for (int r = 0; r < R; ++r) lds.store_slot(sb + Lds::off(r * Ns), w[r]);
      lds.sync();
      const int lb = lds.slot(t) + buf;
#pragma unroll
      for (int e = 0; e < R; ++e) v[e] = lds.load_slot(lb + Lds::off(e * T));
      buf = ROW - buf;
      fft_stages_2row<Real, N, R, ROW, Ns * R>(v, t, lds, buf, tw);
    }
  }
}

template <int N, typename Real>
struct MultiCfg {
  static constexpr int R = N <= 8 ? N : 8;
  static constexpr int T = N / R;
  static constexpr bool POW = N == 8 || N == 64 || N == 512 || N == 4096;  // N a power of R
  static constexpr bool BASE = sizeof(Real) == 8 && POW && N > R;
  // row padding: one element after every 2^SH (one per 8 for the single
  // double-precision row; one per 16 where the base-value twiddles share LDS
  // with two rows, measured equal to one per 8 there)
  static constexpr int SH = (sizeof(Real) == 8 && !BASE) ? 3 : 4;
  static constexpr int ROW = RowPad<N, T, SH>::ROW;
  using TW = std::conditional_t<BASE, BaseTwiddles<N, R>, StagedTwiddles<Real, N, R>>;
  using TWE = std::conditional_t<BASE, Cx<double>, TabEntry<Real>>;
  static constexpr int TW_ENTRIES = TW::SIZE > 0 ? TW::SIZE : 1;
  static constexpr int TW_BYTES = TW_ENTRIES * int(sizeof(TWE));
  static constexpr int ROW_BYTES = ROW * int(sizeof(Cx<Real>));
  static constexpr bool TWO_ROWS = POW && 2 * ROW_BYTES + TW_BYTES <= 160 * 1024;
  static_assert(!BASE || TWO_ROWS, "the base-value twiddles serve the two-row form");
  static constexpr int ROWS = TWO_ROWS ? 2 : 1;
  static constexpr bool fits() { return ROWS * ROW_BYTES + TW_BYTES <= 160 * 1024; }
};

// Forward FFT, multiply by the per-element factors ph[e] (and the uniform zq
// when given), inverse FFT through conj(FFT(conj(.))).
template <typename Real, int N, class Lds, class TW>
__device__ __forceinline__ void fft_regphase_ifft(Cx<Real>* v, int t, Lds& lds, int& buf, const TW& tw,
                                                  const TabEntry<Real> (&ph)[MultiCfg<N, Real>::R],
                                                  const TabEntry<Real>* zq) {
  using Cfg = MultiCfg<N, Real>;
  constexpr int R = Cfg::R;
  auto fft = [&]() {
    if constexpr (Cfg::TWO_ROWS)
      fft_stages_2row<Real, N, R, Cfg::ROW, 1>(v, t, lds, buf, tw);
    else
      fft_pencil<Real, N, R>(v, t, lds, tw);
  };
  fft();
#pragma unroll
  for (int e = 0; e < R; ++e) {
    Cx<Real> x = mul_tab(v[e], ph[e]);
    if (zq) x = mul_tab(x, *zq);
    v[e] = conj(x);
  }
  fft();
#pragma unroll
  for (int e = 0; e < R; ++e) v[e] = conj(v[e]);
}

template <typename Real, int N, bool ENABLED = MultiCfg<N, Real>::fits()>
__global__ __launch_bounds__((MultiCfg<N, Real>::T)) void k_x1d_multi(XPassArgs a, int K, double dt, int open_half,
                                                                       int close_half) {
 if constexpr (ENABLED) {
  using C = Cx<Real>;
  using Cfg = MultiCfg<N, Real>;
  using TW = typename Cfg::TW;
  using TWE = typename Cfg::TWE;
  constexpr int R = Cfg::R, T = Cfg::T, SH = Cfg::SH;
  __shared__ C lds[Cfg::ROWS * Cfg::ROW];
  __shared__ TWE stw[Cfg::TW_ENTRIES];
  const int t = threadIdx.x;
  TabEntry<Real> ph[R];
  TabEntry<Real> zq;
  {
    const TabEntry<Real>* gtw = static_cast<const TabEntry<Real>*>(a.tw);
    const TabEntry<Real>* gph = static_cast<const TabEntry<Real>*>(a.ph) + N;  // m = 0 row
    for (int i = t; i < TW::SIZE; i += T) {
      if constexpr (Cfg::BASE) {
        const TabEntry<Real> w = gtw[TW::exponent(i)];
        stw[i] = C{w.hr, w.hi};
      } else {
        stw[i] = gtw[TW::exponent(i)];
      }
    }
#pragma unroll
    for (int e = 0; e < R; ++e) ph[e] = gph[t + e * T];
    double sn, cs;
    sincos(a.q * dt, &sn, &cs);
    store_tab(&zq, wave_uniform(cs), -wave_uniform(sn));  // the same in every lane
    __syncthreads();
  }
  RowLds<Real, N, T, (T <= 64), SH> L{lds};
  int buf = 0;
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
      // one site at a time: interleaving the eight sites' updates would need
      // registers the double-precision form does not have at 512 threads
      if constexpr (sizeof(Real) == 8) __builtin_amdgcn_sched_barrier(0);
    }
  };
  for (int k = 0; k < K; ++k) {
    local_all(Real((k == 0 && open_half) ? 0.5 * dt : dt));
    // an offset the compiler cannot see through keeps the twiddle reads in
    // the step loop (see above)
    int keep = 0, tk = t;
    asm volatile("" : "+v"(keep), "+v"(tk));
    const TW tw{stw + keep};
    fft_regphase_ifft<Real, N>(v[0], tk, L, buf, tw, ph, &zq);
    fft_regphase_ifft<Real, N>(v[1], tk, L, buf, tw, ph, static_cast<const TabEntry<Real>*>(nullptr));
    fft_regphase_ifft<Real, N>(v[2], tk, L, buf, tw, ph, &zq);
  }
  if (close_half) local_all(Real(0.5 * dt));
#pragma unroll
  for (int m = 0; m < 3; ++m)
#pragma unroll
    for (int e = 0; e < R; ++e) psi[m * a.sites + e * T] = v[m][e];
 }
}

// --------------------------------------------------------------------------
// 1D, latency form: the three components of a sample in three thread groups
// of T = min(64, N/2) lanes (one wavefront each from N = 128 on), so the three
// transforms of a step run side by side instead of one after another.  The
// local update regroups the components through LDS: each group writes its
// component into its LDS row in natural order, the workgroup synchronises,
// every thread updates whole sites (all three components), and each group
// reads its component back.  A group's transforms exchange only within its
// own row and wavefront.
// --------------------------------------------------------------------------
template <int N>
struct SplitCfg {
  static constexpr int R = N / 64 > 16 ? 16 : (N / 64 > 2 ? N / 64 : 2);
  static constexpr int T = N / R;
  static constexpr int THREADS = 3 * T;
  static constexpr int ROW = RowPad<N, T>::ROW;
  // three rows, staged twiddles and the half phase table in 160 KB of LDS
  template <typename Real>
  static constexpr bool fits() {
    return 3 * ROW * int(sizeof(Cx<Real>)) + (N - R + N / 2 + 2) * int(sizeof(TabEntry<Real>)) <= 160 * 1024;
  }
};

template <typename Real, int N, bool ENABLED = SplitCfg<N>::template fits<Real>()>
__global__ __launch_bounds__((SplitCfg<N>::THREADS)) void k_x1d_split(XPassArgs a, int K, double dt, int open_half,
                                                                       int close_half) {
 if constexpr (ENABLED) {
  using C = Cx<Real>;
  using Cfg = SplitCfg<N>;
  constexpr int R = Cfg::R, T = Cfg::T, ROW = Cfg::ROW;
  using TW = StagedTwiddles<Real, N, R>;
  __shared__ C rows[3 * ROW];
  __shared__ TabEntry<Real> stw[TW::SIZE > 0 ? TW::SIZE : 1];
  __shared__ TabEntry<Real> ph0[N / 2 + 1];
  __shared__ TabEntry<Real> zq;
  const int tid = threadIdx.x;
  const int m = tid / T, t = tid - m * T;
  {
    const TabEntry<Real>* gtw = static_cast<const TabEntry<Real>*>(a.tw);
    const TabEntry<Real>* gph = static_cast<const TabEntry<Real>*>(a.ph) + N;  // m = 0 row
    for (int i = tid; i < TW::SIZE; i += Cfg::THREADS) stw[i] = gtw[TW::exponent(i)];
    for (int i = tid; i <= N / 2; i += Cfg::THREADS) ph0[i] = gph[i];
    if (tid == 0) {
      double sn, cs;
      sincos(a.q * dt, &sn, &cs);
      store_tab(&zq, cs, -sn);
    }
    __syncthreads();
  }
  // up to T = 64 a group never straddles a wavefront (T is a power of two) and
  // exchanges within it; longer rows synchronise the workgroup, which every
  // group reaches equally often
  RowLds<Real, N, T, (T <= 64)> L{rows + m * ROW};
  C* psi = static_cast<C*>(a.psi) + int64_t(blockIdx.x) * 3 * a.sites + m * a.sites + t;
  C v[R];
#pragma unroll
  for (int e = 0; e < R; ++e) v[e] = psi[e * T];
  const Real c0 = Real(a.c0), c1 = Real(a.c1);
  const TabEntry<Real>* zm = m == 1 ? nullptr : &zq;
  auto local_all = [&](Real tau) {
#pragma unroll
    for (int e = 0; e < R; ++e) L.store(t + e * T, v[e]);
    __syncthreads();
    for (int s = tid; s < N; s += Cfg::THREADS) {
      const int i = RowPad<N, T>::at(s);
      C site[3] = {rows[i], rows[ROW + i], rows[2 * ROW + i]};
      local_update(site, tau, c0, c1);
      rows[i] = site[0];
      rows[ROW + i] = site[1];
      rows[2 * ROW + i] = site[2];
    }
    __syncthreads();
#pragma unroll
    for (int e = 0; e < R; ++e) v[e] = L.load(t + e * T);
    // the group's next LDS writes (its own row) follow these reads in order
  };
  for (int k = 0; k < K; ++k) {
    local_all(Real((k == 0 && open_half) ? 0.5 * dt : dt));
    fft_halfphase_ifft<Real, N, R>(v, t, L, TW{stw}, ph0, zm);
  }
  if (close_half) local_all(Real(0.5 * dt));
#pragma unroll
  for (int e = 0; e < R; ++e) psi[e * T] = v[e];
 }
}

// --------------------------------------------------------------------------
// launchers
// --------------------------------------------------------------------------
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
  if constexpr (sizeof(Real) == 4) {
    if (a.dither) {
      const int64_t grid = stream_grid(k_xpass_grouped<Real, true>, GroupedX<Real>::THREADS, a.item_end);
      (void)launch_kernel((k_xpass_grouped<Real, true>), dim3(unsigned(grid)), dim3(GroupedX<Real>::THREADS), 0, st, a);
      return hipGetLastError();
    }
  }
  const int64_t grid = stream_grid(k_xpass_grouped<Real, false>, GroupedX<Real>::THREADS, a.item_end);
  (void)launch_kernel((k_xpass_grouped<Real, false>), dim3(unsigned(grid)), dim3(GroupedX<Real>::THREADS), 0, st, a);
  return hipGetLastError();
}

hipError_t launch_xpass_grouped(hipStream_t st, bool dbl, const XGroupArgs& a) {
  return dbl ? xpass_grouped_t<double>(st, a) : xpass_grouped_t<float>(st, a);
}

template <typename Real, int N>
static hipError_t x1d_multi_n(hipStream_t st, const XPassArgs& a, int K, double dt, bool open_half, bool close_half,
                              bool split) {
  // the latency form where its LDS fits (every size but 4096), else the pencil form
  if (split && SplitCfg<N>::template fits<Real>())
    (void)launch_kernel((k_x1d_split<Real, N>), dim3(unsigned(a.S)), dim3(SplitCfg<N>::THREADS), 0, st, a, K, dt,
                       int(open_half), int(close_half));
  else if (!MultiCfg<N, Real>::fits())
    return hipErrorInvalidValue;
  else
    (void)launch_kernel((k_x1d_multi<Real, N>), dim3(unsigned(a.S)), dim3(MultiCfg<N, Real>::T), 0, st, a, K, dt,
                       int(open_half), int(close_half));
  return hipGetLastError();
}

template <typename Real>
static hipError_t x1d_multi_t(hipStream_t st, int n, const XPassArgs& a, int K, double dt, bool oh, bool ch,
                               bool sp) {
  switch (n) {
    case 8: return x1d_multi_n<Real, 8>(st, a, K, dt, oh, ch, sp);
    case 16: return x1d_multi_n<Real, 16>(st, a, K, dt, oh, ch, sp);
    case 32: return x1d_multi_n<Real, 32>(st, a, K, dt, oh, ch, sp);
    case 64: return x1d_multi_n<Real, 64>(st, a, K, dt, oh, ch, sp);
    case 128: return x1d_multi_n<Real, 128>(st, a, K, dt, oh, ch, sp);
    case 256: return x1d_multi_n<Real, 256>(st, a, K, dt, oh, ch, sp);
    case 512: return x1d_multi_n<Real, 512>(st, a, K, dt, oh, ch, sp);
    case 1024: return x1d_multi_n<Real, 1024>(st, a, K, dt, oh, ch, sp);
    case 2048: return x1d_multi_n<Real, 2048>(st, a, K, dt, oh, ch, sp);
    case 4096: return x1d_multi_n<Real, 4096>(st, a, K, dt, oh, ch, sp);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_x1d_multi(hipStream_t st, bool dbl, int n, const XPassArgs& a, int K, double dt, bool open_half,
                            bool close_half, bool split) {
  return dbl ? x1d_multi_t<double>(st, n, a, K, dt, open_half, close_half, split)
             : x1d_multi_t<float>(st, n, a, K, dt, open_half, close_half, split);
}

}  // namespace spin1
