// Device building blocks of the spin-1 split-step library (gfx950).
//
//  * Cx<Real>        interleaved complex value (complex64 / complex128 layout)
//  * dft<Real, R>    in-register radix-R DFT, R = 1, 2, 4, 8, 16, 32
//  * fft_pencil      Stockham autosort FFT of one pencil of length N, held as
//                    R values per thread (thread t owns indices t + e*N/R),
//                    exchanging through LDS between stages
//  * local_update    exact local (c0, c1) flow over tau at one site
//  * philox4x64_10   counter-based generator for the Wigner noise
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

namespace spin1 {

template <typename Real>
struct alignas(2 * sizeof(Real)) Cx {
  Real re, im;
};

// Store of one complex value; NT: non-temporal (the line is not kept in the
// caches: for fields that the next pass cannot find in the last-level cache
// anyway)
template <bool NT, typename Real>
__device__ __forceinline__ void put(Cx<Real>* p, Cx<Real> c) {
  if constexpr (NT) {
    typedef Real V __attribute__((ext_vector_type(2)));
    const V v = {c.re, c.im};
    __builtin_nontemporal_store(v, reinterpret_cast<V*>(p));
  } else {
    *p = c;
  }
}

template <typename Real>
__device__ __forceinline__ Cx<Real> operator+(Cx<Real> a, Cx<Real> b) { return {a.re + b.re, a.im + b.im}; }
template <typename Real>
__device__ __forceinline__ Cx<Real> operator-(Cx<Real> a, Cx<Real> b) { return {a.re - b.re, a.im - b.im}; }
template <typename Real>
__device__ __forceinline__ Cx<Real> operator*(Cx<Real> a, Cx<Real> b) {
  return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
template <typename Real>
__device__ __forceinline__ Cx<Real> scale(Cx<Real> a, Real s) { return {a.re * s, a.im * s}; }
template <typename Real>
__device__ __forceinline__ Cx<Real> conj(Cx<Real> a) { return {a.re, -a.im}; }
// conj(a) * b
template <typename Real>
__device__ __forceinline__ Cx<Real> cmulc(Cx<Real> a, Cx<Real> b) {
  return {a.re * b.re + a.im * b.im, a.re * b.im - a.im * b.re};
}
template <typename Real>
__device__ __forceinline__ Real norm2(Cx<Real> a) { return a.re * a.re + a.im * a.im; }
// a p + sign b conj(q) (sign = +1 or -1) as one chain of fused multiply-adds
// per part: one product and three FMAs, each part rounded once at its end
template <int SIGN, typename Real>
__device__ __forceinline__ Cx<Real> mul_add_conj(Cx<Real> a, Cx<Real> p, Cx<Real> b, Cx<Real> q) {
  static_assert(SIGN == 1 || SIGN == -1, "sign");
  const Real sb = Real(SIGN);
  // b conj(q) = (b.re q.re + b.im q.im) + i (b.im q.re - b.re q.im)
  const Real re = fma(a.re, p.re, fma(-a.im, p.im, sb * fma(b.re, q.re, b.im * q.im)));
  const Real im = fma(a.re, p.im, fma(a.im, p.re, sb * fma(b.im, q.re, -(b.re * q.im))));
  return {re, im};
}

// ---------------------------------------------------------------------------
// Table entries (twiddles, phase factors).  They are computed in FP64; the
// single-precision path keeps each value as an unevaluated sum hi + lo of two
// floats.  A kernel either multiplies by hi + lo (compensated: no rounding of
// the constant) or builds plain floats from them per step with dither_round.
// A constant rounded once would repeat the same relative error in every step,
// and the errors would add up linearly over a run.
// ---------------------------------------------------------------------------
template <typename Real>
struct TabEntry;
template <>
struct alignas(16) TabEntry<float> {
  float hr, hi, lr, li;
};
template <>
struct alignas(16) TabEntry<double> {
  double hr, hi;
};

__device__ __forceinline__ Cx<float> mul_tab(Cx<float> x, TabEntry<float> w) {
  const float cre = x.re * w.lr - x.im * w.li;
  const float cim = x.re * w.li + x.im * w.lr;
  return {fmaf(x.re, w.hr, fmaf(-x.im, w.hi, cre)), fmaf(x.re, w.hi, fmaf(x.im, w.hr, cim))};
}
__device__ __forceinline__ Cx<double> mul_tab(Cx<double> x, TabEntry<double> w) {
  return {x.re * w.hr - x.im * w.hi, x.re * w.hi + x.im * w.hr};
}

// One of the two floats next to the FP64 value h + l (h = nearest float, l the
// remainder), chosen per tick so that the running mean of the choices over
// consecutive ticks tracks h + l (error diffusion with a per-entry offset
// `salt`): the rounding of a constant used once per step then does not add up
// step after step.
__device__ __forceinline__ float dither_round(float h, float l, int64_t tick, uint32_t salt) {
  if (l == 0.0f) return h;
  const float alt = nextafterf(h, l > 0.0f ? __builtin_inff() : -__builtin_inff());
  const float p = l / (alt - h);  // in (0, 1/2]
  // the pattern repeats every 2^16 steps; within that, float holds p * tick
  // to well under one unit
  const float k = float(tick & 0xffff), off = float(salt >> 8) * (1.0f / 16777216.0f);
  const bool up = floorf(fmaf(p, k + 1.0f, off)) > floorf(fmaf(p, k, off));
  return up ? alt : h;
}
__device__ __forceinline__ uint32_t dither_salt(uint32_t i) { return i * 2654435761u; }

// multiply by a table value kept as one plain complex number (rounded once)
template <typename Real>
__device__ __forceinline__ Cx<Real> mul_tab(Cx<Real> x, Cx<Real> w) {
  return x * w;
}

// x * (c_hi + c_lo) for a real constant given in FP64, compensated in FP32
template <typename Real>
__device__ __forceinline__ Real mul_const(Real x, double c) {
  if constexpr (sizeof(Real) == 8) {
    return x * c;
  } else {
    const float hi = float(c);
    const float lo = float(c - double(hi));
    return fmaf(x, hi, x * lo);
  }
}
// x*c + y*s for FP64 constants c, s, compensated in FP32
template <typename Real>
__device__ __forceinline__ Real dot_const(Real x, double c, Real y, double s) {
  if constexpr (sizeof(Real) == 8) {
    return x * c + y * s;
  } else {
    const float ch = float(c), cl = float(c - double(ch));
    const float sh = float(s), sl = float(s - double(sh));
    return fmaf(x, ch, fmaf(y, sh, x * cl + y * sl));
  }
}

// ---------------------------------------------------------------------------
// In-register DFT: out[k] = sum_r v[r] exp(-2 pi i r k / R), radix-2 split
// into even and odd halves, constant twiddles specialised at compile time.
// ---------------------------------------------------------------------------
// cos(pi k / 16), k = 0..8; the other angles of a radix <= 32 DFT follow by
// symmetry (cos(pi (16 - k)/16) = -cos(pi k/16), sin(pi k/16) = cos(pi (8 - k)/16))
__device__ constexpr double kCos32[9] = {1.0,
                                         0.98078528040323044912618223613424,
                                         0.92387953251128675612818318939679,
                                         0.83146961230254523707878837761791,
                                         0.70710678118654752440084436210485,
                                         0.55557023301960222474283081394853,
                                         0.38268343236508977172845998403040,
                                         0.19509032201612826784828486847702,
                                         0.0};

constexpr double cos_pi16(int i) { return i <= 8 ? kCos32[i] : -kCos32[16 - i]; }
constexpr double sin_pi16(int i) { return i <= 8 ? kCos32[8 - i] : kCos32[i - 8]; }

// v * exp(-2 pi i K / R) = v * exp(-i pi I / 16), I = K * 32 / R < 16; the
// irrational constants go through mul_const / dot_const so the single-
// precision path uses them at full FP64 accuracy
template <typename Real, int R, int K>
__device__ __forceinline__ Cx<Real> twiddle_const(Cx<Real> v) {
  static_assert(R <= 32 && 2 * K < R, "twiddle of a radix <= 32 half");
  constexpr int I = K * (32 / R);
  constexpr double h = 0.70710678118654752440;
  if constexpr (I == 0) {
    return v;
  } else if constexpr (I == 8) {
    return {v.im, -v.re};
  } else if constexpr (I == 4) {
    return {mul_const<Real>(v.re + v.im, h), mul_const<Real>(v.im - v.re, h)};
  } else if constexpr (I == 12) {
    return {mul_const<Real>(v.im - v.re, h), -mul_const<Real>(v.re + v.im, h)};
  } else {
    constexpr double c = cos_pi16(I);
    constexpr double s = sin_pi16(I);
    return {dot_const<Real>(v.re, c, v.im, s), dot_const<Real>(v.im, c, v.re, -s)};
  }
}

template <typename Real, int R, int K>
__device__ __forceinline__ void dft_combine(Cx<Real>* v, const Cx<Real>* e, const Cx<Real>* o) {
  if constexpr (K < R / 2) {
    const Cx<Real> t = twiddle_const<Real, R, K>(o[K]);
    v[K] = e[K] + t;
    v[K + R / 2] = e[K] - t;
    dft_combine<Real, R, K + 1>(v, e, o);
  }
}

template <typename Real, int R>
__device__ __forceinline__ void dft(Cx<Real>* v) {
  static_assert(R == 1 || R == 2 || R == 4 || R == 8 || R == 16 || R == 32, "radix");
  if constexpr (R == 2) {
    const Cx<Real> a = v[0], b = v[1];
    v[0] = a + b;
    v[1] = a - b;
  } else if constexpr (R > 2) {
    Cx<Real> e[R / 2], o[R / 2];
#pragma unroll
    for (int i = 0; i < R / 2; ++i) {
      e[i] = v[2 * i];
      o[i] = v[2 * i + 1];
    }
    dft<Real, R / 2>(e);
    dft<Real, R / 2>(o);
    dft_combine<Real, R, 0>(v, e, o);
  }
}

// ---------------------------------------------------------------------------
// Stockham FFT of one pencil.  Stage s has radix Rs (R, except a smaller last
// radix when N is not a power of R) and sub-transform size Ns = product of the
// earlier radices.  Butterfly b reads indices b + r*N/Rs, multiplies element r
// by w^(j r) with j = b mod Ns and w = exp(-2 pi i / (Ns Rs)), applies the
// radix-Rs DFT and writes to (b / Ns) * Ns * Rs + j + r * Ns.  Thread t runs
// the R/Rs butterflies b = t + u*N/R; the elements it reads are always its own
// indices t + e*N/R, and in the last stage the outputs land on those same
// indices, so input and output stay in registers in natural order.
//
// Lds: slot(i) (the LDS element of index i), off(k) (the slot step of a
// compile-time index step k), store_slot / load_slot and sync() (a workgroup
// barrier, or a wavefront one where the pencil lies in one wavefront).
// tw: table exp(-2 pi i m / N), m < N, in global memory.
// ---------------------------------------------------------------------------
template <int N, int R, int Ns>
struct StageRadix {
  static constexpr int value = ((N / Ns) % R == 0) ? R : (N / Ns);
};

// Twiddle w^(j r N/(Ns Rs)) of butterfly j, element r, in the stage with
// sub-transform size Ns and radix Rs.  Default: TW indexable by the exponent
// m < N (a pointer to the full table, or HalfTwiddles).
template <int N, int Ns, int Rs, class TW>
__device__ __forceinline__ auto tw_at(const TW& tw, int j, int r) {
  return tw[j * r * (N / (Ns * Rs))];
}

// Twiddles laid out stage by stage: for the stage with Ns (a power of R) the
// entries (r - 1) * Ns + j, r = 1..Rs-1, j < Ns, follow each other from offset
// Ns - R (the earlier stages hold (R - 1)(R + R^2 + ... + Ns/R) entries); N - R
// entries in all.  The lanes of a pencil read consecutive entries, which keeps
// LDS reads free of bank conflicts where the exponent-indexed table puts the
// butterflies of a stage N/(Ns Rs) entries apart.
template <typename Real, int N, int R>
struct StagedTwiddles {
  const TabEntry<Real>* t;
  static constexpr int SIZE = N - R;
  // exponent of entry i (table construction)
  __device__ static __forceinline__ int exponent(int i) {
    int ns = R;
    while (i >= ns * ((N / ns) % R == 0 ? R - 1 : N / ns - 1)) {
      i -= ns * ((N / ns) % R == 0 ? R - 1 : N / ns - 1);
      ns *= R;
    }
    const int rs = (N / ns) % R == 0 ? R : N / ns;
    const int r = i / ns + 1, j = i % ns;
    return j * r * (N / (ns * rs));
  }
};
template <int N, int Ns, int Rs, typename Real, int R>
__device__ __forceinline__ TabEntry<Real> tw_at(const StagedTwiddles<Real, N, R>& tw, int j, int r) {
  static_assert(Ns >= R, "the first stage has no twiddles");
  return tw.t[(Ns - R) + (r - 1) * Ns + j];
}

// the same layout with each twiddle rounded once to a plain complex value
template <typename Real, int N, int R>
struct StagedTwiddlesPlain {
  const Cx<Real>* t;
};
template <int N, int Ns, int Rs, typename Real, int R>
__device__ __forceinline__ Cx<Real> tw_at(const StagedTwiddlesPlain<Real, N, R>& tw, int j, int r) {
  static_assert(Ns >= R, "the first stage has no twiddles");
  return tw.t[(Ns - R) + (r - 1) * Ns + j];
}

// TW: see tw_at
template <typename Real, int N, int R, int Ns, class Lds, class TW>
__device__ __forceinline__ void fft_stages(Cx<Real>* v, int t, Lds& lds, const TW& tw) {
  if constexpr (Ns < N) {
    constexpr int Rs = StageRadix<N, R, Ns>::value;
    constexpr int U = R / Rs;
    constexpr int T = N / R;
    constexpr bool last = (Ns * Rs == N);
    static_assert(R % Rs == 0, "stage radix must divide R");
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int b = t + u * T;
      const int j = b & (Ns - 1);
      Cx<Real> w[Rs];
#pragma unroll
      for (int r = 0; r < Rs; ++r) w[r] = v[u + r * U];
      if constexpr (Ns > 1) {
#pragma unroll
        for (int r = 1; r < Rs; ++r) w[r] = mul_tab(w[r], tw_at<N, Ns, Rs>(tw, j, r));
      }
      dft<Real, Rs>(w);
      if constexpr (last) {
#pragma unroll
        for (int r = 0; r < Rs; ++r) v[u + r * U] = w[r];
      } else {
        const int sb = lds.slot((b / Ns) * Ns * Rs + j);
#pragma unroll
        for (int r = 0; r < Rs; ++r) lds.store_slot(sb + Lds::off(r * Ns), w[r]);
      }
    }
    if constexpr (!last) {
      lds.sync();
      const int lb = lds.slot(t);
#pragma unroll
      for (int e = 0; e < R; ++e) v[e] = lds.load_slot(lb + Lds::off(e * T));
      lds.sync();
      fft_stages<Real, N, R, Ns * Rs>(v, t, lds, tw);
    }
  }
}

template <typename Real, int N, int R, class Lds, class TW>
__device__ __forceinline__ void fft_pencil(Cx<Real>* v, int t, Lds& lds, const TW& tw) {
  static_assert((N & (N - 1)) == 0 && N >= R, "N must be a power of two >= R");
  fft_stages<Real, N, R, 1>(v, t, lds, tw);
}

// Forward FFT, multiply by ph[k] (which carries the 1/N of the inverse),
// inverse FFT through conj(FFT(conj(.))).  ph is in natural k order; its
// entries are TabEntry (hi + lo) or plain complex values (PE).
template <typename Real, int N, int R, class Lds, class TW, class PE>
__device__ __forceinline__ void fft_phase_ifft(Cx<Real>* v, int t, Lds& lds, const TW& tw,
                                               const PE* __restrict__ ph) {
  constexpr int T = N / R;
  fft_pencil<Real, N, R>(v, t, lds, tw);
#pragma unroll
  for (int e = 0; e < R; ++e) v[e] = conj(mul_tab(v[e], ph[t + e * T]));
  fft_pencil<Real, N, R>(v, t, lds, tw);
#pragma unroll
  for (int e = 0; e < R; ++e) v[e] = conj(v[e]);
}

// Twiddles exp(-2 pi i m / N) from the half table m <= N/2 (conjugate symmetry
// w^(N-m) = conj(w^m)), for kernels that keep their tables in LDS.
template <typename Real, int N>
struct HalfTwiddles {
  const TabEntry<Real>* t;
  __device__ __forceinline__ TabEntry<Real> operator[](int m) const {
    if (m <= N / 2) return t[m];
    TabEntry<Real> w = t[N - m];
    w.hi = -w.hi;
    if constexpr (sizeof(Real) == 4) w.li = -w.li;
    return w;
  }
};

// Forward FFT, multiply by ph0[min(k, N-k)] (the kinetic phase with 1/N, even
// in k) and, when zq is given, by the uniform factor *zq, inverse FFT.
// Element e of thread t is k = t + e*N/R: below N/2 for e < R/2, at or above
// it otherwise, so the mirror choice is static.
template <typename Real, int N, int R, class Lds, class TW, class PE>
__device__ __forceinline__ void fft_halfphase_ifft(Cx<Real>* v, int t, Lds& lds, const TW& tw,
                                                   const PE* __restrict__ ph0, const PE* zq) {
  constexpr int T = N / R;
  static_assert(R >= 2, "the static mirror split needs two halves");
  fft_pencil<Real, N, R>(v, t, lds, tw);
#pragma unroll
  for (int e = 0; e < R; ++e) {
    const int k = e < R / 2 ? t + e * T : N - t - e * T;
    Cx<Real> x = mul_tab(v[e], ph0[k]);
    if (zq) x = mul_tab(x, *zq);
    v[e] = conj(x);
  }
  fft_pencil<Real, N, R>(v, t, lds, tw);
#pragma unroll
  for (int e = 0; e < R; ++e) v[e] = conj(v[e]);
}

// ---------------------------------------------------------------------------
// Exact local flow over tau of i d_t psi = (c0 n + c1 F.f) psi at one site.
// n and F are constant along it, and with M = F.f one has M^3 = |F|^2 M, so
//   exp(-i theta M) = 1 - i s M + c M^2,  theta = c1 tau,
//   s = sin(|F| theta)/|F| = theta sinc(x/2) cos(x/2),
//   c = (cos(|F| theta) - 1)/|F|^2 = -theta^2/2 sinc(x/2)^2,  x = |F| theta,
// and the c0 part is the scalar phase exp(-i c0 n tau).  Applied to the state
// psi that defines F, M takes a closed form: with the singlet-pair amplitude
// Theta = 2 psi_{+1} psi_{-1} - psi_0^2 and the time-reversed spinor
// tpsi_m = (-1)^m conj(psi_{-m}),
//   M psi = n psi + Theta tpsi,  M tpsi = -n tpsi - conj(Theta) psi,
// hence M^2 psi = (n^2 - |Theta|^2) psi = |F|^2 psi (the spin-1 identity
// |F|^2 + |Theta|^2 = n^2), and
//   exp(-i theta M) psi = (cos x - i n s) psi - i s Theta tpsi.
// The general form (apply_M below, with g = F_+/sqrt2:
//   (Mv)_{+1} = Fz v_{+1} + g* v_0,  (Mv)_0 = g v_{+1} + g* v_{-1},
//   (Mv)_{-1} = g v_0 - Fz v_{-1})
// serves the reverse mode and the paper's scheme.
// ---------------------------------------------------------------------------
// Series kernels on u = y^2 for |y| <= pi/4 (Taylor series): sinc(y) =
// sin(y)/y to u^4 (remainder below 2.2e-9 relative) and cos(y) to u^5
// (remainder below 2.5e-8 absolute), both under the single-precision ulp.
__device__ __forceinline__ float sinc_series(float u) {
  float p = fmaf(u, -1.0f / 362880.0f, 1.0f / 5040.0f);
  p = fmaf(u, p, -1.0f / 120.0f);
  p = fmaf(u, p, 1.0f / 6.0f);
  return fmaf(-u, p, 1.0f);
}
__device__ __forceinline__ float cos_series(float u) {
  float q = fmaf(u, -1.0f / 3628800.0f, 1.0f / 40320.0f);
  q = fmaf(u, q, -1.0f / 720.0f);
  q = fmaf(u, q, 1.0f / 24.0f);
  q = fmaf(u, q, -0.5f);
  return fmaf(u, q, 1.0f);
}

// The same series one term shorter, for |y| < 0.52 (u < 0.27): sinc to u^3
// (remainder below 1.5e-8 relative) and cos to u^4 (below 4e-10 absolute).
// The common path of the local update takes these; its arguments are small
// (c1 tau |F| / 2 and c0 n tau).
constexpr float kShortSeriesU = 0.27f;
__device__ __forceinline__ float sinc_series_short(float u) {
  float p = fmaf(u, -1.0f / 5040.0f, 1.0f / 120.0f);
  p = fmaf(u, p, -1.0f / 6.0f);
  return fmaf(u, p, 1.0f);
}
__device__ __forceinline__ float cos_series_short(float u) {
  float q = fmaf(u, 1.0f / 40320.0f, -1.0f / 720.0f);
  q = fmaf(u, q, 1.0f / 24.0f);
  q = fmaf(u, q, -0.5f);
  return fmaf(u, q, 1.0f);
}

struct SinCos {
  float s, c;
};

// |y| > 1e5: FP64 library evaluation, out of line and returned by value so
// that the hot path neither inlines it nor touches scratch memory.
__device__ __noinline__ SinCos sincos_huge(float y) {
  double s, c;
  sincos(double(y), &s, &c);
  return SinCos{float(s), float(c)};
}

// sin and cos of a float of any size: Cody-Waite reduction by pi/2 with a
// three-part constant (remainder exact to ~1e-12 for |y| <= 1e5), series on
// the remainder, quadrant swap.
__device__ __forceinline__ SinCos sincos_reduced(float y) {
  if (!(fabsf(y) <= 1.0e5f)) return sincos_huge(y);
  constexpr double kPio2 = 1.57079632679489661923;
  constexpr float c1 = float(kPio2);
  constexpr float c2 = float(kPio2 - double(c1));
  constexpr float c3 = float(kPio2 - double(c1) - double(c2));
  const float k = rintf(y * float(0.63661977236758134308));
  float r = fmaf(-k, c1, y);
  r = fmaf(-k, c2, r);
  r = fmaf(-k, c3, r);
  const float u = r * r;
  const float sr = r * sinc_series(u), cr = cos_series(u);
  const int q = int(k) & 3;
  const float s0 = (q & 1) ? cr : sr, c0 = (q & 1) ? sr : cr;
  return SinCos{(q & 2) ? -s0 : s0, ((q + 1) & 2) ? -c0 : c0};
}

// sin(y), cos(y) from y itself (single precision)
__device__ __forceinline__ void sincos_small(float y, float* s, float* c) {
  const float u = y * y;
  if (u < kShortSeriesU) {  // |y| < 0.52; beyond, the reduction (k = 0 up to pi/4) and full series
    *s = y * sinc_series_short(u);
    *c = cos_series_short(u);
  } else {
    const SinCos r = sincos_reduced(y);
    *s = r.s;
    *c = r.c;
  }
}

// sinc(y) and cos(y) from u = y^2 >= 0 (single precision): no square root on
// the common path
__device__ __forceinline__ void sinc_cos_from_square(float u, float* sc, float* c) {
  if (u < kShortSeriesU) {
    *sc = sinc_series_short(u);
    *c = cos_series_short(u);
  } else {
    const float y = sqrtf(u);
    const SinCos r = sincos_reduced(y);
    *c = r.c;
    *sc = r.s / y;
  }
}

// Double precision: Taylor series below |y| = 0.52 (u < 0.27), sinc to u^6
// (remainder below 8.1e-17 relative) and cos to u^7 (below 1.4e-18), and the
// library sincos, out of line, beyond (the local update's arguments c1 tau
// |F| / 2 and c0 n tau stay below it in every workload here).
// A double constant cannot be an immediate operand of a VALU instruction, and
// the compiler keeps such constants in vector registers (one pair each, live
// across the kernel's loops); passed through a scalar register pair at the
// point of use they cost a scalar move instead.
__device__ __forceinline__ double sreg(double c) {
  asm volatile("" : "+s"(c));
  return c;
}
constexpr double kShortSeriesUD = 0.27;
__device__ __forceinline__ double sinc_series_short(double u) {
  double p = fma(u, sreg(1.0 / 6227020800.0), sreg(-1.0 / 39916800.0));
  p = fma(u, p, sreg(1.0 / 362880.0));
  p = fma(u, p, sreg(-1.0 / 5040.0));
  p = fma(u, p, sreg(1.0 / 120.0));
  p = fma(u, p, sreg(-1.0 / 6.0));
  return fma(u, p, 1.0);
}
__device__ __forceinline__ double cos_series_short(double u) {
  double q = fma(u, sreg(-1.0 / 87178291200.0), sreg(1.0 / 479001600.0));
  q = fma(u, q, sreg(-1.0 / 3628800.0));
  q = fma(u, q, sreg(1.0 / 40320.0));
  q = fma(u, q, sreg(-1.0 / 720.0));
  q = fma(u, q, sreg(1.0 / 24.0));
  q = fma(u, q, -0.5);
  return fma(u, q, 1.0);
}
struct SinCosD {
  double s, c;
};
__device__ __noinline__ SinCosD sincos_lib(double y) {
  SinCosD r;
  sincos(y, &r.s, &r.c);
  return r;
}
__device__ __forceinline__ void sincos_small(double y, double* s, double* c) {
  const double u = y * y;
  if (u < kShortSeriesUD) {
    *s = y * sinc_series_short(u);
    *c = cos_series_short(u);
  } else {
    const SinCosD r = sincos_lib(y);
    *s = r.s;
    *c = r.c;
  }
}
__device__ __forceinline__ void sinc_cos_from_square(double u, double* sc, double* c) {
  if (u < kShortSeriesUD) {
    *sc = sinc_series_short(u);
    *c = cos_series_short(u);
  } else {
    const double y = sqrt(u);
    const SinCosD r = sincos_lib(y);
    *c = r.c;
    *sc = r.s / y;
  }
}

template <typename Real>
__device__ __forceinline__ void apply_M(const Cx<Real>* a, Cx<Real>* out, Cx<Real> g, Real fz) {
  out[0] = scale(a[0], fz) + cmulc(g, a[1]);
  out[1] = g * a[0] + cmulc(g, a[2]);
  out[2] = g * a[1] - scale(a[2], fz);
}

// s = theta sinc(x/2) cos(x/2) and c = -theta^2/2 sinc(x/2)^2 for x = |F| theta,
// |F|^2 = f2, and the phase exp(-i c0 n tau) as (cos, sin) of c0 n tau.
template <typename Real>
__device__ __forceinline__ void rotation_coeffs(Real f2, Real theta, Real* s, Real* c) {
  Real sc, ch;
  // f2 times a factor that is the same for every site (kept out of site loops)
  sinc_cos_from_square(f2 * (Real(0.25) * theta * theta), &sc, &ch);
  *s = theta * (sc * ch);
  *c = (Real(-0.5) * theta * theta) * (sc * sc);
}

template <typename Real>
__device__ __forceinline__ void angle_sincos(Real a, Real* sn, Real* cs) {
  sincos_small(a, sn, cs);
}

// The phase angle V tau of a trap potential for a kernel in precision Real:
// reduced to [-pi, pi] in FP64 first, so that its single-precision rounding
// stays ~1e-7 rad however deep the trap
template <typename Real>
__device__ __forceinline__ Real pot_angle(double v, double tau) {
  const double a = v * tau;
  if constexpr (sizeof(Real) == 8) {
    return a;
  } else {
    constexpr double kTwoPi = 6.283185307179586476925;
    return Real(a - kTwoPi * rint(a * (1.0 / kTwoPi)));
  }
}

template <typename Real>
__device__ __forceinline__ void local_update(Cx<Real>* psi, Real tau, Real c0, Real c1) {
  const Real d1 = norm2(psi[0]), d0 = norm2(psi[1]), dm = norm2(psi[2]);
  const Real n = d1 + d0 + dm;
  // Theta = 2 psi_{+1} psi_{-1} - psi_0^2
  const Cx<Real> pp = psi[0] * psi[2];
  const Cx<Real> th = {Real(2) * pp.re - (psi[1].re * psi[1].re - psi[1].im * psi[1].im),
                       Real(2) * (pp.im - psi[1].re * psi[1].im)};
  // |F|^2 = n^2 - |Theta|^2: its rounding (a few ulp of n^2) only enters
  // through x^2 = |F|^2 theta^2, i.e. relative to the step as (n theta)^2
  const Real f2 = fmax(n * n - norm2(th), Real(0));
  const Real theta = c1 * tau;
  // sinc(x/2) and cos(x/2) from u = (x/2)^2
  const Real u = f2 * (Real(0.25) * theta * theta);
  Real sc, ch;
  sinc_cos_from_square(u, &sc, &ch);
  const Real s = theta * (sc * ch);           // sin(x) / |F|
  const Real cm1 = Real(-2) * (u * sc) * sc;  // cos(x) - 1 = -2 sin^2(x/2)
  Real sp, cp;
  angle_sincos(n * (c0 * tau), &sp, &cp);
  // psi_m <- a psi_m + b (-1)^m conj(psi_{-m}),
  // a = exp(-i c0 n tau) (1 + (cos x - 1) - i n s), b = exp(-i c0 n tau) (-i s Theta).
  // The small part (cos x - 1 - i n s) is multiplied by the phase factor and
  // added to it last: rounding cos x itself (1 less a few ulp) to single
  // precision biased the norm by ~1e-9 per step.
  const Real ns = n * s;
  const Cx<Real> a = {cp + (cp * cm1 - sp * ns), -sp - (sp * cm1 + cp * ns)};
  const Cx<Real> b = Cx<Real>{cp, -sp} * Cx<Real>{s * th.im, -s * th.re};
  const Cx<Real> p1 = psi[0], p0 = psi[1], pm = psi[2];
  psi[0] = mul_add_conj<-1>(a, p1, b, pm);
  psi[1] = mul_add_conj<1>(a, p0, b, p0);
  psi[2] = mul_add_conj<-1>(a, pm, b, p1);
}

// ---------------------------------------------------------------------------
// The paper's own local sub-steps over dt, in its order (Lie scheme, Sec. 2.2):
//  (4) diagonal phases exp(-i f_m dt) with f_{+1} = q + (c0 + c1) n - 2 c1 |psi_-1|^2,
//      f_0 = (c0 + c1) n - c1 |psi_0|^2, f_{-1} = q + (c0 + c1) n - 2 c1 |psi_1|^2,
//      densities of the field they act on;
//  (5) off-diagonal mixing exp(-i theta S(a, b)), theta = c1 dt, with
//      S(a, b) = [[0, a, 0], [a*, 0, b], [0, b*, 0]] and the couplings averaged
//      over the field and a predictor: a0 = psi_-1* psi_0, b0 = psi_0* psi_1,
//      tpsi = psi - i theta S(a0, b0) psi, a = (a0 + tpsi_-1* tpsi_0)/2,
//      b = (b0 + tpsi_0* tpsi_1)/2.  With lambda^2 = |a|^2 + |b|^2 and
//      S^3 = lambda^2 S the exponential is 1 - i s S + c S^2, s = sin(x)/lambda,
//      c = (cos x - 1)/lambda^2, x = lambda theta (same coefficients as the
//      exact rotation, from the half-angle sinc).
// ---------------------------------------------------------------------------
// exp(-i V tau) on the three components of a site: the trap potential V is a
// multiple of the identity, so it commutes with the local flow and joins it
// exactly as this extra phase (vtau from pot_angle)
template <typename Real>
__device__ __forceinline__ void potential_phase(Cx<Real>* psi, Real vtau) {
  Real sn, cs;
  angle_sincos(vtau, &sn, &cs);
  const Cx<Real> ph = {cs, -sn};
#pragma unroll
  for (int m = 0; m < 3; ++m) psi[m] = ph * psi[m];
}

template <typename Real>
__device__ __forceinline__ void paper_local_update(Cx<Real>* psi, Real dt, Real c0, Real c1, Real q,
                                                   Real vdt = Real(0)) {
  const Real d1 = norm2(psi[0]), d0 = norm2(psi[1]), dm = norm2(psi[2]);
  const Real n = d1 + d0 + dm;
  const Real base = (c0 + c1) * n;
  const Real f[3] = {q + base - Real(2) * c1 * dm, base - c1 * d0, q + base - Real(2) * c1 * d1};
#pragma unroll
  for (int m = 0; m < 3; ++m) {
    Real sn, cs;
    angle_sincos(f[m] * dt + vdt, &sn, &cs);  // vdt = V dt, the V_m of Eq. (4)
    psi[m] = psi[m] * Cx<Real>{cs, -sn};
  }
  const Real theta = c1 * dt;
  // S(a, b) v
  auto apply_S = [](Cx<Real> a, Cx<Real> b, const Cx<Real>* v, Cx<Real>* out) {
    out[0] = a * v[1];
    out[1] = cmulc(a, v[0]) + b * v[2];
    out[2] = cmulc(b, v[1]);
  };
  const Cx<Real> a0 = cmulc(psi[2], psi[1]), b0 = cmulc(psi[1], psi[0]);
  Cx<Real> sv[3], tp[3];
  apply_S(a0, b0, psi, sv);
#pragma unroll
  for (int m = 0; m < 3; ++m) tp[m] = {psi[m].re + theta * sv[m].im, psi[m].im - theta * sv[m].re};
  const Cx<Real> a = scale(a0 + cmulc(tp[2], tp[1]), Real(0.5));
  const Cx<Real> b = scale(b0 + cmulc(tp[1], tp[0]), Real(0.5));
  Real s, c;
  rotation_coeffs(norm2(a) + norm2(b), theta, &s, &c);
  Cx<Real> s1[3], s2[3];
  apply_S(a, b, psi, s1);
  apply_S(a, b, s1, s2);
#pragma unroll
  for (int m = 0; m < 3; ++m)
    psi[m] = {psi[m].re + s * s1[m].im + c * s2[m].re, psi[m].im - s * s1[m].re + c * s2[m].im};
}

// ---------------------------------------------------------------------------
// Vector-Jacobian product of the local update (reverse mode).  Gradients use
// the real convention G = dL/dRe + i dL/dIm, so dL = Re<G, dpsi> with
// <a, b> = sum conj(a) b.  For psi' = exp(-i c0 n tau) U psi with
// U = 1 - i s M + c M^2, M = F.f, s = s(|F|), c = c(|F|):
//   G_in = U^H Gt + 2 lambda_n psi + 2 (alpha M psi + (B.f) psi),
//   Gt = exp(+i c0 n tau) G',  lambda_n = c0 tau Im<G', psi'>,
//   alpha = sigma1 Im<Gt, M psi> + sigma2 Re<Gt, M^2 psi>,
//   B_a = Re<Gt, f_a u> + c Re<M Gt, f_a psi>,  u = -i s psi + c M psi,
// with sigma1 = s'(r)/r and sigma2 = c'(r)/r (r = |F|); n and F change with
// psi (dn = 2 Re<psi, dpsi>, dF_a = 2 Re<f_a psi, dpsi>).  With x = r theta:
//   sigma1 = theta^3 (x cos x - sin x) / x^3,
//   sigma2 = theta^4 (2 - 2 cos x - x sin x) / x^4,
// evaluated by their Taylor series for small x.
// ---------------------------------------------------------------------------
template <typename Real>
struct SpinOps {
  // Re<a, f_a b> for a = x, y, z
  __device__ static __forceinline__ void expect(const Cx<Real>* a, const Cx<Real>* b, Real* out) {
    const Real h = Real(0.70710678118654752440);
    // f_x b = h (b0, b+1 + b-1, b0); f_y b = h (-i b0, i (b+1 - b-1), i b0); f_z b = (b+1, 0, -b-1)
    const Cx<Real> fx0 = scale(b[1], h), fx1 = scale(b[0] + b[2], h), fx2 = scale(b[1], h);
    const Cx<Real> fy0 = {h * b[1].im, -h * b[1].re};
    const Cx<Real> d = b[0] - b[2];
    const Cx<Real> fy1 = {-h * d.im, h * d.re};
    const Cx<Real> fy2 = {-h * b[1].im, h * b[1].re};
    out[0] = cmulc(a[0], fx0).re + cmulc(a[1], fx1).re + cmulc(a[2], fx2).re;
    out[1] = cmulc(a[0], fy0).re + cmulc(a[1], fy1).re + cmulc(a[2], fy2).re;
    out[2] = cmulc(a[0], b[0]).re - cmulc(a[2], b[2]).re;
  }
  // (B.f) v for a real vector B
  __device__ static __forceinline__ void apply(Real bx, Real by, Real bz, const Cx<Real>* v, Cx<Real>* out) {
    const Real h = Real(0.70710678118654752440);
    // B.f = [[bz, h(bx - i by), 0], [h(bx + i by), 0, h(bx - i by)], [0, h(bx + i by), -bz]]
    const Cx<Real> lo = {h * bx, -h * by}, up = {h * bx, h * by};
    out[0] = scale(v[0], bz) + lo * v[1];
    out[1] = up * v[0] + lo * v[2];
    out[2] = up * v[1] - scale(v[2], bz);
  }
};

template <typename Real>
__device__ __forceinline__ void sigma_coeffs(Real theta, Real x, Real* s1, Real* s2) {
  const Real x2 = x * x;
  const Real t3 = theta * theta * theta, t4 = t3 * theta;
  if (fabs(x) < Real(0.5)) {
    // sum_k (-1)^k 2k x^(2k-2) / (2k+1)!  and  sum_k (-1)^k (2k-2) x^(2k-4) / (2k)!
    Real p = Real(-16.0 / 355687428096000.0);
    p = p * x2 + Real(14.0 / 1307674368000.0);
    p = p * x2 + Real(-12.0 / 6227020800.0);
    p = p * x2 + Real(10.0 / 39916800.0);
    p = p * x2 + Real(-8.0 / 362880.0);
    p = p * x2 + Real(6.0 / 5040.0);
    p = p * x2 + Real(-4.0 / 120.0);
    p = p * x2 + Real(2.0 / 6.0);
    *s1 = -t3 * p;
    Real q = Real(14.0 / 20922789888000.0);
    q = q * x2 + Real(-12.0 / 87178291200.0);
    q = q * x2 + Real(10.0 / 479001600.0);
    q = q * x2 + Real(-8.0 / 3628800.0);
    q = q * x2 + Real(6.0 / 40320.0);
    q = q * x2 + Real(-4.0 / 720.0);
    q = q * x2 + Real(2.0 / 24.0);
    *s2 = t4 * q;
  } else {
    Real sx, cx;
    if constexpr (sizeof(Real) == 4) {
      const SinCos r = sincos_reduced(x);
      sx = r.s;
      cx = r.c;
    } else {
      sincos(x, &sx, &cx);
    }
    const Real x3 = x2 * x;
    *s1 = t3 * (x * cx - sx) / x3;
    *s2 = t4 * (Real(2) - Real(2) * cx - x * sx) / (x3 * x);
  }
}

// Gradient at the input psi of R(tau) from the gradient gout at its output
// (psi' = R(tau) psi is passed in as pout).  Returns G_in in gin.
template <typename Real>
__device__ __forceinline__ void local_update_vjp(const Cx<Real>* psi, const Cx<Real>* pout, const Cx<Real>* gout,
                                                 Cx<Real>* gin, Real tau, Real c0, Real c1) {
  const Real d1 = norm2(psi[0]), d0 = norm2(psi[1]), dm = norm2(psi[2]);
  const Real n = d1 + d0 + dm;
  const Cx<Real> g = cmulc(psi[0], psi[1]) + cmulc(psi[1], psi[2]);
  const Real fz = d1 - dm;
  const Real f2 = Real(2) * norm2(g) + fz * fz;
  const Real theta = c1 * tau;
  const Real x = sqrt(f2) * theta;
  Real s, c, sp, cp;
  rotation_coeffs(f2, theta, &s, &c);
  Real s1, s2;
  sigma_coeffs(theta, x, &s1, &s2);
  angle_sincos(n * (c0 * tau), &sp, &cp);
  // Gt = exp(+i c0 n tau) G'
  Cx<Real> gt[3];
  const Cx<Real> ph = {cp, sp};
#pragma unroll
  for (int m = 0; m < 3; ++m) gt[m] = ph * gout[m];
  // lambda_n = c0 tau Im<G', psi'>
  Real im_gp = Real(0);
#pragma unroll
  for (int m = 0; m < 3; ++m) im_gp += cmulc(gout[m], pout[m]).im;
  const Real lam_n = c0 * tau * im_gp;
  Cx<Real> phi[3], chi[3], mg[3], m2g[3];
  apply_M(psi, phi, g, fz);
  apply_M(phi, chi, g, fz);
  apply_M(gt, mg, g, fz);
  apply_M(mg, m2g, g, fz);
  Real im_phi = Real(0), re_chi = Real(0);
#pragma unroll
  for (int m = 0; m < 3; ++m) {
    im_phi += cmulc(gt[m], phi[m]).im;
    re_chi += cmulc(gt[m], chi[m]).re;
  }
  const Real alpha = s1 * im_phi + s2 * re_chi;
  Cx<Real> u[3];
#pragma unroll
  for (int m = 0; m < 3; ++m) u[m] = Cx<Real>{s * psi[m].im + c * phi[m].re, -s * psi[m].re + c * phi[m].im};
  Real b1[3], b2[3];
  SpinOps<Real>::expect(gt, u, b1);
  SpinOps<Real>::expect(mg, psi, b2);
  Cx<Real> bf[3];
  SpinOps<Real>::apply(b1[0] + c * b2[0], b1[1] + c * b2[1], b1[2] + c * b2[2], psi, bf);
#pragma unroll
  for (int m = 0; m < 3; ++m) {
    // U^H Gt = Gt + i s M Gt + c M^2 Gt
    const Cx<Real> uh = {gt[m].re - s * mg[m].im + c * m2g[m].re, gt[m].im + s * mg[m].re + c * m2g[m].im};
    gin[m] = uh + scale(psi[m], Real(2) * lam_n) + scale(phi[m], Real(2) * alpha) + scale(bf[m], Real(2));
  }
}

// ---------------------------------------------------------------------------
// Philox4x64-10 (Salmon et al., SC'11): two 64x64->128 multiplies per round,
// Weyl key schedule.
// ---------------------------------------------------------------------------
struct U64x4 {
  uint64_t v[4];
};

__device__ __forceinline__ U64x4 philox4x64_10(U64x4 c, uint64_t k0, uint64_t k1) {
  const uint64_t M0 = 0xD2E7470EE14C6C93ull, M1 = 0xCA5A826395121157ull;
  const uint64_t W0 = 0x9E3779B97F4A7C15ull, W1 = 0xBB67AE8584CAA73Bull;
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    if (r > 0) {
      k0 += W0;
      k1 += W1;
    }
    const uint64_t hi0 = __umul64hi(M0, c.v[0]), lo0 = M0 * c.v[0];
    const uint64_t hi1 = __umul64hi(M1, c.v[2]), lo1 = M1 * c.v[2];
    U64x4 n;
    n.v[0] = hi1 ^ c.v[1] ^ k0;
    n.v[1] = lo1;
    n.v[2] = hi0 ^ c.v[3] ^ k1;
    n.v[3] = lo0;
    c = n;
  }
  return c;
}

// (floor(x / 2^12) + 1/2) * 2^-52: exact, in (0, 1)
__device__ __forceinline__ double open_unit(uint64_t x) { return (double(x >> 12) + 0.5) * 0x1p-52; }

}  // namespace spin1
