// Batched complex FFTs in LDS for the sine/cosine transforms and the zero-padded
// convolution of the cavity solver (the Fourier expansions (E123F) sampled on uniform
// nodes, and the FFT evaluation of the singular integrals in Section 5).
//
// Engine: Stockham autosort stages whose radix may be composite (up to 32) or one of the
// odd primes 7, 11, 13.  A composite radix R = R1 R2 is computed in registers by one
// Cooley-Tukey split (R2 DFTs of length R1, constant twiddles, R1 DFTs of length R2), so a
// length-625 transform takes two LDS round trips (25 x 25) instead of four.  C transforms of a block are interleaved in LDS,
// element (pos, col) at buf[pos * C + col] with C a power of two, so consecutive lanes
// work on the same butterfly of consecutive transforms and share its twiddles.
//
// The sine/cosine series sampled on x_i = i len / L, i = 0..L, are transforms of type I:
//   SYN_cos(c)_i = sum_m c_m cos(pi m i / L)        = (F(even ext of c)_i + c_0 + (-1)^i c_L) / 2
//   SYN_sin(c)_i = sum_m c_m sin(pi m i / L)        = (i / 2) F(odd ext of c)_i
//   ANA_cos(u)_m = sum_i tau_i u_i cos(pi m i / L)  = F(even ext of u)_m / 2   (tau = 1/2 at ends)
//   ANA_sin(u)_m = sum_i u_i sin(pi m i / L)        = (i / 2) F(odd ext of u)_m
// with F the forward DFT of length 2L of the even (or odd) extension.
#pragma once

#include <type_traits>

#include <hip/hip_runtime.h>

#include <utility>

#include "device.hpp"

namespace cav {

// ---- compile-time twiddles ---------------------------------------------------------
// cos and sin of 2 pi e / R for small integers, evaluated by the compiler: the angle is
// reduced exactly to |r| <= pi/4 around a multiple q of pi/2 (integer arithmetic), then
// the Taylor series of sin and cos of r are summed to below one ulp.
constexpr double ct_pi = 3.14159265358979323846264338327950288;
constexpr double ct_sin_red(double x) {
  double x2 = x * x, term = x, sum = x;
  for (int i = 1; i < 16; ++i) {
    term *= -x2 / ((2.0 * i) * (2.0 * i + 1.0));
    sum += term;
  }
  return sum;
}
constexpr double ct_cos_red(double x) {
  double x2 = x * x, term = 1.0, sum = 1.0;
  for (int i = 1; i < 16; ++i) {
    term *= -x2 / ((2.0 * i - 1.0) * (2.0 * i));
    sum += term;
  }
  return sum;
}
// angle 2 pi e / R = (pi/4) (8e/R) = q pi/2 + (pi/4)(8e - 2qR)/R
constexpr int ct_quadrant(int e, int R) { return ((8 * (e % R) + R) / (2 * R)); }
constexpr double ct_rem(int e, int R) {
  return ct_pi * (double)(8 * (e % R) - 2 * ct_quadrant(e, R) * R) / (4.0 * R);
}
constexpr double ct_cos(int e, int R) {
  const int q = ct_quadrant(e, R) & 3;
  const double r = ct_rem(e, R);
  return q == 0 ? ct_cos_red(r) : q == 1 ? -ct_sin_red(r) : q == 2 ? -ct_cos_red(r) : ct_sin_red(r);
}
constexpr double ct_sin(int e, int R) {
  const int q = ct_quadrant(e, R) & 3;
  const double r = ct_rem(e, R);
  return q == 0 ? ct_sin_red(r) : q == 1 ? ct_cos_red(r) : q == 2 ? -ct_sin_red(r) : -ct_cos_red(r);
}

// ---- small DFTs in registers ---------------------------------------------------------
// Forward: X_k = sum_j x_j e^{-2 pi i jk/R};  INV: e^{+2 pi i jk/R}.
template <int R, typename T, bool INV>
struct Dft;

template <typename T, bool INV>
struct Dft<1, T, INV> {
  __device__ static inline void run(cx<T>*) {}
};

template <typename T, bool INV>
struct Dft<2, T, INV> {
  __device__ static inline void run(cx<T>* v) {
    const cx<T> a = v[0], b = v[1];
    v[0] = a + b;
    v[1] = a - b;
  }
};

template <typename T, bool INV>
struct Dft<3, T, INV> {
  __device__ static inline void run(cx<T>* v) {
    const T s3 = (T)0.86602540378443864676;  // sin(2 pi / 3)
    const cx<T> t1 = v[1] + v[2];
    const cx<T> t2 = v[0] - (T)0.5 * t1;
    const cx<T> t3 = s3 * (v[1] - v[2]);
    v[0] = v[0] + t1;
    v[1] = INV ? t2 + mul_i(t3) : t2 + mul_mi(t3);
    v[2] = INV ? t2 + mul_mi(t3) : t2 + mul_i(t3);
  }
};

template <typename T, bool INV>
struct Dft<4, T, INV> {
  __device__ static inline void run(cx<T>* v) {
    const cx<T> a = v[0] + v[2], b = v[0] - v[2];
    const cx<T> c = v[1] + v[3], d = v[1] - v[3];
    v[0] = a + c;
    v[2] = a - c;
    v[1] = INV ? b + mul_i(d) : b + mul_mi(d);
    v[3] = INV ? b + mul_mi(d) : b + mul_i(d);
  }
};

template <typename T, bool INV>
struct Dft<5, T, INV> {
  __device__ static inline void run(cx<T>* v) {
    const T c1 = (T)0.30901699437494742410;   // cos(2 pi / 5)
    const T c2 = (T)-0.80901699437494742410;  // cos(4 pi / 5)
    const T s1 = (T)0.95105651629515357212;   // sin(2 pi / 5)
    const T s2 = (T)0.58778525229247312917;   // sin(4 pi / 5)
    const cx<T> a1 = v[1] + v[4], b1 = v[1] - v[4];
    const cx<T> a2 = v[2] + v[3], b2 = v[2] - v[3];
    const cx<T> x0 = v[0];
    const cx<T> p1 = x0 + c1 * a1 + c2 * a2;
    const cx<T> p2 = x0 + c2 * a1 + c1 * a2;
    const cx<T> q1 = s1 * b1 + s2 * b2;
    const cx<T> q2 = s2 * b1 - s1 * b2;
    v[0] = x0 + a1 + a2;
    v[1] = INV ? p1 + mul_i(q1) : p1 + mul_mi(q1);
    v[4] = INV ? p1 + mul_mi(q1) : p1 + mul_i(q1);
    v[2] = INV ? p2 + mul_i(q2) : p2 + mul_mi(q2);
    v[3] = INV ? p2 + mul_mi(q2) : p2 + mul_i(q2);
  }
};

// Odd prime R (7, 11, 13): with a_j = x_j + x_{R-j}, b_j = x_j - x_{R-j} (j = 1..H,
// H = (R-1)/2) the outputs pair up as
//   X_k, X_{R-k} = x_0 + sum_j cos(2 pi jk/R) a_j  -/+ i sum_j sin(2 pi jk/R) b_j
// (signs swapped for the inverse), H^2 real multiplies per output pair instead of R^2.
template <int R>
struct OddTrig {
  static constexpr int H = (R - 1) / 2;
  double c[H][H];
  double s[H][H];
  constexpr OddTrig() : c(), s() {
    for (int k = 1; k <= H; ++k)
      for (int j = 1; j <= H; ++j) {
        c[k - 1][j - 1] = ct_cos((j * k) % R, R);
        s[k - 1][j - 1] = ct_sin((j * k) % R, R);
      }
  }
};

template <int R, typename T, bool INV>
struct DftOddPrime {
  __device__ static inline void run(cx<T>* v) {
    constexpr int H = (R - 1) / 2;
    constexpr OddTrig<R> tb{};
    cx<T> a[H], b[H];
#pragma unroll
    for (int j = 1; j <= H; ++j) {
      a[j - 1] = v[j] + v[R - j];
      b[j - 1] = v[j] - v[R - j];
    }
    const cx<T> x0 = v[0];
    cx<T> sum = x0;
#pragma unroll
    for (int j = 0; j < H; ++j) sum = sum + a[j];
    v[0] = sum;
#pragma unroll
    for (int k = 1; k <= H; ++k) {
      cx<T> p = x0, q = mk<T>(0, 0);
#pragma unroll
      for (int j = 1; j <= H; ++j) {
        p = p + (T)tb.c[k - 1][j - 1] * a[j - 1];
        q = q + (T)tb.s[k - 1][j - 1] * b[j - 1];
      }
      v[k] = INV ? p + mul_i(q) : p + mul_mi(q);
      v[R - k] = INV ? p + mul_mi(q) : p + mul_i(q);
    }
  }
};

template <typename T, bool INV> struct Dft<7, T, INV> : DftOddPrime<7, T, INV> {};
template <typename T, bool INV> struct Dft<11, T, INV> : DftOddPrime<11, T, INV> {};
template <typename T, bool INV> struct Dft<13, T, INV> : DftOddPrime<13, T, INV> {};

// Multiply y[I] (I = r2 R1 + k1) by W_R^{r2 k1}, with the trivial factors 1, -1, +-i
// done by sign and swap.
template <int R1, int R2, typename T, bool INV, int I>
__device__ inline void ct_twiddle_one(cx<T>* y) {
  constexpr int R = R1 * R2;
  constexpr int e = ((I / R1) * (I % R1)) % R;
  if constexpr (e == 0) {
    return;
  } else if constexpr (2 * e == R) {
    y[I] = mk<T>(-y[I].re, -y[I].im);
  } else if constexpr (4 * e == R) {
    y[I] = INV ? mul_i(y[I]) : mul_mi(y[I]);
  } else if constexpr (4 * e == 3 * R) {
    y[I] = INV ? mul_mi(y[I]) : mul_i(y[I]);
  } else {
    constexpr double c = ct_cos(e, R), s = ct_sin(e, R);
    y[I] = y[I] * mk<T>((T)c, INV ? (T)s : (T)-s);
  }
}
template <int R1, int R2, typename T, bool INV, int... I>
__device__ inline void ct_twiddles(cx<T>* y, std::integer_sequence<int, I...>) {
  (ct_twiddle_one<R1, R2, T, INV, I>(y), ...);
}

// DFT of length R1 R2 by one Cooley-Tukey split:
//   X[k1 + R1 k2] = sum_{r2} W_{R2}^{r2 k2} W_R^{r2 k1} sum_{r1} x[R2 r1 + r2] W_{R1}^{r1 k1}.
template <int R1, int R2, typename T, bool INV>
struct DftCt {
  __device__ static inline void run(cx<T>* v) {
    constexpr int R = R1 * R2;
    cx<T> y[R];
#pragma unroll
    for (int r2 = 0; r2 < R2; ++r2) {
      cx<T> t[R1];
#pragma unroll
      for (int r1 = 0; r1 < R1; ++r1) t[r1] = v[R2 * r1 + r2];
      Dft<R1, T, INV>::run(t);
#pragma unroll
      for (int k1 = 0; k1 < R1; ++k1) y[r2 * R1 + k1] = t[k1];
    }
    ct_twiddles<R1, R2, T, INV>(y, std::make_integer_sequence<int, R>{});
#pragma unroll
    for (int k1 = 0; k1 < R1; ++k1) {
      cx<T> t[R2];
#pragma unroll
      for (int r2 = 0; r2 < R2; ++r2) t[r2] = y[r2 * R1 + k1];
      Dft<R2, T, INV>::run(t);
#pragma unroll
      for (int k2 = 0; k2 < R2; ++k2) v[k1 + R1 * k2] = t[k2];
    }
  }
};

template <typename T, bool INV> struct Dft<6, T, INV> : DftCt<2, 3, T, INV> {};
template <typename T, bool INV> struct Dft<8, T, INV> : DftCt<2, 4, T, INV> {};
template <typename T, bool INV> struct Dft<9, T, INV> : DftCt<3, 3, T, INV> {};
template <typename T, bool INV> struct Dft<10, T, INV> : DftCt<2, 5, T, INV> {};
template <typename T, bool INV> struct Dft<12, T, INV> : DftCt<3, 4, T, INV> {};
template <typename T, bool INV> struct Dft<15, T, INV> : DftCt<3, 5, T, INV> {};
template <typename T, bool INV> struct Dft<16, T, INV> : DftCt<4, 4, T, INV> {};
template <typename T, bool INV> struct Dft<20, T, INV> : DftCt<4, 5, T, INV> {};
template <typename T, bool INV> struct Dft<25, T, INV> : DftCt<5, 5, T, INV> {};
template <typename T, bool INV> struct Dft<32, T, INV> : DftCt<4, 8, T, INV> {};

// Radices the planner may choose (host and device agree on this list).
#define CAV_FFT_RADICES(X) \
  X(2) X(3) X(4) X(5) X(6) X(7) X(8) X(9) X(10) X(11) X(12) X(13) X(15) X(16) X(20) X(25) X(32)

// ---- FFT plan -----------------------------------------------------------------------
// Factorisation of n into the radices of its Stockham stages, applied in order, and the
// layout of its stage twiddle table: stage s (s >= 1; span ns = radix[0] ... radix[s-1],
// radix R) keeps the R - 1 twiddles of butterfly k (0 <= k < ns) side by side at
// twoff[s] + k (R - 1), so a work item loads its twiddles from one place; ntw entries in
// all.  Entry r - 1 of butterfly k is W_n^{r k n/(ns R)} = exp(-2 pi i r k / (ns R)).
struct FftPlan {
  int n;
  int nst;
  int radix[20];
  int twoff[20];
  int ntw;
};

// One Stockham stage of radix R over C = 2^lc interleaved transforms of length n with
// span ns: butterfly j (0 <= j < n/R) of transform col reads in[(j + r n/R) C + col],
// scales input r by W_{ns R}^{r (j mod ns)} (tw: this stage's part of the stage twiddle
// table, see FftPlan), and writes out[((j - k) R + k + r ns) C + col].
template <int R, typename T, bool INV>
__device__ inline void fft_stage(const cx<T>* __restrict__ in, cx<T>* __restrict__ out, int n,
                                 int ns, int lc, const cx<T>* __restrict__ tw, int tid, int nthr) {
  const int nb = n / R;
  const int total = nb << lc;
  const int cmask = (1 << lc) - 1;
  // Uniform strides: input r of work item w sits at w + r istride, output r at
  // (d << lc) + col + r ostride, so each access is one add to a per-thread base.
  const int istride = nb << lc, ostride = ns << lc;
  // j / ns from a float reciprocal: (j + 1/2) / ns lies at least 1/(2 ns) from an integer
  // and the float rounding error stays below (j + ns) 2^-23 / ns, so the quotient is exact
  // while j + ns < 2^22 (transforms here have at most a few thousand points).
  const float inv_ns = 1.0f / (float)ns;
  for (int w = tid; w < total; w += nthr) {
    const int j = w >> lc;
    const int col = w & cmask;
    const int q = (int)(((float)j + 0.5f) * inv_ns);
    const int k = j - q * ns;
    const cx<T>* ip = in + w;
    cx<T> v[R];
#pragma unroll
    for (int r = 0; r < R; ++r) v[r] = ip[r * istride];
    if (ns > 1) {
      const cx<T>* tp = tw + k * (R - 1);
#pragma unroll
      for (int r = 1; r < R; ++r) {
        const cx<T> w2 = tp[r - 1];
        v[r] = v[r] * (INV ? conj(w2) : w2);
      }
    }
    Dft<R, T, INV>::run(v);
    cx<T>* op = out + ((((q * R) * ns + k) << lc) + col);
#pragma unroll
    for (int r = 0; r < R; ++r) op[r * ostride] = v[r];
  }
}

// 2^lc interleaved length-n transforms held in LDS buffer `a` (scratch `b` of the same
// size).  Every thread of the block must call this with the same plan and lc (it contains
// __syncthreads).  Returns the buffer that holds the result.  Unnormalised.  Only radices
// up to MAXR are compiled in (they set the register footprint of the calling kernel); the
// plan must not use larger ones.
template <typename T, bool INV, int MAXR = 32>
__device__ cx<T>* fft_lds(cx<T>* a, cx<T>* b, const FftPlan& p, const cx<T>* __restrict__ tw,
                          int tid, int nthr, int lc) {
  int ns = 1;
  cx<T>* in = a;
  cx<T>* out = b;
  for (int s = 0; s < p.nst; ++s) {
    const int rdx = p.radix[s];
    switch (rdx) {
#define CAV_FFT_CASE(R)                                                 \
  case R:                                                               \
    if constexpr (R <= MAXR) fft_stage<R, T, INV>(in, out, p.n, ns, lc, tw + p.twoff[s], tid, nthr); \
    break;
      CAV_FFT_RADICES(CAV_FFT_CASE)
#undef CAV_FFT_CASE
      default: break;
    }
    __syncthreads();
    cx<T>* t = in;
    in = out;
    out = t;
    ns *= rdx;
  }
  return in;
}

// The stage above with its outputs handed to `put(dst, pos, col, v)` (pos: output
// position within transform col) instead of stored at out[(pos << lc) + col]: lets the
// last stage of a transform apply a pointwise product or write global memory directly.
template <int R, typename T, bool INV, class Put>
__device__ inline void fft_stage_put(const cx<T>* __restrict__ in, cx<T>* dst, int n, int ns,
                                     int lc, const cx<T>* __restrict__ tw, int tid, int nthr,
                                     const Put& put) {
  const int nb = n / R;
  const int total = nb << lc;
  const int cmask = (1 << lc) - 1;
  const int istride = nb << lc;
  const float inv_ns = 1.0f / (float)ns;
  for (int w = tid; w < total; w += nthr) {
    const int j = w >> lc;
    const int col = w & cmask;
    const int q = (int)(((float)j + 0.5f) * inv_ns);
    const int k = j - q * ns;
    const cx<T>* ip = in + w;
    cx<T> v[R];
#pragma unroll
    for (int r = 0; r < R; ++r) v[r] = ip[r * istride];
    if (ns > 1) {
      const cx<T>* tp = tw + k * (R - 1);
#pragma unroll
      for (int r = 1; r < R; ++r) {
        const cx<T> w2 = tp[r - 1];
        v[r] = v[r] * (INV ? conj(w2) : w2);
      }
    }
    Dft<R, T, INV>::run(v);
    const int p0 = q * R * ns + k;
#pragma unroll
    for (int r = 0; r < R; ++r) put(dst, p0 + r * ns, col, v[r]);
  }
}

// fft_lds whose last stage hands its outputs to `put` (see fft_stage_put) with dst the
// buffer that stage would have written; ends with a barrier and returns dst.
template <typename T, bool INV, int MAXR, class Put>
__device__ cx<T>* fft_lds_put(cx<T>* a, cx<T>* b, const FftPlan& p, const cx<T>* __restrict__ tw,
                              int tid, int nthr, int lc, const Put& put) {
  int ns = 1;
  cx<T>* in = a;
  cx<T>* out = b;
  for (int s = 0; s < p.nst; ++s) {
    const int rdx = p.radix[s];
    const bool last = s == p.nst - 1;
    switch (rdx) {
#define CAV_FFT_CASE_PUT(R)                                                              \
  case R:                                                                                \
    if constexpr (R <= MAXR) {                                                           \
      if (last) fft_stage_put<R, T, INV>(in, out, p.n, ns, lc, tw + p.twoff[s], tid, nthr, put); \
      else fft_stage<R, T, INV>(in, out, p.n, ns, lc, tw + p.twoff[s], tid, nthr);     \
    }                                                                                    \
    break;
      CAV_FFT_RADICES(CAV_FFT_CASE_PUT)
#undef CAV_FFT_CASE_PUT
      default: break;
    }
    __syncthreads();
    cx<T>* t = in;
    in = out;
    out = t;
    ns *= rdx;
  }
  return in;
}

// ---- transforms with a plan fixed at compile time ----------------------------------
// The same Stockham stages with the length, the radices, the span and the batch 2^LC of a
// block of NT threads known to the compiler: strides become immediate LDS offsets and the
// work-item index arithmetic constant divisions, which takes the integer work of a stage
// off the vector ALU.  Used for the transform shapes the hot kernels run at most (the
// generic forms above cover every plan).
template <int... Rs>
struct CtRadices {};

struct NoPut {};

// One stage (see fft_stage); with LAST and a Put handler its outputs go to put(dst, pos,
// col, v) (see fft_stage_put).
template <int R, int N, int NS, int LC, int NT, typename T, bool INV, bool LAST, class Put>
__device__ inline void fft_stage_ct(const cx<T>* __restrict__ in, cx<T>* out,
                                    const cx<T>* __restrict__ tw, int tid, const Put& put) {
  constexpr int NB = N / R;
  constexpr int TOTAL = NB << LC;
  constexpr int ISTR = NB << LC, OSTR = NS << LC;
  constexpr int CM = (1 << LC) - 1;
#pragma unroll
  for (int w0 = 0; w0 < TOTAL; w0 += NT) {
    const int w = w0 + tid;
    if (TOTAL % NT == 0 || w < TOTAL) {
      const int j = w >> LC;
      const int col = w & CM;
      const int q = j / NS, k = j - q * NS;
      const cx<T>* ip = in + w;
      cx<T> v[R];
#pragma unroll
      for (int r = 0; r < R; ++r) v[r] = ip[r * ISTR];
      if constexpr (NS > 1) {
        const cx<T>* tp = tw + k * (R - 1);
#pragma unroll
        for (int r = 1; r < R; ++r) {
          const cx<T> w2 = tp[r - 1];
          v[r] = v[r] * (INV ? conj(w2) : w2);
        }
      }
      Dft<R, T, INV>::run(v);
      if constexpr (LAST) {
        const int p0 = q * R * NS + k;
#pragma unroll
        for (int r = 0; r < R; ++r) put(out, p0 + r * NS, col, v[r]);
      } else {
        cx<T>* op = out + (((q * R * NS + k) << LC) + col);
#pragma unroll
        for (int r = 0; r < R; ++r) op[r * OSTR] = v[r];
      }
    }
  }
}

template <int N, int NS, int LC, int NT, typename T, bool INV, class Put, int S, int R,
          int... Rest>
__device__ inline cx<T>* fft_ct_stages(cx<T>* in, cx<T>* out, const FftPlan& p,
                                       const cx<T>* __restrict__ tw, int tid, const Put& put) {
  constexpr bool last = sizeof...(Rest) == 0;
  constexpr bool use_put = last && !std::is_same<Put, NoPut>::value;
  fft_stage_ct<R, N, NS, LC, NT, T, INV, use_put, Put>(in, out, tw + p.twoff[S], tid, put);
  __syncthreads();
  if constexpr (last)
    return out;
  else
    return fft_ct_stages<N, NS * R, LC, NT, T, INV, Put, S + 1, Rest...>(out, in, p, tw, tid,
                                                                          put);
}

// fft_lds / fft_lds_put for a plan with the radices Rs (p must be that plan: its stage
// twiddle table is used); put = NoPut{} for a plain transform.  Returns the buffer the
// last stage wrote (or would have written), after a barrier.
template <typename T, bool INV, int LC, int NT, class Put, int... Rs>
__device__ inline cx<T>* fft_ct(cx<T>* a, cx<T>* b, CtRadices<Rs...>, const FftPlan& p,
                                const cx<T>* __restrict__ tw, int tid, const Put& put) {
  constexpr int N = (Rs * ...);
  return fft_ct_stages<N, 1, LC, NT, T, INV, Put, 0, Rs...>(a, b, p, tw, tid, put);
}

// In-place stage with the shape fixed at compile time (see fft_stage_ip): every work item
// (at most one per thread) loads, transforms, waits for the block, then overwrites.
template <int R, int N, int NS, int LC, int NT, typename T, bool INV>
__device__ inline void fft_stage_ct_ip(cx<T>* buf, const cx<T>* __restrict__ tw, int tid) {
  constexpr int NB = N / R;
  constexpr int TOTAL = NB << LC;
  static_assert(TOTAL <= NT, "in-place stages need at most one work item per thread");
  constexpr int ISTR = NB << LC, OSTR = NS << LC;
  constexpr int CM = (1 << LC) - 1;
  const bool act = TOTAL == NT || tid < TOTAL;
  cx<T> v[R];
  cx<T>* op = buf;
  if (act) {
    const int j = tid >> LC;
    const int col = tid & CM;
    const int q = j / NS, k = j - q * NS;
    const cx<T>* ip = buf + tid;
#pragma unroll
    for (int r = 0; r < R; ++r) v[r] = ip[r * ISTR];
    if constexpr (NS > 1) {
      const cx<T>* tp = tw + k * (R - 1);
#pragma unroll
      for (int r = 1; r < R; ++r) {
        const cx<T> w2 = tp[r - 1];
        v[r] = v[r] * (INV ? conj(w2) : w2);
      }
    }
    Dft<R, T, INV>::run(v);
    op = buf + (((q * R * NS + k) << LC) + col);
  }
  __syncthreads();
  if (act) {
#pragma unroll
    for (int r = 0; r < R; ++r) op[r * OSTR] = v[r];
  }
}

template <int N, int NS, int LC, int NT, typename T, bool INV, int S, int R, int... Rest>
__device__ inline void fft_ct_ip_stages(cx<T>* buf, const FftPlan& p,
                                        const cx<T>* __restrict__ tw, int tid) {
  fft_stage_ct_ip<R, N, NS, LC, NT, T, INV>(buf, tw + p.twoff[S], tid);
  __syncthreads();
  if constexpr (sizeof...(Rest) > 0)
    fft_ct_ip_stages<N, NS * R, LC, NT, T, INV, S + 1, Rest...>(buf, p, tw, tid);
}

// fft_lds_ip for a plan with the radices Rs; the result is in buf, after a barrier.
template <typename T, bool INV, int LC, int NT, int... Rs>
__device__ inline void fft_ct_ip(cx<T>* buf, CtRadices<Rs...>, const FftPlan& p,
                                 const cx<T>* __restrict__ tw, int tid) {
  constexpr int N = (Rs * ...);
  fft_ct_ip_stages<N, 1, LC, NT, T, INV, 0, Rs...>(buf, p, tw, tid);
}

// Whether every stage of a length-(Rs product) transform with radices Rs, 2^LC of them
// interleaved, has at most NT work items (the in-place form's condition).
template <int LC, int NT, int... Rs>
constexpr bool ct_ip_fits() {
  constexpr int N = (Rs * ...);
  return ((((N / Rs) << LC) <= NT) && ...);
}

// Whether plan p has exactly the radices Rs.
template <int... Rs>
__host__ __device__ inline bool plan_is(const FftPlan& p) {
  constexpr int rs[] = {Rs...};
  if (p.nst != (int)sizeof...(Rs)) return false;
  for (int s = 0; s < p.nst; ++s)
    if (p.radix[s] != rs[s]) return false;
  return true;
}

// In-place form of a Stockham stage for one LDS buffer: work item w < (n/R) 2^lc (at most
// one per thread) loads its R inputs, applies the twiddles and the butterfly in registers,
// the block synchronises, and the outputs overwrite the buffer.  Half the LDS of the
// ping-pong form for one more barrier per stage.
template <int R, typename T, bool INV>
__device__ inline void fft_stage_ip(cx<T>* buf, int n, int ns, int lc,
                                    const cx<T>* __restrict__ tw, int tid) {
  const int nb = n / R;
  const int total = nb << lc;
  const int istride = nb << lc, ostride = ns << lc;
  const bool act = tid < total;
  cx<T> v[R];
  cx<T>* op = buf;
  if (act) {
    const int j = tid >> lc;
    const int col = tid & ((1 << lc) - 1);
    const int q = (int)(((float)j + 0.5f) * (1.0f / (float)ns));
    const int k = j - q * ns;
    const cx<T>* ip = buf + tid;
#pragma unroll
    for (int r = 0; r < R; ++r) v[r] = ip[r * istride];
    if (ns > 1) {
      const cx<T>* tp = tw + k * (R - 1);
#pragma unroll
      for (int r = 1; r < R; ++r) {
        const cx<T> w2 = tp[r - 1];
        v[r] = v[r] * (INV ? conj(w2) : w2);
      }
    }
    Dft<R, T, INV>::run(v);
    op = buf + ((((q * R) * ns + k) << lc) + col);
  }
  __syncthreads();
  if (act) {
#pragma unroll
    for (int r = 0; r < R; ++r) op[r * ostride] = v[r];
  }
}

// 2^lc interleaved length-n transforms in place in LDS buffer `buf`; needs
// (n / smallest radix) 2^lc <= blockDim.x (see fft_max_items).  Same calling rules as
// fft_lds; the result is in buf.
template <typename T, bool INV, int MAXR = 32>
__device__ void fft_lds_ip(cx<T>* buf, const FftPlan& p, const cx<T>* __restrict__ tw, int tid,
                           int lc) {
  int ns = 1;
  for (int s = 0; s < p.nst; ++s) {
    const int rdx = p.radix[s];
    switch (rdx) {
#define CAV_FFT_CASE_IP(R)                                                         \
  case R:                                                                          \
    if constexpr (R <= MAXR) fft_stage_ip<R, T, INV>(buf, p.n, ns, lc, tw + p.twoff[s], tid); \
    break;
      CAV_FFT_RADICES(CAV_FFT_CASE_IP)
#undef CAV_FFT_CASE_IP
      default: break;
    }
    __syncthreads();
    ns *= rdx;
  }
}

// Work items of the busiest stage of one transform (n over the smallest radix).
inline int fft_max_items(const FftPlan& p) {
  int m = 0;
  for (int s = 0; s < p.nst; ++s) m = p.n / p.radix[s] > m ? p.n / p.radix[s] : m;
  return m;
}

// Even (cos) or odd (sin) extension of entry idx (0 <= idx <= L) of transform col into a
// length-2L buffer of 2^lc interleaved transforms (entries never stored stay zero).
template <typename T>
__device__ inline void store_extension(cx<T>* buf, int L, bool is_cos, int idx, cx<T> x, int lc,
                                       int col) {
  if (is_cos) {
    buf[(idx << lc) + col] = x;
    if (idx > 0 && idx < L) buf[((2 * L - idx) << lc) + col] = x;
  } else {
    if (idx == 0 || idx == L) {
      buf[(idx << lc) + col] = mk<T>(0, 0);
    } else {
      buf[(idx << lc) + col] = x;
      buf[((2 * L - idx) << lc) + col] = mk<T>(-x.re, -x.im);
    }
  }
}

// Even extension of xc plus odd extension of xs (entry idx, 0 <= idx <= L, of transform
// col): one transform of the sum yields the cosine series of one sequence and the sine
// series of another, F_k = E_k + O_k with E even and O odd in k, so
// E_k = (F_k + F_{2L-k}) / 2 and O_k = (F_k - F_{2L-k}) / 2.
template <typename T>
__device__ inline void store_pair_extension(cx<T>* buf, int L, int idx, cx<T> xc, cx<T> xs,
                                            int lc, int col) {
  if (idx == 0 || idx == L) {
    buf[(idx << lc) + col] = xc;
  } else {
    buf[(idx << lc) + col] = xc + xs;
    buf[((2 * L - idx) << lc) + col] = xc - xs;
  }
}

}  // namespace cav

namespace cav {

// Host planner: the factorisation of n into the fewest stages with radices from
// CAV_FFT_RADICES not above max_radix, ties broken towards balanced radices (smallest sum
// of squares); stages ordered by decreasing radix so the largest runs without twiddles.
// Returns nst = 0 when n has a prime factor other than 2, 3, 5, 7, 11, 13 or does not fit.
inline FftPlan plan_fft(int n, int max_radix) {
  FftPlan p{};
  p.n = n;
  p.nst = 0;
  static const int rad[] = {
#define CAV_FFT_LIST(R) R,
      CAV_FFT_RADICES(CAV_FFT_LIST)
#undef CAV_FFT_LIST
  };
  const int nr = (int)(sizeof(rad) / sizeof(rad[0]));
  if (n < 1) return p;
  if (n == 1) return p;
  // dynamic programme over the divisors of n (n is at most a few thousand)
  struct Best { int stages; long long sq; int first; };
  Best* best = new Best[n + 1];
  for (int m = 0; m <= n; ++m) best[m] = {1 << 29, 0, 0};
  best[1] = {0, 0, 0};
  for (int m = 2; m <= n; ++m) {
    if (n % m) continue;
    for (int i = 0; i < nr; ++i) {
      const int r = rad[i];
      if (r > max_radix || m % r) continue;
      const Best& s = best[m / r];
      if (s.stages >= (1 << 29)) continue;
      const Best cand{s.stages + 1, s.sq + (long long)r * r, r};
      if (cand.stages < best[m].stages ||
          (cand.stages == best[m].stages && cand.sq < best[m].sq))
        best[m] = cand;
    }
  }
  if (best[n].stages < (1 << 29) && best[n].stages <= 20) {
    int m = n;
    while (m > 1) {
      p.radix[p.nst++] = best[m].first;
      m /= best[m].first;
    }
    for (int i = 0; i < p.nst; ++i)
      for (int j = i + 1; j < p.nst; ++j)
        if (p.radix[j] > p.radix[i]) {
          const int t = p.radix[i];
          p.radix[i] = p.radix[j];
          p.radix[j] = t;
        }
  }
  delete[] best;
  int ns = 1, off = 0;
  for (int s = 0; s < p.nst; ++s) {
    p.twoff[s] = off;
    if (s > 0) off += ns * (p.radix[s] - 1);
    ns *= p.radix[s];
  }
  p.ntw = off;
  return p;
}

// Stage twiddle table of plan p (layout in FftPlan) from the plain table
// table[t] = exp(-2 pi i t / n): entry r - 1 of butterfly k of stage s is table[r k n/(ns R)].
template <typename C>
inline void fill_stage_twiddles(const FftPlan& p, const C* table, C* out) {
  int ns = p.nst > 0 ? p.radix[0] : 1;
  for (int s = 1; s < p.nst; ++s) {
    const int R = p.radix[s];
    const int tstep = p.n / (ns * R);
    for (int k = 0; k < ns; ++k)
      for (int r = 1; r < R; ++r) out[p.twoff[s] + k * (R - 1) + (r - 1)] = table[r * k * tstep];
    ns *= R;
  }
}

}  // namespace cav
