// Device-side building blocks shared by the cavity kernels: complex arithmetic,
// a mixed-radix (2, 3, 4, 5) Stockham FFT that runs in LDS, and the sine/cosine
// transforms of type I built on it.
//
// The sine/cosine series of the paper's Fourier expansions (E123F), sampled on the
// uniform nodes x_i = i L_len / L, i = 0..L, are transforms of type I:
//   SYN_cos(c)_i = sum_m c_m cos(pi m i / L)        = (F(even ext of c)_i + c_0 + (-1)^i c_L) / 2
//   SYN_sin(c)_i = sum_m c_m sin(pi m i / L)        = (i / 2) F(odd ext of c)_i
//   ANA_cos(u)_m = sum_i tau_i u_i cos(pi m i / L)  = F(even ext of u)_m / 2   (tau = 1/2 at ends)
//   ANA_sin(u)_m = sum_i u_i sin(pi m i / L)        = (i / 2) F(odd ext of u)_m
// with F the forward DFT of length 2L of the even (or odd) extension.
#pragma once

#include <hip/hip_runtime.h>

// Dynamic LDS of a kernel, sized at launch.
#ifndef CAV_DYN_SMEM
#define CAV_DYN_SMEM(name) extern __shared__ __align__(16) unsigned char name[]
#endif

namespace cav {

template <typename R>
struct cx {
  R re, im;
};

template <typename R>
__host__ __device__ inline cx<R> mk(R a, R b) { return cx<R>{a, b}; }
template <typename R>
__host__ __device__ inline cx<R> operator+(cx<R> a, cx<R> b) { return {a.re + b.re, a.im + b.im}; }
template <typename R>
__host__ __device__ inline cx<R> operator-(cx<R> a, cx<R> b) { return {a.re - b.re, a.im - b.im}; }
template <typename R>
__host__ __device__ inline cx<R> operator*(cx<R> a, cx<R> b) {
  return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
template <typename R>
__host__ __device__ inline cx<R> operator*(R s, cx<R> a) { return {s * a.re, s * a.im}; }
template <typename R>
__host__ __device__ inline cx<R> conj(cx<R> a) { return {a.re, -a.im}; }
template <typename R>
__host__ __device__ inline cx<R> mul_i(cx<R> a) { return {-a.im, a.re}; }      // i * a
template <typename R>
__host__ __device__ inline cx<R> mul_mi(cx<R> a) { return {a.im, -a.re}; }     // -i * a
template <typename R>
__host__ __device__ inline cx<R> cdiv(cx<R> a, cx<R> b) {
  // Smith's algorithm
  if (fabs(b.re) >= fabs(b.im)) {
    R r = b.im / b.re, d = b.re + b.im * r;
    return {(a.re + a.im * r) / d, (a.im - a.re * r) / d};
  } else {
    R r = b.re / b.im, d = b.im + b.re * r;
    return {(a.re * r + a.im) / d, (a.im * r - a.re) / d};
  }
}
template <typename R>
__host__ __device__ inline R cabs2(cx<R> a) { return a.re * a.re + a.im * a.im; }

typedef cx<double> zd;

// ---------------------------------------------------------------------------------
// FFT plan: factorisation of n into radices, most 4s first.
// ---------------------------------------------------------------------------------
struct FftPlan {
  int n;
  int nst;
  int radix[20];
};

// Twiddle table layout: tw[t] = exp(-2 pi i t / n), t = 0..n-1 (double precision).

template <typename R, bool INV>
__device__ inline void dft2(cx<R>* v) {
  cx<R> a = v[0], b = v[1];
  v[0] = a + b;
  v[1] = a - b;
}

template <typename R, bool INV>
__device__ inline void dft3(cx<R>* v) {
  const R s3 = (R)0.86602540378443864676;  // sin(2 pi / 3)
  cx<R> t1 = v[1] + v[2];
  cx<R> t2 = v[0] - (R)0.5 * t1;
  cx<R> t3 = s3 * (v[1] - v[2]);
  v[0] = v[0] + t1;
  if (!INV) {
    v[1] = t2 + mul_mi(t3);
    v[2] = t2 + mul_i(t3);
  } else {
    v[1] = t2 + mul_i(t3);
    v[2] = t2 + mul_mi(t3);
  }
}

template <typename R, bool INV>
__device__ inline void dft4(cx<R>* v) {
  cx<R> a = v[0] + v[2], b = v[0] - v[2];
  cx<R> c = v[1] + v[3], d = v[1] - v[3];
  v[0] = a + c;
  v[2] = a - c;
  if (!INV) {
    v[1] = b + mul_mi(d);
    v[3] = b + mul_i(d);
  } else {
    v[1] = b + mul_i(d);
    v[3] = b + mul_mi(d);
  }
}

template <typename R, bool INV>
__device__ inline void dft5(cx<R>* v) {
  const R c1 = (R)0.30901699437494742410;   // cos(2 pi / 5)
  const R c2 = (R)-0.80901699437494742410;  // cos(4 pi / 5)
  const R s1 = (R)0.95105651629515357212;   // sin(2 pi / 5)
  const R s2 = (R)0.58778525229247312917;   // sin(4 pi / 5)
  cx<R> a1 = v[1] + v[4], b1 = v[1] - v[4];
  cx<R> a2 = v[2] + v[3], b2 = v[2] - v[3];
  cx<R> x0 = v[0];
  cx<R> p1 = x0 + c1 * a1 + c2 * a2;
  cx<R> p2 = x0 + c2 * a1 + c1 * a2;
  cx<R> q1 = s1 * b1 + s2 * b2;
  cx<R> q2 = s2 * b1 - s1 * b2;
  v[0] = x0 + a1 + a2;
  if (!INV) {
    v[1] = p1 + mul_mi(q1);
    v[4] = p1 + mul_i(q1);
    v[2] = p2 + mul_mi(q2);
    v[3] = p2 + mul_i(q2);
  } else {
    v[1] = p1 + mul_i(q1);
    v[4] = p1 + mul_mi(q1);
    v[2] = p2 + mul_i(q2);
    v[3] = p2 + mul_mi(q2);
  }
}

template <int RDX, typename R, bool INV>
__device__ inline void dft_r(cx<R>* v) {
  if constexpr (RDX == 2) dft2<R, INV>(v);
  else if constexpr (RDX == 3) dft3<R, INV>(v);
  else if constexpr (RDX == 4) dft4<R, INV>(v);
  else dft5<R, INV>(v);
}

// One Stockham stage of radix RDX over C interleaved transforms: element (pos, col) of
// the batch sits at buf[pos * C + col].  Work item w = j * C + col, so consecutive
// threads handle the same butterfly of consecutive transforms: LDS accesses are
// contiguous and each twiddle is shared by C lanes.
template <int RDX, typename R, bool INV>
__device__ inline void fft_stage(const cx<R>* __restrict__ in, cx<R>* __restrict__ out, int n,
                                 int ns, int C, const zd* __restrict__ tw, int tid, int nthr) {
  const int nb = n / RDX;
  const int tstep = n / (ns * RDX);
  const int total = nb * C;
  for (int w = tid; w < total; w += nthr) {
    const int j = w / C;
    const int col = w - j * C;
    const int k = j % ns;
    cx<R> v[RDX];
#pragma unroll
    for (int r = 0; r < RDX; ++r) v[r] = in[(j + r * nb) * C + col];
    if (k > 0) {
#pragma unroll
      for (int r = 1; r < RDX; ++r) {
        zd w2 = tw[r * k * tstep];
        v[r] = v[r] * mk<R>((R)w2.re, INV ? -(R)w2.im : (R)w2.im);
      }
    }
    dft_r<RDX, R, INV>(v);
    const int d = (j / ns) * ns * RDX + k;
#pragma unroll
    for (int r = 0; r < RDX; ++r) out[(d + r * ns) * C + col] = v[r];
  }
}

// C interleaved length-n transforms held in LDS buffer `a` (scratch `b` of the same size).
// Threads tid = 0..nthr-1 cooperate; every thread of the block must call this with the
// same plan and C (it contains __syncthreads).  Returns the buffer that holds the result.
// Forward: X_k = sum_j x_j e^{-2 pi i jk/n};  INV: e^{+2 pi i jk/n}, unnormalised.
template <typename R, bool INV>
__device__ cx<R>* fft_lds(cx<R>* a, cx<R>* b, const FftPlan& p, const zd* __restrict__ tw,
                          int tid, int nthr, int C = 1) {
  int ns = 1;
  cx<R>* in = a;
  cx<R>* out = b;
  for (int s = 0; s < p.nst; ++s) {
    const int rdx = p.radix[s];
    switch (rdx) {
      case 2: fft_stage<2, R, INV>(in, out, p.n, ns, C, tw, tid, nthr); break;
      case 3: fft_stage<3, R, INV>(in, out, p.n, ns, C, tw, tid, nthr); break;
      case 4: fft_stage<4, R, INV>(in, out, p.n, ns, C, tw, tid, nthr); break;
      default: fft_stage<5, R, INV>(in, out, p.n, ns, C, tw, tid, nthr); break;
    }
    __syncthreads();
    cx<R>* t = in;
    in = out;
    out = t;
    ns *= rdx;
  }
  return in;
}

// Even (cos) or odd (sin) extension of entry idx (0 <= idx <= L) of transform col into a
// length-2L batch buffer with C interleaved transforms (entries never stored stay zero).
template <typename R>
__device__ inline void store_extension(cx<R>* buf, int L, bool is_cos, int idx, cx<R> x,
                                       int C = 1, int col = 0) {
  if (is_cos) {
    buf[idx * C + col] = x;
    if (idx > 0 && idx < L) buf[(2 * L - idx) * C + col] = x;
  } else {
    if (idx == 0 || idx == L) {
      buf[idx * C + col] = mk<R>(0, 0);
    } else {
      buf[idx * C + col] = x;
      buf[(2 * L - idx) * C + col] = mk<R>(-x.re, -x.im);
    }
  }
}

}  // namespace cav
