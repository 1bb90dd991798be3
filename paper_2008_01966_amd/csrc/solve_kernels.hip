// Solve-time kernels: right-hand side (Section 3 (nosig), Appendix A), the matrix-free
// reduced aperture operator with its three single-layer families applied by FFT
// convolution (Sections 3, 5), Krylov building blocks, back-substitution and field
// synthesis (EInter), and the aperture transforms behind the RCS (Section 7).
//
// Mode grids are (M+1) x (N+1), m-major (mn = m (N+1) + n).  A padded aperture vector is
// three such grids [E1 | E2 | E3]; entries outside N1, N2, N3 stay zero.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdlib>

#include "kernels.hpp"

namespace cav {

// Elements per thread per trip of the global-to-LDS load loops: the trip's loads are all
// issued before its LDS stores, so their latencies overlap.
constexpr int kLoadBatch = 4;

// Lengths of the transforms the compile-time kernel variants are built for (the host
// dispatches them only for plans of exactly these radices): extension 8 x 8 x 8 = 2 L with
// L = 256, box 5 x 5 x 5 x 5 = P.
constexpr int kCtHalfExt = 256;
constexpr int kCtBox = 625;

// 2^lc interleaved transforms of plan p in LDS, in place in a (ip) or ping-pong between a
// and b; returns the buffer holding the result.  CTLC > 0: the plan has the radices Rs and
// lc == CTLC, both fixed at compile time (fft_ct, fft_ct_ip); ip then needs ct_ip_fits.
template <typename T, bool INV, int MR, int CTLC, int... Rs>
__device__ inline cx<T>* lds_fft(cx<T>* a, cx<T>* b, CtRadices<Rs...> rs, const FftPlan& p,
                                 const cx<T>* __restrict__ tw, int tid, int nt, int lc, int ip) {
  if constexpr (CTLC > 0) {
    if constexpr (ct_ip_fits<CTLC, 256, Rs...>()) {
      if (ip) {
        fft_ct_ip<T, INV, CTLC, 256>(a, rs, p, tw, tid);
        return a;
      }
    }
    return fft_ct<T, INV, CTLC, 256>(a, b, rs, p, tw, tid, NoPut{});
  } else {
    if (ip) {
      fft_lds_ip<T, INV, MR>(a, p, tw, tid, lc);
      return a;
    }
    return fft_lds<T, INV, MR>(a, b, p, tw, tid, nt, lc);
  }
}

// Sum over the 64 lanes of a wave.
__device__ inline double wave_sum(double v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

__device__ inline zd exp_int(double w, double len) {
  const double th = 0.5 * w * len;
  double s, c;
  sincos(th, &s, &c);
  double sinc;
  if (fabs(th) < 1e-4) {
    const double t2 = th * th;
    sinc = 1.0 - t2 * (1.0 / 6.0) + t2 * t2 * (1.0 / 120.0);
  } else {
    sinc = s / th;
  }
  return mk(len * c * sinc, len * s * sinc);
}
// int_0^len cos(f x) e^{i alpha x} dx and int_0^len sin(f x) e^{i alpha x} dx
__device__ inline zd cos_proj(double alpha, double f, double len) {
  return 0.5 * (exp_int(alpha + f, len) + exp_int(alpha - f, len));
}
__device__ inline zd sin_proj(double alpha, double f, double len) {
  const zd d = exp_int(alpha + f, len) - exp_int(alpha - f, len);
  return mk(0.5 * d.im, -0.5 * d.re);  // d / (2i)
}

// ---------------------------------------------------------------------------------
// Right-hand side: g1 = (h/q) 2i (alpha1 p3 + beta p1) C_m(alpha1) S_n(alpha2) on N1,
//                  g2 = (h/c) 2i (alpha2 p3 + beta p2) S_m(alpha1) C_n(alpha2) on N2.
// One right-hand side per blockIdx.y; vectors of length 3 NM, consecutive.
// ---------------------------------------------------------------------------------
__global__ void k_rhs(Geo g, const Wave* __restrict__ waves, zd* __restrict__ b) {
  const int mn = blockIdx.x * blockDim.x + threadIdx.x;
  if (mn >= g.NM) return;
  const Wave wv = waves[blockIdx.y];
  zd* out = b + (long long)blockIdx.y * 3 * g.NM;
  const int m = mn / (g.N + 1), n = mn % (g.N + 1);
  const double mu = M_PI * m / g.a, nu = M_PI * n / g.b;
  zd g1 = mk(0.0, 0.0), g2 = mk(0.0, 0.0);
  if (n >= 1) {
    const double q = (m == 0 ? 0.5 : 0.25) * g.a * g.b;
    const double amp = 2.0 * (wv.alpha1 * wv.p3 + wv.beta * wv.p1) * wv.h / q;
    const zd pr = cos_proj(wv.alpha1, mu, g.a) * sin_proj(wv.alpha2, nu, g.b);
    g1 = mk(-amp * pr.im, amp * pr.re);  // i * amp * pr
  }
  if (m >= 1) {
    const double c = (n == 0 ? 0.5 : 0.25) * g.a * g.b;
    const double amp = 2.0 * (wv.alpha2 * wv.p3 + wv.beta * wv.p2) * wv.h / c;
    const zd pr = sin_proj(wv.alpha1, mu, g.a) * cos_proj(wv.alpha2, nu, g.b);
    g2 = mk(-amp * pr.im, amp * pr.re);
  }
  out[mn] = g1;
  out[g.NM + mn] = g2;
  out[2LL * g.NM + mn] = mk(0.0, 0.0);
}

hipError_t launch_rhs(const Geo& g, const Wave* waves, int nb, zd* b, hipStream_t st) {
  const int blk = 256;
  hipLaunchKernelGGL(k_rhs, dim3((g.NM + blk - 1) / blk, nb), dim3(blk), 0, st, g, waves, b);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------------
// TBC single-layer families f: 0 = cos-sin (acts on E1), 1 = sin-cos (E2), 2 = cos-cos
// (sigma = nu E1 - mu E2, the cos-cos coefficients of div_Gamma(z x E)).
//   (S^f c)_mn = hq1 hq2 ANA1 ANA2 [ IFFT( FFT( w1 w2 SYN1 SYN2 c ) K^s ) ]
// on the (s Nx + 1) x (s Ny + 1) trapezoid grid, zero-padded to P1 x P2.
// Three passes: rows forward (SYN along y, FFT along y), columns (SYN, FFT, multiply,
// inverse FFT, ANA along x), rows backward (inverse FFT along y, ANA along y).
// blockIdx.z selects the right-hand side; a block whose right-hand side is inactive
// returns at once.
// ---------------------------------------------------------------------------------
__device__ inline bool fam_xcos(int f) { return f != 1; }
__device__ inline bool fam_ycos(int f) { return f != 0; }

// Each FFT kernel holds C = 2^lc transforms of a block interleaved in LDS, element
// (pos, c) at buf[(pos << lc) + c]; global loads and stores map consecutive lanes to
// consecutive addresses, and blocks are renumbered so neighbouring strips share an XCD.
// The last block of a grid may hold fewer live transforms (Cb); its other LDS columns
// hold zeros and are never stored.  T is the precision of the workspaces X, Y, of the
// transforms and of the TBC results S (double, or float for the mixed-precision inner
// solve); the input vector is stored in double or single precision (VI) and read into
// double.

// Pass 1: rows m0 .. m0+Cb-1 of one family.  fam_fixed >= 0: `v` is the coefficient grid
// of that family (inspection path); otherwise `v` is a padded aperture vector, optionally
// preconditioned first (in double precision whatever its storage precision VI).
template <typename T, int MR, int CTLC = 0, typename VI = double>
__global__ __launch_bounds__(256) void k_tbc_rows_fwd(Geo g, Fft ext2, Fft box2,
                                                      const zd* __restrict__ pinv_all,
                                                      long long pcs, int precond,
                                                      int fam_fixed, int lc_arg, int ip,
                                                      const cx<VI>* __restrict__ vall, long long vs,
                                                      cx<T>* __restrict__ Xall,
                                                      const int* __restrict__ active) {
  CAV_DYN_SMEM(smem_raw);
  __shared__ cx<T> c0s[64];
  // strip-major order: the 3 family blocks of a row strip read the same aperture entries
  // and preconditioner blocks, next to each other on one XCD
  const BlockId bid = xcd_block_x_slow();
  const int rhs = bid.z;
  if (active && !active[rhs]) return;
  const cx<VI>* v = vall + rhs * vs;
  const zd* pinv = pinv_all + rhs * pcs;
  const int nf = fam_fixed >= 0 ? 1 : 3;
  cx<T>* X = Xall + (long long)rhs * nf * (g.M + 1) * g.ldx;
  const int lc = CTLC > 0 ? CTLC : lc_arg;
  const int C = 1 << lc;
  const int m0 = bid.x << lc;
  const int Cb = min(C, g.M + 1 - m0);
  const int f = fam_fixed >= 0 ? fam_fixed : bid.y;
  const int slot = fam_fixed >= 0 ? 0 : bid.y;
  const int L = CTLC > 0 ? kCtHalfExt : g.nq2, P = CTLC > 0 ? kCtBox : g.P2;
  const DivBy div_p(P);
  // ping-pong: two buffers of P; in place: the extension transform's 2L, then the box's P
  cx<T>* a = reinterpret_cast<cx<T>*>(smem_raw);
  cx<T>* b = a + ((long long)(ip ? 2 * L : P) << lc);
  const bool ycos = fam_ycos(f);
  const int tid = threadIdx.x, nt = blockDim.x;
  for (int i = tid; i < (2 * L) << lc; i += nt) a[i] = mk<T>(0, 0);
  __syncthreads();
  const int rowlen = g.N + 1;
  const DivBy div_row(rowlen);
  for (int w = tid; w < rowlen * Cb; w += nt) {
    const int c = div_row.quot(w), n = w - c * div_row.d;
    const int m = m0 + c;
    const long long mn = (long long)m * rowlen + n;
    zd val;
    if (fam_fixed >= 0) {
      val = widen(v[mn]);
    } else if (precond) {
      zd z[3] = {widen(v[mn]), widen(v[g.NM + mn]), widen(v[2LL * g.NM + mn])};
      zd y[3];
      for (int r = 0; r < 3; ++r)
        y[r] = pinv[(3 * r) * (long long)g.NM + mn] * z[0] +
               pinv[(3 * r + 1) * (long long)g.NM + mn] * z[1] +
               pinv[(3 * r + 2) * (long long)g.NM + mn] * z[2];
      const double mu = g.pa * m, nu = g.pb * n;
      val = f == 0 ? y[0] : (f == 1 ? y[1] : (nu * y[0] - mu * y[1]));
    } else {   // only the components the family uses (f is uniform over the block)
      const double mu = g.pa * m, nu = g.pb * n;
      val = f == 0 ? widen(v[mn])
                   : (f == 1 ? widen(v[g.NM + mn])
                             : (nu * widen(v[mn]) - mu * widen(v[g.NM + mn])));
    }
    const cx<T> tv = cvt<T>(val);
    store_extension(a, L, ycos, n, tv, lc, c);
    if (n == 0) c0s[c] = tv;
  }
  __syncthreads();
  cx<T>* r = lds_fft<T, false, MR, CTLC>(a, b, CtRadices<8, 8, 8>{}, ext2.p, twiddles<T>(ext2),
                                         tid, nt, lc, ip);
  cx<T>* o = (r == a) ? b : a;
  const T hq = (T)g.hq2;
  for (int w = tid; w < P << lc; w += nt) {
    const int i = w >> lc, c = w & (C - 1);
    cx<T> val = mk<T>(0, 0);
    if (i <= L && c < Cb) {
      const cx<T> F = r[w];
      const cx<T> sy = ycos ? (T)0.5 * (F + c0s[c]) : (T)0.5 * mul_i(F);
      val = ((i == 0 || i == L) ? (T)0.5 * hq : hq) * sy;
    }
    o[w] = val;
  }
  __syncthreads();
  cx<T>* r2 = lds_fft<T, false, MR, CTLC>(o, r, CtRadices<5, 5, 5, 5>{}, box2.p,
                                          twiddles<T>(box2), tid, nt, lc, ip);
  cx<T>* dst = X + ((long long)slot * (g.M + 1) + m0) * g.ldx;
  for (int w = tid; w < P * Cb; w += nt) {
    const int c = div_p.quot(w), k = w - c * div_p.d;
    dst[(long long)c * g.ldx + k] = r2[(k << lc) + c];
  }
}

// Pass 2: columns k0 .. k0+Cb-1 of one family.
// Last-stage output handlers of the column pass (see fft_lds_put).
// dst[(k1 << lc) + c] = v * K-hat[k1][k0 + c] for the block's Cb live columns.
template <typename T>
struct SpectrumProduct {
  const cx<T>* khat;   // K-hat + k0
  int P2, Cb, lc;
  __device__ void operator()(cx<T>* dst, int k1, int c, cx<T> v) const {
    dst[(k1 << lc) + c] = c < Cb ? v * khat[(long long)k1 * P2 + c] : v;
  }
};

// Synthesis along x on the trapezoid grid, trapezoid weights and zero padding, in one:
// dst[(i << lc) + c] = w_i hq (cosine: (F + c0) / 2, sine: i F / 2) for i <= L, 0 for
// L < i < 2L (positions 2L..P-1 are zero from the start).
template <typename T>
struct WeightPad {
  const cx<T>* c0s;
  int L, lc;
  bool xcos;
  T hq;
  __device__ void operator()(cx<T>* dst, int i, int c, cx<T> F) const {
    cx<T> val = mk<T>(0, 0);
    if (i <= L) {
      const cx<T> sx = xcos ? (T)0.5 * (F + c0s[c]) : (T)0.5 * mul_i(F);
      val = ((i == 0 || i == L) ? (T)0.5 * hq : hq) * sx;
    }
    dst[(i << lc) + c] = val;
  }
};

// Crop to the trapezoid grid and extend for the projection's transform: entry i <= L of
// the inverse box transform goes to position i and (mirrored, negated for sine) 2L - i.
template <typename T>
struct ExtendCrop {
  int L, lc;
  bool xcos;
  __device__ void operator()(cx<T>* dst, int i, int c, cx<T> v) const {
    if (i <= L) store_extension(dst, L, xcos, i, v, lc, c);
  }
};

// Y[m][k0 + c] = hq * (cosine: F / 2, sine: i F / 2) for m <= M and the live columns.
template <typename T>
struct ColumnStore {
  cx<T>* Y;            // Y + k0
  int ld, rows, Cb;   // ld: row stride of Y
  bool xcos;
  T hq;
  __device__ void operator()(cx<T>*, int m, int c, cx<T> F) const {
    if (m >= rows || c >= Cb) return;
    const cx<T> s = xcos ? (T)0.5 * F : (T)0.5 * mul_i(F);
    Y[(long long)m * ld + c] = hq * s;
  }
};

// CTLC > 0: the transform shapes fixed at compile time (extension 8 x 8 x 8 = 512, box
// 5 x 5 x 5 x 5 = 625, 2^CTLC columns per block; fft_ct) for the plans that have them.
template <typename T, int MR, int CTLC = 0>
__global__ __launch_bounds__(256) void k_tbc_cols(Geo g, Fft ext1, Fft box1,
                                                  const cx<T>* __restrict__ khat, int fam_fixed,
                                                  int lc_arg, const cx<T>* __restrict__ Xall,
                                                  cx<T>* __restrict__ Yall,
                                                  const int* __restrict__ active) {
  CAV_DYN_SMEM(smem_raw);
  __shared__ cx<T> c0s[64];
  const int lc = CTLC > 0 ? CTLC : lc_arg;
  // the strips of one 128-byte line of X and Y run together (their blocks share the line),
  // and the nb x 3 blocks of a strip, which share its K-hat columns, stay close
  const BlockId bid = xcd_block_x_grouped(max(1, 128 / ((int)sizeof(cx<T>) << lc)));
  const int rhs = bid.z;
  if (active && !active[rhs]) return;
  const int nf = fam_fixed >= 0 ? 1 : 3;
  const long long wsz = (long long)nf * (g.M + 1) * g.ldx;
  const int f = fam_fixed >= 0 ? fam_fixed : bid.y;
  const int slot = fam_fixed >= 0 ? 0 : bid.y;
  const cx<T>* X = Xall + rhs * wsz + (long long)slot * (g.M + 1) * g.ldx;
  cx<T>* Y = Yall + rhs * wsz + (long long)slot * (g.M + 1) * g.ldx;
  const int C = 1 << lc;
  const int k0 = bid.x << lc;
  const int Cb = min(C, g.P2 - k0);
  const int L = CTLC > 0 ? kCtHalfExt : g.nq1, P = CTLC > 0 ? kCtBox : g.P1;
  // two ping-pong buffers of P (> 2L) entries per column
  cx<T>* a = reinterpret_cast<cx<T>*>(smem_raw);
  cx<T>* b = a + ((long long)P << lc);
  const bool xcos = fam_xcos(f);
  const int tid = threadIdx.x, nt = blockDim.x;
  // zero the first transform's input (entries the extension does not set) and, in both
  // buffers, the padding 2L..P-1 of the box transform, which no later step writes
  for (int i = tid; i < (2 * L) << lc; i += nt) a[i] = mk<T>(0, 0);
  for (int i = tid; i < (P - 2 * L) << lc; i += nt) {
    a[((2 * L) << lc) + i] = mk<T>(0, 0);
    b[((2 * L) << lc) + i] = mk<T>(0, 0);
  }
  for (int c = tid; c < C; c += nt) c0s[c] = mk<T>(0, 0);
  __syncthreads();
  // kLoadBatch elements per thread per trip with every load issued before the stores
  for (int w0 = tid; w0 < (g.M + 1) << lc; w0 += kLoadBatch * nt) {
    cx<T> xv[kLoadBatch];
#pragma unroll
    for (int u = 0; u < kLoadBatch; ++u) {   // indices clamped in range: no conditional loads
      const int w = w0 + u * nt, m = min(w >> lc, g.M), c = min(w & (C - 1), Cb - 1);
      xv[u] = X[(long long)m * g.ldx + k0 + c];
    }
#pragma unroll
    for (int u = 0; u < kLoadBatch; ++u) {
      const int w = w0 + u * nt, m = w >> lc, c = w & (C - 1);
      if (m > g.M || c >= Cb) continue;
      store_extension(a, L, xcos, m, xv[u], lc, c);
      if (m == 0) c0s[c] = xv[u];
    }
  }
  __syncthreads();
  const cx<T>* tw_e = twiddles<T>(ext1);
  const cx<T>* tw_b = twiddles<T>(box1);
  const T hq = (T)g.hq1;
  cx<T>* o;
  cx<T>* r;
  if constexpr (CTLC > 0) {
    o = fft_ct<T, false, CTLC, 256>(a, b, CtRadices<8, 8, 8>{}, ext1.p, tw_e, tid,
                                    WeightPad<T>{c0s, L, lc, xcos, hq});
    r = (o == a) ? b : a;
  } else if constexpr (MR <= kSmallRadix) {
    // synthesis along x; its last stage applies the trapezoid weights and pads to P
    o = fft_lds_put<T, false, MR>(a, b, ext1.p, tw_e, tid, nt, lc,
                                  WeightPad<T>{c0s, L, lc, xcos, hq});
    r = (o == a) ? b : a;
  } else {
    // with the larger radices the extra last-stage forms cost registers (spills): the
    // weights and padding take a pass of their own
    r = fft_lds<T, false, MR>(a, b, ext1.p, tw_e, tid, nt, lc);
    o = (r == a) ? b : a;
    for (int w = tid; w < P << lc; w += nt) {
      const int i = w >> lc, c = w & (C - 1);
      cx<T> val = mk<T>(0, 0);
      if (i <= L) {
        const cx<T> F = r[w];
        const cx<T> sx = xcos ? (T)0.5 * (F + c0s[c]) : (T)0.5 * mul_i(F);
        val = ((i == 0 || i == L) ? (T)0.5 * hq : hq) * sx;
      }
      o[w] = val;
    }
    __syncthreads();
  }
  // the product with K-hat rides on the transform's last stage
  cx<T>* r2;
  if constexpr (CTLC > 0)
    r2 = fft_ct<T, false, CTLC, 256>(o, r, CtRadices<5, 5, 5, 5>{}, box1.p, tw_b, tid,
                                     SpectrumProduct<T>{khat + k0, g.P2, Cb, lc});
  else
    r2 = fft_lds_put<T, false, MR>(o, r, box1.p, tw_b, tid, nt, lc,
                                   SpectrumProduct<T>{khat + k0, g.P2, Cb, lc});
  cx<T>* o3;
  cx<T>* r3;
  if constexpr (CTLC > 0) {
    o3 = fft_ct<T, true, CTLC, 256>(r2, (r2 == a) ? b : a, CtRadices<5, 5, 5, 5>{}, box1.p, tw_b,
                                    tid, ExtendCrop<T>{L, lc, xcos});
    r3 = (o3 == a) ? b : a;
  } else if constexpr (MR <= kSmallRadix) {
    // inverse transform; its last stage crops to the grid and writes the extension
    o3 = fft_lds_put<T, true, MR>(r2, (r2 == a) ? b : a, box1.p, tw_b, tid, nt, lc,
                                  ExtendCrop<T>{L, lc, xcos});
    r3 = (o3 == a) ? b : a;
  } else {
    r3 = fft_lds<T, true, MR>(r2, (r2 == a) ? b : a, box1.p, tw_b, tid, nt, lc);
    o3 = (r3 == a) ? b : a;
    for (int w = tid; w < (L + 1) << lc; w += nt) {
      const int i = w >> lc, c = w & (C - 1);
      store_extension(o3, L, xcos, i, r3[w], lc, c);
    }
    __syncthreads();
  }
  // the last stage writes the projected entries m = 0..M straight to Y
  if constexpr (CTLC > 0)
    fft_ct<T, false, CTLC, 256>(o3, r3, CtRadices<8, 8, 8>{}, ext1.p, tw_e, tid,
                                ColumnStore<T>{Y + k0, g.ldx, g.M + 1, Cb, xcos, hq});
  else
    fft_lds_put<T, false, MR>(o3, r3, ext1.p, tw_e, tid, nt, lc,
                              ColumnStore<T>{Y + k0, g.ldx, g.M + 1, Cb, xcos, hq});
}

// Pass 3: rows m0 .. m0+Cb-1 backward; writes S[slot][mn] in precision T.
template <typename T, int MR, int CTLC = 0>
__global__ __launch_bounds__(256) void k_tbc_rows_bwd(Geo g, Fft ext2, Fft box2, int fam_fixed,
                                                      int lc_arg, int ip,
                                                      const cx<T>* __restrict__ Yall,
                                                      cx<T>* __restrict__ Sall,
                                                      const int* __restrict__ active) {
  CAV_DYN_SMEM(smem_raw);
  const BlockId bid = xcd_block();
  const int rhs = bid.z;
  if (active && !active[rhs]) return;
  const int nf = fam_fixed >= 0 ? 1 : 3;
  const int f = fam_fixed >= 0 ? fam_fixed : bid.y;
  const int slot = fam_fixed >= 0 ? 0 : bid.y;
  const cx<T>* Y =
      Yall + (long long)rhs * nf * (g.M + 1) * g.ldx + (long long)slot * (g.M + 1) * g.ldx;
  cx<T>* S = Sall + (long long)rhs * nf * g.NM + (long long)slot * g.NM;
  const int lc = CTLC > 0 ? CTLC : lc_arg;
  const int C = 1 << lc;
  const int m0 = bid.x << lc;
  const int Cb = min(C, g.M + 1 - m0);
  const int L = CTLC > 0 ? kCtHalfExt : g.nq2, P = CTLC > 0 ? kCtBox : g.P2;
  const DivBy div_p(P);
  cx<T>* a = reinterpret_cast<cx<T>*>(smem_raw);
  cx<T>* b = a + ((long long)P << lc);
  const bool ycos = fam_ycos(f);
  const int tid = threadIdx.x, nt = blockDim.x;
  for (int w0 = tid; w0 < P << lc; w0 += kLoadBatch * nt) {
    cx<T> yv[kLoadBatch];
#pragma unroll
    for (int u = 0; u < kLoadBatch; ++u) {   // indices clamped in range: no conditional loads
      const int w = min(w0 + u * nt, (P << lc) - 1), c = div_p.quot(w), k = w - c * div_p.d;
      yv[u] = Y[(long long)(m0 + min(c, Cb - 1)) * g.ldx + k];
    }
#pragma unroll
    for (int u = 0; u < kLoadBatch; ++u) {
      const int w = w0 + u * nt, c = div_p.quot(w), k = w - c * div_p.d;
      if (w < P << lc) a[(k << lc) + c] = c < Cb ? yv[u] : mk<T>(0, 0);
    }
  }
  __syncthreads();
  // in place: a holds the box transform (P), b the extension transform (2L)
  cx<T>* r = lds_fft<T, true, MR, CTLC>(a, b, CtRadices<5, 5, 5, 5>{}, box2.p, twiddles<T>(box2),
                                        tid, nt, lc, ip);
  cx<T>* o = (r == a) ? b : a;
  for (int w = tid; w < (L + 1) << lc; w += nt) {
    const int i = w >> lc, c = w & (C - 1);
    store_extension(o, L, ycos, i, r[w], lc, c);
  }
  __syncthreads();
  cx<T>* r2 = lds_fft<T, false, MR, CTLC>(o, r, CtRadices<8, 8, 8>{}, ext2.p,
                                          twiddles<T>(ext2), tid, nt, lc, ip);
  const int rowlen = g.N + 1;
  const DivBy div_row(rowlen);
  for (int w = tid; w < rowlen * Cb; w += nt) {
    const int c = div_row.quot(w), n = w - c * div_row.d;
    const cx<T> F = r2[(n << lc) + c];
    const zd s = widen(ycos ? (T)0.5 * F : (T)0.5 * mul_i(F));
    S[(long long)(m0 + c) * rowlen + n] = cvt<T>(g.hq2 * s);
  }
}

// Pass 4: the local (mode-diagonal) terms of the three aperture rows plus the TBC terms.
//  r1 = (rho_d - 1) z1 + mu (T + h) z3 + (h/q) (2k^2 S^cs z1 - 2 nu S^cc sigma)   on N1
//  r2 = (rho_d - 1) z2 + nu (T + h) z3 + (h/c) (2k^2 S^sc z2 + 2 mu S^cc sigma)   on N2
//  r3 = (rho_n - 1) z3 + mu h z1 + nu h z2                                        on N3
// Operator result of mode mn of right-hand side rhs (the three components r1, r2, r3 of y)
// from its input v (P^{-1} applied first when precond) and the TBC results S: rows 1-3 of
// the reduced system with the per-mode column data.
template <typename VI, typename ST>
__device__ inline void epilogue_mode(const Geo& g, const Cols& cl, int precond, const cx<VI>* v,
                                     const cx<ST>* S, int rhs, int mn, zd* out) {
  const long long co = rhs * cl.cs;
  const zd* __restrict__ rho_d = cl.rho_d + co;
  const zd* __restrict__ T = cl.T + co;
  const zd* __restrict__ rho_n = cl.rho_n + co;
  const zd* __restrict__ pinv = cl.pinv + co;
  const int m = mn / (g.N + 1), n = mn % (g.N + 1);
  const double h = cl.hs ? cl.hs[rhs] : g.h;
  const double mu = g.pa * m, nu = g.pb * n, k2 = g.k * g.k;
  zd z[3] = {widen(v[mn]), widen(v[g.NM + mn]), widen(v[2LL * g.NM + mn])};
  if (precond) {
    zd t[3];
    for (int r = 0; r < 3; ++r)
      t[r] = pinv[(3 * r) * (long long)g.NM + mn] * z[0] +
             pinv[(3 * r + 1) * (long long)g.NM + mn] * z[1] +
             pinv[(3 * r + 2) * (long long)g.NM + mn] * z[2];
    z[0] = t[0]; z[1] = t[1]; z[2] = t[2];
  }
  const zd scs = widen(S[mn]), ssc = widen(S[g.NM + mn]), scc = widen(S[2LL * g.NM + mn]);
  const zd rd = rho_d[mn] - mk(1.0, 0.0), rn = rho_n[mn] - mk(1.0, 0.0);
  const zd th = T[mn] + mk(h, 0.0);
  const double hq = h * ((m == 0 ? 2.0 : 4.0) * g.iab);
  const double hc = h * ((n == 0 ? 2.0 : 4.0) * g.iab);
  zd r1 = mk(0.0, 0.0), r2 = mk(0.0, 0.0), r3 = mk(0.0, 0.0);
  if (n >= 1) r1 = rd * z[0] + mu * (th * z[2]) + hq * ((2.0 * k2) * scs - (2.0 * nu) * scc);
  if (m >= 1) r2 = rd * z[1] + nu * (th * z[2]) + hc * ((2.0 * k2) * ssc + (2.0 * mu) * scc);
  if (m >= 1 && n >= 1) r3 = rn * z[2] + (mu * h) * z[0] + (nu * h) * z[1];
  out[0] = r1;
  out[1] = r2;
  out[2] = r3;
}

template <typename VI, typename ST>
__global__ void k_operator_epilogue(Geo g, Cols cl, int precond, const cx<VI>* __restrict__ vall,
                                    long long vs, const cx<ST>* __restrict__ Sall,
                                    zd* __restrict__ yall, long long ys,
                                    const int* __restrict__ active) {
  const int rhs = blockIdx.y;
  if (active && !active[rhs]) return;
  const int mn = blockIdx.x * blockDim.x + threadIdx.x;
  if (mn >= g.NM) return;
  zd r[3];
  epilogue_mode(g, cl, precond, vall + rhs * vs, Sall + 3LL * rhs * g.NM, rhs, mn, r);
  zd* y = yall + rhs * ys;
  y[mn] = r[0];
  y[g.NM + mn] = r[1];
  y[2LL * g.NM + mn] = r[2];
}

// The epilogue fused with the first Gram-Schmidt pass of an Arnoldi step: y = A v as
// above, and from the same registers the per-block partial sums of conj(V_t) y over the
// nv <= G basis vectors (V_t of right-hand side rhs at V + t ldj + rhs 3 NM) in k_dots'
// layout, partial[(rhs nvmax + t) gridDim.x + block].  Blocks stride over the modes; each
// thread sums its modes in order, the three components of a mode in order.  S and the
// basis are in the operator's precision VT, v is stored in VI and y in WT; the sums run
// in double from y before it is rounded to WT.
template <typename VT, int G, typename VI, typename WT>
__global__ __launch_bounds__(256) void k_epilogue_dots(Geo g, Cols cl, int precond,
                                                       const cx<VI>* __restrict__ vall,
                                                       long long vs,
                                                       const cx<VT>* __restrict__ Sall,
                                                       cx<WT>* __restrict__ yall, long long ys,
                                                       const cx<VT>* __restrict__ V,
                                                       long long ldj, int nv, int nvmax,
                                                       zd* __restrict__ partial,
                                                       const int* __restrict__ active) {
  __shared__ zd red[G][4];
  const int rhs = blockIdx.y;
  if (active && !active[rhs]) return;
  const cx<VI>* v = vall + rhs * vs;
  const cx<VT>* S = Sall + 3LL * rhs * g.NM;
  cx<WT>* y = yall + rhs * ys;
  const cx<VT>* Vr = V + rhs * 3LL * g.NM;
  zd acc[G];
  for (int t = 0; t < G; ++t) acc[t] = mk(0.0, 0.0);
  for (int mn = blockIdx.x * blockDim.x + threadIdx.x; mn < g.NM;
       mn += gridDim.x * blockDim.x) {
    zd r[3];
    epilogue_mode(g, cl, precond, v, S, rhs, mn, r);
    y[mn] = cvt<WT>(r[0]);
    y[g.NM + mn] = cvt<WT>(r[1]);
    y[2LL * g.NM + mn] = cvt<WT>(r[2]);
#pragma unroll
    for (int t = 0; t < G; ++t)
      if (t < nv) {
        const cx<VT>* Vt = Vr + t * ldj;
        const cx<VT> a0 = Vt[mn], a1 = Vt[g.NM + mn], a2 = Vt[2LL * g.NM + mn];
        acc[t] = acc[t] + conj(widen(a0)) * r[0];
        acc[t] = acc[t] + conj(widen(a1)) * r[1];
        acc[t] = acc[t] + conj(widen(a2)) * r[2];
      }
  }
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
  for (int t = 0; t < G; ++t) {
    const zd sum = mk(wave_sum(acc[t].re), wave_sum(acc[t].im));
    if (lane == 0) red[t][wv] = sum;
  }
  __syncthreads();
  if (threadIdx.x < nv) {
    const int t = threadIdx.x;
    partial[((long long)rhs * nvmax + t) * gridDim.x + blockIdx.x] =
        red[t][0] + red[t][1] + red[t][2] + red[t][3];
  }
}

// log2 of the transforms per block for an FFT kernel whose two LDS buffers hold len
// elements of elem bytes each: the largest power of two within the LDS budget (at least
// one transform, at most the next power of two above `cap`, at most 64).  budget 0: the
// default (40000 bytes, or CAVITY_LDS_BUDGET).
static int batch_log2(int len, int elem, int cap, int budget_bytes = 0) {
  static long long deflt = -1;
  if (deflt < 0) {
    const char* e = getenv("CAVITY_LDS_BUDGET");
    deflt = e ? atoll(e) : 40000;
  }
  const long long budget = budget_bytes > 0 ? budget_bytes : deflt;
  int lc = 0;
  while (lc < 6 && (1 << lc) < cap && 2LL * len * elem * (2LL << lc) <= budget) ++lc;
  return lc;
}

// Batch of one TBC pass: 2^lc transforms per block of the extension transform (length
// 2L) and the box transform (length P), in place (buffers of 2L and P, every thread one
// work item per stage) when allowed and the busiest stage has at most one item per
// thread, else in the ping-pong form (two buffers of P).  Measured at 256x256 modes: the
// row passes gain 14-19 % in place; the column pass, whose four transforms per column
// then run two columns per block instead of four, loses 20 %, so it stays ping-pong.  For
// the row passes the plan's autotuner picks the form (one transform per block in place
// can lose to two in the ping-pong form on larger boxes).
struct TbcShape {
  int lc, ip;
  size_t smem;
};
static TbcShape tbc_shape(const FftPlan& ext, const FftPlan& box, int L, int P, int elem,
                          int cap, int budget, bool allow_ip) {
  const int items = std::max(fft_max_items(ext), fft_max_items(box));
  if (allow_ip && items <= 256) {
    int lc = batch_log2((2 * L + P + 1) / 2, elem, cap, budget);
    while (lc > 0 && (items << lc) > 256) --lc;
    return {lc, 1, (size_t)(2 * L + P) * elem << lc};
  }
  const int lc = batch_log2(P, elem, cap, budget);
  return {lc, 0, (size_t)2 * P * elem << lc};
}

template <typename T, typename VI = double>
static hipError_t tbc_passes(const Geo& g, const Trig& t, const cx<T>* khat, const zd* pinv,
                             long long pcs, int precond, int fam_fixed, int nb, const cx<VI>* v,
                             long long vs,
                             cx<T>* X, cx<T>* Y, cx<T>* S, const int* active, hipStream_t st) {
  const int nf = fam_fixed >= 0 ? 1 : 3;
  const double zb = sizeof(zd), tb = sizeof(cx<T>);
  const double xbytes = tb * nb * nf * (g.M + 1) * (double)g.P2;   // one X or Y workspace
  const double vin = nb * (sizeof(cx<VI>) * (fam_fixed >= 0 ? 1.0 : 3.0) * g.NM) +
                     (precond ? zb * 9.0 * g.NM : 0.0);
  const bool single = sizeof(T) == sizeof(float);
  const int id_fwd = single ? K_TBC_ROWS_FWD_F32 : K_TBC_ROWS_FWD;
  const int id_cols = single ? K_TBC_COLS_F32 : K_TBC_COLS;
  const int id_bwd = single ? K_TBC_ROWS_BWD_F32 : K_TBC_ROWS_BWD;
  const TbcShape sr =
      tbc_shape(t.ext2.p, t.box2.p, g.nq2, g.P2, (int)tb, g.M + 1, g.lds_budget, g.rows_ip);
  const int gr = (g.M + 1 + (1 << sr.lc) - 1) >> sr.lc;
  // transforms fixed at compile time for the extension 8 x 8 x 8 and box 5 x 5 x 5 x 5 plans
  // of the radix-8 build (CAVITY_FFT_MAXR=16 keeps the generic kernels); the in-place form,
  // which tbc_shape allows only when every stage fits the block, exists for 2^1 transforms
  // per block
  const bool ct_rows = t.maxr <= kSmallRadix && plan_is<8, 8, 8>(t.ext2.p) &&
                       plan_is<5, 5, 5, 5>(t.box2.p);
  probe_begin(id_fwd, st);
  if (ct_rows && sr.lc == 2 && !sr.ip)
    hipLaunchKernelGGL((k_tbc_rows_fwd<T, 8, 2, VI>), dim3(gr, nf, nb), dim3(256), sr.smem, st, g,
                       t.ext2, t.box2, pinv, pcs, precond, fam_fixed, sr.lc, sr.ip, v, vs, X,
                       active);
  else if (ct_rows && sr.lc == 1)
    hipLaunchKernelGGL((k_tbc_rows_fwd<T, 8, 1, VI>), dim3(gr, nf, nb), dim3(256), sr.smem, st, g,
                       t.ext2, t.box2, pinv, pcs, precond, fam_fixed, sr.lc, sr.ip, v, vs, X,
                       active);
  else if (t.maxr <= 8)
    hipLaunchKernelGGL((k_tbc_rows_fwd<T, 8, 0, VI>), dim3(gr, nf, nb), dim3(256), sr.smem, st, g, t.ext2,
                       t.box2, pinv, pcs, precond, fam_fixed, sr.lc, sr.ip, v, vs, X, active);
  else
    hipLaunchKernelGGL((k_tbc_rows_fwd<T, kMaxRadix, 0, VI>), dim3(gr, nf, nb), dim3(256), sr.smem, st, g,
                       t.ext2, t.box2, pinv, pcs, precond, fam_fixed, sr.lc, sr.ip, v, vs, X,
                       active);
  probe_end(id_fwd, st, vin + xbytes);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  // the column pass has only the two-buffer form (its last stages carry the K-hat product
  // and the store to Y)
  const TbcShape sc =
      tbc_shape(t.ext1.p, t.box1.p, g.nq1, g.P1, (int)tb, g.P2, g.lds_budget, false);
  probe_begin(id_cols, st);
  const dim3 gc((g.P2 + (1 << sc.lc) - 1) >> sc.lc, nf, nb);
  const bool ct = t.maxr <= kSmallRadix && plan_is<8, 8, 8>(t.ext1.p) &&
                  plan_is<5, 5, 5, 5>(t.box1.p);
  if (ct && sc.lc == 2)
    hipLaunchKernelGGL((k_tbc_cols<T, 8, 2>), gc, dim3(256), sc.smem, st, g, t.ext1, t.box1, khat,
                       fam_fixed, sc.lc, X, Y, active);
  else if (ct && sc.lc == 1)
    hipLaunchKernelGGL((k_tbc_cols<T, 8, 1>), gc, dim3(256), sc.smem, st, g, t.ext1, t.box1, khat,
                       fam_fixed, sc.lc, X, Y, active);
  else if (t.maxr <= 8)
    hipLaunchKernelGGL((k_tbc_cols<T, 8>), gc, dim3(256), sc.smem, st, g, t.ext1, t.box1, khat,
                       fam_fixed, sc.lc, X, Y, active);
  else
    hipLaunchKernelGGL((k_tbc_cols<T, kMaxRadix>), gc, dim3(256), sc.smem, st, g, t.ext1, t.box1,
                       khat, fam_fixed, sc.lc, X, Y, active);
  probe_end(id_cols, st, 2.0 * xbytes + tb * (double)g.P1 * g.P2);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  probe_begin(id_bwd, st);
  if (ct_rows && sr.lc == 2 && !sr.ip)
    hipLaunchKernelGGL((k_tbc_rows_bwd<T, 8, 2>), dim3(gr, nf, nb), dim3(256), sr.smem, st, g,
                       t.ext2, t.box2, fam_fixed, sr.lc, sr.ip, Y, S, active);
  else if (ct_rows && sr.lc == 1)
    hipLaunchKernelGGL((k_tbc_rows_bwd<T, 8, 1>), dim3(gr, nf, nb), dim3(256), sr.smem, st, g,
                       t.ext2, t.box2, fam_fixed, sr.lc, sr.ip, Y, S, active);
  else if (t.maxr <= 8)
    hipLaunchKernelGGL((k_tbc_rows_bwd<T, 8>), dim3(gr, nf, nb), dim3(256), sr.smem, st, g, t.ext2,
                       t.box2, fam_fixed, sr.lc, sr.ip, Y, S, active);
  else
    hipLaunchKernelGGL((k_tbc_rows_bwd<T, kMaxRadix>), dim3(gr, nf, nb), dim3(256), sr.smem, st, g,
                       t.ext2, t.box2, fam_fixed, sr.lc, sr.ip, Y, S, active);
  probe_end(id_bwd, st, xbytes + tb * nb * nf * g.NM);
  return hipGetLastError();
}

static hipError_t launch_tbc_passes(const Geo& g, const Trig& t, const zd* khat, const zd* pinv,
                                    int precond, int fam_fixed, int nb, const zd* v, long long vs,
                                    zd* X, zd* Y, zd* S, const int* active, hipStream_t st) {
  return tbc_passes<double>(g, t, khat, pinv, 0, precond, fam_fixed, nb, v, vs, X, Y, S, active,
                            st);
}

// S (3 NM entries per right-hand side in the workspace of that many double entries) holds
// the TBC results in the operator's precision T.
template <typename T, typename VI>
static hipError_t operator_impl(const Geo& g, const Trig& t, const cx<T>* khat, const Cols& c,
                                int precond, int nb, const cx<VI>* v, long long vs, cx<T>* X,
                                cx<T>* Y, zd* S, zd* y, long long ys, const int* active,
                                hipStream_t st) {
  cx<T>* St = reinterpret_cast<cx<T>*>(S);
  hipError_t e = tbc_passes<T, VI>(g, t, khat, c.pinv, c.cs, precond, -1, nb, v, vs, X, Y, St,
                                   active, st);
  if (e != hipSuccess) return e;
  const int blk = 256;
  probe_begin(K_EPILOGUE, st);
  hipLaunchKernelGGL((k_operator_epilogue<VI, T>), dim3((g.NM + blk - 1) / blk, nb), dim3(blk), 0,
                     st, g, c, precond, v, vs, St, y, ys, active);
  probe_end(K_EPILOGUE, st, (sizeof(zd) + sizeof(cx<VI>) + sizeof(cx<T>)) * 3.0 * g.NM * nb +
                                sizeof(zd) * (double)g.NM * (3.0 + (precond ? 9.0 : 0.0)));
  return hipGetLastError();
}

// The operator with the spectral single-layer operators (D_spec) in place of the
// trapezoid ones; same epilogue.
hipError_t launch_operator_spec(const Geo& g, const SpecMats& sm, const zd* khat, const Cols& c,
                                int precond, int nb, const zd* v, long long vs, zd* X, zd* Y,
                                zd* U, zd* S, zd* y, long long ys, const int* active,
                                hipStream_t st) {
  // one cavity per call (the column data of a group have cs > 0 only on the FFT operator)
  hipError_t e = launch_spec_passes(g, sm, khat, c.pinv, precond, -1, nb, v, vs, X, Y, U, S,
                                    active, st);
  if (e != hipSuccess) return e;
  const int blk = 256;
  hipLaunchKernelGGL((k_operator_epilogue<double, double>), dim3((g.NM + blk - 1) / blk, nb),
                     dim3(blk), 0, st, g, c, precond, v, vs, S, y, ys, active);
  return hipGetLastError();
}

hipError_t launch_operator(const Geo& g, const Trig& t, const zd* khat, const Cols& c,
                           int precond, int nb, const zd* v, long long vs, zd* X, zd* Y, zd* S,
                           zd* y, long long ys, const int* active, hipStream_t st) {
  return operator_impl<double, double>(g, t, khat, c, precond, nb, v, vs, X, Y, S, y, ys, active,
                                       st);
}

hipError_t launch_operator_f32(const Geo& g, const Trig& t, const zf* khat_f, const Cols& c,
                               int precond, int nb, const zd* v, long long vs, zf* Xf, zf* Yf,
                               zd* S, zd* y, long long ys, const int* active, hipStream_t st) {
  return operator_impl<float, double>(g, t, khat_f, c, precond, nb, v, vs, Xf, Yf, S, y, ys,
                                      active, st);
}

hipError_t launch_operator_f32(const Geo& g, const Trig& t, const zf* khat_f, const Cols& c,
                               int precond, int nb, const zf* v, long long vs, zf* Xf, zf* Yf,
                               zd* S, zd* y, long long ys, const int* active, hipStream_t st) {
  return operator_impl<float, float>(g, t, khat_f, c, precond, nb, v, vs, Xf, Yf, S, y, ys,
                                     active, st);
}

__global__ void k_reduce_cols(const zd* __restrict__ partial, int nblk, int nvmax,
                              zd* __restrict__ out, long long ostride, zd* __restrict__ acc,
                              long long astride, const int* __restrict__ active);

// The operator on input v (P^{-1} applied to it first when precond) followed by the
// epilogue fused with the first Gram-Schmidt dot products against the nv <= 16 basis
// vectors V (k_epilogue_dots), the nblk per-block partial sums reduced into
// out[r * ostride + t].  v is stored in double or in single precision (VI); S, in the
// workspace of 3 NM double entries per right-hand side, holds the TBC results in
// precision T.
template <typename T, typename VI, typename WT>
static hipError_t operator_dots_impl(const Geo& g, const Trig& t, const cx<T>* khat,
                                     const Cols& c, int precond, int nb, const cx<VI>* v,
                                     long long vs, cx<T>* X, cx<T>* Y, zd* S, cx<WT>* y,
                                     long long ys,
                                     const cx<T>* V, long long ldj, int nv, int nvmax,
                                     zd* partial, int nblk, zd* out, long long ostride,
                                     const int* active, hipStream_t st) {
  if (nv < 1 || nv > 16) return hipErrorInvalidValue;
  cx<T>* St = reinterpret_cast<cx<T>*>(S);
  hipError_t e =
      tbc_passes<T, VI>(g, t, khat, c.pinv, c.cs, precond, -1, nb, v, vs, X, Y, St, active, st);
  if (e != hipSuccess) return e;
  probe_begin(K_EPILOGUE, st);
  if (nv <= 8)
    hipLaunchKernelGGL((k_epilogue_dots<T, 8, VI, WT>), dim3(nblk, nb), dim3(256), 0, st, g, c,
                       precond, v, vs, St, y, ys, V, ldj, nv, nvmax, partial, active);
  else
    hipLaunchKernelGGL((k_epilogue_dots<T, 16, VI, WT>), dim3(nblk, nb), dim3(256), 0, st, g, c,
                       precond, v, vs, St, y, ys, V, ldj, nv, nvmax, partial, active);
  probe_end(K_EPILOGUE, st,
            (sizeof(cx<VI>) + sizeof(cx<T>) + sizeof(cx<WT>)) * 3.0 * g.NM * nb +
                sizeof(zd) * (double)g.NM * (3.0 + (precond ? 9.0 : 0.0)) +
                sizeof(cx<T>) * 3.0 * g.NM * nb * nv);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_reduce_cols, dim3(nv, nb), dim3(256), 0, st, partial, nblk, nvmax, out,
                     ostride, nullptr, 0, active);
  return hipGetLastError();
}

hipError_t launch_operator_dots(const Geo& g, const Trig& t, const zd* khat, const Cols& c,
                                int precond, int nb, const zd* v, long long vs, zd* X, zd* Y,
                                zd* S, zd* y, long long ys, const zd* V, long long ldj, int nv,
                                int nvmax, zd* partial, int nblk, zd* out, long long ostride,
                                const int* active, hipStream_t st) {
  return operator_dots_impl<double, double, double>(g, t, khat, c, precond, nb, v, vs, X, Y, S, y, ys, V,
                                            ldj, nv, nvmax, partial, nblk, out, ostride, active,
                                            st);
}

hipError_t launch_operator_dots_f32(const Geo& g, const Trig& t, const zf* khat_f, const Cols& c,
                                    int precond, int nb, const zd* v, long long vs, zf* Xf,
                                    zf* Yf, zd* S, zd* y, long long ys, const zf* V,
                                    long long ldj, int nv, int nvmax, zd* partial, int nblk,
                                    zd* out, long long ostride, const int* active,
                                    hipStream_t st) {
  return operator_dots_impl<float, double, double>(g, t, khat_f, c, precond, nb, v, vs, Xf, Yf, S, y, ys,
                                           V, ldj, nv, nvmax, partial, nblk, out, ostride, active,
                                           st);
}

hipError_t launch_operator_dots_f32(const Geo& g, const Trig& t, const zf* khat_f, const Cols& c,
                                    int precond, int nb, const zf* v, long long vs, zf* Xf,
                                    zf* Yf, zd* S, zd* y, long long ys, const zf* V,
                                    long long ldj, int nv, int nvmax, zd* partial, int nblk,
                                    zd* out, long long ostride, const int* active,
                                    hipStream_t st) {
  return operator_dots_impl<float, float, double>(g, t, khat_f, c, precond, nb, v, vs, Xf, Yf, S,
                                                  y, ys, V, ldj, nv, nvmax, partial, nblk, out,
                                                  ostride, active, st);
}

hipError_t launch_operator_dots_f32(const Geo& g, const Trig& t, const zf* khat_f, const Cols& c,
                                    int precond, int nb, const zf* v, long long vs, zf* Xf,
                                    zf* Yf, zd* S, zf* y, long long ys, const zf* V,
                                    long long ldj, int nv, int nvmax, zd* partial, int nblk,
                                    zd* out, long long ostride, const int* active,
                                    hipStream_t st) {
  return operator_dots_impl<float, float, float>(g, t, khat_f, c, precond, nb, v, vs, Xf, Yf, S, y,
                                                 ys, V, ldj, nv, nvmax, partial, nblk, out,
                                                 ostride, active, st);
}

__global__ void k_to_f32(const zd* __restrict__ in, zf* __restrict__ out, long long n) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x)
    out[i] = cvt<float>(in[i]);
}

hipError_t launch_to_f32(const zd* in, zf* out, long long n, hipStream_t st) {
  const long long blocks = std::min<long long>((n + 255) / 256, 4096);
  hipLaunchKernelGGL(k_to_f32, dim3((unsigned)std::max<long long>(blocks, 1)), dim3(256), 0, st,
                     in, out, n);
  return hipGetLastError();
}

hipError_t launch_single_family(const Geo& g, const Trig& t, const zd* khat, int family,
                                const zd* in, zd* X, zd* Y, zd* out, hipStream_t st) {
  return launch_tbc_passes(g, t, khat, nullptr, 0, family, 1, in, 0, X, Y, out, nullptr, st);
}

// ---------------------------------------------------------------------------------
// Krylov building blocks for nb right-hand sides iterating in lockstep.  Vector r of a
// set lives at base + r * n; basis vector i of right-hand side r at V + i * ldj + r * n.
// Reductions are two-stage and deterministic.  Inactive right-hand sides are skipped.
// ---------------------------------------------------------------------------------
constexpr int kDotGroup = 8;
constexpr int kDotUnroll = 4;
constexpr int kDotGroupWide = 16;   // basis vectors per group beyond kDotGroup
constexpr int kDotUnrollWide = 2;



// partial[(r * nvmax + vi) * nblk + blk] = sum over the block's slice of conj(V_vi,r) w_r,
// for the G basis vectors of group blockIdx.y.  VT: precision of the stored basis (double,
// or float in the mixed-precision solve).  Each thread sums its elements i, i + stride,
// i + 2 stride, ..., U of them per trip with every load of a trip issued before the
// products.  The variant is chosen from nv alone, so a solve's sums do not depend on how
// many right-hand sides share the launch.
template <typename VT, int G, int U>
__global__ __launch_bounds__(256) void k_dots(const cx<VT>* __restrict__ V, long long ldj, int nv,
                                              int nvmax, const zd* __restrict__ wall, long long n,
                                              zd* __restrict__ partial,
                                              const int* __restrict__ active) {
  __shared__ zd red[G][4];
  const int r = blockIdx.z;
  if (active && !active[r]) return;
  const int grp = blockIdx.y;
  const zd* w = wall + r * n;
  const cx<VT>* Vr = V + r * n;
  const int nvg = min(G, nv - grp * G);
  const cx<VT>* Vg = Vr + (long long)grp * G * ldj;
  zd acc[G];
  for (int t = 0; t < G; ++t) acc[t] = mk(0.0, 0.0);
  const long long stride = (long long)gridDim.x * blockDim.x;
  long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  for (; i + (U - 1) * stride < n; i += U * stride) {
    zd wi[U];
#pragma unroll
    for (int u = 0; u < U; ++u) wi[u] = w[i + u * stride];
#pragma unroll
    for (int t = 0; t < G; ++t) {
      if (t < nvg) {
        cx<VT> v[U];
#pragma unroll
        for (int u = 0; u < U; ++u) v[u] = Vg[t * ldj + i + u * stride];
#pragma unroll
        for (int u = 0; u < U; ++u) acc[t] = acc[t] + conj(widen(v[u])) * wi[u];
      }
    }
  }
  for (; i < n; i += stride) {
    const zd wi = w[i];
#pragma unroll
    for (int t = 0; t < G; ++t)
      if (t < nvg) acc[t] = acc[t] + conj(widen(Vg[t * ldj + i])) * wi;
  }
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
  for (int t = 0; t < G; ++t) {
    const zd sum = mk(wave_sum(acc[t].re), wave_sum(acc[t].im));
    if (lane == 0) red[t][wv] = sum;
  }
  __syncthreads();
  if (threadIdx.x < nvg) {
    const int t = threadIdx.x;
    partial[((long long)r * nvmax + grp * G + t) * gridDim.x + blockIdx.x] =
        red[t][0] + red[t][1] + red[t][2] + red[t][3];
  }
}

// out[r * ostride + vi] = sum_b partial;  when acc is given the sum is also added into
// acc[r * astride + vi]
__global__ void k_reduce_cols(const zd* __restrict__ partial, int nblk, int nvmax,
                              zd* __restrict__ out, long long ostride, zd* __restrict__ acc,
                              long long astride, const int* __restrict__ active) {
  __shared__ zd red[256];
  const int vi = blockIdx.x, r = blockIdx.y;
  if (active && !active[r]) return;
  zd s = mk(0.0, 0.0);
  const zd* p = partial + ((long long)r * nvmax + vi) * nblk;
  for (int i = threadIdx.x; i < nblk; i += blockDim.x) s = s + p[i];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int k = blockDim.x / 2; k > 0; k >>= 1) {
    if (threadIdx.x < k) red[threadIdx.x] = red[threadIdx.x] + red[threadIdx.x + k];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    out[r * ostride + vi] = red[0];
    if (acc) acc[r * astride + vi] = acc[r * astride + vi] + red[0];
  }
}

template <typename VT>
static hipError_t dots_impl(const cx<VT>* V, long long ldj, int nv, int nvmax, const zd* w,
                            long long n, int nb, zd* partial, int nblk, zd* out,
                            long long ostride, zd* acc, long long astride, const int* active,
                            hipStream_t st) {
  // groups of 8 basis vectors while there are at most 8, else of 16 (w read once per group)
  if (nv <= kDotGroup) {
    hipLaunchKernelGGL((k_dots<VT, kDotGroup, kDotUnroll>), dim3(nblk, 1, nb), dim3(256), 0, st,
                       V, ldj, nv, nvmax, w, n, partial, active);
  } else {
    const int ng = (nv + kDotGroupWide - 1) / kDotGroupWide;
    hipLaunchKernelGGL((k_dots<VT, kDotGroupWide, kDotUnrollWide>), dim3(nblk, ng, nb), dim3(256),
                       0, st, V, ldj, nv, nvmax, w, n, partial, active);
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_reduce_cols, dim3(nv, nb), dim3(256), 0, st, partial, nblk, nvmax, out,
                     ostride, acc, astride, active);
  return hipGetLastError();
}

hipError_t launch_dots(const zd* V, long long ldj, int nv, int nvmax, const zd* w, long long n,
                       int nb, zd* partial, int nblk, zd* out, long long ostride, zd* acc,
                       long long astride, const int* active, hipStream_t st) {
  return dots_impl<double>(V, ldj, nv, nvmax, w, n, nb, partial, nblk, out, ostride, acc,
                           astride, active, st);
}

hipError_t launch_dots(const zf* V, long long ldj, int nv, int nvmax, const zd* w, long long n,
                       int nb, zd* partial, int nblk, zd* out, long long ostride, zd* acc,
                       long long astride, const int* active, hipStream_t st) {
  return dots_impl<float>(V, ldj, nv, nvmax, w, n, nb, partial, nblk, out, ostride, acc,
                          astride, active, st);
}

// w_r -= sum_i h[r * hstride + i] V_i,r
template <typename VT>
__global__ __launch_bounds__(256) void k_update(const cx<VT>* __restrict__ V, long long ldj, int nv,
                                                const zd* __restrict__ h, long long hstride,
                                                zd* __restrict__ wall, long long n,
                                                const int* __restrict__ active) {
  __shared__ zd hs[256];
  const int r = blockIdx.y;
  if (active && !active[r]) return;
  for (int i = threadIdx.x; i < nv; i += blockDim.x) hs[i] = h[r * hstride + i];
  __syncthreads();
  zd* w = wall + r * n;
  const cx<VT>* Vr = V + r * n;
  const long long stride = (long long)gridDim.x * blockDim.x;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
    zd a = w[i];
    for (int vi = 0; vi < nv; ++vi) a = a - hs[vi] * widen(Vr[vi * ldj + i]);
    w[i] = a;
  }
}

template <typename VT>
static hipError_t update_impl(const cx<VT>* V, long long ldj, int nv, const zd* h,
                              long long hstride, zd* w, long long n, int nb, const int* active,
                              hipStream_t st) {
  int nblk = (int)((n + 255) / 256);
  if (nblk > 1024) nblk = 1024;
  hipLaunchKernelGGL((k_update<VT>), dim3(nblk, nb), dim3(256), 0, st, V, ldj, nv, h, hstride, w,
                     n, active);
  return hipGetLastError();
}

// First Gram-Schmidt update fused with the second pass's dot products, for nv <= G basis
// vectors: w_r -= sum_i h[r * hstride + i] V_i,r, then the per-block partial sums of
// conj(V_i,r) w_r (updated w) in k_dots' layout, from the same loads of V (one pass over
// the basis instead of two).
template <typename VT, int G, int U>
__global__ __launch_bounds__(256) void k_update_dots(const cx<VT>* __restrict__ V, long long ldj,
                                                     int nv, int nvmax,
                                                     const zd* __restrict__ h, long long hstride,
                                                     zd* __restrict__ wall, long long n,
                                                     zd* __restrict__ partial,
                                                     const int* __restrict__ active) {
  __shared__ zd hs[G];
  __shared__ zd red[G][4];
  const int r = blockIdx.y;
  if (active && !active[r]) return;
  if (threadIdx.x < nv) hs[threadIdx.x] = h[r * hstride + threadIdx.x];
  __syncthreads();
  zd* w = wall + r * n;
  const cx<VT>* Vr = V + r * n;
  zd acc[G];
  for (int t = 0; t < G; ++t) acc[t] = mk(0.0, 0.0);
  const long long stride = (long long)gridDim.x * blockDim.x;
  long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  for (; i + (U - 1) * stride < n; i += U * stride) {
    zd a[U];
    cx<VT> v[G][U];
#pragma unroll
    for (int u = 0; u < U; ++u) a[u] = w[i + u * stride];
#pragma unroll
    for (int t = 0; t < G; ++t)
      if (t < nv) {
#pragma unroll
        for (int u = 0; u < U; ++u) v[t][u] = Vr[t * ldj + i + u * stride];
#pragma unroll
        for (int u = 0; u < U; ++u) a[u] = a[u] - hs[t] * widen(v[t][u]);
      }
#pragma unroll
    for (int u = 0; u < U; ++u) w[i + u * stride] = a[u];
#pragma unroll
    for (int t = 0; t < G; ++t)
      if (t < nv) {
#pragma unroll
        for (int u = 0; u < U; ++u) acc[t] = acc[t] + conj(widen(v[t][u])) * a[u];
      }
  }
  for (; i < n; i += stride) {
    cx<VT> v[G];
    zd a = w[i];
#pragma unroll
    for (int t = 0; t < G; ++t)
      if (t < nv) {
        v[t] = Vr[t * ldj + i];
        a = a - hs[t] * widen(v[t]);
      }
    w[i] = a;
#pragma unroll
    for (int t = 0; t < G; ++t)
      if (t < nv) acc[t] = acc[t] + conj(widen(v[t])) * a;
  }
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
  for (int t = 0; t < G; ++t) {
    const zd sum = mk(wave_sum(acc[t].re), wave_sum(acc[t].im));
    if (lane == 0) red[t][wv] = sum;
  }
  __syncthreads();
  if (threadIdx.x < nv) {
    const int t = threadIdx.x;
    partial[((long long)r * nvmax + t) * gridDim.x + blockIdx.x] =
        red[t][0] + red[t][1] + red[t][2] + red[t][3];
  }
}

// Up to 8 basis vectors: 4 elements per trip; up to 16: 2 (single-precision basis) or 1
// (double) elements per trip, which keeps the loaded basis values within the registers.
template <typename VT>
static hipError_t update_dots_impl(const cx<VT>* V, long long ldj, int nv, int nvmax,
                                   const zd* h, long long hstride, zd* w, long long n, int nb,
                                   zd* partial, int nblk, zd* out, long long ostride, zd* acc,
                                   long long astride, const int* active, hipStream_t st) {
  if (nv < 1 || nv > kDotGroupWide) return hipErrorInvalidValue;
  constexpr int kUw = sizeof(VT) == sizeof(float) ? kDotUnrollWide : 1;
  if (nv <= kDotGroup)
    hipLaunchKernelGGL((k_update_dots<VT, kDotGroup, kDotUnroll>), dim3(nblk, nb), dim3(256), 0,
                       st, V, ldj, nv, nvmax, h, hstride, w, n, partial, active);
  else
    hipLaunchKernelGGL((k_update_dots<VT, kDotGroupWide, kUw>), dim3(nblk, nb), dim3(256), 0, st,
                       V, ldj, nv, nvmax, h, hstride, w, n, partial, active);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_reduce_cols, dim3(nv, nb), dim3(256), 0, st, partial, nblk, nvmax, out,
                     ostride, acc, astride, active);
  return hipGetLastError();
}

hipError_t launch_update_dots(const zd* V, long long ldj, int nv, int nvmax, const zd* h,
                              long long hstride, zd* w, long long n, int nb, zd* partial,
                              int nblk, zd* out, long long ostride, zd* acc, long long astride,
                              const int* active, hipStream_t st) {
  return update_dots_impl<double>(V, ldj, nv, nvmax, h, hstride, w, n, nb, partial, nblk, out,
                                  ostride, acc, astride, active, st);
}

hipError_t launch_update_dots(const zf* V, long long ldj, int nv, int nvmax, const zd* h,
                              long long hstride, zd* w, long long n, int nb, zd* partial,
                              int nblk, zd* out, long long ostride, zd* acc, long long astride,
                              const int* active, hipStream_t st) {
  return update_dots_impl<float>(V, ldj, nv, nvmax, h, hstride, w, n, nb, partial, nblk, out,
                                 ostride, acc, astride, active, st);
}

hipError_t launch_update(const zd* V, long long ldj, int nv, const zd* h, long long hstride,
                         zd* w, long long n, int nb, const int* active, hipStream_t st) {
  return update_impl<double>(V, ldj, nv, h, hstride, w, n, nb, active, st);
}

hipError_t launch_update(const zf* V, long long ldj, int nv, const zd* h, long long hstride,
                         zd* w, long long n, int nb, const int* active, hipStream_t st) {
  return update_impl<float>(V, ldj, nv, h, hstride, w, n, nb, active, st);
}

__global__ void k_norm2(const zd* __restrict__ wall, long long n, double* __restrict__ partial,
                        const int* __restrict__ active) {
  __shared__ double red[256];
  const int r = blockIdx.y;
  if (active && !active[r]) return;
  const zd* w = wall + r * n;
  double acc = 0.0;
  const long long stride = (long long)gridDim.x * blockDim.x;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride)
    acc += cabs2(w[i]);
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int s = blockDim.x / 2; s > 0; s >>= 1) {
    if (threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[(long long)r * gridDim.x + blockIdx.x] = red[0];
}

__global__ void k_reduce_d(const double* __restrict__ partial, int nblk, double* __restrict__ out,
                           const int* __restrict__ active) {
  __shared__ double red[256];
  const int r = blockIdx.x;
  if (active && !active[r]) return;
  double acc = 0.0;
  for (int i = threadIdx.x; i < nblk; i += blockDim.x) acc += partial[(long long)r * nblk + i];
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int s = blockDim.x / 2; s > 0; s >>= 1) {
    if (threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[r] = red[0];
}

hipError_t launch_norm2(const zd* w, long long n, int nb, double* partial, int nblk, double* out,
                        const int* active, hipStream_t st) {
  hipLaunchKernelGGL(k_norm2, dim3(nblk, nb), dim3(256), 0, st, w, n, partial, active);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_reduce_d, dim3(nb), dim3(256), 0, st, partial, nblk, out, active);
  return hipGetLastError();
}

// v_r = w_r / sqrt(nrm2[r]); v may alias w (element-wise, same index).
__global__ void k_scale_copy(const zd* wall, const double* __restrict__ nrm2, zd* vall, long long n,
                             long long vstride, const int* __restrict__ active) {
  const int r = blockIdx.y;
  if (active && !active[r]) return;
  const double s2 = nrm2[r];
  const double sc = s2 > 0.0 ? 1.0 / sqrt(s2) : 0.0;
  const zd* w = wall + r * n;
  zd* v = vall + r * vstride;
  const long long stride = (long long)gridDim.x * blockDim.x;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride)
    v[i] = sc * w[i];
}

hipError_t launch_scale_copy(const zd* w, const double* nrm2, zd* v, long long n,
                             long long vstride, int nb, const int* active, hipStream_t st) {
  int nblk = (int)((n + 255) / 256);
  if (nblk > 2048) nblk = 2048;
  hipLaunchKernelGGL(k_scale_copy, dim3(nblk, nb), dim3(256), 0, st, w, nrm2, v, n, vstride,
                     active);
  return hipGetLastError();
}

__global__ void k_sub(const zd* __restrict__ b, const zd* __restrict__ w, zd* __restrict__ out,
                      long long n, long long total) {
  const long long stride = (long long)gridDim.x * blockDim.x;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += stride)
    out[i] = b[i] - w[i];
}

hipError_t launch_sub(const zd* b, const zd* w, zd* r, long long total, hipStream_t st) {
  int nblk = (int)((total + 255) / 256);
  if (nblk > 4096) nblk = 4096;
  hipLaunchKernelGGL(k_sub, dim3(nblk), dim3(256), 0, st, b, w, r, total, total);
  return hipGetLastError();
}

// Givens step of GMRES for column j of every active right-hand side (one thread each).
// H[(r * restart + j) * (restart + 1) + i]: column j of the Hessenberg matrix, rotated in
// place into R.  Rotation [[c, s], [-conj(s), conj(c)]] with c = conj(a)/d, s = conj(b)/d.
__device__ inline void givens_step(const Krylov& kv, int r, int j, double nrm2) {
  const int R = kv.restart;
  zd* col = kv.H + ((long long)r * R + j) * (R + 1);
  zd* cs = kv.cs + (long long)r * R;
  zd* sn = kv.sn + (long long)r * R;
  zd* gv = kv.g + (long long)r * (R + 1);
  col[j + 1] = mk(sqrt(fmax(nrm2, 0.0)), 0.0);
  for (int i = 0; i < j; ++i) {
    const zd t = cs[i] * col[i] + sn[i] * col[i + 1];
    col[i + 1] = conj(sn[i]) * col[i] * mk(-1.0, 0.0) + conj(cs[i]) * col[i + 1];
    col[i] = t;
  }
  const double den = sqrt(cabs2(col[j]) + cabs2(col[j + 1]));
  zd c, s;
  if (den == 0.0) {
    c = mk(1.0, 0.0);
    s = mk(0.0, 0.0);
  } else {
    c = (1.0 / den) * conj(col[j]);
    s = (1.0 / den) * conj(col[j + 1]);
  }
  cs[j] = c;
  sn[j] = s;
  col[j] = mk(den, 0.0);
  col[j + 1] = mk(0.0, 0.0);
  const zd gj = gv[j];
  gv[j + 1] = mk(-1.0, 0.0) * conj(s) * gj;
  gv[j] = c * gj;
  const bool conv = sqrt(cabs2(gv[j + 1])) <= kv.thr[r] || den == 0.0;
  kv.jcount[r] = j + 1;
  const bool stop = conv || j + 1 >= R;
  if (stop) kv.active[r] = 0;
  if (kv.hflags) {
    kv.hflags[(long long)j * kv.nbh + r] = stop ? 0 : 1;
    kv.hratio[(long long)j * kv.nbh + r] = sqrt(cabs2(gv[j + 1])) / fmax(kv.thr[r], 1e-300);
  }
}

__global__ void k_givens(Krylov kv, int j, int nb) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= nb || !kv.active[r]) return;
  givens_step(kv, r, j, kv.nrm2[r]);
}

hipError_t launch_givens(const Krylov& kv, int j, int nb, hipStream_t st) {
  hipLaunchKernelGGL(k_givens, dim3((nb + 63) / 64), dim3(64), 0, st, kv, j, nb);
  return hipGetLastError();
}

__global__ void k_krylov_init(Krylov kv, int nb) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= nb) return;
  kv.bnorm[r] = sqrt(fmax(kv.nrm2[r], 0.0));
  kv.iters[r] = 0;
  kv.relres[r] = 0.0;
  kv.jcount[r] = 0;
}

__global__ void k_cycle_start(Krylov kv, int nb, int max_iter, double inner) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= nb) return;
  const double b = kv.bnorm[r];
  const double beta = sqrt(fmax(kv.nrm2[r], 0.0));
  const double rel = b > 0.0 ? beta / b : 0.0;
  kv.relres[r] = rel;
  const bool done = b == 0.0 || rel <= kv.tol || kv.iters[r] >= max_iter;
  kv.active[r] = done ? 0 : 1;
  kv.incycle[r] = done ? 0 : 1;
  kv.jcount[r] = 0;
  kv.g[(long long)r * (kv.restart + 1)] = mk(beta, 0.0);
  kv.thr[r] = fmax(kv.tol * b, inner * beta);
}

__global__ void k_cycle_end(Krylov kv, int nb) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= nb || !kv.incycle[r]) return;
  kv.iters[r] += kv.jcount[r];
}

hipError_t launch_krylov_init(const Krylov& kv, int nb, hipStream_t st) {
  hipLaunchKernelGGL(k_krylov_init, dim3((nb + 63) / 64), dim3(64), 0, st, kv, nb);
  return hipGetLastError();
}

hipError_t launch_cycle_start(const Krylov& kv, int nb, int max_iter, double inner,
                              hipStream_t st) {
  hipLaunchKernelGGL(k_cycle_start, dim3((nb + 63) / 64), dim3(64), 0, st, kv, nb, max_iter, inner);
  return hipGetLastError();
}

hipError_t launch_cycle_end(const Krylov& kv, int nb, hipStream_t st) {
  hipLaunchKernelGGL(k_cycle_end, dim3((nb + 63) / 64), dim3(64), 0, st, kv, nb);
  return hipGetLastError();
}

// Back-substitution R y = g on the first jcount[r] columns (one thread per rhs).
__global__ void k_solve_y(Krylov kv, int nb) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= nb || !kv.incycle[r]) return;
  const int R = kv.restart;
  const int jc = kv.jcount[r];
  const zd* Hr = kv.H + (long long)r * R * (R + 1);
  const zd* gv = kv.g + (long long)r * (R + 1);
  zd* y = kv.y + (long long)r * R;
  for (int i = jc - 1; i >= 0; --i) {
    zd acc = gv[i];
    for (int c = i + 1; c < jc; ++c) acc = acc - Hr[(long long)c * (R + 1) + i] * y[c];
    y[i] = cdiv(acc, Hr[(long long)i * (R + 1) + i]);
  }
}

hipError_t launch_solve_y(const Krylov& kv, int nb, hipStream_t st) {
  hipLaunchKernelGGL(k_solve_y, dim3((nb + 63) / 64), dim3(64), 0, st, kv, nb);
  return hipGetLastError();
}

// x_r += P^{-1} (sum_{i < jcount[r]} y[r][i] V_i,r)
template <typename VT>
__global__ void k_combine(Geo g, Krylov kv, const cx<VT>* __restrict__ V, long long ldj,
                          const zd* __restrict__ pinv_all, long long pcs, zd* __restrict__ xall) {
  __shared__ zd ys[256];
  const int r = blockIdx.y;
  if (!kv.incycle[r]) return;
  const zd* __restrict__ pinv = pinv_all + r * pcs;
  const int jc = kv.jcount[r];
  for (int i = threadIdx.x; i < jc; i += blockDim.x) ys[i] = kv.y[(long long)r * kv.restart + i];
  __syncthreads();
  const int mn = blockIdx.x * blockDim.x + threadIdx.x;
  if (mn >= g.NM) return;
  const long long n = 3LL * g.NM;
  const cx<VT>* Vr = V + r * n;
  zd* x = xall + r * n;
  zd u[3] = {mk(0.0, 0.0), mk(0.0, 0.0), mk(0.0, 0.0)};
  for (int vi = 0; vi < jc; ++vi) {
    const cx<VT>* col = Vr + vi * ldj;
    for (int c = 0; c < 3; ++c) u[c] = u[c] + ys[vi] * widen(col[(long long)c * g.NM + mn]);
  }
  for (int k = 0; k < 3; ++k) {
    const zd z = pinv[(3 * k) * (long long)g.NM + mn] * u[0] +
                 pinv[(3 * k + 1) * (long long)g.NM + mn] * u[1] +
                 pinv[(3 * k + 2) * (long long)g.NM + mn] * u[2];
    x[(long long)k * g.NM + mn] = x[(long long)k * g.NM + mn] + z;
  }
}

template <typename VT>
static hipError_t combine_impl(const Geo& g, const Krylov& kv, const cx<VT>* V, long long ldj,
                               const Cols& c, zd* x, int nb, hipStream_t st) {
  const int blk = 256;
  hipLaunchKernelGGL((k_combine<VT>), dim3((g.NM + blk - 1) / blk, nb), dim3(blk), 0, st, g, kv,
                     V, ldj, c.pinv, c.cs, x);
  return hipGetLastError();
}

hipError_t launch_combine(const Geo& g, const Krylov& kv, const zd* V, long long ldj,
                          const Cols& c, zd* x, int nb, hipStream_t st) {
  return combine_impl<double>(g, kv, V, ldj, c, x, nb, st);
}

hipError_t launch_combine(const Geo& g, const Krylov& kv, const zf* V, long long ldj,
                          const Cols& c, zd* x, int nb, hipStream_t st) {
  return combine_impl<float>(g, kv, V, ldj, c, x, nb, st);
}

// ---------------------------------------------------------------------------------
// Fused Arnoldi steps: the second Gram-Schmidt update with the norm of the result, and the
// normalisation with the Givens step and the preconditioner.
// ---------------------------------------------------------------------------------
// w_r -= sum_i h[r * hstride + i] V_i,r (in double precision, w stored in precision WT),
// then partial[r * gridDim.x + block] = block's share of |w_r|^2.
template <typename VT, typename WT>
__global__ __launch_bounds__(256) void k_update_norm(const cx<VT>* __restrict__ V, long long ldj, int nv,
                                                     const zd* __restrict__ h, long long hstride,
                                                     cx<WT>* __restrict__ wall, long long n,
                                                     double* __restrict__ partial,
                                                     const int* __restrict__ active) {
  __shared__ zd hs[256];
  __shared__ double red[4];
  const int r = blockIdx.y;
  if (active && !active[r]) return;
  for (int i = threadIdx.x; i < nv; i += blockDim.x) hs[i] = h[r * hstride + i];
  __syncthreads();
  cx<WT>* w = wall + r * n;
  const cx<VT>* Vr = V + r * n;
  double nrm = 0.0;
  const long long stride = (long long)gridDim.x * blockDim.x;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
    zd a = widen(w[i]);
    for (int vi = 0; vi < nv; ++vi) a = a - hs[vi] * widen(Vr[vi * ldj + i]);
    w[i] = cvt<WT>(a);
    nrm += cabs2(a);
  }
  nrm = wave_sum(nrm);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = nrm;
  __syncthreads();
  if (threadIdx.x == 0)
    partial[(long long)r * gridDim.x + blockIdx.x] = red[0] + red[1] + red[2] + red[3];
}

template <typename VT, typename WT>
static hipError_t update_norm_impl(const cx<VT>* V, long long ldj, int nv, const zd* h,
                                   long long hstride, cx<WT>* w, long long n, int nb,
                                   double* partial, int nblk, const int* active, hipStream_t st) {
  hipLaunchKernelGGL((k_update_norm<VT, WT>), dim3(nblk, nb), dim3(256), 0, st, V, ldj, nv, h,
                     hstride, w, n, partial, active);
  return hipGetLastError();
}

hipError_t launch_update_norm(const zd* V, long long ldj, int nv, const zd* h, long long hstride,
                              zd* w, long long n, int nb, double* partial, int nblk,
                              const int* active, hipStream_t st) {
  return update_norm_impl<double, double>(V, ldj, nv, h, hstride, w, n, nb, partial, nblk, active,
                                          st);
}

hipError_t launch_update_norm(const zf* V, long long ldj, int nv, const zd* h, long long hstride,
                              zd* w, long long n, int nb, double* partial, int nblk,
                              const int* active, hipStream_t st) {
  return update_norm_impl<float, double>(V, ldj, nv, h, hstride, w, n, nb, partial, nblk, active,
                                         st);
}

hipError_t launch_update_norm(const zf* V, long long ldj, int nv, const zd* h, long long hstride,
                              zf* w, long long n, int nb, double* partial, int nblk,
                              const int* active, hipStream_t st) {
  return update_norm_impl<float, float>(V, ldj, nv, h, hstride, w, n, nb, partial, nblk, active,
                                        st);
}

// Next basis vector: |w_r|^2 from the nparts partials of k_update_norm (nparts == 0: from
// kv.nrm2), then (j >= 0) the Givens step of column j by block 0, and v_r = w_r / |w_r|
// with its preconditioned copy z_r = P^{-1} v_r, computed in double precision and stored
// in precision ZT.  Threads run over modes; vectors are
// component-major.  Blocks read the active flag before block 0 may clear it; a rhs that
// stops here never uses the vector written for it.
template <typename VT, typename ZT, typename WT>
__global__ __launch_bounds__(256) void k_next_vector(Geo g, Krylov kv, int j,
                                                     const double* __restrict__ npart, int nparts,
                                                     const cx<WT>* __restrict__ wall,
                                                     cx<VT>* __restrict__ vall, long long vstride,
                                                     const zd* __restrict__ pinv_all,
                                                     long long pcs, cx<ZT>* __restrict__ zall) {
  __shared__ double red[4];
  __shared__ double s_nrm;
  const int r = blockIdx.y;
  if (!kv.active[r]) {
    if (j >= 0 && kv.hflags && blockIdx.x == 0 && threadIdx.x == 0)
      kv.hflags[(long long)j * kv.nbh + r] = 0;
    return;
  }
  if (nparts > 0) {
    double acc = 0.0;
    for (int i = threadIdx.x; i < nparts; i += blockDim.x) acc += npart[(long long)r * nparts + i];
    acc = wave_sum(acc);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) s_nrm = red[0] + red[1] + red[2] + red[3];
  } else if (threadIdx.x == 0) {
    s_nrm = kv.nrm2[r];
  }
  __syncthreads();
  const double nrm2 = s_nrm;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    kv.nrm2[r] = nrm2;
    if (j >= 0) givens_step(kv, r, j, nrm2);
  }
  const double sc = nrm2 > 0.0 ? 1.0 / sqrt(nrm2) : 0.0;
  const long long n = 3LL * g.NM;
  const cx<WT>* w = wall + r * n;
  cx<VT>* v = vall + r * vstride;
  cx<ZT>* z = zall + r * n;
  const zd* __restrict__ pinv = pinv_all + r * pcs;
  const long long stride = (long long)gridDim.x * blockDim.x;
  for (long long mn = (long long)blockIdx.x * blockDim.x + threadIdx.x; mn < g.NM; mn += stride) {
    zd u[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const cx<VT> t = cvt<VT>(sc * widen(w[c * g.NM + mn]));
      v[c * g.NM + mn] = t;
      u[c] = widen(t);   // z from the stored (possibly rounded) basis vector
    }
#pragma unroll
    for (int k = 0; k < 3; ++k)
      z[k * g.NM + mn] = cvt<ZT>(pinv[(3 * k) * (long long)g.NM + mn] * u[0] +
                                 pinv[(3 * k + 1) * (long long)g.NM + mn] * u[1] +
                                 pinv[(3 * k + 2) * (long long)g.NM + mn] * u[2]);
  }
}

template <typename VT, typename ZT, typename WT>
static hipError_t next_vector_impl(const Geo& g, const Krylov& kv, int j, const double* npart,
                                   int nparts, const cx<WT>* w, cx<VT>* v, long long vstride,
                                   const Cols& c, cx<ZT>* z, int nb, hipStream_t st) {
  int nblk = (g.NM + 255) / 256;
  if (nblk > 1024) nblk = 1024;
  hipLaunchKernelGGL((k_next_vector<VT, ZT, WT>), dim3(nblk, nb), dim3(256), 0, st, g, kv, j,
                     npart, nparts, w, v, vstride, c.pinv, c.cs, z);
  return hipGetLastError();
}

hipError_t launch_next_vector(const Geo& g, const Krylov& kv, int j, const double* npart,
                              int nparts, const zd* w, zd* v, long long vstride, const Cols& c,
                              zd* z, int nb, hipStream_t st) {
  return next_vector_impl<double, double, double>(g, kv, j, npart, nparts, w, v, vstride, c, z, nb,
                                                  st);
}

hipError_t launch_next_vector(const Geo& g, const Krylov& kv, int j, const double* npart,
                              int nparts, const zd* w, zf* v, long long vstride, const Cols& c,
                              zd* z, int nb, hipStream_t st) {
  return next_vector_impl<float, double, double>(g, kv, j, npart, nparts, w, v, vstride, c, z, nb,
                                                 st);
}

hipError_t launch_next_vector(const Geo& g, const Krylov& kv, int j, const double* npart,
                              int nparts, const zd* w, zf* v, long long vstride, const Cols& c,
                              zf* z, int nb, hipStream_t st) {
  return next_vector_impl<float, float, double>(g, kv, j, npart, nparts, w, v, vstride, c, z, nb,
                                                st);
}

hipError_t launch_next_vector(const Geo& g, const Krylov& kv, int j, const double* npart,
                              int nparts, const zf* w, zf* v, long long vstride, const Cols& c,
                              zf* z, int nb, hipStream_t st) {
  return next_vector_impl<float, float, float>(g, kv, j, npart, nparts, w, v, vstride, c, z, nb,
                                               st);
}

// ---------------------------------------------------------------------------------
// Back-substitution and synthesis (EInter): at level j the mode values are
//   E1 = Pi_j a1 + mu_m Theta_j a3,  E2 = Pi_j a2 + nu_n Theta_j a3,  E3 = Pi3_j a3,
// then the 2D sine/cosine series is summed on the output nodes: rows along y, then
// columns along x with TK adjacent columns per block.  Along either axis one of E1, E2
// takes the cosine series and the other the sine series, so both come from one transform
// of the even extension of one plus the odd extension of the other (store_pair_extension):
// two transforms per level and axis instead of three.
// One launch pair covers nr right-hand sides (solutions at xap + r xs) and jn levels from
// j0; the staging slab is tbuf[r][l][jj][m][i2], jj = j - j0.  The profiles do not depend
// on the right-hand side: a row block (row strip, level, E1+E2 or E3) takes kSynthRhsPerBlock
// right-hand sides in turn, and the blocks of one strip run next to each other on one XCD,
// so each profile strip comes from HBM about once per launch.
// ---------------------------------------------------------------------------------
constexpr int kSynthRhsPerBlock = 4;

template <int MR, int CTLC = 0>
__global__ __launch_bounds__(256) void k_synth_rows(Geo g, Fft out2, int lc_arg, int ip,
                                                    const zd* __restrict__ pi_d,
                                                    const zd* __restrict__ theta_d,
                                                    const zd* __restrict__ pi_n,
                                                    const zd* __restrict__ xap, long long xs,
                                                    int nr, int j0, int jn,
                                                    zd* __restrict__ tbuf) {
  CAV_DYN_SMEM(smem_raw);
  __shared__ zd c0s[64];
  const BlockId bid = xcd_block_x_slow();
  // blockIdx.y = 2 jj + q: q = 0 sums E1 (sine along y) and E2 (cosine along y) in one
  // transform of the paired extension, q = 1 sums E3 (sine along y)
  const int jj = bid.y >> 1, q = bid.y & 1;
  const int j = j0 + jj;
  const int lc = CTLC > 0 ? CTLC : lc_arg;
  const int C = 1 << lc;
  const int m0 = bid.x << lc;
  const int Cb = min(C, g.M + 1 - m0);
  const int L = g.ny;
  const DivBy div_l1(L + 1);
  zd* a = reinterpret_cast<zd*>(smem_raw);
  zd* b = a + ((2LL * L) << lc);   // second buffer of the ping-pong form only
  const int tid = threadIdx.x, nt = blockDim.x;
  const long long NM = g.NM;
  const int rowlen = g.N + 1;
  const DivBy div_row(rowlen);
  const int r0 = bid.z * kSynthRhsPerBlock;
  const int r1 = min(nr, r0 + kSynthRhsPerBlock);
  const long long slab = (long long)jn * (g.M + 1) * (g.ny + 1);   // one component's slab
  for (int r = r0; r < r1; ++r) {
    const zd* x = xap + r * xs;
    for (int i = tid; i < (2 * L) << lc; i += nt) a[i] = mk(0.0, 0.0);
    __syncthreads();
    // two elements per thread per trip, every load of a trip issued before its stores
    // (indices clamped in range: no conditional loads)
    const long long jNM = (long long)j * NM;
    for (int w0 = tid; w0 < rowlen * Cb; w0 += 2 * nt) {
      long long mn[2];
#pragma unroll
      for (int u = 0; u < 2; ++u) {
        const int w = min(w0 + u * nt, rowlen * Cb - 1);
        const int c = div_row.quot(w), n = w - c * div_row.d;
        mn[u] = (long long)(m0 + c) * rowlen + n;
      }
      if (q == 0) {
        zd pv[2], xa[2], xb[2], tv[2], x3[2];
#pragma unroll
        for (int u = 0; u < 2; ++u) {
          pv[u] = pi_d[jNM + mn[u]];
          xa[u] = x[mn[u]];
          xb[u] = x[NM + mn[u]];
          if (theta_d) {
            tv[u] = theta_d[jNM + mn[u]];
            x3[u] = x[2 * NM + mn[u]];
          }
        }
#pragma unroll
        for (int u = 0; u < 2; ++u) {
          const int w = w0 + u * nt;
          if (w >= rowlen * Cb) continue;
          const int c = div_row.quot(w), n = w - c * div_row.d;
          zd v1 = pv[u] * xa[u], v2 = pv[u] * xb[u];
          if (theta_d) {
            const zd t = tv[u] * x3[u];
            v1 = v1 + (g.pa * (m0 + c)) * t;
            v2 = v2 + (g.pb * n) * t;
          }
          store_pair_extension(a, L, n, v2, v1, lc, c);
          if (n == 0) c0s[c] = v2;
        }
      } else {
        zd pv[2], x3[2];
#pragma unroll
        for (int u = 0; u < 2; ++u) {
          pv[u] = pi_n[jNM + mn[u]];
          x3[u] = x[2 * NM + mn[u]];
        }
#pragma unroll
        for (int u = 0; u < 2; ++u) {
          const int w = w0 + u * nt;
          if (w >= rowlen * Cb) continue;
          const int c = div_row.quot(w), n = w - c * div_row.d;
          store_extension(a, L, false, n, pv[u] * x3[u], lc, c);
        }
      }
    }
    __syncthreads();
    zd* rr = lds_fft<double, false, MR, CTLC>(a, b, CtRadices<8, 8, 8>{}, out2.p, out2.tw, tid,
                                              nt, lc, ip);
    zd* dst = tbuf + ((((long long)r * 3 + (q == 0 ? 0 : 2)) * jn + jj) * (g.M + 1) + m0) *
                         (g.ny + 1);
    for (int w = tid; w < (L + 1) * Cb; w += nt) {
      const int c = div_l1.quot(w), i = w - c * div_l1.d;
      const zd F = rr[(i << lc) + c];
      const long long o = (long long)c * (g.ny + 1) + i;
      if (q == 0) {
        const zd Fm = rr[((i == 0 ? 0 : 2 * L - i) << lc) + c];
        dst[o] = 0.5 * mul_i(0.5 * (F - Fm));            // E1: sine series
        dst[slab + o] = 0.5 * (0.5 * (F + Fm) + c0s[c]);  // E2: cosine series
      } else {
        dst[o] = 0.5 * mul_i(F);
      }
    }
    __syncthreads();
  }
}

// Columns: blockIdx.y = 2 jj + q (q = 0: E1, cosine along x, with E2, sine along x, in
// one transform; q = 1: E3, sine along x), blockIdx.z = right-hand side r; field r at
// eout + r es.
template <int MR, int CTLC = 0>
__device__ inline void synth_cols_body(Geo g, Fft out1, int lc_arg, int ip, int j0, int jn,
                                       const zd* __restrict__ tbuf, zd* __restrict__ eout,
                                       long long es);

template <int MR>
__global__ __launch_bounds__(256) void k_synth_cols(Geo g, Fft out1, int lc_arg, int ip, int j0,
                                                    int jn, const zd* __restrict__ tbuf,
                                                    zd* __restrict__ eout, long long es) {
  synth_cols_body<MR, 0>(g, out1, lc_arg, ip, j0, jn, tbuf, eout, es);
}

// The compile-time form (extension transform 8 x 8 x 8, 4 columns per block, in place) as a
// kernel of its own, so that its bound of 5 waves per SIMD holds the fully unrolled stages
// to about 66 registers (about 114 without the bound, and fewer waves per SIMD).
__global__ __launch_bounds__(256, 5) void k_synth_cols_ct(Geo g, Fft out1, int lc_arg, int ip,
                                                          int j0, int jn,
                                                          const zd* __restrict__ tbuf,
                                                          zd* __restrict__ eout, long long es) {
  synth_cols_body<8, 2>(g, out1, lc_arg, ip, j0, jn, tbuf, eout, es);
}

template <int MR, int CTLC>
__device__ inline void synth_cols_body(Geo g, Fft out1, int lc_arg, int ip, int j0, int jn,
                                       const zd* __restrict__ tbuf, zd* __restrict__ eout,
                                       long long es) {
  CAV_DYN_SMEM(smem_raw);
  __shared__ zd c0s[64];
  const BlockId bid = xcd_block();
  const int jj = bid.y >> 1, q = bid.y & 1, r = bid.z;
  const int j = j0 + jj;
  const int lc = CTLC > 0 ? CTLC : lc_arg;
  const int C = 1 << lc;
  const int i0 = bid.x << lc;
  const int Cb = min(C, g.ny + 1 - i0);
  const int L = g.nx;
  const DivBy div_l1(L + 1);
  zd* a = reinterpret_cast<zd*>(smem_raw);
  zd* b = a + ((2LL * L) << lc);   // second buffer of the ping-pong form only
  const long long slab = (long long)jn * (g.M + 1) * (g.ny + 1);   // one component's slab
  const zd* src = tbuf + (((long long)r * 3 + (q == 0 ? 0 : 2)) * jn + jj) * (g.M + 1) * (g.ny + 1);
  const int tid = threadIdx.x, nt = blockDim.x;
  for (int i = tid; i < (2 * L) << lc; i += nt) a[i] = mk(0.0, 0.0);
  __syncthreads();
  for (int w0 = tid; w0 < (g.M + 1) << lc; w0 += kLoadBatch * nt) {
    zd x1[kLoadBatch], x2[kLoadBatch];
#pragma unroll
    for (int u = 0; u < kLoadBatch; ++u) {   // indices clamped in range: no conditional loads
      const int w = w0 + u * nt, m = min(w >> lc, g.M), c = min(w & (C - 1), Cb - 1);
      const long long o = (long long)m * (g.ny + 1) + i0 + c;
      x1[u] = src[o];
      x2[u] = src[(q == 0 ? slab : 0) + o];
    }
#pragma unroll
    for (int u = 0; u < kLoadBatch; ++u) {
      const int w = w0 + u * nt, m = w >> lc, c = w & (C - 1);
      if (m > g.M || c >= Cb) continue;
      if (q == 0) {
        store_pair_extension(a, L, m, x1[u], x2[u], lc, c);
        if (m == 0) c0s[c] = x1[u];
      } else {
        store_extension(a, L, false, m, x1[u], lc, c);
      }
    }
  }
  __syncthreads();
  zd* rr = lds_fft<double, false, MR, CTLC>(a, b, CtRadices<8, 8, 8>{}, out1.p, out1.tw, tid, nt,
                                            lc, ip);
  const long long plane = (long long)(g.Nz + 1) * (g.ny + 1) * (g.nx + 1);   // one component
  zd* dst = eout + r * es + (q == 0 ? 0 : 2 * plane) +
            ((long long)j * (g.ny + 1) + i0) * (g.nx + 1);
  for (int w = tid; w < (L + 1) * Cb; w += nt) {
    const int c = div_l1.quot(w), i = w - c * div_l1.d;
    const zd F = rr[(i << lc) + c];
    const long long o = (long long)c * (g.nx + 1) + i;
    if (q == 0) {
      const zd Fm = rr[((i == 0 ? 0 : 2 * L - i) << lc) + c];
      dst[o] = 0.5 * (0.5 * (F + Fm) + c0s[c]);           // E1: cosine series
      dst[plane + o] = 0.5 * mul_i(0.5 * (F - Fm));      // E2: sine series
    } else {
      dst[o] = 0.5 * mul_i(F);
    }
  }
}

// Batch of one synthesis pass: transforms of length 2 len per block (at most `cap`) and
// whether they run in place (one LDS buffer, every thread one work item per stage) or in
// the ping-pong form (two buffers; used when a stage has more work items than threads).
struct SynthShape {
  int lc, ip;
  size_t smem;
};
static SynthShape synth_shape(const FftPlan& p, int len, int cap, int budget) {
  const int items = fft_max_items(p);
  if (items <= 256) {
    int lc = batch_log2(len, (int)sizeof(zd), cap, budget);   // one buffer of 2 len
    while (lc > 0 && (items << lc) > 256) --lc;
    return {lc, 1, (size_t)2 * len * sizeof(zd) << lc};
  }
  const int lc = batch_log2(2 * len, (int)sizeof(zd), cap, budget);
  return {lc, 0, (size_t)4 * len * sizeof(zd) << lc};
}

hipError_t launch_synthesis(const Geo& g, const Trig& t, const zd* pi_d, const zd* theta_d,
                            const zd* pi_n, const zd* xap, long long xs, int nr, int j0, int j1,
                            zd* tbuf, zd* eout, long long es, hipStream_t st) {
  const int jn = j1 - j0;
  const double zb = sizeof(zd);
  const double tb = zb * 3.0 * nr * jn * (g.M + 1) * (double)(g.ny + 1);   // staging slab
  const double prof = zb * (double)jn * g.NM * (theta_d ? 3.0 : 2.0);
  static const int synth_budget = [] {
    const char* e = getenv("CAVITY_SYNTH_LDS");
    return e ? atoi(e) : 0;
  }();
  const SynthShape sr = synth_shape(t.out2.p, g.ny, g.M + 1, synth_budget);
  const int rgroups = (nr + kSynthRhsPerBlock - 1) / kSynthRhsPerBlock;
  probe_begin(K_SYNTH_ROWS, st);
  const dim3 grs((g.M + 1 + (1 << sr.lc) - 1) >> sr.lc, 2 * jn, rgroups);
  if (t.maxr <= kSmallRadix && plan_is<8, 8, 8>(t.out2.p) && sr.ip && sr.lc == 2)
    hipLaunchKernelGGL((k_synth_rows<8, 2>), grs, dim3(256), sr.smem, st, g, t.out2, sr.lc, sr.ip,
                       pi_d, theta_d, pi_n, xap, xs, nr, j0, jn, tbuf);
  else if (t.maxr <= 8)
    hipLaunchKernelGGL(k_synth_rows<8>, grs, dim3(256), sr.smem, st, g, t.out2, sr.lc, sr.ip, pi_d,
                       theta_d, pi_n, xap, xs, nr, j0, jn, tbuf);
  else
    hipLaunchKernelGGL(k_synth_rows<kMaxRadix>, grs, dim3(256), sr.smem, st, g, t.out2, sr.lc,
                       sr.ip, pi_d, theta_d, pi_n, xap, xs, nr, j0, jn, tbuf);
  probe_end(K_SYNTH_ROWS, st, prof + zb * 3.0 * g.NM * nr + tb);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const SynthShape sc = synth_shape(t.out1.p, g.nx, g.ny + 1, synth_budget);
  probe_begin(K_SYNTH_COLS, st);
  const dim3 gcs((g.ny + 1 + (1 << sc.lc) - 1) >> sc.lc, 2 * jn, nr);
  if (t.maxr <= kSmallRadix && plan_is<8, 8, 8>(t.out1.p) && sc.ip && sc.lc == 2)
    hipLaunchKernelGGL(k_synth_cols_ct, gcs, dim3(256), sc.smem, st, g, t.out1, sc.lc, sc.ip, j0,
                       jn, tbuf, eout, es);
  else if (t.maxr <= 8)
    hipLaunchKernelGGL(k_synth_cols<8>, gcs, dim3(256), sc.smem, st, g, t.out1, sc.lc, sc.ip, j0,
                       jn, tbuf, eout, es);
  else
    hipLaunchKernelGGL(k_synth_cols<kMaxRadix>, gcs, dim3(256), sc.smem, st, g, t.out1, sc.lc,
                       sc.ip, j0, jn, tbuf, eout, es);
  probe_end(K_SYNTH_COLS, st, tb + zb * 3.0 * nr * jn * (g.ny + 1) * (double)(g.nx + 1));
  return hipGetLastError();
}

// ---------------------------------------------------------------------------------
// Aperture transforms E^1(u) = sum E1_mn C_m(-u1) S_n(-u2), E^2(u) = sum E2_mn S_m(-u1) C_n(-u2)
// ---------------------------------------------------------------------------------
// Query q (blockIdx.y): solution q.rhs (at xall + rhs * n) at transform point (u1, u2);
// partial[(q * gridDim.x + block) * 2 + {0, 1}] = this block's share of (E^1, E^2).
__global__ void k_rcs_partial(Geo g, const zd* __restrict__ xall, long long n,
                              const RcsQuery* __restrict__ queries, zd* __restrict__ partial) {
  __shared__ zd red[2][256];
  const RcsQuery q = queries[blockIdx.y];
  const zd* xap = xall + (long long)q.rhs * n;
  const double u1 = q.u1, u2 = q.u2;
  zd s1 = mk(0.0, 0.0), s2 = mk(0.0, 0.0);
  const long long stride = (long long)gridDim.x * blockDim.x;
  for (long long mn = (long long)blockIdx.x * blockDim.x + threadIdx.x; mn < g.NM; mn += stride) {
    const int m = (int)(mn / (g.N + 1)), n = (int)(mn % (g.N + 1));
    const double mu = M_PI * m / g.a, nu = M_PI * n / g.b;
    if (n >= 1) s1 = s1 + xap[mn] * (cos_proj(-u1, mu, g.a) * sin_proj(-u2, nu, g.b));
    if (m >= 1) s2 = s2 + xap[g.NM + mn] * (sin_proj(-u1, mu, g.a) * cos_proj(-u2, nu, g.b));
  }
  red[0][threadIdx.x] = s1;
  red[1][threadIdx.x] = s2;
  __syncthreads();
  for (int s = blockDim.x / 2; s > 0; s >>= 1) {
    if (threadIdx.x < s) {
      red[0][threadIdx.x] = red[0][threadIdx.x] + red[0][threadIdx.x + s];
      red[1][threadIdx.x] = red[1][threadIdx.x] + red[1][threadIdx.x + s];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    zd* out = partial + 2 * ((long long)blockIdx.y * gridDim.x + blockIdx.x);
    out[0] = red[0][0];
    out[1] = red[1][0];
  }
}

hipError_t launch_rcs_partial(const Geo& g, const zd* xall, long long n, const RcsQuery* queries,
                              int nq, zd* partial, int nblk, hipStream_t st) {
  hipLaunchKernelGGL(k_rcs_partial, dim3(nblk, nq), dim3(256), 0, st, g, xall, n, queries,
                     partial);
  return hipGetLastError();
}

// Padded (three mode grids) <-> compact paper order (E1 on N1, E2 on N2, E3 on N3).
__device__ inline long long compact_index(const Geo& g, int c, int m, int n) {
  const long long M = g.M, N = g.N;
  if (c == 0) return (n >= 1) ? m * N + (n - 1) : -1;
  if (c == 1) return (m >= 1) ? (M + 1) * N + (m - 1) * (N + 1) + n : -1;
  return (m >= 1 && n >= 1) ? (M + 1) * N + M * (N + 1) + (m - 1) * N + (n - 1) : -1;
}

__global__ void k_pack(Geo g, const zd* __restrict__ xpad, zd* __restrict__ xc) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= 3LL * g.NM) return;
  const int c = (int)(i / g.NM);
  const int mn = (int)(i % g.NM);
  const long long ci = compact_index(g, c, mn / (g.N + 1), mn % (g.N + 1));
  if (ci >= 0) xc[ci] = xpad[i];
}

__global__ void k_unpack(Geo g, const zd* __restrict__ xc, zd* __restrict__ xpad) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= 3LL * g.NM) return;
  const int c = (int)(i / g.NM);
  const int mn = (int)(i % g.NM);
  const long long ci = compact_index(g, c, mn / (g.N + 1), mn % (g.N + 1));
  xpad[i] = ci >= 0 ? xc[ci] : mk(0.0, 0.0);
}

hipError_t launch_pack(const Geo& g, const zd* xpad, zd* xcompact, hipStream_t st) {
  const long long n = 3LL * g.NM;
  hipLaunchKernelGGL(k_pack, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, g, xpad,
                     xcompact);
  return hipGetLastError();
}

hipError_t launch_unpack(const Geo& g, const zd* xcompact, zd* xpad, hipStream_t st) {
  const long long n = 3LL * g.NM;
  hipLaunchKernelGGL(k_unpack, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, g, xcompact,
                     xpad);
  return hipGetLastError();
}

}  // namespace cav
