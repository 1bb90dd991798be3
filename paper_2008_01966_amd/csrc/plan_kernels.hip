// Plan-time kernels: truncated-kernel spectrum (Section 5.2), per-mode z-elimination
// (Sections 3-4), and the per-mode block preconditioner of the aperture system.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "kernels.hpp"

namespace cav {

// ---------------------------------------------------------------------------------
// Spectrum.  G^_R(rho) = 1/2 int_0^R J0(rho r) e^{ikr} dr is evaluated through
// J0(x) = (1/pi) int_0^pi e^{i x cos t} dt as (1/(2 pi)) int_0^pi E_R(k + rho cos t) dt,
// E_R(w) = (e^{iwR} - 1)/(iw) = R e^{i wR/2} sinc(wR/2).  The t-integrand is analytic and
// even-periodic, so the midpoint rule with n_t > rho R / 2 nodes converges geometrically.
// One thread per lattice point of the first quadrant (|j1|, |j2|); K^ depends on |xi|
// only and is scattered to the mirror points.
// ---------------------------------------------------------------------------------
__device__ inline zd exp_integral(double w, double len) {
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

// Asymptotic form for large rho (Case 2 of Section 5.2).  With Z = rho R and a = k / rho,
//   int_0^R J0(rho r) e^{ikr} dr = 1/sqrt(rho^2 - k^2) - sqrt(2/pi)/rho * T,
// T the tail beyond Z of [cos(z - pi/4) z^{-1/2} + sin(z - pi/4) z^{-3/2} / 8] e^{iaz}
// (two-term Hankel expansion of J0).  Splitting cos and sin into exponentials leaves
// tails F(p) = int_Z^inf e^{ipz} z^{-1/2} dz and, by parts, int_Z^inf e^{iqz} z^{-3/2} dz
// = 2 e^{iqZ}/sqrt(Z) + 2iq F(q); F(p) = sqrt(pi/(2|p|)) (1 - 2C(t) + i (1 - 2S(t))),
// t = sqrt(2|p|Z/pi) (conjugated for p < 0), with the two-term asymptotic expansions of
// the Fresnel integrals C, S.
constexpr double kAsymptoticSwitch = 100.0;   // applies where (rho - k) R >= this

__device__ inline zd fresnel_tail(double p, double Z) {
  const double ap = fabs(p);
  const double t = sqrt(2.0 * ap * Z / M_PI);
  const double x = M_PI * t * t, x2 = x * x;
  const double f = (1.0 - 3.0 / x2) / (M_PI * t);
  const double gg = (1.0 - 15.0 / x2) / (M_PI * M_PI * t * t * t);
  double sp, cp;
  sincos(ap * Z, &sp, &cp);
  const double amp = sqrt(M_PI / (2.0 * ap));
  const double re = amp * (-2.0 * f * sp + 2.0 * gg * cp);
  const double im = amp * (2.0 * f * cp + 2.0 * gg * sp);
  return mk(re, p > 0 ? im : -im);
}

__device__ inline zd tail_32(double q, double Z) {
  double s, c;
  sincos(q * Z, &s, &c);
  const double w = 2.0 / sqrt(Z);
  const zd F = fresnel_tail(q, Z);
  // 2 e^{iqZ}/sqrt(Z) + 2 i q F
  return mk(w * c - 2.0 * q * F.im, w * s + 2.0 * q * F.re);
}

__device__ inline zd ghat_asymptotic(double rho, double k, double R) {
  const double Z = rho * R, a = k / rho;
  const double h = 0.70710678118654752440;   // cos(pi/4) = sin(pi/4)
  const zd em = mk(h, -h), ep = mk(h, h);
  const zd t1 = em * fresnel_tail(1.0 + a, Z), t2 = ep * fresnel_tail(a - 1.0, Z);
  const zd d = em * tail_32(1.0 + a, Z) - ep * tail_32(a - 1.0, Z);
  // T = (t1 + t2) / 2 + d / (16 i)
  const zd T = mk(0.5 * (t1.re + t2.re) + d.im / 16.0, 0.5 * (t1.im + t2.im) - d.re / 16.0);
  const double inf = 1.0 / sqrt(rho * rho - k * k);
  const double c = sqrt(2.0 / M_PI) / rho;
  return mk(0.5 * (inf - c * T.re), -0.5 * c * T.im);
}

// `split` consecutive lanes (a power of two up to 64) share one lattice point and split
// its quadrature nodes: the node count grows with rho, so one lane per point left the far
// corner's lanes with most of the work.  Measured at P = 625: 537 us with one lane per
// point, 343 / 306 / 281 / 283 us with 4 / 8 / 16 / 32; with the asymptotic form (one lane
// of each group evaluates it) 95 / 25 / 35 / 55 / 95 us.
constexpr int kSpecSplitQuadrature = 16;
constexpr int kSpecSplitAsymptotic = 4;

__global__ void k_spectrum(Geo g, double R, double scale, int method, int split, zd* __restrict__ khat) {
  const int s = threadIdx.x & (split - 1);
  const int u1 = blockIdx.y * blockDim.y + threadIdx.y;
  const int u2 = blockIdx.x * (blockDim.x / split) + threadIdx.x / split;
  const bool live = u1 <= g.P1 / 2 && u2 <= g.P2 / 2;   // every lane takes part in the sums
  const double L1 = g.P1 * g.hq1, L2 = g.P2 * g.hq2;
  const double x1 = 2.0 * M_PI * u1 / L1, x2 = 2.0 * M_PI * u2 / L2;
  const double rho = sqrt(x1 * x1 + x2 * x2);
  const bool asym = method == 1 && (rho - g.k) * R >= kAsymptoticSwitch;
  const int nt = (int)ceil(0.5 * (rho + g.k) * R) + 48;
  double sr = 0.0, si = 0.0;
  if (live && !asym) {
    for (int i = s; i < nt; i += split) {
      const double ct = cospi((i + 0.5) / nt);
      const zd e = exp_integral(g.k + rho * ct, R);
      sr += e.re;
      si += e.im;
    }
  }
  for (int o = 1; o < split; o <<= 1) {
    sr += __shfl_xor(sr, o, 64);
    si += __shfl_xor(si, o, 64);
  }
  if (!live || s != 0) return;
  zd val;
  if (asym) {
    const zd v = ghat_asymptotic(rho, g.k, R);
    val = mk(scale * v.re, scale * v.im);
  } else {
    val = mk(scale * sr / (2.0 * nt), scale * si / (2.0 * nt));
  }
  const int i1a = u1, i1b = (g.P1 - u1) % g.P1;
  const int i2a = u2, i2b = (g.P2 - u2) % g.P2;
  khat[(long long)i1a * g.P2 + i2a] = val;
  khat[(long long)i1a * g.P2 + i2b] = val;
  khat[(long long)i1b * g.P2 + i2a] = val;
  khat[(long long)i1b * g.P2 + i2b] = val;
}

hipError_t launch_spectrum(const Geo& g, double R, double scale, int method, zd* khat,
                           hipStream_t st) {
  dim3 blk(64, 4);   // 64 / split points of a lattice row per wavefront, 4 rows per block
  const int split = method == 1 ? kSpecSplitAsymptotic : kSpecSplitQuadrature;
  const int per_row = blk.x / split;
  dim3 grd((g.P2 / 2 + 1 + per_row - 1) / per_row, (g.P1 / 2 + 1 + blk.y - 1) / blk.y);
  probe_begin(K_SPECTRUM, st);
  hipLaunchKernelGGL(k_spectrum, grd, blk, 0, st, g, R, scale, method, split, khat);
  probe_end(K_SPECTRUM, st, sizeof(zd) * (double)g.P1 * g.P2);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------------
// Elimination.  One thread per mode (m, n); profiles laid out [node][mode] so that a
// wavefront touches 64 consecutive modes (coalesced).
//
// E3 (Neumann bottom, E3_0 = E3_1): relation V(j-1) = alpha_j V(j) within a layer;
//   interior node: alpha_{j+1} = -1 / (alpha_j - 2 + h_l^2 lambda_l), h_l the layer's step
//   interface node (derivative continuity with eps_up E3^+ = eps_lo E3^-, each one-sided
//   difference over its own layer's step, q = h_up / h_lo):
//                  alpha_{j+1} = 1 / (1 + (1 - alpha_j) q eps_up / eps_lo)
// E1/E2 (Dirichlet bottom): E_{j-1} = alpha_j E_j + b_j E3_top (times mu_m or nu_n);
//   interior: pivot alpha_j - 2 + h_l^2 lambda_l, no source;
//   interface: row q E_{j-1} - (1 + q) E_j + E_{j+1} = h_up (1 - eps_up/eps_lo) Pi3_s
//   (tangential-curl continuity with one-sided differences): pivot q alpha_j - (1 + q),
//   b_{j+1} = (source - q b_j) / pivot.  With one step everywhere q = 1.
// rho = alpha_Nz, T = b_Nz; profiles by back-substitution from the aperture (value 1).
// The back-substitution needs the alphas (and b) in reverse order.  The up-sweep keeps
// only the first value of every segment of kElimSeg levels (checkpoints, in the profile
// slot of that level); the down-sweep recomputes a segment's values from its checkpoint
// with the same per-level step, holds them in registers and walks them backwards, so each
// profile entry is written once instead of written, read back and overwritten.
// ---------------------------------------------------------------------------------
constexpr int kElimSeg = 8;

// E3 step at node j: alpha_{j+1} from alpha_j (piv: the pivot).
__device__ inline zd elim_e3_step(const Layers& ly, int j, double mn2, zd al, zd* piv) {
  const int code = ly.node_code[j];
  if (code >= 0) {
    const zd k2 = ly.kappa2[code];
    const double h2 = ly.h[code] * ly.h[code];
    *piv = mk(al.re - 2.0 + h2 * (k2.re - mn2), al.im + h2 * k2.im);
    return cdiv(mk(-1.0, 0.0), *piv);
  }
  const int s = -code - 1;
  const double q = ly.h[s + 1] / ly.h[s];
  const zd r = ly.ratio[s];
  const zd one_m = mk(1.0 - al.re, -al.im);
  *piv = mk(1.0, 0.0) + one_m * (q * r);
  return cdiv(mk(1.0, 0.0), *piv);
}

// E1/E2 step at node j: (alpha, b)_{j+1} from (alpha, b)_j; p3 = Pi3_j (read at interfaces
// only, when has3).
__device__ inline void elim_d_step(const Layers& ly, int j, double mn2, bool has3,
                                   const zd* __restrict__ pi_n_j, zd* al, zd* bb, zd* piv) {
  const int code = ly.node_code[j];
  zd f = mk(0.0, 0.0);
  double q = 1.0;
  if (code >= 0) {
    const zd k2 = ly.kappa2[code];
    const double h2 = ly.h[code] * ly.h[code];
    *piv = mk(al->re - 2.0 + h2 * (k2.re - mn2), al->im + h2 * k2.im);
  } else {
    const int s = -code - 1;
    const double h_up = ly.h[s + 1];
    q = h_up / ly.h[s];
    *piv = mk(q * al->re - (1.0 + q), q * al->im);
    if (has3) {
      const zd r = ly.ratio[s];
      f = h_up * (mk(1.0 - r.re, -r.im) * *pi_n_j);
    }
  }
  const zd inv = cdiv(mk(1.0, 0.0), *piv);
  *al = mk(-inv.re, -inv.im);
  *bb = (f - q * *bb) * inv;
}

__global__ void k_elimination(Geo g, Layers ly, zd* __restrict__ rho_d, zd* __restrict__ Tout,
                              zd* __restrict__ rho_n, zd* __restrict__ pi_d,
                              zd* __restrict__ theta_d, zd* __restrict__ pi_n,
                              double* __restrict__ pivmin) {
  const int mn = blockIdx.x * blockDim.x + threadIdx.x;
  if (mn >= g.NM) return;
  const int m = mn / (g.N + 1), n = mn % (g.N + 1);
  const double mu = M_PI * m / g.a, nu = M_PI * n / g.b;
  const double mn2 = mu * mu + nu * nu;
  const long long NM = g.NM;
  const int Nz = g.Nz;
  const bool has3 = (m >= 1 && n >= 1);
  double pmin = 1e300;
  constexpr int K = kElimSeg;
  const int nseg = (Nz + K - 1) / K;   // segment s: alphas of levels s K + 1 .. (s + 1) K

  // ---- E3 column ----
  if (has3) {
    zd al = mk(1.0, 0.0);   // alpha_1
    pi_n[1 * NM + mn] = al;
    for (int j = 1; j < Nz; ++j) {
      zd piv;
      al = elim_e3_step(ly, j, mn2, al, &piv);
      pmin = fmin(pmin, sqrt(cabs2(piv)));
      if (j % K == 0) pi_n[(long long)(j + 1) * NM + mn] = al;   // checkpoint alpha_{j+1}
    }
    rho_n[mn] = al;
    zd cur = mk(1.0, 0.0);
    for (int sg = nseg - 1; sg >= 0; --sg) {
      const int j0 = sg * K + 1, cnt = min(K, Nz - j0 + 1);
      zd A[K];
      A[0] = pi_n[(long long)j0 * NM + mn];
#pragma unroll
      for (int t = 1; t < K; ++t) {
        zd piv;
        if (t < cnt) A[t] = elim_e3_step(ly, j0 + t - 1, mn2, A[t - 1], &piv);
      }
#pragma unroll
      for (int t = K - 1; t >= 0; --t) {
        if (t >= cnt) continue;
        const int j = j0 + t;
        pi_n[(long long)j * NM + mn] = cur;
        const int code = ly.node_code[j];
        const zd aj = code < 0 ? A[t] * ly.ratio[-code - 1] : A[t];
        cur = aj * cur;
      }
    }
    pi_n[mn] = cur;
  } else {
    for (int j = 0; j <= Nz; ++j) pi_n[(long long)j * NM + mn] = mk(0.0, 0.0);
    rho_n[mn] = mk(0.0, 0.0);
  }

  // ---- E1/E2 column ----
  zd al = mk(0.0, 0.0), bb = mk(0.0, 0.0);   // alpha_1, b_1
  pi_d[1 * NM + mn] = al;
  if (ly.layered) theta_d[1 * NM + mn] = bb;
  for (int j = 1; j < Nz; ++j) {
    zd piv;
    elim_d_step(ly, j, mn2, has3, pi_n + (long long)j * NM + mn, &al, &bb, &piv);
    if (mn != 0) pmin = fmin(pmin, sqrt(cabs2(piv)));
    if (j % K == 0) {   // checkpoint (alpha, b)_{j+1}
      pi_d[(long long)(j + 1) * NM + mn] = al;
      if (ly.layered) theta_d[(long long)(j + 1) * NM + mn] = bb;
    }
  }
  rho_d[mn] = al;
  Tout[mn] = has3 ? bb : mk(0.0, 0.0);
  zd cp = mk(1.0, 0.0), ct = mk(0.0, 0.0);
  for (int sg = nseg - 1; sg >= 0; --sg) {
    const int j0 = sg * K + 1, cnt = min(K, Nz - j0 + 1);
    zd A[K], B[K];
    A[0] = pi_d[(long long)j0 * NM + mn];
    B[0] = ly.layered ? theta_d[(long long)j0 * NM + mn] : mk(0.0, 0.0);
#pragma unroll
    for (int t = 1; t < K; ++t) {
      if (t >= cnt) continue;
      zd a = A[t - 1], b = B[t - 1], piv;
      elim_d_step(ly, j0 + t - 1, mn2, has3, pi_n + (long long)(j0 + t - 1) * NM + mn, &a, &b,
                  &piv);
      A[t] = a;
      B[t] = b;
    }
#pragma unroll
    for (int t = K - 1; t >= 0; --t) {
      if (t >= cnt) continue;
      const int j = j0 + t;
      pi_d[(long long)j * NM + mn] = cp;
      zd bj = mk(0.0, 0.0);
      if (ly.layered) {
        bj = B[t];
        theta_d[(long long)j * NM + mn] = has3 ? ct : mk(0.0, 0.0);
      }
      ct = A[t] * ct + bj;
      cp = A[t] * cp;
    }
  }
  pi_d[mn] = cp;
  if (ly.layered) theta_d[mn] = mk(0.0, 0.0);
  pivmin[mn] = pmin;
}

hipError_t launch_elimination(const Geo& g, const Layers& ly, zd* rho_d, zd* T, zd* rho_n,
                              zd* pi_d, zd* theta_d, zd* pi_n, double* pivmin,
                              hipStream_t st) {
  const int blk = 128;
  probe_begin(K_ELIMINATION, st);
  hipLaunchKernelGGL(k_elimination, dim3((g.NM + blk - 1) / blk), dim3(blk), 0, st, g, ly,
                     rho_d, T, rho_n, pi_d, theta_d, pi_n, pivmin);
  // profiles written once (Pi, Pi3, and Theta when layered) plus the Schur data
  probe_end(K_ELIMINATION, st,
            sizeof(zd) * (double)g.NM * ((g.Nz + 1.0) * (ly.layered ? 3.0 : 2.0) + 3.0));
  return hipGetLastError();
}

// ---------------------------------------------------------------------------------
// Exact diagonal of the discrete single-layer operators (used by the preconditioner).
// S_aa = sum_j K^s[j] |A1_m(j1)|^2 |A2_n(j2)|^2 with A_m(j) = sum_i w_i psi_m(x_i)
// e^{-2 pi i j i / P} (the padded DFT of the trapezoid-weighted mode), K^s the scaled
// spectrum.  Kinds: 0 = cos, 1 = sin.  pw1[kind][m][j1]; pw2[kind][j2][n] (transposed).
// ---------------------------------------------------------------------------------
__global__ void k_basis_power(Geo g, Fft box1, Fft box2, double* __restrict__ pw1,
                              double* __restrict__ pw2) {
  CAV_DYN_SMEM(smem_raw);
  zd* buf = reinterpret_cast<zd*>(smem_raw);
  const int axis = blockIdx.y >> 1, kind = blockIdx.y & 1;
  const int m = blockIdx.x;
  const int nmodes = axis == 0 ? g.M + 1 : g.N + 1;
  if (m >= nmodes) return;
  const Fft& F = axis == 0 ? box1 : box2;
  const int P = F.p.n;
  const int nq = axis == 0 ? g.nq1 : g.nq2;
  const double hq = axis == 0 ? g.hq1 : g.hq2;
  zd* a = buf;
  zd* b = buf + P;
  for (int i = threadIdx.x; i < P; i += blockDim.x) {
    zd v = mk(0.0, 0.0);
    if (i <= nq) {
      const long long t = ((long long)m * i) % (2LL * nq);
      const double arg = (double)t / nq;
      const double psi = kind == 0 ? cospi(arg) : sinpi(arg);
      const double w = (i == 0 || i == nq) ? 0.5 * hq : hq;
      v = mk(w * psi, 0.0);
    }
    a[i] = v;
  }
  __syncthreads();
  zd* r = fft_lds<double, false, kMaxRadix>(a, b, F.p, F.tw, threadIdx.x, blockDim.x, 0);
  for (int j = threadIdx.x; j < P; j += blockDim.x) {
    const double p = cabs2(r[j]);
    if (axis == 0)
      pw1[((long long)kind * (g.M + 1) + m) * P + j] = p;
    else
      pw2[((long long)kind * P + j) * (g.N + 1) + m] = p;
  }
}

hipError_t launch_basis_power(const Geo& g, const Trig& t, double* pw1, double* pw2,
                              hipStream_t st) {
  const int rows = (g.M > g.N ? g.M : g.N) + 1;
  const int pmax = g.P1 > g.P2 ? g.P1 : g.P2;
  hipLaunchKernelGGL(k_basis_power, dim3(rows, 4), dim3(256), 2 * pmax * sizeof(zd), st, g,
                     t.box1, t.box2, pw1, pw2);
  return hipGetLastError();
}

// tmp[kind2][j1][n] = sum_j2 khat[j1][j2] pw2[kind2][j2][n]
__global__ void k_contract_a(Geo g, const zd* __restrict__ khat, const double* __restrict__ pw2,
                             zd* __restrict__ tmp) {
  const int n = blockIdx.x * blockDim.x + threadIdx.x;
  const int j1 = blockIdx.y;
  const int kind = blockIdx.z;
  if (n > g.N) return;
  double sr = 0.0, si = 0.0;
  const zd* krow = khat + (long long)j1 * g.P2;
  const double* col = pw2 + (long long)kind * g.P2 * (g.N + 1) + n;
  for (int j2 = 0; j2 < g.P2; ++j2) {
    const double p = col[(long long)j2 * (g.N + 1)];
    const zd kv = krow[j2];
    sr += kv.re * p;
    si += kv.im * p;
  }
  tmp[((long long)kind * g.P1 + j1) * (g.N + 1) + n] = mk(sr, si);
}

// diag[f][m][n] = sum_j1 pw1[k1(f)][m][j1] tmp[k2(f)][j1][n]
__global__ void k_contract_b(Geo g, const double* __restrict__ pw1, const zd* __restrict__ tmp,
                             zd* __restrict__ diag) {
  const int n = blockIdx.x * blockDim.x + threadIdx.x;
  const int m = blockIdx.y;
  const int f = blockIdx.z;
  if (n > g.N) return;
  const int k1 = (f == 1) ? 1 : 0;   // cs: cos, sc: sin, cc: cos along x1
  const int k2 = (f == 0) ? 1 : 0;   // cs: sin, sc: cos, cc: cos along x2
  const double* row = pw1 + ((long long)k1 * (g.M + 1) + m) * g.P1;
  const zd* col = tmp + (long long)k2 * g.P1 * (g.N + 1) + n;
  double sr = 0.0, si = 0.0;
  for (int j1 = 0; j1 < g.P1; ++j1) {
    const double p = row[j1];
    const zd t = col[(long long)j1 * (g.N + 1)];
    sr += p * t.re;
    si += p * t.im;
  }
  diag[(long long)f * g.NM + (long long)m * (g.N + 1) + n] = mk(sr, si);
}

hipError_t launch_diag_contract(const Geo& g, const zd* khat, const double* pw1,
                                const double* pw2, zd* tmp, zd* diag, hipStream_t st) {
  const int blk = 64;
  const int gx = (g.N + 1 + blk - 1) / blk;
  hipLaunchKernelGGL(k_contract_a, dim3(gx, g.P1, 2), dim3(blk), 0, st, g, khat, pw2, tmp);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_contract_b, dim3(gx, g.M + 1, 3), dim3(blk), 0, st, g, pw1, tmp, diag);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------------
// Block preconditioner: per mode the 3x3 block of the reduced aperture operator with
// each S^f replaced by its diagonal; components outside their mode set get identity
// rows/columns.  Stored inverted, pinv[e][mn], e = 3*row + col.
// ---------------------------------------------------------------------------------
__global__ void k_precond_build(Geo g, const zd* __restrict__ rho_d, const zd* __restrict__ T,
                                const zd* __restrict__ rho_n, const zd* __restrict__ diag,
                                zd* __restrict__ pinv) {
  const int mn = blockIdx.x * blockDim.x + threadIdx.x;
  if (mn >= g.NM) return;
  const int m = mn / (g.N + 1), n = mn % (g.N + 1);
  const double mu = M_PI * m / g.a, nu = M_PI * n / g.b, h = g.h, k2 = g.k * g.k;
  const double hq = h / ((m == 0 ? 0.5 : 0.25) * g.a * g.b);
  const double hc = h / ((n == 0 ? 0.5 : 0.25) * g.a * g.b);
  const zd dcs = diag[mn], dsc = diag[g.NM + mn], dcc = diag[2LL * g.NM + mn];
  const zd rd = rho_d[mn], rn = rho_n[mn], t = T[mn];
  const zd one = mk(1.0, 0.0);
  zd A[3][3];
  A[0][0] = (rd - one) + hq * ((2.0 * k2) * dcs - (2.0 * nu * nu) * dcc);
  A[0][1] = (hq * 2.0 * nu * mu) * dcc;
  A[0][2] = mu * (t + mk(h, 0.0));
  A[1][0] = (hc * 2.0 * mu * nu) * dcc;
  A[1][1] = (rd - one) + hc * ((2.0 * k2) * dsc - (2.0 * mu * mu) * dcc);
  A[1][2] = nu * (t + mk(h, 0.0));
  A[2][0] = mk(mu * h, 0.0);
  A[2][1] = mk(nu * h, 0.0);
  A[2][2] = rn - one;
  const bool valid[3] = {n >= 1, m >= 1, m >= 1 && n >= 1};
  for (int c = 0; c < 3; ++c) {
    if (!valid[c]) {
      for (int e = 0; e < 3; ++e) {
        A[c][e] = mk(0.0, 0.0);
        A[e][c] = mk(0.0, 0.0);
      }
      A[c][c] = one;
    }
  }
  // Gauss-Jordan with partial pivoting on [A | I]
  zd B[3][3];
  for (int r = 0; r < 3; ++r)
    for (int c = 0; c < 3; ++c) B[r][c] = (r == c) ? one : mk(0.0, 0.0);
  for (int col = 0; col < 3; ++col) {
    int piv = col;
    double best = cabs2(A[col][col]);
    for (int r = col + 1; r < 3; ++r) {
      const double v = cabs2(A[r][col]);
      if (v > best) {
        best = v;
        piv = r;
      }
    }
    if (piv != col) {
      for (int c = 0; c < 3; ++c) {
        zd tmp = A[col][c]; A[col][c] = A[piv][c]; A[piv][c] = tmp;
        tmp = B[col][c]; B[col][c] = B[piv][c]; B[piv][c] = tmp;
      }
    }
    const zd inv = cdiv(one, A[col][col]);
    for (int c = 0; c < 3; ++c) {
      A[col][c] = A[col][c] * inv;
      B[col][c] = B[col][c] * inv;
    }
    for (int r = 0; r < 3; ++r) {
      if (r == col) continue;
      const zd f = A[r][col];
      for (int c = 0; c < 3; ++c) {
        A[r][c] = A[r][c] - f * A[col][c];
        B[r][c] = B[r][c] - f * B[col][c];
      }
    }
  }
  for (int r = 0; r < 3; ++r)
    for (int c = 0; c < 3; ++c) pinv[(long long)(3 * r + c) * g.NM + mn] = B[r][c];
}

hipError_t launch_precond_build(const Geo& g, const zd* rho_d, const zd* T, const zd* rho_n,
                                const zd* diag, zd* pinv, hipStream_t st) {
  const int blk = 128;
  hipLaunchKernelGGL(k_precond_build, dim3((g.NM + blk - 1) / blk), dim3(blk), 0, st, g, rho_d,
                     T, rho_n, diag, pinv);
  return hipGetLastError();
}

// out[0] = min over v[0..n) of non-negative values: block minima combined by an atomic
// minimum on the IEEE bit patterns (which order like the values for non-negative doubles);
// out[0] starts as a large positive value.
__global__ void k_min(const double* __restrict__ v, long long n, double* __restrict__ out) {
  __shared__ double red[256];
  double m = 1e300;
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x)
    m = fmin(m, v[i]);
  red[threadIdx.x] = m;
  __syncthreads();
  for (int s = blockDim.x / 2; s > 0; s >>= 1) {
    if (threadIdx.x < s) red[threadIdx.x] = fmin(red[threadIdx.x], red[threadIdx.x + s]);
    __syncthreads();
  }
  if (threadIdx.x == 0)
    atomicMin(reinterpret_cast<unsigned long long*>(out),
              (unsigned long long)__double_as_longlong(red[0]));
}

hipError_t launch_min(const double* v, long long n, double* out, hipStream_t st) {
  hipError_t e = hipMemsetAsync(out, 0x7f, sizeof(double), st);
  if (e != hipSuccess) return e;
  const long long blocks = std::min<long long>(1024, (n + 255) / 256);
  hipLaunchKernelGGL(k_min, dim3((unsigned)std::max<long long>(blocks, 1)), dim3(256), 0, st, v,
                     n, out);
  return hipGetLastError();
}

}  // namespace cav
