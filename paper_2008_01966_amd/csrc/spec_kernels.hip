// Spectral discrete TBC operator (D_spec): the single-layer operators with the exact
// Fourier transforms of the trial functions on the kernel-spectrum lattice (Section 5.2,
// with the outer integral's transform in closed form as well):
//   (S^f c) = (1/(L1 L2)) F1^H [ K^ .* (F1 c F2^T) ] conj(F2),
// F1[j1][m] = int_0^a psi_m(x) e^{-i xi_j1 x} dx (cos or sin by family), F2 likewise along
// y.  Four batched complex matrix products per family and right-hand side; the products
// run in double precision in both precision modes of the solver.
#include <hip/hip_runtime.h>

#include "device.hpp"
#include "kernels.hpp"

namespace cav {

// Tiled complex matrix product over a batch b = rhs * nf + slot:
//   C_b(i, j) = sum_k opA_b(i, k) opB_b(k, j)  [ * khat(i, j) * kscale when khat is set ]
// Each operand is addressed by strides (element (i, k) at base + i si + k sk), with a base
// per family (F matrices) or per slot and right-hand side (data), and an optional conjugate.
struct SpecOperand {
  const zd* base[3];   // by family f
  long long sr;        // stride per right-hand side
  long long ss;        // stride per slot
  long long si, sk;    // element strides
  int conj;
};
struct SpecOut {
  zd* base;
  long long sr, ss, si, sj;
};

constexpr int kSpecT = 32;    // output tile (kSpecT x kSpecT per block)
constexpr int kSpecK = 16;    // depth of one staged slice

__global__ __launch_bounds__(256) void k_spec_gemm(int rows, int cols, int depth, int nf,
                                                   int fam_fixed, SpecOperand A, SpecOperand B,
                                                   SpecOut C, const zd* __restrict__ khat,
                                                   long long khat_si, double kscale,
                                                   const int* __restrict__ active) {
  __shared__ zd As[kSpecT][kSpecK + 1];
  __shared__ zd Bs[kSpecK][kSpecT + 1];
  const int b = blockIdx.z;
  const int rhs = b / nf, slot = b - rhs * nf;
  if (active && !active[rhs]) return;
  const int f = fam_fixed >= 0 ? fam_fixed : slot;
  const zd* pa = A.base[f] + rhs * A.sr + slot * A.ss;
  const zd* pb = B.base[f] + rhs * B.sr + slot * B.ss;
  const int i0 = blockIdx.y * kSpecT, j0 = blockIdx.x * kSpecT;
  const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
  zd acc[2][2];
  for (int u = 0; u < 2; ++u)
    for (int v = 0; v < 2; ++v) acc[u][v] = mk(0.0, 0.0);
  for (int k0 = 0; k0 < depth; k0 += kSpecK) {
    for (int e = threadIdx.x; e < kSpecT * kSpecK; e += blockDim.x) {
      const int ii = e / kSpecK, kk = e - ii * kSpecK;
      const int i = i0 + ii, k = k0 + kk;
      zd va = mk(0.0, 0.0);
      if (i < rows && k < depth) {
        va = pa[i * A.si + k * A.sk];
        if (A.conj) va = conj(va);
      }
      As[ii][kk] = va;
    }
    for (int e = threadIdx.x; e < kSpecK * kSpecT; e += blockDim.x) {
      const int kk = e / kSpecT, jj = e - kk * kSpecT;
      const int k = k0 + kk, j = j0 + jj;
      zd vb = mk(0.0, 0.0);
      if (k < depth && j < cols) {
        vb = pb[k * B.si + j * B.sk];
        if (B.conj) vb = conj(vb);
      }
      Bs[kk][jj] = vb;
    }
    __syncthreads();
#pragma unroll 4
    for (int kk = 0; kk < kSpecK; ++kk) {
      const zd a0 = As[ty][kk], a1 = As[ty + 16][kk];
      const zd b0 = Bs[kk][tx], b1 = Bs[kk][tx + 16];
      acc[0][0] = acc[0][0] + a0 * b0;
      acc[0][1] = acc[0][1] + a0 * b1;
      acc[1][0] = acc[1][0] + a1 * b0;
      acc[1][1] = acc[1][1] + a1 * b1;
    }
    __syncthreads();
  }
  zd* pc = C.base + rhs * C.sr + slot * C.ss;
  for (int u = 0; u < 2; ++u)
    for (int v = 0; v < 2; ++v) {
      const int i = i0 + ty + 16 * u, j = j0 + tx + 16 * v;
      if (i >= rows || j >= cols) continue;
      zd r = acc[u][v];
      if (khat) r = kscale * (r * khat[i * khat_si + j]);
      pc[i * C.si + j * C.sj] = r;
    }
}

// The same product on the matrix cores: each wave of the block owns one 16 x 16 quarter of
// the 32 x 32 output tile and accumulates it with v_mfma_f64_16x16x4f64, four real products
// per complex step (re re - im im, re im + im re).  Operand layout of that instruction on
// gfx950 (measured): lane l gives A(l mod 16, l div 16) and B(l div 16, l mod 16) and holds
// D(l div 16 + 4 v, l mod 16) for v = 0..3.
typedef double v4d __attribute__((ext_vector_type(4)));

__global__ __launch_bounds__(256) void k_spec_gemm_mfma(int rows, int cols, int depth, int nf,
                                                        int fam_fixed, SpecOperand A,
                                                        SpecOperand B, SpecOut C,
                                                        const zd* __restrict__ khat,
                                                        long long khat_si, double kscale,
                                                        const int* __restrict__ active) {
  __shared__ zd As[kSpecT][kSpecK + 1];
  __shared__ zd Bs[kSpecK][kSpecT + 1];
  const int b = blockIdx.z;
  const int rhs = b / nf, slot = b - rhs * nf;
  if (active && !active[rhs]) return;
  const int f = fam_fixed >= 0 ? fam_fixed : slot;
  const zd* pa = A.base[f] + rhs * A.sr + slot * A.ss;
  const zd* pb = B.base[f] + rhs * B.sr + slot * B.ss;
  const int i0 = blockIdx.y * kSpecT, j0 = blockIdx.x * kSpecT;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int wi = (wave >> 1) * 16, wj = (wave & 1) * 16;
  const int lr = lane & 15, lk = lane >> 4;
  v4d cr = {0.0, 0.0, 0.0, 0.0}, ci = {0.0, 0.0, 0.0, 0.0};
  for (int k0 = 0; k0 < depth; k0 += kSpecK) {
    for (int e = threadIdx.x; e < kSpecT * kSpecK; e += blockDim.x) {
      const int ii = e / kSpecK, kk = e - ii * kSpecK;
      const int i = i0 + ii, k = k0 + kk;
      zd va = mk(0.0, 0.0);
      if (i < rows && k < depth) {
        va = pa[i * A.si + k * A.sk];
        if (A.conj) va = conj(va);
      }
      As[ii][kk] = va;
    }
    for (int e = threadIdx.x; e < kSpecK * kSpecT; e += blockDim.x) {
      const int kk = e / kSpecT, jj = e - kk * kSpecT;
      const int k = k0 + kk, j = j0 + jj;
      zd vb = mk(0.0, 0.0);
      if (k < depth && j < cols) {
        vb = pb[k * B.si + j * B.sk];
        if (B.conj) vb = conj(vb);
      }
      Bs[kk][jj] = vb;
    }
    __syncthreads();
#pragma unroll
    for (int ks = 0; ks < kSpecK; ks += 4) {
      const zd a = As[wi + lr][ks + lk];
      const zd bv = Bs[ks + lk][wj + lr];
      cr = __builtin_amdgcn_mfma_f64_16x16x4f64(a.re, bv.re, cr, 0, 0, 0);
      cr = __builtin_amdgcn_mfma_f64_16x16x4f64(-a.im, bv.im, cr, 0, 0, 0);
      ci = __builtin_amdgcn_mfma_f64_16x16x4f64(a.re, bv.im, ci, 0, 0, 0);
      ci = __builtin_amdgcn_mfma_f64_16x16x4f64(a.im, bv.re, ci, 0, 0, 0);
    }
    __syncthreads();
  }
  zd* pc = C.base + rhs * C.sr + slot * C.ss;
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const int i = i0 + wi + lk + 4 * v, j = j0 + wj + lr;
    if (i >= rows || j >= cols) continue;
    zd r = mk(cr[v], ci[v]);
    if (khat) r = kscale * (r * khat[i * khat_si + j]);
    pc[i * C.si + j * C.sj] = r;
  }
}

static hipError_t spec_gemm(int rows, int cols, int depth, int nb, int nf, int fam_fixed,
                            const SpecOperand& A, const SpecOperand& B, const SpecOut& C,
                            const zd* khat, long long khat_si, double kscale,
                            const int* active, hipStream_t st) {
  static const bool mfma = [] {
    const char* e = getenv("CAVITY_SPEC_MFMA");
    return !(e && atoi(e) == 0);
  }();
  const dim3 grid((cols + kSpecT - 1) / kSpecT, (rows + kSpecT - 1) / kSpecT, nb * nf);
  if (mfma)
    hipLaunchKernelGGL(k_spec_gemm_mfma, grid, dim3(256), 0, st, rows, cols, depth, nf, fam_fixed,
                       A, B, C, khat, khat_si, kscale, active);
  else
    hipLaunchKernelGGL(k_spec_gemm, grid, dim3(256), 0, st, rows, cols, depth, nf, fam_fixed, A,
                       B, C, khat, khat_si, kscale, active);
  return hipGetLastError();
}

// x_r = F p_r for r < nb, with F column-major n x n (F[k n + i] = F(i, k)) and p, x stored
// per right-hand side (p[r n + k]): computed as X^T = P^T F^T with the same matrix-core
// product, every operand then read along its contiguous index.
hipError_t launch_dense_product(const zd* F, long long n, const zd* p, int nb, zd* x,
                                hipStream_t st) {
  const SpecOperand A{{p, p, p}, 0, 0, n, 1, 0};   // (r, k) at r n + k
  const SpecOperand B{{F, F, F}, 0, 0, n, 1, 0};   // (k, i) = F(i, k) at k n + i
  const SpecOut C{x, 0, 0, n, 1};                  // (r, i) at r n + i
  return spec_gemm(nb, (int)n, (int)n, 1, 1, 0, A, B, C, nullptr, 0, 0.0, nullptr, st);
}

// Family inputs on the mode grid: c_f = z1 (cs), z2 (sc), nu z1 - mu z2 (cc), z = P^{-1} v
// when precond, else v.  out[rhs][slot][mn].
__global__ void k_spec_input(Geo g, const zd* __restrict__ pinv, int precond, int fam_fixed,
                             const zd* __restrict__ vall, long long vs, zd* __restrict__ out,
                             const int* __restrict__ active) {
  const int rhs = blockIdx.y;
  if (active && !active[rhs]) return;
  const int mn = blockIdx.x * blockDim.x + threadIdx.x;
  if (mn >= g.NM) return;
  const zd* v = vall + rhs * vs;
  const int nf = fam_fixed >= 0 ? 1 : 3;
  zd* o = out + (long long)rhs * nf * g.NM;
  if (fam_fixed >= 0) {
    o[mn] = v[mn];
    return;
  }
  zd z[3] = {v[mn], v[g.NM + mn], v[2LL * g.NM + mn]};
  if (precond) {
    zd y[3];
    for (int r = 0; r < 3; ++r)
      y[r] = pinv[(3 * r) * (long long)g.NM + mn] * z[0] +
             pinv[(3 * r + 1) * (long long)g.NM + mn] * z[1] +
             pinv[(3 * r + 2) * (long long)g.NM + mn] * z[2];
    z[0] = y[0]; z[1] = y[1]; z[2] = y[2];
  }
  const int m = mn / (g.N + 1), n = mn - m * (g.N + 1);
  const double mu = g.pa * m, nu = g.pb * n;
  o[mn] = z[0];
  o[g.NM + mn] = z[1];
  o[2LL * g.NM + mn] = nu * z[0] - mu * z[1];
}

// The three single-layer operators (or the fixed family) of D_spec for nb right-hand
// sides: c (M+1 x N+1, in Y) -> Z = c F2^T (M+1 x P2, in X) -> U = K^ .* (F1 Z) / (L1 L2)
// (P1 x P2, in U) -> W = F1^H U (M+1 x P2, in Y) -> S = W conj(F2) (M+1 x N+1, in S).
hipError_t launch_spec_passes(const Geo& g, const SpecMats& sm, const zd* khat, const zd* pinv,
                              int precond, int fam_fixed, int nb, const zd* v, long long vs,
                              zd* X, zd* Y, zd* U, zd* S, const int* active, hipStream_t st) {
  const int nf = fam_fixed >= 0 ? 1 : 3;
  const long long NM = g.NM, M1 = g.M + 1, N1 = g.N + 1, P1 = g.P1, P2 = g.P2;
  const long long xs = M1 * P2, us = P1 * P2;
  // family f: x basis cos for cs and cc, sin for sc; y basis sin for cs, cos for sc and cc
  const zd* f1[3] = {sm.f1c, sm.f1s, sm.f1c};
  const zd* f2[3] = {sm.f2s, sm.f2c, sm.f2c};
  hipLaunchKernelGGL(k_spec_input, dim3((unsigned)((NM + 255) / 256), nb), dim3(256), 0, st, g,
                     pinv, precond, fam_fixed, v, vs, Y, active);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  // Z(m, j2) = sum_n c(m, n) F2(j2, n)          [F2 stored [j2][n]]
  SpecOperand c{{Y, Y, Y}, nf * NM, NM, N1, 1, 0};
  SpecOperand f2t{{f2[0], f2[1], f2[2]}, 0, 0, 1, N1, 0};
  SpecOut z{X, nf * xs, xs, P2, 1};
  if ((e = spec_gemm((int)M1, (int)P2, (int)N1, nb, nf, fam_fixed, c, f2t, z, nullptr, 0, 0.0,
                     active, st)) != hipSuccess)
    return e;
  // U(j1, j2) = K^(j1, j2) / (L1 L2) sum_m F1(j1, m) Z(m, j2)     [F1 stored [j1][m]]
  // (the plan stores K^ / (hq1 hq2 P1 P2) = K^ / (L1 L2), the factor is already in it)
  SpecOperand f1n{{f1[0], f1[1], f1[2]}, 0, 0, M1, 1, 0};
  SpecOperand zin{{X, X, X}, nf * xs, xs, P2, 1, 0};
  SpecOut uo{U, nf * us, us, P2, 1};
  if ((e = spec_gemm((int)P1, (int)P2, (int)M1, nb, nf, fam_fixed, f1n, zin, uo, khat, P2, 1.0,
                     active, st)) != hipSuccess)
    return e;
  // W(m, j2) = sum_j1 conj(F1(j1, m)) U(j1, j2)
  SpecOperand f1h{{f1[0], f1[1], f1[2]}, 0, 0, 1, M1, 1};
  SpecOperand uin{{U, U, U}, nf * us, us, P2, 1, 0};
  SpecOut w{Y, nf * xs, xs, P2, 1};
  if ((e = spec_gemm((int)M1, (int)P2, (int)P1, nb, nf, fam_fixed, f1h, uin, w, nullptr, 0, 0.0,
                     active, st)) != hipSuccess)
    return e;
  // S(m, n) = sum_j2 W(m, j2) conj(F2(j2, n))
  SpecOperand win{{Y, Y, Y}, nf * xs, xs, P2, 1, 0};
  SpecOperand f2c{{f2[0], f2[1], f2[2]}, 0, 0, N1, 1, 1};
  SpecOut so{S, nf * NM, NM, N1, 1};
  return spec_gemm((int)M1, (int)N1, (int)P2, nb, nf, fam_fixed, win, f2c, so, nullptr, 0, 0.0,
                   active, st);
}

}  // namespace cav
