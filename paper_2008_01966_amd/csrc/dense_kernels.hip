// Direct solve of the reduced aperture system for small cavities.  The paper builds the
// aperture matrix explicitly (Step 1 of its algorithm summary, Section 6) and solves it by
// Gaussian elimination (Step 3); here the matrix is assembled column by column from the
// matrix-free operator (the same TBC convolutions and local 3x3 blocks the iterative path
// applies), inverted once per plan by Gauss-Jordan elimination with partial pivoting, and
// every later right-hand side costs one matrix-vector product with the inverse.
//
// Storage: n x n complex matrices column-major, element (i, j) at A[j * n + i], with
// n = 3 NM (the padded aperture vector; entries of absent modes carry an identity row and
// column so the matrix is nonsingular and those entries of the solution stay zero).
#include <hip/hip_runtime.h>

#include "device.hpp"
#include "kernels.hpp"

namespace cav {

// Matrix-core complex product of the spectral-operator kernels (x_r = F p_r, F column-major).
hipError_t launch_dense_product(const zd* F, long long n, const zd* p, int nb, zd* x,
                                hipStream_t st);

// x[r * n + i] = (i == k0 + r), r < nb: columns k0 .. k0 + nb - 1 of the identity.
__global__ void k_unit_vectors(long long n, long long k0, int nb, zd* __restrict__ x) {
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (long long)nb * n) return;
  const long long r = t / n, i = t - r * n;
  x[t] = mk(i == k0 + r ? 1.0 : 0.0, 0.0);
}

hipError_t launch_unit_vectors(long long n, long long k0, int nb, zd* x, hipStream_t st) {
  const long long tot = (long long)nb * n;
  hipLaunchKernelGGL(k_unit_vectors, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st, n,
                     k0, nb, x);
  return hipGetLastError();
}

// Unit diagonal on the entries of absent modes: E1 needs n >= 1, E2 m >= 1, E3 both.
__global__ void k_dense_fix(Geo g, zd* __restrict__ A) {
  const int mn = blockIdx.x * blockDim.x + threadIdx.x;
  if (mn >= g.NM) return;
  const int m = mn / (g.N + 1), nn = mn % (g.N + 1);
  const long long n = 3LL * g.NM;
  const bool absent[3] = {nn == 0, m == 0, m == 0 || nn == 0};
  for (int c = 0; c < 3; ++c)
    if (absent[c]) {
      const long long d = (long long)c * g.NM + mn;
      A[d * n + d] = mk(1.0, 0.0);
    }
}

hipError_t launch_dense_fix(const Geo& g, zd* A, hipStream_t st) {
  hipLaunchKernelGGL(k_dense_fix, dim3((g.NM + 255) / 256), dim3(256), 0, st, g, A);
  return hipGetLastError();
}

// Block-wide choice of the candidate (value v, row i) with the largest v (ties: the lowest
// row; i < 0 marks no candidate).  Same result in every thread; deterministic order.
__device__ int block_argmax(double v, int i) {
  __shared__ double sv[256];
  __shared__ int si[256];
  sv[threadIdx.x] = v;
  si[threadIdx.x] = i;
  __syncthreads();
  for (int s = blockDim.x / 2; s > 0; s >>= 1) {
    if (threadIdx.x < s) {
      const double v2 = sv[threadIdx.x + s];
      const int i2 = si[threadIdx.x + s];
      const int i1 = si[threadIdx.x];
      if (i2 >= 0 && (i1 < 0 || v2 > sv[threadIdx.x] || (v2 == sv[threadIdx.x] && i2 < i1))) {
        sv[threadIdx.x] = v2;
        si[threadIdx.x] = i2;
      }
    }
    __syncthreads();
  }
  const int r = si[0];
  __syncthreads();
  return r;
}

// Per-thread part of the pivot search: keep the larger |a|^2 (strictly, so the first of
// equal values in this thread's increasing rows wins; zero and NaN never qualify).
__device__ inline void pivot_candidate(zd a, long long i, double* best, int* bi) {
  const double v = cabs2(a);
  if (v > *best) {
    *best = v;
    *bi = (int)i;
  }
}

__global__ __launch_bounds__(256) void k_gj_pivot0(const zd* __restrict__ A, long long n,
                                                   int* __restrict__ piv) {
  double best = 0.0;
  int bi = -1;
  for (long long i = threadIdx.x; i < n; i += blockDim.x) pivot_candidate(A[i], i, &best, &bi);
  const int p = block_argmax(best, bi);
  if (threadIdx.x == 0) piv[0] = p;
}

// Gauss-Jordan step k (in-place inversion scheme, double-buffered): rows k and p = piv[k]
// of src are exchanged, then with a = src after the exchange and d = a_kk,
//   dst_kk = 1/d,  dst_kj = a_kj / d,  dst_ik = -a_ik / d,  dst_ij = a_ij - a_ik a_kj / d.
// Block j computes column j; block k+1 also picks the pivot of step k+1 among the rows
// k+1 .. n-1 of its new column.  After n steps dst holds (P A)^{-1}, P the product of the
// row exchanges, so A^{-1} b = dst (P b).  A pivot of -1 (no nonzero candidate) turns this
// and every later step into no-ops.
__global__ __launch_bounds__(256) void k_gj_step(const zd* __restrict__ src, zd* __restrict__ dst,
                                                 long long n, int k, int* __restrict__ piv) {
  const int j = blockIdx.x;
  const int p = piv[k];
  if (p < k || p >= n) return;
  const zd* ck = src + (long long)k * n;   // column k
  const zd* cj = src + (long long)j * n;   // column j
  zd* out = dst + (long long)j * n;
  const zd d = ck[p];
  const double q = 1.0 / cabs2(d);
  const zd dinv = mk(d.re * q, -d.im * q);
  const bool next = j == k + 1;
  double best = 0.0;
  int bi = -1;
  if (j == k) {
    for (long long i = threadIdx.x; i < n; i += blockDim.x) {
      const long long si = i == k ? p : (i == p ? k : i);
      out[i] = i == k ? dinv : (-1.0) * (ck[si] * dinv);
    }
  } else {
    const zd akj = cj[p] * dinv;           // scaled pivot-row entry of column j
    for (long long i = threadIdx.x; i < n; i += blockDim.x) {
      const long long si = i == k ? p : (i == p ? k : i);
      const zd v = i == k ? akj : cj[si] - ck[si] * akj;
      out[i] = v;
      if (next && i > k) pivot_candidate(v, i, &best, &bi);
    }
  }
  if (next) {
    const int pn = block_argmax(best, bi);
    if (threadIdx.x == 0) piv[k + 1] = pn;
  }
}

hipError_t launch_gj_invert(zd* A, zd* B, long long n, int* piv, zd** result, hipStream_t st) {
  hipError_t e = hipMemsetAsync(piv, 0xff, (size_t)n * sizeof(int), st);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_gj_pivot0, dim3(1), dim3(256), 0, st, A, n, piv);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  zd* src = A;
  zd* dst = B;
  for (long long k = 0; k < n; ++k) {
    hipLaunchKernelGGL(k_gj_step, dim3((unsigned)n), dim3(256), 0, st, src, dst, n, (int)k, piv);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    zd* t = src;
    src = dst;
    dst = t;
  }
  *result = src;
  return hipSuccess;
}

// pb[r * n + i] = b[r * n + perm[i]]
__global__ void k_dense_gather(const zd* __restrict__ b, const int* __restrict__ perm,
                               long long n, int nb, zd* __restrict__ pb) {
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (long long)nb * n) return;
  const long long r = t / n, i = t - r * n;
  pb[t] = b[r * n + perm[i]];
}

// x_r = F (P b_r): gather by the row permutation, then the matrix-core product.
hipError_t launch_dense_apply(const zd* F, const int* perm, long long n, const zd* b, int nb,
                              zd* pb, zd* x, hipStream_t st) {
  const long long tot = (long long)nb * n;
  hipLaunchKernelGGL(k_dense_gather, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st, b,
                     perm, n, nb, pb);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  return launch_dense_product(F, n, pb, nb, x, st);
}

// x += y (total entries)
__global__ void k_add(zd* __restrict__ x, const zd* __restrict__ y, long long total) {
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t < total) x[t] = x[t] + y[t];
}

hipError_t launch_add(zd* x, const zd* y, long long total, hipStream_t st) {
  hipLaunchKernelGGL(k_add, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, st, x, y, total);
  return hipGetLastError();
}

}  // namespace cav
