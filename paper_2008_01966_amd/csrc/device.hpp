// Device-side building blocks shared by the cavity kernels: complex arithmetic on
// interleaved (re, im) pairs.
#pragma once

#include <hip/hip_runtime.h>

// Dynamic LDS of a kernel, sized at launch.
#ifndef CAV_DYN_SMEM
#define CAV_DYN_SMEM(name) extern __shared__ __align__(16) unsigned char name[]
#endif

namespace cav {

// Aligned to its size, so that a complex value moves as one 8- or 16-byte access (LDS
// ds_read_b64 / ds_read_b128 rather than two half-width accesses).
template <typename R>
struct alignas(2 * sizeof(R)) cx {
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
typedef cx<float> zf;

template <typename T>
__host__ __device__ inline cx<T> cvt(zd a) { return cx<T>{(T)a.re, (T)a.im}; }
template <typename T>
__host__ __device__ inline zd widen(cx<T> a) { return zd{(double)a.re, (double)a.im}; }

// Quotient and remainder by a runtime divisor d from a float reciprocal: (w + 1/2) / d lies
// at least 1/(2 d) from an integer and the float rounding error is below (w + d) 2^-23 / d,
// so the quotient is exact while w + d < 2^22 (a few instructions instead of an integer
// division in the load and store loops of the transform kernels).
struct DivBy {
  int d;
  float inv;
  __device__ explicit DivBy(int dd) : d(dd), inv(1.0f / (float)dd) {}
  __device__ int quot(int w) const { return (int)(((float)w + 0.5f) * inv); }
};

struct BlockId {
  int x, y, z;
};

// Logical block index of a 3D grid, renumbered so that each of the 8 XCDs (which receive
// workgroups round-robin in linear dispatch order) runs one contiguous range of logical
// blocks: neighbouring strips of an array then meet in the same L2.
__device__ inline int xcd_logical() {
  const int gx = gridDim.x, gy = gridDim.y;
  const int G = gx * gy * gridDim.z;
  const int lin = blockIdx.x + gx * (blockIdx.y + gy * blockIdx.z);
  const int q = G >> 3, r = G & 7, x = lin & 7;
  return x * q + (x < r ? x : r) + (lin >> 3);
}

// Logical order with x fastest.
__device__ inline BlockId xcd_block() {
  const int gx = gridDim.x, gy = gridDim.y;
  const int l = xcd_logical();
  return BlockId{l % gx, (l / gx) % gy, l / (gx * gy)};
}

// Same ranges, with y and z running fastest: the blocks that share x (the same strip of a
// table every (y, z) reads) run on one XCD, next to each other in dispatch order.
__device__ inline BlockId xcd_block_x_slow() {
  const int gy = gridDim.y, gyz = gridDim.y * gridDim.z;
  const int l = xcd_logical();
  const int x = l / gyz, t = l - x * gyz;
  return BlockId{x, t % gy, t / gy};
}

// Strips in groups of W: the W x (y, z) blocks of a group run next to each other on one
// XCD, x fastest within the group.  A kernel whose blocks each own a strip narrower than a
// cache line (W strips per line) then has the W sharers of a line in flight together, so
// the line is fetched from (and written back to) memory once, while the blocks that share
// a strip's table entries still sit within W (y, z) rows of each other.  The last group
// holds the gridDim.x mod W strips left over when W does not divide gridDim.x.
__device__ inline BlockId xcd_block_x_grouped(int W) {
  const int gx = gridDim.x, gy = gridDim.y, gyz = gridDim.y * gridDim.z;
  const int l = xcd_logical();
  const int span = W * gyz;
  const int sg = l / span;
  const int w = min(W, gx - sg * W);
  const int t = l - sg * span;
  const int yz = t / w;
  return BlockId{sg * W + (t - yz * w), yz % gy, yz / gy};
}

}  // namespace cav
