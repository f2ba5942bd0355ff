// Small device-side linear algebra and rotation helpers.
#pragma once

#include <hip/hip_runtime.h>

#include "common.hpp"

namespace bamg {

// sin(x)/x without a division by zero (no cancellation anywhere).
__device__ __forceinline__ double sinc(double x) { return x == 0.0 ? 1.0 : sin(x) / x; }

// R(w) = I + a [w]x + b [w]x^2 with a = sin(th)/th and
// b = (1 - cos th)/th^2 = 1/2 (sin(th/2)/(th/2))^2 (half-angle form, no cancellation).
// Also returns b (needed by the right Jacobian).
__device__ __forceinline__ void rotation(const double w[3], double R[9], double* b_out) {
  const double th = sqrt(w[0] * w[0] + w[1] * w[1] + w[2] * w[2]);
  const double a = sinc(th);
  const double h = sinc(0.5 * th);
  const double b = 0.5 * h * h;
  const double xx = w[0] * w[0], yy = w[1] * w[1], zz = w[2] * w[2];
  const double xy = w[0] * w[1], xz = w[0] * w[2], yz = w[1] * w[2];
  // [w]x^2 = w w^T - th^2 I
  R[0] = 1.0 + b * (-yy - zz);
  R[1] = -a * w[2] + b * xy;
  R[2] = a * w[1] + b * xz;
  R[3] = a * w[2] + b * xy;
  R[4] = 1.0 + b * (-xx - zz);
  R[5] = -a * w[0] + b * yz;
  R[6] = -a * w[1] + b * xz;
  R[7] = a * w[0] + b * yz;
  R[8] = 1.0 + b * (-xx - yy);
  if (b_out) *b_out = b;
}

// Right Jacobian of SO(3): R(w + d) = R(w) exp([J_r(w) d]x) + O(d^2),
// J_r = I - b [w]x + c [w]x^2, b = (1 - cos th)/th^2, c = (th - sin th)/th^3.
// Then d(R X)/dw = -R [X]x J_r.
__device__ __forceinline__ void right_jacobian(const double w[3], double b, double J[9]) {
  const double t2 = w[0] * w[0] + w[1] * w[1] + w[2] * w[2];
  const double th = sqrt(t2);
  double c;
  if (th < 0.25) {
    // sum_n (-1)^n th^2n / (2n+3)!
    c = 1.0 / 6.0 + t2 * (-1.0 / 120.0 + t2 * (1.0 / 5040.0 + t2 * (-1.0 / 362880.0 + t2 * (1.0 / 39916800.0))));
  } else {
    c = (th - sin(th)) / (t2 * th);
  }
  const double xx = w[0] * w[0], yy = w[1] * w[1], zz = w[2] * w[2];
  const double xy = w[0] * w[1], xz = w[0] * w[2], yz = w[1] * w[2];
  J[0] = 1.0 + c * (-yy - zz);
  J[1] = b * w[2] + c * xy;
  J[2] = -b * w[1] + c * xz;
  J[3] = -b * w[2] + c * xy;
  J[4] = 1.0 + c * (-xx - zz);
  J[5] = b * w[0] + c * yz;
  J[6] = b * w[1] + c * xz;
  J[7] = -b * w[0] + c * yz;
  J[8] = 1.0 + c * (-xx - yy);
}

// Inverse right Jacobian: J_r^-1 = I + 1/2 [w]x + e [w]x^2,
// e = 1/th^2 - cot(th/2) / (2 th); series 1/12 + th^2/720 + th^4/30240 + ... near 0.
__device__ __forceinline__ void right_jacobian_inv(const double w[3], double J[9]) {
  const double t2 = w[0] * w[0] + w[1] * w[1] + w[2] * w[2];
  const double th = sqrt(t2);
  double e;
  if (th < 0.25) {
    e = 1.0 / 12.0 + t2 * (1.0 / 720.0 + t2 * (1.0 / 30240.0 + t2 * (1.0 / 1209600.0 + t2 * (1.0 / 47900160.0))));
  } else {
    const double hh = 0.5 * th;
    e = 1.0 / t2 - cos(hh) / (2.0 * th * sin(hh));
  }
  const double xx = w[0] * w[0], yy = w[1] * w[1], zz = w[2] * w[2];
  const double xy = w[0] * w[1], xz = w[0] * w[2], yz = w[1] * w[2];
  J[0] = 1.0 + e * (-yy - zz);
  J[1] = -0.5 * w[2] + e * xy;
  J[2] = 0.5 * w[1] + e * xz;
  J[3] = 0.5 * w[2] + e * xy;
  J[4] = 1.0 + e * (-xx - zz);
  J[5] = -0.5 * w[0] + e * yz;
  J[6] = -0.5 * w[1] + e * xz;
  J[7] = 0.5 * w[0] + e * yz;
  J[8] = 1.0 + e * (-xx - yy);
}

// In-place Cholesky of an n x n SPD matrix held row-major in `a` (lower factor
// written to the lower triangle). Returns false if a pivot is <= 0 or not finite.
template <int N, class T>
__device__ __forceinline__ bool cholesky(T* a) {
  for (int j = 0; j < N; ++j) {
    T d = a[j * N + j];
    for (int k = 0; k < j; ++k) d -= a[j * N + k] * a[j * N + k];
    if (!(d > T(0))) return false;
    const T l = sqrt(d);
    a[j * N + j] = l;
    const T il = T(1) / l;
    for (int i = j + 1; i < N; ++i) {
      T s = a[i * N + j];
      for (int k = 0; k < j; ++k) s -= a[i * N + k] * a[j * N + k];
      a[i * N + j] = s * il;
    }
  }
  return true;
}

// Inverse of an SPD matrix from its Cholesky factor L (lower triangle of a):
// inv = L^-T L^-1, written to `out` (full, row-major). `a` is destroyed.
template <int N, class T>
__device__ __forceinline__ void cholesky_inverse(T* a, T* out) {
  // invert L in place (lower triangle)
  for (int j = 0; j < N; ++j) {
    a[j * N + j] = T(1) / a[j * N + j];
    for (int i = j + 1; i < N; ++i) {
      T s = 0;
      for (int k = j; k < i; ++k) s -= a[i * N + k] * a[k * N + j];
      a[i * N + j] = s / a[i * N + i];
    }
  }
  // out = Linv^T Linv
  for (int i = 0; i < N; ++i)
    for (int j = 0; j <= i; ++j) {
      T s = 0;
      for (int k = i; k < N; ++k) s += a[k * N + i] * a[k * N + j];
      out[i * N + j] = s;
      out[j * N + i] = s;
    }
}

// Wave-wide sum (64 lanes).
// Workgroups are dealt round-robin to the 8 XCDs of the chip (each with its
// own L2). For a grid of 8 ceil(n / 8) workgroups over n work items whose
// neighbours share data, map workgroup b to item (b % 8) ceil(n / 8) + b / 8:
// every XCD then works through one contiguous range. Items >= n are idle.
__device__ __forceinline__ int xcd_block(int b, int n) {
  const int per = (n + 7) / 8;
  return (b % 8) * per + b / 8;
}
__host__ __device__ constexpr int xcd_grid(int n) { return (n + 7) / 8 * 8; }

template <class T>
__device__ __forceinline__ T wave_sum(T v) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// One halving step of a wave reduce-scatter: lanes whose `off` bit is set keep
// the upper half of v[0 .. 2H), the others the lower half, each adding the
// partner lane's copy of the half it keeps.
template <int H>
__device__ __forceinline__ void reduce_scatter_step(double* v, int off, bool upper) {
#pragma unroll
  for (int k = 0; k < H; ++k) {
    const double send = upper ? v[k] : v[H + k];
    const double keep = upper ? v[H + k] : v[k];
    v[k] = keep + __shfl_xor(send, off, 64);
  }
}

// Sums N = 32 m per-lane values over the 64 lanes of a wave with 63 m / 2
// exchanges (instead of 6 N for N separate butterflies). On return lane l holds
// in v[0 .. m) the wave totals of entries m (l >> 1) .. m (l >> 1) + m - 1
// (both lanes of a pair hold the same totals).
template <int N>
__device__ __forceinline__ void wave_reduce_scatter(double (&v)[N]) {
  static_assert(N % 32 == 0, "N must be a multiple of 32");
  const int lane = threadIdx.x & 63;
  reduce_scatter_step<N / 2>(v, 32, lane & 32);
  reduce_scatter_step<N / 4>(v, 16, lane & 16);
  reduce_scatter_step<N / 8>(v, 8, lane & 8);
  reduce_scatter_step<N / 16>(v, 4, lane & 4);
  reduce_scatter_step<N / 32>(v, 2, lane & 2);
#pragma unroll
  for (int k = 0; k < N / 32; ++k) v[k] += __shfl_xor(v[k], 1, 64);
}

}  // namespace bamg
