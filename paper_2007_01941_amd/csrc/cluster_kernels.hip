// Visibility-based block Jacobi (the comparison preconditioner of Section 2.2):
// the inverse of the block-diagonal part of S over clusters of cameras, the
// clusters being the level-0 aggregates of Algorithm 2. Each cluster of m
// cameras holds a dense n x n block (n = 9m, row-major) at off[a] in one
// array: gathered from the explicit level-0 S, inverted in place, applied as a
// dense product per cluster.
#include "kernels.hpp"

namespace bamg {

// Block (i, j) of the level-0 BSR operator, or -1 when i and j share no point.
__device__ __forceinline__ int bsr_find(const int32_t* __restrict__ rowptr, const int32_t* __restrict__ col,
                                        int i, int j) {
  int lo = rowptr[i], hi = rowptr[i + 1];
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    const int c = col[mid];
    if (c == j) return mid;
    if (c < j) lo = mid + 1;
    else hi = mid;
  }
  return -1;
}

// One workgroup per cluster: out[off[a] + (9 p + r) n + 9 q + c] = S0(i_p, i_q)[r][c]
// for the cluster's members i_0 < i_1 < ... (zero where the cameras share no point).
__global__ __launch_bounds__(256) void k_cj_gather(const int32_t* __restrict__ agg_ptr,
                                                   const int32_t* __restrict__ agg_mem,
                                                   const int32_t* __restrict__ rowptr,
                                                   const int32_t* __restrict__ col, const double* __restrict__ S,
                                                   const int64_t* __restrict__ off, double* __restrict__ out) {
  const int a = blockIdx.x;
  const int beg = agg_ptr[a], m = agg_ptr[a + 1] - beg, n = 9 * m;
  double* blk = out + off[a];
  for (int t = threadIdx.x; t < m * m * 81; t += blockDim.x) {
    const int pair = t / 81, e = t - pair * 81;
    const int p = pair / m, q = pair - p * m;
    const int r = e / 9, c = e - r * 9;
    const int pos = bsr_find(rowptr, col, agg_mem[beg + p], agg_mem[beg + q]);
    blk[(size_t)(9 * p + r) * n + 9 * q + c] = pos >= 0 ? S[(size_t)pos * 81 + r * 9 + c] : 0.0;
  }
}

// In-place Gauss-Jordan inversion of every cluster's SPD block (no pivoting:
// the pivots of an SPD matrix stay positive). Step k:
//   a_ij -= a_ik a_kj / p (i, j != k);  a_kj /= p;  a_ik = -a_ik / p;  a_kk = 1 / p.
// The first phase reads only row and column k, which it does not write.
__global__ __launch_bounds__(256) void k_cj_invert(const int32_t* __restrict__ agg_ptr,
                                                   const int64_t* __restrict__ off, double* __restrict__ inv,
                                                   uint32_t* err) {
  const int a = blockIdx.x;
  const int n = 9 * (agg_ptr[a + 1] - agg_ptr[a]);
  double* A = inv + off[a];
  for (int k = 0; k < n; ++k) {
    double piv = A[(size_t)k * n + k];
    if (!(piv > 0.0)) {
      if (threadIdx.x == 0) atomicOr(err, ERRF_NOT_SPD);
      piv = 1.0;   // keep going; the step reports the failure
    }
    for (int t = threadIdx.x; t < n * n; t += blockDim.x) {
      const int i = t / n, j = t - i * n;
      if (i != k && j != k) A[t] -= A[(size_t)i * n + k] * A[(size_t)k * n + j] / piv;
    }
    __syncthreads();
    for (int t = threadIdx.x; t < n; t += blockDim.x) {
      if (t != k) {
        A[(size_t)k * n + t] /= piv;
        A[(size_t)t * n + k] = -A[(size_t)t * n + k] / piv;
      }
    }
    __syncthreads();
    if (threadIdx.x == 0) A[(size_t)k * n + k] = 1.0 / piv;
    __syncthreads();
  }
}

// z = M^-1 r: per cluster, gather r of the members into LDS (n doubles of
// dynamic shared memory) and multiply by the cluster's inverse.
__global__ __launch_bounds__(256) void k_cj_apply(const int32_t* __restrict__ agg_ptr,
                                                  const int32_t* __restrict__ agg_mem,
                                                  const int64_t* __restrict__ off,
                                                  const double* __restrict__ inv, const double* __restrict__ r,
                                                  double* __restrict__ z, const int* done) {
  if (done && *done) return;
  extern __shared__ double rs[];
  const int a = blockIdx.x;
  const int beg = agg_ptr[a], n = 9 * (agg_ptr[a + 1] - beg);
  for (int t = threadIdx.x; t < n; t += blockDim.x) rs[t] = r[(size_t)9 * agg_mem[beg + t / 9] + t % 9];
  __syncthreads();
  const double* A = inv + off[a];
  for (int i = threadIdx.x; i < n; i += blockDim.x) {
    const double* row = A + (size_t)i * n;
    double acc = 0.0;
    for (int j = 0; j < n; ++j) acc += row[j] * rs[j];
    z[(size_t)9 * agg_mem[beg + i / 9] + i % 9] = acc;
  }
}

}  // namespace bamg
