// The implicit Schur product y = S x = A x - F^T E C^-1 E^T F x (Section 3.6 of
// Konolige and Brown, "Multigrid for Bundle Adjustment"): the operator of PCG
// and, when selected, of level-0 smoothing. Observation planes are point-major
// (see step_kernels.hip for the layout).
#include "kernels.hpp"

namespace bamg {

// ---------------------------------------------------------------- implicit Schur product

// y_c = A_c x_c (packed symmetric A), one thread per (camera, row).
template <class T>
__global__ __launch_bounds__(256) void k_apply_A(int n_cam, const T* __restrict__ A,
                                                 const T* __restrict__ x, T* __restrict__ y) {
  const int gid = blockIdx.x * 252 + threadIdx.x;
  const int c = gid / 9, i = gid % 9;
  if (threadIdx.x >= 252 || c >= n_cam) return;
  const T* a = A + (size_t)c * 45;
  const T* xv = x + (size_t)c * 9;
  T s = 0;
#pragma unroll
  for (int j = 0; j < 9; ++j) s += a[i <= j ? sym_index(9, i, j) : sym_index(9, j, i)] * xv[j];
  y[(size_t)c * 9 + i] = s;
}

// y -= F^T E C^-1 E^T F x, one workgroup per tile of <= TILE_OBS observations
// belonging to whole points. Camera vectors of the tile's cameras are staged
// in LDS (x) and accumulated in LDS (y) before one global atomic add per
// (tile, camera, component); point sums E^T F x are accumulated in LDS.
template <class T>
__global__ __launch_bounds__(256) void k_schur_tiles(
    const int32_t* __restrict__ tile_obs, const int32_t* __restrict__ tile_pt,
    const int32_t* __restrict__ tile_coff, const int32_t* __restrict__ tile_cams,
    const uint32_t* __restrict__ obs_slot, const T* __restrict__ F, const T* __restrict__ E,
    int64_t stride, const T* __restrict__ Cinv, const T* __restrict__ x, T* __restrict__ y,
    const int* __restrict__ done) {
  if (done && *done) return;
  __shared__ T xs[TILE_SLOTS * 9];
  __shared__ T ys[TILE_SLOTS * 9];
  __shared__ T zs[(TILE_OBS / 2) * 3];
  const int t = blockIdx.x;
  const int o0 = tile_obs[t], o1 = tile_obs[t + 1];
  const int q0 = tile_pt[t], np = tile_pt[t + 1] - q0;
  const int c0 = tile_coff[t], nc = tile_coff[t + 1] - c0;
  const int ncs = nc < TILE_SLOTS ? nc : TILE_SLOTS;
  for (int i = threadIdx.x; i < ncs * 9; i += 256) {
    const int s = i / 9, k = i - s * 9;
    xs[i] = x[(size_t)tile_cams[c0 + s] * 9 + k];
    ys[i] = T(0);
  }
  for (int i = threadIdx.x; i < np * 3; i += 256) zs[i] = T(0);
  __syncthreads();

  const int o = o0 + threadIdx.x;
  const bool act = o < o1;
  T f[18], e[6];
  int slot = 0, pl = 0;
  if (act) {
#pragma unroll
    for (int k = 0; k < 18; ++k) f[k] = F[k * stride + o];
#pragma unroll
    for (int k = 0; k < 6; ++k) e[k] = E[k * stride + o];
    const uint32_t w = obs_slot[o];
    slot = (int)(w & 0xffffu);
    pl = (int)(w >> 16);
    const T* xv = slot < TILE_SLOTS ? &xs[slot * 9] : &x[(size_t)tile_cams[c0 + slot] * 9];
    T s0 = 0, s1 = 0;
#pragma unroll
    for (int k = 0; k < 9; ++k) { s0 += f[k] * xv[k]; s1 += f[9 + k] * xv[k]; }
#pragma unroll
    for (int k = 0; k < 3; ++k) atomicAdd(&zs[pl * 3 + k], e[k] * s0 + e[3 + k] * s1);
  }
  // observations beyond one per thread (only a single point with > TILE_OBS views)
  for (int oo = o0 + 256 + threadIdx.x; oo < o1; oo += 256) {
    const uint32_t w = obs_slot[oo];
    const int sl = (int)(w & 0xffffu), pq = (int)(w >> 16);
    const T* xv = sl < TILE_SLOTS ? &xs[sl * 9] : &x[(size_t)tile_cams[c0 + sl] * 9];
    T s0 = 0, s1 = 0;
    for (int k = 0; k < 9; ++k) { s0 += F[k * stride + oo] * xv[k]; s1 += F[(9 + k) * stride + oo] * xv[k]; }
    for (int k = 0; k < 3; ++k) atomicAdd(&zs[pq * 3 + k], E[k * stride + oo] * s0 + E[(3 + k) * stride + oo] * s1);
  }
  __syncthreads();
  for (int i = threadIdx.x; i < np; i += 256) {
    const T* ci = Cinv + (size_t)(q0 + i) * 6;
    const T z0 = zs[i * 3], z1 = zs[i * 3 + 1], z2 = zs[i * 3 + 2];
    zs[i * 3 + 0] = ci[0] * z0 + ci[1] * z1 + ci[2] * z2;
    zs[i * 3 + 1] = ci[1] * z0 + ci[3] * z1 + ci[4] * z2;
    zs[i * 3 + 2] = ci[2] * z0 + ci[4] * z1 + ci[5] * z2;
  }
  __syncthreads();
  if (act) {
    const T u0 = zs[pl * 3], u1 = zs[pl * 3 + 1], u2 = zs[pl * 3 + 2];
    const T w0 = e[0] * u0 + e[1] * u1 + e[2] * u2;
    const T w1 = e[3] * u0 + e[4] * u1 + e[5] * u2;
    if (slot < TILE_SLOTS) {
#pragma unroll
      for (int k = 0; k < 9; ++k) atomicAdd(&ys[slot * 9 + k], -(f[k] * w0 + f[9 + k] * w1));
    } else {
      T* yv = y + (size_t)tile_cams[c0 + slot] * 9;
#pragma unroll
      for (int k = 0; k < 9; ++k) unsafeAtomicAdd(&yv[k], -(f[k] * w0 + f[9 + k] * w1));
    }
  }
  for (int oo = o0 + 256 + threadIdx.x; oo < o1; oo += 256) {
    const uint32_t w = obs_slot[oo];
    const int sl = (int)(w & 0xffffu), pq = (int)(w >> 16);
    const T u0 = zs[pq * 3], u1 = zs[pq * 3 + 1], u2 = zs[pq * 3 + 2];
    const T w0 = E[0 * stride + oo] * u0 + E[1 * stride + oo] * u1 + E[2 * stride + oo] * u2;
    const T w1 = E[3 * stride + oo] * u0 + E[4 * stride + oo] * u1 + E[5 * stride + oo] * u2;
    for (int k = 0; k < 9; ++k) {
      const T v = -(F[k * stride + oo] * w0 + F[(9 + k) * stride + oo] * w1);
      if (sl < TILE_SLOTS) atomicAdd(&ys[sl * 9 + k], v);
      else unsafeAtomicAdd(&y[(size_t)tile_cams[c0 + sl] * 9 + k], v);
    }
  }
  __syncthreads();
  for (int i = threadIdx.x; i < ncs * 9; i += 256) {
    const int s = i / 9, k = i - s * 9;
    unsafeAtomicAdd(&y[(size_t)tile_cams[c0 + s] * 9 + k], ys[i]);
  }
}

template __global__ void k_schur_tiles<double>(const int32_t*, const int32_t*, const int32_t*,
                                               const int32_t*, const uint32_t*, const double*,
                                               const double*, int64_t, const double*, const double*,
                                               double*, const int*);
template __global__ void k_schur_tiles<float>(const int32_t*, const int32_t*, const int32_t*,
                                              const int32_t*, const uint32_t*, const float*,
                                              const float*, int64_t, const float*, const float*,
                                              float*, const int*);
template __global__ void k_apply_A<double>(int, const double*, const double*, double*);
template __global__ void k_apply_A<float>(int, const float*, const float*, float*);

}  // namespace bamg
