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
// belonging to whole points (one thread per observation, coalesced plane
// reads; every load of the tile is issued before the first barrier).
//  1. s_o = F_o x_c(o) with x staged in LDS for the tile's first TILE_SLOTS
//     cameras; each thread leaves E_o^T s_o in LDS.
//  2. One thread per point adds its observations' terms in order and applies
//     C_p^-1: u_p.
//  3. The camera terms -F_o^T E_o u_p are summed per (tile, camera) in LDS and
//     added to y with one global atomic per (tile, camera, component). FP64:
//     LDS atomic adds into per-camera slots. FP32: each thread leaves its
//     terms at its observation's rank in the tile's camera-sorted order and
//     one thread per (camera, component) adds its camera's run (FP32 LDS
//     atomics contend badly when many lanes share a camera).
// A tile of more than TILE_OBS observations (a single point) adds its camera
// terms to y with global atomics directly.
//
// DET (deterministic): no floating-point atomics anywhere. Every (tile,
// camera) sum is formed by the camera-sorted runs (both precisions) and
// stored to part[(tile_coff[t] + slot) * 9 + k]; k_schur_gather then adds each
// camera's partials to y in tile order. A single-point tile has one
// observation per camera, so its terms are stored the same way.
//
// Tiles are numbered in point order, so neighbouring tiles share cameras; the
// launch maps workgroups to tiles with xcd_block (each XCD takes one
// contiguous range), so the x reads and y atomics of neighbouring tiles meet
// in the same L2.
template <class T, bool DET>
__global__ __launch_bounds__(256) void k_schur_tiles(
    const int32_t* __restrict__ tile_obs, const int32_t* __restrict__ tile_pt,
    const int32_t* __restrict__ tile_coff, const int32_t* __restrict__ tile_cams,
    const int32_t* __restrict__ tile_cseg, const int32_t* __restrict__ pt_off,
    const uint32_t* __restrict__ obs_slot, const T* __restrict__ F, const T* __restrict__ E, int64_t stride,
    const T* __restrict__ Cinv, const T* __restrict__ x, T* __restrict__ y, T* __restrict__ part, int n_tiles,
    const int* __restrict__ done) {
  if (done && *done) return;
  constexpr bool lds_atomics = sizeof(T) == 8 && !DET;
  __shared__ T xs[TILE_SLOTS * 9];
  __shared__ T ys[lds_atomics ? TILE_SLOTS * 9 : 1];
  // E^T F x terms [3][TILE_OBS]; FP32 then the camera terms [TILE_OBS][9]
  __shared__ T buf[lds_atomics ? 3 * TILE_OBS : 9 * TILE_OBS];
  __shared__ T us[(TILE_OBS / 2) * 3];
  __shared__ int segs[lds_atomics ? 1 : TILE_OBS + 1];
  const int t = xcd_block(blockIdx.x, n_tiles);
  if (t >= n_tiles) return;
  const int o0 = tile_obs[t], o1 = tile_obs[t + 1];
  const int q0 = tile_pt[t], np = tile_pt[t + 1] - q0;
  const int c0 = tile_coff[t], nc = tile_coff[t + 1] - c0;
  const int ncs = nc < TILE_SLOTS ? nc : TILE_SLOTS;
  const bool big = o1 - o0 > TILE_OBS;
  const int o = o0 + threadIdx.x;
  const bool act = o < o1;
  T f[18], e[6];
  uint32_t w = 0;
  if (act) {
    w = obs_slot[o];
#pragma unroll
    for (int k = 0; k < 18; ++k) f[k] = F[k * stride + o];
#pragma unroll
    for (int k = 0; k < 6; ++k) e[k] = E[k * stride + o];
  }
  T ci[6];
  int l0 = 0, l1 = 0;
  if (threadIdx.x < np) {
    const int q = q0 + threadIdx.x;
#pragma unroll
    for (int k = 0; k < 6; ++k) ci[k] = Cinv[(size_t)q * 6 + k];
    l0 = pt_off[q] - o0;
    l1 = pt_off[q + 1] - o0;
  }
  if (!lds_atomics && !big)
    for (int i = threadIdx.x; i <= nc; i += 256) segs[i] = i < nc ? tile_cseg[c0 + i] : o1 - o0;
  for (int i = threadIdx.x; i < ncs * 9; i += 256) {
    const int sl = i / 9, k = i - sl * 9;
    xs[i] = x[(size_t)tile_cams[c0 + sl] * 9 + k];
    if (lds_atomics) ys[i] = T(0);
  }
  __syncthreads();

  const int slot = (int)(w & 0xffffu), pl = (int)((w >> 16) & 0xffu), rank = (int)(w >> 24);
  T z0 = 0, z1 = 0, z2 = 0;
  if (act) {
    const T* xv = slot < TILE_SLOTS ? &xs[slot * 9] : &x[(size_t)tile_cams[c0 + slot] * 9];
    T s0 = 0, s1 = 0;
#pragma unroll
    for (int k = 0; k < 9; ++k) { s0 += f[k] * xv[k]; s1 += f[9 + k] * xv[k]; }
    z0 = e[0] * s0 + e[3] * s1;
    z1 = e[1] * s0 + e[4] * s1;
    z2 = e[2] * s0 + e[5] * s1;
  }
  for (int oo = o0 + 256 + threadIdx.x; oo < o1; oo += 256) {
    const uint32_t ww = obs_slot[oo];
    const int sl = (int)(ww & 0xffffu);
    const T* xv = sl < TILE_SLOTS ? &xs[sl * 9] : &x[(size_t)tile_cams[c0 + sl] * 9];
    T s0 = 0, s1 = 0;
    for (int k = 0; k < 9; ++k) { s0 += F[k * stride + oo] * xv[k]; s1 += F[(9 + k) * stride + oo] * xv[k]; }
    z0 += E[0 * stride + oo] * s0 + E[3 * stride + oo] * s1;
    z1 += E[1 * stride + oo] * s0 + E[4 * stride + oo] * s1;
    z2 += E[2 * stride + oo] * s0 + E[5 * stride + oo] * s1;
  }
  buf[0 * TILE_OBS + threadIdx.x] = z0;
  buf[1 * TILE_OBS + threadIdx.x] = z1;
  buf[2 * TILE_OBS + threadIdx.x] = z2;
  __syncthreads();
  if (threadIdx.x < np) {
    if (l1 - l0 > TILE_OBS) { l0 = 0; l1 = TILE_OBS; }
    T a0 = 0, a1 = 0, a2 = 0;
    for (int l = l0; l < l1; ++l) { a0 += buf[l]; a1 += buf[TILE_OBS + l]; a2 += buf[2 * TILE_OBS + l]; }
    us[threadIdx.x * 3 + 0] = ci[0] * a0 + ci[1] * a1 + ci[2] * a2;
    us[threadIdx.x * 3 + 1] = ci[1] * a0 + ci[3] * a1 + ci[4] * a2;
    us[threadIdx.x * 3 + 2] = ci[2] * a0 + ci[4] * a1 + ci[5] * a2;
  }
  __syncthreads();
  if (big) {
    for (int oo = o0 + threadIdx.x; oo < o1; oo += 256) {
      const uint32_t ww = obs_slot[oo];
      const int sl = (int)(ww & 0xffffu), pq = (int)((ww >> 16) & 0xffu);
      const T u0 = us[pq * 3], u1 = us[pq * 3 + 1], u2 = us[pq * 3 + 2];
      const T w0 = E[0 * stride + oo] * u0 + E[1 * stride + oo] * u1 + E[2 * stride + oo] * u2;
      const T w1 = E[3 * stride + oo] * u0 + E[4 * stride + oo] * u1 + E[5 * stride + oo] * u2;
      if (DET) {
        T* pv = part + (size_t)(c0 + sl) * 9;
        for (int k = 0; k < 9; ++k) pv[k] = -(F[k * stride + oo] * w0 + F[(9 + k) * stride + oo] * w1);
      } else {
        T* yv = y + (size_t)tile_cams[c0 + sl] * 9;
        for (int k = 0; k < 9; ++k) unsafeAtomicAdd(&yv[k], -(F[k * stride + oo] * w0 + F[(9 + k) * stride + oo] * w1));
      }
    }
    return;
  }
  if (lds_atomics) {
    if (act) {
      const T u0 = us[pl * 3], u1 = us[pl * 3 + 1], u2 = us[pl * 3 + 2];
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
    __syncthreads();
    for (int i = threadIdx.x; i < ncs * 9; i += 256) {
      const int sl = i / 9, k = i - sl * 9;
      unsafeAtomicAdd(&y[(size_t)tile_cams[c0 + sl] * 9 + k], ys[i]);
    }
  } else {
    if (act) {
      const T u0 = us[pl * 3], u1 = us[pl * 3 + 1], u2 = us[pl * 3 + 2];
      const T w0 = e[0] * u0 + e[1] * u1 + e[2] * u2;
      const T w1 = e[3] * u0 + e[4] * u1 + e[5] * u2;
#pragma unroll
      for (int k = 0; k < 9; ++k) buf[rank * 9 + k] = -(f[k] * w0 + f[9 + k] * w1);
    }
    __syncthreads();
    for (int i = threadIdx.x; i < nc * 9; i += 256) {
      const int sl = i / 9, k = i - sl * 9;
      T acc = 0;
      for (int l = segs[sl]; l < segs[sl + 1]; ++l) acc += buf[l * 9 + k];
      if (DET) part[(size_t)(c0 + sl) * 9 + k] = acc;
      else unsafeAtomicAdd(&y[(size_t)tile_cams[c0 + sl] * 9 + k], acc);
    }
  }
}

// Deterministic completion of the product: y_c += the partial sums of camera
// c's (tile, camera) entries in tile order (te_ptr/te list them per camera).
// One thread per (camera, component).
template <class T>
__global__ __launch_bounds__(256) void k_schur_gather(int n_cam, const int32_t* __restrict__ te_ptr,
                                                      const int32_t* __restrict__ te, const T* __restrict__ part,
                                                      T* __restrict__ y, const int* __restrict__ done) {
  if (done && *done) return;
  const int gid = blockIdx.x * 252 + threadIdx.x;
  const int c = gid / 9, k = gid % 9;
  if (threadIdx.x >= 252 || c >= n_cam) return;
  T acc = 0;
  for (int i = te_ptr[c]; i < te_ptr[c + 1]; ++i) acc += part[(size_t)te[i] * 9 + k];
  y[(size_t)c * 9 + k] += acc;
}

#define BAMG_SCHUR_INST(T, DET)                                                                              \
  template __global__ void k_schur_tiles<T, DET>(const int32_t*, const int32_t*, const int32_t*, const int32_t*, \
                                                 const int32_t*, const int32_t*, const uint32_t*, const T*,       \
                                                 const T*, int64_t, const T*, const T*, T*, T*, int, const int*);
BAMG_SCHUR_INST(double, false)
BAMG_SCHUR_INST(double, true)
BAMG_SCHUR_INST(float, false)
BAMG_SCHUR_INST(float, true)
#undef BAMG_SCHUR_INST
template __global__ void k_schur_gather<double>(int, const int32_t*, const int32_t*, const double*, double*,
                                                const int*);
template __global__ void k_schur_gather<float>(int, const int32_t*, const int32_t*, const float*, float*,
                                               const int*);
template __global__ void k_apply_A<double>(int, const double*, const double*, double*);
template __global__ void k_apply_A<float>(int, const float*, const float*, float*);

}  // namespace bamg
