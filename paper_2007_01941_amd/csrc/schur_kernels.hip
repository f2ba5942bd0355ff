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

// y -= F^T E C^-1 E^T F x. Observations are cut (at plan time) into tiles of
// at most TILE_OBS observations of whole points, and consecutive tiles into
// groups whose cameras fit GROUP_SLOTS; one workgroup of 256 threads works
// through one group, one tile at a time, one thread per observation:
//  1. s_o = F_o x_c(o) with the group's x staged in LDS once; each thread
//     leaves E_o^T s_o in LDS.
//  2. One thread per point adds its observations' terms in order and applies
//     C_p^-1: u_p.
//  3. The camera terms -F_o^T E_o u_p are summed per camera into the group's
//     LDS accumulators: FP64 by LDS atomic adds; FP32 (whose LDS atomics
//     contend badly when many lanes share a camera) and the deterministic
//     mode by runs: each thread leaves its terms at its observation's rank in
//     the tile's camera-sorted order, and one thread per (camera, component)
//     adds its camera's run (in four interleaved partial sums).
// At the end of the group each (camera, component) sum is added to y with one global
// atomic (DET: stored to part[(grp_coff[g] + slot) * 9 + k] and added in
// group order by k_schur_gather). Groups are tiles of whole points ordered by
// their lowest camera, so neighbouring tiles share most cameras and a group
// issues far fewer atomics than its tiles would one by one.
//
// A group of one tile may hold more cameras than GROUP_SLOTS: the others read
// x from global memory and add their sums to y directly (DET: store them). A
// tile of more than TILE_OBS observations (a single point) is a group of its
// own, with one camera per observation: each term goes to y (or part) directly.
//
// The launch maps workgroups to groups with xcd_block (each XCD takes one
// contiguous range), so the x reads and y atomics of neighbouring groups meet
// in the same L2.
template <class T>
struct TileRegs {
  T f[18], e[6];   // this thread's observation
  uint32_t w;      // its slot word: group slot | point slot << 16 | camera-sorted rank << 24
  T ci[6];         // this thread's point (threads below the tile's point count)
  int l0, l1;      //   and its observation range within the tile
  int seg, cslot;  // this thread's tile camera: first rank, group slot (run sums)
};

template <class T, bool RUNS>
__device__ __forceinline__ void load_tile(int t, const int32_t* __restrict__ tile_obs,
                                          const int32_t* __restrict__ tile_pt,
                                          const int32_t* __restrict__ tile_coff,
                                          const int32_t* __restrict__ tile_cseg,
                                          const int32_t* __restrict__ tile_cslot,
                                          const int32_t* __restrict__ pt_off,
                                          const uint32_t* __restrict__ obs_slot, const T* __restrict__ F,
                                          const T* __restrict__ E, int64_t stride, const T* __restrict__ Cinv,
                                          TileRegs<T>& r) {
  const int tid = threadIdx.x;
  const int o0 = tile_obs[t], o = o0 + tid;
  r.w = 0;
  if (o < tile_obs[t + 1]) {
    r.w = obs_slot[o];
#pragma unroll
    for (int k = 0; k < 18; ++k) r.f[k] = F[k * stride + o];
#pragma unroll
    for (int k = 0; k < 6; ++k) r.e[k] = E[k * stride + o];
  }
  const int q0 = tile_pt[t];
  r.l0 = r.l1 = 0;
  if (tid < tile_pt[t + 1] - q0) {
    const int q = q0 + tid;
#pragma unroll
    for (int k = 0; k < 6; ++k) r.ci[k] = Cinv[(size_t)q * 6 + k];
    r.l0 = pt_off[q] - o0;
    r.l1 = pt_off[q + 1] - o0;
  }
  if (RUNS) {
    const int c0 = tile_coff[t];
    if (tid < tile_coff[t + 1] - c0) {
      r.seg = tile_cseg[c0 + tid];
      r.cslot = tile_cslot[c0 + tid];
    }
  }
}

template <class T, bool DET>
__global__ __launch_bounds__(256) void k_schur_groups(
    const int32_t* __restrict__ grp_tile, const int32_t* __restrict__ grp_coff,
    const int32_t* __restrict__ grp_cams, const int32_t* __restrict__ tile_obs,
    const int32_t* __restrict__ tile_pt, const int32_t* __restrict__ tile_coff,
    const int32_t* __restrict__ tile_cseg, const int32_t* __restrict__ tile_cslot,
    const int32_t* __restrict__ pt_off, const uint32_t* __restrict__ obs_slot, const T* __restrict__ F,
    const T* __restrict__ E, int64_t stride, const T* __restrict__ Cinv, const T* __restrict__ x,
    T* __restrict__ y, T* __restrict__ part, int n_groups, const int* __restrict__ done) {
  if (done && *done) return;
  constexpr bool RUNS = sizeof(T) == 4 || DET;
  __shared__ T xs[GROUP_SLOTS * 9];
  __shared__ T ys[GROUP_SLOTS * 9];
  // E^T F x terms [3][TILE_OBS]; with RUNS then the camera terms [TILE_OBS][9]
  __shared__ T buf[RUNS ? 9 * TILE_OBS : 3 * TILE_OBS];
  __shared__ T us[(TILE_OBS / 2) * 3];
  __shared__ int segs[RUNS ? TILE_OBS + 1 : 1];
  __shared__ int cslots[RUNS ? TILE_OBS : 1];
  const int g = xcd_block(blockIdx.x, n_groups);
  if (g >= n_groups) return;
  const int tid = threadIdx.x;
  const int t0 = grp_tile[g], t1 = grp_tile[g + 1];
  const bool single = t1 == t0 + 1;
  const int gc0 = grp_coff[g];
  const int gns = min(grp_coff[g + 1] - gc0, GROUP_SLOTS);

  if (tile_obs[t0 + 1] - tile_obs[t0] > TILE_OBS) {
    // one point seen by more than TILE_OBS cameras (one camera per observation)
    const int o0 = tile_obs[t0], o1 = tile_obs[t0 + 1];
    const int q = tile_pt[t0];
    T z0 = 0, z1 = 0, z2 = 0;
    for (int oo = o0 + tid; oo < o1; oo += 256) {
      const int sl = (int)(obs_slot[oo] & 0xffffu);
      const T* xv = &x[(size_t)grp_cams[gc0 + sl] * 9];
      T s0 = 0, s1 = 0;
      for (int k = 0; k < 9; ++k) { s0 += F[k * stride + oo] * xv[k]; s1 += F[(9 + k) * stride + oo] * xv[k]; }
      z0 += E[0 * stride + oo] * s0 + E[3 * stride + oo] * s1;
      z1 += E[1 * stride + oo] * s0 + E[4 * stride + oo] * s1;
      z2 += E[2 * stride + oo] * s0 + E[5 * stride + oo] * s1;
    }
    buf[tid] = z0;
    buf[TILE_OBS + tid] = z1;
    buf[2 * TILE_OBS + tid] = z2;
    __syncthreads();
    if (tid == 0) {
      T a0 = 0, a1 = 0, a2 = 0;
      for (int l = 0; l < 256; ++l) { a0 += buf[l]; a1 += buf[TILE_OBS + l]; a2 += buf[2 * TILE_OBS + l]; }
      const T* ci = Cinv + (size_t)q * 6;
      us[0] = ci[0] * a0 + ci[1] * a1 + ci[2] * a2;
      us[1] = ci[1] * a0 + ci[3] * a1 + ci[4] * a2;
      us[2] = ci[2] * a0 + ci[4] * a1 + ci[5] * a2;
    }
    __syncthreads();
    const T u0 = us[0], u1 = us[1], u2 = us[2];
    for (int oo = o0 + tid; oo < o1; oo += 256) {
      const int sl = (int)(obs_slot[oo] & 0xffffu);
      const T w0 = E[0 * stride + oo] * u0 + E[1 * stride + oo] * u1 + E[2 * stride + oo] * u2;
      const T w1 = E[3 * stride + oo] * u0 + E[4 * stride + oo] * u1 + E[5 * stride + oo] * u2;
      for (int k = 0; k < 9; ++k) {
        const T v = -(F[k * stride + oo] * w0 + F[(9 + k) * stride + oo] * w1);
        if (DET) part[(size_t)(gc0 + sl) * 9 + k] = v;
        else unsafeAtomicAdd(&y[(size_t)grp_cams[gc0 + sl] * 9 + k], v);
      }
    }
    return;
  }

  for (int i = tid; i < gns * 9; i += 256) {
    const int sl = i / 9;
    xs[i] = x[(size_t)grp_cams[gc0 + sl] * 9 + (i - sl * 9)];
    if (!(RUNS && single)) ys[i] = T(0);
  }
  TileRegs<T> cur;
  for (int t = t0; t < t1; ++t) {
    const int n = tile_obs[t + 1] - tile_obs[t];
    const int np = tile_pt[t + 1] - tile_pt[t];
    const int nc = tile_coff[t + 1] - tile_coff[t];
    load_tile<T, RUNS>(t, tile_obs, tile_pt, tile_coff, tile_cseg, tile_cslot, pt_off, obs_slot, F, E, stride,
                       Cinv, cur);
    __syncthreads();   // x staged; the previous tile's LDS reads are done
    if (RUNS) {
      if (tid < nc) {
        segs[tid] = cur.seg;
        cslots[tid] = cur.cslot;
      }
      if (tid == 0) segs[nc] = n;
    }
    const bool act = tid < n;
    const int slot = (int)(cur.w & 0xffffu), pl = (int)((cur.w >> 16) & 0xffu), rank = (int)(cur.w >> 24);
    T z0 = 0, z1 = 0, z2 = 0;
    if (act) {
      T xv[9];
      if (slot < GROUP_SLOTS) {
#pragma unroll
        for (int k = 0; k < 9; ++k) xv[k] = xs[slot * 9 + k];
      } else {
        const T* xg = &x[(size_t)grp_cams[gc0 + slot] * 9];
#pragma unroll
        for (int k = 0; k < 9; ++k) xv[k] = xg[k];
      }
      T s0 = 0, s1 = 0;
#pragma unroll
      for (int k = 0; k < 9; ++k) { s0 += cur.f[k] * xv[k]; s1 += cur.f[9 + k] * xv[k]; }
      z0 = cur.e[0] * s0 + cur.e[3] * s1;
      z1 = cur.e[1] * s0 + cur.e[4] * s1;
      z2 = cur.e[2] * s0 + cur.e[5] * s1;
    }
    buf[tid] = z0;
    buf[TILE_OBS + tid] = z1;
    buf[2 * TILE_OBS + tid] = z2;
    __syncthreads();
    if (tid < np) {
      T a0 = 0, a1 = 0, a2 = 0;
      for (int l = cur.l0; l < cur.l1; ++l) { a0 += buf[l]; a1 += buf[TILE_OBS + l]; a2 += buf[2 * TILE_OBS + l]; }
      us[tid * 3 + 0] = cur.ci[0] * a0 + cur.ci[1] * a1 + cur.ci[2] * a2;
      us[tid * 3 + 1] = cur.ci[1] * a0 + cur.ci[3] * a1 + cur.ci[4] * a2;
      us[tid * 3 + 2] = cur.ci[2] * a0 + cur.ci[4] * a1 + cur.ci[5] * a2;
    }
    __syncthreads();
    T w0 = 0, w1 = 0;
    if (act) {
      const T u0 = us[pl * 3], u1 = us[pl * 3 + 1], u2 = us[pl * 3 + 2];
      w0 = cur.e[0] * u0 + cur.e[1] * u1 + cur.e[2] * u2;
      w1 = cur.e[3] * u0 + cur.e[4] * u1 + cur.e[5] * u2;
    }
    if (!RUNS) {
      if (act) {
        if (slot < GROUP_SLOTS) {
#pragma unroll
          for (int k = 0; k < 9; ++k) atomicAdd(&ys[slot * 9 + k], -(cur.f[k] * w0 + cur.f[9 + k] * w1));
        } else {
          T* yv = y + (size_t)grp_cams[gc0 + slot] * 9;
#pragma unroll
          for (int k = 0; k < 9; ++k) unsafeAtomicAdd(&yv[k], -(cur.f[k] * w0 + cur.f[9 + k] * w1));
        }
      }
    } else {
      if (act) {
#pragma unroll
        for (int k = 0; k < 9; ++k) buf[rank * 9 + k] = -(cur.f[k] * w0 + cur.f[9 + k] * w1);
      }
      __syncthreads();
      for (int i = tid; i < nc * 9; i += 256) {
        const int j = i / 9, k = i - j * 9;
        // four partial sums keep four LDS reads of the run in flight
        const int lb = segs[j], le = segs[j + 1];
        T a0 = 0, a1 = 0, a2 = 0, a3 = 0;
        int l = lb;
        for (; l + 4 <= le; l += 4) {
          a0 += buf[l * 9 + k];
          a1 += buf[(l + 1) * 9 + k];
          a2 += buf[(l + 2) * 9 + k];
          a3 += buf[(l + 3) * 9 + k];
        }
        for (; l < le; ++l) a0 += buf[l * 9 + k];
        const T acc = (a0 + a1) + (a2 + a3);
        const int sl = cslots[j];
        // a group of one tile flushes its sums directly
        if (sl < GROUP_SLOTS && !single) ys[sl * 9 + k] += acc;
        else if (DET) part[(size_t)(gc0 + sl) * 9 + k] = acc;
        else unsafeAtomicAdd(&y[(size_t)grp_cams[gc0 + sl] * 9 + k], acc);
      }
    }
  }
  if (RUNS && single) return;
  __syncthreads();
  for (int i = tid; i < gns * 9; i += 256) {
    const int sl = i / 9, k = i - sl * 9;
    if (DET) part[(size_t)(gc0 + sl) * 9 + k] = ys[i];
    else unsafeAtomicAdd(&y[(size_t)grp_cams[gc0 + sl] * 9 + k], ys[i]);
  }
}

// The same product with F_o and E_o recomputed from the camera and the point
// (project_jacobian, as the Jacobian kernel computes them, times the robust
// weight when there is one) instead of read from the observation planes. Per
// observation the product then reads its 4-byte slot word (and its 8-byte
// weight with a robust loss), per point its record [X | C_p^-1], and per
// group its cameras' 24 parameters, staged in LDS with x: a few dozen bytes
// per observation instead of 24 scalars, for the projection's arithmetic
// (about 150 FP64 operations), which the chip has more of than bandwidth.
// The FP32 form rounds the recomputed blocks exactly as the stored FP32
// copies are rounded. Otherwise as k_schur_groups.
constexpr int CPS = 26;   // LDS stride of a camera's parameters (24 used; 16-byte rows)
// The parameters of the group's first RC_SLOTS cameras are staged in LDS (the
// others are read from the cache), so that LDS (36 KB) and registers (the
// launch bound) both allow four workgroups per CU: 102 -> 92 us on the city grid.
constexpr int RC_SLOTS = 48;

template <class T>
__device__ __forceinline__ void recompute_blocks(const double* __restrict__ cp, const double X[3], double wgt,
                                                 T f[18], T e[6]) {
  double pi[2], Fo[18], Eo[6], z;
  project_jacobian(cp, X, pi, Fo, Eo, &z);
#pragma unroll
  for (int k = 0; k < 18; ++k) f[k] = (T)(Fo[k] * wgt);
#pragma unroll
  for (int k = 0; k < 6; ++k) e[k] = (T)(Eo[k] * wgt);
}

template <class T, bool DET>
__global__ __launch_bounds__(256, 4) void k_schur_groups_rc(
    const int32_t* __restrict__ grp_tile, const int32_t* __restrict__ grp_coff,
    const int32_t* __restrict__ grp_cams, const int32_t* __restrict__ tile_obs,
    const int32_t* __restrict__ tile_pt, const int32_t* __restrict__ tile_coff,
    const int32_t* __restrict__ tile_cseg, const int32_t* __restrict__ tile_cslot,
    const int32_t* __restrict__ pt_off, const uint32_t* __restrict__ obs_slot,
    const double* __restrict__ campre, const double* __restrict__ prec, const double* __restrict__ wsq,
    const T* __restrict__ Cinv, const T* __restrict__ x, T* __restrict__ y, T* __restrict__ part, int n_groups,
    const int* __restrict__ done) {
  if (done && *done) return;
  constexpr bool RUNS = sizeof(T) == 4 || DET;
  __shared__ T xs[GROUP_SLOTS * 9];
  __shared__ T ys[GROUP_SLOTS * 9];
  __shared__ T buf[RUNS ? 9 * TILE_OBS : 3 * TILE_OBS];
  __shared__ T us[(TILE_OBS / 2) * 3];
  __shared__ int segs[RUNS ? TILE_OBS + 1 : 1];
  __shared__ int cslots[RUNS ? TILE_OBS : 1];
  __shared__ double cps[RC_SLOTS * CPS];        // the group's camera parameters
  __shared__ double xp[(TILE_OBS / 2) * 3];     // the tile's points
  const int g = xcd_block(blockIdx.x, n_groups);
  if (g >= n_groups) return;
  const int tid = threadIdx.x;
  const int t0 = grp_tile[g], t1 = grp_tile[g + 1];
  const bool single = t1 == t0 + 1;
  const int gc0 = grp_coff[g];
  const int gns = min(grp_coff[g + 1] - gc0, GROUP_SLOTS);

  if (tile_obs[t0 + 1] - tile_obs[t0] > TILE_OBS) {
    // one point seen by more than TILE_OBS cameras (one camera per observation)
    const int o0 = tile_obs[t0], o1 = tile_obs[t0 + 1];
    const int q = tile_pt[t0];
    const double X[3] = {prec[(size_t)q * PREC], prec[(size_t)q * PREC + 1], prec[(size_t)q * PREC + 2]};
    T z0 = 0, z1 = 0, z2 = 0;
    for (int oo = o0 + tid; oo < o1; oo += 256) {
      const int cam = grp_cams[gc0 + (int)(obs_slot[oo] & 0xffffu)];
      T f[18], e[6];
      recompute_blocks<T>(campre + (size_t)cam * 24, X, wsq ? wsq[oo] : 1.0, f, e);
      const T* xv = &x[(size_t)cam * 9];
      T s0 = 0, s1 = 0;
      for (int k = 0; k < 9; ++k) { s0 += f[k] * xv[k]; s1 += f[9 + k] * xv[k]; }
      z0 += e[0] * s0 + e[3] * s1;
      z1 += e[1] * s0 + e[4] * s1;
      z2 += e[2] * s0 + e[5] * s1;
    }
    buf[tid] = z0;
    buf[TILE_OBS + tid] = z1;
    buf[2 * TILE_OBS + tid] = z2;
    __syncthreads();
    if (tid == 0) {
      T a0 = 0, a1 = 0, a2 = 0;
      for (int l = 0; l < 256; ++l) { a0 += buf[l]; a1 += buf[TILE_OBS + l]; a2 += buf[2 * TILE_OBS + l]; }
      const T* ci = Cinv + (size_t)q * 6;
      us[0] = ci[0] * a0 + ci[1] * a1 + ci[2] * a2;
      us[1] = ci[1] * a0 + ci[3] * a1 + ci[4] * a2;
      us[2] = ci[2] * a0 + ci[4] * a1 + ci[5] * a2;
    }
    __syncthreads();
    const T u0 = us[0], u1 = us[1], u2 = us[2];
    for (int oo = o0 + tid; oo < o1; oo += 256) {
      const int sl = (int)(obs_slot[oo] & 0xffffu);
      const int cam = grp_cams[gc0 + sl];
      T f[18], e[6];
      recompute_blocks<T>(campre + (size_t)cam * 24, X, wsq ? wsq[oo] : 1.0, f, e);
      const T w0 = e[0] * u0 + e[1] * u1 + e[2] * u2;
      const T w1 = e[3] * u0 + e[4] * u1 + e[5] * u2;
      for (int k = 0; k < 9; ++k) {
        const T v = -(f[k] * w0 + f[9 + k] * w1);
        if (DET) part[(size_t)(gc0 + sl) * 9 + k] = v;
        else unsafeAtomicAdd(&y[(size_t)cam * 9 + k], v);
      }
    }
    return;
  }

  for (int i = tid; i < gns * 9; i += 256) {
    const int sl = i / 9;
    xs[i] = x[(size_t)grp_cams[gc0 + sl] * 9 + (i - sl * 9)];
    if (!(RUNS && single)) ys[i] = T(0);
  }
  for (int i = tid; i < min(gns, RC_SLOTS) * 24; i += 256) {
    const int sl = i / 24, k = i - sl * 24;
    cps[sl * CPS + k] = campre[(size_t)grp_cams[gc0 + sl] * 24 + k];
  }
  for (int t = t0; t < t1; ++t) {
    const int o0 = tile_obs[t];
    const int n = tile_obs[t + 1] - o0;
    const int q0 = tile_pt[t];
    const int np = tile_pt[t + 1] - q0;
    const int c0 = tile_coff[t];
    const int nc = tile_coff[t + 1] - c0;
    const bool act = tid < n;
    uint32_t wd = 0;
    double wgt = 1.0;
    if (act) {
      wd = obs_slot[o0 + tid];
      if (wsq) wgt = wsq[o0 + tid];
    }
    T ci[6];
    int l0 = 0, l1 = 0;
    if (tid < np) {
      const int q = q0 + tid;
#pragma unroll
      for (int k = 0; k < 6; ++k) ci[k] = Cinv[(size_t)q * 6 + k];
      l0 = pt_off[q] - o0;
      l1 = pt_off[q + 1] - o0;
      // the previous tile's reads of xp ended before its last barrier
#pragma unroll
      for (int k = 0; k < 3; ++k) xp[tid * 3 + k] = prec[(size_t)q * PREC + k];
    }
    int seg = 0, cslot = 0;
    if (RUNS && tid < nc) {
      seg = tile_cseg[c0 + tid];
      cslot = tile_cslot[c0 + tid];
    }
    __syncthreads();   // x, the cameras and the points staged; the previous tile's LDS reads are done
    if (RUNS) {
      if (tid < nc) {
        segs[tid] = seg;
        cslots[tid] = cslot;
      }
      if (tid == 0) segs[nc] = n;
    }
    const int slot = (int)(wd & 0xffffu), pl = (int)((wd >> 16) & 0xffu), rank = (int)(wd >> 24);
    T f[18], e[6];
    T z0 = 0, z1 = 0, z2 = 0;
    if (act) {
      double cpr[24];
      if (slot < RC_SLOTS) {
#pragma unroll
        for (int k = 0; k < 24; ++k) cpr[k] = cps[slot * CPS + k];
      } else {
        const double* cg = campre + (size_t)grp_cams[gc0 + slot] * 24;
#pragma unroll
        for (int k = 0; k < 24; ++k) cpr[k] = cg[k];
      }
      const double X[3] = {xp[pl * 3], xp[pl * 3 + 1], xp[pl * 3 + 2]};
      // x_c from LDS (or, past the staged slots, global memory), by explicit
      // branches so that each load uses its own address space
      T xv[9];
      if (slot < GROUP_SLOTS) {
#pragma unroll
        for (int k = 0; k < 9; ++k) xv[k] = xs[slot * 9 + k];
      } else {
        const T* xg = &x[(size_t)grp_cams[gc0 + slot] * 9];
#pragma unroll
        for (int k = 0; k < 9; ++k) xv[k] = xg[k];
      }
      recompute_blocks<T>(cpr, X, wgt, f, e);
      T s0 = 0, s1 = 0;
#pragma unroll
      for (int k = 0; k < 9; ++k) { s0 += f[k] * xv[k]; s1 += f[9 + k] * xv[k]; }
      z0 = e[0] * s0 + e[3] * s1;
      z1 = e[1] * s0 + e[4] * s1;
      z2 = e[2] * s0 + e[5] * s1;
    }
    buf[tid] = z0;
    buf[TILE_OBS + tid] = z1;
    buf[2 * TILE_OBS + tid] = z2;
    __syncthreads();
    if (tid < np) {
      T a0 = 0, a1 = 0, a2 = 0;
      for (int l = l0; l < l1; ++l) { a0 += buf[l]; a1 += buf[TILE_OBS + l]; a2 += buf[2 * TILE_OBS + l]; }
      us[tid * 3 + 0] = ci[0] * a0 + ci[1] * a1 + ci[2] * a2;
      us[tid * 3 + 1] = ci[1] * a0 + ci[3] * a1 + ci[4] * a2;
      us[tid * 3 + 2] = ci[2] * a0 + ci[4] * a1 + ci[5] * a2;
    }
    __syncthreads();
    T w0 = 0, w1 = 0;
    if (act) {
      const T u0 = us[pl * 3], u1 = us[pl * 3 + 1], u2 = us[pl * 3 + 2];
      w0 = e[0] * u0 + e[1] * u1 + e[2] * u2;
      w1 = e[3] * u0 + e[4] * u1 + e[5] * u2;
    }
    if (!RUNS) {
      if (act) {
        if (slot < GROUP_SLOTS) {
#pragma unroll
          for (int k = 0; k < 9; ++k) atomicAdd(&ys[slot * 9 + k], -(f[k] * w0 + f[9 + k] * w1));
        } else {
          T* yv = y + (size_t)grp_cams[gc0 + slot] * 9;
#pragma unroll
          for (int k = 0; k < 9; ++k) unsafeAtomicAdd(&yv[k], -(f[k] * w0 + f[9 + k] * w1));
        }
      }
    } else {
      if (act) {
#pragma unroll
        for (int k = 0; k < 9; ++k) buf[rank * 9 + k] = -(f[k] * w0 + f[9 + k] * w1);
      }
      __syncthreads();
      for (int i = tid; i < nc * 9; i += 256) {
        const int j = i / 9, k = i - j * 9;
        // four partial sums keep four LDS reads of the run in flight
        const int lb = segs[j], le = segs[j + 1];
        T a0 = 0, a1 = 0, a2 = 0, a3 = 0;
        int l = lb;
        for (; l + 4 <= le; l += 4) {
          a0 += buf[l * 9 + k];
          a1 += buf[(l + 1) * 9 + k];
          a2 += buf[(l + 2) * 9 + k];
          a3 += buf[(l + 3) * 9 + k];
        }
        for (; l < le; ++l) a0 += buf[l * 9 + k];
        const T acc = (a0 + a1) + (a2 + a3);
        const int sl = cslots[j];
        if (sl < GROUP_SLOTS && !single) ys[sl * 9 + k] += acc;
        else if (DET) part[(size_t)(gc0 + sl) * 9 + k] = acc;
        else unsafeAtomicAdd(&y[(size_t)grp_cams[gc0 + sl] * 9 + k], acc);
      }
    }
  }
  if (RUNS && single) return;
  __syncthreads();
  for (int i = tid; i < gns * 9; i += 256) {
    const int sl = i / 9, k = i - sl * 9;
    if (DET) part[(size_t)(gc0 + sl) * 9 + k] = ys[i];
    else unsafeAtomicAdd(&y[(size_t)grp_cams[gc0 + sl] * 9 + k], ys[i]);
  }
}

// Deterministic completion of the product: y_c += the partial sums of camera
// c's (group, camera) entries (te_ptr/te list them per camera in group
// order). One wave per camera: lane l adds entries l, l + 64, ... in order,
// then the lanes' sums are combined by a fixed butterfly, so the result does
// not depend on timing.
template <class T>
__global__ __launch_bounds__(256) void k_schur_gather(int n_cam, const int32_t* __restrict__ te_ptr,
                                                      const int32_t* __restrict__ te, const T* __restrict__ part,
                                                      T* __restrict__ y, const int* __restrict__ done) {
  if (done && *done) return;
  const int c = blockIdx.x * 4 + (threadIdx.x >> 6), lane = threadIdx.x & 63;
  if (c >= n_cam) return;
  T acc[9];
#pragma unroll
  for (int k = 0; k < 9; ++k) acc[k] = 0;
  for (int i = te_ptr[c] + lane; i < te_ptr[c + 1]; i += 64) {
    const T* pv = part + (size_t)te[i] * 9;
#pragma unroll
    for (int k = 0; k < 9; ++k) acc[k] += pv[k];
  }
#pragma unroll
  for (int k = 0; k < 9; ++k) acc[k] = wave_sum(acc[k]);
  if (lane < 9) {
    T v = acc[0];
#pragma unroll
    for (int k = 1; k < 9; ++k) v = lane == k ? acc[k] : v;
    y[(size_t)c * 9 + lane] += v;
  }
}

#define BAMG_SCHUR_INST(T, DET)                                                                               \
  template __global__ void k_schur_groups<T, DET>(const int32_t*, const int32_t*, const int32_t*, const int32_t*, \
                                                  const int32_t*, const int32_t*, const int32_t*, const int32_t*, \
                                                  const int32_t*, const uint32_t*, const T*, const T*, int64_t,   \
                                                  const T*, const T*, T*, T*, int, const int*);
BAMG_SCHUR_INST(double, false)
BAMG_SCHUR_INST(double, true)
BAMG_SCHUR_INST(float, false)
BAMG_SCHUR_INST(float, true)
#undef BAMG_SCHUR_INST
#define BAMG_SCHUR_RC_INST(T, DET)                                                                            \
  template __global__ void k_schur_groups_rc<T, DET>(                                                         \
      const int32_t*, const int32_t*, const int32_t*, const int32_t*, const int32_t*, const int32_t*,        \
      const int32_t*, const int32_t*, const int32_t*, const uint32_t*, const double*, const double*,         \
      const double*, const T*, const T*, T*, T*, int, const int*);
BAMG_SCHUR_RC_INST(double, false)
BAMG_SCHUR_RC_INST(double, true)
BAMG_SCHUR_RC_INST(float, false)
BAMG_SCHUR_RC_INST(float, true)
#undef BAMG_SCHUR_RC_INST
template __global__ void k_schur_gather<double>(int, const int32_t*, const int32_t*, const double*, double*,
                                                const int*);
template __global__ void k_schur_gather<float>(int, const int32_t*, const int32_t*, const float*, float*,
                                               const int*);
template __global__ void k_apply_A<double>(int, const double*, const double*, double*);
template __global__ void k_apply_A<float>(int, const float*, const float*, float*);

}  // namespace bamg
