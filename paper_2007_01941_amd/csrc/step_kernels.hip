// Per-step kernels: residual and Jacobian, normal-block assembly, the implicit
// Schur product, block Jacobi and back-substitution (Section 2.1 and 3.6 of
// Konolige and Brown, "Multigrid for Bundle Adjustment").
//
// Layout (see plan.hpp): observations are stored point-major (points reordered
// by their lowest observing camera, each point's observations by camera).
// Per-observation blocks are SoA planes with stride `stride`:
//   F[k * stride + o], k = r*9 + c  (F_o = d pi_o / d camera, 2 x 9)
//   E[k * stride + o], k = r*3 + c  (E_o = d pi_o / d point,  2 x 3)
//   f[r * stride + o]               (residual pi_o - u_o)
#include "kernels.hpp"

namespace bamg {

// ---------------------------------------------------------------- cameras

// campre[c] = R (9) | J_r (9) | t (3) | f, k1, k2
__global__ void k_campre(int n_cam, const double* __restrict__ cams, double* __restrict__ campre,
                         uint32_t* err) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= n_cam) return;
  double w[3] = {cams[c * 9 + 0], cams[c * 9 + 1], cams[c * 9 + 2]};
  double R[9], J[9], b;
  rotation(w, R, &b);
  right_jacobian(w, b, J);
  double* o = campre + (size_t)c * 24;
  bool fin = true;
  for (int k = 0; k < 9; ++k) { o[k] = R[k]; o[9 + k] = J[k]; fin &= isfinite(cams[c * 9 + k]); }
  for (int k = 0; k < 3; ++k) o[18 + k] = cams[c * 9 + 3 + k];
  o[21] = cams[c * 9 + 6];
  o[22] = cams[c * 9 + 7];
  o[23] = cams[c * 9 + 8];
  if (!fin) atomicOr(err, ERRF_NONFINITE);
}

// ---------------------------------------------------------------- residual + Jacobian

// The projection pi = f r p with p = -(x, y)/z, r = 1 + k1|p|^2 + k2|p|^4 and
// x_cam = R X + t. With M = d pi / d x_cam:
//   M = -(1/z) (f (r I + (2k1 + 4k2|p|^2) p p^T)) [I2 | p],
//   d pi/dt = M, E = d pi/dX = M R, d pi/dw = -E [X]x J_r,
//   d pi/df = r p, d pi/dk1 = f |p|^2 p, d pi/dk2 = f |p|^4 p.
__device__ __forceinline__ void project_jacobian(const double* __restrict__ cp, const double X[3],
                                                 double pi[2], double Fo[18], double Eo[6],
                                                 double* zcam) {
  const double* R = cp;
  const double* J = cp + 9;
  const double xc = R[0] * X[0] + R[1] * X[1] + R[2] * X[2] + cp[18];
  const double yc = R[3] * X[0] + R[4] * X[1] + R[5] * X[2] + cp[19];
  const double zc = R[6] * X[0] + R[7] * X[1] + R[8] * X[2] + cp[20];
  *zcam = zc;
  const double f = cp[21], k1 = cp[22], k2 = cp[23];
  const double iz = 1.0 / zc;
  const double p0 = -xc * iz, p1 = -yc * iz;
  const double n2 = p0 * p0 + p1 * p1;
  const double r = 1.0 + n2 * (k1 + k2 * n2);
  pi[0] = f * r * p0;
  pi[1] = f * r * p1;
  const double d = 2.0 * k1 + 4.0 * k2 * n2;
  const double m00 = f * (r + d * p0 * p0), m01 = f * d * p0 * p1, m11 = f * (r + d * p1 * p1);
  // M = -iz [[m00, m01, m00 p0 + m01 p1], [m01, m11, m01 p0 + m11 p1]]
  double M[6];
  M[0] = -iz * m00;
  M[1] = -iz * m01;
  M[2] = -iz * (m00 * p0 + m01 * p1);
  M[3] = -iz * m01;
  M[4] = -iz * m11;
  M[5] = -iz * (m01 * p0 + m11 * p1);
#pragma unroll
  for (int rr = 0; rr < 2; ++rr) {
#pragma unroll
    for (int c = 0; c < 3; ++c)
      Eo[rr * 3 + c] = M[rr * 3 + 0] * R[0 * 3 + c] + M[rr * 3 + 1] * R[1 * 3 + c] + M[rr * 3 + 2] * R[2 * 3 + c];
    // g = E_r x X  (row vector E_r [X]x), then d pi_r / dw = -g J_r
    const double e0 = Eo[rr * 3 + 0], e1 = Eo[rr * 3 + 1], e2 = Eo[rr * 3 + 2];
    const double g0 = e1 * X[2] - e2 * X[1];
    const double g1 = e2 * X[0] - e0 * X[2];
    const double g2 = e0 * X[1] - e1 * X[0];
#pragma unroll
    for (int c = 0; c < 3; ++c) Fo[rr * 9 + c] = -(g0 * J[0 * 3 + c] + g1 * J[1 * 3 + c] + g2 * J[2 * 3 + c]);
#pragma unroll
    for (int c = 0; c < 3; ++c) Fo[rr * 9 + 3 + c] = M[rr * 3 + c];
    const double pr = rr == 0 ? p0 : p1;
    Fo[rr * 9 + 6] = r * pr;
    Fo[rr * 9 + 7] = f * n2 * pr;
    Fo[rr * 9 + 8] = f * n2 * n2 * pr;
  }
}

__global__ __launch_bounds__(256) void k_jacobian(
    int n_obs, const int32_t* __restrict__ obs_cam, const int32_t* __restrict__ obs_pt,
    const int32_t* __restrict__ obs_orig, const int32_t* __restrict__ pt_orig,
    const double* __restrict__ campre, const double* __restrict__ pts, const double* __restrict__ uv,
    int64_t stride, double* __restrict__ F, double* __restrict__ E, double* __restrict__ fres,
    float* __restrict__ F32, float* __restrict__ E32, uint32_t* err) {
  const int o = blockIdx.x * blockDim.x + threadIdx.x;
  if (o >= n_obs) return;
  const int c = obs_cam[o];
  const int q = pt_orig[obs_pt[o]];
  const int oo = obs_orig[o];
  const double X[3] = {pts[q * 3 + 0], pts[q * 3 + 1], pts[q * 3 + 2]};
  double pi[2], Fo[18], Eo[6], z;
  project_jacobian(campre + (size_t)c * 24, X, pi, Fo, Eo, &z);
  const double r0 = pi[0] - uv[(size_t)oo * 2 + 0];
  const double r1 = pi[1] - uv[(size_t)oo * 2 + 1];
  if (!(z < 0.0)) atomicOr(err, ERRF_GEOMETRY);
  if (!isfinite(r0) || !isfinite(r1) || !isfinite(X[0] + X[1] + X[2])) atomicOr(err, ERRF_NONFINITE);
  fres[o] = r0;
  fres[stride + o] = r1;
#pragma unroll
  for (int k = 0; k < 18; ++k) F[k * stride + o] = Fo[k];
#pragma unroll
  for (int k = 0; k < 6; ++k) E[k * stride + o] = Eo[k];
  if (F32) {
#pragma unroll
    for (int k = 0; k < 18; ++k) F32[k * stride + o] = (float)Fo[k];
#pragma unroll
    for (int k = 0; k < 6; ++k) E32[k * stride + o] = (float)Eo[k];
  }
}

// Point-major planes -> caller-order arrays (f [n][2], F [n][2][9], E [n][2][3]).
__global__ void k_scatter_jacobian(int n_obs, const int32_t* __restrict__ obs_orig, int64_t stride,
                                   const double* __restrict__ F, const double* __restrict__ E,
                                   const double* __restrict__ fres, double* f_out, double* F_out,
                                   double* E_out) {
  const int o = blockIdx.x * blockDim.x + threadIdx.x;
  if (o >= n_obs) return;
  const size_t oo = obs_orig[o];
  if (f_out) { f_out[oo * 2] = fres[o]; f_out[oo * 2 + 1] = fres[stride + o]; }
  if (F_out) for (int k = 0; k < 18; ++k) F_out[oo * 18 + k] = F[k * stride + o];
  if (E_out) for (int k = 0; k < 6; ++k) E_out[oo * 6 + k] = E[k * stride + o];
}

// ---------------------------------------------------------------- point blocks

// C_p = sum E_o^T E_o + D_p, g_p = sum E_o^T f_o; C_p^-1 (packed), v_p = C_p^-1 g_p.
// D_p = lambda diag(sum E^T E), or the explicit diagonal Dexp (caller order).
__global__ __launch_bounds__(256) void k_point_blocks(
    int n_pt, const int32_t* __restrict__ pt_off, const int32_t* __restrict__ pt_orig, int64_t stride,
    const double* __restrict__ E, const double* __restrict__ fres, double lambda,
    const double* __restrict__ Dexp, int n_cam, double* __restrict__ Cinv, float* __restrict__ Cinv32,
    double* __restrict__ vgp, double* __restrict__ gp_out, double* __restrict__ Dp_out, uint32_t* err) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= n_pt) return;
  double C[6] = {0, 0, 0, 0, 0, 0}, g[3] = {0, 0, 0};
  for (int o = pt_off[q]; o < pt_off[q + 1]; ++o) {
    double e[6];
#pragma unroll
    for (int k = 0; k < 6; ++k) e[k] = E[k * stride + o];
    const double f0 = fres[o], f1 = fres[stride + o];
    C[0] += e[0] * e[0] + e[3] * e[3];
    C[1] += e[0] * e[1] + e[3] * e[4];
    C[2] += e[0] * e[2] + e[3] * e[5];
    C[3] += e[1] * e[1] + e[4] * e[4];
    C[4] += e[1] * e[2] + e[4] * e[5];
    C[5] += e[2] * e[2] + e[5] * e[5];
    g[0] += e[0] * f0 + e[3] * f1;
    g[1] += e[1] * f0 + e[4] * f1;
    g[2] += e[2] * f0 + e[5] * f1;
  }
  double d[3];
  if (Dexp) {
    const int qo = pt_orig[q];
    for (int k = 0; k < 3; ++k) d[k] = Dexp[(size_t)9 * n_cam + 3 * qo + k];
  } else {
    d[0] = lambda * C[0];
    d[1] = lambda * C[3];
    d[2] = lambda * C[5];
  }
  double a[9] = {C[0] + d[0], C[1], C[2], C[1], C[3] + d[1], C[4], C[2], C[4], C[5] + d[2]};
  double inv[9];
  if (!cholesky<3>(a)) {
    atomicOr(err, ERRF_NOT_SPD);
    for (int k = 0; k < 9; ++k) inv[k] = 0.0;
  } else {
    cholesky_inverse<3>(a, inv);
  }
  const double ci[6] = {inv[0], inv[1], inv[2], inv[4], inv[5], inv[8]};
  for (int k = 0; k < 6; ++k) {
    Cinv[(size_t)q * 6 + k] = ci[k];
    if (Cinv32) Cinv32[(size_t)q * 6 + k] = (float)ci[k];
  }
  for (int k = 0; k < 3; ++k) {
    vgp[(size_t)q * 3 + k] = inv[k * 3 + 0] * g[0] + inv[k * 3 + 1] * g[1] + inv[k * 3 + 2] * g[2];
    gp_out[(size_t)q * 3 + k] = g[k];
    Dp_out[(size_t)q * 3 + k] = d[k];
  }
}

// ---------------------------------------------------------------- camera blocks

template <int NV>
__device__ __forceinline__ void block_reduce(double (&acc)[NV], double* red /*[4][NV]*/) {
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
  for (int k = 0; k < NV; ++k) acc[k] = wave_sum(acc[k]);
  if (lane == 0)
    for (int k = 0; k < NV; ++k) red[wid * NV + k] = acc[k];
  __syncthreads();
  for (int k = threadIdx.x; k < NV; k += blockDim.x)
    red[k] = red[k] + red[NV + k] + red[2 * NV + k] + red[3 * NV + k];
  __syncthreads();
}

// One workgroup (256 threads) per camera c, over its observations (camera-major):
//   A0 = sum F^T F, g_c = sum F^T f                                  (pass 1)
//   A = A0 + D_c, D_c = lambda diag(A0) (or explicit)
//   T = sum Y C_p^-1 Y^T, u = sum Y v_p, Y = F^T E                    (pass 2)
//   b = -g_c + u   (reduced right-hand side -g_c + W C^-1 g_p)
//   S_cc = A - T   (diagonal block of S) and its inverse (block Jacobi).
__global__ __launch_bounds__(256) void k_camera_blocks(
    const int32_t* __restrict__ cam_off, const int32_t* __restrict__ cam_obs,
    const int32_t* __restrict__ obs_pt, int64_t stride, const double* __restrict__ F,
    const double* __restrict__ E, const double* __restrict__ fres, const double* __restrict__ Cinv,
    const double* __restrict__ vgp, double lambda, const double* __restrict__ Dexp,
    double* __restrict__ A_out, float* __restrict__ A32, double* __restrict__ Dc_out,
    double* __restrict__ b_out, double* __restrict__ gc_out, double* __restrict__ Scc_out,
    double* __restrict__ Sinv, float* __restrict__ Sinv32, uint32_t* err) {
  __shared__ double red[4 * 54];
  __shared__ double S[81];
  __shared__ double Adiag[9], Ad[45];
  const int c = blockIdx.x;
  const int beg = cam_off[c], end = cam_off[c + 1];
  double acc[54];
  // ---- pass 1: A0 (45 packed) and g_c (9)
#pragma unroll
  for (int k = 0; k < 54; ++k) acc[k] = 0.0;
  for (int i = beg + threadIdx.x; i < end; i += blockDim.x) {
    const int o = cam_obs[i];
    double f[18];
#pragma unroll
    for (int k = 0; k < 18; ++k) f[k] = F[k * stride + o];
    const double r0 = fres[o], r1 = fres[stride + o];
    int idx = 0;
#pragma unroll
    for (int a = 0; a < 9; ++a)
#pragma unroll
      for (int bb = a; bb < 9; ++bb) acc[idx++] += f[a] * f[bb] + f[9 + a] * f[9 + bb];
#pragma unroll
    for (int a = 0; a < 9; ++a) acc[45 + a] += f[a] * r0 + f[9 + a] * r1;
  }
  block_reduce<54>(acc, red);
  if (threadIdx.x < 45) Ad[threadIdx.x] = red[threadIdx.x];
  if (threadIdx.x < 9) {
    const int a = threadIdx.x;
    const double a0 = red[sym_index(9, a, a)];
    const double dd = Dexp ? Dexp[(size_t)c * 9 + a] : lambda * a0;
    Adiag[a] = dd;
    Dc_out[(size_t)c * 9 + a] = dd;
    gc_out[(size_t)c * 9 + a] = red[45 + a];
  }
  __syncthreads();
  double gcv = threadIdx.x < 9 ? red[45 + threadIdx.x] : 0.0;
  if (threadIdx.x < 45) {
    // add damping on the diagonal of the packed matrix
    int i = 0, rem = threadIdx.x;
    while (rem >= 9 - i) { rem -= 9 - i; ++i; }
    const int j = i + rem;
    double v = Ad[threadIdx.x] + (i == j ? Adiag[i] : 0.0);
    Ad[threadIdx.x] = v;
    A_out[(size_t)c * 45 + threadIdx.x] = v;
    if (A32) A32[(size_t)c * 45 + threadIdx.x] = (float)v;
  }
  __syncthreads();
  // ---- pass 2: T = sum Y C^-1 Y^T (45 packed) and u = sum Y v_p (9)
#pragma unroll
  for (int k = 0; k < 54; ++k) acc[k] = 0.0;
  for (int i = beg + threadIdx.x; i < end; i += blockDim.x) {
    const int o = cam_obs[i];
    const int q = obs_pt[o];
    double f[18], e[6];
#pragma unroll
    for (int k = 0; k < 18; ++k) f[k] = F[k * stride + o];
#pragma unroll
    for (int k = 0; k < 6; ++k) e[k] = E[k * stride + o];
    const double* ci = Cinv + (size_t)q * 6;
    const double C[9] = {ci[0], ci[1], ci[2], ci[1], ci[3], ci[4], ci[2], ci[4], ci[5]};
    double Y[27], YC[27];
#pragma unroll
    for (int a = 0; a < 9; ++a)
#pragma unroll
      for (int k = 0; k < 3; ++k) Y[a * 3 + k] = f[a] * e[k] + f[9 + a] * e[3 + k];
#pragma unroll
    for (int a = 0; a < 9; ++a)
#pragma unroll
      for (int k = 0; k < 3; ++k)
        YC[a * 3 + k] = Y[a * 3 + 0] * C[0 * 3 + k] + Y[a * 3 + 1] * C[1 * 3 + k] + Y[a * 3 + 2] * C[2 * 3 + k];
    int idx = 0;
#pragma unroll
    for (int a = 0; a < 9; ++a)
#pragma unroll
      for (int bb = a; bb < 9; ++bb)
        acc[idx++] += YC[a * 3 + 0] * Y[bb * 3 + 0] + YC[a * 3 + 1] * Y[bb * 3 + 1] + YC[a * 3 + 2] * Y[bb * 3 + 2];
    const double v0 = vgp[(size_t)q * 3], v1 = vgp[(size_t)q * 3 + 1], v2 = vgp[(size_t)q * 3 + 2];
#pragma unroll
    for (int a = 0; a < 9; ++a) acc[45 + a] += Y[a * 3 + 0] * v0 + Y[a * 3 + 1] * v1 + Y[a * 3 + 2] * v2;
  }
  block_reduce<54>(acc, red);
  if (threadIdx.x < 9) b_out[(size_t)c * 9 + threadIdx.x] = -gcv + red[45 + threadIdx.x];
  if (threadIdx.x < 81) {
    const int i = threadIdx.x / 9, j = threadIdx.x % 9;
    const int a = i < j ? i : j, bb = i < j ? j : i;
    const int si = sym_index(9, a, bb);
    const double v = Ad[si] - red[si];
    S[threadIdx.x] = v;
    Scc_out[(size_t)c * 81 + threadIdx.x] = v;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double a[81], inv[81];
    for (int k = 0; k < 81; ++k) a[k] = S[k];
    if (!cholesky<9>(a)) {
      atomicOr(err, ERRF_NOT_SPD);
      for (int k = 0; k < 81; ++k) inv[k] = 0.0;
    } else {
      cholesky_inverse<9>(a, inv);
    }
    for (int k = 0; k < 81; ++k) S[k] = inv[k];
  }
  __syncthreads();
  if (threadIdx.x < 81) {
    Sinv[(size_t)c * 81 + threadIdx.x] = S[threadIdx.x];
    if (Sinv32) Sinv32[(size_t)c * 81 + threadIdx.x] = (float)S[threadIdx.x];
  }
}

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

// ---------------------------------------------------------------- camera-side half products

// out_c = sum_{o in c} F_o^T E_o v_{p(o)} (camera-major, one workgroup per camera).
// Used for right-hand sides b = r_c - W C^-1 r_p with v = C^-1 r_p.
__global__ __launch_bounds__(256) void k_cam_FtEv(const int32_t* __restrict__ cam_off,
                                                  const int32_t* __restrict__ cam_obs,
                                                  const int32_t* __restrict__ obs_pt, int64_t stride,
                                                  const double* __restrict__ F,
                                                  const double* __restrict__ E,
                                                  const double* __restrict__ v,
                                                  const double* __restrict__ base, double scale,
                                                  double* __restrict__ out) {
  __shared__ double red[4 * 9];
  const int c = blockIdx.x;
  double acc[9];
#pragma unroll
  for (int k = 0; k < 9; ++k) acc[k] = 0.0;
  for (int i = cam_off[c] + threadIdx.x; i < cam_off[c + 1]; i += blockDim.x) {
    const int o = cam_obs[i];
    const int q = obs_pt[o];
    const double v0 = v[(size_t)q * 3], v1 = v[(size_t)q * 3 + 1], v2 = v[(size_t)q * 3 + 2];
    const double w0 = E[0 * stride + o] * v0 + E[1 * stride + o] * v1 + E[2 * stride + o] * v2;
    const double w1 = E[3 * stride + o] * v0 + E[4 * stride + o] * v1 + E[5 * stride + o] * v2;
#pragma unroll
    for (int k = 0; k < 9; ++k) acc[k] += F[k * stride + o] * w0 + F[(9 + k) * stride + o] * w1;
  }
  block_reduce<9>(acc, red);
  if (threadIdx.x < 9)
    out[(size_t)c * 9 + threadIdx.x] = (base ? base[(size_t)c * 9 + threadIdx.x] : 0.0) + scale * red[threadIdx.x];
}

// Point recovery: x_p = C_p^-1 (r_p - sum_{o in p} E_o^T F_o x_c(o)), written in caller order.
// r_p is given in reordered point order (rp, may be NULL for 0) scaled by rscale.
__global__ __launch_bounds__(256) void k_recover_points(
    int n_pt, const int32_t* __restrict__ pt_off, const int32_t* __restrict__ pt_orig,
    const int32_t* __restrict__ obs_cam, int64_t stride, const double* __restrict__ F,
    const double* __restrict__ E, const double* __restrict__ Cinv, const double* __restrict__ rp,
    double rscale, const double* __restrict__ xc, double* __restrict__ out) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= n_pt) return;
  double z0 = 0, z1 = 0, z2 = 0;
  for (int o = pt_off[q]; o < pt_off[q + 1]; ++o) {
    const double* xv = xc + (size_t)obs_cam[o] * 9;
    double s0 = 0, s1 = 0;
#pragma unroll
    for (int k = 0; k < 9; ++k) { s0 += F[k * stride + o] * xv[k]; s1 += F[(9 + k) * stride + o] * xv[k]; }
    z0 += E[0 * stride + o] * s0 + E[3 * stride + o] * s1;
    z1 += E[1 * stride + o] * s0 + E[4 * stride + o] * s1;
    z2 += E[2 * stride + o] * s0 + E[5 * stride + o] * s1;
  }
  const double r0 = (rp ? rscale * rp[(size_t)q * 3] : 0.0) - z0;
  const double r1 = (rp ? rscale * rp[(size_t)q * 3 + 1] : 0.0) - z1;
  const double r2 = (rp ? rscale * rp[(size_t)q * 3 + 2] : 0.0) - z2;
  const double* ci = Cinv + (size_t)q * 6;
  const size_t qo = pt_orig[q];
  out[qo * 3 + 0] = ci[0] * r0 + ci[1] * r1 + ci[2] * r2;
  out[qo * 3 + 1] = ci[1] * r0 + ci[3] * r1 + ci[4] * r2;
  out[qo * 3 + 2] = ci[2] * r0 + ci[4] * r1 + ci[5] * r2;
}

// v_p = C_p^-1 r_p for a point vector given in caller order (gathered into reordered order).
__global__ void k_point_solve(int n_pt, const int32_t* __restrict__ pt_orig,
                              const double* __restrict__ Cinv, const double* __restrict__ r,
                              double* __restrict__ v, double* __restrict__ r_reordered) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= n_pt) return;
  const size_t qo = pt_orig[q];
  const double r0 = r[qo * 3], r1 = r[qo * 3 + 1], r2 = r[qo * 3 + 2];
  const double* ci = Cinv + (size_t)q * 6;
  v[(size_t)q * 3 + 0] = ci[0] * r0 + ci[1] * r1 + ci[2] * r2;
  v[(size_t)q * 3 + 1] = ci[1] * r0 + ci[3] * r1 + ci[4] * r2;
  v[(size_t)q * 3 + 2] = ci[2] * r0 + ci[4] * r1 + ci[5] * r2;
  if (r_reordered) {
    r_reordered[(size_t)q * 3] = r0;
    r_reordered[(size_t)q * 3 + 1] = r1;
    r_reordered[(size_t)q * 3 + 2] = r2;
  }
}

// C^-1 unpacked to [n][3][3] in caller point order.
__global__ void k_unpack_cinv(int n_pt, const int32_t* __restrict__ pt_orig,
                              const double* __restrict__ Cinv, double* __restrict__ out) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= n_pt) return;
  const double* ci = Cinv + (size_t)q * 6;
  double* o = out + (size_t)pt_orig[q] * 9;
  o[0] = ci[0]; o[1] = ci[1]; o[2] = ci[2];
  o[3] = ci[1]; o[4] = ci[3]; o[5] = ci[4];
  o[6] = ci[2]; o[7] = ci[4]; o[8] = ci[5];
}

}  // namespace bamg
