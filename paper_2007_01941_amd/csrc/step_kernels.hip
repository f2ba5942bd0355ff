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

// ---------------------------------------------------------------- robust loss

// The Huber loss of Section 5.4 on s = |f_o|^2 with scale a: rho(s) = s for
// s <= a^2, 2 a sqrt(s) - a^2 above (the squared loss is rho(s) = s).
__device__ __forceinline__ double loss_value(double s, int loss, double a) {
  return (loss == BA_LOSS_HUBER && s > a * a) ? 2.0 * a * sqrt(s) - a * a : s;
}

// sqrt(rho'(s)): the weight of an observation's residual and Jacobian rows in
// the reweighted step (rho' = a / sqrt(s) above the threshold).
__device__ __forceinline__ double loss_sqrt_weight(double s, int loss, double a) {
  return (loss == BA_LOSS_HUBER && s > a * a) ? sqrt(a / sqrt(s)) : 1.0;
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

// ---------------------------------------------------------------- Jacobian + point blocks

// C_p^-1 and the derived point quantities from the sums C0 = sum E^T E (packed 6)
// and g = sum E^T f of one point q (reordered index; qo = caller index).
// D_p = lambda diag(C0), or the explicit diagonal Dexp (caller order).
__device__ __forceinline__ void finish_point(int q, int qo, const double C[6], const double g[3], double lambda,
                                             const double* __restrict__ Dexp, int n_cam,
                                             const double* __restrict__ pts, double* __restrict__ Cinv,
                                             float* __restrict__ Cinv32, double* __restrict__ vgp,
                                             double* __restrict__ gp_out, double* __restrict__ Dp_out,
                                             double* __restrict__ prec, uint32_t* err) {
  double d[3];
  if (Dexp) {
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
  double v[3];
  for (int k = 0; k < 3; ++k) v[k] = inv[k * 3 + 0] * g[0] + inv[k * 3 + 1] * g[1] + inv[k * 3 + 2] * g[2];
  double* rec = prec + (size_t)q * PREC;
  for (int k = 0; k < 3; ++k) rec[k] = pts[(size_t)qo * 3 + k];
  for (int k = 0; k < 6; ++k) {
    Cinv[(size_t)q * 6 + k] = ci[k];
    rec[3 + k] = ci[k];
    if (Cinv32) Cinv32[(size_t)q * 6 + k] = (float)ci[k];
  }
  for (int k = 0; k < 3; ++k) {
    vgp[(size_t)q * 3 + k] = v[k];
    rec[9 + k] = v[k];
    gp_out[(size_t)q * 3 + k] = g[k];
    Dp_out[(size_t)q * 3 + k] = d[k];
  }
}

// Residual, Jacobian blocks and the point side of the normal equations in one
// pass, one workgroup per tile of whole points (one thread per observation):
// writes f, F, E (and FP32 copies); sums C0 = sum E^T E and g_p = sum E^T f per
// point in LDS; then per point C_p = C0 + D_p, C_p^-1 (packed), v_p = C_p^-1 g_p,
// and the point record [X | C_p^-1 | v_p] read by the camera-side kernels.
// With a robust loss (wsq non-null) every observation's rows are scaled by
// sqrt(rho'(|f_o|^2)), stored in wsq for the kernels that recompute F_o, E_o.
// F, E may be NULL: the planes are then not written (the step recomputes the
// blocks where it needs them).
__global__ __launch_bounds__(256) void k_jacobian_tiles(
    const int32_t* __restrict__ tile_obs, const int32_t* __restrict__ tile_pt,
    const int32_t* __restrict__ pt_off, const uint32_t* __restrict__ obs_slot,
    const int32_t* __restrict__ obs_cam, const int32_t* __restrict__ obs_orig,
    const int32_t* __restrict__ pt_orig,
    const double* __restrict__ campre, const double* __restrict__ pts, const double* __restrict__ uv,
    int64_t stride, double lambda, const double* __restrict__ Dexp, int n_cam, double* __restrict__ F,
    double* __restrict__ E, double* __restrict__ fres, float* __restrict__ F32, float* __restrict__ E32,
    double* __restrict__ Cinv, float* __restrict__ Cinv32, double* __restrict__ vgp,
    double* __restrict__ gp_out, double* __restrict__ Dp_out, double* __restrict__ prec, int n_tiles,
    int loss, double loss_a, double* __restrict__ wsq, uint32_t* err) {
  // per-observation contributions [E^T E (6) | E^T f (3)], summed per point in
  // observation order afterwards (deterministic, no atomics)
  __shared__ double part[9][TILE_OBS];
  const int t = xcd_block(blockIdx.x, n_tiles);
  if (t >= n_tiles) return;
  const int o0 = tile_obs[t], o1 = tile_obs[t + 1];
  const int q0 = tile_pt[t], np = tile_pt[t + 1] - q0;
  double sum[9];
#pragma unroll
  for (int k = 0; k < 9; ++k) sum[k] = 0.0;
  // more than TILE_OBS observations only for a tile holding one point
  for (int o = o0 + threadIdx.x; o < o1; o += TILE_OBS) {
    const int c = obs_cam[o];
    const int pl = (int)((obs_slot[o] >> 16) & 0xffu);
    const int qo = pt_orig[q0 + pl];
    const int oo = obs_orig[o];
    const double X[3] = {pts[(size_t)qo * 3 + 0], pts[(size_t)qo * 3 + 1], pts[(size_t)qo * 3 + 2]};
    double pi[2], Fo[18], e[6], z;
    project_jacobian(campre + (size_t)c * 24, X, pi, Fo, e, &z);
    double r0 = pi[0] - uv[(size_t)oo * 2 + 0];
    double r1 = pi[1] - uv[(size_t)oo * 2 + 1];
    if (!(z < 0.0)) atomicOr(err, ERRF_GEOMETRY);
    if (!isfinite(r0) || !isfinite(r1) || !isfinite(X[0] + X[1] + X[2])) atomicOr(err, ERRF_NONFINITE);
    if (wsq) {
      // robust loss: the reweighted rows sqrt(rho') [f_o | F_o | E_o]
      const double sw = loss_sqrt_weight(r0 * r0 + r1 * r1, loss, loss_a);
      wsq[o] = sw;
      r0 *= sw;
      r1 *= sw;
#pragma unroll
      for (int k = 0; k < 18; ++k) Fo[k] *= sw;
#pragma unroll
      for (int k = 0; k < 6; ++k) e[k] *= sw;
    }
    fres[o] = r0;
    fres[stride + o] = r1;
    if (F) {
#pragma unroll
      for (int k = 0; k < 18; ++k) F[k * stride + o] = Fo[k];
#pragma unroll
      for (int k = 0; k < 6; ++k) E[k * stride + o] = e[k];
    }
    if (F32) {
#pragma unroll
      for (int k = 0; k < 18; ++k) F32[k * stride + o] = (float)Fo[k];
#pragma unroll
      for (int k = 0; k < 6; ++k) E32[k * stride + o] = (float)e[k];
    }
    sum[0] += e[0] * e[0] + e[3] * e[3];
    sum[1] += e[0] * e[1] + e[3] * e[4];
    sum[2] += e[0] * e[2] + e[3] * e[5];
    sum[3] += e[1] * e[1] + e[4] * e[4];
    sum[4] += e[1] * e[2] + e[4] * e[5];
    sum[5] += e[2] * e[2] + e[5] * e[5];
    sum[6] += e[0] * r0 + e[3] * r1;
    sum[7] += e[1] * r0 + e[4] * r1;
    sum[8] += e[2] * r0 + e[5] * r1;
  }
#pragma unroll
  for (int k = 0; k < 9; ++k) part[k][threadIdx.x] = sum[k];
  __syncthreads();
  for (int i = threadIdx.x; i < np; i += 256) {
    const int q = q0 + i;
    int l0 = pt_off[q] - o0, l1 = pt_off[q + 1] - o0;
    if (l1 - l0 > TILE_OBS) { l0 = 0; l1 = TILE_OBS; }
    double C[6] = {0, 0, 0, 0, 0, 0}, g[3] = {0, 0, 0};
    for (int l = l0; l < l1; ++l) {
#pragma unroll
      for (int k = 0; k < 6; ++k) C[k] += part[k][l];
#pragma unroll
      for (int k = 0; k < 3; ++k) g[k] += part[6 + k][l];
    }
    finish_point(q, pt_orig[q], C, g, lambda, Dexp, n_cam, pts, Cinv, Cinv32, vgp, gp_out, Dp_out, prec,
                 err);
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

// Workgroup (256 threads) sum of 64 per-thread values: wave reduce-scatter,
// then the 4 waves' totals through LDS. On return red[0 .. 64) holds the sums.
__device__ __forceinline__ void block_reduce64(double (&acc)[64], double* red /*[4][64]*/) {
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  wave_reduce_scatter<64>(acc);
  if (!(lane & 1)) {
    red[wid * 64 + (lane & ~1)] = acc[0];
    red[wid * 64 + (lane & ~1) + 1] = acc[1];
  }
  __syncthreads();
  if (threadIdx.x < 64)
    red[threadIdx.x] = red[threadIdx.x] + red[64 + threadIdx.x] + red[128 + threadIdx.x] + red[192 + threadIdx.x];
  __syncthreads();
}

// One workgroup (256 threads) per camera c over its observations (camera-major
// list), recomputing F_o and E_o from the camera and the point record instead
// of gathering them from the point-major planes:
//   pass 1:  A0 = sum F^T F;  A = A0 + D_c, D_c = lambda diag(A0) (or explicit)
//   pass 2:  T = sum F^T M F with M = E C_p^-1 E^T (2 x 2), the camera's share
//            of W C^-1 W^T;  b = sum F^T (E v_p - f) = -g_c + W C^-1 g_p
//   S_cc = A - T (diagonal block of S) and its inverse (block Jacobi).
// With a robust loss the recomputed rows are scaled by the stored sqrt(rho').
__global__ __launch_bounds__(256) void k_camera_blocks(
    const int32_t* __restrict__ cam_off, const int32_t* __restrict__ cam_obs,
    const int32_t* __restrict__ cam_q, int64_t stride, const double* __restrict__ campre,
    const double* __restrict__ prec, const double* __restrict__ fres, double lambda,
    const double* __restrict__ Dexp, double* __restrict__ A_out, float* __restrict__ A32,
    double* __restrict__ Dc_out, double* __restrict__ b_out, double* __restrict__ Scc_out,
    double* __restrict__ Sinv, float* __restrict__ Sinv32, int n_cam, const double* __restrict__ wsq,
    uint32_t* err) {
  __shared__ double red[4 * 64];
  __shared__ double S[81];
  __shared__ double Adiag[9], Ad[45];
  const int c = xcd_block(blockIdx.x, n_cam);
  if (c >= n_cam) return;
  const int beg = cam_off[c], end = cam_off[c + 1];
  const double* cp = campre + (size_t)c * 24;
  double acc[64];
  // ---- pass 1: A0 (45 packed)
#pragma unroll
  for (int k = 0; k < 64; ++k) acc[k] = 0.0;
  for (int i = beg + threadIdx.x; i < end; i += blockDim.x) {
    const double* rec = prec + (size_t)cam_q[i] * PREC;
    const double X[3] = {rec[0], rec[1], rec[2]};
    double pi[2], f[18], e[6], z;
    project_jacobian(cp, X, pi, f, e, &z);
    if (wsq) {
      const double sw = wsq[cam_obs[i]];
#pragma unroll
      for (int k = 0; k < 18; ++k) f[k] *= sw;
    }
    int idx = 0;
#pragma unroll
    for (int a = 0; a < 9; ++a)
#pragma unroll
      for (int bb = a; bb < 9; ++bb) acc[idx++] += f[a] * f[bb] + f[9 + a] * f[9 + bb];
  }
  block_reduce64(acc, red);
  if (threadIdx.x < 45) Ad[threadIdx.x] = red[threadIdx.x];
  if (threadIdx.x < 9) {
    const int a = threadIdx.x;
    const double a0 = red[sym_index(9, a, a)];
    const double dd = Dexp ? Dexp[(size_t)c * 9 + a] : lambda * a0;
    Adiag[a] = dd;
    Dc_out[(size_t)c * 9 + a] = dd;
  }
  __syncthreads();
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
  // ---- pass 2: T (45 packed) and b (9)
#pragma unroll
  for (int k = 0; k < 64; ++k) acc[k] = 0.0;
  for (int i = beg + threadIdx.x; i < end; i += blockDim.x) {
    const int o = cam_obs[i];
    const double* rec = prec + (size_t)cam_q[i] * PREC;
    const double X[3] = {rec[0], rec[1], rec[2]};
    const double C[9] = {rec[3], rec[4], rec[5], rec[4], rec[6], rec[7], rec[5], rec[7], rec[8]};
    const double v0 = rec[9], v1 = rec[10], v2 = rec[11];
    const double f0 = fres[o], f1 = fres[stride + o];
    double pi[2], f[18], e[6], z;
    project_jacobian(cp, X, pi, f, e, &z);
    if (wsq) {
      const double sw = wsq[o];
#pragma unroll
      for (int k = 0; k < 18; ++k) f[k] *= sw;
#pragma unroll
      for (int k = 0; k < 6; ++k) e[k] *= sw;
    }
    double ec[6];
#pragma unroll
    for (int r = 0; r < 2; ++r)
#pragma unroll
      for (int k = 0; k < 3; ++k)
        ec[r * 3 + k] = e[r * 3 + 0] * C[0 * 3 + k] + e[r * 3 + 1] * C[1 * 3 + k] + e[r * 3 + 2] * C[2 * 3 + k];
    const double m00 = ec[0] * e[0] + ec[1] * e[1] + ec[2] * e[2];
    const double m01 = ec[0] * e[3] + ec[1] * e[4] + ec[2] * e[5];
    const double m11 = ec[3] * e[3] + ec[4] * e[4] + ec[5] * e[5];
    double mf[18];
#pragma unroll
    for (int k = 0; k < 9; ++k) {
      mf[k] = m00 * f[k] + m01 * f[9 + k];
      mf[9 + k] = m01 * f[k] + m11 * f[9 + k];
    }
    int idx = 0;
#pragma unroll
    for (int a = 0; a < 9; ++a)
#pragma unroll
      for (int bb = a; bb < 9; ++bb) acc[idx++] += f[a] * mf[bb] + f[9 + a] * mf[9 + bb];
    const double w0 = e[0] * v0 + e[1] * v1 + e[2] * v2 - f0;
    const double w1 = e[3] * v0 + e[4] * v1 + e[5] * v2 - f1;
#pragma unroll
    for (int a = 0; a < 9; ++a) acc[45 + a] += f[a] * w0 + f[9 + a] * w1;
  }
  block_reduce64(acc, red);
  if (threadIdx.x < 9) b_out[(size_t)c * 9 + threadIdx.x] = red[45 + threadIdx.x];
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

// Point recovery: x_p = C_p^-1 (rscale r_p - sum_{o in p} E_o^T F_o x_c(o)), written
// in caller order; r_p is in reordered point order (rp may be NULL for 0). One
// workgroup per tile of whole points, one thread per observation (coalesced
// plane reads); per-observation terms are summed per point in order.
// F == NULL: F_o and E_o are recomputed from the camera (campre) and the
// point record (prec) with the Jacobian kernel's projection, times the robust
// weight wsq[o] when wsq is given, instead of read from the planes.
__global__ __launch_bounds__(256) void k_recover_tiles(
    const int32_t* __restrict__ tile_obs, const int32_t* __restrict__ tile_pt,
    const int32_t* __restrict__ pt_off, const int32_t* __restrict__ pt_orig,
    const int32_t* __restrict__ obs_cam, int64_t stride, const double* __restrict__ F,
    const double* __restrict__ E, const int32_t* __restrict__ obs_pt, const double* __restrict__ campre,
    const double* __restrict__ prec, const double* __restrict__ wsq, const double* __restrict__ Cinv,
    const double* __restrict__ rp, double rscale, const double* __restrict__ xc, double* __restrict__ out,
    int n_tiles) {
  __shared__ double part[3][TILE_OBS];
  const int t = xcd_block(blockIdx.x, n_tiles);
  if (t >= n_tiles) return;
  const int o0 = tile_obs[t], o1 = tile_obs[t + 1];
  const int q0 = tile_pt[t], np = tile_pt[t + 1] - q0;
  double z0 = 0, z1 = 0, z2 = 0;
  for (int o = o0 + threadIdx.x; o < o1; o += TILE_OBS) {
    const int c = obs_cam[o];
    const double* xv = xc + (size_t)c * 9;
    double f[18], e[6];
    if (F) {
#pragma unroll
      for (int k = 0; k < 18; ++k) f[k] = F[k * stride + o];
#pragma unroll
      for (int k = 0; k < 6; ++k) e[k] = E[k * stride + o];
    } else {
      const double* rec = prec + (size_t)obs_pt[o] * PREC;
      const double X[3] = {rec[0], rec[1], rec[2]};
      double pi[2], z;
      project_jacobian(campre + (size_t)c * 24, X, pi, f, e, &z);
      if (wsq) {
        const double w = wsq[o];
#pragma unroll
        for (int k = 0; k < 18; ++k) f[k] *= w;
#pragma unroll
        for (int k = 0; k < 6; ++k) e[k] *= w;
      }
    }
    double s0 = 0, s1 = 0;
#pragma unroll
    for (int k = 0; k < 9; ++k) { s0 += f[k] * xv[k]; s1 += f[9 + k] * xv[k]; }
    z0 += e[0] * s0 + e[3] * s1;
    z1 += e[1] * s0 + e[4] * s1;
    z2 += e[2] * s0 + e[5] * s1;
  }
  part[0][threadIdx.x] = z0;
  part[1][threadIdx.x] = z1;
  part[2][threadIdx.x] = z2;
  __syncthreads();
  for (int i = threadIdx.x; i < np; i += 256) {
    const int q = q0 + i;
    int l0 = pt_off[q] - o0, l1 = pt_off[q + 1] - o0;
    if (l1 - l0 > TILE_OBS) { l0 = 0; l1 = TILE_OBS; }
    double y0 = 0, y1 = 0, y2 = 0;
    for (int l = l0; l < l1; ++l) { y0 += part[0][l]; y1 += part[1][l]; y2 += part[2][l]; }
    const double r0 = (rp ? rscale * rp[(size_t)q * 3] : 0.0) - y0;
    const double r1 = (rp ? rscale * rp[(size_t)q * 3 + 1] : 0.0) - y1;
    const double r2 = (rp ? rscale * rp[(size_t)q * 3 + 2] : 0.0) - y2;
    const double* ci = Cinv + (size_t)q * 6;
    const size_t qo = pt_orig[q];
    out[qo * 3 + 0] = ci[0] * r0 + ci[1] * r1 + ci[2] * r2;
    out[qo * 3 + 1] = ci[1] * r0 + ci[3] * r1 + ci[4] * r2;
    out[qo * 3 + 2] = ci[2] * r0 + ci[4] * r1 + ci[5] * r2;
  }
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
