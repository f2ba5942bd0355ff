// Adjoint of one LM step (differentiation form; not part of the paper).
//
// With f = pi(x) - u, H = J^T J + lam diag(J^T J), H delta = -J^T f and an
// upstream gradient gbar = dL/d delta, mu = H^-1 gbar gives
//   dL/du_o = J_o mu_o,
//   dL/dx   = -J^T (J mu) - sum_o sum_r Hess(pi_{o,r}) w_{o,r},
//   w_{o,r} = (f_{o,r} + (J_o delta_o)_r) mu_o + (J_o mu_o)_r delta_o
//             + 2 lam (mu_o * delta_o * J_o[r, :])    (dropped when D is frozen),
// mu_o, delta_o being the 12-vectors (camera, point) of observation o.
// Hess(pi_{o,r}) w is the directional derivative of row r of J_o along w,
// computed here by evaluating the Jacobian on 2-tangent dual numbers.
#include "kernels.hpp"

namespace bamg {

// value + two tangents
struct Dual2 {
  double v, d0, d1;
};
__device__ __forceinline__ Dual2 D2(double v) { return {v, 0.0, 0.0}; }
__device__ __forceinline__ Dual2 operator+(Dual2 a, Dual2 b) { return {a.v + b.v, a.d0 + b.d0, a.d1 + b.d1}; }
__device__ __forceinline__ Dual2 operator-(Dual2 a, Dual2 b) { return {a.v - b.v, a.d0 - b.d0, a.d1 - b.d1}; }
__device__ __forceinline__ Dual2 operator-(Dual2 a) { return {-a.v, -a.d0, -a.d1}; }
__device__ __forceinline__ Dual2 operator*(Dual2 a, Dual2 b) {
  return {a.v * b.v, a.d0 * b.v + a.v * b.d0, a.d1 * b.v + a.v * b.d1};
}
__device__ __forceinline__ Dual2 operator/(Dual2 a, Dual2 b) {
  const double iv = 1.0 / b.v, q = a.v * iv;
  return {q, (a.d0 - q * b.d0) * iv, (a.d1 - q * b.d1) * iv};
}
__device__ __forceinline__ Dual2 operator+(Dual2 a, double b) { return {a.v + b, a.d0, a.d1}; }
__device__ __forceinline__ Dual2 operator+(double b, Dual2 a) { return {a.v + b, a.d0, a.d1}; }
__device__ __forceinline__ Dual2 operator-(Dual2 a, double b) { return {a.v - b, a.d0, a.d1}; }
__device__ __forceinline__ Dual2 operator-(double b, Dual2 a) { return {b - a.v, -a.d0, -a.d1}; }
__device__ __forceinline__ Dual2 operator*(Dual2 a, double b) { return {a.v * b, a.d0 * b, a.d1 * b}; }
__device__ __forceinline__ Dual2 operator*(double b, Dual2 a) { return {a.v * b, a.d0 * b, a.d1 * b}; }
__device__ __forceinline__ Dual2 operator/(Dual2 a, double b) { return {a.v / b, a.d0 / b, a.d1 / b}; }
__device__ __forceinline__ Dual2 operator/(double a, Dual2 b) { return D2(a) / b; }
__device__ __forceinline__ Dual2 dsin(Dual2 a) {
  const double c = cos(a.v);
  return {sin(a.v), c * a.d0, c * a.d1};
}
__device__ __forceinline__ Dual2 dcos(Dual2 a) {
  const double s = -sin(a.v);
  return {cos(a.v), s * a.d0, s * a.d1};
}
__device__ __forceinline__ Dual2 dsqrt(Dual2 a) {
  const double r = sqrt(a.v);
  const double h = r > 0.0 ? 0.5 / r : 0.0;
  return {r, h * a.d0, h * a.d1};
}
__device__ __forceinline__ double dval(Dual2 a) { return a.v; }
__device__ __forceinline__ double dval(double a) { return a; }
__device__ __forceinline__ double dsin(double a) { return sin(a); }
__device__ __forceinline__ double dcos(double a) { return cos(a); }
__device__ __forceinline__ double dsqrt(double a) { return sqrt(a); }

// Reprojection Jacobian straight from the camera parameters, generic in the
// scalar type (same model as the forward kernel: R = I + a[w]x + b[w]x^2,
// d pi/dw = -E [X]x J_r, J_r = I - b [w]x + c [w]x^2).
template <class T>
__device__ __forceinline__ void jacobian_generic(const T cam[9], const T X[3], T Fo[18], T Eo[6]) {
  const T w0 = cam[0], w1 = cam[1], w2 = cam[2];
  const T t2 = w0 * w0 + w1 * w1 + w2 * w2;
  const T th = dsqrt(t2);
  const double thv = dval(th);
  // a = sin(th)/th, b = (1 - cos th)/th^2 = 1/2 sinc(th/2)^2, c = (th - sin th)/th^3
  T a, b, c;
  if (thv < 0.25) {
    a = 1.0 + t2 * (-1.0 / 6.0 + t2 * (1.0 / 120.0 + t2 * (-1.0 / 5040.0 + t2 * (1.0 / 362880.0))));
    b = 0.5 + t2 * (-1.0 / 24.0 + t2 * (1.0 / 720.0 + t2 * (-1.0 / 40320.0 + t2 * (1.0 / 3628800.0))));
    c = 1.0 / 6.0 + t2 * (-1.0 / 120.0 + t2 * (1.0 / 5040.0 + t2 * (-1.0 / 362880.0 + t2 * (1.0 / 39916800.0))));
  } else {
    const T s = dsin(th);
    a = s / th;
    const T h = dsin(th * 0.5) / (th * 0.5);
    b = 0.5 * h * h;
    c = (th - s) / (t2 * th);
  }
  const T xx = w0 * w0, yy = w1 * w1, zz = w2 * w2, xy = w0 * w1, xz = w0 * w2, yz = w1 * w2;
  T R[9], J[9];
  R[0] = 1.0 - b * (yy + zz); R[1] = -(a * w2) + b * xy;   R[2] = a * w1 + b * xz;
  R[3] = a * w2 + b * xy;     R[4] = 1.0 - b * (xx + zz);  R[5] = -(a * w0) + b * yz;
  R[6] = -(a * w1) + b * xz;  R[7] = a * w0 + b * yz;      R[8] = 1.0 - b * (xx + yy);
  J[0] = 1.0 - c * (yy + zz); J[1] = b * w2 + c * xy;      J[2] = -(b * w1) + c * xz;
  J[3] = -(b * w2) + c * xy;  J[4] = 1.0 - c * (xx + zz);  J[5] = b * w0 + c * yz;
  J[6] = b * w1 + c * xz;     J[7] = -(b * w0) + c * yz;   J[8] = 1.0 - c * (xx + yy);
  const T xc = R[0] * X[0] + R[1] * X[1] + R[2] * X[2] + cam[3];
  const T yc = R[3] * X[0] + R[4] * X[1] + R[5] * X[2] + cam[4];
  const T zc = R[6] * X[0] + R[7] * X[1] + R[8] * X[2] + cam[5];
  const T f = cam[6], k1 = cam[7], k2 = cam[8];
  const T iz = 1.0 / zc;
  const T p0 = -(xc * iz), p1 = -(yc * iz);
  const T n2 = p0 * p0 + p1 * p1;
  const T r = 1.0 + n2 * (k1 + k2 * n2);
  const T d = 2.0 * k1 + 4.0 * k2 * n2;
  const T m00 = f * (r + d * p0 * p0), m01 = f * d * p0 * p1, m11 = f * (r + d * p1 * p1);
  T M[6];
  M[0] = -(iz * m00);
  M[1] = -(iz * m01);
  M[2] = -(iz * (m00 * p0 + m01 * p1));
  M[3] = -(iz * m01);
  M[4] = -(iz * m11);
  M[5] = -(iz * (m01 * p0 + m11 * p1));
  for (int rr = 0; rr < 2; ++rr) {
    for (int cc = 0; cc < 3; ++cc)
      Eo[rr * 3 + cc] = M[rr * 3 + 0] * R[cc] + M[rr * 3 + 1] * R[3 + cc] + M[rr * 3 + 2] * R[6 + cc];
    const T e0 = Eo[rr * 3 + 0], e1 = Eo[rr * 3 + 1], e2 = Eo[rr * 3 + 2];
    const T g0 = e1 * X[2] - e2 * X[1];
    const T g1 = e2 * X[0] - e0 * X[2];
    const T g2 = e0 * X[1] - e1 * X[0];
    for (int cc = 0; cc < 3; ++cc) Fo[rr * 9 + cc] = -(g0 * J[cc] + g1 * J[3 + cc] + g2 * J[6 + cc]);
    for (int cc = 0; cc < 3; ++cc) Fo[rr * 9 + 3 + cc] = M[rr * 3 + cc];
    const T pr = rr == 0 ? p0 : p1;
    Fo[rr * 9 + 6] = r * pr;
    Fo[rr * 9 + 7] = f * n2 * pr;
    Fo[rr * 9 + 8] = f * n2 * n2 * pr;
  }
}

// Per observation: dL/du, and the 12-vector -J_o^T J_o mu_o - sum_r Hess_r w_r,
// written as planes tcam[9][stride], tpt[3][stride] (reduced afterwards).
__global__ __launch_bounds__(256) void k_adjoint_obs(
    int n_obs, const int32_t* __restrict__ obs_cam, const int32_t* __restrict__ obs_pt,
    const int32_t* __restrict__ obs_orig, const int32_t* __restrict__ pt_orig, int64_t stride,
    const double* __restrict__ F, const double* __restrict__ E, const double* __restrict__ fres,
    const double* __restrict__ cams, const double* __restrict__ pts, const double* __restrict__ mu_c,
    const double* __restrict__ mu_p, const double* __restrict__ de_c, const double* __restrict__ de_p,
    double lambda, int freeze, double* __restrict__ g_uv, double* __restrict__ tcam,
    double* __restrict__ tpt) {
  const int o = blockIdx.x * blockDim.x + threadIdx.x;
  if (o >= n_obs) return;
  const int c = obs_cam[o];
  const int qo = pt_orig[obs_pt[o]];
  double Jr[2][12], mu[12], de[12];
  for (int k = 0; k < 9; ++k) {
    Jr[0][k] = F[k * stride + o];
    Jr[1][k] = F[(9 + k) * stride + o];
    mu[k] = mu_c[(size_t)c * 9 + k];
    de[k] = de_c[(size_t)c * 9 + k];
  }
  for (int k = 0; k < 3; ++k) {
    Jr[0][9 + k] = E[k * stride + o];
    Jr[1][9 + k] = E[(3 + k) * stride + o];
    mu[9 + k] = mu_p[(size_t)qo * 3 + k];
    de[9 + k] = de_p[(size_t)qo * 3 + k];
  }
  double Jmu[2], Jde[2];
  for (int r = 0; r < 2; ++r) {
    double a = 0.0, b = 0.0;
    for (int k = 0; k < 12; ++k) { a += Jr[r][k] * mu[k]; b += Jr[r][k] * de[k]; }
    Jmu[r] = a;
    Jde[r] = b;
  }
  const size_t oo = obs_orig[o];
  g_uv[oo * 2] = Jmu[0];
  g_uv[oo * 2 + 1] = Jmu[1];
  // directions w_{o,0}, w_{o,1} as the two tangents
  const double fr[2] = {fres[o], fres[stride + o]};
  Dual2 cam[9], X[3];
  for (int k = 0; k < 12; ++k) {
    double w[2];
    for (int r = 0; r < 2; ++r) {
      w[r] = (fr[r] + Jde[r]) * mu[k] + Jmu[r] * de[k];
      if (!freeze) w[r] += 2.0 * lambda * mu[k] * de[k] * Jr[r][k];
    }
    const double v = k < 9 ? cams[(size_t)c * 9 + k] : pts[(size_t)qo * 3 + (k - 9)];
    const Dual2 dv = {v, w[0], w[1]};
    if (k < 9) cam[k] = dv; else X[k - 9] = dv;
  }
  Dual2 Fd[18], Ed[6];
  jacobian_generic<Dual2>(cam, X, Fd, Ed);
  for (int k = 0; k < 12; ++k) {
    const double h0 = k < 9 ? Fd[k].d0 : Ed[k - 9].d0;          // row 0, tangent 0
    const double h1 = k < 9 ? Fd[9 + k].d1 : Ed[3 + k - 9].d1;  // row 1, tangent 1
    const double first = -(Jr[0][k] * Jmu[0] + Jr[1][k] * Jmu[1]);
    const double t = first - h0 - h1;
    if (k < 9) tcam[k * stride + o] = t;
    else tpt[(k - 9) * stride + o] = t;
  }
}

// g_pts[orig(q)] = sum over the point's observations of tpt
__global__ void k_adjoint_points(int n_pt, const int32_t* __restrict__ pt_off, const int32_t* __restrict__ pt_orig,
                                 int64_t stride, const double* __restrict__ tpt, double* __restrict__ g_pts) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= n_pt) return;
  double s[3] = {0, 0, 0};
  for (int o = pt_off[q]; o < pt_off[q + 1]; ++o)
    for (int k = 0; k < 3; ++k) s[k] += tpt[k * stride + o];
  const size_t qo = pt_orig[q];
  for (int k = 0; k < 3; ++k) g_pts[qo * 3 + k] = s[k];
}

// g_cams[c] = sum over the camera's observations of tcam (one workgroup per camera)
__global__ __launch_bounds__(256) void k_adjoint_cameras(const int32_t* __restrict__ cam_off,
                                                         const int32_t* __restrict__ cam_obs, int64_t stride,
                                                         const double* __restrict__ tcam,
                                                         double* __restrict__ g_cams) {
  __shared__ double red[4 * 9];
  const int c = blockIdx.x;
  double acc[9];
  for (int k = 0; k < 9; ++k) acc[k] = 0.0;
  for (int i = cam_off[c] + threadIdx.x; i < cam_off[c + 1]; i += blockDim.x) {
    const int o = cam_obs[i];
    for (int k = 0; k < 9; ++k) acc[k] += tcam[k * stride + o];
  }
  block_reduce<9>(acc, red);
  if (threadIdx.x < 9) g_cams[(size_t)c * 9 + threadIdx.x] = red[threadIdx.x];
}

}  // namespace bamg
