// Kernels of the Levenberg-Marquardt outer loop (Section 2.1): the cost
// 1/2 sum |f_o|^2 at candidate parameters, the decrease of the Gauss-Newton
// model m(delta) = 1/2 |f + J delta|^2 predicted for a step, and the
// candidate update x + delta. Sums are deterministic (per-block partials added
// in block order by the last block, as in the PCG kernels).
#include "kernels.hpp"

namespace bamg {

struct LmScal {
  double cost;       // 1/2 sum |f_o|^2 at the evaluated parameters
  double model;      // m(0) - m(delta)
  unsigned invalid;  // observations with x_cam.z >= 0 or a non-finite residual
  unsigned camflag;  // non-finite camera parameters (ERRF_NONFINITE)
  unsigned count[2];
};

__global__ void k_lm_clear(LmScal* s) {
  if (threadIdx.x == 0) {
    s->invalid = 0u;
    s->camflag = 0u;
    s->count[0] = s->count[1] = 0u;
  }
}

// Cost 1/2 sum rho(|f_o|^2) at (campre, pts) over the point-major observations.
// uv is in the caller's observation order (obs_orig maps to it), pts in caller
// point order.
__global__ __launch_bounds__(256) void k_lm_cost(int n_obs, const int32_t* __restrict__ obs_cam,
                                                 const int32_t* __restrict__ obs_pt,
                                                 const int32_t* __restrict__ pt_orig,
                                                 const int32_t* __restrict__ obs_orig,
                                                 const double* __restrict__ campre, const double* __restrict__ pts,
                                                 const double* __restrict__ uv, int loss, double loss_a,
                                                 double* __restrict__ partial, LmScal* s) {
  double v = 0.0;
  unsigned bad = 0;
  for (int o = blockIdx.x * 256 + threadIdx.x; o < n_obs; o += gridDim.x * 256) {
    const int c = obs_cam[o];
    const size_t p = (size_t)pt_orig[obs_pt[o]];
    const size_t i = (size_t)obs_orig[o];
    const double X[3] = {pts[3 * p], pts[3 * p + 1], pts[3 * p + 2]};
    double pi[2], Fo[18], Eo[6], z;
    project_jacobian(campre + (size_t)c * 24, X, pi, Fo, Eo, &z);
    const double f0 = pi[0] - uv[2 * i], f1 = pi[1] - uv[2 * i + 1];
    const double e = loss_value(f0 * f0 + f1 * f1, loss, loss_a);
    if (z < 0.0 && isfinite(e)) v += e;
    else ++bad;
  }
  if (bad) atomicAdd(&s->invalid, bad);
  double tot;
  if (!last_block_sum(v, partial, &s->count[0], &tot)) return;
  s->cost = 0.5 * tot;
}

// m(0) - m(delta) = -sum_o r_o . (f_o + r_o / 2) with r_o = F_o dc_c + E_o dp_p,
// from the Jacobian planes of the prepared step (point-major, stride `stride`).
// dc [n_cam][9], dp [n_pt][3] in the caller's order.
__global__ __launch_bounds__(256) void k_lm_model(int n_obs, int64_t stride, const int32_t* __restrict__ obs_cam,
                                                  const int32_t* __restrict__ obs_pt,
                                                  const int32_t* __restrict__ pt_orig,
                                                  const double* __restrict__ F, const double* __restrict__ E,
                                                  const double* __restrict__ fres, const double* __restrict__ dc,
                                                  const double* __restrict__ dp, double* __restrict__ partial,
                                                  LmScal* s) {
  double v = 0.0;
  for (int o = blockIdx.x * 256 + threadIdx.x; o < n_obs; o += gridDim.x * 256) {
    const double* x = dc + (size_t)obs_cam[o] * 9;
    const double* y = dp + (size_t)pt_orig[obs_pt[o]] * 3;
    double r[2];
#pragma unroll
    for (int k = 0; k < 2; ++k) {
      double a = 0.0;
#pragma unroll
      for (int j = 0; j < 9; ++j) a += F[(size_t)(k * 9 + j) * stride + o] * x[j];
#pragma unroll
      for (int j = 0; j < 3; ++j) a += E[(size_t)(k * 3 + j) * stride + o] * y[j];
      r[k] = a;
    }
    v -= r[0] * (fres[o] + 0.5 * r[0]) + r[1] * (fres[stride + o] + 0.5 * r[1]);
  }
  double tot;
  if (!last_block_sum(v, partial, &s->count[1], &tot)) return;
  s->model = tot;
}

}  // namespace bamg
