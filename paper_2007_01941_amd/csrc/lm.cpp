// The Levenberg-Marquardt outer loop (Section 2.1) with the solver settings of
// Section 5: a trust region whose radius starts at 1e4 (damping
// D = diag(J^T J) / radius) and, optionally, the Nash-Sofer forcing rule for
// the inner PCG. The paper leaves the radius update to its nonlinear solver;
// this loop uses the update of Madsen, Nielsen and Tingleff, "Methods for
// non-linear least squares problems" (2004), Section 3.2, in radius form:
// a step with rho > min_relative_decrease is accepted,
// radius /= max(1/3, 1 - (2 rho - 1)^3) and nu = 2; otherwise radius /= nu
// and nu *= 2. Parameters are updated additively; a candidate that puts a
// point at or behind an observing camera, or whose cost is not finite, is
// rejected like any other failed step, and so is a step whose damped system is
// not numerically positive definite. With the Huber loss the cost is
// 1/2 sum rho(|f_o|^2) and the model that of the reweighted step.
namespace bamg {

static LmWork& lm_work(ba_plan* P) { return *P->lm; }

// Enqueue the cost at (cams, pts) into L.scal (cost, invalid, camflag).
static void enqueue_cost(ba_plan* P, LmWork& L, const ba_opts* o, const double* cams, const double* pts,
                         const double* uv, hipStream_t s) {
  const int loss = o ? o->loss : BA_LOSS_SQUARED;
  const double a = o ? o->loss_scale : 1.0;
  Scratch& W = *P->scratch;
  hipLaunchKernelGGL(k_lm_clear, dim3(1), dim3(64), 0, s, L.scal.p);
  hipLaunchKernelGGL(k_campre, dim3(ceil_div(P->n_cam, 256)), dim3(256), 0, s, P->n_cam, cams, L.campre.p,
                     &L.scal.p->camflag);
  hipLaunchKernelGGL(k_lm_cost, dim3(red_grid((int)P->n_obs)), dim3(256), 0, s, (int)P->n_obs, P->obs_cam.p,
                     P->obs_pt.p, P->pt_orig.p, P->obs_orig.p, L.campre.p, pts, uv, loss, a, W.partial.p, L.scal.p);
  BA_LAUNCH_CHECK();
}

// |a|^2 into dots[k] (FP64, deterministic)
static void enqueue_norm2(ba_plan* P, const double* a, int n, double* out, hipStream_t s) {
  Scratch& W = *P->scratch;
  hipLaunchKernelGGL((k_dot<DOT_PLAIN, double>), dim3(red_grid(n)), dim3(256), 0, s, n, a, a, W.partial.p, W.scal.p,
                     out);
}

static void read_scalars(LmWork& L, const double* dots, hipStream_t s) {
  BA_HIP(hipMemcpyAsync(L.h_scal, L.scal.p, sizeof(LmScal), hipMemcpyDeviceToHost, s));
  if (dots) BA_HIP(hipMemcpyAsync(L.h_dots, dots, 4 * sizeof(double), hipMemcpyDeviceToHost, s));
  BA_HIP(hipStreamSynchronize(s));
}

static ba_status lm_solve(ba_plan* P, const ba_opts* o_in, const ba_lm_opts* lo, double* cams, double* pts,
                          const double* uv, ba_lm_iter* history, ba_lm_summary* sum, hipStream_t s) {
  LmWork& L = lm_work(P);
  Scratch& W = *P->scratch;
  const int nc = 9 * P->n_cam, np = 3 * P->n_pt;
  double* dots = W.dots.p + 4;   // |dc|^2, |dp|^2, |cams|^2, |pts|^2
  ba_lm_summary out{};
  Timer total(s);

  enqueue_cost(P, L, o_in, cams, pts, uv, s);
  read_scalars(L, nullptr, s);
  BA_CHECK(!L.h_scal->camflag && std::isfinite(L.h_scal->cost), BA_ERR_GEOMETRY,
           "non-finite initial parameters or cost");
  BA_CHECK(L.h_scal->invalid == 0u, BA_ERR_GEOMETRY,
           "initial parameters put a point at or behind an observing camera (x_cam.z >= 0)");
  double cost = L.h_scal->cost;
  out.cost0 = cost;
  out.termination = BA_TERM_MAX_ITERS;
  double radius = lo->radius0, nu = 2.0;
  ba_opts o = *o_in;
  for (int it = 0; it < lo->max_iters; ++it) {
    Timer ti(s);
    o.lambda = 1.0 / radius;
    ba_stats st{};
    ba_status ss = BA_OK;
    try {
      prepare(P, &o, cams, pts, uv, nullptr, &st, s, true);   // the model decrease reads the planes
      ss = solve(P, &o, L.dc.p, L.dp.p, &st, s);
    } catch (const Fail& f) {
      if (f.st != BA_ERR_NOT_SPD) throw;
      // the damped system is not numerically positive definite (a block, the
      // coarse matrix or PCG broke down): a failed step, handled as a rejection.
      // Drain the plan's streams before the next attempt reuses its buffers.
      BA_HIP(hipStreamSynchronize(P->side));
      BA_HIP(hipStreamSynchronize(P->side2));
      BA_HIP(hipStreamSynchronize(P->side3));
      BA_HIP(hipMemsetAsync(P->errflag.p, 0, sizeof(uint32_t), s));
      BA_HIP(hipStreamSynchronize(s));
      if (history) {
        ba_lm_iter& r = history[out.iters];
        r = ba_lm_iter{};
        r.cost = cost;
        r.cost_candidate = INFINITY;
        r.rho = -INFINITY;
        r.radius = radius;
        r.pcg_iters = st.iters;
        r.t_ms = ti.ms();
      }
      out.iters += 1;
      out.pcg_iters += st.iters;
      radius /= nu;
      nu *= 2.0;
      if (radius < lo->min_radius) {
        out.termination = BA_TERM_RADIUS;
        break;
      }
      continue;
    }
    if (ss < 0) return ss;   // cams, pts hold the last accepted parameters
    // predicted decrease, candidate, its cost and the norms of the stopping rules
    hipLaunchKernelGGL(k_lm_clear, dim3(1), dim3(64), 0, s, L.scal.p);
    hipLaunchKernelGGL(k_lm_model, dim3(red_grid((int)P->n_obs)), dim3(256), 0, s, (int)P->n_obs, P->n_obs_pad,
                       P->obs_cam.p, P->obs_pt.p, P->pt_orig.p, P->F.p, P->E.p, P->fres.p, L.dc.p, L.dp.p,
                       W.partial.p, L.scal.p);
    enqueue_norm2(P, L.dc.p, nc, dots + 0, s);
    enqueue_norm2(P, L.dp.p, np, dots + 1, s);
    enqueue_norm2(P, cams, nc, dots + 2, s);
    enqueue_norm2(P, pts, np, dots + 3, s);
    hipLaunchKernelGGL(k_axpby, dim3(ceil_div(nc, 256)), dim3(256), 0, s, nc, (const double*)cams, 1.0,
                       (const double*)L.dc.p, L.cams_new.p);
    hipLaunchKernelGGL(k_axpby, dim3(ceil_div(np, 256)), dim3(256), 0, s, np, (const double*)pts, 1.0,
                       (const double*)L.dp.p, L.pts_new.p);
    hipLaunchKernelGGL(k_campre, dim3(ceil_div(P->n_cam, 256)), dim3(256), 0, s, P->n_cam,
                       (const double*)L.cams_new.p, L.campre.p, &L.scal.p->camflag);
    hipLaunchKernelGGL(k_lm_cost, dim3(red_grid((int)P->n_obs)), dim3(256), 0, s, (int)P->n_obs, P->obs_cam.p,
                       P->obs_pt.p, P->pt_orig.p, P->obs_orig.p, L.campre.p, (const double*)L.pts_new.p, uv,
                       o.loss, o.loss_scale, W.partial.p, L.scal.p);
    BA_LAUNCH_CHECK();
    read_scalars(L, dots, s);
    const LmScal h = *L.h_scal;
    const double step_norm = std::sqrt(L.h_dots[0] + L.h_dots[1]);
    const double x_norm = std::sqrt(L.h_dots[2] + L.h_dots[3]);
    out.pcg_iters += st.iters;
    if (step_norm <= lo->parameter_tol * (x_norm + lo->parameter_tol)) {
      out.termination = BA_TERM_PARAMETER;
      break;
    }
    const double md = h.model;
    const bool valid = !h.camflag && h.invalid == 0u && std::isfinite(h.cost);
    const double cost_new = valid ? h.cost : INFINITY;
    const double rho = (md > 0.0 && valid) ? (cost - cost_new) / md : -INFINITY;
    const bool accepted = rho > lo->min_relative_decrease;
    if (history) {
      ba_lm_iter& r = history[out.iters];
      r.cost = cost;
      r.cost_candidate = cost_new;
      r.model_decrease = md;
      r.rho = rho;
      r.radius = radius;
      r.step_norm = step_norm;
      r.accepted = accepted ? 1 : 0;
      r.pcg_iters = st.iters;
    }
    out.iters += 1;
    if (accepted) {
      radius = std::min(lo->max_radius, radius / std::max(1.0 / 3.0, 1.0 - std::pow(2.0 * rho - 1.0, 3)));
      nu = 2.0;
      BA_HIP(hipMemcpyAsync(cams, L.cams_new.p, (size_t)nc * sizeof(double), hipMemcpyDeviceToDevice, s));
      BA_HIP(hipMemcpyAsync(pts, L.pts_new.p, (size_t)np * sizeof(double), hipMemcpyDeviceToDevice, s));
      out.accepted += 1;
      const double decrease = cost - cost_new;
      cost = cost_new;
      if (history) history[out.iters - 1].t_ms = ti.ms();
      if (decrease <= lo->function_tol * (cost + decrease)) {
        out.termination = BA_TERM_FUNCTION;
        break;
      }
    } else {
      radius /= nu;
      nu *= 2.0;
      if (history) history[out.iters - 1].t_ms = ti.ms();
      if (radius < lo->min_radius) {
        out.termination = BA_TERM_RADIUS;
        break;
      }
    }
  }
  BA_HIP(hipStreamSynchronize(s));
  out.cost = cost;
  out.t_ms = total.ms();
  if (sum) *sum = out;
  return BA_OK;
}

}  // namespace bamg
