// Backward pass of one LM step: mu = H^-1 gbar with the same Schur system and
// preconditioner as the forward step (residual and Jacobian recomputed), then
// dL/du = J mu and dL/dx from the first- and second-order terms.
namespace bamg {

static ba_status backward(ba_plan* P, const ba_opts* o, const double* cams, const double* pts, const double* uv,
                          const double* D, const double* delta_cam, const double* delta_pt, const double* gd_cam,
                          const double* gd_pt, double* g_cams, double* g_pts, double* g_uv, ba_stats* st,
                          hipStream_t s) {
  if (st) std::memset(st, 0, sizeof(*st));
  prepare(P, o, cams, pts, uv, D, st, s, true);   // the adjoint kernels read the planes
  Scratch& W = *P->scratch;
  Backward& B = *P->bwd;
  Timer ts(s);
  // right-hand side of the Schur system for H [mu_c; mu_p] = [gd_cam; gd_pt]
  hipLaunchKernelGGL(k_point_solve, dim3(grid_of<double>(P->n_pt)), dim3(256), 0, s, P->n_pt, P->pt_orig.p,
                     P->Cinv.p, gd_pt, W.pt_a.p, W.pt_b.p);
  hipLaunchKernelGGL(k_cam_FtEv, dim3(P->n_cam), dim3(256), 0, s, P->cam_off.p, P->cam_obs.p, P->obs_pt.p,
                     P->n_obs_pad, P->F.p, P->E.p, W.pt_a.p, gd_cam, -1.0, W.bref.p);
  BA_LAUNCH_CHECK();
  const ba_status status = solve_camera_system(P, o, W.bref.p, st, s);
  // mu_p = C^-1 (gd_p - W^T mu_c), caller order
  hipLaunchKernelGGL(k_recover_tiles, dim3(xcd_grid(P->n_tiles)), dim3(256), 0, s, P->tile_obs.p, P->tile_pt.p, P->pt_off.p,
                     P->pt_orig.p, P->obs_cam.p, P->n_obs_pad, (const double*)P->F.p, (const double*)P->E.p,
                     P->obs_pt.p, (const double*)nullptr, (const double*)nullptr, (const double*)nullptr, P->Cinv.p,
                     W.pt_b.p, 1.0, W.x.p, B.mu_p.p, P->n_tiles);
  hipLaunchKernelGGL(k_adjoint_obs, dim3(grid_of<double>(P->n_obs)), dim3(256), 0, s, (int)P->n_obs, P->obs_cam.p,
                     P->obs_pt.p, P->obs_orig.p, P->pt_orig.p, P->n_obs_pad, P->F.p, P->E.p, P->fres.p, cams, pts,
                     W.x.p, B.mu_p.p, delta_cam, delta_pt, o->lambda, (D || o->freeze_damping_in_grad) ? 1 : 0, g_uv, B.tcam.p,
                     B.tpt.p);
  hipLaunchKernelGGL(k_adjoint_points, dim3(grid_of<double>(P->n_pt)), dim3(256), 0, s, P->n_pt, P->pt_off.p,
                     P->pt_orig.p, P->n_obs_pad, B.tpt.p, g_pts);
  hipLaunchKernelGGL(k_adjoint_cameras, dim3(P->n_cam), dim3(256), 0, s, P->cam_off.p, P->cam_obs.p,
                     P->n_obs_pad, B.tcam.p, g_cams);
  BA_LAUNCH_CHECK();
  const double t = ts.ms();
  if (st) st->t_solve_ms = t;
  prepare_times(P, st);
  return status;
}

}  // namespace bamg
