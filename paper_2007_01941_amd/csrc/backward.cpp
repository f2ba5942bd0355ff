// Backward pass of one LM step.
namespace bamg {

static ba_status backward(ba_plan* P, const ba_opts* o, const double* cams, const double* pts, const double* uv,
                          const double* delta_cam, const double* delta_pt, const double* gd_cam,
                          const double* gd_pt, double* g_cams, double* g_pts, double* g_uv, ba_stats* st,
                          hipStream_t s) {
  BA_CHECK(false, BA_ERR_ARG, "backward is not available yet");
  return BA_ERR_ARG;
}

}  // namespace bamg
