// C ABI of the bamg library: plan lifetime, the LM step and its stages.
#include <cmath>
#include <cstdarg>
#include <cstring>

#include "kernels.hpp"

namespace bamg {

static thread_local char g_err[1024] = "";

void set_error(const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof(g_err), fmt, ap);
  va_end(ap);
}

thread_local const Allocator* tl_alloc = nullptr;

void* dev_alloc(size_t bytes) {
  void* p = nullptr;
  if (tl_alloc && tl_alloc->alloc) {
    p = tl_alloc->alloc(bytes, tl_alloc->ctx);
    BA_CHECK(p, BA_ERR_HIP, "the allocation callback returned NULL for %zu bytes", bytes);
    BA_CHECK(((uintptr_t)p & 255) == 0, BA_ERR_ARG, "the allocation callback returned memory not aligned to 256 bytes");
  } else {
    BA_HIP(hipMalloc(&p, bytes));
  }
  return p;
}

void dev_free(void* p, const Allocator* a) {
  if (a && a->release) a->release(p, a->ctx);
  else if (!a || !a->alloc) (void)hipFree(p);
}

// PCG and refinement vectors of a step (views into the workspace) and the
// pinned host copy of the PCG scalars (owned by the plan).
struct Scratch {
  int n = 0;  // 9 * n_cam
  DBuf<double> x, r, z, p, q, t, bref, e;
  DBuf<float> fx, fr, fz, fp, fq, fb;
  DBuf<double> partial;
  DBuf<PcgScal> scal;
  // reduction scratch of the Lanczos estimates, one slice per setup stream
  // (levels on different streams run concurrently)
  DBuf<double> lz_partial;   // [3][RED_BLOCKS]
  DBuf<PcgScal> lz_scal;     // [3] (only the reduction counters are used)
  DBuf<double> dots;     // plain dot results
  DBuf<double> pt_a, pt_b;
  PcgScal* h_scal = nullptr;
  // one PCG iteration captured as a graph, per precision (0: FP64, 1: FP32),
  // with the bytes of everything its launches depend on
  hipGraphExec_t it_exec[2] = {nullptr, nullptr};
  std::string it_key[2];
  ~Scratch() {
    if (h_scal) (void)hipHostFree(h_scal);
    for (hipGraphExec_t e : it_exec) if (e) (void)hipGraphExecDestroy(e);
  }
};

// Adjoint buffers of a step (workspace views).
struct Backward {
  DBuf<double> mu_p;   // [n_pt][3] caller order
  DBuf<double> tcam;   // [9][stride]
  DBuf<double> tpt;    // [3][stride]
};

// Levenberg-Marquardt loop buffers (workspace views) and pinned host scalars.
struct LmWork {
  DBuf<double> dc, dp;            // step
  DBuf<double> cams_new, pts_new; // candidate
  DBuf<double> campre;            // camera precomputation of the candidate
  DBuf<LmScal> scal;
  LmScal* h_scal = nullptr;       // pinned copy of scal and the four norms
  double* h_dots = nullptr;
  ~LmWork() {
    if (h_scal) (void)hipHostFree(h_scal);
    if (h_dots) (void)hipHostFree(h_dots);
  }
};

static int red_grid(int n) { return std::max(1, std::min(RED_BLOCKS, ceil_div(n, 256))); }

// Read and clear the device error bits; bits outside `mask` are ignored.
static void check_errflag(ba_plan* P, hipStream_t s, const char* stage = "", uint32_t mask = ~0u) {
  uint32_t e = 0;
  BA_HIP(hipMemcpyAsync(&e, P->errflag.p, sizeof(e), hipMemcpyDeviceToHost, s));
  BA_HIP(hipStreamSynchronize(s));
  if (e) BA_HIP(hipMemsetAsync(P->errflag.p, 0, sizeof(uint32_t), s));
  e &= mask;
  BA_CHECK(!(e & ERRF_NONFINITE), BA_ERR_GEOMETRY, "non-finite camera, point, observation or residual");
  BA_CHECK(!(e & ERRF_GEOMETRY), BA_ERR_GEOMETRY,
           "a point lies at or behind an observing camera (x_cam.z >= 0)");
  BA_CHECK(!(e & ERRF_NOT_SPD), BA_ERR_NOT_SPD, "%s: a block is not positive definite", stage);
  BA_CHECK(!(e & ERRF_LIMIT), BA_ERR_LIMIT, "%s: a kernel capacity was exceeded", stage);
}

struct Timer {
  hipEvent_t a, b;
  hipStream_t s;
  explicit Timer(hipStream_t st) : s(st) {
    BA_HIP(hipEventCreate(&a));
    BA_HIP(hipEventCreate(&b));
    BA_HIP(hipEventRecord(a, s));
  }
  double ms() {
    float t = 0;
    BA_HIP(hipEventRecord(b, s));
    BA_HIP(hipEventSynchronize(b));
    BA_HIP(hipEventElapsedTime(&t, a, b));
    return t;
  }
  ~Timer() {
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
  }
};

// ---------------------------------------------------------------- implicit S

template <class T>
static void schur_apply_dev(ba_plan* P, const T* x, T* y, const int* done, hipStream_t s);

// y -= F^T E C^-1 E^T F x (the tile kernel alone; y already holds A x).
template <class T> static T* te_part_of(ba_plan* P);
template <> double* te_part_of<double>(ba_plan* P) { return P->te_part.p; }
template <> float* te_part_of<float>(ba_plan* P) { return P->te_part32.p; }
template <class T> struct Planes;
template <> struct Planes<double> {
  static const double* F(const ba_plan* P) { return P->F.p; }
  static const double* E(const ba_plan* P) { return P->E.p; }
  static const double* Cinv(const ba_plan* P) { return P->Cinv.p; }
};
template <> struct Planes<float> {
  static const float* F(const ba_plan* P) { return P->F32.p; }
  static const float* E(const ba_plan* P) { return P->E32.p; }
  static const float* Cinv(const ba_plan* P) { return P->Cinv32.p; }
};

// With P->det (deterministic step) the group kernel stores its (group,
// camera) sums and k_schur_gather adds them in group order; otherwise it adds
// them to y with atomics. The FP64 product recomputes F_o and E_o from the
// cameras and points (k_schur_groups_rc) rather than reading the stored
// planes (k_schur_groups): about a tenth of the bytes for the projection's
// arithmetic (136 -> 102 us on the 3.5M-observation city grid). The FP32
// product reads its half-width planes (85 us; recomputing, 96 us).
constexpr bool SCHUR_RECOMPUTE = true;

template <class T>
static void schur_tiles_dev(ba_plan* P, const T* x, T* y, const int* done, hipStream_t s) {
  if (SCHUR_RECOMPUTE && sizeof(T) == 8) {
    const double* wsq = P->robust ? P->wsq.p : nullptr;
    T* part = P->det ? te_part_of<T>(P) : nullptr;
    if (P->det)
      hipLaunchKernelGGL((k_schur_groups_rc<T, true>), dim3(xcd_grid(P->n_groups)), dim3(256), 0, s, P->grp_tile.p,
                         P->grp_coff.p, P->grp_cams.p, P->tile_obs.p, P->tile_pt.p, P->tile_coff.p,
                         P->tile_cseg.p, P->tile_cslot.p, P->pt_off.p, P->obs_slot.p, (const double*)P->campre.p,
                         (const double*)P->prec.p, wsq, Planes<T>::Cinv(P), x, y, part, P->n_groups, done);
    else
      hipLaunchKernelGGL((k_schur_groups_rc<T, false>), dim3(xcd_grid(P->n_groups)), dim3(256), 0, s, P->grp_tile.p,
                         P->grp_coff.p, P->grp_cams.p, P->tile_obs.p, P->tile_pt.p, P->tile_coff.p,
                         P->tile_cseg.p, P->tile_cslot.p, P->pt_off.p, P->obs_slot.p, (const double*)P->campre.p,
                         (const double*)P->prec.p, wsq, Planes<T>::Cinv(P), x, y, (T*)nullptr, P->n_groups, done);
    if (P->det)
      hipLaunchKernelGGL((k_schur_gather<T>), dim3(ceil_div(P->n_cam, 4)), dim3(256), 0, s, P->n_cam,
                         P->cam_te_ptr.p, P->cam_te.p, (const T*)part, y, done);
    return;
  }
  if (P->det) {
    T* part = te_part_of<T>(P);
    hipLaunchKernelGGL((k_schur_groups<T, true>), dim3(xcd_grid(P->n_groups)), dim3(256), 0, s, P->grp_tile.p,
                       P->grp_coff.p, P->grp_cams.p, P->tile_obs.p, P->tile_pt.p, P->tile_coff.p, P->tile_cseg.p,
                       P->tile_cslot.p, P->pt_off.p, P->obs_slot.p, Planes<T>::F(P), Planes<T>::E(P), P->n_obs_pad,
                       Planes<T>::Cinv(P), x, y, part, P->n_groups, done);
    hipLaunchKernelGGL((k_schur_gather<T>), dim3(ceil_div(P->n_cam, 4)), dim3(256), 0, s, P->n_cam,
                       P->cam_te_ptr.p, P->cam_te.p, (const T*)part, y, done);
  } else {
    hipLaunchKernelGGL((k_schur_groups<T, false>), dim3(xcd_grid(P->n_groups)), dim3(256), 0, s, P->grp_tile.p,
                       P->grp_coff.p, P->grp_cams.p, P->tile_obs.p, P->tile_pt.p, P->tile_coff.p, P->tile_cseg.p,
                       P->tile_cslot.p, P->pt_off.p, P->obs_slot.p, Planes<T>::F(P), Planes<T>::E(P), P->n_obs_pad,
                       Planes<T>::Cinv(P), x, y, (T*)nullptr, P->n_groups, done);
  }
}

template <>
void schur_apply_dev<double>(ba_plan* P, const double* x, double* y, const int* done, hipStream_t s) {
  hipLaunchKernelGGL(k_apply_A<double>, dim3(ceil_div(9 * P->n_cam, 252)), dim3(256), 0, s, P->n_cam, P->A.p, x, y);
  schur_tiles_dev<double>(P, x, y, done, s);
}

template <>
void schur_apply_dev<float>(ba_plan* P, const float* x, float* y, const int* done, hipStream_t s) {
  hipLaunchKernelGGL(k_apply_A<float>, dim3(ceil_div(9 * P->n_cam, 252)), dim3(256), 0, s, P->n_cam, P->A32.p, x, y);
  schur_tiles_dev<float>(P, x, y, done, s);
}

}  // namespace bamg

#include "solver.cpp"

using namespace bamg;

#define BA_API_BEGIN try {
#define BA_API_END                                                 \
  }                                                                \
  catch (const Fail& f) {                                          \
    return f.st;                                                   \
  }                                                                \
  catch (const std::bad_alloc&) {                                  \
    set_error("host out of memory");                               \
    return BA_ERR_HIP;                                             \
  }                                                                \
  return BA_OK;

extern "C" {

ba_status ba_opts_default(ba_opts* o) {
  if (!o) return BA_ERR_ARG;
  std::memset(o, 0, sizeof(*o));
  o->precond = BA_PC_MULTIGRID;
  o->precision = BA_FP64;
  o->lambda = 1e-4;
  o->rtol = 1e-6;
  o->max_iter = 2000;
  o->max_refine = 10;
  o->inner_rtol = 1e-3;
  o->agg_cap = 20;
  o->cheb_degree = 2;
  o->lanczos_steps = 5;
  o->coarse_max_nodes = 128;
  o->max_levels = 12;
  o->cheb_lo = 0.3;
  o->cheb_hi = 1.1;
  o->min_coarsen_ratio = 0.9;
  o->level0_op = BA_OP_AUTO;
  o->freeze_damping_in_grad = 0;
  o->check_every = 4;
  o->deterministic = 0;
  o->stop_rule = BA_STOP_RESIDUAL;
  o->forcing = 0.1;
  o->loss = BA_LOSS_SQUARED;
  o->loss_scale = 1.0;
  o->prolongator = BA_PROLONG_TENTATIVE;
  o->graph = 0;
  o->smooth_omega = 4.0 / 3.0;
  return BA_OK;
}

static void validate_opts(const ba_opts* o) {
  BA_CHECK(o, BA_ERR_ARG, "opts is NULL");
  BA_CHECK(o->precond == BA_PC_BLOCK_JACOBI || o->precond == BA_PC_MULTIGRID ||
               o->precond == BA_PC_CLUSTER_JACOBI, BA_ERR_ARG, "bad precond");
  BA_CHECK(o->precond != BA_PC_CLUSTER_JACOBI || o->precision == BA_FP64, BA_ERR_ARG,
           "the cluster preconditioner is FP64 only");
  BA_CHECK(o->precision == BA_FP64 || o->precision == BA_MIXED, BA_ERR_ARG, "bad precision");
  BA_CHECK(o->lambda >= 0.0, BA_ERR_ARG, "lambda must be >= 0");
  BA_CHECK(o->rtol > 0.0 && o->rtol < 1.0, BA_ERR_ARG, "rtol must be in (0, 1)");
  BA_CHECK(o->max_iter >= 1, BA_ERR_ARG, "max_iter must be >= 1");
  BA_CHECK(o->agg_cap >= 2, BA_ERR_ARG, "agg_cap must be >= 2");
  BA_CHECK(o->cheb_degree >= 1 && o->cheb_degree <= 16, BA_ERR_ARG, "cheb_degree must be in [1, 16]");
  BA_CHECK(o->lanczos_steps >= 1 && o->lanczos_steps <= 32, BA_ERR_ARG, "lanczos_steps must be in [1, 32]");
  BA_CHECK(o->coarse_max_nodes >= 1, BA_ERR_ARG, "coarse_max_nodes must be >= 1");
  BA_CHECK(o->max_levels >= 1 && o->max_levels <= 16, BA_ERR_ARG, "max_levels must be in [1, 16]");
  BA_CHECK(o->cheb_hi > o->cheb_lo && o->cheb_lo > 0.0, BA_ERR_ARG, "bad Chebyshev interval");
  BA_CHECK(o->check_every >= 1, BA_ERR_ARG, "check_every must be >= 1");
  BA_CHECK(o->deterministic == 0 || o->deterministic == 1, BA_ERR_ARG, "deterministic must be 0 or 1");
  BA_CHECK(o->stop_rule == BA_STOP_RESIDUAL || o->stop_rule == BA_STOP_NASH_SOFER, BA_ERR_ARG, "bad stop_rule");
  BA_CHECK(o->stop_rule != BA_STOP_NASH_SOFER || (o->forcing >= 0.0 && o->precision == BA_FP64), BA_ERR_ARG,
           "the Nash-Sofer rule needs forcing >= 0 and BA_FP64");
  BA_CHECK(o->loss == BA_LOSS_SQUARED || o->loss == BA_LOSS_HUBER, BA_ERR_ARG, "bad loss");
  BA_CHECK(o->loss == BA_LOSS_SQUARED || o->loss_scale > 0.0, BA_ERR_ARG, "loss_scale must be > 0");
  BA_CHECK(o->graph == 0 || o->graph == 1, BA_ERR_ARG, "graph must be 0 or 1");
  BA_CHECK(o->prolongator == BA_PROLONG_TENTATIVE || o->prolongator == BA_PROLONG_SMOOTHED, BA_ERR_ARG,
           "bad prolongator");
  BA_CHECK(o->prolongator == BA_PROLONG_TENTATIVE || (o->smooth_omega > 0.0 && o->smooth_omega < 2.0), BA_ERR_ARG,
           "smooth_omega must be in (0, 2)");
  BA_CHECK(o->prolongator == BA_PROLONG_TENTATIVE || o->precond != BA_PC_MULTIGRID || o->precision == BA_FP64,
           BA_ERR_ARG, "the smoothed prolongator is FP64 only");
  BA_CHECK(o->precision != BA_MIXED || (o->max_refine >= 1 && o->inner_rtol > 0.0 && o->inner_rtol < 1.0),
           BA_ERR_ARG, "bad refinement options");
}

ba_status ba_plan_create(int32_t n_cam, int32_t n_pt, int64_t n_obs, const int32_t* obs_cam,
                         const int32_t* obs_pt, const ba_opts* o, ba_alloc_fn alloc, ba_free_fn release,
                         void* ctx, void* stream, ba_plan** out) {
  BA_API_BEGIN
  BA_CHECK(out, BA_ERR_ARG, "out is NULL");
  *out = nullptr;
  validate_opts(o);
  BA_CHECK(n_cam >= 2 && n_pt >= 1 && n_obs >= 2, BA_ERR_ARG, "need n_cam >= 2, n_pt >= 1, n_obs >= 2");
  BA_CHECK(n_obs < (int64_t)INT32_MAX - 1024, BA_ERR_LIMIT, "n_obs must be below 2^31");
  BA_CHECK(obs_cam && obs_pt, BA_ERR_ARG, "observation index arrays are NULL");
  BA_CHECK((alloc == nullptr) == (release == nullptr), BA_ERR_ARG, "give both allocation callbacks or neither");
  hipStream_t s = (hipStream_t)stream;
  ba_plan* P = new ba_plan();
  P->alloc.alloc = alloc;
  P->alloc.release = release;
  P->alloc.ctx = ctx;
  try {
    AllocScope scope(&P->alloc);
    P->n_cam = n_cam;
    P->n_pt = n_pt;
    P->n_obs = n_obs;
    P->n_obs_pad = (n_obs + 63) / 64 * 64;
    P->sa = o->prolongator == BA_PROLONG_SMOOTHED;
    P->errflag.alloc(1);
    BA_HIP(hipMemsetAsync(P->errflag.p, 0, sizeof(uint32_t), s));
    std::vector<int32_t> oc(n_obs), op(n_obs);
    BA_HIP(hipMemcpyAsync(oc.data(), obs_cam, n_obs * sizeof(int32_t), hipMemcpyDeviceToHost, s));
    BA_HIP(hipMemcpyAsync(op.data(), obs_pt, n_obs * sizeof(int32_t), hipMemcpyDeviceToHost, s));
    BA_HIP(hipStreamSynchronize(s));
    build_observation_layout(P, oc, op, s);
    build_hierarchy(P, o, s);
    create_runtime(P);
    BA_HIP(hipStreamSynchronize(s));
    *out = P;
  } catch (...) {
    delete P;
    throw;
  }
  BA_API_END
}

size_t ba_workspace_bytes(const ba_plan* P, const ba_opts* o, int32_t uses) {
  try {
    BA_CHECK(P, BA_ERR_ARG, "plan is NULL");
    validate_opts(o);
    BA_CHECK(uses >= 0 && uses <= (BA_USE_BACKWARD | BA_USE_LM), BA_ERR_ARG, "bad `uses`");
    return layout_ws(const_cast<ba_plan*>(P), ws_key(o, uses), nullptr);
  } catch (const Fail&) {
    return 0;
  }
}

void ba_plan_destroy(ba_plan* p) {
  if (!p) return;
  (void)hipDeviceSynchronize();   // no work of the plan may still use its memory
  for (hipStream_t st : {p->side, p->side2, p->side3, p->cap}) {
    if (!st) continue;
    (void)hipStreamSynchronize(st);
    (void)hipStreamDestroy(st);
  }
  for (hipEvent_t e : p->ev_qr) if (e) (void)hipEventDestroy(e);
  for (hipEvent_t e : p->ev_lvl) if (e) (void)hipEventDestroy(e);
  if (p->ev_fork) (void)hipEventDestroy(p->ev_fork);
  for (hipEvent_t e : p->ev_lz) if (e) (void)hipEventDestroy(e);
  for (hipEvent_t e : p->ev_t) if (e) (void)hipEventDestroy(e);
  if (p->h_err) (void)hipHostFree(p->h_err);
  delete p->scratch;
  delete p->bwd;
  delete p->lm;
  delete p;
}

size_t ba_plan_bytes(const ba_plan* P) {
  if (!P) return 0;
  return plan_bytes(P);
}

ba_status ba_eval_jacobian(ba_plan* P, const double* cams, const double* pts, const double* uv, void* ws,
                           size_t ws_bytes, double* f, double* F, double* E, void* stream) {
  BA_API_BEGIN
  BA_CHECK(P && cams && pts && uv, BA_ERR_ARG, "null argument");
  hipStream_t s = (hipStream_t)stream;
  AllocScope scope(&P->alloc);
  bind_ws(P, 0u, ws, ws_bytes, s);
  eval_jacobian(P, cams, pts, uv, s);
  hipLaunchKernelGGL(k_scatter_jacobian, dim3(ceil_div(P->n_obs, 256)), dim3(256), 0, s, (int)P->n_obs,
                     P->obs_orig.p, P->n_obs_pad, P->F.p, P->E.p, P->fres.p, f, F, E);
  BA_LAUNCH_CHECK();
  BA_HIP(hipStreamSynchronize(s));
  // the per-observation planes of a prepared step were overwritten
  P->prepared = false;
  P->prepared_mg = false;
  P->prepared_cj = false;
  BA_API_END
}

ba_status ba_step_prepare(ba_plan* P, const ba_opts* o, const double* cams, const double* pts,
                          const double* uv, const double* D, void* ws, size_t ws_bytes, ba_stats* st,
                          void* stream) {
  BA_API_BEGIN
  BA_CHECK(P && cams && pts && uv, BA_ERR_ARG, "null argument");
  validate_opts(o);
  if (st) std::memset(st, 0, sizeof(*st));
  AllocScope scope(&P->alloc);
  bind_ws(P, ws_key(o, 0), ws, ws_bytes, (hipStream_t)stream);
  prepare(P, o, cams, pts, uv, D, st, (hipStream_t)stream);
  check_errflag(P, (hipStream_t)stream, "normal blocks or preconditioner setup");
  prepare_times(P, st);
  BA_API_END
}

ba_status ba_step_solve(ba_plan* P, const ba_opts* o, double* delta_cam, double* delta_pt,
                        ba_stats* st, void* stream) {
  BA_API_BEGIN
  BA_CHECK(P && delta_cam && delta_pt, BA_ERR_ARG, "null argument");
  validate_opts(o);
  BA_CHECK(P->prepared, BA_ERR_ARG, "ba_step_prepare has not been called");
  return solve(P, o, delta_cam, delta_pt, st, (hipStream_t)stream);
  BA_API_END
}

ba_status ba_lm_step(ba_plan* P, const ba_opts* o, const double* cams, const double* pts,
                     const double* uv, const double* D, void* ws, size_t ws_bytes, double* delta_cam,
                     double* delta_pt, ba_stats* st, void* stream) {
  BA_API_BEGIN
  BA_CHECK(P && cams && pts && uv && delta_cam && delta_pt, BA_ERR_ARG, "null argument");
  validate_opts(o);
  hipStream_t s = (hipStream_t)stream;
  if (st) std::memset(st, 0, sizeof(*st));
  AllocScope scope(&P->alloc);
  bind_ws(P, ws_key(o, 0), ws, ws_bytes, s);
  prepare(P, o, cams, pts, uv, D, st, s);
  const ba_status r = solve(P, o, delta_cam, delta_pt, st, s);
  prepare_times(P, st);
  return r;
  BA_API_END
}

ba_status ba_schur_apply(ba_plan* P, int32_t precision, const double* x, double* y, void* stream) {
  BA_API_BEGIN
  BA_CHECK(P && x && y, BA_ERR_ARG, "null argument");
  BA_CHECK(P->prepared, BA_ERR_ARG, "ba_step_prepare has not been called");
  hipStream_t s = (hipStream_t)stream;
  const int n = 9 * P->n_cam;
  if (precision == BA_MIXED) {
    BA_CHECK(P->have_mixed, BA_ERR_ARG, "step was prepared without BA_MIXED");
    Scratch& W = *P->scratch;
    hipLaunchKernelGGL((k_convert<double, float>), dim3(ceil_div(n, 256)), dim3(256), 0, s, n, x, W.fx.p);
    schur_apply_dev<float>(P, W.fx.p, W.fq.p, nullptr, s);
    hipLaunchKernelGGL((k_convert<float, double>), dim3(ceil_div(n, 256)), dim3(256), 0, s, n, W.fq.p, y);
  } else {
    schur_apply_dev<double>(P, x, y, nullptr, s);
  }
  BA_LAUNCH_CHECK();
  BA_API_END
}

ba_status ba_schur_offdiag_apply(ba_plan* P, int32_t precision, const double* x, double* y, void* stream) {
  BA_API_BEGIN
  BA_CHECK(P && x && y, BA_ERR_ARG, "null argument");
  BA_CHECK(P->prepared, BA_ERR_ARG, "ba_step_prepare has not been called");
  hipStream_t s = (hipStream_t)stream;
  const int n = 9 * P->n_cam;
  if (precision == BA_MIXED) {
    BA_CHECK(P->have_mixed, BA_ERR_ARG, "step was prepared without BA_MIXED");
    Scratch& W = *P->scratch;
    hipLaunchKernelGGL((k_convert<double, float>), dim3(ceil_div(n, 256)), dim3(256), 0, s, n, x, W.fx.p);
    hipLaunchKernelGGL((k_convert<double, float>), dim3(ceil_div(n, 256)), dim3(256), 0, s, n, (const double*)y,
                       W.fq.p);
    schur_tiles_dev<float>(P, W.fx.p, W.fq.p, nullptr, s);
    hipLaunchKernelGGL((k_convert<float, double>), dim3(ceil_div(n, 256)), dim3(256), 0, s, n, W.fq.p, y);
  } else {
    schur_tiles_dev<double>(P, x, y, nullptr, s);
  }
  BA_LAUNCH_CHECK();
  BA_API_END
}

ba_status ba_precond_apply(ba_plan* P, const ba_opts* o, int32_t precision, const double* r,
                           double* z, void* stream) {
  BA_API_BEGIN
  BA_CHECK(P && r && z, BA_ERR_ARG, "null argument");
  validate_opts(o);
  BA_CHECK(P->prepared, BA_ERR_ARG, "ba_step_prepare has not been called");
  precond_apply_fp64boundary(P, o, precision, r, z, (hipStream_t)stream);
  BA_API_END
}

ba_status ba_step_blocks(ba_plan* P, double* b, double* Cinv, double* Scc, void* stream) {
  BA_API_BEGIN
  BA_CHECK(P, BA_ERR_ARG, "null plan");
  BA_CHECK(P->prepared, BA_ERR_ARG, "ba_step_prepare has not been called");
  hipStream_t s = (hipStream_t)stream;
  if (b) BA_HIP(hipMemcpyAsync(b, P->b.p, P->b.bytes(), hipMemcpyDeviceToDevice, s));
  if (Scc) BA_HIP(hipMemcpyAsync(Scc, P->Scc.p, P->Scc.bytes(), hipMemcpyDeviceToDevice, s));
  if (Cinv)
    hipLaunchKernelGGL(k_unpack_cinv, dim3(ceil_div(P->n_pt, 256)), dim3(256), 0, s, P->n_pt, P->pt_orig.p,
                       P->Cinv.p, Cinv);
  BA_LAUNCH_CHECK();
  BA_HIP(hipStreamSynchronize(s));
  BA_API_END
}

ba_status ba_mg_levels(const ba_plan* P, int32_t* n_levels, int32_t* nodes) {
  BA_API_BEGIN
  BA_CHECK(P && n_levels, BA_ERR_ARG, "null argument");
  *n_levels = (int32_t)P->levels.size();
  if (nodes)
    for (size_t l = 0; l < P->levels.size() && l < 16; ++l) nodes[l] = P->levels[l].n;
  BA_API_END
}

ba_status ba_mg_aggregates(const ba_plan* P, int32_t level, int32_t* agg) {
  BA_API_BEGIN
  BA_CHECK(P && agg, BA_ERR_ARG, "null argument");
  BA_CHECK(level >= 0 && level + 1 < (int)P->levels.size(), BA_ERR_ARG, "level has no aggregates");
  const Level& L = P->levels[level];
  BA_HIP(hipMemcpy(agg, L.agg.p, L.n * sizeof(int32_t), hipMemcpyDeviceToDevice));
  BA_API_END
}

ba_status ba_mg_covisibility(const ba_plan* P, int32_t level, int64_t* nnz, int64_t* row_ptr,
                             int32_t* col, int64_t* val) {
  BA_API_BEGIN
  BA_CHECK(P && nnz, BA_ERR_ARG, "null argument");
  BA_CHECK(level >= 0 && level < (int)P->levels.size(), BA_ERR_ARG, "bad level");
  const Level& L = P->levels[level];
  *nnz = L.wnnz;
  if (row_ptr) BA_HIP(hipMemcpy(row_ptr, L.wrowptr.p, (L.n + 1) * sizeof(int64_t), hipMemcpyDeviceToDevice));
  if (col) BA_HIP(hipMemcpy(col, L.wcol.p, L.wnnz * sizeof(int32_t), hipMemcpyDeviceToDevice));
  if (val) BA_HIP(hipMemcpy(val, L.wval.p, L.wnnz * sizeof(int64_t), hipMemcpyDeviceToDevice));
  BA_API_END
}

ba_status ba_mg_level_data(const ba_plan* P, int32_t level, int32_t what, double* out, void* stream) {
  BA_API_BEGIN
  BA_CHECK(P && out, BA_ERR_ARG, "null argument");
  BA_CHECK(level >= 0 && level < (int)P->levels.size(), BA_ERR_ARG, "bad level");
  BA_CHECK(P->inspectable_mg, BA_ERR_ARG, "no multigrid step has been prepared");
  level_data(P, level, what, out, (hipStream_t)stream);
  BA_API_END
}

ba_status ba_lm_step_backward(ba_plan* P, const ba_opts* o, const double* cams, const double* pts,
                              const double* uv, const double* D, const double* delta_cam, const double* delta_pt,
                              const double* gd_cam, const double* gd_pt, void* ws, size_t ws_bytes,
                              double* g_cams, double* g_pts, double* g_uv, ba_stats* st, void* stream) {
  BA_API_BEGIN
  BA_CHECK(P && cams && pts && uv && delta_cam && delta_pt && gd_cam && gd_pt && g_cams && g_pts && g_uv,
           BA_ERR_ARG, "null argument");
  validate_opts(o);
  BA_CHECK(o->loss == BA_LOSS_SQUARED, BA_ERR_ARG, "the backward pass supports the squared loss only");
  AllocScope scope(&P->alloc);
  bind_ws(P, ws_key(o, BA_USE_BACKWARD), ws, ws_bytes, (hipStream_t)stream);
  return backward(P, o, cams, pts, uv, D, delta_cam, delta_pt, gd_cam, gd_pt, g_cams, g_pts, g_uv, st,
                  (hipStream_t)stream);
  BA_API_END
}

ba_status ba_lm_opts_default(ba_lm_opts* lo) {
  if (!lo) return BA_ERR_ARG;
  std::memset(lo, 0, sizeof(*lo));
  lo->max_iters = 100;
  lo->radius0 = 1e4;
  lo->min_relative_decrease = 1e-3;
  lo->function_tol = 1e-6;
  lo->parameter_tol = 1e-8;
  lo->min_radius = 1e-32;
  lo->max_radius = 1e16;
  return BA_OK;
}

ba_status ba_cost(ba_plan* P, const ba_opts* o, const double* cams, const double* pts, const double* uv,
                  void* ws, size_t ws_bytes, double* cost, int64_t* n_invalid, void* stream) {
  BA_API_BEGIN
  BA_CHECK(P && cams && pts && uv && cost, BA_ERR_ARG, "null argument");
  if (o) validate_opts(o);
  hipStream_t s = (hipStream_t)stream;
  AllocScope scope(&P->alloc);
  bind_ws(P, o ? ws_key(o, BA_USE_LM) : (uint32_t)WS_LM, ws, ws_bytes, s);
  LmWork& L = lm_work(P);
  enqueue_cost(P, L, o, cams, pts, uv, s);
  read_scalars(L, nullptr, s);
  *cost = L.h_scal->cost;
  if (n_invalid) *n_invalid = (int64_t)L.h_scal->invalid;
  BA_API_END
}

ba_status ba_lm_solve(ba_plan* P, const ba_opts* o, const ba_lm_opts* lo, double* cams, double* pts,
                      const double* uv, void* ws, size_t ws_bytes, ba_lm_iter* history, ba_lm_summary* summary,
                      void* stream) {
  BA_API_BEGIN
  BA_CHECK(P && lo && cams && pts && uv, BA_ERR_ARG, "null argument");
  validate_opts(o);
  AllocScope scope(&P->alloc);
  bind_ws(P, ws_key(o, BA_USE_LM), ws, ws_bytes, (hipStream_t)stream);
  BA_CHECK(lo->max_iters >= 0 && lo->radius0 > 0.0 && lo->max_radius >= lo->radius0 && lo->min_radius >= 0.0 &&
               lo->function_tol >= 0.0 && lo->parameter_tol >= 0.0 && lo->min_relative_decrease >= 0.0,
           BA_ERR_ARG, "bad LM options");
  return lm_solve(P, o, lo, cams, pts, uv, history, summary, (hipStream_t)stream);
  BA_API_END
}

ba_status ba_selftest_tile_mma(const double* X, const double* Y, double* C, int32_t mode, void* stream) {
  BA_API_BEGIN
  BA_CHECK(X && Y && C && mode >= 0 && mode <= 2, BA_ERR_ARG, "bad argument");
  hipStream_t s = (hipStream_t)stream;
  hipLaunchKernelGGL(k_mfma_probe, dim3(1), dim3(64), 0, s, X, Y, C, mode);
  BA_LAUNCH_CHECK();
  BA_HIP(hipStreamSynchronize(s));
  BA_API_END
}

const char* ba_status_str(ba_status e) {
  switch (e) {
    case BA_OK: return "BA_OK";
    case BA_NOT_CONVERGED: return "BA_NOT_CONVERGED";
    case BA_ERR_ARG: return "BA_ERR_ARG";
    case BA_ERR_INDEX: return "BA_ERR_INDEX";
    case BA_ERR_STRUCTURE: return "BA_ERR_STRUCTURE";
    case BA_ERR_GEOMETRY: return "BA_ERR_GEOMETRY";
    case BA_ERR_NOT_SPD: return "BA_ERR_NOT_SPD";
    case BA_ERR_WORKSPACE: return "BA_ERR_WORKSPACE";
    case BA_ERR_HIP: return "BA_ERR_HIP";
    case BA_ERR_LIMIT: return "BA_ERR_LIMIT";
  }
  return "unknown status";
}

const char* ba_last_error(void) { return g_err; }

}  // extern "C"
