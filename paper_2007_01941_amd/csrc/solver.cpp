// Host orchestration of one LM step on the device: evaluation, numeric
// multigrid setup, the V-cycle, PCG and mixed-precision refinement.
// (Included by api.cpp inside namespace-level scope.)
#include <algorithm>
#include <cmath>
#include <string>
#include <thread>
#include <type_traits>

namespace bamg {

template <class T>
static int grid_of(int64_t n, int per = 256) { return std::max(1, ceil_div(n, per)); }

// Device bytes the plan owns: its persistent arrays and its own workspace.
static size_t plan_bytes(const ba_plan* P) {
  size_t b = 0;
  b += P->obs_cam.bytes() + P->obs_pt.bytes() + P->obs_orig.bytes() + P->pt_off.bytes() + P->pt_orig.bytes();
  b += P->pt_new.bytes() + P->cam_off.bytes() + P->cam_obs.bytes() + P->obs_rank.bytes();
  b += P->tile_obs.bytes() + P->tile_pt.bytes() + P->tile_coff.bytes() + P->tile_cams.bytes() + P->tile_cseg.bytes() + P->obs_slot.bytes();
  b += P->tile_cslot.bytes() + P->grp_tile.bytes() + P->grp_coff.bytes() + P->grp_cams.bytes();
  b += P->s0_ptr.bytes() + P->s0_q.bytes() + P->cam_q.bytes() + P->s0_chunk_e.bytes() + P->s0_chunk_beg.bytes();
  b += P->s0_blk_e.bytes() + P->s0_blk_ch.bytes() + P->cam_te_ptr.bytes() + P->cam_te.bytes() + P->cj_off.bytes();
  b += P->errflag.bytes() + P->own_ws.bytes();
  for (const Level& L : P->levels) {
    b += L.wrowptr.bytes() + L.wcol.bytes() + L.rowptr32.bytes() + L.col.bytes() + L.wval.bytes() + L.wdiag.bytes() +
         L.order.bytes();
    b += L.diag_pos.bytes() + L.trans_pos.bytes() + L.row_of.bytes() + L.agg.bytes() + L.agg_ptr.bytes();
    b += L.agg_mem.bytes() + L.agg_pos.bytes() + L.slot_of.bytes() + L.gal_ptr.bytes() + L.gal_fine.bytes();
    for (const DBuf<int32_t>* v : {&L.ps_ptr, &L.ps_col, &L.ps_row, &L.ps_self, &L.ps_src_ptr, &L.ps_src, &L.pst_ptr,
                                   &L.pst_e, &L.t_src_ptr, &L.t_src_op, &L.t_src_ps, &L.cg_ptr, &L.cg_ps, &L.cg_t})
      b += v->bytes();
  }
  return b;
}

// ---------------------------------------------------------------- workspace

// What a workspace holds beyond the plain FP64 step.
enum : uint32_t {
  WS_MIXED = 1u, WS_ROBUST = 2u, WS_DET = 4u, WS_MG = 8u, WS_CJ = 16u, WS_BWD = 32u, WS_LM = 64u,
};

static uint32_t ws_key(const ba_opts* o, int32_t uses) {
  uint32_t k = 0;
  if (o->precision == BA_MIXED) k |= WS_MIXED;
  if (o->loss != BA_LOSS_SQUARED) k |= WS_ROBUST;
  if (o->deterministic) k |= WS_DET;
  if (o->precond == BA_PC_MULTIGRID) k |= WS_MG;
  if (o->precond == BA_PC_CLUSTER_JACOBI) k |= WS_CJ;
  if (uses & BA_USE_BACKWARD) k |= WS_BWD;
  if (uses & BA_USE_LM) k |= WS_LM;
  return k;
}

// Places every per-step buffer of `key` in the workspace at `base` (or, with
// base == nullptr, only adds up the bytes). Buffers a key does not need are
// left empty.
static size_t layout_ws(ba_plan* P, uint32_t key, char* base) {
  Carve c;
  c.base = base;
  const int64_t st = P->n_obs_pad;
  const size_t nc = P->n_cam, np = P->n_pt, n = 9 * nc;
  const bool mixed = key & WS_MIXED, mg = key & WS_MG, cj = key & WS_CJ, det = key & WS_DET;
  if (base) {
    // drop the views a key may leave out, so that they are empty
    for (DBuf<float>* v : {&P->F32, &P->E32, &P->Cinv32, &P->A32, &P->Sinv32, &P->te_part32}) v->view(nullptr, 0);
    for (DBuf<double>* v : {&P->wsq, &P->te_part, &P->s0_part, &P->cj_inv}) v->view(nullptr, 0);
  }
  c.take(P->campre, nc * 24);
  c.take(P->F, 18 * st);
  c.take(P->E, 6 * st);
  c.take(P->fres, 2 * st);
  c.take(P->Cinv, np * 6);
  c.take(P->vgp, np * 3);
  c.take(P->gp, np * 3);
  c.take(P->Dp, np * 3);
  c.take(P->A, nc * 45);
  c.take(P->Dc, nc * 9);
  c.take(P->b, nc * 9);
  c.take(P->prec, np * PREC);
  c.take(P->Scc, nc * 81);
  c.take(P->Sinv, nc * 81);
  Scratch& W = *P->scratch;
  for (DBuf<double>* v : {&W.x, &W.r, &W.z, &W.p, &W.q, &W.t, &W.bref, &W.e}) c.take(*v, n);
  c.take(W.partial, RED_BLOCKS);
  c.take(W.scal, 2);
  c.take(W.lz_partial, 3 * RED_BLOCKS);
  c.take(W.lz_scal, 3);
  c.take(W.dots, 8);
  c.take(W.pt_a, 3 * np);
  c.take(W.pt_b, 3 * np);
  if (mixed) {
    c.take(P->F32, 18 * st);
    c.take(P->E32, 6 * st);
    c.take(P->Cinv32, np * 6);
    c.take(P->A32, nc * 45);
    c.take(P->Sinv32, nc * 81);
    for (DBuf<float>* v : {&W.fx, &W.fr, &W.fz, &W.fp, &W.fq, &W.fb}) c.take(*v, n);
  } else {
    for (DBuf<float>* v : {&W.fx, &W.fr, &W.fz, &W.fp, &W.fq, &W.fb}) if (base) v->view(nullptr, 0);
  }
  if (key & WS_ROBUST) c.take(P->wsq, st);
  if (det) {
    c.take(P->te_part, (size_t)P->n_te * 9);
    if (mixed) c.take(P->te_part32, (size_t)P->n_te * 9);
    if (mg || cj) c.take(P->s0_part, (size_t)P->s0_chunks * 81);
  }
  const int nl = (int)P->levels.size();
  for (int l = 0; l < nl; ++l) {
    Level& L = P->levels[l];
    const size_t nv = (size_t)L.n * L.bs;
    const bool last = l + 1 == nl;
    const bool use = mg || (cj && l == 0);   // the cluster blocks come from the explicit level-0 S
    if (base) {
      for (DBuf<double>* v : {&L.S, &L.K, &L.P, &L.Dinv, &L.dense, &L.inv, &L.gj_scale, &L.gj_piv, &L.vb, &L.vx,
                              &L.vr, &L.vd, &L.vt, &L.vpart, &L.vd2, &L.vx2, &L.lz_u, &L.lz_v, &L.lz_up, &L.lz_vp,
                              &L.lz_av, &L.lz_dav, &L.lz_w, &L.lz_dw, &L.lz_s, &L.Ps, &L.Tsp})
        v->view(nullptr, 0);
      for (DBuf<float>* v : {&L.S32, &L.P32, &L.Dinv32, &L.fb, &L.fx, &L.fr, &L.fd, &L.ft, &L.fpart, &L.fd2, &L.fx2})
        v->view(nullptr, 0);
    }
    if (!use) continue;
    c.take(L.S, (size_t)L.nnz * L.bs * L.bs);
    if (!mg) continue;
    c.take(L.K, nv * NS);
    if (!last) {
      c.take(L.P, nv * NS);
      if (l > 0) c.take(L.Dinv, (size_t)L.n * L.bs * L.bs);
      c.take(L.vpart, (size_t)L.n * NS);
      c.take(L.vd2, nv);
      c.take(L.vx2, nv);
      for (DBuf<double>* v : {&L.lz_u, &L.lz_v, &L.lz_up, &L.lz_vp, &L.lz_av, &L.lz_dav, &L.lz_w, &L.lz_dw})
        c.take(*v, nv);
      c.take(L.lz_s, LZ_SIZE);
      if (P->sa) {
        c.take(L.Ps, (size_t)L.nnz_ps * L.bs * NS);
        c.take(L.Tsp, (size_t)L.nnz_t * L.bs * NS);
      }
    } else {
      L.nd = (int)((nv + GJB - 1) / GJB * GJB);
      c.take(L.dense, (size_t)L.nd * L.nd);
      c.take(L.inv, (size_t)L.nd * L.nd);
      c.take(L.gj_scale, L.nd);
      c.take(L.gj_piv, 2 * GJB * GJB);
    }
    for (DBuf<double>* v : {&L.vb, &L.vx, &L.vr, &L.vd, &L.vt}) c.take(*v, nv);
    if (mixed && l == 0) {
      // the FP32 V-cycle runs level 0 in FP32 and the coarse levels in FP64
      c.take(L.S32, (size_t)L.nnz * L.bs * L.bs);
      if (!last) {
        c.take(L.P32, nv * NS);
        c.take(L.fpart, (size_t)L.n * NS);
        c.take(L.fd2, nv);
        c.take(L.fx2, nv);
      }
      for (DBuf<float>* v : {&L.fb, &L.fx, &L.fr, &L.fd, &L.ft}) c.take(*v, nv);
    } else if (mixed && l == 1) {
      // level 1 in FP32: the restricted residual and the coarse correction as
      // level 0's FP32 V-cycle hands them over (widened to / narrowed from FP64)
      c.take(L.fb, nv);
      c.take(L.fx, nv);
    }
  }
  if (cj && nl > 1) c.take(P->cj_inv, (size_t)P->cj_total);
  if (key & WS_BWD) {
    Backward& B = *P->bwd;
    c.take(B.mu_p, np * 3);
    c.take(B.tcam, 9 * st);
    c.take(B.tpt, 3 * st);
  }
  if (key & WS_LM) {
    LmWork& L = *P->lm;
    c.take(L.dc, 9 * nc);
    c.take(L.dp, 3 * np);
    c.take(L.cams_new, 9 * nc);
    c.take(L.pts_new, 3 * np);
    c.take(L.campre, 24 * nc);
    c.take(L.scal, 1);
  }
  return (c.off + 255) / 256 * 256;
}

static void invalidate_step(ba_plan* P) {
  P->prepared = false;
  P->prepared_mg = false;
  P->prepared_cj = false;
  P->inspectable_mg = false;
  P->have_mixed = false;
}

// Binds the step buffers of options `key` to the caller's workspace (ws) or
// to the plan's own (ws == NULL, allocated through the plan's callbacks and
// only ever grown). Rebinding drops the prepared step; binding the same
// workspace with the same key keeps it.
static void bind_ws(ba_plan* P, uint32_t key, void* ws, size_t ws_bytes, hipStream_t s) {
  char* base;
  uint32_t k;
  if (ws) {
    BA_CHECK(((uintptr_t)ws & 255) == 0, BA_ERR_ARG, "the workspace is not aligned to 256 bytes");
    const size_t need = layout_ws(P, key, nullptr);
    BA_CHECK(ws_bytes >= need, BA_ERR_WORKSPACE, "workspace of %zu bytes; these options need %zu", ws_bytes, need);
    // the same workspace, already laid out for these options and more, and
    // still holding all of that layout
    if (ws == P->ws_base && (P->ws_key & key) == key && ws_bytes >= P->ws_span) return;
    base = static_cast<char*>(ws);
    k = key;
  } else {
    k = P->own_key | key;
    if (!P->own_ws.p || k != P->own_key) {
      const size_t need = layout_ws(P, k, nullptr);
      if (P->own_ws.p) BA_HIP(hipStreamSynchronize(s));
      P->ws_base = nullptr;
      P->own_ws.alloc(need);
      P->own_key = k;
    }
    base = P->own_ws.p;
  }
  if (P->ws_base == base && P->ws_key == k) return;
  BA_HIP(hipStreamSynchronize(s));
  invalidate_step(P);
  P->ws_span = layout_ws(P, k, base);
  P->ws_base = base;
  P->ws_key = k;
  // the reduction counters in the scalar blocks start at zero
  BA_HIP(hipMemsetAsync(P->scratch->scal.p, 0, 2 * sizeof(PcgScal), s));
  BA_HIP(hipMemsetAsync(P->scratch->lz_scal.p, 0, 3 * sizeof(PcgScal), s));
  if (k & WS_LM) BA_HIP(hipMemsetAsync(P->lm->scal.p, 0, sizeof(LmScal), s));
}

// Host-side runtime of a plan: side streams, events, pinned scalar copies and
// the work structs whose device buffers are workspace views.
static void create_runtime(ba_plan* P) {
  P->scratch = new Scratch();
  P->scratch->n = 9 * P->n_cam;
  BA_HIP(hipHostMalloc((void**)&P->scratch->h_scal, 2 * sizeof(PcgScal), hipHostMallocDefault));
  P->bwd = new Backward();
  P->lm = new LmWork();
  BA_HIP(hipHostMalloc((void**)&P->lm->h_scal, sizeof(LmScal), hipHostMallocDefault));
  BA_HIP(hipHostMalloc((void**)&P->lm->h_dots, 4 * sizeof(double), hipHostMallocDefault));
  BA_HIP(hipHostMalloc((void**)&P->h_err, sizeof(uint32_t), hipHostMallocDefault));
  for (hipEvent_t& e : P->ev_t) BA_HIP(hipEventCreate(&e));
  BA_HIP(hipStreamCreateWithFlags(&P->side, hipStreamNonBlocking));
  BA_HIP(hipStreamCreateWithFlags(&P->side2, hipStreamNonBlocking));
  BA_HIP(hipStreamCreateWithFlags(&P->side3, hipStreamNonBlocking));
  BA_HIP(hipEventCreateWithFlags(&P->ev_fork, hipEventDisableTiming));
  for (hipEvent_t& e : P->ev_lz) BA_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
  P->ev_qr.assign(P->levels.size(), nullptr);
  P->ev_lvl.assign(P->levels.size(), nullptr);
  for (hipEvent_t& e : P->ev_qr) BA_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
  for (hipEvent_t& e : P->ev_lvl) BA_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
  // offsets of the cluster blocks (visibility-based block Jacobi): level-0
  // aggregates of 9 m dofs hold (9 m)^2 doubles each
  if (P->levels.size() > 1) {
    const Level& L0 = P->levels[0];
    std::vector<int32_t> cnt(L0.n_agg, 0);
    for (int i = 0; i < L0.n; ++i) ++cnt[L0.h_agg[i]];
    std::vector<int64_t> off((size_t)L0.n_agg + 1, 0);
    int max_n = 0;
    for (int a = 0; a < L0.n_agg; ++a) {
      const int m = 9 * cnt[a];
      off[a + 1] = off[a] + (int64_t)m * m;
      max_n = std::max(max_n, m);
    }
    P->cj_max_n = max_n;
    P->cj_total = off.back();
    P->cj_off.upload(off, nullptr);
    BA_HIP(hipStreamSynchronize(nullptr));
  }
}

template <class T, class U>
static void convert(size_t n, const T* a, U* b, hipStream_t s) {
  if (n) hipLaunchKernelGGL((k_convert<T, U>), dim3(grid_of<T>(n)), dim3(256), 0, s, (int)n, a, b);
}

// Residual and Jacobian planes by the step's own kernel (k_jacobian_tiles),
// without robust weighting; its point-side outputs (C^-1 with the default
// damping, g_p, point records) are written too and discarded by the caller.
static void eval_jacobian(ba_plan* P, const double* cams, const double* pts, const double* uv, hipStream_t s) {
  hipLaunchKernelGGL(k_campre, dim3(grid_of<double>(P->n_cam)), dim3(256), 0, s, P->n_cam, cams, P->campre.p,
                     P->errflag.p);
  hipLaunchKernelGGL(k_jacobian_tiles, dim3(xcd_grid(P->n_tiles)), dim3(256), 0, s, P->tile_obs.p, P->tile_pt.p,
                     P->pt_off.p, P->obs_slot.p, P->obs_cam.p, P->obs_orig.p, P->pt_orig.p, P->campre.p, pts, uv,
                     P->n_obs_pad, 1e-4, (const double*)nullptr, P->n_cam, P->F.p, P->E.p, P->fres.p,
                     (float*)nullptr, (float*)nullptr, P->Cinv.p, (float*)nullptr, P->vgp.p, P->gp.p, P->Dp.p,
                     P->prec.p, P->n_tiles, BA_LOSS_SQUARED, 1.0, (double*)nullptr, P->errflag.p);
  BA_LAUNCH_CHECK();
  // a point block that is not positive definite does not concern this call
  check_errflag(P, s, "residual and Jacobian", ~ERRF_NOT_SPD);
}

// ---------------------------------------------------------------- level operators

static bool level0_explicit(const ba_plan* P, const ba_opts* o, int s_bytes) {
  if (o->level0_op == BA_OP_EXPLICIT) return true;
  if (o->level0_op == BA_OP_IMPLICIT) return false;
  const Level& L = P->levels[0];
  const double implicit = (double)P->n_obs * (24.0 * s_bytes + 4) + (double)P->n_pt * (6.0 * s_bytes + 4) +
                          (double)P->n_cam * 63.0 * s_bytes;
  const double expl = (double)L.nnz * (81.0 * s_bytes + 4) + (double)P->n_cam * 18.0 * s_bytes;
  return expl < implicit;
}

template <class T> static const T* lvS(const Level& L);
template <> const double* lvS<double>(const Level& L) { return L.S.p; }
template <> const float* lvS<float>(const Level& L) { return L.S32.p; }
template <class T> static const T* lvP(const Level& L);
template <> const double* lvP<double>(const Level& L) { return L.P.p; }
template <> const float* lvP<float>(const Level& L) { return L.P32.p; }
template <class T> static const T* lvDinv(const ba_plan* P, int l);
template <> const double* lvDinv<double>(const ba_plan* P, int l) { return l == 0 ? P->Sinv.p : P->levels[l].Dinv.p; }
template <> const float* lvDinv<float>(const ba_plan* P, int l) { return l == 0 ? P->Sinv32.p : P->levels[l].Dinv32.p; }
template <class T> struct LvVec;
template <> struct LvVec<double> {
  static double* b(Level& L) { return L.vb.p; }
  static double* x(Level& L) { return L.vx.p; }
  static double* r(Level& L) { return L.vr.p; }
  static double* d(Level& L) { return L.vd.p; }
  static double* t(Level& L) { return L.vt.p; }
  static double* part(Level& L) { return L.vpart.p; }
  static double* d2(Level& L) { return L.vd2.p; }
  static double* x2(Level& L) { return L.vx2.p; }
};
template <> struct LvVec<float> {
  static float* b(Level& L) { return L.fb.p; }
  static float* x(Level& L) { return L.fx.p; }
  static float* r(Level& L) { return L.fr.p; }
  static float* d(Level& L) { return L.fd.p; }
  static float* t(Level& L) { return L.ft.p; }
  static float* part(Level& L) { return L.fpart.p; }
  static float* d2(Level& L) { return L.fd2.p; }
  static float* x2(Level& L) { return L.fx2.p; }
};

template <class T>
static void op_apply(ba_plan* P, int l, const T* x, T* y, const int* done, hipStream_t s) {
  Level& L = P->levels[l];
  if (l == 0 && !L.explicit_op) {
    schur_apply_dev<T>(P, x, y, done, s);
    return;
  }
  if (L.bs == 9)
    hipLaunchKernelGGL((k_bsr_row<9, T, EP_STORE>), dim3(L.n), dim3(256), 0, s, L.n, L.rowptr32.p, L.col.p, lvS<T>(L),
                       x, y, (const T*)nullptr, (const T*)nullptr, (T*)nullptr, (const T*)nullptr, (T*)nullptr,
                       (const T*)nullptr, (T*)nullptr, T(0), T(0), (const double*)nullptr, (const T*)nullptr,
                       (const int32_t*)nullptr, (T*)nullptr, ProlongTo<T>(), done);
  else
    hipLaunchKernelGGL((k_bsr_row<16, T, EP_STORE>), dim3(L.n), dim3(256), 0, s, L.n, L.rowptr32.p, L.col.p,
                       lvS<T>(L), x, y, (const T*)nullptr, (const T*)nullptr, (T*)nullptr, (const T*)nullptr,
                       (T*)nullptr, (const T*)nullptr, (T*)nullptr, T(0), T(0), (const double*)nullptr,
                       (const T*)nullptr, (const int32_t*)nullptr, (T*)nullptr, ProlongTo<T>(), done);
}

// Block-row product with the explicit operator of level l and a fused epilogue
// (see k_bsr_row): v is the product's input; c2 is for lambda_max = 1 (the
// kernel scales it by the level's 1 / lambda_max on the device).
template <int BS, class T, int EP>
static void row_op(ba_plan* P, int l, const T* v, const T* b, T* r, const T* d_in, T* d_out, const T* x_in,
                   T* x_out, double c1, double c2, T* part, const int* done, hipStream_t s,
                   ProlongTo<T> pro = ProlongTo<T>()) {
  Level& L = P->levels[l];
  hipLaunchKernelGGL((k_bsr_row<BS, T, EP>), dim3(L.n), dim3(256), 0, s, L.n, L.rowptr32.p, L.col.p, lvS<T>(L), v,
                     (T*)nullptr, lvDinv<T>(P, l), b, r, d_in, d_out, x_in, x_out, (T)c1, (T)c2,
                     (const double*)(L.lz_s.p + LZ_ILMAX), part ? lvP<T>(L) : (const T*)nullptr,
                     part ? L.slot_of.p : (const int32_t*)nullptr, part, pro, done);
}

template <int BS, class T>
static void blockdiag_apply(ba_plan* P, int l, const T* r, T* z, const int* done, hipStream_t s) {
  const Level& L = P->levels[l];
  hipLaunchKernelGGL((k_blockdiag<BS, T>), dim3(grid_of<T>((int64_t)L.n * BS)), dim3(256), 0, s, L.n,
                     lvDinv<T>(P, l), r, z, done);
}

// The restriction of the finer level's residual, when it is still in the
// form of per-node partials (fused into the finer level's residual update):
// b_i = sum of part over [agg_ptr[i], agg_ptr[i+1]).
template <class T>
struct Pending {
  const int32_t* agg_ptr = nullptr;
  const T* part = nullptr;
};

template <int BS, class T>
static void vcycle_level(ba_plan* P, const ba_opts* o, int l, T* b, T* x, Pending<T> pend, const int* done,
                         hipStream_t s, ProlongTo<T> pro);

// x = M_l b: the V-cycle from level l (Algorithm 1), x overwritten. With
// pend.part set, b is first formed from the finer level's partials; with
// pro.x set, x is finally prolonged into the finer level (x_f += P x), inside
// the kernel that finishes x.
template <class T>
static void vcycle(ba_plan* P, const ba_opts* o, int l, T* b, T* x, Pending<T> pend, const int* done,
                   hipStream_t s, ProlongTo<T> pro = ProlongTo<T>()) {
  Level& L = P->levels[l];
  if (l + 1 == (int)P->levels.size()) {
    const int nv = L.n * L.bs;
    if constexpr (std::is_same<T, double>::value) {
      if (l > 0 && nv <= 4096) {
        hipLaunchKernelGGL(k_coarse_solve_fused, dim3(L.n), dim3(1024), 0, s, L.n, L.nd, (const double*)L.inv.p, b,
                           pend.agg_ptr, pend.part, x, pro, done);
        return;
      }
    }
    if (pend.part)
      hipLaunchKernelGGL((k_restrict_sum<T>), dim3(grid_of<T>((int64_t)L.n * NS)), dim3(256), 0, s, L.n,
                         pend.agg_ptr, pend.part, b, done);
    hipLaunchKernelGGL((k_dense_solve<T>), dim3(grid_of<T>(nv, 4)), dim3(256), 0, s, nv, L.nd, L.inv.p,
                       (const T*)b, x, done);
    BA_CHECK(!pro.x, BA_ERR_ARG, "internal: a prolongation pending at an unfused coarsest solve");
    return;
  }
  if (L.bs == 9) vcycle_level<9, T>(P, o, l, b, x, pend, done, s, pro);
  else vcycle_level<16, T>(P, o, l, b, x, pend, done, s, pro);
}

// Coarse-grid correction of level l: xc = V-cycle of level l+1 on the restricted
// residual (given as the pending partials `pend`, or, with pend.part null, as
// bc). Coarse levels always run in FP64: their 16 x 16 diagonal blocks are
// nearly singular along the aggregates' rigid motions (held only by the
// damping), so FP32 block inverses there are meaningless; in the FP32 V-cycle
// the level-0 partials (or bc) are widened and the correction narrowed back.
template <class T>
static void coarse_correction(ba_plan* P, const ba_opts* o, int l, T* bc, T* xc, Pending<T> pend, const int* done,
                              hipStream_t s);

template <>
void coarse_correction<double>(ba_plan* P, const ba_opts* o, int l, double* bc, double* xc, Pending<double> pend,
                               const int* done, hipStream_t s) {
  vcycle<double>(P, o, l + 1, bc, xc, pend, done, s);
}

// The FP64 coarse-grid correction with level l's prolongation fused into the
// coarse level's last kernel (x += P xc without a launch of its own). Whether
// level l+1 can take it: its V-cycle must end in a Chebyshev row update
// (degree >= 2) or be the fused coarsest solve.
static bool can_fuse_prolong(const ba_plan* P, const ba_opts* o, int l) {
  if (P->sa) return false;
  const int c = l + 1;
  if (c + 1 == (int)P->levels.size()) return c > 0 && P->levels[c].n * NS <= 4096;
  return o->cheb_degree >= 2;
}

template <>
void coarse_correction<float>(ba_plan* P, const ba_opts* o, int l, float* bc, float* xc, Pending<float> pend,
                              const int* done, hipStream_t s) {
  Level& L = P->levels[l];
  Level& C = P->levels[l + 1];
  Pending<double> wide;
  if (pend.part) {
    convert((size_t)L.n * NS, pend.part, L.vpart.p, s);
    wide.agg_ptr = pend.agg_ptr;
    wide.part = L.vpart.p;
  } else {
    convert((size_t)C.n * C.bs, (const float*)bc, C.vb.p, s);
  }
  vcycle<double>(P, o, l + 1, C.vb.p, C.vx.p, wide, done, s);
  convert((size_t)C.n * C.bs, (const double*)C.vx.p, xc, s);
}

// Restriction and prolongation with the smoothed prolongator of level l
// (FP64 only: plans built for it reject BA_MIXED multigrid steps).
template <int BS, class T>
static void sa_restrict(ba_plan* P, int l, const T* r, const T* t, T* bc, const int* done, hipStream_t s) {
  if constexpr (std::is_same<T, double>::value) {
    const Level& L = P->levels[l];
    hipLaunchKernelGGL((k_sa_restrict<BS>), dim3(grid_of<double>((int64_t)L.n_agg * NS)), dim3(256), 0, s, L.n_agg,
                       L.pst_ptr.p, L.pst_e.p, L.ps_row.p, (const double*)L.Ps.p, r, t, bc, done);
  } else {
    BA_CHECK(false, BA_ERR_ARG, "the smoothed prolongator is FP64 only");
  }
}

template <int BS, class T>
static void sa_prolong(ba_plan* P, int l, const T* xc, T* x, const int* done, hipStream_t s) {
  if constexpr (std::is_same<T, double>::value) {
    const Level& L = P->levels[l];
    hipLaunchKernelGGL((k_sa_prolong<BS>), dim3(grid_of<double>((int64_t)L.n * BS)), dim3(256), 0, s, L.n,
                       L.ps_ptr.p, L.ps_col.p, (const double*)L.Ps.p, xc, x, done);
  } else {
    BA_CHECK(false, BA_ERR_ARG, "the smoothed prolongator is FP64 only");
  }
}

// One V-cycle level (Algorithm 1) with the explicit level operator: every
// Chebyshev step after the first is one fused block-row launch (product and
// update), with the direction d and, in post-smoothing, the iterate
// ping-ponged between two buffers so that no launch writes its product's input.
template <int BS, class T>
static void vcycle_level_fused(ba_plan* P, const ba_opts* o, int l, T* b, T* x, Pending<T> pend, const int* done,
                               hipStream_t s, ProlongTo<T> pro) {
  Level& L = P->levels[l];
  Level& C = P->levels[l + 1];
  T* r = LvVec<T>::r(L);
  T* dA = LvVec<T>::d(L);
  T* dB = LvVec<T>::d2(L);
  T* x2 = LvVec<T>::x2(L);
  const T* Dinv = lvDinv<T>(P, l);
  // Chebyshev coefficients for lambda_max = 1: the kernels scale the ones
  // that depend on it by the level's 1 / lambda_max, read on the device
  const double* il = L.lz_s.p + LZ_ILMAX;
  const double theta = 0.5 * (o->cheb_hi + o->cheb_lo);
  const double delta = 0.5 * (o->cheb_hi - o->cheb_lo);
  const double sigma1 = theta / delta;
  const int m = o->cheb_degree;
  const int nb = std::max(1, ceil_div(L.n, 256 / BS));
  // pre-smoothing from x = 0: r = b, d = D^-1 b / theta, x = d
  double rho = 1.0 / sigma1;
  hipLaunchKernelGGL((k_cheb_first<BS, T>), dim3(nb), dim3(256), 0, s, L.n, pend.part ? 2 : 0, Dinv, b,
                     (const T*)nullptr, r, dA, x, (T)(1.0 / theta), il, pend.agg_ptr, pend.part, done);
  T* part = P->sa ? nullptr : LvVec<T>::part(L);
  for (int k = 0; k < m; ++k) {
    if (k == m - 1) {
      // last pre-smoothing residual update r -= S d (the V-cycle residual),
      // with each node's restriction partial P_i^T r_i (unsmoothed P)
      row_op<BS, T, EP_RESID>(P, l, dA, nullptr, r, nullptr, nullptr, nullptr, nullptr, 0.0, 0.0, part, done, s);
      break;
    }
    const double rn = 1.0 / (2.0 * sigma1 - rho);
    row_op<BS, T, EP_CHEB>(P, l, dA, nullptr, r, dA, dB, x, x, rn * rho, 2.0 * rn / delta, nullptr, done, s);
    std::swap(dA, dB);
    rho = rn;
  }
  T* bc = LvVec<T>::b(C);
  T* xc = LvVec<T>::x(C);
  if (P->sa) {
    sa_restrict<BS, T>(P, l, r, nullptr, bc, done, s);
    coarse_correction<T>(P, o, l, bc, xc, Pending<T>(), done, s);
    sa_prolong<BS, T>(P, l, xc, x, done, s);
  } else {
    // the coarse right-hand side is summed from the partials by the next level
    Pending<T> next;
    next.agg_ptr = L.agg_ptr.p;
    next.part = part;
    bool fused = false;
    if constexpr (std::is_same<T, double>::value) {
      if (can_fuse_prolong(P, o, l)) {
        // x += P xc happens in the coarse level's last kernel
        ProlongTo<double> mine;
        mine.ptr = L.agg_ptr.p;
        mine.mem = L.agg_mem.p;
        mine.P = L.P.p;
        mine.x = x;
        mine.bs = BS;
        vcycle<double>(P, o, l + 1, bc, xc, next, done, s, mine);
        fused = true;
      }
    }
    if (!fused) {
      coarse_correction<T>(P, o, l, bc, xc, next, done, s);
      hipLaunchKernelGGL((k_prolong<BS, T>), dim3(grid_of<T>((int64_t)L.n * BS)), dim3(256), 0, s, L.n, L.agg.p,
                         lvP<T>(L), (const T*)xc, x, done);
    }
  }
  // post-smoothing from x: r = b - S x, d = D^-1 r / theta, iterate -> x2
  rho = 1.0 / sigma1;
  row_op<BS, T, EP_CHEB_POST>(P, l, x, b, r, nullptr, dA, x, x2, 0.0, 1.0 / theta, nullptr, done, s);
  if (m == 1) {
    BA_CHECK(!pro.x, BA_ERR_ARG, "internal: a fused prolongation needs two smoothing steps");
    hipLaunchKernelGGL((k_convert<T, T>), dim3(grid_of<T>((int64_t)L.n * BS)), dim3(256), 0, s, L.n * BS,
                       (const T*)x2, x);
    return;
  }
  for (int k = 0; k < m - 1; ++k) {
    const double rn = 1.0 / (2.0 * sigma1 - rho);
    T* xo = k == m - 2 ? x : x2;
    // the last step finishes x: the finer level's prolongation goes with it
    row_op<BS, T, EP_CHEB>(P, l, dA, nullptr, r, dA, dB, x2, xo, rn * rho, 2.0 * rn / delta, nullptr, done, s,
                           k == m - 2 ? pro : ProlongTo<T>());
    std::swap(dA, dB);
    rho = rn;
  }
}

template <int BS, class T>
static void vcycle_level(ba_plan* P, const ba_opts* o, int l, T* b, T* x, Pending<T> pend, const int* done,
                         hipStream_t s, ProlongTo<T> pro) {
  Level& L = P->levels[l];
  if (l > 0 || L.explicit_op) {
    vcycle_level_fused<BS, T>(P, o, l, b, x, pend, done, s, pro);
    return;
  }
  BA_CHECK(!pro.x, BA_ERR_ARG, "internal: level 0 has no finer level");
  Level& C = P->levels[l + 1];
  T* r = LvVec<T>::r(L);
  T* d = LvVec<T>::d(L);
  T* t = LvVec<T>::t(L);
  const T* Dinv = lvDinv<T>(P, l);
  // Chebyshev coefficients for lambda_max = 1: the kernels scale the ones
  // that depend on it by the level's 1 / lambda_max, read on the device
  const double* il = L.lz_s.p + LZ_ILMAX;
  const double theta = 0.5 * (o->cheb_hi + o->cheb_lo);
  const double delta = 0.5 * (o->cheb_hi - o->cheb_lo);
  const double sigma1 = theta / delta;
  const int m = o->cheb_degree;
  const int nb = std::max(1, ceil_div(L.n, 256 / BS));
  // pre-smoothing from x = 0
  double rho = 1.0 / sigma1;
  hipLaunchKernelGGL((k_cheb_first<BS, T>), dim3(nb), dim3(256), 0, s, L.n, 0, Dinv, b, (const T*)nullptr, r, d, x,
                     (T)(1.0 / theta), il, (const int32_t*)nullptr, (const T*)nullptr, done);
  for (int k = 0; k < m; ++k) {
    op_apply<T>(P, l, d, t, done, s);
    if (k == m - 1) break;
    const double rn = 1.0 / (2.0 * sigma1 - rho);
    hipLaunchKernelGGL((k_cheb_next<BS, T>), dim3(nb), dim3(256), 0, s, L.n, Dinv, (const T*)t, r, d, x,
                       (T)(rn * rho), (T)(2.0 * rn / delta), il, done);
    rho = rn;
  }
  // restriction of the pre-smoother's residual r - t
  T* bc = LvVec<T>::b(C);
  T* xc = LvVec<T>::x(C);
  if (P->sa) {
    sa_restrict<BS, T>(P, l, r, t, bc, done, s);
    coarse_correction<T>(P, o, l, bc, xc, Pending<T>(), done, s);
    sa_prolong<BS, T>(P, l, xc, x, done, s);
  } else {
    T* part = LvVec<T>::part(L);
    hipLaunchKernelGGL((k_restrict_nodes<BS, T>), dim3(grid_of<T>((int64_t)L.n * NS)), dim3(256), 0, s, L.n,
                       L.slot_of.p, lvP<T>(L), (const T*)r, (const T*)t, part, done);
    hipLaunchKernelGGL((k_restrict_sum<T>), dim3(grid_of<T>((int64_t)C.n * NS)), dim3(256), 0, s, C.n,
                       L.agg_ptr.p, (const T*)part, bc, done);
    bool fused = false;
    if constexpr (std::is_same<T, double>::value) {
      if (can_fuse_prolong(P, o, l)) {
        ProlongTo<double> mine;
        mine.ptr = L.agg_ptr.p;
        mine.mem = L.agg_mem.p;
        mine.P = L.P.p;
        mine.x = x;
        mine.bs = BS;
        vcycle<double>(P, o, l + 1, bc, xc, Pending<double>(), done, s, mine);
        fused = true;
      }
    }
    if (!fused) {
      coarse_correction<T>(P, o, l, bc, xc, Pending<T>(), done, s);
      hipLaunchKernelGGL((k_prolong<BS, T>), dim3(grid_of<T>((int64_t)L.n * BS)), dim3(256), 0, s, L.n, L.agg.p,
                         lvP<T>(L), (const T*)xc, x, done);
    }
  }
  // post-smoothing from x
  op_apply<T>(P, l, x, t, done, s);
  rho = 1.0 / sigma1;
  hipLaunchKernelGGL((k_cheb_first<BS, T>), dim3(nb), dim3(256), 0, s, L.n, 1, Dinv, b, (const T*)t, r, d, x,
                     (T)(1.0 / theta), il, (const int32_t*)nullptr, (const T*)nullptr, done);
  for (int k = 0; k < m - 1; ++k) {
    op_apply<T>(P, l, d, t, done, s);
    const double rn = 1.0 / (2.0 * sigma1 - rho);
    hipLaunchKernelGGL((k_cheb_next<BS, T>), dim3(nb), dim3(256), 0, s, L.n, Dinv, (const T*)t, r, d, x,
                       (T)(rn * rho), (T)(2.0 * rn / delta), il, done);
    rho = rn;
  }
}

template <class T> static const T* Sinv_of(const ba_plan* P);
template <> const double* Sinv_of<double>(const ba_plan* P) { return P->Sinv.p; }
template <> const float* Sinv_of<float>(const ba_plan* P) { return P->Sinv32.p; }
template <class T> static const T* A_of(const ba_plan* P);
template <> const double* A_of<double>(const ba_plan* P) { return P->A.p; }
template <> const float* A_of<float>(const ba_plan* P) { return P->A32.p; }

static void cluster_apply(ba_plan* P, const double* r, double* z, const int* done, hipStream_t s) {
  BA_CHECK(P->prepared_cj, BA_ERR_ARG, "the step was prepared without the cluster preconditioner");
  if (P->levels.size() < 2) {   // no aggregates: every camera is its own cluster
    hipLaunchKernelGGL((k_bj_apply<double>), dim3(grid_of<double>(9 * P->n_cam, 252)), dim3(256), 0, s, P->n_cam,
                       P->Sinv.p, r, z, done);
    return;
  }
  const Level& L0 = P->levels[0];
  hipLaunchKernelGGL(k_cj_apply, dim3(L0.n_agg), dim3(256), (size_t)P->cj_max_n * sizeof(double), s,
                     L0.agg_ptr.p, L0.agg_mem.p, P->cj_off.p, P->cj_inv.p, r, z, done);
}
static void cluster_apply(ba_plan*, const float*, float*, const int*, hipStream_t) {
  BA_CHECK(false, BA_ERR_ARG, "the cluster preconditioner is FP64 only");
}

template <class T>
static void precond_apply(ba_plan* P, const ba_opts* o, const T* r, T* z, const int* done, hipStream_t s) {
  if (o->precond == BA_PC_CLUSTER_JACOBI) {
    cluster_apply(P, r, z, done, s);
  } else if (o->precond == BA_PC_BLOCK_JACOBI) {
    hipLaunchKernelGGL((k_bj_apply<T>), dim3(grid_of<T>(9 * P->n_cam, 252)), dim3(256), 0, s, P->n_cam,
                       Sinv_of<T>(P), r, z, done);
  } else {
    BA_CHECK(P->prepared_mg, BA_ERR_ARG, "the step was prepared without the multigrid preconditioner");
    // level 0 has no pending restriction, so r is only read
    vcycle<T>(P, o, 0, const_cast<T*>(r), z, Pending<T>(), done, s);
  }
}

static void precond_apply_fp64boundary(ba_plan* P, const ba_opts* o, int precision, const double* r, double* z,
                                       hipStream_t s) {
  const int n = 9 * P->n_cam;
  if (precision == BA_MIXED) {
    BA_CHECK(P->have_mixed, BA_ERR_ARG, "step was prepared without BA_MIXED");
    Scratch& W = *P->scratch;
    convert(n, r, W.fr.p, s);
    precond_apply<float>(P, o, W.fr.p, W.fz.p, nullptr, s);
    convert(n, W.fz.p, z, s);
  } else {
    precond_apply<double>(P, o, r, z, nullptr, s);
  }
  BA_LAUNCH_CHECK();
}

// ---------------------------------------------------------------- Lanczos

static double plain_dot(ba_plan* P, int n, const double* a, const double* b, hipStream_t s) {
  Scratch& W = *P->scratch;
  hipLaunchKernelGGL((k_dot<DOT_PLAIN, double>), dim3(red_grid(n)), dim3(256), 0, s, n, a, b, W.partial.p,
                     W.scal.p + 1, W.dots.p);
  double v = 0;
  BA_HIP(hipMemcpyAsync(&v, W.dots.p, sizeof(double), hipMemcpyDeviceToHost, s));
  BA_HIP(hipStreamSynchronize(s));
  return v;
}

// lambda_max of D^-1 S on one level: `lanczos_steps` steps of generalized
// Lanczos in the D inner product, then the largest eigenvalue of the
// tridiagonal matrix (k_lanczos_finish). Everything stays on the device
// (L.lz_s): the V-cycle's kernels read 1 / lambda_max from there.
static void lanczos_launch(ba_plan* P, const ba_opts* o, int l, hipStream_t s, int slot) {
  Level& L = P->levels[l];
  const int n = L.n * L.bs;
  Scratch& W = *P->scratch;
  double* partial = W.lz_partial.p + (size_t)slot * RED_BLOCKS;
  PcgScal* red = W.lz_scal.p + slot;
  double* lz = L.lz_s.p;
  BA_HIP(hipMemsetAsync(lz, 0, LZ_SIZE * sizeof(double), s));
  BA_HIP(hipMemsetAsync(L.lz_up.p, 0, n * sizeof(double), s));
  BA_HIP(hipMemsetAsync(L.lz_vp.p, 0, n * sizeof(double), s));
  const int g = grid_of<double>(n);
  const int rg = red_grid(n);
  auto dinv = [&](const double* in, double* out) {
    if (L.bs == 9) blockdiag_apply<9, double>(P, l, in, out, nullptr, s);
    else blockdiag_apply<16, double>(P, l, in, out, nullptr, s);
  };
  auto dot = [&](const double* a, const double* b, int at) {
    hipLaunchKernelGGL((k_dot<DOT_PLAIN, double>), dim3(rg), dim3(256), 0, s, n, a, b, partial, red, lz + at);
  };
  hipLaunchKernelGGL(k_lanczos_start, dim3(g), dim3(256), 0, s, n, l, L.lz_u.p);
  dinv(L.lz_u.p, L.lz_v.p);
  dot(L.lz_v.p, L.lz_u.p, LZ_NRM);
  hipLaunchKernelGGL(k_lanczos_normalize, dim3(g), dim3(256), 0, s, n, L.lz_v.p, L.lz_u.p, (const double*)lz);
  const int steps = o->lanczos_steps;
  for (int j = 0; j < steps; ++j) {
    op_apply<double>(P, l, L.lz_v.p, L.lz_av.p, nullptr, s);
    dot(L.lz_av.p, L.lz_v.p, LZ_ALPHA + j);
    if (j == steps - 1) break;
    dinv(L.lz_av.p, L.lz_dav.p);
    hipLaunchKernelGGL(k_lanczos_update, dim3(g), dim3(256), 0, s, n, j, L.lz_dav.p, L.lz_av.p, L.lz_v.p, L.lz_vp.p,
                       L.lz_u.p, L.lz_up.p, (const double*)lz, L.lz_w.p, L.lz_dw.p);
    dot(L.lz_w.p, L.lz_dw.p, LZ_B2);
    hipLaunchKernelGGL(k_lanczos_record, dim3(1), dim3(1), 0, s, j, lz);
    hipLaunchKernelGGL(k_lanczos_advance, dim3(g), dim3(256), 0, s, n, j, L.lz_v.p, L.lz_vp.p, L.lz_u.p, L.lz_up.p,
                       (const double*)L.lz_w.p, (const double*)L.lz_dw.p, (const double*)lz);
  }
  hipLaunchKernelGGL(k_lanczos_finish, dim3(1), dim3(64), 0, s, steps, lz, P->errflag.p);
  BA_LAUNCH_CHECK();
}

// ---------------------------------------------------------------- multigrid setup

// Dense FP64 inverse of the coarsest level's operator (Algorithm 1's direct
// solve): the equilibrated s S s (s = diag^-1/2) by blocked Gauss-Jordan,
// scaled back: inv = s (s S s)^-1 s.
static void coarse_inverse(ba_plan* P, const ba_opts* o, hipStream_t s) {
  Level& Lc = P->levels.back();
  // The steps alternate between the two matrices; start in the one that makes
  // the last step write Lc.inv, so that the inverse always lands in the same
  // buffer (a captured V-cycle reads it by address).
  const int nbk = Lc.nd / GJB;
  double* src = nbk % 2 == 0 ? Lc.inv.p : Lc.dense.p;
  double* dst = nbk % 2 == 0 ? Lc.dense.p : Lc.inv.p;
  BA_HIP(hipMemsetAsync(src, 0, (size_t)Lc.nd * Lc.nd * sizeof(double), s));
  const int64_t tot = Lc.nnz * Lc.bs * Lc.bs + Lc.nd;
  hipLaunchKernelGGL(k_bsr_to_dense, dim3(grid_of<double>(tot)), dim3(256), 0, s, Lc.n, Lc.bs, Lc.nd, Lc.row_of.p,
                     Lc.col.p, Lc.nnz, Lc.S.p, src);
  DBuf<double>& scl = Lc.gj_scale;
  const int64_t nd2 = (int64_t)Lc.nd * Lc.nd;
  hipLaunchKernelGGL(k_dense_diag, dim3(grid_of<double>(Lc.nd)), dim3(256), 0, s, Lc.nd, src, scl.p,
                     P->errflag.p);
  hipLaunchKernelGGL(k_dense_scale, dim3(grid_of<double>(nd2)), dim3(256), 0, s, Lc.nd, src, scl.p, 0.0);
  // P_0 = A_00^-1 (one workgroup); then step k updates every block with P_k
  // and inverts the next pivot block into P_{k+1} (two alternating buffers).
  hipLaunchKernelGGL(k_gj_pivot<GJB>, dim3(1), dim3(256), 0, s, Lc.nd, (const double*)src, 0, Lc.gj_piv.p,
                     P->errflag.p);
  for (int k = 0; k < nbk; ++k) {
    const double* pk = Lc.gj_piv.p + (size_t)(k & 1) * GJB * GJB;
    double* pn = Lc.gj_piv.p + (size_t)((k + 1) & 1) * GJB * GJB;
    hipLaunchKernelGGL(k_gj_step<GJB>, dim3(nbk * (nbk + 1) / 2), dim3(256), 0, s, Lc.nd, (const double*)src, dst, k, pk,
                       pn, P->errflag.p);
    std::swap(src, dst);
  }
  hipLaunchKernelGGL(k_dense_scale, dim3(grid_of<double>(nd2)), dim3(256), 0, s, Lc.nd, Lc.inv.p, scl.p, 0.0);
  BA_LAUNCH_CHECK();
}


// Numeric multigrid setup as a small task graph on four streams (forked from
// and joined back into s with events):
//   side : near-nullspace, then QR of every level in turn (QR(l+1) needs only
//          the coarse K of QR(l));
//   s    : explicit level-0 S, then per level the Galerkin product (after
//          QR(l)) and the next level's block inverses, then the coarsest
//          level's dense inverse;
//   side2, side, side3: the Lanczos estimate of level l on the (l mod 3)-th,
//          once that level's operator and block inverses are ready.
// Explicit level-0 Schur complement (Section 3.6): diagonal blocks S_cc, then
// the off-diagonal blocks from the shared points of every camera pair.
static void assemble_s0(ba_plan* P, hipStream_t s) {
  Level& L0 = P->levels[0];
  hipLaunchKernelGGL(k_s0_init, dim3(grid_of<double>(L0.nnz * 81)), dim3(256), 0, s, (int64_t)L0.nnz * 81,
                     L0.row_of.p, L0.col.p, P->Scc.p, L0.S.p);
  if (P->s0_chunks == 0) return;
  double* part = P->det ? P->s0_part.p : nullptr;
  hipLaunchKernelGGL(k_explicit_s0, dim3(P->s0_chunks), dim3(64), 0, s, part, P->s0_chunk_e.p, P->s0_chunk_beg.p,
                     L0.row_of.p, L0.col.p, L0.trans_pos.p, P->s0_ptr.p, P->s0_q.p, P->campre.p, P->prec.p,
                     P->pt_off.p, P->obs_cam.p, P->robust ? P->wsq.p : nullptr, L0.S.p);
  if (P->det)
    hipLaunchKernelGGL(k_s0_gather, dim3(ceil_div((int64_t)P->s0_blocks * 81, 243)), dim3(256), 0, s, P->s0_blocks,
                       P->s0_blk_e.p, P->s0_blk_ch.p, L0.trans_pos.p, (const double*)P->s0_part.p, L0.S.p);
}

// Visibility-based block Jacobi: the level-0 aggregates' blocks of S, inverted.
// With a single-level hierarchy every camera is its own cluster and the
// block-Jacobi inverses of the step are used as they are.
static void cluster_setup(ba_plan* P, hipStream_t s) {
  if (P->levels.size() < 2) {
    P->prepared_cj = true;
    return;
  }
  Level& L0 = P->levels[0];
  BA_CHECK((size_t)P->cj_max_n * sizeof(double) <= 64 * 1024, BA_ERR_LIMIT,
           "a cluster of %d cameras exceeds the cluster kernel's LDS", P->cj_max_n / 9);
  assemble_s0(P, s);
  hipLaunchKernelGGL(k_cj_gather, dim3(L0.n_agg), dim3(256), 0, s, L0.agg_ptr.p, L0.agg_mem.p, L0.rowptr32.p,
                     L0.col.p, L0.S.p, P->cj_off.p, P->cj_inv.p);
  hipLaunchKernelGGL(k_cj_invert, dim3(L0.n_agg), dim3(256), 0, s, L0.agg_ptr.p, P->cj_off.p, P->cj_inv.p,
                     P->errflag.p);
  BA_LAUNCH_CHECK();
  check_errflag(P, s, "cluster blocks");
  P->prepared_cj = true;
}

// Numeric setup with the smoothed prolongator, level by level on one stream:
// each level's P_s needs lambda_max of that level's operator (read back to the
// host), and the next level's operator needs P_s. Per level: QR (P_t and the
// coarse K), Lanczos, P_s = (I - w/lambda D^-1 S) P_t, T = S P_s, C = P_s^T T
// and C's smoother blocks; then the coarsest level's dense inverse.
static void mg_setup_sa(ba_plan* P, const ba_opts* o, const double* cams, hipStream_t s) {
  const int nl = (int)P->levels.size();
  Level& L0 = P->levels[0];
  hipLaunchKernelGGL(k_nullspace0, dim3(grid_of<double>(P->n_cam)), dim3(256), 0, s, P->n_cam, cams, P->campre.p,
                     L0.K.p);
  assemble_s0(P, s);
  L0.explicit_op = level0_explicit(P, o, 8);
  std::vector<double> h(1);
  for (int l = 0; l + 1 < nl; ++l) {
    Level& F = P->levels[l];
    Level& C = P->levels[l + 1];
    const size_t lds = (size_t)2 * F.max_agg * F.bs * NS * sizeof(double);
    BA_CHECK(lds <= 160 * 1024, BA_ERR_LIMIT, "aggregate with %d nodes exceeds the QR kernel's LDS", F.max_agg);
    hipLaunchKernelGGL(k_qr_aggregates, dim3(F.n_agg), dim3(64), lds, s, F.bs, F.agg_ptr.p, F.agg_mem.p, F.K.p,
                       F.P.p, C.K.p);
    lanczos_launch(P, o, l, s, 0);
    BA_HIP(hipMemcpyAsync(h.data(), F.lz_s.p + LZ_LMAX, sizeof(double), hipMemcpyDeviceToHost, s));
    check_errflag(P, s, "multigrid setup (QR, smoother blocks, lambda_max)");
    F.lmax = h[0];
    const double c = o->smooth_omega / F.lmax;
    const double* Dinv = lvDinv<double>(P, l);
    if (F.bs == 9) {
      hipLaunchKernelGGL((k_sa_product<9, true>), dim3((unsigned)F.nnz_ps), dim3(256), 0, s, F.ps_src_ptr.p,
                         F.ps_src.p, F.col.p, F.S.p, F.P.p, F.ps_row.p, F.ps_self.p, F.P.p, Dinv, c, F.Ps.p);
      hipLaunchKernelGGL((k_sa_product<9, false>), dim3((unsigned)F.nnz_t), dim3(256), 0, s, F.t_src_ptr.p,
                         F.t_src_op.p, F.t_src_ps.p, F.S.p, F.Ps.p, (const int32_t*)nullptr,
                         (const int32_t*)nullptr, (const double*)nullptr, (const double*)nullptr, 0.0, F.Tsp.p);
      hipLaunchKernelGGL((k_sa_galerkin<9>), dim3((unsigned)C.nnz), dim3(256), 0, s, F.cg_ptr.p, F.cg_ps.p,
                         F.cg_t.p, F.Ps.p, F.Tsp.p, C.S.p);
    } else {
      hipLaunchKernelGGL((k_sa_product<16, true>), dim3((unsigned)F.nnz_ps), dim3(256), 0, s, F.ps_src_ptr.p,
                         F.ps_src.p, F.col.p, F.S.p, F.P.p, F.ps_row.p, F.ps_self.p, F.P.p, Dinv, c, F.Ps.p);
      hipLaunchKernelGGL((k_sa_product<16, false>), dim3((unsigned)F.nnz_t), dim3(256), 0, s, F.t_src_ptr.p,
                         F.t_src_op.p, F.t_src_ps.p, F.S.p, F.Ps.p, (const int32_t*)nullptr,
                         (const int32_t*)nullptr, (const double*)nullptr, (const double*)nullptr, 0.0, F.Tsp.p);
      hipLaunchKernelGGL((k_sa_galerkin<16>), dim3((unsigned)C.nnz), dim3(256), 0, s, F.cg_ptr.p, F.cg_ps.p,
                         F.cg_t.p, F.Ps.p, F.Tsp.p, C.S.p);
    }
    if (l + 1 < nl - 1)
      hipLaunchKernelGGL(k_diag_inverse16, dim3(C.n), dim3(64), 0, s, C.diag_pos.p, C.S.p, C.Dinv.p, P->errflag.p);
    BA_LAUNCH_CHECK();
  }
  coarse_inverse(P, o, s);
  BA_LAUNCH_CHECK();
  P->inspectable_mg = true;
  check_errflag(P, s, "multigrid setup (smoothed prolongator, Galerkin, coarse inverse)");
  P->prepared_mg = true;
}

static void mg_setup(ba_plan* P, const ba_opts* o, const double* cams, bool mixed, hipStream_t s) {
  const int nl = (int)P->levels.size();
  Level& L0 = P->levels[0];
  BA_HIP(hipEventRecord(P->ev_fork, s));
  // ---- side: near-nullspace and the QR chain
  BA_HIP(hipStreamWaitEvent(P->side, P->ev_fork, 0));
  hipLaunchKernelGGL(k_nullspace0, dim3(grid_of<double>(P->n_cam)), dim3(256), 0, P->side, P->n_cam, cams,
                     P->campre.p, L0.K.p);
  for (int l = 0; l + 1 < nl; ++l) {
    Level& F = P->levels[l];
    Level& C = P->levels[l + 1];
    const size_t lds = (size_t)2 * F.max_agg * F.bs * NS * sizeof(double);
    BA_CHECK(lds <= 160 * 1024, BA_ERR_LIMIT, "aggregate with %d nodes exceeds the QR kernel's LDS", F.max_agg);
    hipLaunchKernelGGL(k_qr_aggregates, dim3(F.n_agg), dim3(64), lds, P->side, F.bs, F.agg_ptr.p, F.agg_mem.p,
                       F.K.p, F.P.p, C.K.p);
    BA_HIP(hipEventRecord(P->ev_qr[l], P->side));
  }
  // ---- s: explicit level-0 S (Section 3.6), needed for the Galerkin product
  // and, when cheaper than the implicit form, for smoothing
  assemble_s0(P, s);
  L0.explicit_op = level0_explicit(P, o, mixed ? 4 : 8);
  BA_HIP(hipEventRecord(P->ev_lvl[0], s));
  for (int l = 0; l + 1 < nl; ++l) {
    Level& F = P->levels[l];
    Level& C = P->levels[l + 1];
    BA_HIP(hipStreamWaitEvent(s, P->ev_qr[l], 0));
    hipLaunchKernelGGL(k_galerkin, dim3((unsigned)C.nnz), dim3(256), 0, s, F.bs, F.gal_ptr.p, F.gal_fine.p,
                       F.row_of.p, F.col.p, F.S.p, F.P.p, C.S.p);
    if (l + 1 < nl - 1)
      hipLaunchKernelGGL(k_diag_inverse16, dim3(C.n), dim3(64), 0, s, C.diag_pos.p, C.S.p, C.Dinv.p, P->errflag.p);
    BA_HIP(hipEventRecord(P->ev_lvl[l + 1], s));
  }
  // ---- Lanczos per level, enqueued from a second host thread (its many
  // small launches would otherwise hold back the coarse inverse's), level l
  // on stream l mod 3 of {side2, side, side3} (side once its QR chain is
  // done), so that the levels' estimates run concurrently: each is a chain
  // of small dependent launches. (Streams beyond the process's hardware
  // queues share one; the short estimate of level 2 then still runs last.)
  // (the error message is thread-local: a failure there is re-raised here
  // with its message)
  bool lz_failed = false;
  ba_status lz_status = BA_OK;
  std::string lz_msg;
  std::thread lz([&]() {
    try {
      const hipStream_t lzs[3] = {P->side2, P->side, P->side3};
      for (int l = 0; l + 1 < nl; ++l) {
        BA_HIP(hipStreamWaitEvent(lzs[l % 3], P->ev_lvl[l], 0));
        lanczos_launch(P, o, l, lzs[l % 3], l % 3);
      }
      for (int i = 0; i < 3; ++i) BA_HIP(hipEventRecord(P->ev_lz[i], lzs[i]));
    } catch (const Fail& f) {
      lz_failed = true;
      lz_status = f.st;
      lz_msg = ba_last_error();
    } catch (...) {
      lz_failed = true;
      lz_status = BA_ERR_HIP;
      lz_msg = "Lanczos enqueue failed";
    }
  });
  // ---- s: coarsest level's dense inverse
  try {
    coarse_inverse(P, o, s);
  } catch (...) {
    lz.join();
    throw;
  }
  lz.join();
  BA_CHECK(!lz_failed, lz_status, "%s", lz_msg.c_str());
  BA_LAUNCH_CHECK();
  P->inspectable_mg = true;
  for (hipEvent_t e : P->ev_lz) BA_HIP(hipStreamWaitEvent(s, e, 0));
  // no readback: lambda_max stays on the device, and the error flags are
  // checked once the solve reads its scalars back
  if (mixed) {
    // FP32 copies of level 0 (the coarse levels of the FP32 V-cycle run in FP64)
    convert((size_t)L0.nnz * L0.bs * L0.bs, L0.S.p, L0.S32.p, s);
    if (nl > 1) convert((size_t)L0.n * L0.bs * NS, L0.P.p, L0.P32.p, s);
  }
  P->prepared_mg = true;
}

// ---------------------------------------------------------------- prepare

// planes: also write the FP64 observation planes F and E (the adjoint and the
// LM loop's model read them); the step itself recomputes the blocks where it
// needs them (Schur product, camera blocks, explicit level-0 S,
// back-substitution), so a plain step skips those 192 bytes per observation.
static void prepare(ba_plan* P, const ba_opts* o, const double* cams, const double* pts, const double* uv,
                    const double* D, ba_stats* st, hipStream_t s, bool planes = false) {
  const bool mixed = o->precision == BA_MIXED;
  const uint32_t need = ws_key(o, 0);
  BA_CHECK((P->ws_key & need) == need, BA_ERR_ARG, "internal: the bound workspace does not fit the options");
  BA_CHECK(o->precond != BA_PC_MULTIGRID || (o->prolongator == BA_PROLONG_SMOOTHED) == P->sa, BA_ERR_ARG,
           "the plan was built for the %s prolongator", P->sa ? "smoothed" : "tentative");
  invalidate_step(P);
  P->lambda = o->lambda;
  P->det = o->deterministic != 0;
  P->robust = o->loss != BA_LOSS_SQUARED;
  double* wsq = P->robust ? P->wsq.p : nullptr;
  BA_HIP(hipEventRecord(P->ev_t[0], s));
  hipLaunchKernelGGL(k_campre, dim3(grid_of<double>(P->n_cam)), dim3(256), 0, s, P->n_cam, cams, P->campre.p,
                     P->errflag.p);
  hipLaunchKernelGGL(k_jacobian_tiles, dim3(xcd_grid(P->n_tiles)), dim3(256), 0, s, P->tile_obs.p, P->tile_pt.p, P->pt_off.p,
                     P->obs_slot.p, P->obs_cam.p, P->obs_orig.p, P->pt_orig.p, P->campre.p, pts, uv, P->n_obs_pad,
                     o->lambda, D, P->n_cam, (planes || !SCHUR_RECOMPUTE) ? P->F.p : nullptr,
                     (planes || !SCHUR_RECOMPUTE) ? P->E.p : nullptr, P->fres.p, mixed ? P->F32.p : nullptr,
                     mixed ? P->E32.p : nullptr, P->Cinv.p, mixed ? P->Cinv32.p : nullptr, P->vgp.p, P->gp.p,
                     P->Dp.p, P->prec.p, P->n_tiles, o->loss, o->loss_scale, wsq, P->errflag.p);
  hipLaunchKernelGGL(k_camera_blocks, dim3(xcd_grid(P->n_cam)), dim3(256), 0, s, P->cam_off.p, P->cam_obs.p, P->cam_q.p,
                     P->n_obs_pad, P->campre.p, P->prec.p, P->fres.p, o->lambda, D, P->A.p,
                     mixed ? P->A32.p : nullptr, P->Dc.p, P->b.p, P->Scc.p, P->Sinv.p,
                     mixed ? P->Sinv32.p : nullptr, P->n_cam, wsq, P->errflag.p);
  BA_LAUNCH_CHECK();
  BA_HIP(hipEventRecord(P->ev_t[1], s));
  // The error flags of the blocks and the setup are read back with the
  // solve's first scalars (pcg_run), so that nothing here waits for the GPU
  // (the smoothed-prolongator and cluster setups read back on their own).
  P->have_mixed = mixed;
  P->prepared = true;
  if (o->precond == BA_PC_MULTIGRID) {
    if (P->sa) mg_setup_sa(P, o, cams, s);
    else mg_setup(P, o, cams, mixed, s);
  }
  if (o->precond == BA_PC_CLUSTER_JACOBI) cluster_setup(P, s);
  BA_HIP(hipEventRecord(P->ev_t[2], s));
  if (st) {
    st->levels = (int)P->levels.size();
    for (size_t l = 0; l < P->levels.size() && l < 16; ++l) {
      const Level& L = P->levels[l];
      st->nodes[l] = L.n;
      const bool has = l + 1 < P->levels.size();
      st->agg_min[l] = has ? L.min_agg : 0;
      st->agg_max[l] = has ? L.max_agg : 0;
      st->agg_mean[l] = has ? L.mean_agg : 0.0;
    }
  }
}

// Phase times of the prepared step into st (waits for the setup to finish).
static void prepare_times(ba_plan* P, ba_stats* st) {
  if (!st) return;
  BA_HIP(hipEventSynchronize(P->ev_t[2]));
  float a = 0.f, b = 0.f;
  BA_HIP(hipEventElapsedTime(&a, P->ev_t[0], P->ev_t[1]));
  BA_HIP(hipEventElapsedTime(&b, P->ev_t[1], P->ev_t[2]));
  st->t_jacobian_ms = a;
  st->t_setup_ms = b;
}

// ---------------------------------------------------------------- PCG

template <class T>
struct PcgVecs { T *x, *r, *z, *p, *q; };

struct PcgOut {
  int iters = 0;
  double rr = 0, bb = 0;
  bool converged = false;
  bool breakdown = false;
};

// One PCG iteration (Saad, Algorithm 9.1): p = z + beta p with q = A p, then
// q -= W C^-1 W^T p, alpha = r.z / p.q, x += alpha p, r -= alpha q (and the
// stop tests), z = M r, beta. Every launch returns at once after `done`.
template <class T>
static void pcg_iteration(ba_plan* P, const ba_opts* o, PcgVecs<T> v, hipStream_t s) {
  Scratch& W = *P->scratch;
  PcgScal* sc = W.scal.p;
  const int* done = &sc->done;
  const int n = W.n;
  const int g = red_grid(n);
  hipLaunchKernelGGL((k_pcg_p_Ap<T>), dim3(grid_of<T>(9 * P->n_cam, 252 / 9 * 9)), dim3(256), 0, s, P->n_cam,
                     (const T*)v.z, v.p, A_of<T>(P), v.q, (const PcgScal*)sc);
  schur_tiles_dev<T>(P, v.p, v.q, done, s);
  hipLaunchKernelGGL((k_dot<DOT_ALPHA, T>), dim3(g), dim3(256), 0, s, n, (const T*)v.p, (const T*)v.q, W.partial.p,
                     sc, (double*)nullptr);
  hipLaunchKernelGGL((k_pcg_xr<T>), dim3(g), dim3(256), 0, s, n, (const T*)v.p, (const T*)v.q, v.x, v.r,
                     W.partial.p, sc);
  precond_apply<T>(P, o, v.r, v.z, done, s);
  hipLaunchKernelGGL((k_dot<DOT_BETA, T>), dim3(g), dim3(256), 0, s, n, (const T*)v.r, (const T*)v.z, W.partial.p,
                     sc, (double*)nullptr);
}

// The bytes of everything an iteration's launches depend on beyond the plan's
// fixed arrays: the workspace binding, the options that choose kernels or
// their arguments, level 0's operator form, and the iteration's vectors.
template <class T>
static std::string iteration_key(const ba_plan* P, const ba_opts* o, const PcgVecs<T>& v) {
  std::string k;
  auto put = [&](const void* p, size_t n) { k.append(static_cast<const char*>(p), n); };
  put(&P->ws_base, sizeof(P->ws_base));
  put(&P->ws_key, sizeof(P->ws_key));
  put(&o->precond, sizeof(o->precond));
  put(&o->cheb_degree, sizeof(o->cheb_degree));
  put(&o->cheb_lo, sizeof(o->cheb_lo));
  put(&o->cheb_hi, sizeof(o->cheb_hi));
  const char flags[3] = {(char)P->det, (char)P->sa, (char)(!P->levels.empty() && P->levels[0].explicit_op)};
  put(flags, sizeof(flags));
  put(&v, sizeof(v));
  return k;
}

// The iteration as an executable graph, captured (on the plan's capture
// stream, which records and runs nothing) when nothing cached matches.
template <class T>
static hipGraphExec_t iteration_graph(ba_plan* P, const ba_opts* o, const PcgVecs<T>& v) {
  Scratch& W = *P->scratch;
  const int ti = sizeof(T) == 4 ? 1 : 0;
  std::string key = iteration_key<T>(P, o, v);
  if (W.it_exec[ti] && W.it_key[ti] == key) return W.it_exec[ti];
  if (W.it_exec[ti]) {
    BA_HIP(hipGraphExecDestroy(W.it_exec[ti]));
    W.it_exec[ti] = nullptr;
  }
  // created on first use: a stream takes one of the process's few hardware
  // queues, which the setup's side streams should have to themselves
  if (!P->cap) BA_HIP(hipStreamCreateWithFlags(&P->cap, hipStreamNonBlocking));
  BA_HIP(hipStreamBeginCapture(P->cap, hipStreamCaptureModeThreadLocal));
  hipGraph_t graph = nullptr;
  try {
    pcg_iteration<T>(P, o, v, P->cap);
  } catch (...) {
    (void)hipStreamEndCapture(P->cap, &graph);
    if (graph) (void)hipGraphDestroy(graph);
    throw;
  }
  BA_HIP(hipStreamEndCapture(P->cap, &graph));
  hipGraphExec_t exec = nullptr;
  const hipError_t e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
  (void)hipGraphDestroy(graph);
  BA_HIP(e);
  W.it_exec[ti] = exec;
  W.it_key[ti] = std::move(key);
  return exec;
}

template <class T>
static PcgOut pcg_run(ba_plan* P, const ba_opts* o, const T* b, PcgVecs<T> v, double rtol, int max_iter,
                      hipStream_t s, double forcing = -1.0) {
  Scratch& W = *P->scratch;
  PcgScal* sc = W.scal.p;
  const int n = W.n;
  const int g = red_grid(n);
  hipLaunchKernelGGL((k_pcg_start<T>), dim3(g), dim3(256), 0, s, n, b, v.x, v.r, v.p, W.partial.p, sc, rtol * rtol,
                     forcing);
  precond_apply<T>(P, o, v.r, v.z, nullptr, s);
  hipLaunchKernelGGL((k_dot<DOT_INIT, T>), dim3(g), dim3(256), 0, s, n, (const T*)v.r, (const T*)v.z, W.partial.p,
                     sc, (double*)nullptr);
  const hipGraphExec_t exec = o->graph ? iteration_graph<T>(P, o, v) : nullptr;
  PcgOut out;
  for (int it = 0; it < max_iter; ++it) {
    if (exec) BA_HIP(hipGraphLaunch(exec, s));
    else pcg_iteration<T>(P, o, v, s);
    if ((it + 1) % o->check_every == 0 || it + 1 == max_iter) {
      BA_HIP(hipMemcpyAsync(W.h_scal, sc, sizeof(PcgScal), hipMemcpyDeviceToHost, s));
      BA_HIP(hipStreamSynchronize(s));
      if (W.h_scal->done) break;
    }
  }
  BA_LAUNCH_CHECK();
  BA_HIP(hipMemcpyAsync(W.h_scal, sc, sizeof(PcgScal), hipMemcpyDeviceToHost, s));
  BA_HIP(hipMemcpyAsync(P->h_err, P->errflag.p, sizeof(uint32_t), hipMemcpyDeviceToHost, s));
  BA_HIP(hipStreamSynchronize(s));
  // an error of the step's blocks or preconditioner setup takes precedence
  // over what the iteration made of it
  if (*P->h_err) check_errflag(P, s, "normal blocks or preconditioner setup");
  out.iters = W.h_scal->iters;
  out.rr = W.h_scal->rr;
  out.bb = W.h_scal->bb;
  out.breakdown = W.h_scal->flag != 0;
  out.converged = W.h_scal->done && !out.breakdown;
  return out;
}

// Solve S x = b (b: FP64 device [n_cam*9]) into W.x; returns status and fills stats.
// forcing >= 0 adds the Nash-Sofer stop rule to the FP64 PCG (the mixed form
// keeps the residual rule: its inner solves have their own tolerances).
static ba_status solve_camera_system(ba_plan* P, const ba_opts* o, const double* b, ba_stats* st, hipStream_t s,
                                     double forcing = -1.0) {
  Scratch& W = *P->scratch;
  const int n = W.n;
  ba_status status = BA_OK;
  if (o->precision == BA_FP64) {
    PcgOut r = pcg_run<double>(P, o, b, PcgVecs<double>{W.x.p, W.r.p, W.z.p, W.p.p, W.q.p}, o->rtol, o->max_iter, s,
                               forcing);
    if (st) {   // also on a breakdown: the iterations spent are reported
      st->iters = r.iters;
      st->rel_res = r.bb > 0 ? std::sqrt(r.rr / r.bb) : 0.0;
    }
    BA_CHECK(!r.breakdown, BA_ERR_NOT_SPD, "PCG breakdown: the operator or preconditioner is not SPD");
    if (!r.converged) status = BA_NOT_CONVERGED;
  } else {
    // FP64 iterative refinement around FP32 PCG
    BA_HIP(hipMemsetAsync(W.x.p, 0, n * sizeof(double), s));
    BA_HIP(hipMemcpyAsync(W.t.p, b, n * sizeof(double), hipMemcpyDeviceToDevice, s));   // t = residual
    const double bb = plain_dot(P, n, b, b, s);
    double rr = bb;
    int iters = 0, ref = 0;
    bool conv = bb == 0.0;
    for (; ref < o->max_refine && !conv; ++ref) {
      convert(n, W.t.p, W.fb.p, s);
      // the inner solve needs to reduce the current residual only to the outer
      // target (with a factor 2 margin), never by less than inner_rtol
      const double need = 0.5 * o->rtol * std::sqrt(bb / rr);
      const double tol = std::min(0.5, std::max(o->inner_rtol, need));
      PcgOut r = pcg_run<float>(P, o, W.fb.p, PcgVecs<float>{W.fx.p, W.fr.p, W.fz.p, W.fp.p, W.fq.p}, tol,
                                o->max_iter, s);
      iters += r.iters;
      if (r.breakdown) {
        // The FP32 operator or preconditioner lost definiteness (S's smallest
        // eigenvalues below FP32 rounding of its terms): keep the iterate
        // reached, and finish with an FP64 PCG on the FP64 residual.
        if (r.iters > 0) {
          hipLaunchKernelGGL(k_add_f32, dim3(grid_of<double>(n)), dim3(256), 0, s, n, W.fx.p, W.x.p);
          schur_apply_dev<double>(P, W.x.p, W.q.p, nullptr, s);
          hipLaunchKernelGGL(k_axpby, dim3(grid_of<double>(n)), dim3(256), 0, s, n, b, -1.0, W.q.p, W.t.p);
          rr = plain_dot(P, n, W.t.p, W.t.p, s);
        }
        const double tol64 = std::min(0.5, o->rtol * std::sqrt(bb / std::max(rr, 1e-300)));
        PcgOut r64 = pcg_run<double>(P, o, W.t.p, PcgVecs<double>{W.e.p, W.r.p, W.z.p, W.p.p, W.q.p}, tol64,
                                     o->max_iter, s);
        iters += r64.iters;
        if (st) st->iters = iters;
        BA_CHECK(!r64.breakdown, BA_ERR_NOT_SPD, "PCG breakdown: the operator or preconditioner is not SPD");
        hipLaunchKernelGGL(k_add_f64, dim3(grid_of<double>(n)), dim3(256), 0, s, n, (const double*)W.e.p, W.x.p);
        if (st) st->fallback_fp64 = 1;
      } else {
        hipLaunchKernelGGL(k_add_f32, dim3(grid_of<double>(n)), dim3(256), 0, s, n, W.fx.p, W.x.p);
      }
      schur_apply_dev<double>(P, W.x.p, W.q.p, nullptr, s);
      hipLaunchKernelGGL(k_axpby, dim3(grid_of<double>(n)), dim3(256), 0, s, n, b, -1.0, W.q.p, W.t.p);
      rr = plain_dot(P, n, W.t.p, W.t.p, s);
      conv = rr <= o->rtol * o->rtol * bb;
      if (r.breakdown) {
        ++ref;
        break;
      }
    }
    if (st) {
      st->iters = iters;
      st->refine_steps = ref;
      st->rel_res = bb > 0 ? std::sqrt(rr / bb) : 0.0;
    }
    if (!conv) status = BA_NOT_CONVERGED;
  }
  return status;
}

static ba_status solve(ba_plan* P, const ba_opts* o, double* delta_cam, double* delta_pt, ba_stats* st,
                       hipStream_t s) {
  BA_CHECK(o->precond != BA_PC_MULTIGRID || P->prepared_mg, BA_ERR_ARG,
           "the step was prepared without the multigrid preconditioner");
  BA_CHECK(o->precond != BA_PC_CLUSTER_JACOBI || P->prepared_cj, BA_ERR_ARG,
           "the step was prepared without the cluster preconditioner");
  BA_CHECK(o->precision == BA_FP64 || P->have_mixed, BA_ERR_ARG, "the step was prepared without BA_MIXED");
  Timer ts(s);
  Scratch& W = *P->scratch;
  const ba_status status =
      solve_camera_system(P, o, P->b.p, st, s, o->stop_rule == BA_STOP_NASH_SOFER ? o->forcing : -1.0);
  BA_HIP(hipMemcpyAsync(delta_cam, W.x.p, (size_t)W.n * sizeof(double), hipMemcpyDeviceToDevice, s));
  // back-substitution delta_p = C^-1 (-g_p - W^T delta_c)
  // (F_o, E_o recomputed from the cameras and point records: the planes may not be written)
  hipLaunchKernelGGL(k_recover_tiles, dim3(xcd_grid(P->n_tiles)), dim3(256), 0, s, P->tile_obs.p, P->tile_pt.p, P->pt_off.p,
                     P->pt_orig.p, P->obs_cam.p, P->n_obs_pad, (const double*)nullptr, (const double*)nullptr,
                     P->obs_pt.p, (const double*)P->campre.p, (const double*)P->prec.p,
                     P->robust ? (const double*)P->wsq.p : nullptr, P->Cinv.p, P->gp.p, -1.0, W.x.p, delta_pt,
                     P->n_tiles);
  BA_LAUNCH_CHECK();
  const double t = ts.ms();
  if (st) st->t_solve_ms = t;
  return status;
}

// ---------------------------------------------------------------- inspection

static void level_data(const ba_plan* Pc, int l, int what, double* out, hipStream_t s) {
  ba_plan* P = const_cast<ba_plan*>(Pc);
  Level& L = P->levels[l];
  const int nl = (int)P->levels.size();
  const size_t nv = (size_t)L.n * L.bs;
  switch (what) {
    case 0: {
      BA_CHECK(nv <= 16384, BA_ERR_LIMIT, "level too large for a dense copy");
      BA_HIP(hipMemsetAsync(out, 0, nv * nv * sizeof(double), s));
      hipLaunchKernelGGL(k_bsr_to_dense, dim3(grid_of<double>(L.nnz * L.bs * L.bs)), dim3(256), 0, s, L.n, L.bs,
                         (int)nv, L.row_of.p, L.col.p, L.nnz, L.S.p, out);
      break;
    }
    case 1:
      BA_CHECK(l + 1 < nl, BA_ERR_ARG, "the coarsest level has no prolongator");
      BA_HIP(hipMemcpyAsync(out, L.P.p, L.P.bytes(), hipMemcpyDeviceToDevice, s));
      break;
    case 2:
      BA_HIP(hipMemcpyAsync(out, L.K.p, L.K.bytes(), hipMemcpyDeviceToDevice, s));
      break;
    case 3:
      BA_CHECK(l + 1 < nl, BA_ERR_ARG, "the coarsest level has no smoother");
      BA_HIP(hipMemcpyAsync(out, lvDinv<double>(P, l), (size_t)L.n * L.bs * L.bs * sizeof(double),
                            hipMemcpyDeviceToDevice, s));
      break;
    case 4:
      BA_CHECK(l + 1 < nl, BA_ERR_ARG, "the coarsest level has no smoother");
      BA_HIP(hipMemcpyAsync(out, L.lz_s.p + LZ_LMAX, sizeof(double), hipMemcpyDeviceToDevice, s));
      break;
    case 5:
      BA_CHECK(l + 1 == nl, BA_ERR_ARG, "only the coarsest level has an inverse");
      BA_HIP(hipMemcpy2DAsync(out, nv * sizeof(double), L.inv.p, (size_t)L.nd * sizeof(double), nv * sizeof(double),
                              nv, hipMemcpyDeviceToDevice, s));
      break;
    case 6: {
      BA_CHECK(P->sa, BA_ERR_ARG, "the plan was not built for the smoothed prolongator");
      BA_CHECK(l + 1 < nl, BA_ERR_ARG, "the coarsest level has no prolongator");
      BA_CHECK(nv <= 16384, BA_ERR_LIMIT, "level too large for a dense copy");
      const int ncols = P->levels[l + 1].n * NS;
      BA_HIP(hipMemsetAsync(out, 0, nv * ncols * sizeof(double), s));
      hipLaunchKernelGGL(k_sa_to_dense, dim3(grid_of<double>(L.nnz_ps * L.bs * NS)), dim3(256), 0, s, L.nnz_ps,
                         L.bs, ncols, L.ps_row.p, L.ps_col.p, L.Ps.p, out);
      break;
    }
    default:
      BA_CHECK(false, BA_ERR_ARG, "bad `what`");
  }
  BA_LAUNCH_CHECK();
  BA_HIP(hipStreamSynchronize(s));
}

}  // namespace bamg

#include "backward.cpp"
#include "lm.cpp"
