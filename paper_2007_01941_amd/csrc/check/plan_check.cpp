// Host-side checker of the library, meant to be built with AddressSanitizer
// and UndefinedBehaviorSanitizer on its host code (the kernels are the
// library's own, unchanged). It drives every C-ABI call that builds or walks
// host-side structures -- plan creation (observation sort, tiles and groups,
// covisibility, aggregation, Galerkin and smoothed-aggregation gather lists),
// workspace layout and binding, steps with every preconditioner and precision,
// the adjoint, the cost, the LM loop, hierarchy inspection and the error paths
// -- on one scene read from a file, and exits non-zero on the first failure.
//
// Usage: plan_check <scene.bin>
//   scene.bin (little endian): int32 n_cam, int32 n_pt, int64 n_obs,
//   int32 obs_cam[n_obs], int32 obs_pt[n_obs], double cams[n_cam][9],
//   double pts[n_pt][3], double uv[n_obs][2].
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <vector>

#include "bamg.h"

// Ends the process without running static destructors: the checker's last
// step has been checked by then, and the HIP runtime's own teardown (not this
// library's code) trips the sanitizer's device-allocator bookkeeping.
[[noreturn]] static void quit(int rc) {
  std::fflush(nullptr);
  std::_Exit(rc);
}

#define HIPOK(x)                                                                   \
  do {                                                                             \
    hipError_t e_ = (x);                                                           \
    if (e_ != hipSuccess) {                                                        \
      std::fprintf(stderr, "[check] %s:%d %s\n", __FILE__, __LINE__, hipGetErrorString(e_)); \
      quit(2);                                                                \
    }                                                                              \
  } while (0)

static void expect(ba_status got, ba_status want, const char* what) {
  if (got != want) {
    std::fprintf(stderr, "[check] %s: %s (want %s): %s\n", what, ba_status_str(got), ba_status_str(want),
                 ba_last_error());
    quit(1);
  }
  std::printf("[check] %s: %s\n", what, ba_status_str(got));
  std::fflush(stdout);
}

static void expect_ok(ba_status got, const char* what) {
  if (got != BA_OK && got != BA_NOT_CONVERGED) expect(got, BA_OK, what);
  std::printf("[check] %s: %s\n", what, ba_status_str(got));
  std::fflush(stdout);
}

// Allocation callbacks that count what is live.
struct Counter {
  long live = 0, total = 0;
};
static void* count_alloc(size_t bytes, void* ctx) {
  void* p = nullptr;
  if (hipMalloc(&p, bytes) != hipSuccess) return nullptr;
  auto* c = static_cast<Counter*>(ctx);
  ++c->live;
  ++c->total;
  return p;
}
static void count_free(void* p, void* ctx) {
  (void)hipFree(p);
  --static_cast<Counter*>(ctx)->live;
}

template <class T>
static T* upload(const std::vector<T>& h) {
  T* d = nullptr;
  HIPOK(hipMalloc(&d, std::max<size_t>(1, h.size()) * sizeof(T)));
  if (!h.empty()) HIPOK(hipMemcpy(d, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice));
  return d;
}

template <class T>
static T* dalloc(size_t n) {
  T* d = nullptr;
  HIPOK(hipMalloc(&d, std::max<size_t>(1, n) * sizeof(T)));
  return d;
}

int main(int argc, char** argv) {
  std::setvbuf(stdout, nullptr, _IOLBF, 0);
  if (argc != 2) {
    std::fprintf(stderr, "usage: plan_check <scene.bin>\n");
    return 2;
  }
  FILE* f = std::fopen(argv[1], "rb");
  if (!f) {
    std::fprintf(stderr, "[check] cannot open %s\n", argv[1]);
    return 2;
  }
  int32_t n_cam = 0, n_pt = 0;
  int64_t n_obs = 0;
  bool ok = std::fread(&n_cam, 4, 1, f) == 1 && std::fread(&n_pt, 4, 1, f) == 1 && std::fread(&n_obs, 8, 1, f) == 1;
  if (!ok || n_cam < 2 || n_pt < 1 || n_obs < 2) {
    std::fprintf(stderr, "[check] bad header\n");
    return 2;
  }
  std::vector<int32_t> oc(n_obs), op(n_obs);
  std::vector<double> cams((size_t)n_cam * 9), pts((size_t)n_pt * 3), uv((size_t)n_obs * 2);
  ok = std::fread(oc.data(), 4, n_obs, f) == (size_t)n_obs && std::fread(op.data(), 4, n_obs, f) == (size_t)n_obs &&
       std::fread(cams.data(), 8, cams.size(), f) == cams.size() &&
       std::fread(pts.data(), 8, pts.size(), f) == pts.size() && std::fread(uv.data(), 8, uv.size(), f) == uv.size();
  std::fclose(f);
  if (!ok) {
    std::fprintf(stderr, "[check] short file\n");
    return 2;
  }
  std::printf("[check] scene: %d cameras, %d points, %lld observations\n", n_cam, n_pt, (long long)n_obs);
  hipStream_t s;
  HIPOK(hipStreamCreate(&s));
  int32_t* d_oc = upload(oc);
  int32_t* d_op = upload(op);
  double* d_cams = upload(cams);
  double* d_pts = upload(pts);
  double* d_uv = upload(uv);
  double* dc = dalloc<double>((size_t)n_cam * 9);
  double* dp = dalloc<double>((size_t)n_pt * 3);

  // ---- error paths of plan creation (checked before or during the layout)
  {
    ba_opts o;
    ba_opts_default(&o);
    ba_plan* p = nullptr;
    std::vector<int32_t> bad = oc;
    bad[n_obs / 2] = n_cam;   // out of range
    int32_t* d_bad = upload(bad);
    expect(ba_plan_create(n_cam, n_pt, n_obs, d_bad, d_op, &o, nullptr, nullptr, nullptr, s, &p), BA_ERR_INDEX,
           "plan with a camera index out of range");
    HIPOK(hipFree(d_bad));
    std::vector<int32_t> dup_c(oc), dup_p(op);
    dup_c.push_back(oc[0]);
    dup_p.push_back(op[0]);   // the same (camera, point) twice
    int32_t* d_dc = upload(dup_c);
    int32_t* d_dp = upload(dup_p);
    expect(ba_plan_create(n_cam, n_pt, n_obs + 1, d_dc, d_dp, &o, nullptr, nullptr, nullptr, s, &p),
           BA_ERR_STRUCTURE, "plan with a duplicate observation");
    HIPOK(hipFree(d_dc));
    HIPOK(hipFree(d_dp));
    std::vector<int32_t> one_p(op);
    for (auto& q : one_p) if (q == n_pt - 1) q = 0;
    // point n_pt - 1 has no observations now (and point 0 may hold duplicates)
    int32_t* d_1p = upload(one_p);
    expect(ba_plan_create(n_cam, n_pt, n_obs, d_oc, d_1p, &o, nullptr, nullptr, nullptr, s, &p), BA_ERR_STRUCTURE,
           "plan with an unobserved point");
    HIPOK(hipFree(d_1p));
  }

  Counter counter;
  for (int smooth = 0; smooth < 2; ++smooth) {
    ba_opts o;
    ba_opts_default(&o);
    o.coarse_max_nodes = 16;
    o.prolongator = smooth ? BA_PROLONG_SMOOTHED : BA_PROLONG_TENTATIVE;
    ba_plan* p = nullptr;
    expect(ba_plan_create(n_cam, n_pt, n_obs, d_oc, d_op, &o, smooth ? count_alloc : nullptr,
                          smooth ? count_free : nullptr, &counter, s, &p),
           BA_OK, smooth ? "plan (smoothed prolongator, counted allocations)" : "plan (tentative prolongator)");
    std::printf("[check] plan bytes %zu\n", ba_plan_bytes(p));
    int32_t nl = 0, nodes[16];
    expect(ba_mg_levels(p, &nl, nodes), BA_OK, "levels");
    // steps: every preconditioner, precision and mode the plan allows
    const int pcs[3] = {BA_PC_BLOCK_JACOBI, BA_PC_MULTIGRID, BA_PC_CLUSTER_JACOBI};
    for (int pc : pcs) {
      for (int prec = 0; prec < 2; ++prec) {
        for (int det = 0; det < 2; ++det) {
          ba_opts so = o;
          so.precond = pc;
          so.precision = prec ? BA_MIXED : BA_FP64;
          so.deterministic = det;
          so.rtol = 1e-8;
          const bool allowed = !(prec && pc == BA_PC_CLUSTER_JACOBI) && !(prec && smooth && pc == BA_PC_MULTIGRID);
          ba_stats st;
          char what[96];
          std::snprintf(what, sizeof(what), "step pc=%d %s det=%d", pc, prec ? "mixed" : "fp64", det);
          ba_status r = ba_lm_step(p, &so, d_cams, d_pts, d_uv, nullptr, nullptr, 0, dc, dp, &st, s);
          if (!allowed) {
            expect(r, BA_ERR_ARG, what);
            continue;
          }
          expect_ok(r, what);
          if (pc == BA_PC_MULTIGRID && st.levels > 1 && !(st.agg_min[0] >= 1 && st.agg_max[0] >= st.agg_min[0])) {
            std::fprintf(stderr, "[check] aggregate statistics missing\n");
            quit(1);
          }
        }
      }
    }
    // the step in a caller's workspace: exact, short and misaligned
    {
      ba_opts so = o;
      const size_t need = ba_workspace_bytes(p, &so, BA_USE_STEP);
      char* ws = dalloc<char>(need + 256);
      expect_ok(ba_lm_step(p, &so, d_cams, d_pts, d_uv, nullptr, ws, need, dc, dp, nullptr, s),
                "step in a caller workspace");
      expect(ba_lm_step(p, &so, d_cams, d_pts, d_uv, nullptr, ws, need - 256, dc, dp, nullptr, s),
             BA_ERR_WORKSPACE, "step in a short workspace");
      expect(ba_lm_step(p, &so, d_cams, d_pts, d_uv, nullptr, ws + 8, need, dc, dp, nullptr, s), BA_ERR_ARG,
             "step in a misaligned workspace");
      HIPOK(hipFree(ws));
    }
    // a step with the other prolongator than the plan's
    {
      ba_opts so = o;
      so.prolongator = smooth ? BA_PROLONG_TENTATIVE : BA_PROLONG_SMOOTHED;
      expect(ba_lm_step(p, &so, d_cams, d_pts, d_uv, nullptr, nullptr, 0, dc, dp, nullptr, s), BA_ERR_ARG,
             "step with the other prolongator");
    }
    // hierarchy inspection after a multigrid step
    expect_ok(ba_lm_step(p, &o, d_cams, d_pts, d_uv, nullptr, nullptr, 0, dc, dp, nullptr, s), "multigrid step");
    for (int l = 0; l < nl; ++l) {
      const int bs = l == 0 ? 9 : 16;
      const size_t nv = (size_t)nodes[l] * bs;
      int64_t nnz = 0;
      expect(ba_mg_covisibility(p, l, &nnz, nullptr, nullptr, nullptr), BA_OK, "covisibility size");
      int64_t* rp = dalloc<int64_t>(nodes[l] + 1);
      int32_t* col = dalloc<int32_t>(nnz);
      int64_t* val = dalloc<int64_t>(nnz);
      expect(ba_mg_covisibility(p, l, &nnz, rp, col, val), BA_OK, "covisibility");
      HIPOK(hipFree(rp));
      HIPOK(hipFree(col));
      HIPOK(hipFree(val));
      if (l + 1 < nl) {
        int32_t* agg = dalloc<int32_t>(nodes[l]);
        expect(ba_mg_aggregates(p, l, agg), BA_OK, "aggregates");
        HIPOK(hipFree(agg));
      }
      const size_t nc = l + 1 < nl ? (size_t)nodes[l + 1] * 16 : 0;
      for (int what = 0; what <= 6; ++what) {
        size_t n = 0;
        bool valid = true;
        switch (what) {
          case 0: n = nv * nv; valid = nv <= 16384; break;
          case 1: case 2: n = nv * 16; valid = what == 2 || l + 1 < nl; break;
          case 3: n = (size_t)nodes[l] * bs * bs; valid = l + 1 < nl; break;
          case 4: n = 1; valid = l + 1 < nl; break;
          case 5: n = nv * nv; valid = l + 1 == nl; break;
          case 6: n = nv * nc; valid = smooth && l + 1 < nl && nv <= 16384; break;
        }
        double* out = dalloc<double>(std::max<size_t>(n, 1));
        char what_s[64];
        std::snprintf(what_s, sizeof(what_s), "level %d data %d", l, what);
        ba_status r = ba_mg_level_data(p, l, what, out, s);
        if (valid) expect(r, BA_OK, what_s);
        else if (r == BA_OK) expect(r, BA_ERR_ARG, what_s);
        HIPOK(hipFree(out));
      }
    }
    // the adjoint
    if (!smooth) {
      double* g_c = dalloc<double>((size_t)n_cam * 9);
      double* g_p = dalloc<double>((size_t)n_pt * 3);
      double* g_u = dalloc<double>((size_t)n_obs * 2);
      expect_ok(ba_lm_step_backward(p, &o, d_cams, d_pts, d_uv, nullptr, dc, dp, dc, dp, nullptr, 0, g_c, g_p, g_u,
                                    nullptr, s),
                "adjoint");
      HIPOK(hipFree(g_c));
      HIPOK(hipFree(g_p));
      HIPOK(hipFree(g_u));
    }
    // cost, and the allocation-free cost
    double cost = 0.0, cost2 = 0.0;
    int64_t bad = -1, bad2 = -1;
    expect(ba_cost(p, &o, d_cams, d_pts, d_uv, nullptr, 0, &cost, &bad, s), BA_OK, "cost");
    if (n_cam <= 32768) {
      expect(ba_cost_noalloc(p, &o, d_cams, d_pts, d_uv, &cost2, &bad2, s), BA_OK, "cost without allocation");
      if (!(std::fabs(cost - cost2) <= 1e-12 * std::fabs(cost)) || bad != bad2) {
        std::fprintf(stderr, "[check] cost %.17g vs %.17g\n", cost, cost2);
        quit(1);
      }
    }
    // a few LM iterations on copies of the parameters
    {
      double* c2 = upload(cams);
      double* p2 = upload(pts);
      ba_lm_opts lo;
      ba_lm_opts_default(&lo);
      lo.max_iters = 4;
      std::vector<ba_lm_iter> hist(lo.max_iters);
      ba_lm_summary sum;
      ba_opts so = o;
      so.stop_rule = BA_STOP_NASH_SOFER;
      so.loss = smooth ? BA_LOSS_SQUARED : BA_LOSS_HUBER;
      expect(ba_lm_solve(p, &so, &lo, c2, p2, d_uv, nullptr, 0, hist.data(), &sum, s), BA_OK, "LM loop");
      std::printf("[check] LM: %d iterations, cost %.6e -> %.6e\n", sum.iters, sum.cost0, sum.cost);
      HIPOK(hipFree(c2));
      HIPOK(hipFree(p2));
    }
    ba_plan_destroy(p);
  }
  if (counter.live != 0 || counter.total == 0) {
    std::fprintf(stderr, "[check] allocation callbacks: %ld live after destroy (%ld total)\n", counter.live,
                 counter.total);
    quit(1);
  }
  std::printf("[check] allocation callbacks balanced (%ld allocations)\n", counter.total);
  for (void* q : {(void*)d_oc, (void*)d_op, (void*)d_cams, (void*)d_pts, (void*)d_uv, (void*)dc, (void*)dp})
    HIPOK(hipFree(q));
  HIPOK(hipStreamDestroy(s));
  std::printf("[check] OK\n");
  quit(0);
}
