// Plan construction: the integer structure of one visibility graph.
//
// Host part (once per visibility structure): validation, point-major order,
// point reordering by lowest observing camera (so that a tile of consecutive
// points touches few cameras), camera-major lists and tiles. Device part: the
// covisibility counts, strength ordering and greedy aggregation of every
// multigrid level (mg_plan_kernels.hip); the host then derives the block
// patterns and Galerkin gather lists from the aggregates.
#include <algorithm>
#include <array>
#include <numeric>

#include "kernels.hpp"

namespace bamg {

static void build_observation_layout(ba_plan* P, const std::vector<int32_t>& oc,
                                     const std::vector<int32_t>& op, hipStream_t s) {
  const int n_cam = P->n_cam, n_pt = P->n_pt;
  const int64_t n_obs = P->n_obs;
  for (int64_t o = 0; o < n_obs; ++o) {
    BA_CHECK(oc[o] >= 0 && oc[o] < n_cam, BA_ERR_INDEX, "observation %lld: camera index %d out of [0, %d)",
             (long long)o, oc[o], n_cam);
    BA_CHECK(op[o] >= 0 && op[o] < n_pt, BA_ERR_INDEX, "observation %lld: point index %d out of [0, %d)",
             (long long)o, op[o], n_pt);
  }
  std::vector<int32_t> cnt(n_pt, 0), ccnt(n_cam, 0);
  for (int64_t o = 0; o < n_obs; ++o) { ++cnt[op[o]]; ++ccnt[oc[o]]; }
  int max_k = 0;
  for (int p = 0; p < n_pt; ++p) {
    BA_CHECK(cnt[p] >= 2, BA_ERR_STRUCTURE, "point %d has %d observation(s); at least 2 are required", p, cnt[p]);
    max_k = std::max(max_k, cnt[p]);
  }
  BA_CHECK(max_k <= 65535, BA_ERR_LIMIT, "a point is seen by %d cameras (limit 65535)", max_k);
  // Every covisibility count of every level is at most sum_p k_p^2 (the sum of
  // all entries of W = V V^T, which Ahat^T W Ahat keeps); the exact strength
  // comparison multiplies three counts in 128 bits, so they must stay < 2^42.
  {
    int64_t wsum = 0;
    for (int p = 0; p < n_pt; ++p) wsum += (int64_t)cnt[p] * cnt[p];
    BA_CHECK(wsum < (int64_t(1) << 42), BA_ERR_LIMIT,
             "sum over points of (observations per point)^2 = %lld exceeds 2^42", (long long)wsum);
  }
  for (int c = 0; c < n_cam; ++c)
    BA_CHECK(ccnt[c] >= 1, BA_ERR_STRUCTURE, "camera %d observes no point", c);
  // point-major, stable in the caller's order, then each point's views by camera
  std::vector<int64_t> off(n_pt + 1, 0);
  for (int p = 0; p < n_pt; ++p) off[p + 1] = off[p] + cnt[p];
  std::vector<int32_t> pm(n_obs);
  {
    std::vector<int64_t> cur(off.begin(), off.end() - 1);
    for (int64_t o = 0; o < n_obs; ++o) pm[cur[op[o]]++] = (int32_t)o;
  }
  for (int p = 0; p < n_pt; ++p) {
    auto b = pm.begin() + off[p], e = pm.begin() + off[p + 1];
    std::sort(b, e, [&](int32_t x, int32_t y) { return oc[x] < oc[y]; });
    for (auto it = b + 1; it < e; ++it)
      BA_CHECK(oc[*it] != oc[*(it - 1)], BA_ERR_STRUCTURE,
               "camera %d observes point %d more than once", oc[*it], p);
  }
  // reorder points by their lowest observing camera (stable)
  std::vector<int32_t> key(n_pt);
  for (int p = 0; p < n_pt; ++p) key[p] = oc[pm[off[p]]];
  std::vector<int64_t> kstart(n_cam + 1, 0);
  for (int p = 0; p < n_pt; ++p) ++kstart[key[p] + 1];
  for (int c = 0; c < n_cam; ++c) kstart[c + 1] += kstart[c];
  P->h_pt_orig.assign(n_pt, 0);
  for (int p = 0; p < n_pt; ++p) P->h_pt_orig[kstart[key[p]]++] = p;
  std::vector<int32_t> pt_new(n_pt);
  for (int q = 0; q < n_pt; ++q) pt_new[P->h_pt_orig[q]] = q;
  // observation arrays in the new order
  P->h_obs_cam.resize(n_obs);
  P->h_obs_pt.resize(n_obs);
  P->h_obs_orig.resize(n_obs);
  P->h_pt_off.assign(n_pt + 1, 0);
  int64_t w = 0;
  for (int q = 0; q < n_pt; ++q) {
    const int p = P->h_pt_orig[q];
    P->h_pt_off[q] = w;
    for (int64_t k = off[p]; k < off[p + 1]; ++k) {
      const int32_t o = pm[k];
      P->h_obs_cam[w] = oc[o];
      P->h_obs_pt[w] = q;
      P->h_obs_orig[w] = o;
      ++w;
    }
  }
  P->h_pt_off[n_pt] = w;
  std::vector<int32_t> rank(n_obs);
  for (int64_t o = 0; o < n_obs; ++o) rank[P->h_obs_orig[o]] = (int32_t)o;
  // camera-major lists of point-major observation indices (ascending)
  P->h_cam_off.assign(n_cam + 1, 0);
  for (int c = 0; c < n_cam; ++c) P->h_cam_off[c + 1] = P->h_cam_off[c] + ccnt[c];
  P->h_cam_obs.resize(n_obs);
  {
    std::vector<int64_t> cur(P->h_cam_off.begin(), P->h_cam_off.end() - 1);
    for (int64_t o = 0; o < n_obs; ++o) P->h_cam_obs[cur[P->h_obs_cam[o]]++] = (int32_t)o;
  }
  // tiles of whole points with <= TILE_OBS observations
  std::vector<int32_t> t_obs{0}, t_pt{0};
  {
    int cur = 0;
    for (int q = 0; q < n_pt; ++q) {
      const int k = (int)(P->h_pt_off[q + 1] - P->h_pt_off[q]);
      if (cur > 0 && cur + k > TILE_OBS) {
        t_obs.push_back((int32_t)P->h_pt_off[q]);
        t_pt.push_back(q);
        cur = 0;
      }
      cur += k;
    }
    t_obs.push_back((int32_t)n_obs);
    t_pt.push_back(n_pt);
  }
  const int n_tiles = (int)t_obs.size() - 1;
  // Per tile: its distinct cameras (ascending; an observation's camera slot is
  // the index in this list), and the tile's observations sorted by slot: the
  // rank of each observation in that order and the first rank of every slot.
  std::vector<int32_t> t_coff{0}, t_cams, t_cseg;
  std::vector<uint32_t> slot(n_obs);
  std::vector<int32_t> mark(n_cam, -1), slot_of(n_cam, 0);
  int max_tc = 0;
  for (int t = 0; t < n_tiles; ++t) {
    std::vector<int32_t> cams;
    for (int64_t o = t_obs[t]; o < t_obs[t + 1]; ++o) {
      const int c = P->h_obs_cam[o];
      if (mark[c] != t) { mark[c] = t; cams.push_back(c); }
    }
    std::sort(cams.begin(), cams.end());
    BA_CHECK(cams.size() <= 65535, BA_ERR_LIMIT, "tile with too many cameras");
    for (size_t i = 0; i < cams.size(); ++i) slot_of[cams[i]] = (int32_t)i;
    std::vector<int32_t> seg(cams.size() + 1, 0);
    for (int64_t o = t_obs[t]; o < t_obs[t + 1]; ++o) ++seg[slot_of[P->h_obs_cam[o]] + 1];
    for (size_t i = 0; i < cams.size(); ++i) seg[i + 1] += seg[i];
    const bool small = t_obs[t + 1] - t_obs[t] <= TILE_OBS;   // else: a single point, no ranks
    std::vector<int32_t> cur(seg.begin(), seg.end() - 1);
    for (int64_t o = t_obs[t]; o < t_obs[t + 1]; ++o) {
      const int sl = slot_of[P->h_obs_cam[o]];
      const uint32_t rank = small ? (uint32_t)cur[sl]++ : 0u;
      slot[o] = (uint32_t)sl | ((uint32_t)(P->h_obs_pt[o] - t_pt[t]) << 16) | (rank << 24);
    }
    t_cseg.insert(t_cseg.end(), seg.begin(), seg.end() - 1);
    t_cams.insert(t_cams.end(), cams.begin(), cams.end());
    t_coff.push_back((int32_t)t_cams.size());
    max_tc = std::max(max_tc, (int)cams.size());
  }
  P->n_tiles = n_tiles;
  P->max_tile_cams = max_tc;
  // Groups of consecutive tiles for the Schur product: a group takes tiles
  // while it has fewer than G of them and the union of their cameras fits
  // GROUP_SLOTS; a tile of one point with more than TILE_OBS observations is a
  // group of its own. Grouping saves atomics but costs parallelism: G keeps at
  // least ~4096 workgroups (16 per compute unit) per product (measured on the
  // 2,000-camera city grid: 3 tiles per group beat 1, 2 and 4 to 8).
  const int G = std::max(1, std::min(GROUP_TILES, n_tiles / 4096));
  std::vector<int32_t> g_tile{0}, g_coff{0}, g_cams, t_cslot(t_cams.size());
  {
    std::vector<int32_t> gmark(n_cam, -1), gslot(n_cam, 0);
    int gid = 0, g_n = 0, g_u = 0;
    bool g_big = false;
    for (int t = 0; t < n_tiles; ++t) {
      const bool big = t_obs[t + 1] - t_obs[t] > TILE_OBS;
      int add = 0;
      for (int e = t_coff[t]; e < t_coff[t + 1]; ++e) add += gmark[t_cams[e]] != gid;
      if (g_n > 0 && (big || g_big || g_n >= G || g_u + add > GROUP_SLOTS)) {
        g_tile.push_back(t);
        g_coff.push_back((int32_t)g_cams.size());
        ++gid;
        g_n = g_u = 0;
      }
      for (int e = t_coff[t]; e < t_coff[t + 1]; ++e) {
        const int c = t_cams[e];
        if (gmark[c] != gid) {
          gmark[c] = gid;
          gslot[c] = g_u++;
          g_cams.push_back(c);
        }
        t_cslot[e] = gslot[c];
      }
      for (int64_t o = t_obs[t]; o < t_obs[t + 1]; ++o)
        slot[o] = (slot[o] & ~0xffffu) | (uint32_t)gslot[P->h_obs_cam[o]];
      ++g_n;
      g_big = big;
    }
    g_tile.push_back(n_tiles);
    g_coff.push_back((int32_t)g_cams.size());
    BA_CHECK(g_cams.size() < (size_t)INT32_MAX / 9, BA_ERR_LIMIT, "too many group camera entries");
  }
  P->n_groups = (int32_t)g_tile.size() - 1;
  P->max_pt_obs = max_k;
  // upload
  std::vector<int32_t> pt_off32(P->h_pt_off.begin(), P->h_pt_off.end());
  std::vector<int32_t> cam_off32(P->h_cam_off.begin(), P->h_cam_off.end());
  P->obs_cam.upload(P->h_obs_cam, s);
  P->obs_pt.upload(P->h_obs_pt, s);
  P->obs_orig.upload(P->h_obs_orig, s);
  P->obs_rank.upload(rank, s);
  P->pt_off.upload(pt_off32, s);
  P->pt_orig.upload(P->h_pt_orig, s);
  P->pt_new.upload(pt_new, s);
  P->cam_off.upload(cam_off32, s);
  P->cam_obs.upload(P->h_cam_obs, s);
  {
    std::vector<int32_t> cq(n_obs);
    for (int64_t i = 0; i < n_obs; ++i) cq[i] = P->h_obs_pt[P->h_cam_obs[i]];
    P->cam_q.upload(cq, s);
  }
  P->tile_obs.upload(t_obs, s);
  P->tile_pt.upload(t_pt, s);
  P->tile_coff.upload(t_coff, s);
  P->tile_cams.upload(t_cams, s);
  P->tile_cseg.upload(t_cseg, s);
  P->tile_cslot.upload(t_cslot, s);
  P->obs_slot.upload(slot, s);
  P->grp_tile.upload(g_tile, s);
  P->grp_coff.upload(g_coff, s);
  P->grp_cams.upload(g_cams, s);
  {
    // per camera, its entries of grp_cams in group order (deterministic product)
    std::vector<int32_t> tptr(n_cam + 1, 0), te(g_cams.size());
    for (int32_t c : g_cams) ++tptr[c + 1];
    for (int c = 0; c < n_cam; ++c) tptr[c + 1] += tptr[c];
    std::vector<int32_t> cur(tptr.begin(), tptr.end() - 1);
    for (size_t e = 0; e < g_cams.size(); ++e) te[cur[g_cams[e]]++] = (int32_t)e;
    P->n_te = (int32_t)g_cams.size();
    P->cam_te_ptr.upload(tptr, s);
    P->cam_te.upload(te, s);
  }
  BA_HIP(hipStreamSynchronize(s));
}

static uint32_t read_err(ba_plan* P, hipStream_t s) {
  uint32_t e = 0;
  BA_HIP(hipMemcpyAsync(&e, P->errflag.p, sizeof(e), hipMemcpyDeviceToHost, s));
  BA_HIP(hipStreamSynchronize(s));
  return e;
}

// Per-level CSR helpers computed on the host from the sorted pattern.
static void finish_level_pattern(Level& L, hipStream_t s) {
  const int n = L.n;
  std::vector<int32_t> diag(n), rowof(L.nnz), trans(L.nnz);
  for (int i = 0; i < n; ++i) {
    for (int64_t e = L.h_rowptr[i]; e < L.h_rowptr[i + 1]; ++e) {
      rowof[e] = i;
      if (L.h_col[e] == i) diag[i] = (int32_t)e;
    }
  }
  for (int i = 0; i < n; ++i) {
    for (int64_t e = L.h_rowptr[i]; e < L.h_rowptr[i + 1]; ++e) {
      const int j = L.h_col[e];
      auto b = L.h_col.begin() + L.h_rowptr[j], en = L.h_col.begin() + L.h_rowptr[j + 1];
      auto it = std::lower_bound(b, en, i);
      trans[e] = (int32_t)(it - L.h_col.begin());
    }
  }
  std::vector<int32_t> rp32(L.h_rowptr.begin(), L.h_rowptr.end());
  L.rowptr32.upload(rp32, s);
  L.diag_pos.upload(diag, s);
  L.row_of.upload(rowof, s);
  L.trans_pos.upload(trans, s);
}

// Covisibility of one level on the device (two passes: sizes, then entries),
// then the row sort and strength order.
template <class LaunchPass>
static void build_covisibility(ba_plan* P, Level& L, LaunchPass launch, hipStream_t s) {
  const int n = L.n;
  DBuf<int32_t> row_nnz;
  row_nnz.alloc(n);
  L.wdiag.alloc(n);
  launch(0, row_nnz.p, L.wdiag.p, (const int64_t*)nullptr, (int32_t*)nullptr, (int64_t*)nullptr);
  BA_LAUNCH_CHECK();
  std::vector<int32_t> h_nnz = row_nnz.download(s);
  uint32_t e = read_err(P, s);
  BA_CHECK(!(e & ERRF_LIMIT), BA_ERR_LIMIT, "a covisibility row exceeds %d entries", HASH_SLOTS * 3 / 4);
  L.h_wrowptr.assign(n + 1, 0);
  for (int i = 0; i < n; ++i) L.h_wrowptr[i + 1] = L.h_wrowptr[i] + h_nnz[i];
  L.wnnz = L.h_wrowptr[n];
  L.wrowptr.upload(L.h_wrowptr, s);
  L.wcol.alloc(L.wnnz);
  L.wval.alloc(L.wnnz);
  L.order.alloc(std::max<int64_t>(1, L.wnnz - n));
  launch(1, row_nnz.p, L.wdiag.p, L.wrowptr.p, L.wcol.p, L.wval.p);
  BA_LAUNCH_CHECK();
  hipLaunchKernelGGL(k_row_sort, dim3(n), dim3(256), 0, s, L.wrowptr.p, L.wcol.p, L.wval.p, L.wdiag.p,
                     L.order.p, P->errflag.p);
  BA_LAUNCH_CHECK();
  e = read_err(P, s);
  BA_CHECK(!(e & ERRF_LIMIT), BA_ERR_LIMIT, "a node is covisible with more than %d others", ROW_SORT_MAX - 1);
  L.h_wcol = L.wcol.download(s);
}

// The operator's block pattern is W's (level 0, and every level above an
// unsmoothed prolongator).
static void op_pattern_from_w(Level& L, hipStream_t s) {
  L.nnz = L.wnnz;
  L.h_rowptr = L.h_wrowptr;
  L.h_col = L.h_wcol;
  L.col.upload(L.h_col, s);
  finish_level_pattern(L, s);
}

// Plan-time gather lists of the smoothed prolongator P_s = (I - w D^-1 S) P_t
// of level F, of T = S P_s and of the Galerkin product P_s^T T that is C's
// operator; C's block pattern is that product's (wider than C's covisibility:
// the fill-in of smoothed aggregation). Every list is in a fixed order, so the
// products are deterministic.
static void build_sa_level(Level& F, Level& C, hipStream_t s) {
  const int n = F.n, na = F.n_agg;
  const std::vector<int32_t>& agg = F.h_agg;
  // P_s: row i holds the aggregates of i's operator neighbours, i included;
  // entry (i, a) sums S_ij P_t[j] over the neighbours j in aggregate a
  std::vector<int32_t> psp(n + 1, 0), pscol, psrow, psself, srcp, src;
  src.reserve(F.nnz);
  {
    std::vector<std::pair<int32_t, int32_t>> tmp;
    for (int i = 0; i < n; ++i) {
      tmp.clear();
      for (int64_t q = F.h_rowptr[i]; q < F.h_rowptr[i + 1]; ++q) tmp.emplace_back(agg[F.h_col[q]], (int32_t)q);
      std::sort(tmp.begin(), tmp.end());
      for (size_t k = 0; k < tmp.size(); ++k) {
        if (k == 0 || tmp[k].first != tmp[k - 1].first) {
          pscol.push_back(tmp[k].first);
          psrow.push_back(i);
          psself.push_back(tmp[k].first == agg[i]);
          srcp.push_back((int32_t)src.size());
        }
        src.push_back(tmp[k].second);
      }
      BA_CHECK(pscol.size() < (size_t)INT32_MAX, BA_ERR_LIMIT, "smoothed prolongator too large");
      psp[i + 1] = (int32_t)pscol.size();
    }
    srcp.push_back((int32_t)src.size());
  }
  const int64_t nps = (int64_t)pscol.size();
  // the entries of every aggregate's column, rows ascending
  std::vector<int32_t> pstp(na + 1, 0), pste(nps);
  for (int64_t e = 0; e < nps; ++e) ++pstp[pscol[e] + 1];
  for (int a = 0; a < na; ++a) pstp[a + 1] += pstp[a];
  {
    std::vector<int32_t> cur(pstp.begin(), pstp.end() - 1);
    for (int64_t e = 0; e < nps; ++e) pste[cur[pscol[e]]++] = (int32_t)e;
  }
  // T = S P_s: entry (i, b) sums S[q] P_s[e'] over operator entries q = (i, j)
  // and P_s entries e' = (j, b)
  std::vector<int64_t> tp(n + 1, 0);
  std::vector<int32_t> tcol, tsp, tso, tsps;
  {
    std::vector<std::array<int32_t, 3>> tmp;
    for (int i = 0; i < n; ++i) {
      tmp.clear();
      for (int64_t q = F.h_rowptr[i]; q < F.h_rowptr[i + 1]; ++q) {
        const int j = F.h_col[q];
        for (int32_t e = psp[j]; e < psp[j + 1]; ++e) tmp.push_back({pscol[e], (int32_t)q, e});
      }
      std::sort(tmp.begin(), tmp.end());
      BA_CHECK(tso.size() + tmp.size() < (size_t)INT32_MAX, BA_ERR_LIMIT, "smoothed Galerkin product too large");
      for (size_t k = 0; k < tmp.size(); ++k) {
        if (k == 0 || tmp[k][0] != tmp[k - 1][0]) {
          tcol.push_back(tmp[k][0]);
          tsp.push_back((int32_t)tso.size());
        }
        tso.push_back(tmp[k][1]);
        tsps.push_back(tmp[k][2]);
      }
      tp[i + 1] = (int64_t)tcol.size();
    }
    tsp.push_back((int32_t)tso.size());
  }
  const int64_t nt = (int64_t)tcol.size();
  BA_CHECK(nt < (int64_t)INT32_MAX && (int64_t)tsp.size() == nt + 1, BA_ERR_LIMIT, "S P_s too large");
  // C = P_s^T T: entry (a, b) sums P_s[e]^T T[t] over rows i with e = (i, a)
  // and t = (i, b)
  C.h_rowptr.assign(na + 1, 0);
  C.h_col.clear();
  std::vector<int32_t> cgp, cgps, cgt;
  {
    std::vector<std::array<int32_t, 3>> tmp;
    for (int a = 0; a < na; ++a) {
      tmp.clear();
      for (int32_t k = pstp[a]; k < pstp[a + 1]; ++k) {
        const int32_t e = pste[k];
        const int i = psrow[e];
        for (int64_t t = tp[i]; t < tp[i + 1]; ++t) tmp.push_back({tcol[t], e, (int32_t)t});
      }
      std::sort(tmp.begin(), tmp.end());
      BA_CHECK(cgps.size() + tmp.size() < (size_t)INT32_MAX, BA_ERR_LIMIT, "smoothed Galerkin product too large");
      for (size_t k = 0; k < tmp.size(); ++k) {
        if (k == 0 || tmp[k][0] != tmp[k - 1][0]) {
          C.h_col.push_back(tmp[k][0]);
          cgp.push_back((int32_t)cgps.size());
        }
        cgps.push_back(tmp[k][1]);
        cgt.push_back(tmp[k][2]);
      }
      C.h_rowptr[a + 1] = (int64_t)C.h_col.size();
    }
    cgp.push_back((int32_t)cgps.size());
  }
  C.nnz = (int64_t)C.h_col.size();
  BA_CHECK((int64_t)cgp.size() == C.nnz + 1, BA_ERR_STRUCTURE, "internal: smoothed Galerkin lists");
  C.col.upload(C.h_col, s);
  finish_level_pattern(C, s);
  F.nnz_ps = nps;
  F.nnz_t = nt;
  F.ps_ptr.upload(psp, s);
  F.ps_col.upload(pscol, s);
  F.ps_row.upload(psrow, s);
  F.ps_self.upload(psself, s);
  F.ps_src_ptr.upload(srcp, s);
  F.ps_src.upload(src, s);
  F.pst_ptr.upload(pstp, s);
  F.pst_e.upload(pste, s);
  F.t_src_ptr.upload(tsp, s);
  F.t_src_op.upload(tso, s);
  F.t_src_ps.upload(tsps, s);
  F.cg_ptr.upload(cgp, s);
  F.cg_ps.upload(cgps, s);
  F.cg_t.upload(cgt, s);
  // the host vectors go out of scope here: the uploads must have completed
  BA_HIP(hipStreamSynchronize(s));
}

// Shared points of every upper off-diagonal block of the level-0 pattern: for
// each point (in order) and each pair a < b of its camera-sorted observations,
// the point goes to block (camera(a), camera(b)).
static void build_s0_pairs(ba_plan* P, const Level& L0, hipStream_t s) {
  const int n_pt = P->n_pt;
  std::vector<int32_t> cnt(L0.nnz + 1, 0);
  auto entry = [&](int ci, int cj) {
    auto b = L0.h_col.begin() + L0.h_rowptr[ci], e = L0.h_col.begin() + L0.h_rowptr[ci + 1];
    return (int32_t)(std::lower_bound(b, e, cj) - L0.h_col.begin());
  };
  int64_t total = 0;
  for (int q = 0; q < n_pt; ++q)
    for (int64_t a = P->h_pt_off[q]; a < P->h_pt_off[q + 1]; ++a)
      for (int64_t b = a + 1; b < P->h_pt_off[q + 1]; ++b) {
        ++cnt[entry(P->h_obs_cam[a], P->h_obs_cam[b]) + 1];
        ++total;
      }
  BA_CHECK(total < INT32_MAX, BA_ERR_LIMIT, "too many covisible observation pairs");
  for (int64_t e = 0; e < L0.nnz; ++e) cnt[e + 1] += cnt[e];
  std::vector<int32_t> pts(std::max<int64_t>(1, total));
  std::vector<int32_t> cur(cnt.begin(), cnt.end() - 1);
  for (int q = 0; q < n_pt; ++q)
    for (int64_t a = P->h_pt_off[q]; a < P->h_pt_off[q + 1]; ++a)
      for (int64_t b = a + 1; b < P->h_pt_off[q + 1]; ++b)
        pts[cur[entry(P->h_obs_cam[a], P->h_obs_cam[b])]++] = q;
  std::vector<int32_t> ce, cb;
  for (int64_t e = 0; e < L0.nnz; ++e)
    for (int32_t h = cnt[e]; h < cnt[e + 1]; h += S0_CHUNK) {
      ce.push_back((int32_t)e);
      cb.push_back(h);
    }
  std::vector<int32_t> be, bch;
  for (size_t c = 0; c < ce.size(); ++c)
    if (c == 0 || ce[c] != ce[c - 1]) {
      be.push_back(ce[c]);
      bch.push_back((int32_t)c);
    }
  bch.push_back((int32_t)ce.size());
  P->s0_blocks = (int32_t)be.size();
  P->s0_blk_e.upload(be, s);
  P->s0_blk_ch.upload(bch, s);
  P->s0_chunks = (int32_t)ce.size();
  P->s0_ptr.upload(cnt, s);
  P->s0_q.upload(pts, s);
  P->s0_chunk_e.upload(ce, s);
  P->s0_chunk_beg.upload(cb, s);
}

static void aggregate_level(ba_plan* P, Level& L, int cap, hipStream_t s) {
  const int n = L.n;
  DBuf<int32_t> agg, nagg;
  agg.alloc(n);
  nagg.alloc(1);
  const size_t lds = (size_t)n * 2 * sizeof(int);
  if (lds <= 150 * 1024) {
    hipLaunchKernelGGL(k_aggregate_lds, dim3(1), dim3(64), lds, s, n, L.wrowptr.p, L.order.p, cap,
                       agg.p, nagg.p);
  } else {
    DBuf<int32_t> size;
    size.alloc(n);
    hipLaunchKernelGGL(k_aggregate_global, dim3(1), dim3(64), 0, s, n, L.wrowptr.p, L.order.p, cap,
                       agg.p, size.p, nagg.p);
    BA_HIP(hipStreamSynchronize(s));
  }
  BA_LAUNCH_CHECK();
  std::vector<int32_t> hn = nagg.download(s);
  L.h_agg = agg.download(s);
  L.n_agg = hn[0];
  L.agg = std::move(agg);
}

static void build_hierarchy(ba_plan* P, const ba_opts* o, hipStream_t s) {
  P->levels.clear();
  P->levels.reserve(std::max(1, o->max_levels));
  P->levels.emplace_back();
  {
    Level& L0 = P->levels[0];
    L0.n = P->n_cam;
    L0.bs = 9;
    build_covisibility(P, L0, [&](int pass, int32_t* nnz, int64_t* wd, const int64_t* rp, int32_t* col, int64_t* val) {
      if (pass == 0)
        hipLaunchKernelGGL(k_covis0<0>, dim3(L0.n), dim3(256), 0, s, P->cam_off.p, P->cam_obs.p, P->obs_pt.p,
                           P->pt_off.p, P->obs_cam.p, nnz, wd, rp, col, val, P->errflag.p);
      else
        hipLaunchKernelGGL(k_covis0<1>, dim3(L0.n), dim3(256), 0, s, P->cam_off.p, P->cam_obs.p, P->obs_pt.p,
                           P->pt_off.p, P->obs_cam.p, nnz, wd, rp, col, val, P->errflag.p);
    }, s);
    op_pattern_from_w(L0, s);
    build_s0_pairs(P, L0, s);
  }
  for (;;) {
    const int l = (int)P->levels.size() - 1;
    Level& L = P->levels[l];
    if (L.n <= o->coarse_max_nodes || (int)P->levels.size() >= o->max_levels) break;
    aggregate_level(P, L, o->agg_cap, s);
    if (L.n_agg > o->min_coarsen_ratio * L.n) {
      L.n_agg = 0;
      L.agg.free();
      L.h_agg.clear();
      break;
    }
    // members of every aggregate, ascending
    std::vector<int32_t> aptr(L.n_agg + 1, 0), amem(L.n), apos(L.n);
    for (int i = 0; i < L.n; ++i) ++aptr[L.h_agg[i] + 1];
    for (int a = 0; a < L.n_agg; ++a) aptr[a + 1] += aptr[a];
    {
      std::vector<int32_t> cur(aptr.begin(), aptr.end() - 1);
      for (int i = 0; i < L.n; ++i) { apos[i] = cur[L.h_agg[i]] - aptr[L.h_agg[i]]; amem[cur[L.h_agg[i]]++] = i; }
    }
    L.max_agg = 0;
    L.min_agg = L.n;
    for (int a = 0; a < L.n_agg; ++a) {
      L.max_agg = std::max(L.max_agg, aptr[a + 1] - aptr[a]);
      L.min_agg = std::min(L.min_agg, aptr[a + 1] - aptr[a]);
    }
    L.mean_agg = (double)L.n / L.n_agg;
    L.agg_ptr.upload(aptr, s);
    L.agg_mem.upload(amem, s);
    L.agg_pos.upload(apos, s);
    std::vector<int32_t> slot(L.n);
    for (int i = 0; i < L.n; ++i) slot[i] = aptr[L.h_agg[i]] + apos[i];
    L.slot_of.upload(slot, s);
    P->levels.emplace_back();
    Level& F = P->levels[l];
    Level& C = P->levels[l + 1];
    C.n = F.n_agg;
    C.bs = NS;
    build_covisibility(P, C, [&](int pass, int32_t* nnz, int64_t* wd, const int64_t* rp, int32_t* col, int64_t* val) {
      if (pass == 0)
        hipLaunchKernelGGL(k_covisL<0>, dim3(C.n), dim3(256), 0, s, F.agg_ptr.p, F.agg_mem.p, F.wrowptr.p, F.wcol.p,
                           F.wval.p, F.agg.p, nnz, wd, rp, col, val, P->errflag.p);
      else
        hipLaunchKernelGGL(k_covisL<1>, dim3(C.n), dim3(256), 0, s, F.agg_ptr.p, F.agg_mem.p, F.wrowptr.p, F.wcol.p,
                           F.wval.p, F.agg.p, nnz, wd, rp, col, val, P->errflag.p);
    }, s);
    if (P->sa) {
      build_sa_level(F, C, s);
      continue;
    }
    op_pattern_from_w(C, s);
    // Galerkin gather lists: coarse entry (A, B) <- fine entries (i, j), agg(i)=A, agg(j)=B
    std::vector<int32_t> cidx(F.nnz);
    std::vector<int32_t> gptr(C.nnz + 1, 0);
    for (int i = 0; i < F.n; ++i) {
      const int A = F.h_agg[i];
      for (int64_t e = F.h_rowptr[i]; e < F.h_rowptr[i + 1]; ++e) {
        const int B = F.h_agg[F.h_col[e]];
        auto b = C.h_col.begin() + C.h_rowptr[A], en = C.h_col.begin() + C.h_rowptr[A + 1];
        auto it = std::lower_bound(b, en, B);
        BA_CHECK(it != en && *it == B, BA_ERR_STRUCTURE, "internal: coarse pattern misses an entry");
        cidx[e] = (int32_t)(it - C.h_col.begin());
        ++gptr[cidx[e] + 1];
      }
    }
    for (int64_t e = 0; e < C.nnz; ++e) gptr[e + 1] += gptr[e];
    std::vector<int32_t> gfine(F.nnz);
    {
      std::vector<int32_t> cur(gptr.begin(), gptr.end() - 1);
      for (int64_t e = 0; e < F.nnz; ++e) gfine[cur[cidx[e]]++] = (int32_t)e;
    }
    F.gal_ptr.upload(gptr, s);
    F.gal_fine.upload(gfine, s);
  }
  BA_HIP(hipStreamSynchronize(s));
}

}  // namespace bamg
