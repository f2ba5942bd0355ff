// The plan: integer structure of one visibility graph (observation layout,
// tiles, multigrid hierarchy pattern) plus the per-step numeric buffers.
#pragma once

#include "common.hpp"

namespace bamg {

// One multigrid level. Nodes are cameras on level 0 and aggregates above.
struct Level {
  int n = 0;    // nodes
  int bs = 9;   // dofs per node: 9 on level 0, 16 above
  // covisibility W of this level (the aggregation graph): CSR with sorted
  // columns, diagonal included
  int64_t wnnz = 0;
  std::vector<int64_t> h_wrowptr;
  std::vector<int32_t> h_wcol;
  DBuf<int64_t> wrowptr;
  DBuf<int32_t> wcol;
  DBuf<int64_t> wval;
  DBuf<int64_t> wdiag;       // W_ii
  DBuf<int32_t> order;       // neighbours by decreasing strength: row i at [wrowptr[i]-i, wrowptr[i+1]-i-1)
  // block pattern of this level's operator: W's pattern, except above a
  // smoothed prolongator, whose Galerkin product fills in (then wider)
  int64_t nnz = 0;
  std::vector<int64_t> h_rowptr;
  std::vector<int32_t> h_col;
  DBuf<int32_t> rowptr32;
  DBuf<int32_t> col;
  DBuf<int32_t> diag_pos;    // CSR position of (i, i)
  DBuf<int32_t> trans_pos;   // CSR position of (j, i) for entry (i, j)
  DBuf<int32_t> row_of;      // row index of every CSR entry
  // aggregation of this level into the next (absent on the coarsest level)
  int n_agg = 0;
  std::vector<int32_t> h_agg;
  DBuf<int32_t> agg;         // aggregate id per node (creation order)
  DBuf<int32_t> agg_ptr;     // members of aggregate a: agg_mem[agg_ptr[a] .. agg_ptr[a+1])
  DBuf<int32_t> agg_mem;     // ascending node ids
  DBuf<int32_t> agg_pos;     // position of node i inside its aggregate
  DBuf<int32_t> slot_of;     // node i's position in aggregate order: agg_ptr[agg[i]] + agg_pos[i]
  int max_agg = 0;           // largest aggregate
  int min_agg = 0;           // smallest aggregate
  double mean_agg = 0.0;     // nodes per aggregate
  // Galerkin map: coarse CSR entry e gathers fine entries gal_fine[gal_ptr[e] .. gal_ptr[e+1])
  DBuf<int32_t> gal_ptr;
  DBuf<int32_t> gal_fine;
  // smoothed prolongator P_s = (I - w D^-1 S) P_t to the next level (plans
  // built for it), CSR by node (row pointer ps_ptr): entry e = (node
  // ps_row[e], aggregate ps_col[e]); its terms S_ij P_t[j] come from the
  // operator entries ps_src[ps_src_ptr[e] ..), and ps_self[e] marks the
  // aggregate of the node itself (P_t's own block).
  int64_t nnz_ps = 0, nnz_t = 0;
  DBuf<int32_t> ps_ptr, ps_col, ps_row, ps_self, ps_src_ptr, ps_src;
  DBuf<int32_t> pst_ptr, pst_e;   // P_s entries by aggregate (rows ascending)
  // T = S P_s (node x aggregate blocks): entry t sums S[t_src_op] P_s[t_src_ps] over t_src_ptr[t] ..
  DBuf<int32_t> t_src_ptr, t_src_op, t_src_ps;
  // the next level's operator P_s^T T: its entry c sums P_s[cg_ps]^T T[cg_t]
  // over cg_ptr[c] ..
  DBuf<int32_t> cg_ptr, cg_ps, cg_t;
  // ---- numeric, per step
  DBuf<double> S;            // nnz * bs * bs  explicit operator (level 0: explicit Schur S)
  DBuf<float> S32;
  DBuf<double> K;            // n * bs * NS near-nullspace rows
  DBuf<double> P;            // n * bs * NS tentative prolongator blocks (to level + 1)
  DBuf<double> Ps;           // nnz_ps * bs * NS smoothed prolongator blocks
  DBuf<double> Tsp;          // nnz_t * bs * NS blocks of S P_s
  DBuf<float> P32;
  DBuf<double> Dinv;         // n * bs * bs inverse diagonal blocks
  DBuf<float> Dinv32;
  double lmax = 0.0;         // host copy of lambda_max of D^-1 S (smoothed-prolongator setup only)
  bool explicit_op = true;   // level 0: use explicit S for smoothing (else implicit)
  // coarsest level: dense inverse of the operator (FP64), padded to nd x nd
  int nd = 0;
  DBuf<double> dense;        // factor workspace nd x nd
  DBuf<double> inv;          // inverse nd x nd
  // V-cycle work vectors, FP64 and FP32 (n * bs each)
  DBuf<double> lz_u, lz_v, lz_up, lz_vp, lz_av, lz_dav, lz_w, lz_dw;   // Lanczos vectors
  DBuf<double> lz_s;         // Lanczos scalars: alpha[32], beta[32], norm, b2, count, stop, lambda_max, 1/lambda_max
  DBuf<double> gj_scale;     // coarsest level: equilibration scales
  DBuf<double> gj_piv;       // coarsest level: inverses of the current and next pivot blocks (2 x GJB x GJB)
  DBuf<double> vb, vx, vr, vd, vt, vpart;
  DBuf<float> fb, fx, fr, fd, ft, fpart;   // vpart/fpart: restriction partials (n * NS)
  DBuf<double> vd2, vx2;     // second Chebyshev direction and iterate (fused block-row products)
  DBuf<float> fd2, fx2;
};

struct Scratch;   // defined in api.cpp
struct Backward;  // defined in backward.cpp
struct LmWork;    // defined in lm.cpp

}  // namespace bamg

struct ba_plan {
  bamg::Allocator alloc;          // where the persistent arrays come from (declared first: freed last)
  int32_t n_cam = 0, n_pt = 0;
  int64_t n_obs = 0;
  int64_t n_obs_pad = 0;     // plane stride of the observation SoA arrays
  // ---- point-major observation layout
  std::vector<int32_t> h_obs_cam, h_obs_pt, h_obs_orig, h_pt_orig;
  std::vector<int64_t> h_pt_off, h_cam_off;
  std::vector<int32_t> h_cam_obs;
  bamg::DBuf<int32_t> obs_cam;    // [n_obs] camera of each observation (point-major)
  bamg::DBuf<int32_t> obs_pt;     // [n_obs] reordered point index
  bamg::DBuf<int32_t> obs_orig;   // [n_obs] caller's observation index
  bamg::DBuf<int32_t> pt_off;     // [n_pt + 1] observation range of each reordered point
  bamg::DBuf<int32_t> pt_orig;    // [n_pt] caller's point index of each reordered point
  bamg::DBuf<int32_t> pt_new;     // [n_pt] reordered index of each caller point
  bamg::DBuf<int32_t> cam_off;    // [n_cam + 1]
  bamg::DBuf<int32_t> cam_obs;    // [n_obs] point-major observation indices, camera-major
  bamg::DBuf<int32_t> cam_q;      // [n_obs] reordered point of each camera-major entry
  bamg::DBuf<int32_t> obs_rank;   // [n_obs] point-major index of caller observation i
  // ---- tiles for the implicit Schur product
  int32_t n_tiles = 0;
  bamg::DBuf<int32_t> tile_obs;   // [n_tiles + 1]
  bamg::DBuf<int32_t> tile_pt;    // [n_tiles + 1]
  bamg::DBuf<int32_t> tile_coff;  // [n_tiles + 1] offsets into tile_cams
  bamg::DBuf<int32_t> tile_cams;  // distinct cameras of each tile, ascending
  bamg::DBuf<int32_t> tile_cseg;  // per tile_cams entry: first rank of that camera's observations
  bamg::DBuf<uint32_t> obs_slot;  // [n_obs] group camera slot | point slot << 16 | rank by camera << 24
  bamg::DBuf<int32_t> tile_cslot; // per tile_cams entry: its camera's slot in the tile's group
  int32_t max_tile_cams = 0;
  // ---- groups of consecutive tiles (one workgroup each in the Schur product)
  int32_t n_groups = 0;
  bamg::DBuf<int32_t> grp_tile;   // [n_groups + 1] tile range of each group
  bamg::DBuf<int32_t> grp_coff;   // [n_groups + 1] offsets into grp_cams
  bamg::DBuf<int32_t> grp_cams;   // cameras of each group, in slot order
  // ---- explicit level-0 S: for every upper off-diagonal block (i, j) of the
  // level-0 pattern, the (reordered) points cameras i and j share
  bamg::DBuf<int32_t> s0_ptr;     // [nnz0 + 1]
  bamg::DBuf<int32_t> s0_q;
  bamg::DBuf<int32_t> s0_chunk_e;    // chunks of <= S0_CHUNK points: block
  bamg::DBuf<int32_t> s0_chunk_beg;  //   and first index into s0_q
  int32_t s0_chunks = 0;
  bamg::DBuf<int32_t> s0_blk_e;      // deterministic mode: every upper block with
  bamg::DBuf<int32_t> s0_blk_ch;     //   shared points, and its chunk range [i, i + 1)
  int32_t s0_blocks = 0;
  bamg::DBuf<double> s0_part;        // deterministic mode: [s0_chunks][81] chunk sums
  // deterministic Schur product: per camera, its (group, camera) entries of
  // grp_cams in group order, and the partial sums of one product
  bamg::DBuf<int32_t> cam_te_ptr;    // [n_cam + 1]
  bamg::DBuf<int32_t> cam_te;        // [total grp_cams entries]
  int32_t n_te = 0;
  bamg::DBuf<double> te_part;        // [n_te][9]
  bamg::DBuf<float> te_part32;
  int32_t max_pt_obs = 0;
  // ---- multigrid hierarchy
  std::vector<bamg::Level> levels;
  // ---- per-step numeric state (FP64 unless suffixed 32)
  bamg::DBuf<double> campre;      // [n_cam][24]: R, J_r, t, f, k1, k2
  bamg::DBuf<double> F, E, fres;  // SoA planes: 18, 6, 2 x n_obs_pad
  bamg::DBuf<float> F32, E32;
  bamg::DBuf<double> Cinv;        // [n_pt][6] packed symmetric C^-1 (reordered points)
  bamg::DBuf<float> Cinv32;
  bamg::DBuf<double> vgp;         // [n_pt][3] C^-1 g_p
  bamg::DBuf<double> prec;        // [n_pt][PREC] point records: X | C^-1 (packed) | C^-1 g_p
  bamg::DBuf<double> gp;          // [n_pt][3] g_p
  bamg::DBuf<double> Dp;          // [n_pt][3] damping of the point block
  bamg::DBuf<double> A;           // [n_cam][45] packed damped A
  bamg::DBuf<float> A32;
  bamg::DBuf<double> Dc;          // [n_cam][9] damping of the camera block
  bamg::DBuf<double> b;           // [n_cam][9]
  bamg::DBuf<double> Scc;         // [n_cam][81] block-Jacobi blocks (before inversion)
  bamg::DBuf<double> Sinv;        // [n_cam][81] inverses
  bamg::DBuf<double> wsq;         // [n_obs_pad] sqrt(rho') per observation (robust loss only)
  bool robust = false;            // the prepared step uses a robust loss
  bamg::DBuf<int64_t> cj_off;     // [n_agg0 + 1] offsets of the cluster blocks in cj_inv
  bamg::DBuf<double> cj_inv;      // cluster blocks of S, inverted (visibility-based block Jacobi)
  int cj_max_n = 0;               // largest cluster block dimension (9 x members)
  int64_t cj_total = 0;           // doubles of all cluster blocks
  bool prepared_cj = false;
  bamg::DBuf<float> Sinv32;
  bamg::DBuf<uint32_t> errflag;   // device error bits
  bool prepared = false;
  bool prepared_mg = false;
  bool inspectable_mg = false;   // hierarchy data readable (also after a failed setup)
  bool have_mixed = false;
  bool det = false;               // the prepared step runs without floating-point atomics
  bool sa = false;                // hierarchy built for the smoothed prolongator (Section 3.5)
  double lambda = 1e-4;
  // ---- workspace binding: the per-step buffers above are views into it
  bamg::DBuf<char> own_ws;        // the plan's own workspace (callers passing ws == NULL)
  uint32_t own_key = 0;           // what own_ws is laid out for
  const void* ws_base = nullptr;  // workspace the views point into
  uint32_t ws_key = 0;            // its layout
  size_t ws_span = 0;             // bytes that layout spans
  hipEvent_t ev_t[3] = {nullptr, nullptr, nullptr};   // step phases: start, blocks done, setup done
  uint32_t* h_err = nullptr;      // pinned copy of the error flags
  hipStream_t cap = nullptr;      // stream the PCG iteration graph is captured on (runs nothing)
  bamg::Scratch* scratch = nullptr;
  // side streams of the multigrid setup (default priority), forked from and
  // joined back into the caller's stream with these events: side runs the QR
  // chain, and the Lanczos estimate of level l runs on the (l mod 3)-th of
  // side2, side and side3, each stream signalling its ev_lz[] when done
  hipStream_t side = nullptr, side2 = nullptr, side3 = nullptr;
  hipEvent_t ev_fork = nullptr;
  hipEvent_t ev_lz[3] = {nullptr, nullptr, nullptr};
  std::vector<hipEvent_t> ev_qr, ev_lvl;   // per level: QR done; operator and block inverses ready
  bamg::Backward* bwd = nullptr;
  bamg::LmWork* lm = nullptr;
};
