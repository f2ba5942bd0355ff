// Multigrid numeric setup (Sections 3.1, 3.3, 3.4, 3.6 of Konolige and Brown):
// camera near-nullspace, per-aggregate QR tentative prolongation, the explicit
// level-0 Schur complement, Galerkin coarse operators P^T S P, smoother block
// inverses, and the dense coarse factorization (the FP64 MFMA site).
#include "kernels.hpp"

namespace bamg {

// ---------------------------------------------------------------- near-nullspace

// K rows of camera c (9 x 16, row-major): columns 0..8 constant in each camera
// parameter; 9..11 world translations tau_k (dt = -R e_k); 12..14 world
// rotations (dw = -J_r(w)^-1 e_k); 15 world scale (dt = t). Section 3.1.
__global__ void k_nullspace0(int n_cam, const double* __restrict__ cams, const double* __restrict__ campre,
                             double* __restrict__ K) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= n_cam) return;
  const double w[3] = {cams[c * 9], cams[c * 9 + 1], cams[c * 9 + 2]};
  double Ji[9];
  right_jacobian_inv(w, Ji);
  const double* R = campre + (size_t)c * 24;
  double* k = K + (size_t)c * 9 * NS;
  for (int i = 0; i < 9 * NS; ++i) k[i] = 0.0;
  for (int i = 0; i < 9; ++i) k[i * NS + i] = 1.0;
  for (int j = 0; j < 3; ++j) {
    for (int i = 0; i < 3; ++i) {
      k[(3 + i) * NS + 9 + j] = -R[i * 3 + j];
      k[i * NS + 12 + j] = -Ji[i * 3 + j];
    }
  }
  for (int i = 0; i < 3; ++i) k[(3 + i) * NS + 15] = cams[c * 9 + 3 + i];
}

// ---------------------------------------------------------------- QR per aggregate

// Householder QR (LAPACK conventions: beta = -sign(alpha) |x|, v_0 = 1) of the
// stacked near-nullspace rows of one aggregate's members (ascending), thin Q,
// then signs flipped so that diag(R) >= 0. One wave per aggregate; the
// aggregate's matrix lives in dynamic LDS.
__global__ __launch_bounds__(64) void k_qr_aggregates(int bs, const int32_t* __restrict__ agg_ptr,
                                                      const int32_t* __restrict__ agg_mem,
                                                      const double* __restrict__ Kf,
                                                      double* __restrict__ P, double* __restrict__ Kc) {
  extern __shared__ double sm[];
  const int a = blockIdx.x;
  const int lane = threadIdx.x;
  const int m0 = agg_ptr[a], nm = agg_ptr[a + 1] - m0;
  const int rows = nm * bs;
  double* A = sm;                    // rows x NS, row-major
  double* Q = sm + rows * NS;        // rows x NS
  __shared__ double tau[NS];
  for (int idx = lane; idx < rows * NS; idx += 64) {
    const int r = idx / NS, c = idx % NS;
    const int mem = agg_mem[m0 + r / bs];
    A[idx] = Kf[((size_t)mem * bs + (r % bs)) * NS + c];
  }
  __syncthreads();
  const int ncol = rows < NS ? rows : NS;
  for (int j = 0; j < ncol; ++j) {
    double s = 0.0;
    for (int r = j + 1 + lane; r < rows; r += 64) s += A[r * NS + j] * A[r * NS + j];
    s = wave_sum(s);
    const double alpha = A[j * NS + j];
    double t = 0.0, beta = alpha, scal = 0.0;
    if (s > 0.0) {
      const double nrm = sqrt(alpha * alpha + s);
      beta = alpha >= 0.0 ? -nrm : nrm;
      t = (beta - alpha) / beta;
      scal = 1.0 / (alpha - beta);
    }
    __syncthreads();
    if (s > 0.0)
      for (int r = j + 1 + lane; r < rows; r += 64) A[r * NS + j] *= scal;
    if (lane == 0) { A[j * NS + j] = beta; tau[j] = t; }
    __syncthreads();
    // apply H_j = I - t v v^T (v = [1; A[j+1:, j]]) to columns j+1..NS-1
    for (int c = j + 1; c < NS; ++c) {
      double w = 0.0;
      for (int r = j + lane; r < rows; r += 64) w += (r == j ? 1.0 : A[r * NS + j]) * A[r * NS + c];
      w = wave_sum(w) * t;
      __syncthreads();
      for (int r = j + lane; r < rows; r += 64) A[r * NS + c] -= w * (r == j ? 1.0 : A[r * NS + j]);
      __syncthreads();
    }
  }
  // Q = H_0 ... H_{ncol-1} [I; 0]
  for (int idx = lane; idx < rows * NS; idx += 64) {
    const int r = idx / NS, c = idx % NS;
    Q[idx] = (r == c) ? 1.0 : 0.0;
  }
  __syncthreads();
  for (int j = ncol - 1; j >= 0; --j) {
    const double t = tau[j];
    for (int c = j; c < NS; ++c) {
      double w = 0.0;
      for (int r = j + lane; r < rows; r += 64) w += (r == j ? 1.0 : A[r * NS + j]) * Q[r * NS + c];
      w = wave_sum(w) * t;
      __syncthreads();
      for (int r = j + lane; r < rows; r += 64) Q[r * NS + c] -= w * (r == j ? 1.0 : A[r * NS + j]);
      __syncthreads();
    }
  }
  // sign convention diag(R) >= 0; R = upper triangle of A's first NS rows
  __shared__ double sgn[NS];
  if (lane < NS) sgn[lane] = (lane < ncol && A[lane * NS + lane] < 0.0) ? -1.0 : 1.0;
  __syncthreads();
  for (int idx = lane; idx < rows * NS; idx += 64) {
    const int r = idx / NS, c = idx % NS;
    const int mem = agg_mem[m0 + r / bs];
    P[((size_t)mem * bs + (r % bs)) * NS + c] = Q[idx] * sgn[c];
  }
  for (int idx = lane; idx < NS * NS; idx += 64) {
    const int r = idx / NS, c = idx % NS;
    Kc[(size_t)a * NS * NS + idx] = (r < ncol && c >= r) ? sgn[r] * A[r * NS + c] : 0.0;
  }
}

// ---------------------------------------------------------------- explicit level-0 S

// Off-diagonal block (i, j), i < j, of S = A - W C^-1 W^T:
//   S_ij = - sum_{p seen by i and j} F_ip^T (E_ip C_p^-1 E_jp^T) F_jp,
// one wave per upper entry, one lane per shared point (the plan lists the
// points of every block). Each lane recomputes both cameras' Jacobian blocks
// from the camera data and the point record [X | C_p^-1], accumulates the 81
// entries, and the wave sums them with a reduce-scatter. Diagonal blocks are
// the block-Jacobi blocks S_cc; both (i, j) and (j, i) are written.
__global__ __launch_bounds__(64) void k_explicit_s0(
    const int32_t* __restrict__ row_of, const int32_t* __restrict__ col,
    const int32_t* __restrict__ trans_pos, const int32_t* __restrict__ s0_ptr,
    const int32_t* __restrict__ s0_q, const double* __restrict__ campre, const double* __restrict__ prec,
    const double* __restrict__ Scc, double* __restrict__ S) {
  const int e = blockIdx.x;
  const int i = row_of[e], j = col[e];
  const int lane = threadIdx.x;
  if (i == j) {
    for (int k = lane; k < 81; k += 64) S[(size_t)e * 81 + k] = Scc[(size_t)i * 81 + k];
    return;
  }
  if (i > j) return;
  const double* ci = campre + (size_t)i * 24;
  const double* cj = campre + (size_t)j * 24;
  double acc[96];
#pragma unroll
  for (int k = 0; k < 96; ++k) acc[k] = 0.0;
  const int end = s0_ptr[e + 1];
  for (int h = s0_ptr[e] + lane; h < end; h += 64) {
    const double* rec = prec + (size_t)s0_q[h] * PREC;
    const double X[3] = {rec[0], rec[1], rec[2]};
    const double C[9] = {rec[3], rec[4], rec[5], rec[4], rec[6], rec[7], rec[5], rec[7], rec[8]};
    double pi[2], fi[18], ei[6], fj[18], ej[6], z;
    project_jacobian(ci, X, pi, fi, ei, &z);
    project_jacobian(cj, X, pi, fj, ej, &z);
    double ec[6];
#pragma unroll
    for (int r = 0; r < 2; ++r)
#pragma unroll
      for (int k = 0; k < 3; ++k)
        ec[r * 3 + k] = ei[r * 3 + 0] * C[0 * 3 + k] + ei[r * 3 + 1] * C[1 * 3 + k] + ei[r * 3 + 2] * C[2 * 3 + k];
    double m[4];
#pragma unroll
    for (int r = 0; r < 2; ++r)
#pragma unroll
      for (int t = 0; t < 2; ++t) m[r * 2 + t] = ec[r * 3 + 0] * ej[t * 3 + 0] + ec[r * 3 + 1] * ej[t * 3 + 1] + ec[r * 3 + 2] * ej[t * 3 + 2];
    double mf[18];
#pragma unroll
    for (int k = 0; k < 9; ++k) {
      mf[k] = m[0] * fj[k] + m[1] * fj[9 + k];
      mf[9 + k] = m[2] * fj[k] + m[3] * fj[9 + k];
    }
#pragma unroll
    for (int r = 0; r < 9; ++r)
#pragma unroll
      for (int c = 0; c < 9; ++c) acc[r * 9 + c] += fi[r] * mf[c] + fi[9 + r] * mf[9 + c];
  }
  wave_reduce_scatter<96>(acc);
  if (!(lane & 1)) {
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      const int idx = 3 * (lane >> 1) + k;
      if (idx < 81) {
        const int r = idx / 9, c = idx % 9;
        S[(size_t)e * 81 + idx] = -acc[k];
        S[(size_t)trans_pos[e] * 81 + c * 9 + r] = -acc[k];
      }
    }
  }
}

// ---------------------------------------------------------------- Galerkin product

// Coarse entry (A, B) = sum over fine entries (i, j) with agg(i) = A, agg(j) = B
// of P_i^T S_ij P_j (fine blocks bs x bs, P blocks bs x 16). One workgroup of
// 256 threads per coarse entry; thread (r, c) owns entry (r, c).
__global__ __launch_bounds__(256) void k_galerkin(int bs, const int32_t* __restrict__ gal_ptr,
                                                  const int32_t* __restrict__ gal_fine,
                                                  const int32_t* __restrict__ row_of,
                                                  const int32_t* __restrict__ col,
                                                  const double* __restrict__ Sf,
                                                  const double* __restrict__ P,
                                                  double* __restrict__ Sc) {
  __shared__ double Ss[NS * NS], Pi[NS * NS], Pj[NS * NS], T[NS * NS];
  const int ec = blockIdx.x;
  const int r = threadIdx.x / NS, c = threadIdx.x % NS;
  double acc = 0.0;
  for (int g = gal_ptr[ec]; g < gal_ptr[ec + 1]; ++g) {
    const int e = gal_fine[g];
    const int i = row_of[e], j = col[e];
    if (threadIdx.x < bs * bs) Ss[threadIdx.x] = Sf[(size_t)e * bs * bs + threadIdx.x];
    if (threadIdx.x < bs * NS) {
      Pi[threadIdx.x] = P[(size_t)i * bs * NS + threadIdx.x];
      Pj[threadIdx.x] = P[(size_t)j * bs * NS + threadIdx.x];
    }
    __syncthreads();
    // T = S_ij P_j  (bs x 16)
    if (r < bs) {
      double s = 0.0;
      for (int k = 0; k < bs; ++k) s += Ss[r * bs + k] * Pj[k * NS + c];
      T[r * NS + c] = s;
    }
    __syncthreads();
    double s = 0.0;
    for (int k = 0; k < bs; ++k) s += Pi[k * NS + r] * T[k * NS + c];
    acc += s;
    __syncthreads();
  }
  Sc[(size_t)ec * NS * NS + threadIdx.x] = acc;
}

// ---------------------------------------------------------------- block inverses

// Inverse of the diagonal 16 x 16 block of every node (one wave per node).
__global__ __launch_bounds__(64) void k_diag_inverse16(const int32_t* __restrict__ diag_pos,
                                                       const double* __restrict__ S,
                                                       double* __restrict__ Dinv, uint32_t* err) {
  __shared__ double a[NS * NS], inv[NS * NS];
  const int i = blockIdx.x;
  const double* blk = S + (size_t)diag_pos[i] * NS * NS;
  for (int k = threadIdx.x; k < NS * NS; k += 64) a[k] = blk[k];
  __syncthreads();
  if (threadIdx.x == 0) {
    if (!cholesky<NS>(a)) {
      atomicOr(err, ERRF_NOT_SPD);
      for (int k = 0; k < NS * NS; ++k) inv[k] = 0.0;
    } else {
      cholesky_inverse<NS>(a, inv);
    }
  }
  __syncthreads();
  for (int k = threadIdx.x; k < NS * NS; k += 64) Dinv[(size_t)i * NS * NS + k] = inv[k];
}

// ---------------------------------------------------------------- coarse level

// Scatter a BSR operator into a dense nd x nd matrix (padding rows get 1 on the
// diagonal). One thread per stored value.
__global__ void k_bsr_to_dense(int n, int bs, int nd, const int32_t* __restrict__ row_of,
                               const int32_t* __restrict__ col, int64_t nnz,
                               const double* __restrict__ S, double* __restrict__ D) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t total = nnz * bs * bs;
  if (idx < total) {
    const int64_t e = idx / (bs * bs);
    const int rc = (int)(idx % (bs * bs));
    const int r = rc / bs, c = rc % bs;
    D[(size_t)(row_of[e] * bs + r) * nd + (size_t)col[e] * bs + c] = S[idx];
  }
  const int64_t pad = idx - total;
  if (pad >= 0 && pad < nd - (int64_t)n * bs) {
    const size_t d = (size_t)n * bs + pad;
    D[d * nd + d] = 1.0;
  }
}

// Equilibration of the coarse matrix: s_i = D_ii^-1/2 (k_dense_diag), then
// A <- s A s + shift I before the factorization and inv <- s inv s after it.
__global__ void k_dense_diag(int nd, const double* __restrict__ A, double* __restrict__ s, uint32_t* err) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nd) return;
  const double d = A[(size_t)i * nd + i];
  if (!(d > 0.0)) {
    atomicOr(err, ERRF_NOT_SPD);
    s[i] = 1.0;
  } else {
    s[i] = 1.0 / sqrt(d);
  }
}

__global__ void k_dense_scale(int nd, double* __restrict__ A, const double* __restrict__ s, double shift) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (int64_t)nd * nd) return;
  const int64_t r = idx / nd, c = idx % nd;
  A[idx] = A[idx] * s[r] * s[c] + (r == c ? shift : 0.0);
}

typedef double d4 __attribute__((ext_vector_type(4)));

// Orders the LDS/global accesses of the lanes of one wave (no block barrier).
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
}

// One 16x16 FP64 tile product on the matrix cores, 4 MFMA 16x16x4 steps:
//   XT = false: C += sx * X Y^T,   XT = true: C += sx * X^T Y,
// X, Y row-major 16 x 16 tiles with leading dimensions ldx, ldy.
// MFMA 16x16x4 f64 operand layout: lane l supplies A[l%16][l/16] and
// B[l/16][l%16]; accumulator element i of lane l is C[4*i + l/16][l%16]
// (rows interleaved across the four lane groups).
template <bool XT>
__device__ __forceinline__ d4 tile_mma(d4 acc, const double* X, int ldx, const double* Y, int ldy,
                                       double sx) {
  const int l = threadIdx.x & 63;
  const int m = l & 15, kq = l >> 4;
#pragma unroll
  for (int kk = 0; kk < 4; ++kk) {
    const int k = kk * 4 + kq;
    const double a = XT ? X[(size_t)k * ldx + m] : X[(size_t)m * ldx + k];
    const double b = XT ? Y[(size_t)k * ldy + m] : Y[(size_t)m * ldy + k];
    acc = __builtin_amdgcn_mfma_f64_16x16x4f64(sx * a, b, acc, 0, 0, 0);
  }
  return acc;
}

// C += sx * X Y (plain product), same layout conventions.
__device__ __forceinline__ d4 tile_mma_nn(d4 acc, const double* X, int ldx, const double* Y, int ldy,
                                          double sx) {
  const int l = threadIdx.x & 63;
  const int m = l & 15, kq = l >> 4;
#pragma unroll
  for (int kk = 0; kk < 4; ++kk) {
    const int k = kk * 4 + kq;
    acc = __builtin_amdgcn_mfma_f64_16x16x4f64(sx * X[(size_t)m * ldx + k], Y[(size_t)k * ldy + m], acc, 0, 0, 0);
  }
  return acc;
}

__device__ __forceinline__ d4 tile_load(const double* C, int ld) {
  const int l = threadIdx.x & 63;
  d4 v;
#pragma unroll
  for (int i = 0; i < 4; ++i) v[i] = C[(size_t)(4 * i + (l >> 4)) * ld + (l & 15)];
  return v;
}

__device__ __forceinline__ void tile_store(double* C, int ld, d4 v) {
  const int l = threadIdx.x & 63;
#pragma unroll
  for (int i = 0; i < 4; ++i) C[(size_t)(4 * i + (l >> 4)) * ld + (l & 15)] = v[i];
}

// Probe of the tile products (checked by a test of the MFMA operand layout):
// mode 0: C += X Y^T, 1: C += X^T Y, 2: C += X Y.
__global__ __launch_bounds__(64) void k_mfma_probe(const double* X, const double* Y, double* C, int mode) {
  d4 acc = tile_load(C, 16);
  if (mode == 0) acc = tile_mma<false>(acc, X, 16, Y, 16, 1.0);
  else if (mode == 1) acc = tile_mma<true>(acc, X, 16, Y, 16, 1.0);
  else acc = tile_mma_nn(acc, X, 16, Y, 16, 1.0);
  tile_store(C, 16, acc);
}

// ---------------------------------------------------------------- coarse inverse

// Dense inverse of the (equilibrated, SPD) coarsest operator by blocked
// Gauss-Jordan elimination with 64 x 64 pivot blocks. With P = A_kk^-1, one
// pivot step maps
//   A_kk <- P,  A_kj <- P A_kj,  A_ik <- -A_ik P,  A_ij <- A_ij - A_ik P A_kj,
// and after every block has served as pivot A holds A^-1. Each step is three
// launches: the 64 x 64 pivot inverse (one workgroup, in LDS), the new pivot
// row and column (one workgroup per block), and the rank-64 update of all
// other blocks (one workgroup per block, 16 waves, each wave one 16 x 16 tile
// on the FP64 matrix cores). nd is a multiple of 64; pivots are the diagonal
// blocks of successive Schur complements, positive definite for SPD A.
constexpr int GJB = 64;

// P = A_kk^-1 by unblocked Gauss-Jordan: 1024 threads, each keeping 4 entries
// of the block in registers (column j = t % 64, rows t / 64 + 16 m); the pivot
// row and column of every step are exchanged through double-buffered LDS, so
// each step costs one barrier.
__global__ __launch_bounds__(1024) void k_gj_pivot(int nd, const double* __restrict__ A, int k,
                                                   double* __restrict__ Pbuf, uint32_t* err) {
  __shared__ double rowp[2][GJB], colp[2][GJB];
  const size_t k0 = (size_t)k * GJB;
  const int t = threadIdx.x, j = t % GJB, i0 = t / GJB;
  double v[4];
#pragma unroll
  for (int m = 0; m < 4; ++m) v[m] = A[(k0 + i0 + 16 * m) * nd + k0 + j];
  bool bad = false;
  for (int p = 0; p < GJB; ++p) {
    const int buf = p & 1;
    if (i0 == (p & 15)) rowp[buf][j] = v[p >> 4];
    if (j == p) {
#pragma unroll
      for (int m = 0; m < 4; ++m) colp[buf][i0 + 16 * m] = v[m];
    }
    __syncthreads();
    const double piv = rowp[buf][p];
    if (!(piv > 0.0)) { bad = true; break; }   // uniform: all threads read the same pivot
    const double ip = 1.0 / piv;
    const double rp = rowp[buf][j] * ip;
#pragma unroll
    for (int m = 0; m < 4; ++m) {
      const int i = i0 + 16 * m;
      const double cp = colp[buf][i];
      if (i == p) v[m] = (j == p) ? ip : rp;
      else v[m] = (j == p) ? -cp * ip : v[m] - cp * rp;
    }
  }
  if (bad) {
    if (t == 0) atomicOr(err, ERRF_NOT_SPD);
    return;
  }
#pragma unroll
  for (int m = 0; m < 4; ++m) Pbuf[(i0 + 16 * m) * GJB + j] = v[m];
}

// One 64 x 64 block product on 16 waves: wave w owns output tile (w/4, w%4);
// acc += sx * X Y (X, Y 64 x 64 row-major, leading dims ldx, ldy).
__device__ __forceinline__ d4 block_mma(d4 acc, const double* X, int ldx, const double* Y, int ldy, double sx) {
  const int w = threadIdx.x >> 6;
  const int tr = w >> 2, tc = w & 3;
#pragma unroll
  for (int t = 0; t < 4; ++t)
    acc = tile_mma_nn(acc, X + (size_t)(tr * 16) * ldx + t * 16, ldx, Y + (size_t)(t * 16) * ldy + tc * 16, ldy, sx);
  return acc;
}

__device__ __forceinline__ double* block_tile(double* B, int ld) {
  const int w = threadIdx.x >> 6;
  return B + (size_t)((w >> 2) * 16) * ld + (w & 3) * 16;
}

// New pivot row and column: for block b != k, Row_b = P A_kb and Col_b = -A_bk P,
// and the old column block kept for the update (Cold_b = A_bk).
__global__ __launch_bounds__(1024) void k_gj_panel(int nd, const double* __restrict__ A, int k,
                                                   const double* __restrict__ Pbuf, double* __restrict__ Row,
                                                   double* __restrict__ Col, double* __restrict__ Cold) {
  const int b = blockIdx.x;
  if (b == k) return;
  const size_t k0 = (size_t)k * GJB, b0 = (size_t)b * GJB;
  const double* Akb = A + k0 * nd + b0;   // row k, block b
  const double* Abk = A + b0 * nd + k0;   // row b, block k
  d4 r = {0, 0, 0, 0}, c = {0, 0, 0, 0};
  r = block_mma(r, Pbuf, GJB, Akb, nd, 1.0);
  c = block_mma(c, Abk, nd, Pbuf, GJB, -1.0);
  tile_store(block_tile(Row + b0, nd), nd, r);          // Row: 64 x nd
  tile_store(block_tile(Col + b0 * GJB, GJB), GJB, c);  // Col: nd x 64
  // copy of the old column block
  for (int idx = threadIdx.x; idx < GJB * GJB; idx += 1024)
    Cold[(b0 + idx / GJB) * GJB + idx % GJB] = Abk[(size_t)(idx / GJB) * nd + idx % GJB];
}

// Rank-64 update of every block (i, j), i, j != k: A_ij -= Cold_i Row_j; the
// pivot row, column and block take their new values.
__global__ __launch_bounds__(1024) void k_gj_update(int nd, double* __restrict__ A, int k,
                                                    const double* __restrict__ Pbuf, const double* __restrict__ Row,
                                                    const double* __restrict__ Col, const double* __restrict__ Cold) {
  const int nb = nd / GJB;
  const int i = blockIdx.x / nb, j = blockIdx.x % nb;
  const size_t i0 = (size_t)i * GJB, j0 = (size_t)j * GJB;
  double* Aij = A + i0 * nd + j0;
  if (i == k && j == k) {
    for (int idx = threadIdx.x; idx < GJB * GJB; idx += 1024) Aij[(size_t)(idx / GJB) * nd + idx % GJB] = Pbuf[idx];
  } else if (i == k) {
    for (int idx = threadIdx.x; idx < GJB * GJB; idx += 1024)
      Aij[(size_t)(idx / GJB) * nd + idx % GJB] = Row[(size_t)(idx / GJB) * nd + j0 + idx % GJB];
  } else if (j == k) {
    for (int idx = threadIdx.x; idx < GJB * GJB; idx += 1024)
      Aij[(size_t)(idx / GJB) * nd + idx % GJB] = Col[(i0 + idx / GJB) * GJB + idx % GJB];
  } else {
    double* t = block_tile(Aij, nd);
    d4 acc = tile_load(t, nd);
    acc = block_mma(acc, Cold + i0 * GJB, GJB, Row + j0, nd, -1.0);
    tile_store(t, nd, acc);
  }
}

}  // namespace bamg
