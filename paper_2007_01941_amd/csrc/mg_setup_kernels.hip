// Multigrid numeric setup (Sections 3.1, 3.3, 3.4, 3.6 of Konolige and Brown):
// camera near-nullspace, per-aggregate QR tentative prolongation, the explicit
// level-0 Schur complement, Galerkin coarse operators P^T S P, smoother block
// inverses, and the dense coarse factorization (the FP64 MFMA site).
#include "kernels.hpp"

namespace bamg {

// Accumulator of one 16 x 16 FP64 MFMA tile (4 entries per lane).
typedef double d4 __attribute__((ext_vector_type(4)));

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
  // lane = (row group g, column c): column sums over rows r = g (mod 4), then
  // two exchanges combine the 4 groups
  const int c = lane & 15, g = lane >> 4;
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
    if (lane == 0) tau[j] = t;
    __syncthreads();
    // apply H_j = I - t v v^T (v = [1; A[j+1:, j]]) to columns j+1..NS-1
    double w = 0.0;
    if (c > j)
      for (int r = j + g; r < rows; r += 4) w += (r == j ? 1.0 : A[r * NS + j]) * A[r * NS + c];
    w += __shfl_xor(w, 16, 64);
    w += __shfl_xor(w, 32, 64);
    w *= t;
    if (c > j)
      for (int r = j + g; r < rows; r += 4) A[r * NS + c] -= w * (r == j ? 1.0 : A[r * NS + j]);
    __syncthreads();
    if (lane == 0) A[j * NS + j] = beta;
    __syncthreads();
  }
  // Q = H_0 ... H_{ncol-1} [I; 0]
  for (int idx = lane; idx < rows * NS; idx += 64) {
    const int r = idx / NS, cc = idx % NS;
    Q[idx] = (r == cc) ? 1.0 : 0.0;
  }
  __syncthreads();
  for (int j = ncol - 1; j >= 0; --j) {
    const double t = tau[j];
    double w = 0.0;
    if (c >= j)
      for (int r = j + g; r < rows; r += 4) w += (r == j ? 1.0 : A[r * NS + j]) * Q[r * NS + c];
    w += __shfl_xor(w, 16, 64);
    w += __shfl_xor(w, 32, 64);
    w *= t;
    if (c >= j)
      for (int r = j + g; r < rows; r += 4) Q[r * NS + c] -= w * (r == j ? 1.0 : A[r * NS + j]);
    __syncthreads();
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

// Level-0 S before the off-diagonal sums: diagonal blocks = the block-Jacobi
// blocks S_cc, every other block 0.
__global__ void k_s0_init(int64_t n, const int32_t* __restrict__ row_of, const int32_t* __restrict__ col,
                          const double* __restrict__ Scc, double* __restrict__ S) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= n) return;
  const int64_t e = idx / 81;
  const int k = (int)(idx - e * 81);
  const int i = row_of[e];
  S[idx] = i == col[e] ? Scc[(size_t)i * 81 + k] : 0.0;
}

// Off-diagonal block (i, j), i < j, of S = A - W C^-1 W^T:
//   S_ij = - sum_{p seen by i and j} F_ip^T (E_ip C_p^-1 E_jp^T) F_jp = - U^T V,
// with U stacking the 2 x 9 blocks F_ip and V the blocks M_p F_jp
// (M_p = E_ip C_p^-1 E_jp^T, 2 x 2) over the shared points p (the plan lists
// them per block and cuts every block's list into chunks of at most
// S0_CHUNK points, so that heavy blocks spread over many waves). One wave per
// chunk: in batches of 64 points each lane recomputes both cameras' Jacobian
// blocks from the camera data and the point record [X | C_p^-1]; the lanes'
// 2 rows of U and V pass through LDS 32 points at a time, and U^T V
// accumulates on the FP64 matrix cores (16 x 16 x 4, 9 x 9 used), two points
// per instruction, in the points' order; the chunk's
// sum is added to blocks (i, j) and (j, i) with global atomics.
// part != NULL (deterministic mode): each chunk stores its 9 x 9 sum to
// part[chunk] instead, and k_s0_gather adds the chunks of every block in
// order; no atomics.
__global__ __launch_bounds__(64) void k_explicit_s0(
    double* __restrict__ part, const int32_t* __restrict__ chunk_e, const int32_t* __restrict__ chunk_beg,
    const int32_t* __restrict__ row_of, const int32_t* __restrict__ col,
    const int32_t* __restrict__ trans_pos, const int32_t* __restrict__ s0_ptr,
    const int32_t* __restrict__ s0_q, const double* __restrict__ campre, const double* __restrict__ prec,
    const int32_t* __restrict__ pt_off, const int32_t* __restrict__ obs_cam, const double* __restrict__ wsq,
    double* __restrict__ S) {
  __shared__ double Us[64 * 9];   // rows of 32 points at a time (LDS per wave
  __shared__ double Vs[64 * 9];   // kept small: more waves per CU)
  const int ch = blockIdx.x;
  const int e = chunk_e[ch];
  const int i = row_of[e], j = col[e];
  const int lane = threadIdx.x;
  const double* ci = campre + (size_t)i * 24;
  const double* cj = campre + (size_t)j * 24;
  const int kq = lane >> 4, cc = lane & 15;
  d4 acc = {0, 0, 0, 0};
  const int beg = chunk_beg[ch];
  const int end = min(s0_ptr[e + 1], beg + S0_CHUNK);
  for (int base = beg; base < end; base += 64) {
    const int nh = end - base < 64 ? end - base : 64;
    double urow[18], vrow[18];   // this lane's point: its 2 rows of U and of V
    if (lane < nh) {
      const int q = s0_q[base + lane];
      const double* rec = prec + (size_t)q * PREC;
      const double X[3] = {rec[0], rec[1], rec[2]};
      const double C[9] = {rec[3], rec[4], rec[5], rec[4], rec[6], rec[7], rec[5], rec[7], rec[8]};
      double pi[2], fi[18], ei[6], fj[18], ej[6], z;
      project_jacobian(ci, X, pi, fi, ei, &z);
      project_jacobian(cj, X, pi, fj, ej, &z);
      if (wsq) {
        // robust loss: the rows of both observations scaled by their sqrt(rho')
        double swi = 1.0, swj = 1.0;
        for (int o = pt_off[q]; o < pt_off[q + 1]; ++o) {
          const int c = obs_cam[o];
          if (c == i) swi = wsq[o];
          if (c == j) swj = wsq[o];
        }
#pragma unroll
        for (int k = 0; k < 18; ++k) {
          fi[k] *= swi;
          fj[k] *= swj;
        }
#pragma unroll
        for (int k = 0; k < 6; ++k) {
          ei[k] *= swi;
          ej[k] *= swj;
        }
      }
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
        for (int t = 0; t < 2; ++t)
          m[r * 2 + t] = ec[r * 3 + 0] * ej[t * 3 + 0] + ec[r * 3 + 1] * ej[t * 3 + 1] + ec[r * 3 + 2] * ej[t * 3 + 2];
#pragma unroll
      for (int k = 0; k < 18; ++k) urow[k] = fi[k];
#pragma unroll
      for (int k = 0; k < 9; ++k) {
        vrow[k] = m[0] * fj[k] + m[1] * fj[9 + k];
        vrow[9 + k] = m[2] * fj[k] + m[3] * fj[9 + k];
      }
    }
    // the batch's points go through LDS in two halves of 32, in order
    for (int n0 = 0; n0 < nh; n0 += 32) {
      const int nn = nh - n0 < 32 ? nh - n0 : 32;
      const int pl = lane - n0;
      if (pl >= 0 && pl < nn) {
#pragma unroll
        for (int k = 0; k < 9; ++k) {
          Us[(2 * pl) * 9 + k] = urow[k];
          Us[(2 * pl + 1) * 9 + k] = urow[9 + k];
          Vs[(2 * pl) * 9 + k] = vrow[k];
          Vs[(2 * pl + 1) * 9 + k] = vrow[9 + k];
        }
      }
      __syncthreads();
      // rows 4 s .. 4 s + 3 of the stacked U, V (points n0 + 2 s, n0 + 2 s + 1)
      for (int st = 0; st < (nn + 1) / 2; ++st) {
        const int row = 4 * st + kq;
        const bool ok = cc < 9 && row < 2 * nn;
        const double a = ok ? Us[row * 9 + cc] : 0.0;
        const double b = ok ? Vs[row * 9 + cc] : 0.0;
        acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc, 0, 0, 0);
      }
      __syncthreads();
    }
  }
  // accumulator element t of lane l holds (U^T V)[4 t + l / 16][l % 16]
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    const int r = 4 * t + kq;
    if (r < 9 && cc < 9) {
      if (part) {
        part[(size_t)ch * 81 + r * 9 + cc] = acc[t];
      } else {
        unsafeAtomicAdd(&S[(size_t)e * 81 + r * 9 + cc], -acc[t]);
        unsafeAtomicAdd(&S[(size_t)trans_pos[e] * 81 + cc * 9 + r], -acc[t]);
      }
    }
  }
}

// Deterministic completion of the explicit level-0 S: block e (upper, listed
// in blk_e with its chunks blk_ch[i] .. blk_ch[i + 1]) and its transpose get
// minus the sum of the chunks' partial products, added in chunk order. One
// thread per (block, entry).
__global__ __launch_bounds__(256) void k_s0_gather(int n_blk, const int32_t* __restrict__ blk_e,
                                                   const int32_t* __restrict__ blk_ch,
                                                   const int32_t* __restrict__ trans_pos,
                                                   const double* __restrict__ part, double* __restrict__ S) {
  const int gid = blockIdx.x * 243 + threadIdx.x;
  const int i = gid / 81, m = gid - i * 81;
  if (threadIdx.x >= 243 || i >= n_blk) return;
  double acc = 0.0;
  for (int ch = blk_ch[i]; ch < blk_ch[i + 1]; ++ch) acc += part[(size_t)ch * 81 + m];
  const int e = blk_e[i], r = m / 9, c = m - r * 9;
  S[(size_t)e * 81 + m] = -acc;
  S[(size_t)trans_pos[e] * 81 + c * 9 + r] = -acc;
}

// ---------------------------------------------------------------- Galerkin product

// Coarse entry (A, B) = sum over fine entries (i, j) with agg(i) = A, agg(j) = B
// of P_i^T S_ij P_j (fine blocks bs x bs, P blocks bs x 16). One workgroup of
// 256 threads per coarse entry; thread (r, c) owns entry (r, c). The fine
// entries are software-pipelined: each thread's elements of the next entry's
// S_ij, P_i and P_j (and the indices of the one after) are loaded while the
// current entry's products run.
__global__ __launch_bounds__(256) void k_galerkin(int bs, const int32_t* __restrict__ gal_ptr,
                                                  const int32_t* __restrict__ gal_fine,
                                                  const int32_t* __restrict__ row_of,
                                                  const int32_t* __restrict__ col,
                                                  const double* __restrict__ Sf,
                                                  const double* __restrict__ P,
                                                  double* __restrict__ Sc) {
  __shared__ double Ss[NS * NS], Pi[NS * NS], Pj[NS * NS], T[NS * NS];
  const int ec = blockIdx.x;
  const int tid = threadIdx.x;
  const int r = tid / NS, c = tid % NS;
  const bool ls = tid < bs * bs, lp = tid < bs * NS;
  const int g0 = gal_ptr[ec], g1 = gal_ptr[ec + 1];
  // indices of entry g (ie, ii, ij) and this thread's elements of it (vs, vi, vj)
  int ie = 0, ii = 0, ij = 0;
  double vs = 0.0, vi = 0.0, vj = 0.0;
  if (g0 < g1) {
    ie = gal_fine[g0];
    ii = row_of[ie];
    ij = col[ie];
    if (ls) vs = Sf[(size_t)ie * bs * bs + tid];
    if (lp) {
      vi = P[(size_t)ii * bs * NS + tid];
      vj = P[(size_t)ij * bs * NS + tid];
    }
  }
  int ne = 0, ni = 0, nj = 0;   // indices of entry g + 1
  if (g0 + 1 < g1) {
    ne = gal_fine[g0 + 1];
    ni = row_of[ne];
    nj = col[ne];
  }
  double acc = 0.0;
  for (int g = g0; g < g1; ++g) {
    if (ls) Ss[tid] = vs;
    if (lp) {
      Pi[tid] = vi;
      Pj[tid] = vj;
    }
    if (g + 1 < g1) {
      if (ls) vs = Sf[(size_t)ne * bs * bs + tid];
      if (lp) {
        vi = P[(size_t)ni * bs * NS + tid];
        vj = P[(size_t)nj * bs * NS + tid];
      }
      if (g + 2 < g1) {
        ne = gal_fine[g + 2];
        ni = row_of[ne];
        nj = col[ne];
      }
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

// Inverse of the diagonal 16 x 16 (SPD) block of every node, one wave per
// node, by Gauss-Jordan without pivoting: lane l keeps column l % 16 of rows
// l / 16 + 4 m (m < 4); the pivot row and column of every step are exchanged
// through double-buffered LDS.
__global__ __launch_bounds__(64) void k_diag_inverse16(const int32_t* __restrict__ diag_pos,
                                                       const double* __restrict__ S,
                                                       double* __restrict__ Dinv, uint32_t* err) {
  __shared__ double rowb[2][NS], colb[2][NS];
  const int i = blockIdx.x;
  const int l = threadIdx.x, c = l % NS, r0 = l / NS;
  const double* blk = S + (size_t)diag_pos[i] * NS * NS;
  double v[4];
#pragma unroll
  for (int m = 0; m < 4; ++m) v[m] = blk[(r0 + 4 * m) * NS + c];
  bool ok = true;
#pragma unroll
  for (int p = 0; p < NS; ++p) {
    const int buf = p & 1;
    if (r0 == (p & 3)) rowb[buf][c] = v[p >> 2];
    if (c == p) {
#pragma unroll
      for (int m = 0; m < 4; ++m) colb[buf][r0 + 4 * m] = v[m];
    }
    __syncthreads();
    const double piv = rowb[buf][p];
    ok = ok && piv > 0.0;
    const double ip = 1.0 / piv;
    const double rp = rowb[buf][c] * ip;
#pragma unroll
    for (int m = 0; m < 4; ++m) {
      const int ii = r0 + 4 * m;
      const double cp = colb[buf][ii];
      if (ii == p) v[m] = (c == p) ? ip : rp;
      else v[m] = (c == p) ? -cp * ip : v[m] - cp * rp;
    }
  }
  if (!ok) {
    if (l == 0) atomicOr(err, ERRF_NOT_SPD);
#pragma unroll
    for (int m = 0; m < 4; ++m) v[m] = 0.0;
  }
#pragma unroll
  for (int m = 0; m < 4; ++m) Dinv[(size_t)i * NS * NS + (r0 + 4 * m) * NS + c] = v[m];
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
// Gauss-Jordan elimination with B x B pivot blocks. With P = A_kk^-1, one
// pivot step maps
//   A_kk <- P,  A_kj <- P A_kj,  A_ik <- -A_ik P,  A_ij <- A_ij - A_ik P A_kj,
// and after every block has served as pivot A holds A^-1. The first pivot
// inverse is a launch of its own (one workgroup); every step is then one
// launch that updates every block (one workgroup per block, reading one copy
// of A and writing the other) and inverts the next pivot. nd is a multiple of
// B; pivots are the diagonal blocks of successive Schur complements,
// positive definite for SPD A. The pivot inverses form the sequential chain
// of the elimination (one per step); each step reads and writes the whole
// matrix. B = 64 (inverted as 2 x 2 blocks of 32, see block_inverse) and
// B = 32 (half the chain per step, twice the steps) measured alike on the
// coarsest operators met here; 64 takes half the launches and traffic.
constexpr int GJB = 64;

// 1 / x for a positive normal x: the hardware reciprocal estimate refined by
// two steps of Newton's iteration r <- r + r (1 - x r) (each step squares the
// relative error), which leaves it within about an ulp of the quotient; a
// shorter dependent chain than the fully rounded division, and the pivots'
// reciprocals are the sequential part of the elimination.
__device__ __forceinline__ double recip_newton(double x) {
  double r = __builtin_amdgcn_rcp(x);
  r = fma(r, fma(-x, r, 1.0), r);
  r = fma(r, fma(-x, r, 1.0), r);
  return r;
}

// In-place inverse of a 4 x 4 SPD matrix (row-major) by Gauss-Jordan without
// pivoting; false if a pivot is not positive (or below the normal range).
__device__ __forceinline__ bool inv4(double (&a)[16]) {
  bool ok = true;
#pragma unroll
  for (int p = 0; p < 4; ++p) {
    const double piv = a[p * 4 + p];
    ok = ok && (piv >= 0x1p-1022);
    const double ip = recip_newton(piv);
#pragma unroll
    for (int j = 0; j < 4; ++j)
      if (j != p) a[p * 4 + j] *= ip;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      if (i == p) continue;
      const double aip = a[i * 4 + p];
#pragma unroll
      for (int j = 0; j < 4; ++j)
        if (j != p) a[i * 4 + j] -= aip * a[p * 4 + j];
      a[i * 4 + p] = -aip * ip;
    }
    a[p * 4 + p] = ip;
  }
  return ok;
}

// v <- inverse of a B x B SPD block held by 256 threads (thread t keeps
// column j = t % B, rows i0 + R m with i0 = t / B, R = 256 / B, m < B / R),
// by Gauss-Jordan on 4 x 4 pivot blocks: pivot block q is rows 4q .. 4q+3,
// i.e. register v[4q / R] of the threads with i0 - 4q mod R in 0 .. 3.
// Pivot rows and columns go through double-buffered LDS (one barrier per
// pivot block); every thread inverts the 4 x 4 pivot itself.
template <int B>
__device__ __forceinline__ bool pivot_inverse(double (&v)[B * B / 256], double (*rowK)[4][B],
                                              double (*colK)[B][4]) {
  constexpr int R = 256 / B, M = B / R;
  const int t = threadIdx.x, j = t % B, i0 = t / B;
  bool ok = true;
#pragma unroll
  for (int q = 0; q < B / 4; ++q) {
    const int buf = q & 1;
    const int mq = (4 * q) / R;          // the register holding the pivot rows
    const int aq = i0 - (4 * q) % R;     // this thread's row within the pivot block
    const bool prow = aq >= 0 && aq < 4;
    if (prow) rowK[buf][aq][j] = v[mq];
    if ((j >> 2) == q) {
#pragma unroll
      for (int m = 0; m < M; ++m) colK[buf][i0 + R * m][j & 3] = v[m];
    }
    __syncthreads();
    double p4[16];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
      for (int bb = 0; bb < 4; ++bb) p4[a * 4 + bb] = rowK[buf][a][4 * q + bb];
    ok = inv4(p4) && ok;
    double tj[4];
    {
      const double r0 = rowK[buf][0][j], r1 = rowK[buf][1][j], r2 = rowK[buf][2][j], r3 = rowK[buf][3][j];
#pragma unroll
      for (int a = 0; a < 4; ++a) tj[a] = p4[a * 4 + 0] * r0 + p4[a * 4 + 1] * r1 + p4[a * 4 + 2] * r2 + p4[a * 4 + 3] * r3;
    }
    const bool jin = (j >> 2) == q;
    const int bj = j & 3;
    double pc[4];   // column bj of the pivot inverse (used when j is a pivot column)
#pragma unroll
    for (int a = 0; a < 4; ++a)
      pc[a] = bj == 0 ? p4[a * 4 + 0] : bj == 1 ? p4[a * 4 + 1] : bj == 2 ? p4[a * 4 + 2] : p4[a * 4 + 3];
    // the coefficients that multiply the pivot column entries of row i
    double w[4];
#pragma unroll
    for (int a = 0; a < 4; ++a) w[a] = jin ? pc[a] : tj[a];
#pragma unroll
    for (int m = 0; m < M; ++m) {
      if (m == mq && prow) {
        // row 4q + aq of the pivot block row
        v[m] = aq == 0 ? w[0] : aq == 1 ? w[1] : aq == 2 ? w[2] : w[3];
      } else {
        const int i = i0 + R * m;
        const double c0 = colK[buf][i][0], c1 = colK[buf][i][1], c2 = colK[buf][i][2], c3 = colK[buf][i][3];
        const double d = c0 * w[0] + c1 * w[1] + c2 * w[2] + c3 * w[3];
        v[m] = jin ? -d : v[m] - d;
      }
    }
  }
  return ok;
}

// Staging of a B x B block into LDS (leading dim B + 1), 256 threads.
template <int B>
__device__ __forceinline__ void stage_block256(double* __restrict__ dst, const double* __restrict__ src, size_t ld) {
#pragma unroll 4
  for (int r = 0; r < B * B / 256; ++r) {
    const int idx = threadIdx.x + 256 * r;
    dst[(idx / B) * (B + 1) + idx % B] = src[(size_t)(idx / B) * ld + idx % B];
  }
}

// The same in two halves: the global loads into registers, and (later) the
// registers into LDS, so that a load can be in flight during other work.
template <int B>
__device__ __forceinline__ void load_block256(double (&r)[B * B / 256], const double* __restrict__ src, size_t ld) {
#pragma unroll
  for (int i = 0; i < B * B / 256; ++i) {
    const int idx = threadIdx.x + 256 * i;
    r[i] = src[(size_t)(idx / B) * ld + idx % B];
  }
}

template <int B>
__device__ __forceinline__ void store_block256(double* __restrict__ dst, const double (&r)[B * B / 256]) {
#pragma unroll
  for (int i = 0; i < B * B / 256; ++i) {
    const int idx = threadIdx.x + 256 * i;
    dst[(idx / B) * (B + 1) + idx % B] = r[i];
  }
}

// acc[u] += sx * (X Y) for this wave's tiles of a B x B product, X and Y in
// LDS (leading dim ld)
template <int B>
__device__ __forceinline__ void wave_tiles_mma(d4 (&acc)[(B / 16) * (B / 16) / 4], const double* X, const double* Y,
                                               int ld, double sx) {
  constexpr int TI = B / 16, NT = TI * TI / 4;
  const int w = threadIdx.x >> 6;
#pragma unroll
  for (int u = 0; u < NT; ++u) {
    const int e = w * NT + u, tr = e / TI, tc = e % TI;
#pragma unroll
    for (int t = 0; t < TI; ++t)
      acc[u] = tile_mma_nn(acc[u], X + (size_t)(tr * 16) * ld + t * 16, ld, Y + (size_t)(t * 16) * ld + tc * 16, ld, sx);
  }
}

// In-place inverse of the SPD B x B block held in LDS X (leading dim B + 1)
// by the 256 threads of the workgroup; Y is LDS scratch of the same size.
// B = 32: pivot_inverse directly. B = 64: by the 2 x 2 partition into
// 32 x 32 blocks [A11 A12; A21 A22]:
//   X11 = A11^-1,  T = X11 A12,  R = A21 X11,  S = A22 - A21 T,  Si = S^-1,
//   inverse = [X11 - T B21, B12; B21, Si] with B12 = -T Si, B21 = -Si R,
// the two 32 x 32 inverses by pivot_inverse<32> (S is the Schur complement
// of A11, SPD with A) and the products on the FP64 matrix cores (wave w:
// tile (w / 2, w % 2) of every 32 x 32 product), so that the sequential
// part is two 32 x 32 eliminations instead of one 64 x 64. False if a pivot
// is not positive.
__device__ __forceinline__ bool inv32_lds(double* A, int ld, double (*rowK)[4][32], double (*colK)[32][4]) {
  const int t = threadIdx.x, j = t % 32, i0 = t / 32;
  double v[4];
#pragma unroll
  for (int m = 0; m < 4; ++m) v[m] = A[(i0 + 8 * m) * ld + j];
  const bool ok = pivot_inverse<32>(v, rowK, colK);
#pragma unroll
  for (int m = 0; m < 4; ++m) A[(i0 + 8 * m) * ld + j] = v[m];
  return ok;
}

template <int B>
__device__ __forceinline__ bool block_inverse(double* X, double* Y, double (*rowK)[4][32], double (*colK)[32][4]) {
  constexpr int LD = B + 1;
  if (B == 32) return inv32_lds(X, LD, rowK, colK);
  const int w = threadIdx.x >> 6, tr = w >> 1, tc = w & 1;
  double* A11 = X;
  double* A12 = X + 32;
  double* A21 = X + 32 * LD;
  double* A22 = X + 32 * LD + 32;
  double* T = Y;             // Y rows 0 .. 31
  double* R = Y + 32 * LD;   // Y rows 32 .. 63
  const size_t me = (size_t)(tr * 16) * LD + tc * 16;   // this wave's tile
  bool ok = inv32_lds(A11, LD, rowK, colK);
  __syncthreads();
  d4 tt = {0, 0, 0, 0}, rr = {0, 0, 0, 0};
#pragma unroll
  for (int kk = 0; kk < 2; ++kk) {
    tt = tile_mma_nn(tt, A11 + (tr * 16) * LD + kk * 16, LD, A12 + (kk * 16) * LD + tc * 16, LD, 1.0);
    rr = tile_mma_nn(rr, A21 + (tr * 16) * LD + kk * 16, LD, A11 + (kk * 16) * LD + tc * 16, LD, 1.0);
  }
  tile_store(T + me, LD, tt);
  tile_store(R + me, LD, rr);
  __syncthreads();
  // S in place of A22 (each wave reads only its own tile of A22)
  d4 ss = tile_load(A22 + me, LD);
#pragma unroll
  for (int kk = 0; kk < 2; ++kk)
    ss = tile_mma_nn(ss, A21 + (tr * 16) * LD + kk * 16, LD, T + (kk * 16) * LD + tc * 16, LD, -1.0);
  tile_store(A22 + me, LD, ss);
  __syncthreads();
  ok = inv32_lds(A22, LD, rowK, colK) && ok;
  __syncthreads();
  d4 b12 = {0, 0, 0, 0}, b21 = {0, 0, 0, 0};
#pragma unroll
  for (int kk = 0; kk < 2; ++kk) {
    b12 = tile_mma_nn(b12, T + (tr * 16) * LD + kk * 16, LD, A22 + (kk * 16) * LD + tc * 16, LD, -1.0);
    b21 = tile_mma_nn(b21, A22 + (tr * 16) * LD + kk * 16, LD, R + (kk * 16) * LD + tc * 16, LD, -1.0);
  }
  tile_store(A12 + me, LD, b12);
  tile_store(A21 + me, LD, b21);
  __syncthreads();
  // X11 - T B21 in place of A11 (each wave reads only its own tile of A11)
  d4 b11 = tile_load(A11 + me, LD);
#pragma unroll
  for (int kk = 0; kk < 2; ++kk)
    b11 = tile_mma_nn(b11, T + (tr * 16) * LD + kk * 16, LD, A21 + (kk * 16) * LD + tc * 16, LD, -1.0);
  tile_store(A11 + me, LD, b11);
  __syncthreads();
  return ok;
}

// P = A_kk^-1 for pivot step k (one workgroup of 256 threads).
template <int B>
__global__ __launch_bounds__(256) void k_gj_pivot(int nd, const double* __restrict__ A, int k,
                                                  double* __restrict__ Pbuf, uint32_t* err) {
  constexpr int LD = B + 1;
  __shared__ double X[B * LD];
  __shared__ double Y[B == 64 ? B * LD : 1];
  __shared__ double rowK[2][4][32];
  __shared__ double colK[2][32][4];
  const size_t k0 = (size_t)k * B;
  stage_block256<B>(X, A + k0 * nd + k0, nd);
  __syncthreads();
  if (!block_inverse<B>(X, Y, rowK, colK) && threadIdx.x == 0) atomicOr(err, ERRF_NOT_SPD);
#pragma unroll
  for (int r = 0; r < B * B / 256; ++r) {
    const int idx = threadIdx.x + 256 * r;
    Pbuf[idx] = X[(idx / B) * LD + idx % B];
  }
}

// Pivot step k of blocked Gauss-Jordan from Ain to Aout, given P = A_kk^-1:
// one workgroup of four waves per B x B block (i, j), i <= j (the block's
// 16 x 16 tiles in row-major order, dealt to the waves in equal consecutive
// shares), writes
//   (k, k): P;   (k, j): P A_kj;   (i, k): -A_ik P;   else A_ij - A_ik (P A_kj),
// operands staged in LDS, products on the FP64 matrix cores. The iterate
// keeps a fixed symmetry: A_ji = s A_ij^T with s = -1 when exactly one of
// i, j has already served as pivot (i, j <= k) and +1 otherwise, so each
// workgroup also writes block (j, i) and only the upper blocks are computed.
// Look-ahead: the workgroup of block (k+1, k+1), the next step's pivot block,
// is dispatched first and also inverts its result into Pnext
// (block_inverse on its 256 threads), so every step after the first is one
// launch and the inverse overlaps the other blocks' updates.
template <int B>
__global__ __launch_bounds__(256) void k_gj_step(int nd, const double* __restrict__ Ain, double* __restrict__ Aout,
                                                 int k, const double* __restrict__ Pbuf, double* __restrict__ Pnext,
                                                 uint32_t* err) {
  constexpr int LD = B + 1, TI = B / 16, NT = TI * TI / 4;
  __shared__ double X[B * LD];
  __shared__ double Y[B * LD];
  __shared__ double rowK[2][4][32];
  __shared__ double colK[2][32][4];
  const int nb = nd / B;
  // upper block number -> (bi, bj), bi <= bj, row by row; the next pivot
  // block (k+1, k+1) goes to workgroup 0
  int e = blockIdx.x;
  if (k + 1 < nb) {
    const int di = (k + 1) * nb - (k + 1) * k / 2;
    e = e == 0 ? di : e <= di ? e - 1 : e;
  }
  int bi = 0, rem = e;
  while (rem >= nb - bi) { rem -= nb - bi; ++bi; }
  const int bj = bi + rem;
  const size_t k0 = (size_t)k * B, i0 = (size_t)bi * B, j0 = (size_t)bj * B;
  const int w = threadIdx.x >> 6;
  d4 acc[NT];
#pragma unroll
  for (int u = 0; u < NT; ++u) acc[u] = d4{0, 0, 0, 0};
  if (bi == k && bj == k) {
    stage_block256<B>(X, Pbuf, B);
    __syncthreads();
#pragma unroll
    for (int u = 0; u < NT; ++u) {
      const int te = w * NT + u;
      acc[u] = tile_load(X + (size_t)((te / TI) * 16) * LD + (te % TI) * 16, LD);
    }
  } else if (bi == k) {
    stage_block256<B>(X, Pbuf, B);
    stage_block256<B>(Y, Ain + k0 * nd + j0, nd);
    __syncthreads();
    wave_tiles_mma<B>(acc, X, Y, LD, 1.0);
  } else if (bj == k) {
    stage_block256<B>(X, Ain + i0 * nd + k0, nd);
    stage_block256<B>(Y, Pbuf, B);
    __syncthreads();
    wave_tiles_mma<B>(acc, X, Y, LD, -1.0);
  } else {
    // A_ik and A_ij are loaded up front, in flight during T = P A_kj
    double aik[B * B / 256];
    load_block256<B>(aik, Ain + i0 * nd + k0, nd);
#pragma unroll
    for (int u = 0; u < NT; ++u) {
      const int te = w * NT + u;
      acc[u] = tile_load(Ain + (i0 + (te / TI) * 16) * nd + j0 + (te % TI) * 16, nd);
    }
    stage_block256<B>(X, Pbuf, B);
    stage_block256<B>(Y, Ain + k0 * nd + j0, nd);
    __syncthreads();
    d4 tk[NT];
#pragma unroll
    for (int u = 0; u < NT; ++u) tk[u] = d4{0, 0, 0, 0};
    wave_tiles_mma<B>(tk, X, Y, LD, 1.0);   // T = P A_kj
    __syncthreads();                         // every wave is done with X and Y
#pragma unroll
    for (int u = 0; u < NT; ++u) {
      const int te = w * NT + u;
      tile_store(Y + (size_t)((te / TI) * 16) * LD + (te % TI) * 16, LD, tk[u]);
    }
    store_block256<B>(X, aik);
    __syncthreads();
    wave_tiles_mma<B>(acc, X, Y, LD, -1.0);
  }
#pragma unroll
  for (int u = 0; u < NT; ++u) {
    const int te = w * NT + u;
    tile_store(Aout + (i0 + (te / TI) * 16) * nd + j0 + (te % TI) * 16, nd, acc[u]);
  }
  if (bi != bj) {
    // block (j, i) = s (block (i, j))^T: tile (tr, tc) goes to tile (tc, tr)
    // of block (j, i), transposed
    const double sgn = ((bi <= k) != (bj <= k)) ? -1.0 : 1.0;
    const int l = threadIdx.x & 63;
#pragma unroll
    for (int u = 0; u < NT; ++u) {
      const int te = w * NT + u, tr = te / TI, tc = te % TI;
      double* T = Aout + (j0 + tc * 16) * nd + i0 + tr * 16;
#pragma unroll
      for (int t = 0; t < 4; ++t) T[(size_t)(l & 15) * nd + 4 * t + (l >> 4)] = sgn * acc[u][t];
    }
  } else if (bi == k + 1) {
    // the next pivot block, inverted here from the values Aout receives
    __syncthreads();   // every wave is done reading X
#pragma unroll
    for (int u = 0; u < NT; ++u) {
      const int te = w * NT + u;
      tile_store(X + (size_t)((te / TI) * 16) * LD + (te % TI) * 16, LD, acc[u]);
    }
    __syncthreads();
    if (!block_inverse<B>(X, Y, rowK, colK) && threadIdx.x == 0) atomicOr(err, ERRF_NOT_SPD);
#pragma unroll
    for (int r = 0; r < B * B / 256; ++r) {
      const int idx = threadIdx.x + 256 * r;
      Pnext[idx] = X[(idx / B) * LD + idx % B];
    }
  }
}

template __global__ void k_gj_pivot<32>(int, const double*, int, double*, uint32_t*);
template __global__ void k_gj_pivot<64>(int, const double*, int, double*, uint32_t*);
template __global__ void k_gj_step<32>(int, const double*, double*, int, const double*, double*, uint32_t*);
template __global__ void k_gj_step<64>(int, const double*, double*, int, const double*, double*, uint32_t*);

}  // namespace bamg
