// Multigrid V-cycle kernels (Algorithm 1 of Konolige and Brown, Chebyshev
// smoothing of Section 3.4): block-sparse products with the explicit level
// operators, point-block-Jacobi applications, the Chebyshev recurrence,
// restriction R = P^T, prolongation and the dense coarse solve.
// Every kernel takes the PCG `done` flag and returns at once when it is set.
#include "kernels.hpp"

namespace bamg {

// Prolongation into the finer level fused into the kernel that finishes a
// coarse node's iterate: x_f,i += P_i x_a for the members i of aggregate a
// (each fine node has one aggregate, so no two workgroups write one x_f,i).
template <class T>
struct ProlongTo {
  const int32_t* ptr = nullptr;   // finer level's members of every aggregate: mem[ptr[a] .. ptr[a+1])
  const int32_t* mem = nullptr;
  const T* P = nullptr;           // its tentative blocks [n_f][bs][16]
  T* x = nullptr;                 // its iterate (null: no prolongation)
  int bs = 0;                     // its block size
};

// x_f,i += P_i xa over the members of aggregate a, on one wave whose lane m
// (m < 16) holds component m of x_a in xv; lanes step over (member, row) pairs.
template <class T>
__device__ __forceinline__ void prolong_members(const ProlongTo<T>& pro, int a, T xv) {
  const int lane = threadIdx.x & 63;
  T xa[NS];
#pragma unroll
  for (int m = 0; m < NS; ++m) xa[m] = __shfl(xv, m, 64);
  const int i0 = pro.ptr[a], cnt = (pro.ptr[a + 1] - i0) * pro.bs;
  for (int q = lane; q < cnt; q += 64) {
    const int i = pro.mem[i0 + q / pro.bs], k = q % pro.bs;
    const T* Pi = pro.P + ((size_t)i * pro.bs + k) * NS;
    T s = 0;
#pragma unroll
    for (int m = 0; m < NS; ++m) s += Pi[m] * xa[m];
    pro.x[(size_t)i * pro.bs + k] += s;
  }
}

// Epilogues of the block-row product t = (S v)_i (one node i per workgroup).
// The Chebyshev coefficient c2 is given for lambda_max = 1 and scaled by
// *ilmax = 1 / lambda_max, which stays on the device:
enum RowEpilogue {
  EP_STORE = 0,     // out_i = t
  EP_RESID = 1,     // r_i -= t;  part_{slot(i)} = P_i^T r_i (restriction partial)
  EP_CHEB = 2,      // v = d_in:  r_i -= t;  d_out_i = c1 d_in_i + c2 D_i^-1 r_i;  x_out_i = x_in_i + d_out_i
  EP_CHEB_POST = 3  // v = x_in:  r_i = b_i - t;  d_out_i = c2 D_i^-1 r_i;  x_out_i = x_in_i + d_out_i
};

// Block-sparse product with the explicit level operator (BS x BS blocks, CSR
// of blocks), one workgroup of 256 threads per block row. A row's blocks are
// contiguous, and the workgroup streams them NB = 256 / BS^2 blocks at a time
// (3 of 9 x 9, 1 of 16 x 16): thread t keeps entry (r, c) of block t / BS^2
// of each group, so that consecutive threads read consecutive scalars, and
// accumulates S_rc v_c; the sums over c (and the NB blocks) give the row's
// component r (16 x 16: a 16-lane butterfly; 9 x 9: 27 partials in LDS). The
// row's Chebyshev update (EP_CHEB, EP_CHEB_POST) or residual update (EP_RESID)
// is then applied in place: the workgroup owns all of node i. The product's
// input v is never written here (d_in, d_out and x_in, x_out are different
// buffers where v is one of them).
template <int BS, class T, int EP>
__global__ __launch_bounds__(256) void k_bsr_row(int n, const int32_t* __restrict__ rowptr,
                                                 const int32_t* __restrict__ col, const T* __restrict__ S,
                                                 const T* __restrict__ v, T* __restrict__ out,
                                                 const T* __restrict__ Dinv, const T* __restrict__ b,
                                                 T* __restrict__ r, const T* __restrict__ d_in,
                                                 T* __restrict__ d_out, const T* __restrict__ x_in,
                                                 T* __restrict__ x_out, T c1, T c2,
                                                 const double* __restrict__ ilmax,
                                                 const T* __restrict__ P, const int32_t* __restrict__ slot_of,
                                                 T* __restrict__ rpart, ProlongTo<T> pro, const int* done) {
  if (done && *done) return;
  constexpr int BB = BS * BS;
  constexpr int NB = 256 / BB;
  __shared__ T red[256];
  __shared__ T rs[BS];
  const int row = blockIdx.x;
  const int comp = threadIdx.x % BS;
  const bool own = threadIdx.x < BS;
  const size_t k = (size_t)row * BS + comp;
  // the epilogue's operands are loaded first, so that their latency overlaps
  // the row product's
  T r0 = 0, d0 = 0, x0 = 0;
  if (own && EP != EP_STORE) {
    r0 = EP == EP_CHEB_POST ? b[k] : r[k];
    if (EP == EP_CHEB) d0 = d_in[k];
    if (EP == EP_CHEB || EP == EP_CHEB_POST) x0 = x_in[k];
  }
  int slot = 0;
  if (EP == EP_RESID && rpart && threadIdx.x < NS) slot = slot_of[row];
  // and so are the epilogue's matrix rows: D_i^-1 row comp (Chebyshev) or
  // column threadIdx.x of P_i (restriction)
  T mrow[BS];
  if ((EP == EP_CHEB || EP == EP_CHEB_POST) && own) {
#pragma unroll
    for (int k2 = 0; k2 < BS; ++k2) mrow[k2] = Dinv[(size_t)row * BS * BS + comp * BS + k2];
  }
  if (EP == EP_RESID && rpart && threadIdx.x < NS) {
#pragma unroll
    for (int k2 = 0; k2 < BS; ++k2) mrow[k2] = P[(size_t)row * BS * NS + k2 * NS + threadIdx.x];
  }
  T acc = 0;
  const int blk = threadIdx.x / BB, rc = threadIdx.x % BB;
  if (blk < NB) {
    const int e1 = rowptr[row + 1];
    const int c = rc % BS;
    // batches of U blocks per thread: the U column indices, then the U operator
    // entries and v entries, are all in flight together
    constexpr int U = 8;
    for (int e = rowptr[row] + blk; e < e1; e += NB * U) {
      int cj[U];
#pragma unroll
      for (int u = 0; u < U; ++u) cj[u] = e + u * NB < e1 ? col[e + u * NB] : -1;
      T sv[U], vv[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        sv[u] = cj[u] >= 0 ? S[(size_t)(e + u * NB) * BB + rc] : T(0);
        vv[u] = cj[u] >= 0 ? v[(size_t)cj[u] * BS + c] : T(0);
      }
#pragma unroll
      for (int u = 0; u < U; ++u) acc += sv[u] * vv[u];
    }
  }
  if (BS == 16) {
    // lanes 16 r .. 16 r + 15 hold row r's terms
#pragma unroll
    for (int off = 8; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 64);
    if ((threadIdx.x & 15) == 0) red[threadIdx.x >> 4] = acc;
  } else {
    red[threadIdx.x] = acc;
  }
  __syncthreads();
  if (own) {
    T tsum = 0;
    if (BS == 16) {
      tsum = red[comp];
    } else {
#pragma unroll
      for (int q = 0; q < NB; ++q)
#pragma unroll
        for (int c = 0; c < BS; ++c) tsum += red[q * BB + comp * BS + c];
    }
    if (EP == EP_STORE) {
      out[k] = tsum;
    } else {
      const T rv = r0 - tsum;
      r[k] = rv;
      rs[comp] = rv;
    }
  }
  if (EP == EP_STORE) return;
  __syncthreads();
  if (EP == EP_RESID) {
    if (rpart && threadIdx.x < NS) {
      T sacc = 0;
#pragma unroll
      for (int k2 = 0; k2 < BS; ++k2) sacc += mrow[k2] * rs[k2];
      rpart[(size_t)slot * NS + threadIdx.x] = sacc;
    }
    return;
  }
  if (threadIdx.x >= 64) return;   // the node's components are on lanes 0 .. BS-1 of wave 0
  T xv = 0;
  if (own) {
    T z = 0;
#pragma unroll
    for (int k2 = 0; k2 < BS; ++k2) z += mrow[k2] * rs[k2];
    const T c2s = c2 * (T)*ilmax;
    const T dv = EP == EP_CHEB ? c1 * d0 + c2s * z : c2s * z;
    d_out[k] = dv;
    xv = x0 + dv;
    x_out[k] = xv;
  }
  if constexpr (EP == EP_CHEB && BS == NS) {
    if (pro.x) prolong_members(pro, row, xv);
  }
}

// z = D^-1 r block by block (BS x BS inverse blocks), one thread per dof.
template <int BS, class T>
__global__ __launch_bounds__(256) void k_blockdiag(int n, const T* __restrict__ Dinv,
                                                   const T* __restrict__ r, T* __restrict__ z,
                                                   const int* done) {
  if (done && *done) return;
  const int g = blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= n * BS) return;
  const int i = g / BS, a = g % BS;
  const T* m = Dinv + (size_t)i * BS * BS + a * BS;
  const T* rv = r + (size_t)i * BS;
  T s = 0;
#pragma unroll
  for (int k = 0; k < BS; ++k) s += m[k] * rv[k];
  z[g] = s;
}

// First Chebyshev step (inv_theta for lambda_max = 1, scaled by *ilmax).
// mode 0 (pre-smoothing from x = 0, r = b):
//   d = D^-1 b / theta; x = d; r = b.
// mode 1 (post-smoothing from x, t = S x): r = b - t; d = D^-1 r / theta; x += d.
// mode 2: as mode 0, with b first formed (and stored) from the finer level's
//   restriction partials: b_i = sum_{q in [agg_ptr[i], agg_ptr[i+1])} part_q.
template <int BS, class T>
__global__ __launch_bounds__(256) void k_cheb_first(int n, int mode, const T* __restrict__ Dinv,
                                                    T* __restrict__ b, const T* __restrict__ t,
                                                    T* __restrict__ r, T* __restrict__ d,
                                                    T* __restrict__ x, T inv_theta,
                                                    const double* __restrict__ ilmax,
                                                    const int32_t* __restrict__ agg_ptr,
                                                    const T* __restrict__ part, const int* done) {
  if (done && *done) return;
  __shared__ T rs[256];
  const int nodes_per_block = 256 / BS;
  const int ln = threadIdx.x / BS, a = threadIdx.x % BS;
  const int i = blockIdx.x * nodes_per_block + ln;
  const bool act = ln < nodes_per_block && i < n;
  if (act) {
    const size_t k = (size_t)i * BS + a;
    T rv;
    if (mode == 2) {
      rv = 0;
      for (int q = agg_ptr[i]; q < agg_ptr[i + 1]; ++q) rv += part[(size_t)q * BS + a];
      b[k] = rv;
    } else {
      rv = mode == 0 ? b[k] : b[k] - t[k];
    }
    rs[ln * BS + a] = rv;
    r[k] = rv;
  }
  __syncthreads();
  if (!act) return;
  const T* m = Dinv + (size_t)i * BS * BS + a * BS;
  T s = 0;
#pragma unroll
  for (int k2 = 0; k2 < BS; ++k2) s += m[k2] * rs[ln * BS + k2];
  const size_t k = (size_t)i * BS + a;
  const T dv = s * (inv_theta * (T)*ilmax);
  d[k] = dv;
  x[k] = mode == 1 ? x[k] + dv : dv;
}

// Later Chebyshev steps: r -= t (t = S d); d = c1 d + c2 D^-1 r; x += d (c2 for
// lambda_max = 1, scaled by *ilmax).
template <int BS, class T>
__global__ __launch_bounds__(256) void k_cheb_next(int n, const T* __restrict__ Dinv, const T* __restrict__ t,
                                                   T* __restrict__ r, T* __restrict__ d, T* __restrict__ x,
                                                   T c1, T c2, const double* __restrict__ ilmax,
                                                   const int* done) {
  if (done && *done) return;
  __shared__ T rs[256];
  const int nodes_per_block = 256 / BS;
  const int ln = threadIdx.x / BS, a = threadIdx.x % BS;
  const int i = blockIdx.x * nodes_per_block + ln;
  const bool act = ln < nodes_per_block && i < n;
  if (act) {
    const size_t k = (size_t)i * BS + a;
    const T rv = r[k] - t[k];
    rs[ln * BS + a] = rv;
    r[k] = rv;
  }
  __syncthreads();
  if (!act) return;
  const T* m = Dinv + (size_t)i * BS * BS + a * BS;
  T s = 0;
#pragma unroll
  for (int k2 = 0; k2 < BS; ++k2) s += m[k2] * rs[ln * BS + k2];
  const size_t k = (size_t)i * BS + a;
  const T dv = c1 * d[k] + (c2 * (T)*ilmax) * s;
  d[k] = dv;
  x[k] += dv;
}

// Restriction b_c[a] = sum_{i in a} P_i^T (r_i - t_i) (t optional: the last
// residual update of the pre-smoother is fused here), in two passes so that
// no thread chases member indices: (1) one thread per (fine node, m) writes
// P_i^T (r_i - t_i) to the node's slot in aggregate order; (2) one thread per
// (aggregate, m) sums its members' contiguous slots.
template <int BS, class T>
__global__ __launch_bounds__(256) void k_restrict_nodes(int n, const int32_t* __restrict__ slot_of,
                                                        const T* __restrict__ P, const T* __restrict__ r,
                                                        const T* __restrict__ t, T* __restrict__ part,
                                                        const int* done) {
  if (done && *done) return;
  const int g = blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= n * NS) return;
  const int i = g / NS, m = g % NS;
  const T* Pi = P + (size_t)i * BS * NS + m;
  const T* ri = r + (size_t)i * BS;
  T s = 0;
  if (t) {
    const T* ti = t + (size_t)i * BS;
#pragma unroll
    for (int k = 0; k < BS; ++k) s += Pi[k * NS] * (ri[k] - ti[k]);
  } else {
#pragma unroll
    for (int k = 0; k < BS; ++k) s += Pi[k * NS] * ri[k];
  }
  part[(size_t)slot_of[i] * NS + m] = s;
}

template <class T>
__global__ __launch_bounds__(256) void k_restrict_sum(int n_agg, const int32_t* __restrict__ agg_ptr,
                                                      const T* __restrict__ part, T* __restrict__ bc,
                                                      const int* done) {
  if (done && *done) return;
  const int g = blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= n_agg * NS) return;
  const int a = g / NS, m = g % NS;
  T s = 0;
  for (int q = agg_ptr[a]; q < agg_ptr[a + 1]; ++q) s += part[(size_t)q * NS + m];
  bc[g] = s;
}

// Prolongation x_i += P_i x_c[agg(i)], one thread per fine dof.
template <int BS, class T>
__global__ __launch_bounds__(256) void k_prolong(int n, const int32_t* __restrict__ agg,
                                                 const T* __restrict__ P, const T* __restrict__ xc,
                                                 T* __restrict__ x, const int* done) {
  if (done && *done) return;
  const int g = blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= n * BS) return;
  const int i = g / BS, k = g % BS;
  const T* Pi = P + (size_t)i * BS * NS + k * NS;
  const T* xv = xc + (size_t)agg[i] * NS;
  T s = 0;
#pragma unroll
  for (int m = 0; m < NS; ++m) s += Pi[m] * xv[m];
  x[g] += s;
}

// Coarse solve x = inv b with the dense FP64 inverse (nd x nd, nd >= nv);
// one wave per row, FP64 accumulation whatever the vector type.
template <class T>
__global__ __launch_bounds__(256) void k_dense_solve(int nv, int nd, const double* __restrict__ inv,
                                                     const T* __restrict__ b, T* __restrict__ x,
                                                     const int* done) {
  if (done && *done) return;
  const int row = blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (row >= nv) return;
  const double* m = inv + (size_t)row * nd;
  double s0 = 0.0, s1 = 0.0;
  // nd is even and rows are 16-byte aligned: lane k reads entries 2k, 2k + 1 of each 128-wide chunk
#pragma unroll 4
  for (int k = 2 * lane; k < nv; k += 128) {
    const double2 mv = *reinterpret_cast<const double2*>(m + k);
    s0 += mv.x * (double)b[k];
    if (k + 1 < nv) s1 += mv.y * (double)b[k + 1];
  }
  double s = wave_sum(s0 + s1);
  if (lane == 0) x[row] = (T)s;
}

// The coarsest solve with its neighbours fused, one workgroup of 16 waves per
// coarsest node (wave w computes row w of the node): b is first summed from
// the finer level's restriction partials (each workgroup forms all of it in
// LDS; workgroup 0 also stores it), x = inv b, then x is prolonged into the
// finer level (pro.x set). nv <= 4096.
__global__ __launch_bounds__(1024) void k_coarse_solve_fused(int n, int nd, const double* __restrict__ inv,
                                                             double* __restrict__ b,
                                                             const int32_t* __restrict__ agg_ptr,
                                                             const double* __restrict__ part, double* __restrict__ x,
                                                             ProlongTo<double> pro, const int* done) {
  if (done && *done) return;
  __shared__ double bs[4096];
  __shared__ double xs[NS];
  const int nv = n * NS;
  const int a = blockIdx.x;
  for (int g = threadIdx.x; g < nv; g += 1024) {
    double v;
    if (part) {
      const int c = g / NS, m = g % NS;
      v = 0.0;
      for (int q = agg_ptr[c]; q < agg_ptr[c + 1]; ++q) v += part[(size_t)q * NS + m];
      if (a == 0) b[g] = v;
    } else {
      v = b[g];
    }
    bs[g] = v;
  }
  __syncthreads();
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int row = a * NS + w;
  const double* m = inv + (size_t)row * nd;
  double s0 = 0.0, s1 = 0.0;
#pragma unroll 4
  for (int k = 2 * lane; k < nv; k += 128) {
    const double2 mv = *reinterpret_cast<const double2*>(m + k);
    s0 += mv.x * bs[k];
    if (k + 1 < nv) s1 += mv.y * bs[k + 1];
  }
  const double sum = wave_sum(s0 + s1);
  if (lane == 0) {
    x[row] = sum;
    xs[w] = sum;
  }
  if (!pro.x) return;
  __syncthreads();
  if (w == 0) prolong_members(pro, a, lane < NS ? xs[lane] : 0.0);
}

// Lanczos start vector on dof i of a level: (splitmix64(seed ^ i) >> 11) 2^-53 - 1/2,
// seed = 0x9E3779B97F4A7C15 ^ level (splitmix64: Steele, Lea and Flood 2014).
__device__ __forceinline__ uint64_t splitmix64(uint64_t x) {
  uint64_t z = x + 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

__global__ void k_lanczos_start(int n, int level, double* __restrict__ v) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const uint64_t seed = 0x9E3779B97F4A7C15ull ^ (uint64_t)level;
  v[i] = (double)(splitmix64(seed ^ (uint64_t)i) >> 11) * 0x1.0p-53 - 0.5;
}

// ---- generalized Lanczos on S x = lambda D x with device-resident scalars
// Scalar slots: alpha[j] = s[j], beta[j] = s[32 + j], s[64] = norm^2,
// s[65] = b2, s[66] = completed steps, s[67] = stop flag, s[68] = lambda_max,
// s[69] = 1 / lambda_max.
constexpr int LZ_ALPHA = 0, LZ_BETA = 32, LZ_NRM = 64, LZ_B2 = 65, LZ_COUNT = 66, LZ_STOP = 67, LZ_LMAX = 68,
              LZ_ILMAX = 69, LZ_SIZE = 72;

// v <- v / sqrt(s[64]), u <- u / sqrt(s[64])
__global__ void k_lanczos_normalize(int n, double* __restrict__ v, double* __restrict__ u,
                                    const double* __restrict__ lz) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double sc = 1.0 / sqrt(lz[LZ_NRM]);
  v[i] *= sc;
  u[i] *= sc;
}

// w = D^-1 A v - alpha_j v - beta_j v_prev ;  Dw = A v - alpha_j u - beta_j u_prev
__global__ void k_lanczos_update(int n, int j, const double* __restrict__ dinv_av, const double* __restrict__ av,
                                 const double* __restrict__ v, const double* __restrict__ vp,
                                 const double* __restrict__ u, const double* __restrict__ up,
                                 const double* __restrict__ lz, double* __restrict__ w, double* __restrict__ dw) {
  if (lz[LZ_STOP] != 0.0) return;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double alpha = lz[LZ_ALPHA + j], beta = j > 0 ? lz[LZ_BETA + j - 1] : 0.0;
  w[i] = dinv_av[i] - alpha * v[i] - beta * vp[i];
  dw[i] = av[i] - alpha * u[i] - beta * up[i];
}

// After step j (unless stopped): (v_prev, u_prev, v, u) <- (v, u, w / beta_j, Dw / beta_j).
__global__ void k_lanczos_advance(int n, int j, double* __restrict__ v, double* __restrict__ vp,
                                  double* __restrict__ u, double* __restrict__ up, const double* __restrict__ w,
                                  const double* __restrict__ dw, const double* __restrict__ lz) {
  if (lz[LZ_STOP] != 0.0) return;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double ib = 1.0 / lz[LZ_BETA + j];
  vp[i] = v[i];
  up[i] = u[i];
  v[i] = w[i] * ib;
  u[i] = dw[i] * ib;
}

// lambda_max of the Lanczos tridiagonal matrix (alpha on the diagonal, beta
// beside it; the steps completed before a breakdown, else `steps`): its
// largest eigenvalue by bisection on the Sturm sequence count, one thread.
// A start vector of non-positive D-norm (a smoother block that is not
// positive definite) sets ERRF_NOT_SPD.
__global__ void k_lanczos_finish(int steps, double* __restrict__ lz, uint32_t* err) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  const double nrm = lz[LZ_NRM];
  if (!(nrm > 0.0) || !isfinite(nrm)) {
    atomicOr(err, ERRF_NOT_SPD);
    lz[LZ_LMAX] = 1.0;
    lz[LZ_ILMAX] = 1.0;
    return;
  }
  const int n = lz[LZ_STOP] != 0.0 ? (int)lz[LZ_COUNT] : steps;
  const double* a = lz + LZ_ALPHA;
  const double* b = lz + LZ_BETA;
  double lo = 1e300, hi = -1e300;
  for (int i = 0; i < n; ++i) {
    const double r = (i > 0 ? fabs(b[i - 1]) : 0.0) + (i + 1 < n ? fabs(b[i]) : 0.0);
    lo = fmin(lo, a[i] - r);
    hi = fmax(hi, a[i] + r);
  }
  for (int it = 0; it < 200; ++it) {
    const double mid = 0.5 * (lo + hi);
    if (mid <= lo || mid >= hi) break;
    int below = 0;   // eigenvalues < mid
    double d = 1.0;
    for (int i = 0; i < n; ++i) {
      d = a[i] - mid - (i > 0 ? b[i - 1] * b[i - 1] / d : 0.0);
      if (d == 0.0) d = -1e-300;
      if (d < 0.0) ++below;
    }
    if (below < n) lo = mid; else hi = mid;
  }
  const double lmax = 0.5 * (lo + hi);
  lz[LZ_LMAX] = lmax;
  lz[LZ_ILMAX] = 1.0 / lmax;
  if (!(lmax > 0.0) || !isfinite(lmax)) atomicOr(err, ERRF_NOT_SPD);
}

// Bookkeeping after step j (one thread): record alpha_j as done, and beta_j or the stop.
__global__ void k_lanczos_record(int j, double* __restrict__ lz) {
  if (lz[LZ_STOP] != 0.0) return;
  lz[LZ_COUNT] = (double)(j + 1);
  const double b2 = lz[LZ_B2], alpha = lz[LZ_ALPHA + j];
  if (!(b2 > 1e-300) || sqrt(b2) <= 1e-14 * fabs(alpha)) lz[LZ_STOP] = 1.0;
  else lz[LZ_BETA + j] = sqrt(b2);
}

}  // namespace bamg
