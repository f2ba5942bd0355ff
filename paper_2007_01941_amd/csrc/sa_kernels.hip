// Smoothed aggregation: the prolongator P_s = (I - w D^-1 S) P_t and the
// coarse operator P_s^T S P_s, the alternative to the unsmoothed prolongator
// that Section 3.5 and the scaling experiment of Section 5.2 compare against.
// Every sum runs over plan-time gather lists in a fixed order (no atomics).
//
// Blocks: S entries BS x BS, P_t / P_s / T entries BS x NS, coarse entries
// NS x NS, all row-major FP64.
#include "kernels.hpp"

namespace bamg {

constexpr int SA_STAGE = 4;   // source pairs staged in LDS per round

// out[e] = sum over g in [ptr[e], ptr[e+1]) of S[op[g]] B[b(g)], where b(g) is
// src[op[g]] (SMOOTH: B = P_t indexed by the operator entry's column node) or
// src[g] (B = P_s indexed by entry). SMOOTH finishes the entry of P_s:
// out[e] = [self[e]] P_t[row[e]] - c Dinv[row[e]] (the sum), c = w / lambda_max.
// One workgroup per output block; thread (r, m) keeps entry (r, m).
template <int BS, bool SMOOTH>
__global__ __launch_bounds__(256) void k_sa_product(const int32_t* __restrict__ ptr, const int32_t* __restrict__ op,
                                                    const int32_t* __restrict__ src, const double* __restrict__ S,
                                                    const double* __restrict__ B, const int32_t* __restrict__ row,
                                                    const int32_t* __restrict__ self, const double* __restrict__ Pt,
                                                    const double* __restrict__ Dinv, double c,
                                                    double* __restrict__ out) {
  __shared__ double As[SA_STAGE][BS * BS], Bs[SA_STAGE][BS * NS];
  const int e = blockIdx.x;
  const int tid = threadIdx.x;
  const int r = tid / NS, m = tid % NS;
  const int g0 = ptr[e], g1 = ptr[e + 1];
  double acc = 0.0;
  for (int g = g0; g < g1; g += SA_STAGE) {
    const int nb = min(SA_STAGE, g1 - g);
    for (int k = tid; k < nb * BS * BS; k += 256) {
      const int q = k / (BS * BS), w = k % (BS * BS);
      As[q][w] = S[(size_t)op[g + q] * BS * BS + w];
    }
    for (int k = tid; k < nb * BS * NS; k += 256) {
      const int q = k / (BS * NS), w = k % (BS * NS);
      const int b = SMOOTH ? src[op[g + q]] : src[g + q];
      Bs[q][w] = B[(size_t)b * BS * NS + w];
    }
    __syncthreads();
    if (r < BS) {
      for (int q = 0; q < nb; ++q) {
#pragma unroll
        for (int k = 0; k < BS; ++k) acc += As[q][r * BS + k] * Bs[q][k * NS + m];
      }
    }
    __syncthreads();
  }
  if (!SMOOTH) {
    if (r < BS) out[(size_t)e * BS * NS + tid] = acc;
    return;
  }
  const int i = row[e];
  if (r < BS) Bs[0][tid] = acc;
  for (int k = tid; k < BS * BS; k += 256) As[0][k] = Dinv[(size_t)i * BS * BS + k];
  __syncthreads();
  if (r < BS) {
    double d = 0.0;
#pragma unroll
    for (int k = 0; k < BS; ++k) d += As[0][r * BS + k] * Bs[0][k * NS + m];
    const double p = self[e] ? Pt[(size_t)i * BS * NS + tid] : 0.0;
    out[(size_t)e * BS * NS + tid] = p - c * d;
  }
}

// Coarse operator entry c = sum over g in [ptr[c], ptr[c+1]) of
// Ps[ps[g]]^T T[t[g]] (NS x NS), T = S P_s.
template <int BS>
__global__ __launch_bounds__(256) void k_sa_galerkin(const int32_t* __restrict__ ptr, const int32_t* __restrict__ ps,
                                                     const int32_t* __restrict__ t, const double* __restrict__ Ps,
                                                     const double* __restrict__ T, double* __restrict__ Sc) {
  __shared__ double Xs[SA_STAGE][BS * NS], Ys[SA_STAGE][BS * NS];
  const int c = blockIdx.x;
  const int tid = threadIdx.x;
  const int r = tid / NS, m = tid % NS;
  const int g0 = ptr[c], g1 = ptr[c + 1];
  double acc = 0.0;
  for (int g = g0; g < g1; g += SA_STAGE) {
    const int nb = min(SA_STAGE, g1 - g);
    for (int k = tid; k < nb * BS * NS; k += 256) {
      const int q = k / (BS * NS), w = k % (BS * NS);
      Xs[q][w] = Ps[(size_t)ps[g + q] * BS * NS + w];
      Ys[q][w] = T[(size_t)t[g + q] * BS * NS + w];
    }
    __syncthreads();
    for (int q = 0; q < nb; ++q) {
#pragma unroll
      for (int k = 0; k < BS; ++k) acc += Xs[q][k * NS + r] * Ys[q][k * NS + m];
    }
    __syncthreads();
  }
  Sc[(size_t)c * NS * NS + tid] = acc;
}

// Restriction with the smoothed prolongator: bc_a = sum over the entries e of
// aggregate a's column (rows ascending) of P_s[e]^T (r - t)_row(e) (t may be
// null). One thread per coarse dof.
template <int BS>
__global__ __launch_bounds__(256) void k_sa_restrict(int n_agg, const int32_t* __restrict__ colptr,
                                                     const int32_t* __restrict__ col_e,
                                                     const int32_t* __restrict__ ps_row,
                                                     const double* __restrict__ Ps, const double* __restrict__ r,
                                                     const double* __restrict__ t, double* __restrict__ bc,
                                                     const int* done) {
  if (done && *done) return;
  const int g = blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= n_agg * NS) return;
  const int a = g / NS, m = g % NS;
  double s = 0.0;
  for (int q = colptr[a]; q < colptr[a + 1]; ++q) {
    const int e = col_e[q];
    const int i = ps_row[e];
    const double* Pe = Ps + (size_t)e * BS * NS + m;
    const double* ri = r + (size_t)i * BS;
    if (t) {
      const double* ti = t + (size_t)i * BS;
#pragma unroll
      for (int k = 0; k < BS; ++k) s += Pe[k * NS] * (ri[k] - ti[k]);
    } else {
#pragma unroll
      for (int k = 0; k < BS; ++k) s += Pe[k * NS] * ri[k];
    }
  }
  bc[g] = s;
}

// Prolongation x_i += sum over the row's entries e of P_s[e] xc[col(e)], one
// thread per fine dof.
template <int BS>
__global__ __launch_bounds__(256) void k_sa_prolong(int n, const int32_t* __restrict__ rowptr,
                                                    const int32_t* __restrict__ ps_col,
                                                    const double* __restrict__ Ps, const double* __restrict__ xc,
                                                    double* __restrict__ x, const int* done) {
  if (done && *done) return;
  const int g = blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= n * BS) return;
  const int i = g / BS, k = g % BS;
  double s = 0.0;
  for (int e = rowptr[i]; e < rowptr[i + 1]; ++e) {
    const double* Pe = Ps + (size_t)e * BS * NS + k * NS;
    const double* xv = xc + (size_t)ps_col[e] * NS;
#pragma unroll
    for (int m2 = 0; m2 < NS; ++m2) s += Pe[m2] * xv[m2];
  }
  x[g] += s;
}

// Scatter of the smoothed prolongator's blocks into a dense
// [n bs][n_agg NS] matrix (zeroed beforehand).
__global__ __launch_bounds__(256) void k_sa_to_dense(int64_t nnz, int bs, int ncols,
                                                     const int32_t* __restrict__ ps_row,
                                                     const int32_t* __restrict__ ps_col,
                                                     const double* __restrict__ Ps, double* __restrict__ out) {
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= nnz * bs * NS) return;
  const int64_t e = g / (bs * NS);
  const int w = (int)(g % (bs * NS));
  const int r = w / NS, m = w % NS;
  out[((int64_t)ps_row[e] * bs + r) * ncols + (int64_t)ps_col[e] * NS + m] = Ps[g];
}

}  // namespace bamg
