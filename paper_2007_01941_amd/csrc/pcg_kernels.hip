// Preconditioned conjugate gradients on the camera system (Saad, Iterative
// Methods for Sparse Linear Systems, Algorithm 9.1) with device-resident
// scalars. Dot products are reduced deterministically: every block writes a
// partial, and the last block to finish sums the partials in block order and
// updates the scalars. Kernels of an iteration return immediately once the
// `done` flag is set, so the host may enqueue several iterations between
// convergence checks.
#include "kernels.hpp"

namespace bamg {

struct PcgScal {
  double rz;      // r . z of the current iterate
  double alpha;
  double beta;
  double bb;      // b . b
  double rr;      // r . r after the latest update
  double pq;
  double q;       // quadratic model 1/2 x^T S x - x^T b of the current iterate
  double rtol2;   // stop when r . r <= rtol2 b . b
  double forcing; // Nash-Sofer tolerance (< 0: rule off)
  int done;       // converged or broke down
  int iters;      // completed iterations
  int flag;       // ERRF_BREAKDOWN on breakdown
  int maxit_hit;
  unsigned count[4];
};

constexpr int RED_BLOCKS = 256;   // grid size of the reduction kernels

enum DotMode { DOT_INIT = 0, DOT_ALPHA = 1, DOT_BETA = 2, DOT_PLAIN = 3 };

__device__ __forceinline__ double load_agent(const double* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Block-reduce v and return true in the last block, whose thread 0 then holds
// the ordered sum of all partials in *out.
__device__ __forceinline__ bool last_block_sum(double v, double* partial, unsigned* counter,
                                               double* out) {
  __shared__ double red[4];
  __shared__ int is_last;
  v = wave_sum(v);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  if (lane == 0) red[wid] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    partial[blockIdx.x] = red[0] + red[1] + red[2] + red[3];
    __threadfence();
    const unsigned prev = atomicAdd(counter, 1u);
    is_last = (prev == gridDim.x - 1);
  }
  __syncthreads();
  if (!is_last) return false;
  __threadfence();
  double s = threadIdx.x < gridDim.x ? load_agent(&partial[threadIdx.x]) : 0.0;
  s = wave_sum(s);
  __syncthreads();
  if (lane == 0) red[wid] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    *out = red[0] + red[1] + red[2] + red[3];
    *counter = 0u;
  }
  return threadIdx.x == 0;
}

// dot(a, b) with a finalize step selected by MODE.
template <int MODE, class T>
__global__ __launch_bounds__(256) void k_dot(int n, const T* __restrict__ a, const T* __restrict__ b,
                                             double* __restrict__ partial, PcgScal* s,
                                             double* plain_out) {
  if (MODE != DOT_INIT && MODE != DOT_PLAIN && s->done) return;
  double v = 0.0;
  for (int i = blockIdx.x * 256 + threadIdx.x; i < n; i += gridDim.x * 256) v += (double)a[i] * (double)b[i];
  double tot;
  if (!last_block_sum(v, partial, &s->count[MODE], &tot)) return;
  if (MODE == DOT_PLAIN) {
    *plain_out = tot;
  } else if (MODE == DOT_INIT) {
    s->rz = tot;
    s->beta = 0.0;
    s->iters = 0;
    s->flag = 0;
    s->done = (s->bb == 0.0) ? 1 : 0;
    if (!(tot > 0.0) && s->bb > 0.0) { s->flag = ERRF_BREAKDOWN; s->done = 1; }
  } else if (MODE == DOT_ALPHA) {
    s->pq = tot;
    if (!(tot > 0.0)) { s->flag = ERRF_BREAKDOWN; s->done = 1; }
    else s->alpha = s->rz / tot;
  } else {  // DOT_BETA
    if (!(tot > 0.0)) { s->flag = ERRF_BREAKDOWN; s->done = 1; }
    else { s->beta = tot / s->rz; s->rz = tot; }
  }
}

// b . b (and zero the iteration state; the stop tolerances go to the device
// scalars, so that an iteration's launches do not depend on them)
template <class T>
__global__ __launch_bounds__(256) void k_pcg_start(int n, const T* __restrict__ b, T* __restrict__ x,
                                                   T* __restrict__ r, T* __restrict__ p,
                                                   double* __restrict__ partial, PcgScal* s, double rtol2,
                                                   double forcing) {
  double v = 0.0;
  for (int i = blockIdx.x * 256 + threadIdx.x; i < n; i += gridDim.x * 256) {
    const T bi = b[i];
    x[i] = T(0);
    r[i] = bi;
    p[i] = T(0);
    v += (double)bi * (double)bi;
  }
  double tot;
  if (!last_block_sum(v, partial, &s->count[3], &tot)) return;
  s->bb = tot;
  s->rr = tot;
  s->q = 0.0;
  s->rtol2 = rtol2;
  s->forcing = forcing;
  s->done = 0;
  s->iters = 0;
  s->flag = 0;
}

// p = z + beta p;  q = A p (camera block diagonal), one thread per (camera, row).
template <class T>
__global__ __launch_bounds__(256) void k_pcg_p_Ap(int n_cam, const T* __restrict__ z, T* __restrict__ p,
                                                  const T* __restrict__ A, T* __restrict__ q,
                                                  const PcgScal* s) {
  if (s->done) return;
  __shared__ T ps[28 * 9];
  const int lc = threadIdx.x / 9, i = threadIdx.x % 9;
  const int c = blockIdx.x * 28 + lc;
  const bool act = threadIdx.x < 252 && c < n_cam;
  const T beta = (T)s->beta;
  if (act) {
    const size_t k = (size_t)c * 9 + i;
    const T v = z[k] + beta * p[k];
    p[k] = v;
    ps[lc * 9 + i] = v;
  }
  __syncthreads();
  if (!act) return;
  const T* a = A + (size_t)c * 45;
  T acc = 0;
#pragma unroll
  for (int j = 0; j < 9; ++j) acc += a[i <= j ? sym_index(9, i, j) : sym_index(9, j, i)] * ps[lc * 9 + j];
  q[(size_t)c * 9 + i] = acc;
}

// x += alpha p; r -= alpha q; convergence test on r . r. With forcing >= 0
// the Nash-Sofer rule of Section 2.1 also stops the iteration: the quadratic
// model falls by alpha_i r_{i-1}.z_{i-1} / 2 in iteration i (Q_0 = 0), and the
// solve ends once i (Q_i - Q_{i-1}) / Q_i <= forcing.
template <class T>
__global__ __launch_bounds__(256) void k_pcg_xr(int n, const T* __restrict__ p, const T* __restrict__ q,
                                                T* __restrict__ x, T* __restrict__ r,
                                                double* __restrict__ partial, PcgScal* s) {
  if (s->done) return;
  const T alpha = (T)s->alpha;
  double v = 0.0;
  for (int i = blockIdx.x * 256 + threadIdx.x; i < n; i += gridDim.x * 256) {
    x[i] += alpha * p[i];
    const T ri = r[i] - alpha * q[i];
    r[i] = ri;
    v += (double)ri * (double)ri;
  }
  double tot;
  if (!last_block_sum(v, partial, &s->count[2], &tot)) return;
  s->rr = tot;
  s->iters += 1;
  if (tot <= s->rtol2 * s->bb) {
    s->done = 1;
  } else if (s->forcing >= 0.0) {
    const double qn = s->q - 0.5 * s->alpha * s->rz;
    if ((double)s->iters * (qn - s->q) / qn <= s->forcing) s->done = 1;
    s->q = qn;
  }
}

// z = Sinv r (block Jacobi, 9x9 per camera); one thread per (camera, row).
template <class T>
__global__ __launch_bounds__(256) void k_bj_apply(int n_cam, const T* __restrict__ Sinv,
                                                  const T* __restrict__ r, T* __restrict__ z,
                                                  const int* done) {
  if (done && *done) return;
  __shared__ T rs[28 * 9];
  const int lc = threadIdx.x / 9, i = threadIdx.x % 9;
  const int c = blockIdx.x * 28 + lc;
  const bool act = threadIdx.x < 252 && c < n_cam;
  if (act) rs[lc * 9 + i] = r[(size_t)c * 9 + i];
  __syncthreads();
  if (!act) return;
  const T* m = Sinv + (size_t)c * 81 + i * 9;
  T acc = 0;
#pragma unroll
  for (int j = 0; j < 9; ++j) acc += m[j] * rs[lc * 9 + j];
  z[(size_t)c * 9 + i] = acc;
}

// ---- small vector kernels
template <class T, class U>
__global__ void k_convert(int n, const T* __restrict__ a, U* __restrict__ b) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) b[i] = (U)a[i];
}

// y = a + s * b  (FP64)
__global__ void k_axpby(int n, const double* __restrict__ a, double s, const double* __restrict__ b,
                        double* __restrict__ y) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) y[i] = a[i] + s * b[i];
}

// x += e (FP64 correction)
__global__ void k_add_f64(int n, const double* __restrict__ e, double* __restrict__ x) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) x[i] += e[i];
}

// x += (double) e (refinement update)
__global__ void k_add_f32(int n, const float* __restrict__ e, double* __restrict__ x) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) x[i] += (double)e[i];
}

}  // namespace bamg
