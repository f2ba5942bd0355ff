// Multigrid plan kernels: covisibility counts, strength ordering and greedy
// aggregation (Section 3.2 and Algorithm 2 of Konolige and Brown).
//
// W = V V^T counts the points two cameras share (W_ii = points seen by i).
// The strength of connection is G_ij = W_ij / sqrt(W_ii W_jj) (the visibility
// cosine). Neighbours of one row are only ever compared with each other, and
// G_ij > G_ik exactly when W_ij^2 W_kk > W_ik^2 W_jj, so the order is decided
// in 128-bit integers without rounding (the plan bounds every count by 2^42,
// so the products stay below 2^126). On coarse levels an
// aggregate's visibility vector is the sum of its members', so
// W_{l+1} = Ahat^T W_l Ahat with Ahat the 0/1 aggregate matrix.
#include "kernels.hpp"

namespace bamg {

constexpr int HASH_SLOTS = 8192;     // LDS hash table of one covisibility row
constexpr int ROW_SORT_MAX = 4096;   // longest covisibility row the row sort handles

__device__ __forceinline__ uint32_t hash_key(int k) { return ((uint32_t)k * 2654435761u) >> 19; }

// Add `w` to the entry `key` of an LDS hash table (open addressing).
__device__ __forceinline__ void hash_add(int* keys, unsigned long long* vals, int* n_used, int key,
                                         unsigned long long w, uint32_t* err) {
  uint32_t h = hash_key(key) & (HASH_SLOTS - 1);
  for (int probe = 0; probe < HASH_SLOTS; ++probe) {
    int k = keys[h];
    if (k == -1) {
      const int old = atomicCAS(&keys[h], -1, key);
      if (old == -1) {
        atomicAdd(n_used, 1);
        atomicAdd(&vals[h], w);
        return;
      }
      k = old;
    }
    if (k == key) {
      atomicAdd(&vals[h], w);
      return;
    }
    h = (h + 1) & (HASH_SLOTS - 1);
  }
  atomicOr(err, ERRF_LIMIT);
}

__device__ __forceinline__ void hash_clear(int* keys, unsigned long long* vals, int* n_used) {
  for (int i = threadIdx.x; i < HASH_SLOTS; i += blockDim.x) { keys[i] = -1; vals[i] = 0ull; }
  if (threadIdx.x == 0) *n_used = 0;
  __syncthreads();
}

// Finish one hash row: PASS 0 writes the number of distinct columns and W_ii;
// PASS 1 writes the (unsorted) entries at rowptr[row].
template <int PASS>
__device__ __forceinline__ void hash_emit(int row, const int* keys, const unsigned long long* vals,
                                          int* n_used, int32_t* row_nnz, int64_t* wdiag,
                                          const int64_t* rowptr, int32_t* col, int64_t* val,
                                          uint32_t* err) {
  __syncthreads();
  if (PASS == 0) {
    if (threadIdx.x == 0) {
      row_nnz[row] = *n_used;
      if (*n_used > HASH_SLOTS * 3 / 4) atomicOr(err, ERRF_LIMIT);
    }
    for (int i = threadIdx.x; i < HASH_SLOTS; i += blockDim.x)
      if (keys[i] == row) wdiag[row] = (int64_t)vals[i];
  } else {
    __shared__ int cursor;
    if (threadIdx.x == 0) cursor = 0;
    __syncthreads();
    const int64_t base = rowptr[row];
    for (int i = threadIdx.x; i < HASH_SLOTS; i += blockDim.x) {
      if (keys[i] != -1) {
        const int pos = atomicAdd(&cursor, 1);
        col[base + pos] = keys[i];
        val[base + pos] = (int64_t)vals[i];
      }
    }
  }
}

// Level 0: row i of W from the points camera i sees and their observers.
template <int PASS>
__global__ __launch_bounds__(256) void k_covis0(const int32_t* __restrict__ cam_off,
                                                const int32_t* __restrict__ cam_obs,
                                                const int32_t* __restrict__ obs_pt,
                                                const int32_t* __restrict__ pt_off,
                                                const int32_t* __restrict__ obs_cam,
                                                int32_t* row_nnz, int64_t* wdiag,
                                                const int64_t* rowptr, int32_t* col, int64_t* val,
                                                uint32_t* err) {
  __shared__ int keys[HASH_SLOTS];
  __shared__ unsigned long long vals[HASH_SLOTS];
  __shared__ int n_used;
  const int row = blockIdx.x;
  hash_clear(keys, vals, &n_used);
  for (int i = cam_off[row] + threadIdx.x; i < cam_off[row + 1]; i += blockDim.x) {
    const int q = obs_pt[cam_obs[i]];
    for (int o = pt_off[q]; o < pt_off[q + 1]; ++o) hash_add(keys, vals, &n_used, obs_cam[o], 1ull, err);
  }
  hash_emit<PASS>(row, keys, vals, &n_used, row_nnz, wdiag, rowptr, col, val, err);
}

// Level l+1: row A of Ahat^T W Ahat from the rows of A's members.
template <int PASS>
__global__ __launch_bounds__(256) void k_covisL(const int32_t* __restrict__ agg_ptr,
                                                const int32_t* __restrict__ agg_mem,
                                                const int64_t* __restrict__ f_rowptr,
                                                const int32_t* __restrict__ f_col,
                                                const int64_t* __restrict__ f_val,
                                                const int32_t* __restrict__ f_agg,
                                                int32_t* row_nnz, int64_t* wdiag,
                                                const int64_t* rowptr, int32_t* col, int64_t* val,
                                                uint32_t* err) {
  __shared__ int keys[HASH_SLOTS];
  __shared__ unsigned long long vals[HASH_SLOTS];
  __shared__ int n_used;
  const int row = blockIdx.x;
  hash_clear(keys, vals, &n_used);
  for (int m = agg_ptr[row]; m < agg_ptr[row + 1]; ++m) {
    const int i = agg_mem[m];
    for (int64_t e = f_rowptr[i] + threadIdx.x; e < f_rowptr[i + 1]; e += blockDim.x)
      hash_add(keys, vals, &n_used, f_agg[f_col[e]], (unsigned long long)f_val[e], err);
  }
  hash_emit<PASS>(row, keys, vals, &n_used, row_nnz, wdiag, rowptr, col, val, err);
}

// True when neighbour a (count wa = W_ia, diagonal da = W_aa) comes after
// neighbour b in row i's order: weaker strength, or equal strength and a
// higher column. Strengths compare as W_ia^2 W_bb against W_ib^2 W_aa.
__device__ __forceinline__ bool weaker(long long wa, long long da, int ca, long long wb, long long db,
                                       int cb) {
  const unsigned __int128 lhs = (unsigned __int128)(uint64_t)wa * (uint64_t)wa * (uint64_t)db;
  const unsigned __int128 rhs = (unsigned __int128)(uint64_t)wb * (uint64_t)wb * (uint64_t)da;
  return lhs < rhs || (lhs == rhs && ca > cb);
}

// Sort one row by column (carrying the counts), then write its neighbours
// (diagonal excluded) by decreasing strength, equal strengths by column.
__global__ __launch_bounds__(256) void k_row_sort(const int64_t* __restrict__ rowptr, int32_t* col,
                                                  int64_t* val, const int64_t* __restrict__ wdiag,
                                                  int32_t* order, uint32_t* err) {
  __shared__ int c_s[ROW_SORT_MAX];
  __shared__ long long v_s[ROW_SORT_MAX];
  __shared__ long long d_s[ROW_SORT_MAX];
  const int row = blockIdx.x;
  const int64_t beg = rowptr[row];
  const int len = (int)(rowptr[row + 1] - beg);
  if (len > ROW_SORT_MAX) {
    if (threadIdx.x == 0) atomicOr(err, ERRF_LIMIT);
    return;
  }
  int m = 1;
  while (m < len) m <<= 1;
  for (int i = threadIdx.x; i < m; i += blockDim.x) {
    if (i < len) { c_s[i] = col[beg + i]; v_s[i] = val[beg + i]; }
    else { c_s[i] = 0x7fffffff; v_s[i] = 0; }
  }
  __syncthreads();
  // bitonic sort by column ascending
  for (int k = 2; k <= m; k <<= 1)
    for (int j = k >> 1; j > 0; j >>= 1) {
      for (int i = threadIdx.x; i < m; i += blockDim.x) {
        const int l = i ^ j;
        if (l > i) {
          const bool up = (i & k) == 0;
          if ((c_s[i] > c_s[l]) == up) {
            const int tc = c_s[i]; c_s[i] = c_s[l]; c_s[l] = tc;
            const long long tv = v_s[i]; v_s[i] = v_s[l]; v_s[l] = tv;
          }
        }
      }
      __syncthreads();
    }
  for (int i = threadIdx.x; i < len; i += blockDim.x) { col[beg + i] = c_s[i]; val[beg + i] = v_s[i]; }
  __syncthreads();
  // the diagonal and the padding get strength 0 (count 0), below every
  // neighbour (counts >= 1); among them the diagonal's column comes first
  for (int i = threadIdx.x; i < m; i += blockDim.x) {
    if (i < len && c_s[i] != row) d_s[i] = wdiag[c_s[i]];
    else { v_s[i] = 0; d_s[i] = 1; }
  }
  __syncthreads();
  // bitonic sort by (strength descending, column ascending)
  for (int k = 2; k <= m; k <<= 1)
    for (int j = k >> 1; j > 0; j >>= 1) {
      for (int i = threadIdx.x; i < m; i += blockDim.x) {
        const int l = i ^ j;
        if (l > i) {
          const bool up = (i & k) == 0;
          if (weaker(v_s[i], d_s[i], c_s[i], v_s[l], d_s[l], c_s[l]) == up) {
            const int tc = c_s[i]; c_s[i] = c_s[l]; c_s[l] = tc;
            const long long tv = v_s[i]; v_s[i] = v_s[l]; v_s[l] = tv;
            const long long td = d_s[i]; d_s[i] = d_s[l]; d_s[l] = td;
          }
        }
      }
      __syncthreads();
    }
  const int64_t obeg = beg - row;   // one diagonal entry per earlier row
  for (int i = threadIdx.x; i < len - 1; i += blockDim.x) order[obeg + i] = c_s[i];
}

// Algorithm 2 on one level, by a single wave: nodes in index order; an
// unaggregated node i takes the first neighbour j (by decreasing strength)
// that is unaggregated (new aggregate {i, j}) or whose aggregate has fewer
// than `cap` nodes (i joins it). Nodes left over join the aggregate of their
// first neighbour; a node without neighbours becomes a singleton.
// agg/size point to LDS (dynamic shared memory) or to global scratch.
__device__ void aggregate_wave(int n, const int64_t* __restrict__ rowptr,
                               const int32_t* __restrict__ order, int cap, volatile int* agg,
                               volatile int* size, int* n_agg_out) {
  const int lane = threadIdx.x;
  for (int i = lane; i < n; i += 64) { agg[i] = -1; size[i] = 0; }
  __threadfence_block();
  int n_agg = 0;
  for (int i = 0; i < n; ++i) {
    if (agg[i] != -1) continue;
    const int64_t beg = rowptr[i] - i, end = rowptr[i + 1] - i - 1;
    for (int64_t base = beg; base < end; base += 64) {
      const int64_t idx = base + lane;
      int j = -1, a = -2;
      bool elig = false;
      if (idx < end) {
        j = order[idx];
        a = agg[j];
        elig = (a == -1) || (size[a] < cap);
      }
      const unsigned long long mask = __ballot(elig);
      if (mask) {
        const int first = __ffsll((long long)mask) - 1;
        const int jj = __shfl(j, first, 64);
        const int aa = __shfl(a, first, 64);
        if (lane == 0) {
          if (aa == -1) {
            agg[i] = n_agg;
            agg[jj] = n_agg;
            size[n_agg] = 2;
          } else {
            agg[i] = aa;
            size[aa] = size[aa] + 1;
          }
        }
        if (aa == -1) ++n_agg;
        __threadfence_block();
        break;
      }
    }
  }
  // leftovers, in ascending order; singletons numbered in that order
  for (int base = 0; base < n; base += 64) {
    const int i = base + lane;
    bool left = false, single = false;
    int target = -1;
    if (i < n && agg[i] == -1) {
      left = true;
      const int64_t beg = rowptr[i] - i, end = rowptr[i + 1] - i - 1;
      if (end > beg) target = agg[order[beg]];
      else single = true;
    }
    const unsigned long long smask = __ballot(single);
    if (single) {
      const unsigned long long below = lane ? (smask & ((1ull << lane) - 1ull)) : 0ull;
      target = n_agg + __popcll(below);
    }
    n_agg += __popcll(smask);
    __threadfence_block();
    if (left) agg[i] = target;
    __threadfence_block();
  }
  if (lane == 0) *n_agg_out = n_agg;
}

__global__ __launch_bounds__(64) void k_aggregate_lds(int n, const int64_t* __restrict__ rowptr,
                                                      const int32_t* __restrict__ order, int cap,
                                                      int32_t* agg_out, int32_t* n_agg_out) {
  extern __shared__ int smem[];
  int* agg = smem;
  int* size = smem + n;
  aggregate_wave(n, rowptr, order, cap, agg, size, n_agg_out);
  __syncthreads();
  for (int i = threadIdx.x; i < n; i += 64) agg_out[i] = agg[i];
}

__global__ __launch_bounds__(64) void k_aggregate_global(int n, const int64_t* __restrict__ rowptr,
                                                         const int32_t* __restrict__ order, int cap,
                                                         int32_t* agg, int32_t* size,
                                                         int32_t* n_agg_out) {
  aggregate_wave(n, rowptr, order, cap, agg, size, n_agg_out);
}

}  // namespace bamg
