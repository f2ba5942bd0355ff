// Shared definitions of the bamg library: status handling, device helpers,
// and the plan structure. Everything here is CDNA4 (gfx950) HIP.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <string>
#include <vector>

#include "../../include/bamg.h"
#include "../../include/bamg_selftest.h"

namespace bamg {

// ------------------------------------------------------------ errors

void set_error(const char* fmt, ...);

struct Fail {
  ba_status st;
};

#define BA_HIP(call)                                                              \
  do {                                                                            \
    hipError_t e_ = (call);                                                       \
    if (e_ != hipSuccess) {                                                       \
      ::bamg::set_error("%s:%d %s -> %s", __FILE__, __LINE__, #call,              \
                        hipGetErrorString(e_));                                   \
      throw ::bamg::Fail{BA_ERR_HIP};                                             \
    }                                                                             \
  } while (0)

#define BA_CHECK(cond, status, ...)                                               \
  do {                                                                            \
    if (!(cond)) {                                                                \
      ::bamg::set_error(__VA_ARGS__);                                             \
      throw ::bamg::Fail{status};                                                 \
    }                                                                             \
  } while (0)

#define BA_LAUNCH_CHECK() BA_HIP(hipGetLastError())

// Device-side error flags (bit set in a device word, read back by the host).
enum : uint32_t {
  ERRF_GEOMETRY = 1u,     // point at or behind a camera
  ERRF_NONFINITE = 2u,    // non-finite input or intermediate
  ERRF_NOT_SPD = 4u,      // a block Cholesky pivot <= 0
  ERRF_BREAKDOWN = 8u,    // PCG breakdown
  ERRF_LIMIT = 16u,       // a kernel capacity was exceeded
};

// ------------------------------------------------------------ device memory

// Where a plan's persistent device memory comes from: the caller's callbacks
// (ba_plan_create), or hipMalloc / hipFree when they are NULL.
struct Allocator {
  ba_alloc_fn alloc = nullptr;
  ba_free_fn release = nullptr;
  void* ctx = nullptr;
};

// The allocator of the plan the calling thread is working on (set for the
// duration of an API call by AllocScope); nullptr means hipMalloc.
extern thread_local const Allocator* tl_alloc;

struct AllocScope {
  const Allocator* prev;
  explicit AllocScope(const Allocator* a) : prev(tl_alloc) { tl_alloc = a; }
  ~AllocScope() { tl_alloc = prev; }
};

void* dev_alloc(size_t bytes);
void dev_free(void* p, const Allocator* a);

// A device buffer of the plan: either owned (allocated through the plan's
// allocator, freed with it) or a view into a workspace (never freed here).
template <class T>
struct DBuf {
  T* p = nullptr;
  size_t n = 0;
  const Allocator* al = nullptr;
  bool own = false;
  void alloc(size_t count) {
    free();
    if (count) {
      p = static_cast<T*>(dev_alloc(count * sizeof(T)));
      al = tl_alloc;
      own = true;
    }
    n = count;
  }
  void view(T* ptr, size_t count) {
    free();
    p = count ? ptr : nullptr;
    n = count;
  }
  void free() {
    if (p && own) dev_free(p, al);
    p = nullptr;
    n = 0;
    own = false;
  }
  size_t bytes() const { return n * sizeof(T); }
  void upload(const std::vector<T>& h, hipStream_t s) {
    alloc(h.size());
    if (!h.empty()) BA_HIP(hipMemcpyAsync(p, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice, s));
  }
  std::vector<T> download(hipStream_t s) const {
    std::vector<T> h(n);
    if (n) {
      BA_HIP(hipMemcpyAsync(h.data(), p, n * sizeof(T), hipMemcpyDeviceToHost, s));
      BA_HIP(hipStreamSynchronize(s));
    }
    return h;
  }
  ~DBuf() { free(); }
  DBuf() = default;
  DBuf(const DBuf&) = delete;
  DBuf& operator=(const DBuf&) = delete;
  DBuf(DBuf&& o) noexcept : p(o.p), n(o.n), al(o.al), own(o.own) {
    o.p = nullptr;
    o.n = 0;
    o.own = false;
  }
  DBuf& operator=(DBuf&& o) noexcept {
    if (this != &o) {
      free();
      p = o.p;
      n = o.n;
      al = o.al;
      own = o.own;
      o.p = nullptr;
      o.n = 0;
      o.own = false;
    }
    return *this;
  }
};

// Carves the per-step buffers out of one workspace: each take() places a
// buffer at the next 256-byte boundary. With base == nullptr it only counts
// the bytes (ba_workspace_bytes).
struct Carve {
  char* base = nullptr;
  size_t off = 0;
  template <class T>
  void take(DBuf<T>& b, size_t count) {
    off = (off + 255) / 256 * 256;
    if (base) b.view(reinterpret_cast<T*>(base + off), count);
    off += count * sizeof(T);
  }
};

// ------------------------------------------------------------ small helpers

// Packed symmetric storage of an n x n matrix: upper triangle row by row.
__host__ __device__ constexpr int sym_index(int n, int i, int j) {
  // requires i <= j
  return i * n - i * (i - 1) / 2 + (j - i);
}

inline int ceil_div(int64_t a, int64_t b) { return (int)((a + b - 1) / b); }

// Tile geometry of the point-major observation layout.
constexpr int TILE_OBS = 256;     // observations per tile (one per thread)
constexpr int S0_CHUNK = 128;    // shared points per wave in the explicit level-0 S
constexpr int PREC = 16;         // doubles per point record (X 3, C^-1 6, C^-1 g_p 3, padding)
constexpr int GROUP_SLOTS = 96;   // cameras of a tile group kept in LDS (others go to global memory)
constexpr int GROUP_TILES = 8;    // most tiles in one group of the Schur product

// Block size of the MG levels above level 0 (16 near-nullspace columns, Section 3.3).
constexpr int NS = 16;

}  // namespace bamg
