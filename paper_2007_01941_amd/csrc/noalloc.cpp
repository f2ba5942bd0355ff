// ba_cost_noalloc: the cost of ba_cost for callers that cannot allocate device
// memory (code under HIP graph capture, tight serving loops, harnesses that
// forbid hipMalloc). Its kernels' scratch -- the camera records, the
// reduction partials and the scalar block with its counters -- lives in the
// file-scope device array below instead of a workspace: each GPU the library
// runs on holds one copy until the process ends, and every call on that GPU
// shares it, so calls that overlap on one GPU (different streams or threads)
// race. Host code never uses the array's name as an address: the address is
// taken per device with hipGetSymbolAddress on the first call there.
#include <mutex>

namespace bamg {

constexpr int NOALLOC_MAX_CAMS = 32768;   // cameras the scratch holds records for
constexpr size_t NOALLOC_CAM_BYTES = (size_t)NOALLOC_MAX_CAMS * 24 * sizeof(double);
constexpr size_t NOALLOC_PART_BYTES = (size_t)RED_BLOCKS * sizeof(double);
constexpr size_t NOALLOC_BYTES = NOALLOC_CAM_BYTES + NOALLOC_PART_BYTES + 256;   // + the scalar block

static __device__ __align__(256) unsigned char scratch[NOALLOC_BYTES];

static std::mutex g_noalloc_mu;
static void* g_noalloc_ptr[64] = {};   // address of `scratch` on each device

static unsigned char* noalloc_scratch() {
  int dev = 0;
  BA_HIP(hipGetDevice(&dev));
  BA_CHECK(dev >= 0 && dev < 64, BA_ERR_LIMIT, "device index %d beyond the library's table", dev);
  std::lock_guard<std::mutex> lock(g_noalloc_mu);
  if (!g_noalloc_ptr[dev]) {
    void* p = nullptr;
    BA_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    BA_CHECK(p, BA_ERR_HIP, "no address for the scratch array on device %d", dev);
    g_noalloc_ptr[dev] = p;
  }
  return static_cast<unsigned char*>(g_noalloc_ptr[dev]);
}

}  // namespace bamg

extern "C" ba_status ba_cost_noalloc(ba_plan* P, const ba_opts* o, const double* cams, const double* pts,
                                     const double* uv, double* cost, int64_t* n_invalid, void* stream) {
  BA_API_BEGIN
  BA_CHECK(P && cams && pts && uv && cost, BA_ERR_ARG, "null argument");
  if (o) validate_opts(o);
  BA_CHECK(P->n_cam <= NOALLOC_MAX_CAMS, BA_ERR_LIMIT,
           "ba_cost_noalloc holds camera records for at most %d cameras (plan has %d)", NOALLOC_MAX_CAMS,
           P->n_cam);
  hipStream_t s = (hipStream_t)stream;
  unsigned char* base = noalloc_scratch();
  double* camrec = reinterpret_cast<double*>(base);
  double* partial = reinterpret_cast<double*>(base + NOALLOC_CAM_BYTES);
  LmScal* scal = reinterpret_cast<LmScal*>(base + NOALLOC_CAM_BYTES + NOALLOC_PART_BYTES);
  const int loss = o ? o->loss : BA_LOSS_SQUARED;
  const double a = o ? o->loss_scale : 1.0;
  // the scalar block (flags and reduction counters) starts at zero on every call
  hipLaunchKernelGGL(k_lm_clear, dim3(1), dim3(64), 0, s, scal);
  hipLaunchKernelGGL(k_campre, dim3(ceil_div(P->n_cam, 256)), dim3(256), 0, s, P->n_cam, cams, camrec,
                     &scal->camflag);
  hipLaunchKernelGGL(k_lm_cost, dim3(red_grid((int)P->n_obs)), dim3(256), 0, s, (int)P->n_obs, P->obs_cam.p,
                     P->obs_pt.p, P->pt_orig.p, P->obs_orig.p, (const double*)camrec, pts, uv, loss, a, partial,
                     scal);
  BA_LAUNCH_CHECK();
  LmScal h{};
  BA_HIP(hipMemcpyAsync(&h, scal, sizeof(LmScal), hipMemcpyDeviceToHost, s));
  BA_HIP(hipStreamSynchronize(s));
  *cost = h.cost;
  if (n_invalid) *n_invalid = (int64_t)h.invalid;
  BA_API_END
}
