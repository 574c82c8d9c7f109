// Device memory bandwidth probe: the reference points the streaming kernels
// are measured against.  One 256 x 16-byte chunk per workgroup, nontemporal
// loads and stores (the forms the transform passes use), best of several
// timed launches.
#include <cfloat>

#include "host.h"

namespace rdm {

namespace {

typedef float f4 __attribute__((ext_vector_type(4)));
constexpr int kProbeThreads = 256;

__device__ __forceinline__ f4 ld(const f4* p) { return __builtin_nontemporal_load(p); }
__device__ __forceinline__ void st(f4 v, f4* p) { __builtin_nontemporal_store(v, p); }

// pattern 0: read a (one value per workgroup is written, only if the sum hits
// an impossible value, so the loads are not removed)
// 1: b = a; 2: d = 1.5 a + b - 0.5 c; 3: c = a - 0.25 b, d = a + b
template <int PATTERN>
__global__ __launch_bounds__(kProbeThreads) void k_probe(const f4* __restrict__ a, const f4* __restrict__ b,
                                                         f4* __restrict__ c, f4* __restrict__ d) {
  const size_t o = (size_t)blockIdx.x * kProbeThreads + threadIdx.x;
  if (PATTERN == 0) {
    const f4 x = ld(a + o);
    if (x.x + x.y + x.z + x.w == -FLT_MAX) c[blockIdx.x] = x;
  } else if (PATTERN == 1) {
    st(ld(a + o), c + o);
  } else if (PATTERN == 2) {
    const f4 x = ld(a + o), y = ld(b + o), z = ld(c + o);
    st(x * 1.5f + y - z * 0.5f, d + o);
  } else {
    const f4 x = ld(a + o), y = ld(b + o);
    st(x - y * 0.25f, c + o);
    st(x + y, d + o);
  }
}

}  // namespace

}  // namespace rdm

using namespace rdm;

extern "C" rdm_status rdm_stream_probe(int32_t pattern, uint64_t bytes, int32_t reps, void* hip_stream,
                                       double* gbs) {
  const uint64_t chunk = (uint64_t)kProbeThreads * sizeof(f4);
  if (pattern < 0 || pattern > 3 || reps < 1 || !gbs || bytes < chunk || bytes % chunk != 0 ||
      bytes / chunk > 0x7fffffffull) {
    set_error("rdm_stream_probe: pattern 0..3, reps >= 1, bytes a positive multiple of 4096");
    return RDM_E_INVALID;
  }
  hipStream_t s = (hipStream_t)hip_stream;
  f4* buf[4] = {nullptr, nullptr, nullptr, nullptr};
  const int narr = pattern == 0 ? 2 : pattern == 1 ? 2 : 4;
  for (int i = 0; i < narr; ++i) {
    if (hipMalloc(&buf[i], bytes) != hipSuccess) {
      for (int q = 0; q < i; ++q) (void)hipFree(buf[q]);
      set_error("rdm_stream_probe: cannot allocate the arrays");
      return RDM_E_NOMEM;
    }
  }
  hipEvent_t e0 = nullptr, e1 = nullptr;
  hipError_t err = hipEventCreate(&e0);
  if (err == hipSuccess) err = hipEventCreate(&e1);
  for (int i = 0; i < narr && err == hipSuccess; ++i) err = hipMemsetAsync(buf[i], 0, bytes, s);
  const unsigned grid = (unsigned)(bytes / chunk);
  auto launch = [&]() {
    switch (pattern) {
      case 0: hipLaunchKernelGGL(k_probe<0>, dim3(grid), dim3(kProbeThreads), 0, s, buf[0], buf[0], buf[1], buf[1]); break;
      case 1: hipLaunchKernelGGL(k_probe<1>, dim3(grid), dim3(kProbeThreads), 0, s, buf[0], buf[0], buf[1], buf[1]); break;
      case 2: hipLaunchKernelGGL(k_probe<2>, dim3(grid), dim3(kProbeThreads), 0, s, buf[0], buf[1], buf[2], buf[3]); break;
      default: hipLaunchKernelGGL(k_probe<3>, dim3(grid), dim3(kProbeThreads), 0, s, buf[0], buf[1], buf[2], buf[3]); break;
    }
    return hipGetLastError();
  };
  float best = 1e30f;
  if (err == hipSuccess) err = launch();  // warm-up
  for (int r = 0; r < reps && err == hipSuccess; ++r) {
    err = hipEventRecord(e0, s);
    if (err == hipSuccess) err = launch();
    if (err == hipSuccess) err = hipEventRecord(e1, s);
    if (err == hipSuccess) err = hipEventSynchronize(e1);
    float ms = 0.f;
    if (err == hipSuccess) err = hipEventElapsedTime(&ms, e0, e1);
    if (err == hipSuccess && ms < best) best = ms;
  }
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  for (int i = 0; i < narr; ++i) (void)hipFree(buf[i]);
  if (err != hipSuccess) {
    set_error(std::string("rdm_stream_probe: ") + hipGetErrorString(err));
    return RDM_E_DEVICE;
  }
  const double moved = (double)bytes * (pattern == 0 ? 1 : pattern == 1 ? 2 : 4);
  *gbs = moved / (best * 1e-3) / 1e9;
  return RDM_OK;
}
