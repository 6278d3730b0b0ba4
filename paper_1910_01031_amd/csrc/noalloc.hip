// Residual resampling that allocates nothing (iewpf_resample_noalloc, declared in iewpf.h).
//
// The resampling kernels need per-particle partial results (the floor counts and the
// cumulative residuals).  Here they live in one file-scope device array, `scratch`, instead of
// a context's workspaces: each GPU the library runs on holds its own copy until the process
// ends.  Its device address is looked up once per device (with that device current) and kept;
// host code passes that address to the kernels, never the array's name (which on the host is
// only a stand-in for the symbol).  Every call on a GPU shares that GPU's array, so calls that
// overlap in time on one GPU race; each call writes every entry it reads before reading it, so
// nothing has to be cleared between calls.
#include <hip/hip_runtime.h>

#include <mutex>
#include <string>

#include "internal.hpp"

namespace iewpf {
namespace {

constexpr int kNoAllocMaxParticles = 65535;
// counts int32 [max] then cumulative residuals float64 [max], each part 256-byte aligned
constexpr size_t kCountsBytes = ((sizeof(int32_t) * kNoAllocMaxParticles + 255) / 256) * 256;
constexpr size_t kScratchBytes = kCountsBytes + sizeof(double) * kNoAllocMaxParticles;

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void* g_scratch[kMaxDevices] = {};

// Device address of `scratch` on the current device (looked up on the first call there).
int scratch_address(void** out) {
  int dev = -1;
  const hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return fail(IEWPF_E_HIP, std::string("hipGetDevice: ") + hipGetErrorString(e));
  if (dev < 0 || dev >= kMaxDevices) return fail(IEWPF_E_HIP, "device index beyond the scratch table");
  std::lock_guard<std::mutex> lock(g_mu);
  if (!g_scratch[dev]) {
    void* p = nullptr;
    const hipError_t es = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (es != hipSuccess || !p)
      return fail(IEWPF_E_HIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(es));
    g_scratch[dev] = p;
  }
  *out = g_scratch[dev];
  return 0;
}

}  // namespace
}  // namespace iewpf

using namespace iewpf;

extern "C" int iewpf_resample_noalloc(int n_particles, size_t floats_per_particle, uint64_t seed,
                                      uint32_t ensemble_id, uint64_t analysis_index,
                                      const double* logw, const float* state_in, float* state_out,
                                      int32_t* parents, void* stream) {
  if (!logw || !state_in || !state_out || !parents || n_particles < 1)
    return fail(IEWPF_E_ARG, "invalid argument");
  if (n_particles > kNoAllocMaxParticles)
    return fail(IEWPF_E_CAPACITY, "more than " + std::to_string(kNoAllocMaxParticles) +
                                      " particles (the size of the resampling scratch array)");
  if (floats_per_particle == 0 || floats_per_particle % 4 != 0)
    return fail(IEWPF_E_SHAPE, "floats per particle must be a positive multiple of 4");
  const size_t bytes = sizeof(float) * floats_per_particle * (size_t)n_particles;
  const char* a = reinterpret_cast<const char*>(state_in);
  const char* b = reinterpret_cast<const char*>(state_out);
  if (a < b + bytes && b < a + bytes) return fail(IEWPF_E_ARG, "state_in and state_out overlap");
  void* base = nullptr;
  if (int rc = scratch_address(&base)) return rc;
  unsigned char* sp = static_cast<unsigned char*>(base);
  int32_t* counts = reinterpret_cast<int32_t*>(sp);
  double* cum = reinterpret_cast<double*>(sp + kCountsBytes);
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  launch_resample(n_particles, seed, analysis_index, ensemble_id, logw, parents, counts, cum, s);
  launch_gather_particles(n_particles, floats_per_particle, parents, state_in, state_out, s);
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(IEWPF_E_HIP, std::string("resample launch: ") + hipGetErrorString(e));
  return 0;
}
