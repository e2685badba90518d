// grffe_check_finite without device allocation: the per-element flags and the
// count live in a fixed, file-scope device array instead of the domain's
// lazily allocated work array.
#include <hip/hip_runtime.h>

#include <mutex>

#include "common.h"

namespace grffe {
void launch_check_finite(const KArgs& a, int nn, int mm, uint8_t* bad, hipStream_t s);
int set_error(int code, const char* msg);
}  // namespace grffe

using namespace grffe;

// Largest element count the fixed array serves: one flag byte per element after
// a 256-byte header that holds the count (1 MiB + 256 B per device, held until
// the process ends).
static constexpr int kMaxElems = 1 << 20;
static constexpr size_t kHeader = 256;
static constexpr int kMaxDevices = 64;

// The array itself.  Host code never passes its name to a kernel or a copy (on the
// host the name is only a stand-in), only the device address hipGetSymbolAddress
// returns for the current device.
static __device__ __align__(256) unsigned char scratch[kHeader + kMaxElems];

namespace {

std::mutex g_mu;
void* g_ptr[kMaxDevices] = {};

// Device address of the current device's copy of `scratch` (looked up once per
// device), or null with the HIP status in *err.
void* scratch_ptr(hipError_t* err) {
  int dev = 0;
  *err = hipGetDevice(&dev);
  if (*err != hipSuccess) return nullptr;
  if (dev < 0 || dev >= kMaxDevices) {
    *err = hipErrorInvalidDevice;
    return nullptr;
  }
  std::lock_guard<std::mutex> lock(g_mu);
  if (!g_ptr[dev]) {
    void* p = nullptr;
    *err = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (*err != hipSuccess) return nullptr;
    g_ptr[dev] = p;
  }
  return g_ptr[dev];
}

// Number of set flags among flags[0 .. E), written to *out by one workgroup (no
// prior clearing needed: the single block writes the final value).
__global__ __launch_bounds__(1024) void k_count_flags(const uint8_t* flags, int E, int32_t* out) {
  __shared__ int32_t part[16];
  int32_t c = 0;
  for (int e = threadIdx.x; e < E; e += 1024) c += flags[e] ? 1 : 0;
  for (int off = 32; off > 0; off >>= 1) c += __shfl_xor(c, off, 64);
  if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = c;
  __syncthreads();
  if (threadIdx.x == 0) {
    int32_t s = 0;
    for (int w = 0; w < 16; ++w) s += part[w];
    *out = s;
  }
}

}  // namespace

extern "C" int grffe_check_finite_noalloc(grffe_domain* d, int32_t* n_bad, void* stream) {
  if (!d) return set_error(GRFFE_EINVAL, "domain is NULL");
  if (d->E > kMaxElems)
    return set_error(GRFFE_EINVAL, "grffe_check_finite_noalloc serves at most 1048576 elements");
  hipError_t err = hipSuccess;
  unsigned char* base = static_cast<unsigned char*>(scratch_ptr(&err));
  if (!base) return set_error(GRFFE_EHIP, hipGetErrorString(err));
  int32_t* count = reinterpret_cast<int32_t*>(base);
  uint8_t* flags = base + kHeader;
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  KArgs a = make_args(d);
  launch_check_finite(a, d->nn, d->mm, flags, st);
  launch_kernel(k_count_flags, dim3(1), dim3(1024), st, (const uint8_t*)flags, d->E, count);
  err = hipGetLastError();
  if (err != hipSuccess) return set_error(GRFFE_EHIP, hipGetErrorString(err));
  int32_t nb = 0;
  err = hipMemcpyAsync(&nb, count, sizeof(int32_t), hipMemcpyDeviceToHost, st);
  if (err == hipSuccess) err = hipStreamSynchronize(st);
  if (err != hipSuccess) return set_error(GRFFE_EHIP, hipGetErrorString(err));
  if (n_bad) *n_bad = nb;
  if (nb) return set_error(GRFFE_ENONFINITE, "element(s) hold non-finite values");
  return GRFFE_OK;
}
