// ddamg_apply_D_noalloc: the canonical-layout Wilson-clover apply for
// callers that cannot allocate device memory (code under HIP graph capture,
// tight serving loops, harnesses that forbid hipMalloc).  ddamg_apply_D with
// the canonical layout converts the batch into two native staging fields
// that the library allocates on first use; this entry point stages through a
// fixed array in the library's device data instead and never allocates.
#include <mutex>

#include "handles.h"

using namespace ddamg;

// The staging memory: the native input batch in the first half, the native
// result in the second.  Every GPU that runs the library holds its own copy
// until the process ends.  In host code `scratch` names a host-side stand-in
// only; kernels get the device address from hipGetSymbolAddress.
static __device__ __align__(256) unsigned char scratch[DDAMG_NOALLOC_SCRATCH_BYTES];

namespace {

constexpr int MAX_DEVICES = 64;
std::mutex g_mu;
void* g_scratch_ptr[MAX_DEVICES] = {};

// device address of this device's `scratch` (looked up once per device, with
// that device current)
void* scratch_ptr() {
  int dev = -1;
  DD_CHECK_HIP(hipGetDevice(&dev));
  DD_REQUIRE(dev >= 0 && dev < MAX_DEVICES, "device index out of range");
  std::lock_guard<std::mutex> lock(g_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || p == nullptr) {
      (void)hipGetLastError();
      throw Error(DDAMG_EHIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    }
    g_scratch_ptr[dev] = p;
  }
  return g_scratch_ptr[dev];
}

template <typename T>
void apply_staged(Context& c, const double2* in, double2* out, int nrhs, void* base, hipStream_t s) {
  const size_t field = (size_t)c.g.V * 12 * sizeof(C<T>);
  DD_REQUIRE(2 * field * (size_t)nrhs <= (size_t)DDAMG_NOALLOC_SCRATCH_BYTES,
             "ddamg_apply_D_noalloc: " + std::to_string(nrhs) + " field(s) of " + std::to_string(c.g.V) +
                 " sites need " + std::to_string(2 * field * (size_t)nrhs) + " bytes of staging, more than the " +
                 std::to_string((size_t)DDAMG_NOALLOC_SCRATCH_BYTES) + " available");
  C<T>* a = static_cast<C<T>*>(base);
  C<T>* b = reinterpret_cast<C<T>*>(static_cast<unsigned char*>(base) + field * (size_t)nrhs);
  fine_to_native<T>(c.g, in, a, nrhs, s);
  dslash<T>(c.view<T>(), a, b, s, nrhs);
  fine_from_native<T>(c.g, b, out, nrhs, s);
}

}  // namespace

extern "C" int ddamg_apply_D_noalloc(ddamg_ctx ctx, const void* in, void* out, int nrhs, int prec,
                                     void* stream) {
  return guarded([&] {
    DD_REQUIRE(ctx && ctx->c, "null context");
    DD_REQUIRE(in && out && in != out, "in/out must be distinct device pointers");
    DD_REQUIRE(nrhs >= 1, "nrhs must be >= 1");
    DD_REQUIRE(prec == DDAMG_F64 || prec == DDAMG_F32, "prec must be DDAMG_F64 or DDAMG_F32");
    void* base = scratch_ptr();
    const hipStream_t s = as_stream(stream);
    if (prec == DDAMG_F64)
      apply_staged<double>(*ctx->c, static_cast<const double2*>(in), static_cast<double2*>(out), nrhs, base, s);
    else
      apply_staged<float>(*ctx->c, static_cast<const double2*>(in), static_cast<double2*>(out), nrhs, base, s);
  });
}
