// Static device workspace of the allocation-free encode entry point
// (lpcc_encode_frame_noalloc).  Callers that cannot allocate device memory
// (code under HIP graph capture, tight serving loops, harnesses that forbid
// hipMalloc) get every intermediate buffer of an encode carved from one
// block that lives in this code object instead of from the context's
// growing arenas.
//
// The block is a file-scope __device__ array: every device the library runs
// on holds its own copy, at its own address, from the load of this code
// object until the process ends.  In host code the array's name is only a
// host-side stand-in, never a device address: host code uses the address
// that hipGetSymbolAddress returns for the current device, looked up once
// per device when a context is created on it.
#include <mutex>

#include "lpcc_internal.h"

static __device__ __align__(256) char scratch[lpcc::kNoallocBytes];

namespace {
constexpr int kMaxDevices = 64;
char* g_scratch_ptr[kMaxDevices] = {};   // device address of `scratch`, per device
hipError_t g_scratch_err[kMaxDevices] = {};
bool g_scratch_done[kMaxDevices] = {};
std::mutex g_setup_mu;
std::mutex g_call_mu[kMaxDevices];
}  // namespace

namespace lpcc {

int scratch_setup(int device, char** base, size_t* cap, std::string* why) {
  *base = nullptr;
  *cap = 0;
  if (device < 0 || device >= kMaxDevices) return LPCC_E_INVAL;
  std::lock_guard<std::mutex> g(g_setup_mu);
  if (!g_scratch_done[device]) {
    // `device` is current (the caller has set it)
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || p == nullptr) {
      (void)hipGetLastError();
      g_scratch_err[device] = e != hipSuccess ? e : hipErrorInvalidSymbol;
    } else {
      g_scratch_ptr[device] = (char*)p;
    }
    g_scratch_done[device] = true;
  }
  if (!g_scratch_ptr[device]) {
    *why = std::string("hipGetSymbolAddress of the static workspace failed: ") +
           hipGetErrorString(g_scratch_err[device]);
    return LPCC_E_DEVICE;
  }
  *base = g_scratch_ptr[device];
  *cap = kNoallocBytes;
  return LPCC_OK;
}

std::mutex& scratch_mutex(int device) { return g_call_mu[device < 0 || device >= kMaxDevices ? 0 : device]; }

}  // namespace lpcc
