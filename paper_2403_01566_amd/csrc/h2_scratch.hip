// Device scratch of the allocation-free entry point (h2_matvec_noalloc).
//
// One file-scope device array per GPU, allocated when the library's code
// object is loaded on that GPU and held until the process ends.  Host code
// never passes `scratch` itself to a kernel or a copy: in host code the name
// is a host-side stand-in.  The device address of each GPU's copy is looked
// up once per device (with that device current) and kept; every user of the
// array takes that address.
#include <mutex>

#include "h2_core.h"

namespace h2 {

namespace {
constexpr size_t kScratchBytes = size_t(H2_MATVEC_SCRATCH_BYTES);
std::mutex g_mu;
std::map<int, char*> g_addr;  // device -> address of its copy of `scratch`
}  // namespace

static __device__ __align__(256) char scratch[kScratchBytes];

char* scratch_address(int device) {
  std::lock_guard<std::mutex> lock(g_mu);
  auto it = g_addr.find(device);
  if (it != g_addr.end()) return it->second;
  int cur = -1;
  H2_HIP(hipGetDevice(&cur));
  if (cur != device) throw Error(H2_ERR_DEVICE, "scratch lookup with another device current");
  void* p = nullptr;
  const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e != hipSuccess || p == nullptr)
    throw Error(H2_ERR_DEVICE, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
  g_addr[device] = static_cast<char*>(p);
  return static_cast<char*>(p);
}

size_t scratch_bytes() { return kScratchBytes; }

}  // namespace h2
