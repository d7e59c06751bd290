// Fixed device scratch for the entry point that allocates nothing
// (lsp_apply_op_noalloc): the FFT work array of the K-matvec lives in a
// file-scope device array of kStaticScratchBytes instead of a caller
// workspace.  Each device the library runs on holds its own copy of the
// array (module load), at its own address; that address is looked up once
// per device with hipGetSymbolAddress, with the device current, and the
// library uses only the looked-up pointer from then on.  Every call on a
// device shares that device's copy: calls that overlap on one device race.
#include <map>
#include <mutex>

#include "lsp_common.h"
#include "static_scratch.h"

namespace lsp {

namespace {

static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

std::mutex g_mu;
std::map<int, void*> g_ptr;  // device -> address of that device's scratch

}  // namespace

void* static_scratch(int device) {
  std::lock_guard<std::mutex> lock(g_mu);
  auto it = g_ptr.find(device);
  if (it != g_ptr.end()) return it->second;
  int cur = -1;
  LSP_HIP(hipGetDevice(&cur));
  if (cur != device) LSP_HIP(hipSetDevice(device));
  void* ptr = nullptr;
  const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
  if (cur != device) (void)hipSetDevice(cur);
  if (e != hipSuccess || ptr == nullptr)
    throw Error(LSP_ERR_HIP, std::string("hipGetSymbolAddress of the static scratch failed: ") +
                                 hipGetErrorString(e));
  g_ptr.emplace(device, ptr);
  return ptr;
}

}  // namespace lsp
