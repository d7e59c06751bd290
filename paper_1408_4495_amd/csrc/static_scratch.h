// Fixed device scratch of the allocation-free entry point (see
// static_scratch.hip).
#pragma once

#include <cstddef>

namespace lsp {

// Size of the per-device static scratch array (32 MiB).
constexpr size_t kStaticScratchBytes = size_t(32) << 20;

// Device address of `device`'s copy of the scratch array; looked up with
// hipGetSymbolAddress on the first call for that device (thread-safe).
// Throws lsp::Error(LSP_ERR_HIP) when the lookup fails.
void* static_scratch(int device);

}  // namespace lsp
