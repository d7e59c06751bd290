"""MI355X (gfx950) solver for the Lippmann-Schwinger equation with the
sparsifying preconditioner: HIP kernels behind the C ABI of include/lsp.h,
with this package as a thin ctypes binding (lsp.py) and build step (build.py).
"""
from .lsp import (Plan, Problem, LspError, load, LSP_FP64, LSP_MIXED,  # noqa: F401
                  LSP_RHS_INCIDENT, LSP_RHS_G, EXPORTED, LIB_PATH)
