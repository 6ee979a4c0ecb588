"""MI355X-native GPMA+: a dynamic graph kept on the GPU as a packed memory
array, updated in batches by the lock-free level-by-level GPMA+ algorithm and
analysed in place (PageRank, BFS, connected components).

The work happens in libgpma.so (hand-written HIP for gfx950, C ABI in
include/gpma.h); this package is its ctypes binding.
"""
from .gpma import (GPMA, CSRRebuild, BatchStats, GpmaError, gpma_bfs, gpma_cc, gpma_create,  # noqa: F401
                   gpma_default_params, gpma_delete_batch, gpma_destroy, gpma_insert_batch,
                   gpma_pagerank, gpma_apply_batches, load_library, LIB_PATH)
