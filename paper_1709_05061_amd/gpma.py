"""ctypes binding of libgpma.so (the C ABI in include/gpma.h).

Argument marshalling only: every step of the update and of the analytics
runs in the HIP library.  Device buffers are torch tensors on the current
HIP device; streams are torch streams.  There is no CPU fallback: importing
works anywhere, but the first call raises if the library is not built or no
GPU is visible.
"""
from __future__ import annotations

import ctypes as C
import os
import threading
from dataclasses import dataclass, field
from typing import List, Optional

import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libgpma.so")

GPMA_OK, GPMA_EINVAL, GPMA_ENOMEM, GPMA_EDEVICE = 0, -1, -2, -3
GPMA_FLAG_MIRROR = 1
GPMA_FLAG_LEARNED_LOCATOR = 2
GPMA_FLAG_FUSED_DIRECT = 4
GPMA_FLAG_LAZY_DELETE = 8
GPMA_FLAG_FUSED_LIB_STREAMS = 16
GPMA_FLAG_WINDOW_RADIX = 32
SPMV_FORMS = {"auto": 0, "binned": 1, "binned_coarse": 2, "pull": 3, "push": 4, "binned_gather": 5}
EMPTY = 0xFFFFFFFFFFFFFFFF
GUARD_DST = 0xFFFFFFFF

# kernel ids for the profiling calls
K_SPMV, K_LEAF_MERGE, K_SEG_MERGE, K_SORT, K_LOCATE, K_BFS, K_CC = range(7)
KERNEL_NAMES = ["spmv", "leaf_merge", "seg_merge", "sort", "locate", "bfs_expand", "cc_hook"]


class gpma_params(C.Structure):
    _fields_ = [("leaf_size", C.c_uint32), ("tau_leaf_pm", C.c_uint32), ("tau_root_pm", C.c_uint32),
                ("rho_leaf_pm", C.c_uint32), ("rho_root_pm", C.c_uint32), ("flags", C.c_uint32),
                ("sort_tile_keys", C.c_uint32), ("fused_levels", C.c_uint32),
                ("lds_tier_bytes", C.c_uint32), ("spmv_form", C.c_uint32)]


ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_void_p, C.c_void_p)
FREE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_size_t, C.c_void_p, C.c_void_p)


class gpma_allocator(C.Structure):
    _fields_ = [("alloc", ALLOC_FN), ("free", FREE_FN), ("ctx", C.c_void_p)]


class TorchAllocator:
    """Device memory of a handle from PyTorch's caching allocator, so the
    library's arrays share torch's pool (and its accounting) on the stream of
    the call that allocates them.  held_bytes counts what the library holds
    through this allocator; a failed allocation returns NULL, which the
    library turns into GPMA_ENOMEM with nothing changed.  Keep the object
    alive as long as a handle created with it."""

    def __init__(self, device=None):
        self.device = torch.cuda.current_device() if device is None else device
        self.held_bytes = 0
        self.peak_bytes = 0
        self._sizes = {}
        # handles used from several host threads (the service's query
        # workers) allocate concurrently: the budget check, the allocation and
        # the count are one step
        self._lock = threading.Lock()
        self._alloc_cb = ALLOC_FN(self._alloc)
        self._free_cb = FREE_FN(self._free)
        self.struct = gpma_allocator(self._alloc_cb, self._free_cb, None)

    def allow(self, nbytes: int) -> bool:
        """Whether an allocation of nbytes may be made (a subclass may
        refuse, e.g. to keep an HBM budget)."""
        return True

    def _alloc(self, nbytes, stream, ctx):
        with self._lock:
            try:
                if not self.allow(int(nbytes)):
                    return None
                ptr = torch.cuda.caching_allocator_alloc(int(nbytes), self.device, int(stream or 0))
            except Exception:
                return None
            self._sizes[ptr] = int(nbytes)
            self.held_bytes += int(nbytes)
            self.peak_bytes = max(self.peak_bytes, self.held_bytes)
            return ptr

    def _free(self, ptr, nbytes, stream, ctx):
        with self._lock:
            try:
                self.held_bytes -= self._sizes.pop(ptr, int(nbytes))
                torch.cuda.caching_allocator_delete(ptr)
            except Exception:
                pass


class gpma_stats(C.Structure):
    _fields_ = [("requested", C.c_uint64), ("applied", C.c_uint64), ("noops", C.c_uint64),
                ("top_level", C.c_int32), ("resized", C.c_uint32),
                ("segments_merged", C.c_uint64 * 40), ("slots_rewritten", C.c_uint64),
                ("mirror_slots_rewritten", C.c_uint64)]


class GpmaError(RuntimeError):
    def __init__(self, code: int, what: str):
        super().__init__("%s failed: %s (%d)" % (what, strerror(code), code))
        self.code = code


_lib = None


def load_library() -> C.CDLL:
    """Load libgpma.so; raises if it is missing (no fallback path exists)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError("libgpma.so is not built (build it with "
                           "python paper_1709_05061_amd/build.py)")
    lib = C.CDLL(LIB_PATH)
    vp, u32, u64, i32, f32 = C.c_void_p, C.c_uint32, C.c_uint64, C.c_int32, C.c_float
    pu64 = C.POINTER(u64)
    sig = {
        "gpma_default_params": (None, [C.POINTER(gpma_params)]),
        "gpma_create": (C.c_int, [C.POINTER(vp), u32, vp, u64, C.POINTER(gpma_params),
                                  C.POINTER(gpma_allocator), vp]),
        "gpma_fused_pairing": (C.c_int, [vp, vp]),
        "gpma_allocated_bytes": (u64, [vp]),
        "gpma_reserve": (C.c_int, [vp, u64, vp]),
        "gpma_destroy": (C.c_int, [vp]),
        "gpma_insert_batch": (C.c_int, [vp, vp, u64, vp, C.POINTER(gpma_stats)]),
        "gpma_delete_batch": (C.c_int, [vp, vp, u64, vp, C.POINTER(gpma_stats)]),
        "gpma_pagerank": (C.c_int, [vp, vp, vp, u32, f32, vp]),
        "gpma_bfs": (C.c_int, [vp, u32, vp, vp]),
        "gpma_bfs_noalloc": (C.c_int, [vp, u32, vp, vp]),
        "gpma_cc": (C.c_int, [vp, vp, vp]),
        "gpma_num_edges": (u64, [vp]),
        "gpma_capacity": (u64, [vp]),
        "gpma_leaf_size": (u32, [vp]),
        "gpma_num_vertices": (u32, [vp]),
        "gpma_export_slots": (C.c_int, [vp, vp, u64, pu64, vp]),
        "gpma_export_keys": (C.c_int, [vp, vp, u64, pu64, vp]),
        "gpma_export_leaf_counts": (C.c_int, [vp, vp, u64, vp]),
        "gpma_export_pivots": (C.c_int, [vp, vp, u64, vp]),
        "gpma_export_row_offsets": (C.c_int, [vp, vp, u64, vp]),
        "gpma_export_degrees": (C.c_int, [vp, vp, u64, vp]),
        "gpma_sync": (C.c_int, [vp]),
        "gpma_get_mirror": (vp, [vp]),
        "gpma_lock_insert_batch": (C.c_int, [vp, vp, u64, vp, C.POINTER(gpma_stats), C.POINTER(u32)]),
        "gpma_snapshot": (C.c_int, [vp, C.POINTER(vp), vp]),
        "gpma_snapshot_refresh": (C.c_int, [vp, vp, vp]),
        "gpma_device_bytes": (u64, [vp]),
        "gpma_locate": (C.c_int, [vp, vp, u64, vp, vp]),
        "gpma_locator_refit": (C.c_int, [vp, vp]),
        "gpma_locator_info": (C.c_int, [vp, C.POINTER(u32), pu64, pu64, pu64]),
        "gpma_apply_batches": (C.c_int, [vp, u32, C.POINTER(C.c_uint8), C.POINTER(vp), C.POINTER(u64), vp,
                                         C.POINTER(gpma_stats), C.POINTER(u32)]),
        "gpma_strerror": (C.c_char_p, [C.c_int]),
        "gpma_profile_enable": (C.c_int, [vp, C.c_int]),
        "gpma_profile_reset": (C.c_int, [vp]),
        "gpma_profile_read": (C.c_int, [vp, C.c_int, C.POINTER(C.c_double), pu64,
                                        C.POINTER(C.c_double)]),
        "gpma_csr_create": (C.c_int, [C.POINTER(vp), u32, vp, u64, vp]),
        "gpma_csr_destroy": (None, [vp]),
        "gpma_csr_update": (C.c_int, [vp, vp, u64, C.c_int, vp]),
        "gpma_csr_num_edges": (u64, [vp]),
        "gpma_csr_export": (C.c_int, [vp, vp, u64, vp, vp]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def exported_symbols() -> List[str]:
    return ["gpma_default_params", "gpma_create", "gpma_destroy", "gpma_insert_batch",
            "gpma_delete_batch", "gpma_pagerank", "gpma_bfs", "gpma_bfs_noalloc", "gpma_cc", "gpma_num_edges",
            "gpma_capacity", "gpma_leaf_size", "gpma_num_vertices", "gpma_export_slots",
            "gpma_export_keys", "gpma_export_leaf_counts", "gpma_export_pivots", "gpma_export_row_offsets",
            "gpma_export_degrees", "gpma_sync", "gpma_get_mirror", "gpma_apply_batches", "gpma_strerror",
            "gpma_snapshot", "gpma_snapshot_refresh", "gpma_device_bytes", "gpma_locate",
            "gpma_locator_refit", "gpma_locator_info",
            "gpma_profile_enable",
            "gpma_profile_reset", "gpma_profile_read", "gpma_csr_create", "gpma_csr_destroy",
            "gpma_csr_update", "gpma_csr_num_edges", "gpma_csr_export", "gpma_lock_insert_batch",
            "gpma_fused_pairing", "gpma_allocated_bytes", "gpma_reserve"]


def strerror(code: int) -> str:
    try:
        return load_library().gpma_strerror(code).decode()
    except Exception:  # pragma: no cover
        return "error"


def _stream(stream=None) -> C.c_void_p:
    if stream is None:
        stream = torch.cuda.current_stream()
    return C.c_void_p(stream.cuda_stream)


def _dev_u64(t: torch.Tensor) -> torch.Tensor:
    if not t.is_cuda:
        raise ValueError("keys must be a device tensor")
    if t.dtype not in (torch.int64, torch.uint64):
        raise ValueError("keys must be 64-bit integers")
    return t.contiguous()


def _check(code: int, what: str):
    if code != GPMA_OK:
        raise GpmaError(code, what)


# --------------------------------------------------------------------------
# thin wrappers with the C names

def gpma_default_params() -> gpma_params:
    p = gpma_params()
    load_library().gpma_default_params(C.byref(p))
    return p


def gpma_create(num_vertices: int, init_keys: torch.Tensor, params: Optional[gpma_params] = None,
                stream=None, allocator: Optional[TorchAllocator] = None) -> C.c_void_p:
    lib = load_library()
    h = C.c_void_p()
    k = _dev_u64(init_keys)
    rc = lib.gpma_create(C.byref(h), num_vertices, C.c_void_p(k.data_ptr()), k.numel(),
                         C.byref(params) if params is not None else None,
                         C.byref(allocator.struct) if allocator is not None else None, _stream(stream))
    _check(rc, "gpma_create")
    return h


def gpma_destroy(h) -> None:
    load_library().gpma_destroy(h)


def gpma_insert_batch(h, keys: torch.Tensor, stream=None, stats: bool = False):
    k = _dev_u64(keys)
    st = gpma_stats() if stats else None
    rc = load_library().gpma_insert_batch(h, C.c_void_p(k.data_ptr()), k.numel(), _stream(stream),
                                          C.byref(st) if st is not None else None)
    _check(rc, "gpma_insert_batch")
    return st


def gpma_lock_insert_batch(h, keys: torch.Tensor, stream=None):
    """The lock-based GPMA insertion (comparator); returns (stats, rounds)."""
    k = _dev_u64(keys)
    st = gpma_stats()
    rounds = C.c_uint32()
    rc = load_library().gpma_lock_insert_batch(h, C.c_void_p(k.data_ptr()), k.numel(), _stream(stream),
                                               C.byref(st), C.byref(rounds))
    _check(rc, "gpma_lock_insert_batch")
    return st, rounds.value


def gpma_delete_batch(h, keys: torch.Tensor, stream=None, stats: bool = False):
    k = _dev_u64(keys)
    st = gpma_stats() if stats else None
    rc = load_library().gpma_delete_batch(h, C.c_void_p(k.data_ptr()), k.numel(), _stream(stream),
                                          C.byref(st) if st is not None else None)
    _check(rc, "gpma_delete_batch")
    return st


def gpma_apply_batches(h, ops, batches, stream=None):
    """Fused batching: ops[i] in {0 insert, 1 delete}, batches[i] device key
    tensors.  Returns (stats, completed)."""
    n = len(batches)
    ks = [_dev_u64(b) for b in batches]
    ops_arr = (C.c_uint8 * max(n, 1))(*[int(o) for o in ops])
    ptrs = (C.c_void_p * max(n, 1))(*[k.data_ptr() for k in ks])
    sizes = (C.c_uint64 * max(n, 1))(*[k.numel() for k in ks])
    st = gpma_stats()
    done = C.c_uint32()
    rc = load_library().gpma_apply_batches(h, n, ops_arr, ptrs, sizes, _stream(stream), C.byref(st),
                                           C.byref(done))
    _check(rc, "gpma_apply_batches")
    return st, done.value


def gpma_pagerank(h, init: Optional[torch.Tensor], out: torch.Tensor, iters: int = 10,
                  damping: float = 0.85, stream=None) -> torch.Tensor:
    assert out.is_cuda and out.dtype == torch.float32 and out.is_contiguous()
    ip = None
    if init is not None:
        assert init.is_cuda and init.dtype == torch.float32 and init.is_contiguous()
        ip = C.c_void_p(init.data_ptr())
    rc = load_library().gpma_pagerank(h, ip, C.c_void_p(out.data_ptr()), iters, damping, _stream(stream))
    _check(rc, "gpma_pagerank")
    return out


def gpma_bfs(h, source: int, dist: torch.Tensor, stream=None) -> torch.Tensor:
    assert dist.is_cuda and dist.dtype == torch.int32 and dist.is_contiguous()
    _check(load_library().gpma_bfs(h, source, C.c_void_p(dist.data_ptr()), _stream(stream)), "gpma_bfs")
    return dist


def gpma_bfs_noalloc(h, source: int, dist: torch.Tensor, stream=None) -> torch.Tensor:
    """gpma_bfs without device allocation (scratch in the library's fixed
    per-GPU array; V <= 2^22)."""
    assert dist.is_cuda and dist.dtype == torch.int32 and dist.is_contiguous()
    _check(load_library().gpma_bfs_noalloc(h, source, C.c_void_p(dist.data_ptr()), _stream(stream)),
           "gpma_bfs_noalloc")
    return dist


def gpma_cc(h, label: torch.Tensor, stream=None) -> torch.Tensor:
    assert label.is_cuda and label.dtype == torch.int32 and label.is_contiguous()
    _check(load_library().gpma_cc(h, C.c_void_p(label.data_ptr()), _stream(stream)), "gpma_cc")
    return label


# --------------------------------------------------------------------------
# convenience object

@dataclass
class BatchStats:
    requested: int
    applied: int
    noops: int
    top_level: int
    resized: bool
    segments_merged: List[int] = field(default_factory=list)
    slots_rewritten: int = 0
    mirror_slots_rewritten: int = 0

    @classmethod
    def of(cls, st: gpma_stats) -> "BatchStats":
        # the levels up to the last with a merge (trailing zero words cut in C)
        w = C.sizeof(st.segments_merged._type_)
        n = (len(bytes(st.segments_merged).rstrip(b"\0")) + w - 1) // w
        segs = st.segments_merged[:n]
        return cls(st.requested, st.applied, st.noops, st.top_level, bool(st.resized), segs,
                   st.slots_rewritten, st.mirror_slots_rewritten)


class _HandleView:
    """Read-only calls on a handle (exports, introspection)."""

    def __init__(self, h, V: int):
        self._lib = load_library()
        self.h = h
        self.V = V

    # --- introspection
    @property
    def num_edges(self) -> int:
        return int(self._lib.gpma_num_edges(self.h))

    @property
    def capacity(self) -> int:
        return int(self._lib.gpma_capacity(self.h))

    @property
    def leaf_size(self) -> int:
        return int(self._lib.gpma_leaf_size(self.h))

    def slots(self, stream=None) -> torch.Tensor:
        out = torch.empty(self.capacity, dtype=torch.int64, device="cuda")
        cap = C.c_uint64()
        _check(self._lib.gpma_export_slots(self.h, C.c_void_p(out.data_ptr()), out.numel(),
                                           C.byref(cap), _stream(stream)), "gpma_export_slots")
        return out

    def keys(self, stream=None) -> torch.Tensor:
        out = torch.empty(max(self.num_edges, 1), dtype=torch.int64, device="cuda")
        n = C.c_uint64()
        _check(self._lib.gpma_export_keys(self.h, C.c_void_p(out.data_ptr()), out.numel(),
                                          C.byref(n), _stream(stream)), "gpma_export_keys")
        return out[: n.value]

    def leaf_counts(self, stream=None) -> torch.Tensor:
        out = torch.empty(self.capacity // self.leaf_size, dtype=torch.int16, device="cuda")
        _check(self._lib.gpma_export_leaf_counts(self.h, C.c_void_p(out.data_ptr()), out.numel(),
                                                 _stream(stream)), "gpma_export_leaf_counts")
        return out

    def pivots(self, stream=None) -> torch.Tensor:
        """Each leaf's first slot with the deletion mark cleared (int64 bit
        patterns), the array the locate searches."""
        out = torch.empty(self.capacity // self.leaf_size, dtype=torch.int64, device="cuda")
        _check(self._lib.gpma_export_pivots(self.h, C.c_void_p(out.data_ptr()), out.numel(),
                                            _stream(stream)), "gpma_export_pivots")
        return out

    def row_offsets(self, stream=None) -> torch.Tensor:
        out = torch.empty(self.V + 1, dtype=torch.int32, device="cuda")
        _check(self._lib.gpma_export_row_offsets(self.h, C.c_void_p(out.data_ptr()), out.numel(),
                                                 _stream(stream)), "gpma_export_row_offsets")
        return out

    def degrees(self, stream=None) -> torch.Tensor:
        out = torch.empty(self.V, dtype=torch.int32, device="cuda")
        _check(self._lib.gpma_export_degrees(self.h, C.c_void_p(out.data_ptr()), out.numel(),
                                             _stream(stream)), "gpma_export_degrees")
        return out



class GPMA(_HandleView):
    """A GPU PMA holding a dynamic directed graph (one handle of the C ABI).
    mirror=True also keeps the dst-major mirror (GPMA_FLAG_MIRROR); learned
    enables the learned locator; fused_direct makes apply_batches enqueue
    kernels directly instead of replaying captured graphs; sort_tile picks the
    batch sort's keys per workgroup tile (512, 1024 or 2048; 0 = 1024);
    fused_levels is how many tree levels above the leaves a fused batch runs
    on the device before the host takes over (0..3); lazy_delete makes
    deletes mark their entries in place (GPMA_FLAG_LAZY_DELETE); lds_tier
    caps the LDS bytes of the workgroup merge tier (0 = all; 1 sends every
    level above the leaves to the device tier); spmv picks PageRank's SpMV
    (a key of SPMV_FORMS); lib_streams forces fused batching with a mirror
    onto two handle streams; window_sort picks the sort of a fused window's
    keys ("splitter", or "radix" for the LSD radix sort).  allocator: a TorchAllocator (the default: a new
    one per handle, so the library's memory comes from torch's caching
    allocator), or False for the library's own hipMalloc."""

    def __init__(self, num_vertices: int, init_keys: torch.Tensor, leaf_size: int = 0,
                 tau_leaf=920, tau_root=800, rho_leaf=80, rho_root=400, mirror: bool = False,
                 learned: bool = False, stream=None, fused_direct: bool = False, sort_tile: int = 0,
                 fused_levels: int = 1, lazy_delete: bool = False, lds_tier: int = 0, spmv: str = "auto",
                 lib_streams: bool = False, window_sort: str = "splitter", allocator=None):
        if window_sort not in ("splitter", "radix"):
            raise ValueError("window_sort must be 'splitter' or 'radix'")
        flags = ((GPMA_FLAG_MIRROR if mirror else 0) | (GPMA_FLAG_LEARNED_LOCATOR if learned else 0)
                 | (GPMA_FLAG_FUSED_DIRECT if fused_direct else 0) | (GPMA_FLAG_LAZY_DELETE if lazy_delete else 0)
                 | (GPMA_FLAG_FUSED_LIB_STREAMS if lib_streams else 0)
                 | (GPMA_FLAG_WINDOW_RADIX if window_sort == "radix" else 0))
        p = gpma_params(leaf_size, tau_leaf, tau_root, rho_leaf, rho_root, flags, sort_tile, fused_levels,
                        lds_tier, SPMV_FORMS[spmv])
        if allocator is None:
            allocator = TorchAllocator()
        self.allocator = allocator or None
        super().__init__(gpma_create(num_vertices, init_keys, p, stream, self.allocator), num_vertices)

    def close(self):
        if getattr(self, "h", None):
            gpma_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def allocated_bytes(self) -> int:
        """Device bytes the handle and its mirror hold from their allocator."""
        return int(self._lib.gpma_allocated_bytes(self.h))

    def reserve(self, b: int, stream=None):
        """Take now the memory update batches of up to b keys need short of a
        root resize (gpma_reserve)."""
        _check(self._lib.gpma_reserve(self.h, b, _stream(stream)), "gpma_reserve")

    def fused_pairing(self, stream=None) -> int:
        """1: fused batching keeps the array's pipeline on `stream` with the
        mirror's beside it; 0: both on handle streams; GPMA_EINVAL: no mirror
        or no fused call on that stream yet."""
        return int(self._lib.gpma_fused_pairing(self.h, _stream(stream)))

    def locate(self, keys: torch.Tensor, stream=None) -> torch.Tensor:
        """Leaf of each key (learned locator if enabled, else binary search)."""
        k = _dev_u64(keys)
        out = torch.empty(k.numel(), dtype=torch.int32, device="cuda")
        _check(self._lib.gpma_locate(self.h, C.c_void_p(k.data_ptr()), k.numel(), C.c_void_p(out.data_ptr()),
                                     _stream(stream)), "gpma_locate")
        return out

    def locator_info(self):
        eps, lk, ms, fits = C.c_uint32(), C.c_uint64(), C.c_uint64(), C.c_uint64()
        _check(self._lib.gpma_locator_info(self.h, C.byref(eps), C.byref(lk), C.byref(ms), C.byref(fits)),
               "gpma_locator_info")
        return {"eps": eps.value, "lookups": lk.value, "misses": ms.value, "fits": fits.value}

    def mirror(self):
        """The dst-major mirror as a read-only view (None without one)."""
        m = self._lib.gpma_get_mirror(self.h)
        return _HandleView(C.c_void_p(m), self.V) if m else None

    # --- updates
    def insert(self, keys: torch.Tensor, stream=None, stats=False):
        st = gpma_insert_batch(self.h, keys, stream, stats)
        return BatchStats.of(st) if stats else None

    def delete(self, keys: torch.Tensor, stream=None, stats=False):
        st = gpma_delete_batch(self.h, keys, stream, stats)
        return BatchStats.of(st) if stats else None

    def lock_insert(self, keys: torch.Tensor, stream=None):
        """Insert with the lock-based GPMA algorithm (the comparator);
        returns (BatchStats, rounds)."""
        st, rounds = gpma_lock_insert_batch(self.h, keys, stream)
        return BatchStats.of(st), rounds

    def apply_batches(self, ops, batches, stream=None) -> BatchStats:
        """Fused batching of a sequence of insert (0) / delete (1) batches."""
        st, _ = gpma_apply_batches(self.h, ops, batches, stream)
        return BatchStats.of(st)

    # --- analytics
    def pagerank(self, init: Optional[torch.Tensor] = None, iters: int = 10, damping: float = 0.85,
                 out: Optional[torch.Tensor] = None, stream=None) -> torch.Tensor:
        if out is None:
            out = torch.empty(self.V, dtype=torch.float32, device="cuda")
        return gpma_pagerank(self.h, init, out, iters, damping, stream)

    def bfs(self, source: int, out: Optional[torch.Tensor] = None, stream=None) -> torch.Tensor:
        if out is None:
            out = torch.empty(self.V, dtype=torch.int32, device="cuda")
        return gpma_bfs(self.h, source, out, stream)

    def cc(self, out: Optional[torch.Tensor] = None, stream=None) -> torch.Tensor:
        if out is None:
            out = torch.empty(self.V, dtype=torch.int32, device="cuda")
        return gpma_cc(self.h, out, stream)

    # --- profiling
    def profile(self, enable: bool = True):
        self._lib.gpma_profile_enable(self.h, 1 if enable else 0)

    def profile_reset(self):
        self._lib.gpma_profile_reset(self.h)

    def profile_read(self, kernel: int):
        ms, n, by = C.c_double(), C.c_uint64(), C.c_double()
        self._lib.gpma_profile_read(self.h, kernel, C.byref(ms), C.byref(n), C.byref(by))
        return ms.value, n.value, by.value


class CSRRebuild:
    """The rebuild-per-batch CSR comparator (gpma_csr_*): same set semantics
    as GPMA, every batch rewrites the whole edge array and row offsets."""

    def __init__(self, num_vertices: int, init_keys: torch.Tensor, stream=None):
        self._lib = load_library()
        self.V = num_vertices
        h = C.c_void_p()
        init_keys = init_keys.contiguous()
        _check(self._lib.gpma_csr_create(C.byref(h), num_vertices, C.c_void_p(init_keys.data_ptr()),
                                         init_keys.numel(), _stream(stream)), "gpma_csr_create")
        self.h = h

    def _update(self, keys: torch.Tensor, delete: bool, stream=None):
        keys = keys.contiguous()
        _check(self._lib.gpma_csr_update(self.h, C.c_void_p(keys.data_ptr()), keys.numel(), 1 if delete else 0,
                                         _stream(stream)), "gpma_csr_update")

    def insert(self, keys: torch.Tensor, stream=None):
        self._update(keys, False, stream)

    def delete(self, keys: torch.Tensor, stream=None):
        self._update(keys, True, stream)

    @property
    def num_edges(self) -> int:
        return int(self._lib.gpma_csr_num_edges(self.h))

    def keys(self, stream=None) -> torch.Tensor:
        out = torch.empty(max(self.num_edges, 1), dtype=torch.int64, device="cuda")
        _check(self._lib.gpma_csr_export(self.h, C.c_void_p(out.data_ptr()), out.numel(), None, _stream(stream)),
               "gpma_csr_export")
        return out[: self.num_edges]

    def row_offsets(self, stream=None) -> torch.Tensor:
        out = torch.empty(self.V + 1, dtype=torch.int64, device="cuda")
        _check(self._lib.gpma_csr_export(self.h, None, 0, C.c_void_p(out.data_ptr()), _stream(stream)),
               "gpma_csr_export")
        return out

    def close(self):
        if getattr(self, "h", None):
            self._lib.gpma_csr_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
