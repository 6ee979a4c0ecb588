"""CPU oracle for the GPMA+ hot path -- TEST INFRASTRUCTURE ONLY.

Only the tests, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package.  The GPU library never calls it and the
two share no code.

The sequential PMA and the analytics live in ``gpma_oracle.c`` (plain C, built
with gcc into ``liboracle.so``); this module is the ctypes binding plus a few
plain numpy read-outs of a slot image (CSR row offsets, leaf counts, the
structural invariants).  Source: Sha, Li, He, Tan, "Accelerating Dynamic
Graph Analytics on GPUs" (arXiv 1709.05061); each function cites the part of
the paper it follows.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "gpma_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

EMPTY = np.uint64(0xFFFFFFFFFFFFFFFF)
GUARD_DST = 0xFFFFFFFF
# density bounds of the figure "PMA insertion example" (Section 4.1), per mille
DEFAULT_PM = dict(tau_leaf=920, tau_root=800, rho_leaf=80, rho_root=400)

_lib = None


def build(force: bool = False) -> str:
    """Compile gpma_oracle.c with gcc (no GPU code involved)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fPIC", "-shared",
                               "-o", tmp, _SRC])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is not None:
        return _lib
    build()
    lib = C.CDLL(_LIB)
    u32, u64, i32 = C.c_uint32, C.c_uint64, C.c_int32
    pu64, pi32 = C.POINTER(u64), C.POINTER(i32)
    lib.orc_create.restype = C.c_void_p
    lib.orc_create.argtypes = [u32, pu64, u64, u32, u32, u32, u32, u32, C.POINTER(C.c_int)]
    lib.orc_set_lazy.restype = C.c_int
    lib.orc_set_lazy.argtypes = [C.c_void_p, C.c_int]
    lib.orc_from_slots.restype = C.c_void_p
    lib.orc_from_slots.argtypes = [pu64, u64, u32, u32, u32, u32, u32, C.POINTER(C.c_int)]
    lib.orc_free.argtypes = [C.c_void_p]
    for name in ("orc_capacity", "orc_size", "orc_log_len", "orc_last_applied", "orc_last_noops"):
        getattr(lib, name).restype = u64
        getattr(lib, name).argtypes = [C.c_void_p]
    lib.orc_leaf_size.restype = u32
    lib.orc_leaf_size.argtypes = [C.c_void_p]
    lib.orc_slots.restype = pu64
    lib.orc_slots.argtypes = [C.c_void_p]
    lib.orc_log_levels.restype = pi32
    lib.orc_log_levels.argtypes = [C.c_void_p]
    lib.orc_log_segs.restype = pu64
    lib.orc_log_segs.argtypes = [C.c_void_p]
    lib.orc_log_counts.restype = pu64
    lib.orc_log_counts.argtypes = [C.c_void_p]
    lib.orc_log_updates.restype = pu64
    lib.orc_log_updates.argtypes = [C.c_void_p]
    lib.orc_insert.restype = C.c_int
    lib.orc_insert.argtypes = [C.c_void_p, pu64, u64]
    lib.orc_delete.restype = C.c_int
    lib.orc_delete.argtypes = [C.c_void_p, pu64, u64]
    lib.orc_level_bounds.restype = C.c_int
    lib.orc_level_bounds.argtypes = [u32, u32, u32, u32, u32, u32, pu64, pu64]
    lib.orc_pagerank.argtypes = [u32, pu64, u64, C.POINTER(C.c_double), u32, C.c_double,
                                 C.POINTER(C.c_double)]
    lib.orc_bfs.argtypes = [u32, pu64, u64, u32, pi32]
    lib.orc_set_create.restype = C.c_void_p
    lib.orc_set_create.argtypes = [pu64, u64]
    lib.orc_set_free.argtypes = [C.c_void_p]
    lib.orc_set_size.restype = u64
    lib.orc_set_size.argtypes = [C.c_void_p]
    lib.orc_set_keys.restype = pu64
    lib.orc_set_keys.argtypes = [C.c_void_p]
    lib.orc_set_apply.restype = C.c_int64
    lib.orc_set_apply.argtypes = [C.c_void_p, pu64, u64, C.c_int]
    lib.orc_cc.argtypes = [u32, pu64, u64, C.POINTER(u32)]
    _lib = lib
    return lib


def _p(a: np.ndarray, ct):
    return a.ctypes.data_as(C.POINTER(ct))


def _keys(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.uint64))


class OracleError(RuntimeError):
    pass


def level_bounds(lf: int, H: int, tau_leaf=920, tau_root=800, rho_leaf=80, rho_root=400):
    """(min_h, max_h) for h = 0..H (Section 4.1, figure "PMA insertion example")."""
    lib = _load()
    mn = np.zeros(H + 1, np.uint64)
    mx = np.zeros(H + 1, np.uint64)
    lib.orc_level_bounds(lf, tau_leaf, tau_root, rho_leaf, rho_root, H,
                         _p(mn, C.c_uint64), _p(mx, C.c_uint64))
    return mn, mx


class OraclePMA:
    """Sequential GPMA+ (Section 5.2, Algorithm "GPMA+ Segment-Oriented
    Insertion", and its dual for deletions).  ``V > 0``: CSR-on-GPMA edge mode
    (guards added, keys checked); ``V == 0``: raw integer keys.  ``lazy``:
    deletions mark entries in place (bit 63) without density maintenance;
    merges drop the marked entries (Section 6, lazy deletion)."""

    def __init__(self, V: int, keys, leaf_size: int, tau_leaf=920, tau_root=800,
                 rho_leaf=80, rho_root=400, _handle=None, lazy: bool = False):
        self._lib = _load()
        if _handle is not None:
            self._h = _handle
            return
        k = _keys(keys)
        err = C.c_int(0)
        h = self._lib.orc_create(V, _p(k, C.c_uint64), k.size, leaf_size,
                                 tau_leaf, tau_root, rho_leaf, rho_root, C.byref(err))
        if not h:
            raise OracleError("orc_create failed (%d)" % err.value)
        self._h = h
        if lazy and self._lib.orc_set_lazy(h, 1) != 0:
            raise OracleError("lazy deletion needs 1 <= V <= 2^31")

    @classmethod
    def from_slots(cls, slots, leaf_size: int, tau_leaf=920, tau_root=800,
                   rho_leaf=80, rho_root=400) -> "OraclePMA":
        lib = _load()
        s = _keys(slots)
        err = C.c_int(0)
        h = lib.orc_from_slots(_p(s, C.c_uint64), s.size, leaf_size, tau_leaf, tau_root,
                               rho_leaf, rho_root, C.byref(err))
        if not h:
            raise OracleError("orc_from_slots failed (%d)" % err.value)
        return cls(0, None, leaf_size, _handle=h)

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            self._lib.orc_free(h)
            self._h = None

    @property
    def capacity(self) -> int:
        return int(self._lib.orc_capacity(self._h))

    @property
    def size(self) -> int:
        return int(self._lib.orc_size(self._h))

    @property
    def leaf_size(self) -> int:
        return int(self._lib.orc_leaf_size(self._h))

    def slots(self) -> np.ndarray:
        cap = self.capacity
        ptr = self._lib.orc_slots(self._h)
        return np.ctypeslib.as_array(ptr, shape=(cap,)).copy()

    def merge_log(self):
        n = int(self._lib.orc_log_len(self._h))
        if n == 0:
            return []
        lv = np.ctypeslib.as_array(self._lib.orc_log_levels(self._h), shape=(n,))
        sg = np.ctypeslib.as_array(self._lib.orc_log_segs(self._h), shape=(n,))
        return [(int(a), int(b)) for a, b in zip(lv, sg)]

    def merge_log_counts(self):
        """Per merge-log entry: (live entries of the segment before the
        merge, updates merged into it); for a root rebuild, (entries of the
        whole array, updates left at the root)."""
        n = int(self._lib.orc_log_len(self._h))
        if n == 0:
            return []
        ns = np.ctypeslib.as_array(self._lib.orc_log_counts(self._h), shape=(n,))
        k = np.ctypeslib.as_array(self._lib.orc_log_updates(self._h), shape=(n,))
        return [(int(a), int(b)) for a, b in zip(ns, k)]

    def last_applied(self) -> int:
        return int(self._lib.orc_last_applied(self._h))

    def last_noops(self) -> int:
        return int(self._lib.orc_last_noops(self._h))

    def insert(self, keys) -> None:
        k = _keys(keys)
        if self._lib.orc_insert(self._h, _p(k, C.c_uint64), k.size) != 0:
            raise OracleError("invalid key in insert batch")

    def delete(self, keys) -> None:
        k = _keys(keys)
        if self._lib.orc_delete(self._h, _p(k, C.c_uint64), k.size) != 0:
            raise OracleError("invalid key in delete batch")


class OracleSet:
    """The semantic layer: the edge set as a sorted vector of unique keys,
    batches merged in (union) or out (difference).  No layout; what the PMA
    must hold after any batch sequence, and a rebuild-style timing
    baseline (Section 6's CSR updated by rebuilding)."""

    def __init__(self, keys):
        self._lib = _load()
        k = _keys(keys)
        self._h = self._lib.orc_set_create(_p(k, C.c_uint64), k.size)
        if not self._h:
            raise OracleError("orc_set_create failed")

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            self._lib.orc_set_free(h)
            self._h = None

    def _apply(self, keys, delete: bool) -> int:
        k = _keys(keys)
        r = int(self._lib.orc_set_apply(self._h, _p(k, C.c_uint64), k.size, 1 if delete else 0))
        if r < 0:
            raise OracleError("out of memory")
        return r

    def insert(self, keys) -> int:
        return self._apply(keys, False)

    def delete(self, keys) -> int:
        return self._apply(keys, True)

    def keys(self) -> np.ndarray:
        n = int(self._lib.orc_set_size(self._h))
        if n == 0:
            return np.zeros(0, np.uint64)
        return np.ctypeslib.as_array(self._lib.orc_set_keys(self._h), shape=(n,)).copy()


# --------------------------------------------------------------------------
# read-outs of a slot image (plain numpy)

TOMB = np.uint64(1 << 63)


def stored(slots: np.ndarray) -> np.ndarray:
    """Live entries in array order (gaps and lazily deleted entries dropped)."""
    return slots[(slots & TOMB) == 0]


def occupied(slots: np.ndarray) -> np.ndarray:
    """Occupied slots in array order, marks cleared (lazily deleted entries
    still order the array)."""
    return slots[slots != EMPTY] & ~TOMB


def edge_keys(slots: np.ndarray) -> np.ndarray:
    """Stored (live) edges in order, guards dropped."""
    s = stored(slots)
    return s[(s & np.uint64(0xFFFFFFFF)) != np.uint64(GUARD_DST)]


def leaf_counts(slots: np.ndarray, lf: int) -> np.ndarray:
    return (slots.reshape(-1, lf) != EMPTY).sum(axis=1).astype(np.int64)


def leaf_pivots(slots: np.ndarray, lf: int) -> np.ndarray:
    """Each leaf's pivot: its first slot, a lazily deleted entry counting by
    its key (the locate rule's search keys, Section 5.1)."""
    return slots.reshape(-1, lf)[:, 0] & ~TOMB


def row_offsets(slots: np.ndarray, V: int) -> np.ndarray:
    """CSR row offsets on the PMA (Section 4.2, "CSR as a case study"): the
    guard of row u ends the row, so offset[u+1] = position(guard_u) + 1 and
    offset[0] = 0.  Row u spans slots [offset[u], offset[u+1])."""
    pos = np.nonzero((slots != EMPTY) & ((slots & np.uint64(0xFFFFFFFF)) == np.uint64(GUARD_DST)))[0]
    src = (slots[pos] >> np.uint64(32)).astype(np.int64)
    off = np.zeros(V + 1, np.int64)
    off[src + 1] = pos + 1
    return off


def out_degrees(edges: np.ndarray, V: int) -> np.ndarray:
    return np.bincount((edges >> np.uint64(32)).astype(np.int64), minlength=V).astype(np.int64)


def check_invariants(slots: np.ndarray, lf: int, V: int = 0, allow_empty_leaves=False):
    """Structural invariants of the PMA after a batch; raises AssertionError.
    (i) stored keys ascend strictly; (ii) every leaf is a packed prefix followed
    by gaps; (iii) no leaf is empty (unless allowed); (iv) in edge mode every
    vertex has exactly one guard and the guards of rows u < w appear in order."""
    assert slots.size % lf == 0
    o = occupied(slots)
    assert np.all(o[1:] > o[:-1]), "keys not strictly ascending"
    s = stored(slots)
    leaves = slots.reshape(-1, lf)
    occ = leaves != EMPTY
    cnt = occ.sum(axis=1)
    prefix = np.arange(lf)[None, :] < cnt[:, None]
    assert np.array_equal(occ, prefix), "a leaf is not a packed prefix"
    if not allow_empty_leaves:
        assert np.all(cnt > 0), "empty leaf"
    if V:
        g = s[(s & np.uint64(0xFFFFFFFF)) == np.uint64(GUARD_DST)]
        assert g.size == V and np.array_equal(g >> np.uint64(32), np.arange(V, dtype=np.uint64))


# --------------------------------------------------------------------------
# analytics (Section 6.1 "Applications"), fp64

def _sorted(edges) -> np.ndarray:
    e = _keys(edges)
    return e if e.size < 2 or bool(np.all(e[1:] >= e[:-1])) else np.sort(e)


def pagerank(V: int, edges, x0=None, iters: int = 10, damping: float = 0.85) -> np.ndarray:
    lib = _load()
    e = _sorted(edges)
    out = np.zeros(V, np.float64)
    if x0 is not None:
        x = np.ascontiguousarray(np.asarray(x0, dtype=np.float64))
        xp = _p(x, C.c_double)
    else:
        xp = None
    lib.orc_pagerank(V, _p(e, C.c_uint64), e.size, xp, iters, damping, _p(out, C.c_double))
    return out


def bfs(V: int, edges, source: int) -> np.ndarray:
    lib = _load()
    e = _sorted(edges)
    out = np.zeros(V, np.int32)
    lib.orc_bfs(V, _p(e, C.c_uint64), e.size, source, _p(out, C.c_int32))
    return out


def cc(V: int, edges) -> np.ndarray:
    lib = _load()
    e = _sorted(edges)
    out = np.zeros(V, np.uint32)
    lib.orc_cc(V, _p(e, C.c_uint64), e.size, _p(out, C.c_uint32))
    return out
