"""gpma_bfs_noalloc (scratch in the library's fixed per-GPU device array,
nothing allocated by the call) against gpma_bfs on the same handle, both
through the C ABI: bit-exact hop distances on two calls in a row, the second
on a smaller graph, with and without the dst-major mirror (whose bottom-up
levels read it), at the array's vertex limit, and the refusal just above it.
"""
import ctypes as C
import sys

import numpy as np
import pytest
import torch

import oracle as O
import synth

pytestmark = pytest.mark.gpu

MAX_V = 1 << 22


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def both(lib, g, src):
    s = torch.cuda.current_stream()
    a = torch.full((g.V,), -7, dtype=torch.int32, device="cuda")
    b = torch.full((g.V,), -9, dtype=torch.int32, device="cuda")
    assert lib.gpma_bfs(g.h, src, C.c_void_p(a.data_ptr()), C.c_void_p(s.cuda_stream)) == 0
    assert lib.gpma_bfs_noalloc(g.h, src, C.c_void_p(b.data_ptr()), C.c_void_p(s.cuda_stream)) == 0
    return a.cpu().numpy(), b.cpu().numpy()


def source_with_edges(keys, V, seed):
    src = np.unique((keys >> np.uint64(32)).astype(np.int64))
    return int(src[seed % src.size])


@pytest.mark.parametrize("mirror", [False, True])
def test_bfs_noalloc_equals_bfs_two_calls(mirror):
    from paper_1709_05061_amd import GPMA
    from paper_1709_05061_amd.gpma import load_library
    lib = load_library()
    for scale, seed in ((18, 3), (11, 4)):      # the second graph is smaller
        say("noalloc bfs: R-MAT scale", scale, "seed", seed, "mirror", mirror)
        st = synth.rmat_stream(scale, 16, seed=seed, device="cuda")
        init = st.initial()
        g = GPMA(st.V, init, mirror=mirror)
        keys = init.cpu().numpy().view(np.uint64)
        for k in range(2):
            src = source_with_edges(keys, st.V, seed + k)
            a, b = both(lib, g, src)
            assert np.array_equal(a, b), (scale, src)
            if scale == 11:
                assert np.array_equal(b, O.bfs(st.V, np.unique(keys), src))
        g.close()


def test_bfs_noalloc_at_the_vertex_limit_and_above():
    from paper_1709_05061_amd import GPMA
    from paper_1709_05061_amd.gpma import GPMA_EINVAL, load_library
    lib = load_library()
    say("noalloc bfs: V = 2^22, random graph")
    init = synth.random_batch(MAX_V, 1 << 22, 21).cuda()
    g = GPMA(MAX_V, init, mirror=True)
    keys = init.cpu().numpy().view(np.uint64)
    a, b = both(lib, g, source_with_edges(keys, MAX_V, 5))
    assert np.array_equal(a, b)
    g.close()
    say("noalloc bfs: V = 2^22 + 1 is refused")
    g = GPMA(MAX_V + 1, init[:1000])
    d = torch.full((MAX_V + 1,), 3, dtype=torch.int32, device="cuda")
    s = torch.cuda.current_stream()
    assert lib.gpma_bfs_noalloc(g.h, 0, C.c_void_p(d.data_ptr()), C.c_void_p(s.cuda_stream)) == GPMA_EINVAL
    assert int((d != 3).sum()) == 0
    g.close()
