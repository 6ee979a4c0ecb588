"""The C-ABI library loads and exports every entry point include/gpma.h
declares (no compute call: runs without a GPU)."""
import ctypes
import os
import re

import pytest

from conftest import ROOT

HEADER = os.path.join(ROOT, "include", "gpma.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"\b(gpma_[a-z_]+)\s*\(", text)
    return sorted(set(names))


def test_header_declares_the_boundary():
    names = declared_functions()
    for must in ("gpma_create", "gpma_insert_batch", "gpma_delete_batch", "gpma_pagerank",
                 "gpma_bfs", "gpma_cc", "gpma_destroy"):
        assert must in names


def test_library_exports_every_declared_symbol():
    from paper_1709_05061_amd import gpma
    if not os.path.exists(gpma.LIB_PATH):
        pytest.skip("libgpma.so not built")
    lib = ctypes.CDLL(gpma.LIB_PATH)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing
    assert sorted(gpma.exported_symbols()) == declared_functions()


def test_product_path_has_no_oracle_dependency():
    pkg = os.path.join(ROOT, "paper_1709_05061_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".h", ".cpp")):
                txt = open(os.path.join(dirpath, f)).read()
                assert "import oracle" not in txt and "from oracle" not in txt, f
                assert "liboracle" not in txt and "gpma_oracle" not in txt, f


def test_thresholds_agree_with_oracle_via_params_validation():
    # host logic without a GPU: default params are the figure's values
    from paper_1709_05061_amd import gpma
    if not os.path.exists(gpma.LIB_PATH):
        pytest.skip("libgpma.so not built")
    p = gpma.gpma_default_params()
    assert (p.leaf_size, p.tau_leaf_pm, p.tau_root_pm, p.rho_leaf_pm, p.rho_root_pm) == (0, 920, 800, 80, 400)


def test_batch_stats_keep_levels_up_to_the_last_merge():
    # host logic of the binding: the per-level merge counts of gpma_stats are
    # cut after the last nonzero level, whatever the values' byte patterns
    import random
    from paper_1709_05061_amd import gpma
    rng = random.Random(5)
    values = [0, 0, 1, 255, 256, 1 << 24, 1 << 32, (1 << 63) + 1, (1 << 64) - 1]
    for _ in range(500):
        st = gpma.gpma_stats()
        L = len(st.segments_merged)
        want = [rng.choice(values) for _ in range(rng.randrange(0, L + 1))]
        for j, v in enumerate(want):
            st.segments_merged[j] = v
        while want and want[-1] == 0:
            want.pop()
        assert gpma.BatchStats.of(st).segments_merged == want
    assert gpma.BatchStats.of(gpma.gpma_stats()).segments_merged == []


def test_missing_library_fails_loudly(monkeypatch):
    # no fallback path: without the built library every entry point raises
    from paper_1709_05061_amd import gpma
    monkeypatch.setattr(gpma, "_lib", None)
    monkeypatch.setattr(gpma, "LIB_PATH", os.path.join(ROOT, "no_such_dir", "libgpma.so"))
    with pytest.raises(RuntimeError, match="not built"):
        gpma.load_library()


@pytest.mark.parametrize("argv,env", [(["--gpus", "2"], {}), (["--gpus", "8"], {}), ([], {"WORLD_SIZE": "2"})])
def test_bench_refuses_more_than_one_gpu(argv, env):
    # one GPU only: the bench exits with a message before it touches a device
    import subprocess
    import sys
    e = dict(os.environ, **env)
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), *argv], capture_output=True, text=True,
                       env=e, timeout=120)
    assert r.returncode == 2
    assert "one GPU only" in r.stderr
    assert r.stdout == ""
