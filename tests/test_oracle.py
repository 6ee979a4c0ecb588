"""Pins of the CPU oracle against what the paper and the mathematics fix.

Nothing here touches the GPU library.  Each test names the passage or the
independent fact it checks; together they are chosen so that a plausible
slip in the oracle (a wrong bound, a wrong re-dispatch, a wrong leaf rule, a
dropped PageRank term, a transposed adjacency, a directed/undirected mix-up)
fails at least one of them.
"""
import itertools
import json
import os
from fractions import Fraction

import numpy as np
import pytest

import oracle as O
from conftest import GOLDEN

U64 = np.uint64
E = 0xFFFFFFFFFFFFFFFF


def golden(name):
    with open(os.path.join(GOLDEN, name)) as f:
        return json.load(f)


def slots_from_json(vals):
    return np.array([E if v is None else v for v in vals], dtype=np.uint64)


def key(u, v):
    return (int(u) << 32) | int(v)


# --------------------------------------------------------------------------
# density bounds: figure "PMA insertion example" (Section 4.1)

def test_threshold_rows_match_figure():
    g = golden("threshold_table.json")
    lf, H = g["leaf_size"], g["height"]
    mn, mx = O.level_bounds(lf, H)
    for h in range(H + 1):
        cap = g["segment_size"][h]
        assert cap == lf << h
        # the printed rho/tau are rounded to two decimals: the integer bounds
        # must be the strict bounds of some rho, tau inside that rounding
        # interval (Algorithm GPMA+ tests (n_s+|U_s|)/cap < tau)
        t_lo, t_hi = Fraction(g["tau"][h]) - Fraction(1, 200), Fraction(g["tau"][h]) + Fraction(1, 200)
        r_lo, r_hi = Fraction(g["rho"][h]) - Fraction(1, 200), Fraction(g["rho"][h]) + Fraction(1, 200)
        assert Fraction(int(mx[h])) < t_hi * cap and Fraction(int(mx[h]) + 1) >= t_lo * cap
        assert Fraction(int(mn[h])) > r_lo * cap and Fraction(int(mn[h]) - 1) <= r_hi * cap
    # where the figure's count rows agree with its rho/tau rows they must match
    assert int(mx[0]) == g["max_entries"][0]
    assert int(mn[0]) == g["min_entries"][0] and int(mn[1]) == g["min_entries"][1]


def test_threshold_interpolation_is_linear_in_height():
    # leaf and root rows of the figure; the middle rows are their linear
    # interpolation rounded to two decimals (0.1867 -> 0.19, 0.2933 -> 0.29)
    g = golden("threshold_table.json")
    H = g["height"]
    for h in range(H + 1):
        rho = Fraction(g["rho"][0]) + (Fraction(g["rho"][H]) - Fraction(g["rho"][0])) * h / H
        tau = Fraction(g["tau"][0]) + (Fraction(g["tau"][H]) - Fraction(g["tau"][0])) * h / H
        assert round(float(rho), 2) == g["rho"][h]
        assert round(float(tau), 2) == g["tau"][h]
    # and the oracle's bound at a big segment converges on tau_h * cap_h
    lf, H2 = 1 << 12, 4
    mn, mx = O.level_bounds(lf, H2)
    for h in range(H2 + 1):
        tau = 0.92 + (0.80 - 0.92) * h / H2
        rho = 0.08 + (0.40 - 0.08) * h / H2
        cap = lf << h
        assert abs(int(mx[h]) - tau * cap) <= 1.0
        assert abs(int(mn[h]) - rho * cap) <= 1.0


def test_single_level_tree_uses_root_bounds():
    mn, mx = O.level_bounds(16, 0)
    assert int(mx[0]) == 12          # largest m < 0.80 * 16 = 12.8
    assert int(mn[0]) == 7           # smallest m > 0.40 * 16 = 6.4


# --------------------------------------------------------------------------
# CSR on GPMA: figure "GPMA based on CSR" (Section 4.2)

def test_csr_example_row_offsets():
    g = golden("csr_example.json")
    V = g["num_vertices"]
    off, col = g["row_offset"], g["column_index"]
    edges = [key(u, col[i]) for u in range(V) for i in range(off[u], off[u + 1])]
    p = O.OraclePMA(V, np.array(edges[::-1], dtype=np.uint64), 16)
    s = p.slots()
    O.check_invariants(s, 16, V)
    comp = O.stored(s)
    guard = (comp & U64(0xFFFFFFFF)) == U64(0xFFFFFFFF)
    # compacted array with guards: [0->0, 0->2, G0, 1->2, G1, 2->0, 2->1, 2->2, G2]
    assert [int(x) for x in np.nonzero(guard)[0]] == [2, 4, 8]
    # row offsets over the compacted array, guards dropped, equal the figure
    rows = (comp >> U64(32)).astype(np.int64)
    plain = np.zeros(V + 1, np.int64)
    np.add.at(plain, rows[~guard] + 1, 1)
    assert list(np.cumsum(plain)) == off
    assert [int(x & U64(0xFFFFFFFF)) for x in comp[~guard]] == col
    # the gapped row offsets bracket exactly the rows' entries and guards
    ro = O.row_offsets(s, V)
    for u in range(V):
        seg = s[ro[u]:ro[u + 1]]
        seg = seg[seg != U64(E)]
        assert int(seg[-1]) == key(u, 0xFFFFFFFF)
        assert [int(x & U64(0xFFFFFFFF)) for x in seg[:-1]] == col[off[u]:off[u + 1]]


# --------------------------------------------------------------------------
# worked examples of the update

def test_example1_sequential_pma_insert_climbs_to_16_31():
    g = golden("example1_pma_insert.json")
    p = O.OraclePMA.from_slots(slots_from_json(g["slots"]), g["leaf_size"])
    p.insert(np.array(g["insert"], dtype=np.uint64))
    assert [list(m) for m in p.merge_log()] == g["expected_merges"]
    h, s = g["expected_merges"][0]
    lo = s * (g["leaf_size"] << h)
    assert [lo, lo + (g["leaf_size"] << h) - 1] == g["expected_segment_interval"]
    out = p.slots()
    # untouched left half; right half re-dispatched evenly: 12 entries, 3 per leaf
    assert np.array_equal(out[:16], slots_from_json(g["slots"])[:16])
    right = out[16:].reshape(4, 4)
    assert list((right != U64(E)).sum(1)) == [3, 3, 3, 3]
    assert [int(x) for x in O.stored(out[16:])] == [40, 45, 47, 48, 50, 52, 54, 56, 60, 62, 70, 72]


def test_example3_gpmaplus_rounds():
    g = golden("example3_gpmaplus_insert.json")
    init = slots_from_json(g["slots"])
    p = O.OraclePMA.from_slots(init, g["leaf_size"])
    p.insert(np.array(g["insert"], dtype=np.uint64))
    assert [list(m) for m in p.merge_log()] == g["expected_merges"]
    out = p.slots()
    want = sorted(set(int(x) for x in O.stored(init)) | set(g["insert"]))
    assert [int(x) for x in O.stored(out)] == want
    assert list((out.reshape(8, 4) != U64(E)).sum(1)) == [3] * 8


def test_example3_under_a_successor_leaf_rule_would_differ():
    # the leaf rule matters: 4 has predecessor 0 (leaf 0) but successor 5
    # (leaf 1); the paper merges {1,4} together at the leaf level
    g = golden("example3_gpmaplus_insert.json")
    p = O.OraclePMA.from_slots(slots_from_json(g["slots"]), g["leaf_size"])
    p.insert(np.array([4], dtype=np.uint64))
    assert p.merge_log() == [(0, 0)]


def test_delete_dual_bounds_at_equality_and_uneven_split():
    """Deletions (the dual of insertions, Section 4.1): a failed leaf hands
    its deletions to its parent, a segment passes when the live count after
    the deletions still reaches min_h (three segments pass exactly at their
    bound), and an odd count is re-dispatched floor-evenly."""
    g = golden("delete_dual_uneven.json")
    lf = g["leaf_size"]
    mn, _ = O.level_bounds(lf, 3)
    assert [int(x) for x in mn] == g["min_entries"]
    p = O.OraclePMA.from_slots(slots_from_json(g["slots"]), lf)
    p.delete(np.array(g["delete"], dtype=np.uint64))
    assert [list(m) for m in p.merge_log()] == g["expected_merges"]
    assert np.array_equal(p.slots(), slots_from_json(g["expected_slots"]))
    assert p.last_applied() == len(g["delete"])


def test_insert_bound_at_equality_and_uneven_split():
    g = golden("insert_uneven_dispatch.json")
    lf = g["leaf_size"]
    _, mx = O.level_bounds(lf, 3)
    assert [int(x) for x in mx] == g["max_entries"]
    p = O.OraclePMA.from_slots(slots_from_json(g["slots"]), lf)
    p.insert(np.array(g["insert"], dtype=np.uint64))
    assert [list(m) for m in p.merge_log()] == g["expected_merges"]
    assert np.array_equal(p.slots(), slots_from_json(g["expected_slots"]))


def test_even_dispatch_counts_closed_form():
    """Bulk load spreads n entries over the L leaves of the array: leaf j
    holds floor((j+1)n/L) - floor(jn/L) of them, in key order, packed at the
    front (the reading of "re-dispatch evenly"), for every n up to a few
    arrays' worth, including the uneven ones."""
    lf = 4
    for n in range(1, 200):
        keys = np.arange(3, 3 + 7 * n, 7, dtype=np.uint64)
        p = O.OraclePMA(0, keys, lf)
        s = p.slots()
        L = s.size // lf
        want = [(j + 1) * n // L - j * n // L for j in range(L)]
        assert list(O.leaf_counts(s, lf)) == want, n
        assert np.array_equal(O.stored(s), keys)
        O.check_invariants(s, lf, allow_empty_leaves=True)


def test_leaf_pivots_are_leaf_minima_and_locate_by_them():
    """A leaf's pivot is the smallest key it holds (marked entries by their
    key), so the pivots ascend, and the predecessor-leaf rule (Example 3:
    the leaf holding the greatest stored key <= k, leaf 0 if none) is a
    search over them: checked by brute force over every leaf for keys
    below, between and above the stored ones, after lazy marks."""
    rng = np.random.default_rng(11)
    lf, V = 8, 40
    keys = np.unique(rng.integers(0, V, 300).astype(np.uint64) << np.uint64(32)
                     | rng.integers(0, V, 300).astype(np.uint64))
    p = O.OraclePMA(V, keys, lf, lazy=True)
    p.delete(keys[::3])
    s = p.slots()
    piv = O.leaf_pivots(s, lf)
    leaves = s.reshape(-1, lf)
    for j in range(leaves.shape[0]):
        occ = leaves[j][leaves[j] != O.EMPTY] & ~O.TOMB
        assert occ.size and piv[j] == occ.min()
    assert np.all(piv[1:] > piv[:-1])
    occ_all = O.occupied(s)
    for k in np.concatenate([occ_all, occ_all + np.uint64(1), [np.uint64(0)]]):
        owner = [j for j in range(leaves.shape[0])
                 if np.any((leaves[j] != O.EMPTY) & ((leaves[j] & ~O.TOMB) <= k))]
        want = max(owner) if owner else 0
        got = max(int(np.searchsorted(piv, k, side="right")) - 1, 0)
        assert got == want, k


def test_eager_mode_keeps_keys_with_the_top_bit():
    """Bit 63 marks a lazily deleted entry only in lazy mode; an eager array
    of raw keys stores, merges and deletes keys >= 2^63 like any other, and
    lazy mode refuses an array whose keys may use that bit."""
    lf = 4
    top = 1 << 63
    init = [top + 5 * i for i in range(20)] + list(range(0, 40, 4))
    p = O.OraclePMA(0, np.array(init, dtype=np.uint64), lf)
    ref = set(init)
    rng = np.random.default_rng(11)
    for t in range(30):
        ks = [int(x) | (top if rng.random() < 0.5 else 0) for x in rng.integers(0, 200, 9)]
        if t % 2:
            p.insert(np.array(ks, dtype=np.uint64))
            ref |= set(ks)
        else:
            p.delete(np.array(ks + sorted(ref)[::5], dtype=np.uint64))
            ref -= set(ks + sorted(ref)[::5])
        s = p.slots()
        assert [int(x) for x in s[s != O.EMPTY]] == sorted(ref)
    with pytest.raises(O.OracleError):
        O.OraclePMA(0, np.array(init, dtype=np.uint64), lf, lazy=True)
    with pytest.raises(O.OracleError):
        O.OraclePMA((1 << 31) + 1, np.array([], dtype=np.uint64), 16)


def _frac_bounds(lf, H, h, pm=O.DEFAULT_PM):
    """rho_h * cap_h and tau_h * cap_h as exact fractions (linear in the
    height between the figure's leaf and root values; one leaf = the root)."""
    cap = Fraction(lf << h)
    if H == 0:
        return Fraction(pm["rho_root"], 1000) * cap, Fraction(pm["tau_root"], 1000) * cap
    rho = (Fraction(pm["rho_leaf"]) * (H - h) + Fraction(pm["rho_root"]) * h) / (1000 * H)
    tau = (Fraction(pm["tau_leaf"]) * (H - h) + Fraction(pm["tau_root"]) * h) / (1000 * H)
    return rho * cap, tau * cap


def assert_merge_log(p, lf, cap_before, delete):
    """Invariants (vi) and (vii) of a batch, from the oracle's merge log and
    exact fractions: every segment merged at height h met its bound at merge
    time (insert: (n_s+k)/cap_h < tau_h; delete: (n_s-k)/cap_h > rho_h); a
    root rebuild leaves n' < tau_root * cap' at the capacity the resize rule
    picks (a grown root is the smallest power of two that holds n'; a shrunk
    root stops halving once n' clears rho_root or the half would overflow)."""
    H = int(np.log2(cap_before // lf))
    for (lvl, seg), (ns, k) in zip(p.merge_log(), p.merge_log_counts()):
        if lvl >= 0:
            assert seg < (cap_before // lf) >> lvl
            rho_c, tau_c = _frac_bounds(lf, H, lvl)
            if delete:
                assert ns - k > rho_c, (lvl, seg, ns, k)
            else:
                assert ns + k < tau_c, (lvl, seg, ns, k)
        else:
            ncap = seg
            n2 = ns - k if delete else ns + k
            Hn = int(np.log2(ncap // lf))
            rho_c, tau_c = _frac_bounds(lf, Hn, Hn)
            assert n2 < tau_c
            if ncap > cap_before:
                assert n2 >= _frac_bounds(lf, Hn - 1, Hn - 1)[1]
            elif ncap < cap_before and ncap > lf:
                assert n2 > rho_c or n2 >= _frac_bounds(lf, Hn - 1, Hn - 1)[1]


# --------------------------------------------------------------------------
# set semantics by brute force, invariants after every batch

def _check(p, ref, V, lf):
    s = p.slots()
    O.check_invariants(s, lf, V)
    assert [int(x) for x in O.edge_keys(s)] == sorted(ref)
    assert p.size == len(ref) + V
    # per-level bounds are checked only where a merge happens, so the root may
    # sit above its own bound after leaf-level merges; only cap bounds size
    assert p.size <= p.capacity


def test_exhaustive_tiny_graphs():
    V, lf = 2, 16
    universe = [key(u, v) for u in range(V) for v in range(V)]
    subsets = [set(c) for r in range(len(universe) + 1) for c in itertools.combinations(universe, r)]
    for init in subsets:
        for batch in subsets:
            for op in ("insert", "delete"):
                p = O.OraclePMA(V, np.array(sorted(init), dtype=np.uint64), lf)
                getattr(p, op)(np.array(sorted(batch) * 2, dtype=np.uint64))
                ref = init | batch if op == "insert" else init - batch
                _check(p, ref, V, lf)
                changed = len(batch - init) if op == "insert" else len(batch & init)
                assert p.last_applied() == changed
                assert p.last_noops() == 2 * len(batch) - changed


@pytest.mark.parametrize("seed,V,lf", [(1, 8, 16), (2, 32, 16), (3, 64, 32), (4, 300, 16)])
def test_random_batches_vs_set(seed, V, lf):
    rng = np.random.default_rng(seed)

    def rnd(n):
        return [key(a, b) for a, b in zip(rng.integers(0, V, n), rng.integers(0, V, n))]

    ref = set(rnd(3 * V))
    p = O.OraclePMA(V, np.array(list(ref), dtype=np.uint64), lf)
    _check(p, ref, V, lf)
    for t in range(40):
        b = int(rng.integers(1, 4 * V))
        cap0 = p.capacity
        if rng.random() < 0.5:
            ins = rnd(b)
            p.insert(np.array(ins, dtype=np.uint64))
            ref |= set(ins)
            assert_merge_log(p, lf, cap0, False)
        else:
            pool = sorted(ref)
            dl = [pool[i] for i in rng.integers(0, len(pool), b)] if pool else []
            dl += rnd(b // 4)     # some absent keys: no-ops
            p.delete(np.array(dl, dtype=np.uint64))
            ref -= set(dl)
            assert_merge_log(p, lf, cap0, True)
        _check(p, ref, V, lf)


def test_growth_and_shrink_resize_rules():
    V, lf = 16, 16
    p = O.OraclePMA(V, [], lf)
    ref = set()
    caps = [p.capacity]
    allk = [key(u, v) for u in range(V) for v in range(V)]
    rng = np.random.default_rng(7)
    rng.shuffle(allk)
    for i in range(0, len(allk), 23):
        cap0 = p.capacity
        p.insert(np.array(allk[i:i + 23], dtype=np.uint64))
        ref |= set(allk[i:i + 23])
        _check(p, ref, V, lf)
        assert_merge_log(p, lf, cap0, False)
        caps.append(p.capacity)
        for lvl, seg in p.merge_log():
            if lvl < 0:    # a root rebuild: the new capacity is the smallest that fits
                mn, mx = O.level_bounds(lf, int(np.log2(seg // lf)))
                assert p.size <= int(mx[-1])
                if seg > lf:
                    mn2, mx2 = O.level_bounds(lf, int(np.log2(seg // 2 // lf)))
                    assert p.size > int(mx2[-1])
    assert caps == sorted(caps) and caps[-1] > caps[0]
    for i in range(0, len(allk), 31):
        cap0 = p.capacity
        p.delete(np.array(allk[i:i + 31], dtype=np.uint64))
        ref -= set(allk[i:i + 31])
        _check(p, ref, V, lf)
        assert_merge_log(p, lf, cap0, True)
        for lvl, seg in p.merge_log():
            if lvl < 0 and seg > lf:
                mn, mx = O.level_bounds(lf, int(np.log2(seg // lf)))
                assert p.size >= int(mn[-1])
    assert p.capacity < caps[-1]


def test_semantic_set_against_python_sets_and_layout_oracle():
    """The sorted-vector set follows Python's set union / difference batch
    by batch (repeats, absent deletes, present inserts), reports how many
    keys changed the set, and holds exactly the layout oracle's edges."""
    rng = np.random.default_rng(12)
    V = 50
    def rnd(n):
        return [key(a, b) for a, b in zip(rng.integers(0, V, n), rng.integers(0, V, n))]
    init = rnd(400)
    s = O.OracleSet(np.array(init, dtype=np.uint64))
    p = O.OraclePMA(V, np.array(init, dtype=np.uint64), 16)
    ref = set(init)
    assert [int(x) for x in s.keys()] == sorted(ref)
    for t in range(60):
        b = rnd(int(rng.integers(0, 300)))
        if t % 3 == 2:
            b += sorted(ref)[::7]
            changed = s.delete(np.array(b, dtype=np.uint64))
            p.delete(np.array(b, dtype=np.uint64))
            assert changed == len(ref & set(b))
            ref -= set(b)
        else:
            changed = s.insert(np.array(b, dtype=np.uint64))
            p.insert(np.array(b, dtype=np.uint64))
            assert changed == len(set(b) - ref)
            ref |= set(b)
        assert [int(x) for x in s.keys()] == sorted(ref)
        assert np.array_equal(s.keys(), O.edge_keys(p.slots()))


def test_invalid_keys_leave_state_unchanged():
    p = O.OraclePMA(4, [key(0, 1), key(1, 2)], 16)
    before = p.slots()
    for bad in (key(4, 0), key(0, 4), key(1, 0xFFFFFFFF)):
        with pytest.raises(O.OracleError):
            p.insert(np.array([key(2, 3), bad], dtype=np.uint64))
        with pytest.raises(O.OracleError):
            p.delete(np.array([key(0, 1), bad], dtype=np.uint64))
    assert np.array_equal(p.slots(), before)


def test_amortized_work_grows_slowly():
    # Lemma (Section 4.1) / Theorem 1 (Section 5.2): work per update is
    # polylogarithmic; the slots rewritten per applied update stay far below
    # the array size as the array grows
    rng = np.random.default_rng(3)
    for V in (64, 256):
        keys = [key(a, b) for a, b in zip(rng.integers(0, V, 20 * V), rng.integers(0, V, 20 * V))]
        p = O.OraclePMA(V, keys[: 10 * V], 16)
        work = applied = 0
        for i in range(10 * V, 20 * V, 32):
            p.insert(np.array(keys[i:i + 32], dtype=np.uint64))
            applied += p.last_applied()
            for lvl, seg in p.merge_log():
                work += (16 << lvl) if lvl >= 0 else seg
        assert applied > 0 and work / applied < p.capacity / 8


# --------------------------------------------------------------------------
# PageRank (Section 6.1): fp64 power iteration

def google_matrix(V, edges, d):
    A = np.zeros((V, V))
    for k in edges:
        A[k >> 32, k & 0xFFFFFFFF] = 1.0
    deg = A.sum(1)
    P = np.where(deg[:, None] > 0, A / np.maximum(deg, 1)[:, None], 1.0 / V)
    return d * P.T + (1 - d) / V


def test_pagerank_cycle_and_edgeless_are_uniform():
    V = 7
    cyc = [key(i, (i + 1) % V) for i in range(V)]
    np.testing.assert_allclose(O.pagerank(V, cyc, iters=10), np.full(V, 1 / V), rtol=1e-14)
    np.testing.assert_allclose(O.pagerank(V, [], iters=10), np.full(V, 1 / V), rtol=1e-14)


def test_pagerank_is_stationary_vector_of_google_matrix():
    rng = np.random.default_rng(5)
    V = 40
    edges = sorted({key(a, b) for a, b in zip(rng.integers(0, V, 150), rng.integers(0, V // 2, 150))})
    x = O.pagerank(V, edges, iters=300)
    G = google_matrix(V, edges, 0.85)
    w, vecs = np.linalg.eig(G)
    v = np.real(vecs[:, np.argmax(np.real(w))])
    v = v / v.sum()
    np.testing.assert_allclose(x, v, rtol=1e-9)
    assert abs(x.sum() - 1) < 1e-12


def test_pagerank_single_step_matches_matrix_form():
    rng = np.random.default_rng(6)
    V = 25
    edges = sorted({key(a, b) for a, b in zip(rng.integers(0, V, 60), rng.integers(0, V, 60))})
    x0 = rng.random(V)
    x0 /= x0.sum()
    got = O.pagerank(V, edges, x0=x0, iters=1, damping=0.7)
    want = google_matrix(V, edges, 0.7) @ x0
    np.testing.assert_allclose(got, want, rtol=1e-12)


# --------------------------------------------------------------------------
# BFS (Algorithm "Breadth-First Search", Section 4.2) and CC (Section 6.1)

def test_bfs_closed_forms():
    V = 10
    path = [key(i, i + 1) for i in range(V - 1)]
    assert list(O.bfs(V, path, 0)) == list(range(V))
    assert list(O.bfs(V, path, 4)) == [-1] * 4 + list(range(V - 4))   # directed
    star = [key(0, i) for i in range(1, V)]
    assert list(O.bfs(V, star, 0)) == [0] + [1] * (V - 1)
    assert list(O.bfs(V, star, 3)) == [-1, -1, -1, 0] + [-1] * (V - 4)


def test_bfs_matches_boolean_matrix_powers():
    rng = np.random.default_rng(8)
    V = 30
    edges = sorted({key(a, b) for a, b in zip(rng.integers(0, V, 45), rng.integers(0, V, 45))})
    A = np.zeros((V, V), dtype=np.int64)
    for k in edges:
        A[k >> 32, k & 0xFFFFFFFF] = 1
    for src in (0, 3, 17):
        want = np.full(V, -1)
        reach = np.zeros(V, dtype=np.int64)
        reach[src] = 1
        seen = reach.copy()
        want[src] = 0
        for dist in range(1, V):
            reach = ((reach @ A) > 0).astype(np.int64) & (1 - seen)
            want[reach > 0] = dist
            seen |= reach
        assert list(O.bfs(V, edges, src)) == list(want)


def test_cc_closed_forms_and_scipy():
    V = 12
    cyc = [key(i, (i + 1) % 4) for i in range(4)] + [key(4 + (i + 1) % 4, 4 + i) for i in range(4)]
    lab = O.cc(V, cyc)
    assert list(lab) == [0] * 4 + [4] * 4 + list(range(8, 12))
    full = [key(u, v) for u in range(V) for v in range(V) if u != v]
    assert list(O.cc(V, full)) == [0] * V
    from scipy.sparse import coo_matrix
    from scipy.sparse.csgraph import connected_components
    rng = np.random.default_rng(9)
    V = 200
    edges = sorted({key(a, b) for a, b in zip(rng.integers(0, V, 150), rng.integers(0, V, 150))})
    src = np.array([k >> 32 for k in edges])
    dst = np.array([k & 0xFFFFFFFF for k in edges])
    M = coo_matrix((np.ones(len(edges)), (src, dst)), shape=(V, V))
    n, comp = connected_components(M, directed=True, connection="weak")
    want = np.array([np.min(np.nonzero(comp == comp[v])[0]) for v in range(V)])
    assert np.array_equal(O.cc(V, edges), want)
    assert len(set(O.cc(V, edges))) == n


def test_stream_generators_explicit_deletions_and_sorted_arrivals():
    """Input recipes of the extended workloads: explicit deletions remove
    distinct edges that are live at that slide; sorted arrivals keep the
    window and order the arrivals by key."""
    import torch

    import synth
    st = synth.rmat_stream(11, 16, 4)
    slides = synth.explicit_deletion_slides(st.initial(), st.order[st.window:], 200, 5, 9)
    live = set(st.initial().tolist())
    for d, i in slides:
        d = d.tolist()
        assert len(set(d)) == len(d) == 200 and set(d) <= live
        live -= set(d)
        live |= set(i.tolist())
    s2 = synth.sorted_stream(st)
    assert torch.equal(s2.initial(), st.initial())
    arr = s2.order[s2.window:]
    assert bool((arr[1:] >= arr[:-1]).all())
    assert sorted(arr.tolist()) == sorted(st.order[st.window:].tolist())


# --------------------------------------------------------------------------
# lazy deletion (Section 6: deleted entries are marked in place, without
# density maintenance, and their slots are recycled by later insertions)

def _lazy_pair(V, init, lf, seed):
    rng = np.random.default_rng(seed)
    lazy = O.OraclePMA(V, init, lf, lazy=True)
    eager = O.OraclePMA(V, init, lf)
    return rng, lazy, eager


def test_lazy_deletion_marks_only_the_deleted_entries():
    V, lf = 64, 16
    init = np.unique(np.array([(a << 32) | b for a in range(V) for b in range(0, V, 5)], np.uint64))
    _, lazy, _ = _lazy_pair(V, init, lf, 0)
    before = lazy.slots()
    dels = init[::7]
    absent = np.array([(3 << 32) | 1], np.uint64)
    lazy.delete(np.concatenate([dels, dels[:5], absent]))
    after = lazy.slots()
    changed = np.nonzero(before != after)[0]
    assert np.array_equal(np.sort(before[changed]), np.sort(dels))      # exactly the deleted keys
    assert np.all(after[changed] == (before[changed] | O.TOMB))          # marked, not moved
    assert lazy.last_applied() == dels.size
    assert lazy.capacity == O.OraclePMA(V, init, lf).capacity           # no density maintenance
    O.check_invariants(after, lf, V)
    assert np.array_equal(O.edge_keys(after), np.setdiff1d(init, dels))


def test_lazy_deletion_against_sets_and_eager_mode():
    """Random sequences of lazy deletes and inserts: the live edges equal a
    Python set (and the eager PMA's edges) after every batch; the structural
    invariants hold with marked entries in place; re-inserting a deleted key
    brings it back."""
    for seed in range(4):
        V, lf = 40, 16
        rng = np.random.default_rng(seed)
        init = np.unique(rng.integers(0, V, (300, 2)).astype(np.uint64) @ np.array([1 << 32, 1], np.uint64))
        lazy = O.OraclePMA(V, init, lf, lazy=True)
        eager = O.OraclePMA(V, init, lf)
        live = set(int(x) for x in init)
        for t in range(40):
            if rng.random() < 0.5 and live:
                pool = np.array(sorted(live), np.uint64)
                b = np.concatenate([pool[rng.choice(pool.size, min(pool.size, int(rng.integers(1, 60))),
                                                   replace=False)],
                                    rng.integers(0, V, (5, 2)).astype(np.uint64) @ np.array([1 << 32, 1],
                                                                                           np.uint64)])
                lazy.delete(b)
                eager.delete(b)
                live -= set(int(x) for x in b)
            else:
                b = rng.integers(0, V, (int(rng.integers(1, 120)), 2)).astype(np.uint64) @ \
                    np.array([1 << 32, 1], np.uint64)
                lazy.insert(b)
                eager.insert(b)
                live |= set(int(x) for x in b)
            s = lazy.slots()
            O.check_invariants(s, lf, V)
            want = np.array(sorted(live), np.uint64)
            assert np.array_equal(O.edge_keys(s), want), (seed, t)
            assert np.array_equal(O.edge_keys(eager.slots()), want)


def test_lazy_insert_merge_recycles_marked_slots():
    """An insert merged into a leaf drops the marked entries of that leaf; a
    deleted key inserted again is live once, mark gone."""
    V, lf = 8, 16
    init = np.array([(0 << 32) | v for v in range(7)], np.uint64)
    lazy = O.OraclePMA(V, init, lf, lazy=True)
    lazy.delete(init[[1, 3, 5]])
    s = lazy.slots()
    assert ((s & O.TOMB) != 0).sum() - (s == O.EMPTY).sum() == 3
    lazy.insert(np.array([init[3]], np.uint64))
    s = lazy.slots()
    assert ((s != O.EMPTY) & ((s & O.TOMB) != 0)).sum() == 0               # marks dropped by the merge
    assert np.array_equal(O.edge_keys(s), np.sort(init[[0, 2, 3, 4, 6]]))
    O.check_invariants(s, lf, V)
