"""Pins of the FP64 oracle against things other than itself.

* a hand-computed worked example (tests/golden/worked_example.json)
* closed forms: single-tip samples, disjoint root subtrees
* brute force (tip sets by walking parent pointers) on random small trees,
  including multifurcations, unary nodes, zero lengths and shuffled ids
* library routines: scipy's weighted Jaccard / Bray-Curtis on star trees, the
  1-Wasserstein distance on caterpillar trees, a scipy.sparse Gram product
* the Gower centring identity for the PCoA means
* invariants and metamorphic relations of the definitions
Each pin is chosen so that a plausible slip (a dropped or extra branch, the
root branch counted, a swapped operand, max vs sum in a denominator, a wrong
index in the layout) fails at least one test.
"""
import json
import os
from fractions import Fraction

import numpy as np
import pytest
import scipy.sparse as sp
from hypothesis import given, settings, strategies as st
from scipy.spatial.distance import braycurtis, jaccard
from scipy.stats import wasserstein_distance

import oracle
import synth
from oracle import brute, core
from tests import _util

HERE = os.path.dirname(os.path.abspath(__file__))
VARIANTS = ("unweighted", "weighted_normalized")


@pytest.fixture(scope="module", autouse=True)
def _build_core():
    core.build(force=False)


# ---------------------------------------------------------------- worked example
def test_worked_example():
    g = json.load(open(os.path.join(HERE, "golden", "worked_example.json")))
    name_to_id = {n: k for k, n in enumerate(g["nodes"])}
    t = _util.tree(g["parent"], g["length"])
    for case in g["cases"]:
        rows = [{name_to_id[k]: v for k, v in g["samples"][s].items()} for s in case["pair"]]
        tab = _util.table(rows)
        for var in VARIANTS:
            want = float(Fraction(case[var]))
            assert oracle.dm(t, tab, var)[0] == pytest.approx(want, abs=1e-15), (case, var)
            assert brute.dm(t.parent, t.length, rows, var)[0] == pytest.approx(want, abs=1e-15)
            assert core.dm(t, tab, var)[0][0] == pytest.approx(want, abs=1e-15)


def test_root_length_is_ignored():
    # the worked-example tree with a non-zero root length: nothing changes
    g = json.load(open(os.path.join(HERE, "golden", "worked_example.json")))
    length = list(g["length"])
    length[4] = 7.5
    t = _util.tree(g["parent"], length)
    tab = _util.table([{0: 1}, {3: 1}])   # A vs D: disjoint root subtrees
    for var in VARIANTS:
        assert oracle.dm(t, tab, var)[0] == pytest.approx(1.0, abs=1e-15)


# ---------------------------------------------------------------- closed forms
def _root_dist_and_anc(t):
    m = t.parent.shape[0]
    anc = []
    dist = np.zeros(m)
    for v in range(m):
        chain, x, d = [], v, 0.0
        while x >= 0:
            chain.append(x)
            if t.parent[x] >= 0:
                d += t.length[x]
            x = t.parent[x]
        anc.append(chain)
        dist[v] = d
    return dist, anc


def test_single_tip_closed_form():
    rng = np.random.default_rng(0)
    t = synth.gen_tree(40, 0.3, seed=21)
    dist, anc = _root_dist_and_anc(t)
    tips = _util.tip_ids(t)
    pairs = [(int(a), int(b)) for a, b in rng.choice(tips, size=(25, 2))]
    rows = []
    for a, b in pairs:
        rows += [{a: int(rng.integers(1, 9))}, {b: int(rng.integers(1, 9))}]
    tab = _util.table(rows)
    n = len(rows)
    dmu = oracle.dm(t, tab, "unweighted")
    dmw = oracle.dm(t, tab, "weighted_normalized")
    for k, (a, b) in enumerate(pairs):
        lca = next(x for x in anc[a] if x in set(anc[b]))
        di, dj, dl = dist[a], dist[b], dist[lca]
        want_u = (di + dj - 2 * dl) / (di + dj - dl) if di + dj - dl > 0 else 0.0
        want_w = (di + dj - 2 * dl) / (di + dj) if di + dj > 0 else 0.0
        idx = oracle.condensed_index(n, 2 * k, 2 * k + 1)
        assert dmu[idx] == pytest.approx(want_u, rel=1e-12, abs=1e-15)
        assert dmw[idx] == pytest.approx(want_w, rel=1e-12, abs=1e-15)


def test_disjoint_root_subtrees_give_one():
    t = synth.gen_tree(60, 0.2, seed=4)
    t.length[-1] = 3.0                          # root length must be ignored
    root = t.n_nodes - 1
    kids = np.nonzero(t.parent == root)[0]
    _, anc = _root_dist_and_anc(t)
    tips = _util.tip_ids(t)
    left = [x for x in tips if kids[0] in anc[x]]
    right = [x for x in tips if kids[1] in anc[x]]
    rng = np.random.default_rng(1)
    rows = _util.random_rows(rng, left, 3) + _util.random_rows(rng, right, 3)
    tab = _util.table(rows)
    for var in VARIANTS:
        d = _util.squareform(oracle.dm(t, tab, var), 6)
        assert np.allclose(d[:3, 3:], 1.0, atol=1e-15)


# ---------------------------------------------------------------- brute force
@st.composite
def small_problem(draw):
    m = draw(st.integers(2, 14))
    # random tree on m nodes: node k>0 attaches to a random earlier node
    par = [-1] + [draw(st.integers(0, k - 1)) for k in range(1, m)]
    lens = [draw(st.sampled_from([0.0, 0.5, 1.0, 2.25, 0.1, 3.0])) for _ in range(m)]
    perm = draw(st.permutations(list(range(m))))      # shuffle ids
    parent = [-1] * m
    length = [0.0] * m
    for old in range(m):
        new = perm[old]
        parent[new] = perm[par[old]] if par[old] >= 0 else -1
        length[new] = lens[old]
    t = _util.tree(parent, length)
    tips = list(_util.tip_ids(t))
    n = draw(st.integers(2, 6))
    rows = []
    for _ in range(n):
        k = draw(st.integers(1, len(tips)))
        chosen = draw(st.permutations(tips))[:k]
        r = {int(x): draw(st.integers(0, 7)) for x in chosen}
        first = int(chosen[0])
        r[first] = max(r[first], 1)
        rows.append(r)
    return t, rows


@settings(max_examples=150, deadline=None)
@given(small_problem())
def test_oracle_matches_brute_force(prob):
    t, rows = prob
    tab = _util.table(rows)
    for var in VARIANTS:
        want = np.asarray(brute.dm(t.parent, t.length, rows, var))
        got = oracle.dm(t, tab, var)
        assert np.allclose(got, want, rtol=0, atol=1e-12), var
        got_c, _ = core.dm(t, tab, var, n_threads=2)
        assert np.allclose(got_c, want, rtol=0, atol=1e-12), var


def test_c_core_matches_python_oracle_c1_slice():
    tr, tab = synth.config("C1", n_samples=48)
    for var in VARIANTS:
        a = oracle.dm(tr, tab, var)
        b, used = core.dm(tr, tab, var)
        assert used >= 1
        assert np.allclose(a, b, rtol=1e-13, atol=1e-15)


# ---------------------------------------------------------------- library pins
def test_star_tree_matches_scipy_weighted_jaccard_and_braycurtis():
    rng = np.random.default_rng(3)
    n_tips = 30
    parent = [n_tips] * n_tips + [-1]
    length = list(rng.exponential(0.5, n_tips)) + [0.0]
    t = _util.tree(parent, length)
    rows = _util.random_rows(rng, range(n_tips), 8, max_nnz=12, zero_prob=0.2)
    tab = _util.table(rows)
    x = tab.dense(n_tips + 1)[:, :n_tips].astype(float)
    w = np.asarray(length[:n_tips])
    du = _util.squareform(oracle.dm(t, tab, "unweighted"), 8)
    dw = _util.squareform(oracle.dm(t, tab, "weighted_normalized"), 8)
    for i in range(8):
        for j in range(i + 1, 8):
            assert du[i, j] == pytest.approx(jaccard(x[i] > 0, x[j] > 0, w=w), abs=1e-13)
            pi, pj = x[i] / x[i].sum(), x[j] / x[j].sum()
            assert dw[i, j] == pytest.approx(braycurtis(pi, pj, w=w), abs=1e-13)


def test_caterpillar_matches_wasserstein():
    # spine s_0 (root) - s_1 - ... - s_{k-1}; tip t_m hangs from s_m with length 0;
    # the branch of s_m has length x_m - x_{m-1}.  Then the numerator of d_W is
    # the 1-Wasserstein distance between the tip distributions on positions x,
    # and the denominator is E_i[x] + E_j[x] (positions measured from x_0 = 0).
    rng = np.random.default_rng(5)
    k = 12
    x = np.concatenate([[0.0], np.cumsum(rng.exponential(1.0, k - 1))])
    parent, length = [-1], [0.0]                 # s_0 = node 0
    for m in range(1, k):
        parent.append(m - 1)                     # s_m = node m
        length.append(x[m] - x[m - 1])
    tip_node = []
    for m in range(k):
        parent.append(m)
        length.append(0.0)
        tip_node.append(k + m)
    t = _util.tree(parent, length)
    rows = []
    for _ in range(6):
        cnt = rng.integers(0, 6, size=k)
        cnt[rng.integers(k)] += 1
        rows.append({tip_node[m]: int(cnt[m]) for m in range(k) if cnt[m] > 0})
    tab = _util.table(rows)
    dw = _util.squareform(oracle.dm(t, tab, "weighted_normalized"), 6)
    for i in range(6):
        for j in range(i + 1, 6):
            pi = np.array([rows[i].get(tip_node[m], 0) for m in range(k)], float)
            pj = np.array([rows[j].get(tip_node[m], 0) for m in range(k)], float)
            pi /= pi.sum()
            pj /= pj.sum()
            num = wasserstein_distance(x, x, pi, pj)
            den = float(pi @ x + pj @ x)
            assert dw[i, j] == pytest.approx(num / den, rel=1e-12, abs=1e-15)


def test_unweighted_equals_sparse_gram_identity():
    # d_U = (w_i + w_j - 2G) / (w_i + w_j - G), G = A diag(l) A^T, w = A l
    tr, tab = synth.config("C1", n_samples=40)
    u, a, length, nonroot = oracle.embedding(tr, tab)
    A = sp.csr_matrix(a[:, nonroot])
    lv = length[nonroot]
    G = (A @ sp.diags(lv) @ A.T).toarray()
    w = A @ lv
    n = a.shape[0]
    d = oracle.dm(tr, tab, "unweighted")
    k = 0
    for i in range(n):
        for j in range(i + 1, n):
            xor = w[i] + w[j] - 2 * G[i, j]
            orr = w[i] + w[j] - G[i, j]
            assert d[k] == pytest.approx(xor / orr, rel=1e-12, abs=1e-14)
            k += 1


def test_weighted_denominator_is_root_distance_sum():
    # sum_v l_v (u_iv + u_jv) = sum_t D_t (p_it + p_jt): D_t = root-to-tip distance
    tr, tab = synth.config("C1", n_samples=5)
    u, a, length, nonroot = oracle.embedding(tr, tab)
    dist, _ = _root_dist_and_anc(tr)
    x = tab.dense(tr.n_nodes).astype(float)
    p = x / x.sum(axis=1, keepdims=True)
    s = (u[:, nonroot] * length[nonroot]).sum(axis=1)
    assert np.allclose(s, p @ dist, rtol=1e-12)


# ---------------------------------------------------------------- PCoA means
def test_pcoa_means_gower_identity():
    rng = np.random.default_rng(2)
    n = 9
    cond = rng.random(n * (n - 1) // 2)
    r, g = oracle.pcoa_means(cond, n)
    d = _util.squareform(cond, n)
    a = -0.5 * d * d
    j = np.eye(n) - np.ones((n, n)) / n
    centred = j @ a @ j
    assert np.allclose(centred, a - r[:, None] - r[None, :] + g, atol=1e-14)
    assert np.allclose(centred.sum(axis=1), 0.0, atol=1e-13)
    assert g == pytest.approx(a.sum() / n / n, abs=1e-15)


# ---------------------------------------------------------------- layouts
@pytest.mark.parametrize("n", [2, 3, 7, 8, 13])
def test_stripes_cover_each_pair(n):
    cond = np.arange(1, n * (n - 1) // 2 + 1, dtype=float)
    s = oracle.to_stripes(cond, n, 0, oracle.n_stripes(n))
    seen = np.bincount(s.reshape(-1).astype(int), minlength=cond.size + 1)[1:]
    if n % 2:
        assert np.all(seen == 1)
    else:
        # the last stripe (partner n/2 away) holds each of its pairs twice
        twice = {oracle.condensed_index(n, i, i + n // 2) for i in range(n // 2)}
        for k in range(cond.size):
            assert seen[k] == (2 if k in twice else 1)


def test_condensed_index_matches_scipy_squareform():
    from scipy.spatial.distance import squareform
    n = 11
    cond = np.arange(n * (n - 1) // 2, dtype=float)
    sq = squareform(cond)
    for i in range(n):
        for j in range(n):
            if i != j:
                assert sq[i, j] == oracle.condensed_index(n, i, j)


# ---------------------------------------------------------------- invariants
def _c1(n=24, seed=101):
    tr = synth.gen_tree(120, 0.1, seed)
    tab = synth.gen_table_uniform(n, np.arange(120), 15, seed)
    return tr, tab


@pytest.mark.parametrize("var", VARIANTS)
def test_basic_invariants(var):
    tr, tab = _c1()
    n = tab.n_samples
    # duplicate sample 0 at the end: d(a, a) = 0
    rows = list(range(n)) + [0]
    tab2 = synth.subset_rows(tab, rows)
    d = _util.squareform(oracle.dm(tr, tab2, var), n + 1)
    assert d[0, n] == pytest.approx(0.0, abs=1e-15)
    assert np.all(d >= 0) and np.all(d <= 1 + 1e-15)
    # sample permutation permutes the matrix
    perm = np.random.default_rng(4).permutation(n)
    dp = _util.squareform(oracle.dm(tr, synth.subset_rows(tab, perm), var), n)
    assert np.allclose(dp, d[:n, :n][np.ix_(perm, perm)], atol=1e-14)


def test_unweighted_triangle_inequality():
    tr, tab = _c1(n=20)
    d = _util.squareform(oracle.dm(tr, tab, "unweighted"), 20)
    for k in range(20):
        assert np.all(d <= d[:, [k]] + d[[k], :] + 1e-12)


@pytest.mark.parametrize("var", VARIANTS)
def test_scaling_invariances(var):
    tr, tab = _c1()
    base = oracle.dm(tr, tab, var)
    tr2 = synth.Tree(parent=tr.parent, length=tr.length * 3.7, n_tips=tr.n_tips)
    assert np.allclose(oracle.dm(tr2, tab, var), base, atol=1e-14)
    tab2 = synth.Table(indptr=tab.indptr, tips=tab.tips, counts=tab.counts * 5)
    assert np.allclose(oracle.dm(tr, tab2, var), base, atol=1e-14)


@pytest.mark.parametrize("var", VARIANTS)
def test_unary_split_and_zero_tip_and_relabel(var):
    tr, tab = _c1(n=12)
    base = oracle.dm(tr, tab, var)
    m = tr.n_nodes
    # split branch of node 5 by a new unary node m (length split 0.3 / 0.7)
    parent = np.append(tr.parent.copy(), tr.parent[5])
    length = np.append(tr.length.copy(), tr.length[5] * 0.7)
    parent[5] = m
    length[5] = tr.length[5] * 0.3
    # add a zero-count tip m+1 under node 200 (an internal node)
    parent = np.append(parent, 200)
    length = np.append(length, 1.5)
    t2 = _util.tree(parent, length)
    assert np.allclose(oracle.dm(t2, tab, var), base, atol=1e-14)
    # relabel every node id (children reorder too)
    perm = np.random.default_rng(8).permutation(m)
    inv = np.empty(m, np.int64)
    inv[perm] = np.arange(m)
    p3 = np.full(m, -1, np.int64)
    l3 = np.zeros(m)
    for old in range(m):
        p3[perm[old]] = perm[tr.parent[old]] if tr.parent[old] >= 0 else -1
        l3[perm[old]] = tr.length[old]
    tab3 = synth.Table(indptr=tab.indptr, tips=perm[tab.tips], counts=tab.counts)
    assert np.allclose(oracle.dm(_util.tree(p3, l3), tab3, var), base, atol=1e-14)


def test_embedding_sum_rules():
    tr, tab = _c1(n=6)
    u, a, length, nonroot = oracle.embedding(tr, tab)
    root = tr.n_nodes - 1
    kids = [np.nonzero(tr.parent == v)[0] for v in range(tr.n_nodes)]
    for v in range(tr.n_nodes):
        if kids[v].size:
            assert np.allclose(u[:, v], u[:, kids[v]].sum(axis=1), atol=1e-14)
    assert np.allclose(u[:, root], 1.0)


# ---------------------------------------------------------------- validation
@pytest.mark.parametrize("parent,length", [
    ([-1, -1, 0], [0, 1, 1]),          # two roots
    ([1, 2, 0, -1], [1, 1, 1, 0]),      # cycle detached from root
    ([2, 2, -1], [1, -1.0, 0]),         # negative length
    ([2, 2, -1], [1, float("nan"), 0]),  # NaN length
    ([2, 5, -1], [1, 1, 0]),            # parent out of range
])
def test_invalid_trees_raise(parent, length):
    with pytest.raises(oracle.TreeError):
        oracle.validate_tree(parent, length)


@pytest.mark.parametrize("rows", [
    [{0: 1}, {2: 1}],                 # feature mapped to an internal node
    [{0: 0}, {1: 1}],                 # zero-total sample
])
def test_invalid_tables_raise(rows):
    t = _util.tree([2, 2, -1], [1.0, 2.0, 0.0])
    with pytest.raises(oracle.TableError):
        oracle.dm(t, _util.table(rows), "unweighted")


def test_duplicate_feature_raises():
    t = _util.tree([2, 2, -1], [1.0, 2.0, 0.0])
    tab = synth.Table(indptr=np.array([0, 2, 3]), tips=np.array([0, 0, 1]), counts=np.array([1, 1, 1]))
    with pytest.raises(oracle.TableError):
        oracle.dm(t, tab, "weighted_normalized")


# ---------------------------------------------------------------- BF16 rounding (split lengths)
# The split-precision lengths of the MFMA Gram path (l = hi + lo, each rounded
# to bfloat16 with ties to even) are part of the oracle the unweighted split and
# the Gram tests compare with.  bfloat16 keeps 8 significant bits (7 stored),
# the FP32 exponent range, and a subnormal grid of spacing 2^-133 below 2^-126.
@pytest.mark.parametrize("x, want", [
    (1.0, 1.0),
    (1.0 + 2.0 ** -8, 1.0),                      # exact tie: to the even neighbour 1.0
    (1.0 + 3 * 2.0 ** -9, 1.0 + 2.0 ** -7),      # 0.75 of a unit: up
    (1.0 + 2.0 ** -9, 1.0),                      # 0.25 of a unit: down
    (1.0 + 3 * 2.0 ** -8, 1.0 + 2.0 ** -6),      # tie between odd 1+2^-7 and even 1+2^-6
    (1.0 + 5 * 2.0 ** -8, 1.0 + 2.0 ** -6),      # tie between even 1+2^-6 and odd 1+3*2^-7
    (-(1.0 + 3 * 2.0 ** -9), -(1.0 + 2.0 ** -7)),  # sign kept, magnitude rounded
    (255.0, 255.0), (257.0, 256.0), (259.0, 260.0),  # 8 significant bits: spacing 2 in [256, 512)
    (0.1, 0.10009765625),                        # 0x3DCD
    (2.0 ** -126, 2.0 ** -126),                  # smallest normal
    (2.0 ** -126 - 2.0 ** -140, 2.0 ** -126),    # just below: the subnormal grid (2^-133) rounds up
    (2.0 ** -134, 0.0),                          # half the smallest subnormal: tie to even 0
    (3 * 2.0 ** -134, 2.0 ** -132),              # 1.5 subnormal units: tie to even 2 units
    (5 * 2.0 ** -135, 2.0 ** -133),              # 1.25 units: down to 1 unit
    (0.0, 0.0),
])
def test_bf16_rounding_hand_computed(x, want):
    from oracle.unifrac import _round_bf16_f64
    assert _round_bf16_f64(np.array([x]))[0] == want


def test_bf16_rounding_matches_torch_on_float32_inputs():
    # torch converts float32 -> bfloat16 with round-to-nearest-even on the bit
    # pattern; on FP32-exact inputs (normal and subnormal) the oracle must agree.
    # The oracle's domain stops below 2^127 (branch lengths are many orders of
    # magnitude smaller; it does not model rounding up to infinity).
    import torch
    from oracle.unifrac import _round_bf16_f64
    rng = np.random.default_rng(0)
    bits = rng.integers(0, 0x7F000000, size=200_000, dtype=np.uint64).astype(np.uint32)
    bits[:1000] = rng.integers(0, 2 ** 23, size=1000).astype(np.uint32)          # subnormals
    # exact ties: the 16 dropped bits are 0x8000
    bits[1000:2000] = ((rng.integers(0, 0x7F00, size=1000) << 16) | 0x8000).astype(np.uint32)
    f32 = bits.view(np.float32)
    f32 = np.concatenate([f32, -f32])
    want = torch.from_numpy(f32.copy()).to(torch.bfloat16).to(torch.float64).numpy()
    got = _round_bf16_f64(f32.astype(np.float64))
    assert np.array_equal(got, want)


def test_gram_split_lengths_residual_and_nearest():
    # hi is the nearest bfloat16 to l (checked against both bfloat16 neighbours),
    # lo the nearest to l - hi, and |l - hi - lo| <= 2^-16 l (8 significant bits
    # per part, half a unit of each)
    import torch
    rng = np.random.default_rng(3)
    length = np.concatenate([rng.exponential(0.05, size=20_000), [0.0, 1e-30, 7.0, 0.1]])
    hi, lo = oracle.gram_split_bf16(length)
    for part in (hi, lo):
        rt = torch.from_numpy(part.astype(np.float32)).to(torch.bfloat16).to(torch.float64).numpy()
        assert np.array_equal(rt, part)                    # exactly representable
    assert np.all(np.abs(length - hi - lo) <= 2.0 ** -16 * length)

    def neighbours(v):
        b = torch.from_numpy(v.astype(np.float32)).to(torch.bfloat16).view(torch.int16)
        up = (b + 1).view(torch.bfloat16).to(torch.float64).numpy()
        dn = (b - 1).view(torch.bfloat16).to(torch.float64).numpy()
        return up, dn

    pos = length > 1e-30
    up, dn = neighbours(hi[pos])
    err = np.abs(length[pos] - hi[pos])
    assert np.all(err <= np.abs(length[pos] - up)) and np.all(err <= np.abs(length[pos] - dn))
