"""C ABI, host side: symbols, validation, degree statistics and tree lookup.
None of these calls touches a GPU."""
import os
import re

import numpy as np
import pytest

import oracle
from oracle import features as ofeat
from oracle import tree as otree
from paper_1708_01159_amd import graphgen as gg
from paper_1708_01159_amd import gsw

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    names = set()
    for fn in os.listdir(os.path.join(ROOT, "include")):
        if not fn.endswith(".h"):
            continue
        text = open(os.path.join(ROOT, "include", fn)).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        for m in re.finditer(r"\b(gsw_\w+)\s*\(", text):
            names.add(m.group(1))
    return sorted(names)


def test_every_declared_symbol_is_exported():
    names = declared_functions()
    assert "gsw_bfs" in names and "gsw_graph_create_host" in names
    lib = gsw.lib()
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing


def test_header_and_binding_agree_on_constants():
    text = open(os.path.join(ROOT, "include", "gsw.h")).read()
    consts = dict((m.group(1), int(m.group(2)))
                  for m in re.finditer(r"GSW_K_(\w+) = (\d+)", text))
    for i, name in enumerate(gsw.KERNEL_NAMES):
        assert consts[name.upper()] == i
        assert gsw.kernel_name(i) == name
    assert gsw.kernel_name(99) == "?"
    assert int(re.search(r"GSW_N_FEATURES (\d+)", text).group(1)) == gsw.N_FEATURES == ofeat.N_FEATURES
    assert gsw.lib().gsw_abi_version() == int(re.search(r"GSW_ABI_VERSION (\d+)", text).group(1))


@pytest.mark.parametrize("offs,cols,msg", [
    ([1, 2], [0], "offs[0]"),
    ([0, 2, 1], [0, 1], "decreases"),
    ([0, 1, 3], [1, 0], "differs"),
    ([0, 1, 2], [1, 2], "out of"),
    ([0, 1, 2], [1, -1], "out of"),
])
def test_validation_errors(offs, cols, msg):
    with pytest.raises(gsw.GswError) as ei:
        gsw.validate(offs, cols)
    assert ei.value.status == gsw.EINVAL and msg in str(ei.value)


def test_validation_zero_vertices():
    with pytest.raises(gsw.GswError):
        gsw.validate(np.zeros(1, dtype=np.int64), np.zeros(0, dtype=np.int32))


def test_symmetry_detection():
    g = gg.rmat(9, 8, seed=3)
    assert gsw.validate(g.offs, g.cols)
    # directed path 0->1->2
    assert not gsw.validate([0, 1, 2, 2], [1, 2])
    # unsorted rows, still symmetric
    assert gsw.validate([0, 2, 3, 4], [2, 1, 0, 0])
    # loops and repeats tolerated
    assert gsw.validate([0, 3, 4], [1, 1, 0, 0])


def test_degree_stats_match_oracle():
    for g in (gg.rmat(10, 16, seed=1), gg.grid(13, 17, 0.1, seed=2), gg.chung_lu(4000, 2.1, 10, seed=3),
              gg.from_edges(5, [0, 1, 2, 3], [1, 2, 3, 4])):
        mine = gsw.degree_stats(g.offs)
        ref = ofeat.graph_features(g.offs)[2:8]
        assert np.array_equal(mine[:5], ref[:5])
        assert mine[5] == pytest.approx(ref[5], rel=1e-12)


def _export(clf, ck):
    t = clf.tree_
    return dict(left=t.children_left.tolist(), right=t.children_right.tolist(),
                feature=t.feature.tolist(), threshold=t.threshold.tolist(),
                value=[list(map(float, v[0])) for v in t.value], class_kernel=list(ck))


def test_tree_predict_matches_oracle_and_sklearn():
    from sklearn.tree import DecisionTreeClassifier

    rng = np.random.default_rng(11)
    X = np.abs(rng.normal(size=(800, gsw.N_FEATURES))) * (10.0 ** rng.integers(0, 8, gsw.N_FEATURES))
    y = (X[:, 8] > np.median(X[:, 8])).astype(int) * 2 + (X[:, 11] > np.median(X[:, 11]))
    y[::7] = 4  # noise so some leaves are mixed
    clf = DecisionTreeClassifier(criterion="gini", max_depth=6, random_state=0).fit(X, y)
    ck = [gsw.PULL_BITMAP, gsw.PUSH_EDGE, gsw.PUSH_WAVE16, gsw.PUSH_VERTEX, gsw.EDGE_SCAN]
    T = _export(clf, ck)
    tr = gsw.Tree(T)
    Xq = np.concatenate([X, np.abs(rng.normal(size=(300, gsw.N_FEATURES))) * 1e4])
    n_unknown = 0
    for x in Xq:
        for prev, level in ((gsw.PUSH_VERTEX, 0), (gsw.PUSH_WAVE64, 3)):
            k, u = tr.predict(x, prev, level)
            k2, u2 = otree.predict(T, x, prev, level, gsw.DEFAULT_KERNEL)
            assert (k, u) == (k2, u2)
            if not u:
                assert k == ck[int(np.searchsorted(clf.classes_, clf.predict(x.reshape(1, -1))[0]))]
            n_unknown += u
    # exact ties are rare on random data; the handmade case below covers them


def test_tree_unknown_rule_handmade():
    T = dict(left=[1, -1, -1], right=[2, -1, -1], feature=[9, -2, -2], threshold=[0.5, -2.0, -2.0],
             value=[[2, 5], [2, 2], [0, 3]], class_kernel=[gsw.PULL_BITMAP, gsw.PUSH_VERTEX])
    tr = gsw.Tree(T)
    x = np.zeros(gsw.N_FEATURES)
    x[9] = 0.9
    assert tr.predict(x, gsw.PUSH_WAVE8, 0) == (gsw.PUSH_VERTEX, False)
    x[9] = 0.1
    assert tr.predict(x, gsw.PUSH_WAVE8, 0) == (gsw.DEFAULT_KERNEL, True)
    assert tr.predict(x, gsw.PUSH_WAVE8, 4) == (gsw.PUSH_WAVE8, True)


def test_tree_float32_threshold_semantics():
    # feature 1 (arcs) above 2^24: compared as float32 like sklearn
    T = dict(left=[1, -1, -1], right=[2, -1, -1], feature=[1, -2, -2],
             threshold=[16777216.5, -2.0, -2.0], value=[[1, 1], [1, 0], [0, 1]],
             class_kernel=[gsw.PUSH_EDGE, gsw.PULL_BITMAP])
    tr = gsw.Tree(T)
    x = np.zeros(gsw.N_FEATURES)
    x[1] = 16777217.0  # float32 -> 16777216 <= threshold -> left
    assert tr.predict(x, 0, 1)[0] == gsw.PUSH_EDGE
    assert otree.predict(T, x, 0, 1, gsw.DEFAULT_KERNEL)[0] == gsw.PUSH_EDGE
    x[1] = 16777218.0
    assert tr.predict(x, 0, 1)[0] == gsw.PULL_BITMAP


@pytest.mark.parametrize("bad", [
    dict(left=[1, -1], right=[0, -1]),   # child pointing backwards
    dict(left=[1, -1], right=[5, -1]),   # child out of range
    dict(left=[-1, -1], right=[1, -1]),  # half leaf
])
def test_tree_create_rejects_malformed(bad):
    T = dict(feature=[0, 0], threshold=[0.0, 0.0], value=[[1.0], [1.0]], class_kernel=[0], **bad)
    with pytest.raises(gsw.GswError):
        gsw.Tree(T)


def test_tree_create_rejects_bad_kernel():
    with pytest.raises(gsw.GswError):
        gsw.Tree(dict(feature=[0], threshold=[0.0], left=[-1], right=[-1], value=[[1.0]],
                      class_kernel=[42]))


def test_graph_create_without_gpu_fails_loudly():
    import torch

    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    g = gg.rmat(6, 4, seed=1)
    with pytest.raises(gsw.GswError) as ei:
        gsw.Graph.from_csr(g.offs, g.cols)
    assert ei.value.status == gsw.EHIP
