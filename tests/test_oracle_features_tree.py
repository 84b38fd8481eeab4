"""Pins of the feature, tree and schedule oracles."""
import numpy as np
import pytest

from oracle import features, schedule, tree
from paper_1708_01159_amd import graphgen as gg


def test_graph_features_closed_forms():
    # star K_{1,9}: degrees [9, 1 x 9]
    g = gg.from_edges(10, [0] * 9, list(range(1, 10)))
    f = features.graph_features(g.offs)
    # sorted degrees 1,1,1,1,1,1,1,1,1,9: linear-interpolated quartiles are 1
    assert f.tolist()[:7] == [10, 18, 1, 1, 1, 1, 9]
    mean = 1.8
    assert f[7] == pytest.approx(np.sqrt((9 * (1 - mean) ** 2 + (9 - mean) ** 2) / 10))
    # path on 5 vertices: degrees 1,2,2,2,1 -> sorted 1,1,2,2,2
    g = gg.from_edges(5, [0, 1, 2, 3], [1, 2, 3, 4])
    f = features.graph_features(g.offs)
    # positions (k-1)*p: q1 at 1.0 -> 1, median at 2.0 -> 2, q3 at 3.0 -> 2
    assert f.tolist()[:7] == [5, 8, 1, 1, 2, 2, 2]
    # four degrees 1,2,3,4 (hand: q1 at 0.75 -> 1.75, med 2.5, q3 at 2.25 -> 3.25)
    offs = np.array([0, 1, 3, 6, 10], dtype=np.int64)
    f = features.graph_features(offs)
    assert f.tolist()[2:7] == [1.0, 1.75, 2.5, 3.25, 4.0]


def test_level_features():
    offs = np.array([0, 1, 3, 6, 10], dtype=np.int64)
    hist = np.array([1, 2, 1])
    x = features.level_features(offs, hist, 1)
    assert x.shape == (features.N_FEATURES,)
    assert x[20:].tolist() == [2.0, 0.5, 3.0, 0.75]
    # symmetric: in- and absolute-degree summaries repeat the out-degree one
    assert x[8:14].tolist() == x[2:8].tolist() == x[14:20].tolist()


def test_directed_degree_features_by_hand():
    """Arcs 0->1, 0->2, 0->3, 1->0.  out = (3,1,0,0), in = (1,1,1,1), absolute
    (distinct neighbours ignoring direction) = (3,1,1,1)."""
    offs = np.array([0, 3, 4, 4, 4], dtype=np.int64)
    cols = np.array([1, 2, 3, 0], dtype=np.int32)
    out, ind, ab = features.degrees(offs, cols)
    assert out.tolist() == [3, 1, 0, 0] and ind.tolist() == [1, 1, 1, 1] and ab.tolist() == [3, 1, 1, 1]
    f = features.graph_features(offs, cols)
    # out sorted 0,0,1,3: q1 at 0.75 -> 0, median at 1.5 -> 0.5, q3 at 2.25 -> 1.5; mean 1, var 1.5
    assert f[:8].tolist() == pytest.approx([4, 4, 0, 0, 0.5, 1.5, 3, np.sqrt(1.5)])
    assert f[8:14].tolist() == [1, 1, 1, 1, 1, 0]
    # absolute sorted 1,1,1,3: q3 at 2.25 -> 1.5; mean 1.5, var 0.75
    assert f[14:20].tolist() == pytest.approx([1, 1, 1, 1.5, 3, np.sqrt(0.75)])
    # a reciprocated pair, a self-loop and a repeated arc: 0->0, 0->1, 0->1, 1->0, 1->2
    offs = np.array([0, 3, 5, 5], dtype=np.int64)
    cols = np.array([0, 1, 1, 0, 2], dtype=np.int32)
    out, ind, ab = features.degrees(offs, cols)
    # in: v0 from rows 0,1 -> 2; v1 twice from row 0 -> 2; v2 once -> 1
    assert out.tolist() == [3, 2, 0] and ind.tolist() == [2, 2, 1]
    # row 0 entries whose reverse exists: 0 (0->0), 1, 1 (1->0): all 3 -> abs 3 + 2 - 3 = 2
    # row 1 entries: 0 (0->1 exists), 2 (2->1 no) -> 1 -> abs 2 + 2 - 1 = 3; v2: 0 + 1 = 1
    assert ab.tolist() == [2, 3, 1]


def _export(clf, class_kernel):
    t = clf.tree_
    return dict(left=t.children_left.tolist(), right=t.children_right.tolist(),
                feature=t.feature.tolist(), threshold=t.threshold.tolist(),
                value=[list(map(float, v[0])) for v in t.value], class_kernel=list(class_kernel))


def test_tree_walk_matches_sklearn():
    from sklearn.tree import DecisionTreeClassifier

    rng = np.random.default_rng(3)
    X = rng.normal(size=(600, 6)) * np.array([1, 10, 100, 1e3, 1e6, 3e7])
    X[:, 5] = np.round(X[:, 5])  # large integer-valued feature (float32 rounding)
    y = (X[:, 0] > 0).astype(int) + 2 * (X[:, 3] > 100) + (X[:, 5] > 1.2e7)
    clf = DecisionTreeClassifier(criterion="gini", random_state=0).fit(X, y)
    ck = [10 + c for c in range(len(clf.classes_))]
    T = _export(clf, ck)
    pred = clf.predict(X)
    Xq = rng.normal(size=(400, 6)) * np.array([1, 10, 100, 1e3, 1e6, 3e7])
    predq = clf.predict(Xq)
    for XX, pp in ((X, pred), (Xq, predq)):
        for x, p in zip(XX, pp):
            k, unknown = tree.predict(T, x, prev_kernel=-5, level=3, default_kernel=-7)
            leaf = tree.leaf_of(T, x)
            assert leaf == clf.apply(x.reshape(1, -1))[0]
            if not unknown:
                assert k == 10 + int(np.searchsorted(clf.classes_, p))


def test_tree_float32_feature_cast():
    from sklearn.tree import DecisionTreeClassifier

    # 16777217 is not a float32; sklearn sees it as 16777216
    X = np.array([[16777216.0], [16777217.0], [16777218.0], [16777220.0]])
    y = np.array([0, 1, 1, 1])
    clf = DecisionTreeClassifier(random_state=0).fit(X, y)
    T = _export(clf, [0, 1])
    for x in X:
        k, unknown = tree.predict(T, x, 0, 1, 0)
        if not unknown:
            assert k == clf.predict(x.reshape(1, -1))[0]
    # the 2^24 and 2^24+1 rows are indistinguishable in float32: same leaf
    assert tree.leaf_of(T, X[0]) == tree.leaf_of(T, X[1])


def test_unknown_rule():
    # root splits feature 0 at 0.5; left leaf tied [2, 2], right leaf [0, 3]
    T = dict(left=[1, -1, -1], right=[2, -1, -1], feature=[0, -2, -2], threshold=[0.5, -2, -2],
             value=[[2, 5], [2, 2], [0, 3]], class_kernel=[4, 6])
    assert tree.predict(T, [1.0], prev_kernel=1, level=0, default_kernel=2) == (6, False)
    # tie at the first level -> edge-centric default
    assert tree.predict(T, [0.0], prev_kernel=1, level=0, default_kernel=2) == (2, True)
    # tie later -> repeat the previous level's choice
    assert tree.predict(T, [0.0], prev_kernel=1, level=5, default_kernel=2) == (1, True)
    # sklearn itself breaks the tie by lowest class: it never says "unknown"
    from sklearn.tree import DecisionTreeClassifier

    clf = DecisionTreeClassifier(max_depth=1, random_state=0).fit([[0], [0], [0], [0]], [0, 1, 0, 1])
    assert clf.predict([[0]])[0] == 0


def test_best_per_level_and_fixed():
    nan = np.nan
    T = np.array([[1.0, 2.0, 3.0],
                  [5.0, 1.0, 1.0],
                  [2.0, 9.0, nan]])
    choice, total = schedule.best_per_level(T)
    assert choice.tolist() == [0, 1, 0] and total == 4.0
    k, tot = schedule.best_fixed(T)
    assert (k, tot) == (0, 8.0)
