"""CPU tests of the tree training: the labelling and its tie rule, the row
weights, the scores, Table II on a hand-made set, and the export round trip
(JSON -> gsw_tree_load -> the same choices as scikit-learn)."""
import numpy as np
import pytest

from oracle import tree as otree
from paper_1708_01159_amd import gsw, train


def test_labels_take_the_fastest_lowest_on_ties_and_skip_unmeasured():
    T = np.array([[3.0, 1.0, 2.0], [1.0, 1.0, 5.0], [-1.0, 4.0, 4.0], [2.0, -1.0, 1.5]])
    assert train.labels(T).tolist() == [1, 0, 1, 2]
    # within the tolerance of the fastest is a tie, beyond it is not
    T = np.array([[1.015, 1.0, 3.0], [1.03, 1.0, 3.0], [5.0, 2.0, 2.03]])
    assert train.labels(T).tolist() == [0, 1, 1]
    assert train.labels(T, tol=0.0).tolist() == [1, 1, 1]


def test_weights():
    T = np.array([[1.0, 2.0, 3.0], [1.0, 1.0, 1.0], [5.0, 1.0, 9.0]])
    g = np.array(["a", "a", "b"])
    assert train._weights(T, g, "none") is None
    w = train._weights(T, g, "regret")  # median - min, + 1e-4, normalised to mean 1
    raw = np.array([1.0, 0.0, 4.0]) + 1e-4
    np.testing.assert_allclose(w, raw / raw.mean())
    w = train._weights(T, g, "graph")  # each graph weighs the same
    assert w[0] == w[1] and w[2] == pytest.approx(2 * w[0])
    with pytest.raises(ValueError):
        train._weights(T, g, "bogus")


def test_scores_by_hand():
    T = np.array([[1.0, 2.0], [4.0, 2.0]])
    acc, slow, ratio = train.scores(np.array([1, 1]), T)
    assert acc == 0.5 and slow == pytest.approx((2.0 + 1.0) / 2) and ratio == pytest.approx(4.0 / 3.0)


def test_table2_by_hand():
    # two traversals of graph g (levels 2 and 1) and one of h; kernels 0 and 1
    T = np.array([[1.0, 3.0], [2.0, 1.0], [1.0, 10.0], [4.0, 1.0]])
    graph = np.array(["g", "g", "g", "h"])
    source = np.array([0, 0, 1, 5])
    # best per level: traversal (g,0) = 1 + 1 = 2, (g,1) = 1, (h,5) = 1
    out = train.table2({"always 0": np.array([0, 0, 0, 0])}, T, graph, source, ["k0", "k1"])
    # kernel 0: (g,0) 3/2, (g,1) 1/1, (h,5) 4/1
    assert out["always 0"]["average"] == pytest.approx((1.5 + 1.0 + 4.0) / 3, abs=1e-3)
    assert out["always 0"]["worst"] == 4.0 and out["always 0"]["optimal"] == pytest.approx(1 / 3, abs=1e-3)
    assert out["k1"]["worst"] == 10.0
    # best fixed kernel per graph: g -> kernel 0 (3 + 1 = 4 vs 4 + 10 = 14), h -> kernel 1
    assert out["best fixed kernel per graph"]["average"] == pytest.approx((1.5 + 1.0 + 1.0) / 3, abs=1e-3)


def test_cost_sensitive_leaves():
    """A leaf whose rows mostly favour kernel 0 by a hair, while one row is
    far slower with it, predicts kernel 1 once relabelled by total time."""
    from sklearn.tree import DecisionTreeClassifier

    X = np.zeros((5, 2))
    X[:, 0] = [0, 0, 0, 0, 1]
    T = np.array([[1.0, 1.1], [1.0, 1.1], [1.0, 1.1], [50.0, 1.2], [3.0, 1.0]])
    y = train.labels(T)
    c = DecisionTreeClassifier(max_depth=1).fit(X, y)
    assert c.predict(np.array([[0.0, 0.0]], dtype=np.float32))[0] == 0  # the majority
    train.relabel_leaves(c, X, T)
    assert c.predict(np.array([[0.0, 0.0]], dtype=np.float32))[0] == 1  # 53 ms against 4.5 ms
    assert c.predict(np.array([[1.0, 0.0]], dtype=np.float32))[0] == 1


def test_fit_export_load_round_trip(tmp_path):
    """A tree fitted on synthetic rows, exported, read back by the library's
    JSON reader, chooses what scikit-learn and the oracle walk choose."""
    rng = np.random.default_rng(0)
    n, K = 600, 4
    X = np.abs(rng.normal(size=(n, gsw.N_FEATURES))) * 10.0 ** rng.integers(0, 6, gsw.N_FEATURES)
    base = np.stack([1 + (X[:, 20] > 300), 1 + (X[:, 21] < 0.3), np.full(n, 1.4), 2 - (X[:, 2] > 5)], 1)
    T = base * rng.uniform(0.9, 1.1, size=(n, K))
    rows = dict(X=X, T=T, graph=np.array(["g%d" % (i % 7) for i in range(n)]),
                source=np.arange(n) % 5, level=np.zeros(n, dtype=int), kernels=np.array([0, 6, 7, 11 + 10]))
    valid = dict(rows)
    grid = [(4, 5, "regret", "majority"), (6, 1, "none", "time")]
    clf, ks, report = train.fit(rows, valid, grid=grid, log=lambda *a: None)
    assert report["params"]["max_depth"] in (4, 6) and report["validation"]["time_ratio"] >= 1.0
    assert set(report["model_variants_on_validation"]) >= {"random forest (64 trees)"}
    assert set(report["graph_split"]["by_family"]) == {"g"} and report["validation"]["by_family"]["g"] >= 1.0
    path = str(tmp_path / "t.json")
    arrays = train.export(clf, ks, path, report)
    loaded = gsw.Tree.load(path)
    for x in X[:150]:
        k, unknown = loaded.predict(x, 0, 1)
        k2, u2 = otree.predict(arrays, x, 0, 1, gsw.DEFAULT_KERNEL)
        assert (k, unknown) == (k2, u2)
        if not unknown:
            assert k == ks[int(clf.predict(x.astype(np.float32).reshape(1, -1))[0])]


def test_family_ratios_by_hand():
    assert [train.family(x) for x in ("rmat22_s200", "er20_d8_s401", "grid1024_del5_s202", "chunglu23_s220")] == \
        ["rmat", "er", "grid", "chunglu"]
    T = np.array([[1.0, 2.0], [4.0, 1.0], [2.0, 2.0], [3.0, -1.0]])
    graph = np.array(["rmat20_s1", "rmat22_s2", "er20_s3", "er21_s4"])
    # rmat: chosen 2 + 1 over best 1 + 1; er: chosen 2 + 3 over best 2 + 3
    assert train.family_ratios(np.array([1, 1, 0, 0]), T, graph) == {"er": 1.0, "rmat": 1.5}


def test_apply_solo_replaces_push_times_on_single_workgroup_rows(tmp_path):
    from paper_1708_01159_amd import gsw, train

    ks = np.arange(gsw.N_KERNELS)
    T = np.full((3, len(ks)), 0.010)
    T[:, gsw.PULL_BITMAP] = 0.008
    solo = np.array([np.nan, 0.003, np.nan])
    T2 = train.apply_solo(T, solo, ks)
    push = [k for k in ks if gsw.kernel_base(int(k)) <= gsw.PUSH_EDGE]
    other = [k for k in ks if gsw.kernel_base(int(k)) > gsw.PUSH_EDGE]
    assert np.allclose(T2[1, push], 0.003 + train.SOLO_LAUNCH_SHARE_MS)
    assert np.array_equal(T2[1, other], T[1, other]) and np.array_equal(T2[[0, 2]], T[[0, 2]])
    assert train.labels(T2)[1] == 0 and train.labels(T)[1] == gsw.PULL_BITMAP  # push now wins that level
    # collect files with the solo pass are corrected on load; without it they are not
    rows = dict(X=np.zeros((3, gsw.N_FEATURES)), T=T, graph=np.array(["a"] * 3), source=np.zeros(3, dtype=np.int64),
                level=np.arange(3), kernels=ks)
    np.savez(tmp_path / "plain.npz", **rows)
    np.savez(tmp_path / "solo.npz", solo_ms=solo, **rows)
    assert np.array_equal(train._load_rows([str(tmp_path / "plain.npz")])["T"], T)
    assert np.array_equal(train._load_rows([str(tmp_path / "solo.npz")])["T"], T2)
