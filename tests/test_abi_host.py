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


def test_library_stamp_matches_sources(monkeypatch):
    """The library carries the digest of the sources it was built from; the
    binding refuses one built from other sources (a stale binary)."""
    from paper_1708_01159_amd import build

    lib = gsw.lib()
    assert lib.gsw_source_digest().decode() == build.source_digest()
    monkeypatch.setattr(gsw, "_lib", None)
    monkeypatch.setattr(build, "source_digest", lambda: "0000000000000000")
    with pytest.raises(RuntimeError, match="other sources"):
        gsw.lib()


def test_header_and_binding_agree_on_constants():
    text = open(os.path.join(ROOT, "include", "gsw.h")).read()
    consts = dict((m.group(1), int(m.group(2)))
                  for m in re.finditer(r"GSW_K_(\w+) = (\d+)", text))
    for i, name in enumerate(gsw.BASE_NAMES):
        assert consts[name.upper()] == i
    assert int(re.search(r"GSW_N_BASE_KERNELS = (\d+)", text).group(1)) == gsw.N_BASE_KERNELS
    counts = dict((m.group(1), int(m.group(2))) for m in re.finditer(r"GSW_COUNT_(\w+) = (\d+)", text))
    assert (counts["WORKGROUP"], counts["WAVE"], counts["THREAD"]) == (
        gsw.COUNT_WORKGROUP, gsw.COUNT_WAVE, gsw.COUNT_THREAD)
    assert len(gsw.KERNEL_NAMES) == gsw.N_KERNELS == 33
    for i, name in enumerate(gsw.KERNEL_NAMES):
        assert gsw.kernel_name(i) == name
        assert gsw.kernel_id(gsw.kernel_base(i), gsw.kernel_count(i)) == i
    assert gsw.kernel_name(gsw.N_KERNELS) == "?" and gsw.kernel_name(-1) == "?"
    assert int(re.search(r"GSW_N_FEATURES (\d+)", text).group(1)) == gsw.N_FEATURES == ofeat.N_FEATURES
    assert int(re.search(r"GSW_N_GRAPH_FEATURES (\d+)", text).group(1)) == gsw.N_GRAPH_FEATURES
    for i, name in enumerate(gsw.FEATURE_NAMES):
        assert gsw.lib().gsw_feature_name(i).decode() == name == ofeat.NAMES[i]
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


def test_graph_features_host_match_oracle():
    """The library's 20 graph features against the oracle's definitions, on
    symmetric graphs and on directed ones (out-, in- and absolute degrees
    differ there)."""
    rng = np.random.default_rng(5)
    cases = [gg.rmat(9, 8, seed=3), gg.from_edges(5, [0, 1, 2, 3], [1, 2, 3, 4])]
    for k in range(6):  # random directed graphs with repeats, loops and some reciprocated arcs
        n = int(rng.integers(2, 40))
        m = int(rng.integers(1, 4 * n))
        src = rng.integers(0, n, m)
        dst = rng.integers(0, n, m)
        order = np.lexsort((dst, src))
        src, dst = src[order], dst[order]
        offs = np.zeros(n + 1, dtype=np.int64)
        np.add.at(offs, src + 1, 1)
        cases.append(type("G", (), dict(offs=np.cumsum(offs), cols=dst.astype(np.int32)))())
    for g in cases:
        mine = gsw.graph_features_host(g.offs, g.cols)
        ref = ofeat.graph_features(g.offs, g.cols)
        np.testing.assert_allclose(mine, ref, rtol=1e-12, atol=0)


def _write(tmp_path, name, obj):
    import json

    p = tmp_path / name
    p.write_text(obj if isinstance(obj, str) else json.dumps(obj))
    return str(p)


def test_tree_load_matches_tree_create(tmp_path):
    """gsw_tree_load reads the JSON export into the same tree that
    gsw_tree_create builds from the arrays (and sklearn predicts)."""
    from sklearn.tree import DecisionTreeClassifier

    rng = np.random.default_rng(3)
    X = np.abs(rng.normal(size=(500, gsw.N_FEATURES))) * 10.0 ** rng.integers(0, 6, gsw.N_FEATURES)
    y = (X[:, 20] > np.median(X[:, 20])).astype(int) + 2 * (X[:, 3] > np.median(X[:, 3]))
    clf = DecisionTreeClassifier(max_depth=5, random_state=0).fit(X, y)
    T = _export(clf, [gsw.PULL_BITMAP, gsw.PUSH_EDGE, gsw.kernel_id(gsw.REV_EDGE_SCAN, gsw.COUNT_THREAD),
                      gsw.PUSH_VERTEX])
    T["feature_names"] = list(gsw.FEATURE_NAMES)
    T["report"] = {"nested": [1, {"a": None, "b": True}], "text": "\u00e9\"x\""}
    path = _write(tmp_path, "t.json", T)
    loaded = gsw.Tree.load(path)
    built = gsw.Tree(T)
    for x in X[:200]:
        for prev, lev in ((0, 0), (gsw.PUSH_WAVE8, 2)):
            assert loaded.predict(x, prev, lev) == built.predict(x, prev, lev)


@pytest.mark.parametrize("text,msg", [
    ("{", "not a JSON object"),
    ("[1, 2]", "not a JSON object"),
    ('{"feature": [0], "threshold": [0.0], "left": [-1], "right": [-1], "value": [[1.0]]}', "class_kernel"),
    ('{"feature": [0, 1], "threshold": [0.0], "left": [-1], "right": [-1], "value": [[1.0]], '
     '"class_kernel": [0]}', "differ in length"),
    ('{"feature": [0], "threshold": [0.0], "left": [-1], "right": [-1], "value": [[1.0, 2.0]], '
     '"class_kernel": [0]}', "classes"),
    ('{"feature": [0.5], "threshold": [0.0], "left": [-1], "right": [-1], "value": [[1.0]], '
     '"class_kernel": [0]}', "non-integer"),
    ('{"feature_names": ["deg_min"], "feature": [0], "threshold": [0.0], "left": [-1], "right": [-1], '
     '"value": [[1.0]], "class_kernel": [0]}', "feature_names"),
    ("[" * 100 + "]" * 100, "not a JSON object"),
])
def test_tree_load_rejects_malformed(tmp_path, text, msg):
    path = _write(tmp_path, "bad.json", text)
    with pytest.raises(gsw.GswError) as ei:
        gsw.Tree.load(path) if not text.startswith("[") and text != "{" else _load_raw(path)
    assert ei.value.status == gsw.EINVAL and msg in str(ei.value)


def _load_raw(path):
    import ctypes

    out = ctypes.c_void_p()
    gsw._check(gsw.lib().gsw_tree_load(os.fsencode(path), ctypes.byref(out)))


def test_tree_load_missing_file(tmp_path):
    with pytest.raises(gsw.GswError) as ei:
        _load_raw(str(tmp_path / "nope.json"))
    assert ei.value.status == gsw.EINVAL


def test_shipped_trees_load():
    from paper_1708_01159_amd import trees

    for name in ("seed", "mi355x"):
        t = gsw.Tree.load(trees.path(name))
        assert t.n_nodes >= 1


class _FakeGraph:
    n = 10
    handle = None


@pytest.mark.parametrize("make,msg", [
    (lambda torch: torch.zeros((1, 10), dtype=torch.int32), "CUDA tensor"),
    (lambda torch: np.zeros((1, 10), dtype=np.int32), "CUDA tensor"),
])
def test_binding_rejects_bad_outputs(make, msg):
    """Output buffers are checked before any C call: a CPU tensor, a numpy
    array where device memory is expected, the wrong dtype, a strided or
    short tensor would otherwise be written out of bounds by the GPU."""
    import torch

    with pytest.raises(ValueError) as ei:
        gsw.check_out(make(torch), "int32", 10, True, "levels")
    assert msg in str(ei.value)


def test_check_out_rules():
    import torch

    ok = np.zeros(20, dtype=np.int32)
    gsw.check_out(ok, "int32", 20, False, "x")
    with pytest.raises(ValueError, match="int8"):
        gsw.check_out(ok, "int8", 20, False, "x")
    with pytest.raises(ValueError, match="need"):
        gsw.check_out(ok, "int32", 21, False, "x")
    with pytest.raises(ValueError, match="contiguous"):
        gsw.check_out(np.zeros(40, dtype=np.int32)[::2], "int32", 20, False, "x")
    with pytest.raises(ValueError, match="host output"):
        gsw.check_out(torch.zeros(20, dtype=torch.int32), "int32", 20, False, "x")
    with pytest.raises(ValueError, match="no buffer"):
        gsw.check_out(None, "int32", 1, True, "x")
    # the public entry points run the checks before touching the library
    with pytest.raises(ValueError):
        gsw.bfs(_FakeGraph(), [0], policy="fixed", kernel=0, device=True,
                out=(torch.zeros((1, 10), dtype=torch.int32), None))
    with pytest.raises(ValueError):
        gsw.msbfs(_FakeGraph(), [0], out=torch.zeros((1, 10), dtype=torch.int8))


def test_components_abi_constants_layout_and_null_arguments():
    """gsw_cc's enums and structs as the binding lays them out, its defaults,
    and its argument checks that need no GPU."""
    import ctypes

    text = open(os.path.join(ROOT, "include", "gsw.h")).read()
    pol = dict((m.group(1), int(m.group(2))) for m in re.finditer(r"GSW_CC_(SWITCH|PUSH|PULL) = (\d+)", text))
    assert (pol["SWITCH"], pol["PUSH"], pol["PULL"]) == (gsw.CC_SWITCH, gsw.CC_PUSH, gsw.CC_PULL)
    ks = dict((m.group(1), int(m.group(2))) for m in re.finditer(r"GSW_CC_K_(BFS|PUSH|PULL) = (\d+)", text))
    assert [ks["BFS"], ks["PUSH"], ks["PULL"]] == [gsw.CC_K_BFS, gsw.CC_K_PUSH, gsw.CC_K_PULL]
    assert gsw.CC_KERNEL_NAMES[gsw.CC_K_PULL] == "pull"
    assert ctypes.sizeof(gsw.CcTrace) == 40 and gsw.CcTrace.ms.offset == 32
    assert ctypes.sizeof(gsw.CcOpts) == 32 and gsw.CcOpts.stream.offset == 24
    o = gsw.CcOpts()
    gsw.lib().gsw_cc_opts_default(ctypes.byref(o))
    assert (o.policy, o.bfs_first, o.device_ptrs) == (gsw.CC_SWITCH, 1, 0)
    assert abs(o.pull_above - 0.05) < 1e-7 and o.tree is None and o.stream is None
    lab = np.zeros(4, dtype=np.int32)
    nc = ctypes.c_int64(-1)
    st = gsw.lib().gsw_cc(None, lab.ctypes.data, ctypes.byref(nc), None, 0, None, ctypes.byref(o))
    assert st == gsw.EINVAL and nc.value == 0 and "null graph" in gsw.last_error()


def test_components_binding_checks_outputs_before_the_call():
    import torch

    with pytest.raises(ValueError, match="CUDA tensor"):
        gsw.components(_FakeGraph(), device=True, out=torch.zeros(10, dtype=torch.int32))
    with pytest.raises(ValueError, match="need"):
        gsw.components(_FakeGraph(), out=np.zeros(9, dtype=np.int32))
    with pytest.raises(ValueError, match="host output"):
        gsw.components(_FakeGraph(), out=torch.zeros(10, dtype=torch.int32))
    with pytest.raises(KeyError):
        gsw.components(_FakeGraph(), policy="sideways")
