"""The profile summary's attribution of level-kernel dispatches to the
variant each ran, from the benchmark's dispatch log (no GPU)."""
from paper_1708_01159_amd import gsw
from paper_1708_01159_amd import profile_summary as ps

K = "gsw::(anonymous namespace)::"


def _d(name):
    return (K + name + "(gsw::BfsBase, gsw::BfsPolicy, int)", 1.0)


def test_align_by_launch_index():
    disp = [(K + "k_init(...)", 1.0), _d("k_level_solo"), _d("k_level_auto"), _d("k_level_auto"),
            _d("k_level_auto"), _d("k_level_solo"), _d("k_level_auto"), _d("k_level_auto"),
            (K + "k_init(...)", 1.0), _d("k_level_solo"), _d("k_level_auto"), _d("k_level_auto")]
    pe, pull, pv = gsw.PUSH_EDGE, gsw.PULL_BITMAP, gsw.PUSH_VERTEX
    calls = [
        {"levels": [  # kernel, frontier, bytes, literal bytes, launch, flags
            [pv, 1, 10, None, 0, 4], [pv, 3, 11, None, 0, 4],   # two levels in one single-workgroup launch
            [pe, 900, 500, None, 2, 0],                          # push_edge in two launches (1 = prefix)
            [pull, 5000, 700, 900, 3, 0],
            [pv, 7, 12, None, 5, 0]]},                           # launch 4 handed its level on
        {"levels": [[pe, 1, 20, None, 1, 0]]},                   # launch 0 handed the hub source on
    ]
    lab = ps._align(disp, calls, gsw.KERNEL_NAMES)
    names = [l[0] if l else None for l in lab]
    assert names == [None, "single-workgroup launch", "push_edge (prefix)", "push_edge (expand)", "pull_bitmap",
                     "(no level completed)", "push_vertex", "(no level completed)",
                     None, "(no level completed)", "push_edge", "(no level completed)"]
    assert lab[3][1] == 500 and lab[4][1:] == (700, 900) and lab[6][1] == 12
