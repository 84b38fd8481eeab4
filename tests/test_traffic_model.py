"""The byte model's per-level counts (C, one pass over the rows) against a
direct numpy walk of every unvisited row, and its totals by hand."""
import numpy as np

import oracle
from paper_1708_01159_amd import graphgen as gg
from paper_1708_01159_amd import traffic


def test_pull_counts_match_row_walk():
    for g in (gg.rmat(12, 16, seed=3), gg.grid(40, 31, 0.05, seed=4), gg.chung_lu(5000, 2.1, 8.0, seed=5),
              gg.from_edges(300, [0, 1, 2, 5], [1, 2, 3, 6])):  # isolated vertices, a small component
        for s in gg.pick_sources(g, 3, 6):
            lv = oracle.levels(g.offs, g.cols, int(s))
            c = traffic.Counts(g.offs, g.cols, lv, int(s))
            nf, ef = traffic.level_sizes(g.offs, lv)
            assert np.array_equal(c.nf[:len(nf)], nf) and np.array_equal(c.ef[:len(ef)], ef)
            for d in range(len(nf)):
                p, u = traffic.pull_probes_reference(g.offs, g.cols, lv, d)
                probes, unv_pos, unv_all = c.pull_terms(d)
                assert (probes, unv_pos) == (p, u), (g.name, int(s), d)
                assert unv_all == int(np.count_nonzero((lv == -1) | (lv > d)))
                words = np.unique(np.flatnonzero(lv == d + 1) >> 6).shape[0]
                assert c.at(c.words, d + 1) == words


def test_isolated_source_and_literal_formula():
    g = gg.from_edges(10, [1, 2], [2, 3])  # vertex 0 isolated
    lv = oracle.levels(g.offs, g.cols, 0)
    c = traffic.Counts(g.offs, g.cols, lv, 0)
    probes, unv_pos, unv_all = c.pull_terms(0)
    assert (probes, unv_pos, unv_all) == (4, 3, 9)  # rows of 1,2,3: 1+2+1 arcs, none in the frontier
    # literal: 1 word * 24 + 9 unvisited * 16 + 4 probes * 12 + 0 found
    assert traffic.pull_bytes_literal(c, 0) == 24 + 9 * 16 + 48
    # model: clear 8 + visited 8 + 3 * 16 + 4 * 12, no discoveries
    assert traffic.level_bytes(traffic.PULL, c, 0) == 8 + 8 + 48 + 48


def test_head_pull_counts_match_walk():
    """The model of the bottom-up level starting from the head, ranked and
    not, against a direct walk: head probes, row reads and row probes per
    level; without ranking a vertex probes max(p_v, h_v) arcs (the head is
    probed whole), so never fewer than the row-order p_v."""
    for g in (gg.rmat(10, 16, seed=3), gg.grid(30, 21, 0.05, seed=4), gg.chung_lu(3000, 2.1, 8.0, seed=5),
              gg.erdos_renyi(2000, 8000, seed=7), gg.from_edges(300, [0, 1, 2, 5], [1, 2, 3, 6])):
        for s in gg.pick_sources(g, 2, 6):
            lv = oracle.levels(g.offs, g.cols, int(s))
            for ranked in (True, False):
                c = traffic.Counts(g.offs, g.cols, lv, int(s), ranked=ranked)
                for d in range(int(lv.max()) + 1):
                    want = traffic.head_probes_reference(g.offs, g.cols, lv, d, ranked)
                    assert c.head_terms(d) == want, (g.name, int(s), d, ranked)
                    if not ranked:
                        assert want[0] >= traffic.pull_probes_reference(g.offs, g.cols, lv, d)[0]


def test_head_ranking_rule():
    """Ranked on skewed degree laws, not on narrow ones, as the library
    decides from its degree statistics."""
    assert traffic.head_is_ranked(gg.rmat(12, 16, seed=3).offs)
    assert traffic.head_is_ranked(gg.chung_lu(5000, 2.1, 8.0, seed=5).offs)
    assert not traffic.head_is_ranked(gg.erdos_renyi(5000, 20000, seed=6).offs)
    assert not traffic.head_is_ranked(gg.grid(40, 31, 0.05, seed=4).offs)
    assert not traffic.head_is_ranked(np.zeros(5, dtype=np.int64))


def test_ranked_head_order():
    # vertex 0's neighbours 1..6 with degrees 1, 3, 2, 3, 1, 4: the head is 6, 2, 4, 3
    src = [0] * 6 + [2, 2, 3, 4, 4, 6, 6, 6]
    dst = [1, 2, 3, 4, 5, 6] + [7, 8, 9, 10, 11, 12, 13, 14]
    g = gg.from_edges(15, src, dst)
    assert traffic.ranked_head(g.offs, g.cols, 0) == [6, 2, 4, 3]
