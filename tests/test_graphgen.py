"""Seeded input generators: determinism, RNG definition, RMAT shape, CSR."""
import numpy as np
import pytest

import graphgen as gg


def test_splitmix64_published_vectors():
    # SplitMix64 started from state 0 emits these three words first; the
    # counter-based draw(seed=0, c) is exactly that stream.
    assert gg.draw(0, 0) == 0xE220A8397B1DCDAF
    assert gg.draw(0, 1) == 0x6E789E6AA1B965F4
    assert gg.draw(0, 2) == 0x06C45D188009454F


def test_draw_python_definition():
    def mix(z):
        m = 2**64 - 1
        z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & m
        z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & m
        return z ^ (z >> 31)

    for seed, c in [(1, 0), (12345, 99), (2**63 + 7, 2**40)]:
        ref = mix((seed + (c + 1) * 0x9E3779B97F4A7C15) & (2**64 - 1))
        assert gg.draw(seed, c) == ref


def test_rmat_deterministic_and_seed_sensitive():
    a = gg.rmat_edges(12, 50000, 7)
    b = gg.rmat_edges(12, 50000, 7)
    c = gg.rmat_edges(12, 50000, 8)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])
    assert not np.array_equal(a[0], c[0])


def test_rmat_quadrant_frequencies():
    scale, m = 10, 200000
    src, dst = gg.rmat_edges(scale, m, 11)
    top = scale - 1
    sb, db = (src >> top) & 1, (dst >> top) & 1
    freq = [np.mean((sb == 0) & (db == 0)), np.mean((sb == 0) & (db == 1)),
            np.mean((sb == 1) & (db == 0)), np.mean((sb == 1) & (db == 1))]
    for f, p in zip(freq, [0.57, 0.19, 0.19, 0.05]):
        sigma = np.sqrt(p * (1 - p) / m)
        assert abs(f - p) < 5 * sigma
    # every level is an independent draw: the lowest bit has the same law
    sb, db = src & 1, dst & 1
    assert abs(np.mean((sb == 0) & (db == 0)) - 0.57) < 5 * np.sqrt(0.57 * 0.43 / m)
    assert src.max() < 2**scale and dst.max() < 2**scale


def test_er_uniform():
    n, m = 1000, 200000
    src, dst = gg.er_edges(n, m, 3)
    assert src.max() < n and dst.max() < n
    counts = np.bincount(src, minlength=n)
    # chi-square against uniform, 999 dof: mean 999, sd ~44.7
    chi2 = np.sum((counts - m / n) ** 2 / (m / n))
    assert chi2 < 999 + 6 * 44.7


def test_csr_matches_edge_multiset():
    n = 300
    src, dst = gg.rmat_edges(8, 5000, 5)
    src = src % n
    dst = dst % n
    off, cols = gg.build_csr(n, src, dst)
    assert off[0] == 0 and off[-1] == len(src)
    assert np.all(np.diff(off.astype(np.int64)) >= 0)
    rows = np.repeat(np.arange(n), np.diff(off.astype(np.int64)))
    got = np.lexsort((cols, rows))
    assert np.all(got == np.arange(len(cols)))  # already sorted by (row, col)
    ref = np.lexsort((dst, src))
    assert np.array_equal(rows, src[ref]) and np.array_equal(cols, dst[ref])


def test_csr_long_rows_sorted():
    # a hub row longer than the radix threshold
    n = 70000
    rng = np.random.default_rng(0)
    dst = rng.integers(0, n, 20000, dtype=np.uint32)
    src = np.zeros_like(dst)
    off, cols = gg.build_csr(n, src, dst)
    assert np.array_equal(cols, np.sort(dst))


def test_csr_rejects_out_of_range():
    with pytest.raises(ValueError):
        gg.build_csr(4, np.array([0, 5], np.uint32), np.array([1, 1], np.uint32))


def test_symmetrize_doubles_multiset():
    src = np.array([0, 1, 2, 2], np.uint32)
    dst = np.array([1, 2, 2, 0], np.uint32)
    s2, d2 = gg.symmetrize(src, dst)
    pairs = sorted(zip(s2.tolist(), d2.tolist()))
    assert pairs == sorted([(0, 1), (1, 0), (1, 2), (2, 1), (2, 2), (2, 2), (2, 0), (0, 2)])


def test_weights_range_and_spread():
    w = gg.edge_weights(100000, 9)
    assert w.min() == 1 and w.max() == 255
    assert abs(w.mean() - 128.0) < 1.0


def test_sources_rule():
    g = gg.rmat_graph(12, 8, 21)
    deg = g.degrees()
    s = gg.pick_sources(g.offsets, 5, 8)
    assert len(s) == 8 and len(set(s.tolist())) == 8
    assert s[0] == int(np.argmax(deg))
    assert all(deg[v] > 0 for v in s)
    assert np.array_equal(s, gg.pick_sources(g.offsets, 5, 8))


def test_empty_and_tiny():
    off, cols = gg.build_csr(3, np.zeros(0, np.uint32), np.zeros(0, np.uint32))
    assert off.tolist() == [0, 0, 0, 0] and cols.size == 0
    assert gg.pick_sources(off, 1, 4).size == 0


def test_permute_vertices_is_an_isomorphism():
    g = gg.rmat_graph(10, 8, seed=gg.BASE_SEED + 123, symmetric=True)
    h, perm = gg.permute_vertices(g, 77)
    assert sorted(perm.tolist()) == list(range(g.n))
    assert h.m == g.m and h.n == g.n
    # degree of v in g equals degree of perm[v] in h
    assert np.array_equal(h.degrees()[perm], g.degrees())
    # edge multisets agree under the relabelling
    src = np.repeat(np.arange(g.n, dtype=np.uint64), g.degrees())
    a = np.sort(perm[src].astype(np.uint64) << 32 | perm[g.cols].astype(np.uint64))
    hsrc = np.repeat(np.arange(h.n, dtype=np.uint64), h.degrees())
    b = np.sort(hsrc << 32 | h.cols.astype(np.uint64))
    assert np.array_equal(a, b)
    # rows stay sorted; the same seed gives the same bytes
    for v in range(0, h.n, 97):
        row = h.cols[h.offsets[v]:h.offsets[v + 1]]
        assert np.all(row[1:] >= row[:-1])
    h2, _ = gg.permute_vertices(g, 77)
    assert np.array_equal(h2.cols, h.cols)


def test_inter_partition_fraction_counts_crossing_entries():
    # path 0-1-2-3 (both directions), partitions of 2 ids: only 1<->2 crosses
    g = gg.from_edges(4, [0, 1, 1, 2, 2, 3], [1, 0, 2, 1, 3, 2])
    assert gg.inter_partition_fraction(g, 1) == 2 / 6
    assert gg.inter_partition_fraction(g, 2) == 0.0
    assert gg.inter_partition_fraction(g, 0) == 1.0
    # a random relabelling of RMAT leaves almost every entry crossing
    r = gg.rmat_graph(12, 8, seed=gg.BASE_SEED + 5, symmetric=True)
    rp, _ = gg.permute_vertices(r, 3)
    assert gg.inter_partition_fraction(rp, 8) > 0.9 > gg.inter_partition_fraction(r, 8)
