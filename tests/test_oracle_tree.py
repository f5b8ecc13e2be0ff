"""Pins of the oracle's tree and lists (Sec. 2.1, 2.2, Table 1, Fig. 1).

* the worked example of Fig. 1 (stored under tests/golden/ with its citation);
* a closed form for the mean interaction-list size on a full 3D grid;
* brute force: cells, depth and lists recomputed from the definitions with
  real-valued geometry on small random inputs;
* the coverage property of the H2 partition: every ordered pair of points is
  in exactly one near block or one interaction-list block.
"""
import itertools
import json
import os

import numpy as np
import pytest

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def grid_points(d, side):
    """One point at the centre of every cell of a side^d grid on [0,1]^d,
    plus the two corners so that the bounding cube is exactly [0,1]^d."""
    c = (np.arange(side) + 0.5) / side
    g = np.array(list(itertools.product(c, repeat=d)))
    return np.vstack([g, np.zeros(d), np.ones(d)])


def cell_index(tree, l, coord):
    cells = tree.cells(l)
    hit = np.where((cells["coord"] == np.array(coord)).all(1))[0]
    assert hit.size == 1
    return int(hit[0])


def test_fig1_worked_example(orc):
    g = json.load(open(os.path.join(GOLDEN, "fig1_lists.json")))
    p = grid_points(2, 8)
    T = orc.Tree(p, leaf_size=3, eta2=tuple(g["eta2"]))
    assert T.kappa == 3
    for case in g["cases"]:
        l = case["level"]
        b = cell_index(T, l, case["cell"])
        nptr, _ = T.lists(l, "nb")
        iptr, _ = T.lists(l, "il")
        assert nptr[b + 1] - nptr[b] == case["neighbours"], case
        assert iptr[b + 1] - iptr[b] == case["interaction_list"], case


def test_mean_interaction_list_closed_form(orc):
    # Full 32^3 grid: per axis the parent-neighbour children span 4 cells at
    # the two first/last positions and 6 elsewhere (mean 5.75); the neighbour
    # span is 2 at the ends and 3 elsewhere (mean 2.9375).  The axes are
    # independent, so the mean |IL| is 5.75^3 - 2.9375^3.
    p = grid_points(3, 32)
    T = orc.Tree(p, leaf_size=3)
    assert T.kappa == 5
    ptr, _ = T.lists(5, "il")
    sizes = np.diff(ptr)
    assert abs(sizes.mean() - (5.75 ** 3 - 2.9375 ** 3)) < 1e-12
    assert sizes.max() == 189
    nptr, _ = T.lists(5, "nb")
    assert abs(np.diff(nptr).mean() - 2.9375 ** 3) < 1e-12


def test_literal_sqrt2_in_3d(orc):
    # eta = sqrt(2) taken literally in 3D: admissible iff sum g^2 >= 2, which
    # gives 27 + 6*9 = 81 neighbours and 8*81 - 81 = 567 cells in the list of
    # an interior cell.
    p = grid_points(3, 16)
    T = orc.Tree(p, leaf_size=3, eta2=(2, 1))
    b = cell_index(T, 4, [8, 8, 8])
    nptr, _ = T.lists(4, "nb")
    iptr, _ = T.lists(4, "il")
    assert nptr[b + 1] - nptr[b] == 81
    assert iptr[b + 1] - iptr[b] == 567


def _brute(p, leaf, eta2):
    n, d = p.shape
    lo = p.min(0)
    L = (p.max(0) - lo).max()
    kmax = 60 // d

    def coords(l):
        u = (p - lo) / L
        return np.minimum(np.floor(u * 2.0 ** l), 2 ** l - 1).astype(np.int64)

    kappa = kmax
    for l in range(kmax + 1):
        _, cnt = np.unique(coords(l), axis=0, return_counts=True)
        if cnt.max() <= leaf:
            kappa = l
            break
    levels = []
    for l in range(kappa + 1):
        levels.append(sorted({tuple(c) for c in coords(l)}))

    def adm(a, b, l):
        h = L / 2 ** l
        diam = h * np.sqrt(d)
        gap = np.maximum(np.abs(np.array(a) - np.array(b)) - 1, 0) * h
        dist = np.sqrt((gap ** 2).sum())
        return diam * diam <= eta2 * dist * dist * (1 + 1e-12)

    nb, il = [], []
    for l in range(kappa + 1):
        cells = levels[l]
        nbl = {c: {o for o in cells if not adm(c, o, l)} for c in cells}
        nb.append(nbl)
        if l == 0:
            il.append({c: set() for c in cells})
            continue
        par = nb[l - 1]
        ill = {}
        for c in cells:
            pc = tuple(v >> 1 for v in c)
            cand = {o for o in cells if tuple(v >> 1 for v in o) in par[pc]}
            ill[c] = {o for o in cand if adm(c, o, l)}
        il.append(ill)
    return kappa, levels, nb, il, coords


@pytest.mark.parametrize("d,n,leaf,eta2", [(2, 400, 5, (2, 1)), (3, 500, 6, (3, 1)), (3, 300, 4, (2, 1)), (2, 300, 4, (1, 2))])
def test_tree_and_lists_brute_force(orc, d, n, leaf, eta2):
    rng = np.random.default_rng(10 + d)
    p = rng.uniform(-1, 1, (n, d))
    p[:3] = p[3]   # duplicates
    T = orc.Tree(p, leaf, eta2=eta2)
    kappa, levels, nb, il, coords = _brute(p, leaf, eta2[0] / eta2[1])
    assert T.kappa == kappa
    order = T.order()
    assert sorted(order.tolist()) == list(range(n))
    for l in range(kappa + 1):
        cells = T.cells(l)
        got = [tuple(c) for c in cells["coord"]]
        assert sorted(got) == levels[l]
        # every point of a cell lies in the cell's contiguous range
        cp = coords(l)[order]
        for b, c in enumerate(got):
            f, k = cells["first"][b], cells["count"][b]
            assert (cp[f:f + k] == np.array(c)).all()
        assert cells["count"].sum() == n
        for which, ref in (("nb", nb[l]), ("il", il[l])):
            ptr, idx = T.lists(l, which)
            for b, c in enumerate(got):
                lst = idx[ptr[b]:ptr[b + 1]]
                assert list(lst) == sorted(lst)
                assert {got[e] for e in lst} == ref[c], (l, which, c)


@pytest.mark.parametrize("d,n,leaf,eta2", [(2, 600, 8, (2, 1)), (3, 700, 10, (3, 1)), (3, 400, 5, (2, 1))])
def test_partition_covers_each_pair_once(orc, d, n, leaf, eta2):
    rng = np.random.default_rng(20 + d)
    p = rng.uniform(-1, 1, (n, d))
    T = orc.Tree(p, leaf, eta2=eta2)
    order = T.order()
    cover = np.zeros((n, n), np.int64)
    for l in range(T.kappa + 1):
        cells = T.cells(l)
        rng_of = [order[f:f + k] for f, k in zip(cells["first"], cells["count"])]
        ptr, idx = T.lists(l, "il")
        for b in range(len(rng_of)):
            for e in idx[ptr[b]:ptr[b + 1]]:
                cover[np.ix_(rng_of[b], rng_of[e])] += 1
        if l == T.kappa:
            ptr, idx = T.lists(l, "nb")
            for b in range(len(rng_of)):
                for e in idx[ptr[b]:ptr[b + 1]]:
                    cover[np.ix_(rng_of[b], rng_of[e])] += 1
    assert (cover == 1).all()


def test_degenerate_trees(orc):
    # all points identical: a single leaf (the direct sum)
    T = orc.Tree(np.ones((50, 3)), 4)
    assert T.kappa == 0 and T.ncell(0) == 1
    # fewer points than the leaf size
    T = orc.Tree(np.random.default_rng(0).uniform(size=(10, 2)), 64)
    assert T.kappa == 0
    # a single point
    T = orc.Tree(np.zeros((1, 3)), 1)
    assert T.kappa == 0
    # many duplicates: depth capped at 60/d, the over-full leaf is kept
    p = np.vstack([np.zeros((20, 2)), np.ones((1, 2))])
    T = orc.Tree(p, 4)
    assert T.kappa == 30
    assert T.cells(30)["count"].max() == 20
