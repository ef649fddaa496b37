"""Pins of the oracle's lattice, horizon, notch and pad geometry against
brute force, closed-form counts and the paper's level table."""
import itertools
import os
from fractions import Fraction

import numpy as np
import pytest

import workloads as W
from oracle import geometry as G

HERE = os.path.dirname(os.path.abspath(__file__))


def brute_force_bonds(shape, dx, delta):
    """O(M^2) pairwise distance test on cell-centred positions."""
    pos = G.node_positions(shape, dx)
    M = len(pos)
    out = set()
    for a in range(M):
        for b in range(a + 1, M):
            d2 = float(np.sum((pos[a] - pos[b]) ** 2))
            if d2 <= delta * delta:
                out.add((a, b))
    return out


@pytest.mark.parametrize("shape", [(2, 2, 2), (4, 4, 4), (7, 5, 3), (5, 1, 6)])
def test_bonds_match_brute_force(shape):
    bi, bj, v = G.unique_bonds(shape, W.M_RATIO)
    got = set(zip(bi.tolist(), bj.tolist()))
    assert got == brute_force_bonds(shape, 1.0, W.M_RATIO)
    assert np.all(bi < bj)
    # the stored offset is the lattice offset of j relative to i
    nx, ny, _ = shape
    gi = np.stack([bi % nx, (bi // nx) % ny, bi // (nx * ny)], 1)
    gj = np.stack([bj % nx, (bj // nx) % ny, bj // (nx * ny)], 1)
    assert np.array_equal(gj - gi, v)


def test_stencil_is_the_122_point_ball():
    st = G.stencil(W.M_RATIO)
    assert len(st) == 122
    # delta = pi dx gives the same neighbourhood (no lattice point between 3.14 and pi)
    assert len(G.stencil(np.pi)) == 122
    assert {tuple(x) for x in st} == {tuple(-x) for x in st}


def closed_form_count(shape, m):
    """Number of unordered neighbour pairs: for each offset v, the number of
    lattice points p with p and p + v both inside is prod_d (n_d - |v_d|)."""
    r = int(np.ceil(m))
    tot = 0
    for v in itertools.product(range(-r, r + 1), repeat=3):
        n2 = sum(x * x for x in v)
        if 0 < n2 <= m * m:
            tot += int(np.prod([max(0, n - abs(x)) for n, x in zip(shape, v)]))
    return tot // 2


@pytest.mark.parametrize("shape", [(35, 10, 10), (70, 20, 20), (9, 4, 7)])
def test_bond_count_closed_form(shape):
    bi, _, _ = G.unique_bonds(shape, W.M_RATIO)
    assert bi.size == closed_form_count(shape, W.M_RATIO)


def test_paper_level_table_node_counts():
    """Cell-centred lattice convention pinned by the paper's level table."""
    rows = [l.split() for l in open(os.path.join(HERE, "golden", "table_discretisation.txt"))
            if l.strip() and not l.startswith("#")]
    for lev, dx_mm, nodes in rows:
        nx, ny, nz = G.grid_shape((350e-3, 1e-3 * float(dx_mm), 100e-3), 1e-3 * float(dx_mm))
        assert ny == 1
        assert nx * nz == int(nodes)


def brute_force_notch(shape, dx, x_notch, a):
    """Rational segment / notch-plane intersection in physical units: the bond
    from p1 to p2 crosses the plane x = x_notch (entering the closed right-hand
    side) at parameter t = (x_notch - x1)/(x2 - x1); it is cut when the
    crossing height is strictly below the tip a."""
    dx = Fraction(dx); x_notch = Fraction(x_notch); a = Fraction(a)
    nx, ny, nz = shape
    def pos(n):
        return ((n % nx) * dx + dx / 2, (n // (nx * ny)) * dx + dx / 2)
    bi, bj, _ = G.unique_bonds(shape, W.M_RATIO)
    out = []
    for p, q in zip(bi.tolist(), bj.tolist()):
        (x1, z1), (x2, z2) = pos(p), pos(q)
        if x1 == x2 or not (min(x1, x2) < x_notch <= max(x1, x2)):
            out.append(False)
            continue
        t = (x_notch - x1) / (x2 - x1)
        out.append(z1 + t * (z2 - z1) < a)
    return np.array(out)


@pytest.mark.parametrize("shape,xn,a", [((8, 2, 6), 4, 2), ((9, 3, 7), 4.5, 3), ((12, 1, 10), 6, 4),
                                        ((7, 2, 8), 3.5, 1)])
def test_notch_cut_matches_rational_brute_force(shape, xn, a):
    bi, bj, _ = G.unique_bonds(shape, W.M_RATIO)
    got = G.notch_cut_mask(shape, 1.0, bi, bj, xn, a)
    ref = brute_force_notch(shape, 1, Fraction(xn).limit_denominator(2), Fraction(a).limit_denominator(2))
    assert got.sum() > 0
    assert np.array_equal(got, ref)


def test_notch_levels_and_pads():
    """Beam levels: cut counts stay consistent and pads cover the same volume
    on every level (10 / 80 / 640 nodes per pad)."""
    for ell, per_pad in ((0, 10), (1, 80)):
        lv = W.level(ell)
        shape = lv.shape
        bi, bj, _ = G.unique_bonds(shape, W.M_RATIO)
        cut = G.notch_cut_mask(shape, lv.dx, bi, bj, 0.5 * lv.beam.length, lv.beam.notch_depth)
        assert 0 < cut.sum() < 0.01 * bi.size
        sup, load = G.beam_pads(shape, lv.dx, lv.beam)
        assert sup.size == 2 * per_pad and load.size == per_pad
        pos = G.node_positions(shape, lv.dx)
        assert np.all(pos[sup, 2] < lv.beam.pad_width)
        assert np.all(pos[load, 2] > lv.beam.depth - lv.beam.pad_width)
