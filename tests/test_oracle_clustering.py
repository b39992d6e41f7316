"""Pins of the oracle's Berger-Rigoutsos clustering (the AMR method's
clustering, Sec. 2.2, as a variant tiler that keeps patches unions of whole
pmin-blocks inside one pmax-block).  Hand-worked examples of the rules
(shrink, efficiency, hole, inflection, bisection), invariants on random
weight grids (disjoint, covering, tight, efficient or single), and adaptive
runs with the clustering (hierarchy invariants, flag coverage, conservation,
reduction to the bounding box at eta = 0)."""
import numpy as np
import pytest

from paper_1603_05211_amd import inputs

from test_oracle_adaptive import check_hierarchy, coarsen_mask

G = 1.4
FULL = 16   # flagged parent cells of a fully flagged 2D sub-block (q = 4)


def boxes(orc, W, eta=0.8, q=4):
    return [tuple(int(v) for v in r) for r in orc.br_cluster(W, q, eta)]


def test_l_shape_worked_example(orc):
    """Row y = 0 and column x = 0 of a 4 x 4 grid flagged (7 of 16): no hole
    and no inflection (second differences 3, 0 along both axes), so the box
    is halved along x (tie: x) into columns 0-1 and 2-3; columns 0-1 (5 of 8)
    are halved along y (the longer) into rows 0-1 and 2-3; rows 0-1 (3 of 4)
    are halved along x into (0, 0..1), emitted (2 of 2), and (1, 0..1),
    shrunk to (1, 0); rows 2-3 shrink to (0, 2..3); columns 2-3 shrink to
    row 0."""
    W = np.zeros((4, 4), np.int32)
    W[0, :] = FULL
    W[:, 0] = FULL
    assert boxes(orc, W) == [(0, 0, 0, 0, 1, 0), (1, 0, 0, 1, 0, 0), (0, 2, 0, 0, 3, 0), (2, 0, 0, 3, 0, 0)]


def test_hole_splits_two_clusters(orc):
    W = np.zeros((4, 4), np.int32)
    W[0, 0] = FULL
    W[3, 3] = 5
    assert boxes(orc, W) == [(0, 0, 0, 0, 0, 0), (3, 3, 0, 3, 3, 0)]
    # a hole nearest the middle: columns 0 and 3 flagged, 1 and 2 empty ->
    # cut at 1 (|2 i - 3| = 1 for i = 1 and 2; the lower one)
    W = np.zeros((4, 4), np.int32)
    W[:, 0] = FULL
    W[:, 3] = FULL
    assert boxes(orc, W) == [(0, 0, 0, 0, 3, 0), (3, 0, 0, 3, 3, 0)]


def test_inflection_then_bisection_worked_example(orc):
    """One row of an 8 x 8 grid with weights 16, 16, 16, 4, 4, 4, 4, 4 (68 of
    128): the second differences 0, -12, 12, 0, 0, 0 change sign between x =
    2 and 3 (strength 24): x 0-2 is emitted (48 of 48); x 3-7 (20 of 80) has
    flat signatures and is halved, the lower part taking the smaller share:
    3-4 then 5-7, which split down to single sub-blocks."""
    W = np.zeros((8, 8), np.int32)
    W[0, :] = [16, 16, 16, 4, 4, 4, 4, 4]
    assert boxes(orc, W) == [(0, 0, 0, 2, 0, 0), (3, 0, 0, 3, 0, 0), (4, 0, 0, 4, 0, 0), (5, 0, 0, 5, 0, 0),
                             (6, 0, 0, 6, 0, 0), (7, 0, 0, 7, 0, 0)]


def test_full_grid_and_eta_zero(orc):
    W = np.full((4, 4), FULL, np.int32)
    assert boxes(orc, W) == [(0, 0, 0, 3, 3, 0)]
    W = np.zeros((4, 4, 4), np.int32)
    W[1, 2, 0] = 3
    W[3, 0, 3] = 1
    # eta = 0: the bounding box of the flagged sub-blocks, once
    assert boxes(orc, W, eta=0.0) == [(0, 0, 1, 3, 2, 3)]
    # 3D: a hole along z (the longest extent) separates them
    assert boxes(orc, W) == [(0, 2, 1, 0, 2, 1), (3, 0, 3, 3, 0, 3)]


@pytest.mark.parametrize("dim,R", [(2, 4), (2, 8), (3, 2), (3, 4)])
def test_invariants_on_random_grids(orc, dim, R):
    """Boxes are disjoint, cover every sub-block with flagged cells, are tight
    (each boundary slice holds one) and reach the efficiency eta unless they
    are a single sub-block."""
    rng = np.random.default_rng(7 + R + dim)
    q = 4
    cap = q ** dim
    for trial in range(60):
        W = np.where(rng.random((R,) * dim) < rng.uniform(0.1, 0.7), rng.integers(1, cap + 1, (R,) * dim), 0)
        W = W.astype(np.int32)
        for eta in (0.5, 0.8, 1.0):
            B = boxes(orc, W, eta=eta, q=q)
            cover = np.zeros(W.shape, np.int32)
            for b in B:
                lo, hi = b[:3][:dim], b[3:][:dim]
                sl = tuple(slice(l, h + 1) for l, h in zip(lo[::-1], hi[::-1]))
                cover[sl] += 1
                sub = W[sl]
                assert sub.sum() > 0
                for ax in range(dim):
                    first = np.take(sub, 0, axis=ax)
                    last = np.take(sub, -1, axis=ax)
                    assert first.sum() > 0 and last.sum() > 0
                single = sub.size == 1
                assert single or sub.sum() >= eta * sub.size * cap
            assert cover.max() <= 1 and (cover[W > 0] == 1).all()


def br_hierarchy(orc, eta=0.8, bc=0, prim_seed=5):
    h = orc.Hierarchy(2, 4, 32, eps=1e-3, eta=eta, bc=bc, tiler=orc.TILER_BR)
    h.init_finest(orc.init_quadrant(256, G, inputs.quadrant_states(prim_seed)))
    return h


def test_adaptive_runs_with_clustering(orc):
    h = br_hierarchy(orc)
    b = orc.Hierarchy(2, 4, 32, eps=1e-3, eta=0.8)
    b.init_finest(orc.init_quadrant(256, G, inputs.quadrant_states(5)))
    for _ in range(4):
        h.step(0.45)
        b.step(0.45)
        P, acts = check_hierarchy(h)
        for l in range(h.L - 1):
            F = h.flags(l).astype(bool)
            assert not (F & ~coarsen_mask(acts[l + 1], 2)).any()
    assert not np.array_equal(h.patches(), b.patches())   # rectangles, not squares


def test_eta_zero_gives_bounding_boxes(orc):
    """eta = 0: every pmax block with flags becomes one patch, the bounding
    box of its flagged pmin-blocks."""
    h = br_hierarchy(orc, eta=0.0)
    P, acts = check_hierarchy(h)
    for lv, ox, oy, oz, sx, sy, sz in P:
        F = h.flags(lv - 1).astype(bool)
        bx, by = ox // 32 * 32, oy // 32 * 32
        blk = F[by // 2:(by + 32) // 2, bx // 2:(bx + 32) // 2]
        ys, xs = np.nonzero(blk.reshape(4, 4, 4, 4).any(axis=(1, 3)))
        assert (ox - bx) // 8 == xs.min() and (ox - bx + sx) // 8 - 1 == xs.max()
        assert (oy - by) // 8 == ys.min() and (oy - by + sy) // 8 - 1 == ys.max()


def test_clustering_conserves_periodic(orc):
    h = br_hierarchy(orc, bc=orc.BC_PERIODIC, prim_seed=6)
    T0 = h.totals()
    for _ in range(8):
        h.step(0.4)
    check_hierarchy(h, periodic=True)
    assert np.all(np.abs(h.totals() - T0) <= 2e-13 * np.maximum(1.0, np.abs(T0)))
