"""Pins of the oracle's preconditioner (Sec. 4.2, eq. localmatix) against
the oracle's Nystrom matrix and hand-built subdomains.

In a medium whose layers share k and eta the reaction part vanishes, so the
Nystrom matrix K restricted to one layer is exactly the matrix the
preconditioner approximates.  With one box per layer the preconditioner is
K^{-1}; with boxes that have no neighbours it is the block inverse; with a
chain of neighbouring boxes it is the sum of the kept rows of the local
inverses over neighbourhoods written down by hand.  A wrong weight (|Gamma|
on the row instead of the column), a wrong self term, a dropped neighbour or a
wrong gather / scatter fails one of these.
"""

import numpy as np
import pytest

from oracle import precond as pre
from oracle.medium import Medium
from oracle.nystrom import Elements, matrix


def _circle(c, r, n, phase=0.0):
    t = phase + 2 * np.pi * np.arange(n) / n
    return np.stack([c[0] + r * np.cos(t), c[1] + r * np.sin(t)], axis=1)


HOMOG = Medium([0.0], [2.0, 2.0])  # w_top = 4


def _chain():
    """Clusters at level-0 cells (0,0), (1,0), (2,0), (4,0) of layer 0 and
    (0,0) of layer 1."""
    polys = [_circle((2.0 + 4.0 * c, 1.5), 0.4, 12, 0.1 * c) for c in (0, 1, 2, 4)]
    polys.append(_circle((2.0, -1.5), 0.4, 12, 0.3))
    return polys


@pytest.fixture(scope="module")
def chain():
    el = Elements(HOMOG, _chain())
    return el, matrix(HOMOG, el)


def test_local_matrix_is_the_homogeneous_nystrom_matrix(chain):
    el, K = chain
    own = np.nonzero(el.layer == 0)[0]
    P = pre.local_matrix(HOMOG, el, own)
    assert np.allclose(P, K[np.ix_(own, own)], rtol=1e-12, atol=1e-14)


def test_cells_of_the_chain(chain):
    el, _ = chain
    grid = pre.BoxGrid(HOMOG, el)
    i, j = grid.cells(0)
    for s, col in enumerate((0, 1, 2, 4, 0)):
        sel = el.scatterer == s
        assert np.all(i[sel] == col) and np.all(j[sel] == 0), s
    assert np.all(el.layer[el.scatterer == 4] == 1) and np.all(el.layer[el.scatterer < 4] == 0)


def test_chain_subdomains_by_hand(chain):
    """Neighbourhoods of the chain written down by hand: cell 0 meets 1,
    cell 1 meets 0 and 2, cell 2 meets 1, cell 4 and the layer-1 cluster
    meet nothing."""
    el, K = chain
    sc = [np.nonzero(el.scatterer == s)[0] for s in range(5)]
    hand = [(sc[0], [sc[0], sc[1]]), (sc[1], [sc[1], sc[0], sc[2]]), (sc[2], [sc[2], sc[1]]),
            (sc[3], [sc[3]]), (sc[4], [sc[4]])]
    M = np.zeros((el.n, el.n), dtype=complex)
    for own, parts in hand:
        J = np.concatenate(parts)
        Zi = np.linalg.inv(K[np.ix_(J, J)])
        M[np.ix_(own, J)] += Zi[: len(own)]
    got = pre.dense(HOMOG, el, 0, 0)
    assert np.allclose(got, M, rtol=1e-10, atol=1e-12 * np.abs(M).max())
    subs = pre.subdomains(HOMOG, el, 0, 0)
    assert sorted(tuple(sorted(o)) for o, _ in subs) == sorted(tuple(sorted(o)) for o, _ in hand)
    rng = np.random.default_rng(7)
    x = rng.standard_normal((3, el.n)) + 1j * rng.standard_normal((3, el.n))
    assert np.allclose(pre.apply(HOMOG, el, 0, 0, x), x @ got.T, rtol=1e-10, atol=1e-12 * np.abs(x @ got.T).max())


def test_one_box_per_layer_is_the_inverse():
    """All of a layer in one level-0 box: the preconditioner is the inverse of
    the layer's block of K."""
    polys = [_circle((1.0, 1.2), 0.5, 20), _circle((2.4, 2.0), 0.3, 16, 0.2)]
    el = Elements(HOMOG, polys)
    K = matrix(HOMOG, el)
    M = pre.dense(HOMOG, el, 0, 0)
    assert np.allclose(M @ K, np.eye(el.n), atol=1e-10)


def test_isolated_boxes_give_the_block_inverse():
    polys = [_circle((2.0 + 8.0 * c, 1.5 + 4.0 * (c % 2)), 0.45, 14, 0.2 * c) for c in range(3)]
    el = Elements(HOMOG, polys)
    K = matrix(HOMOG, el)
    M = pre.dense(HOMOG, el, 0, 0)
    ref = np.zeros_like(M)
    for s in range(3):
        b = np.nonzero(el.scatterer == s)[0]
        ref[np.ix_(b, b)] = np.linalg.inv(K[np.ix_(b, b)])
    assert np.allclose(M, ref, rtol=1e-10, atol=1e-12 * np.abs(ref).max())


def test_levels_and_ancestors():
    """Coarser subdomains are unions of finer ones; the automatic level keeps
    neighbourhoods within the limit; c >= 2 steps c - 1 levels up."""
    med = Medium([0.0, 1.3], [2.0, 3.5, 2.5], [1.0, 2.0, 1.5])
    rng = np.random.default_rng(3)
    polys = [_circle((rng.uniform(-4, 4), rng.uniform(-3, 2)), 0.25, 24, rng.uniform(0, 6)) for _ in range(12)]
    el = Elements(med, polys)
    lev, lf = pre.level_for(med, el, 1, leaf_size=8)
    assert lev == lf >= 2
    assert pre.level_for(med, el, 2, leaf_size=8)[0] == lf - 1
    fine = {tuple(sorted(o)) for o, _ in pre.subdomains(med, el, lf, lf)}
    coarse = [set(o) for o, _ in pre.subdomains(med, el, lf - 1, lf)]
    for f in fine:
        assert sum(set(f) <= c for c in coarse) == 1
    assert sum(len(c) for c in coarse) == el.n
    for own, J in pre.subdomains(med, el, lf - 1, lf):
        assert np.all(el.layer[J] == el.layer[own[0]])
        assert list(J[: len(own)]) == list(own)
    auto, _ = pre.level_for(med, el, -1, leaf_size=8)
    assert auto == 0  # 288 elements: the top level fits
