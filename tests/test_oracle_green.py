"""Pins of the oracle's layered Green's function.

* Sommerfeld identity: the quadrature machinery applied to the free-space
  plane-wave integrand reproduces (i/4) H_0^(1) (scipy) over the whole range
  of horizontal offsets and decay distances the workloads produce.
* Transmission conditions [G] = 0 and [eta dG/dy] = 0 at every interface for
  sources in every layer (the defining property of G, Sec. 3.1).
* eta-weighted reciprocity eta_l G_{l l'}(r, r') = eta_{l'} G_{l' l}(r', r).
* Homogeneous limit (reaction part vanishes within a layer, G_{l l'} = G^f
  across layers) and the image limits eta_1/eta_0 -> inf / 0.
"""

import numpy as np
import pytest
from scipy.special import hankel1

from oracle.green import LayeredGreen, free_space
from oracle.medium import Medium
from oracle.quadrature import bin_index, node_set, sommerfeld


def _free_integral(X, D, k, kmax):
    ix, idd = int(bin_index(X)), int(bin_index(D))
    nodes = node_set(kmax, ix, idd)
    facs = []
    for lam in (nodes[0], nodes[2], nodes[4]):
        if lam.size == 0:
            facs.append(None)
            continue
        ky = np.sqrt(k * k - lam * lam + 0j)
        ky = np.where(ky.imag < 0, -ky, ky)
        facs.append((1j / (2 * ky) * np.exp(1j * ky * D))[None, :])
    return sommerfeld(np.array([X]), facs[0], facs[1], facs[2], nodes)[0]


@pytest.mark.parametrize("X", [0.0, 1e-6, 1e-3, 0.05, 0.4, 1.0, 3.0, 10.0, 20.0, 45.0])
@pytest.mark.parametrize("D", [1e-6, 1e-3, 0.02, 0.3, 1.0, 4.0])
def test_sommerfeld_identity(X, D):
    k = 3.0
    got = _free_integral(X, D, k, kmax=8.0)
    ref = 0.25j * hankel1(0, k * np.hypot(X, D))
    assert abs(got - ref) <= 5e-13 * abs(ref)


GUIDED = Medium([0.0, 2.0], [5.0, 7.0, 4.0])           # interior layer fastest: real-axis poles
ETA3 = Medium([0.0, 1.3], [2.0, 3.5, 2.5], [1.0, 2.0, 1.5])
FIVE = Medium([0.0, 1.0, 2.0, 3.0], [3.2, 2.5, 5.1, 8.6, 6.9], [1.0, 2.0, 3.0, 4.0, 5.0])


def _src_in(med, l):
    if l == 0:
        return -med.d[0] + 0.6
    if l == med.L:
        return -med.d[-1] - 0.45
    return -0.5 * (med.d[l - 1] + med.d[l]) + 0.1


@pytest.mark.parametrize("med", [GUIDED, ETA3, FIVE], ids=["guided", "eta3", "five"])
def test_transmission_conditions(med):
    G = LayeredGreen(med)
    xs = 0.3
    for lp in range(med.L + 1):
        ys = _src_in(med, lp)
        for m in range(med.L):
            yi = -med.d[m]
            for x in (0.0, 1.3, 6.0):
                ga, dga = G.green(x, yi, [xs], [ys], l=m, lp=lp, dy=True)
                gb, dgb = G.green(x, yi, [xs], [ys], l=m + 1, lp=lp, dy=True)
                assert abs(ga[0] - gb[0]) <= 1e-12 * abs(ga[0]) + 1e-14, (lp, m, x)
                ja = med.eta[m] * dga[0]
                jb = med.eta[m + 1] * dgb[0]
                assert abs(ja - jb) <= 1e-11 * abs(ja) + 1e-13, (lp, m, x)


@pytest.mark.parametrize("med", [GUIDED, ETA3, FIVE], ids=["guided", "eta3", "five"])
def test_eta_weighted_reciprocity(med):
    G = LayeredGreen(med)
    rng = np.random.default_rng(0)
    for l in range(med.L + 1):
        for lp in range(med.L + 1):
            y, ys = _src_in(med, l) - 0.05, _src_in(med, lp) + 0.03
            x, xs = rng.uniform(-2, 2, 2)
            a = med.eta[l] * G.green(x, y, [xs], [ys], l=l, lp=lp)[0]
            b = med.eta[lp] * G.green(xs, ys, [x], [y], l=lp, lp=l)[0]
            assert abs(a - b) <= 1e-12 * abs(a), (l, lp)


def test_homogeneous_limit():
    med = Medium([0.0, 1.5], [3.0, 3.0, 3.0])
    G = LayeredGreen(med)
    xs = np.array([0.2, 1.4, -3.0])
    for l, y in ((0, 0.4), (1, -0.7), (2, -2.2)):
        for lp in range(3):
            ys = np.full(3, _src_in(med, lp))
            g = G.green(0.1, y, xs, ys, l=l, lp=lp)
            ref = free_space(3.0, 0.1, y, xs, ys)
            assert np.allclose(g, ref, rtol=1e-12, atol=1e-15)
            if l == lp:
                assert np.max(np.abs(G.reaction(l, lp, 0.1, y, xs, ys))) < 1e-15


@pytest.mark.parametrize("ratio,sign", [(1e12, -1.0), (1e-12, 1.0)])
def test_image_limits(ratio, sign):
    """eta_1/eta_0 -> inf: R -> -1 and G_00 -> G^f(r,r') - G^f(r, image);
    eta_1/eta_0 -> 0: R -> +1 and the image enters with +."""
    med = Medium([0.5], [2.0, 3.0], [1.0, ratio])
    G = LayeredGreen(med)
    x, y = 0.3, 0.2
    xs, ys = np.array([-0.4, 2.0]), np.array([0.9, -0.2])
    g = G.green(x, y, xs, ys, l=0, lp=0)
    ref = free_space(2.0, x, y, xs, ys) + sign * free_space(2.0, x, y, xs, -2 * 0.5 - ys)
    assert np.allclose(g, ref, rtol=1e-10, atol=1e-12)


def test_g_independent_of_y_shift():
    """Translating the whole stack vertically translates G (checks that the
    absolute interface positions enter only through tau and the phases)."""
    a = Medium([0.0, 2.0], [5.0, 7.0, 4.0])
    b = Medium([1.25, 3.25], [5.0, 7.0, 4.0])
    Ga, Gb = LayeredGreen(a), LayeredGreen(b)
    for l, y in ((0, 0.3), (1, -1.2), (2, -2.7)):
        for lp, ys in ((0, 0.8), (1, -0.4), (2, -3.5)):
            ga = Ga.green(0.7, y, [-0.5], [ys], l=l, lp=lp)[0]
            gb = Gb.green(0.7, y - 1.25, [-0.5], [ys - 1.25], l=l, lp=lp)[0]
            assert abs(ga - gb) <= 1e-12 * abs(ga)
