"""Pins of the oracle's spectrally accurate Nystrom rule (oracle/kress.py):

* the logarithmic weights integrate ln(4 sin^2((t - s)/2)) against cos(m s)
  and sin(m s) exactly: the integrals are -2 pi cos(m t)/m and
  -2 pi sin(m t)/m for m >= 1 and 0 for m = 0 (Fourier series of
  ln(4 sin^2(u/2)) = -2 sum cos(m u)/m);
* the spectral derivative of an ellipse's samples equals the analytic one;
* a sound-soft disk in a homogeneous medium: the scattered field against the
  Bessel series u^s = -sum i^n J_n(ka)/H_n(ka) H_n(kr) e^{in(phi - alpha)},
  with errors falling faster than any power of N (and far below the
  first-order rule's at the same N);
* a three-layer eta != 1 medium with a scatterer in each layer: Dirichlet
  data from a point source inside one scatterer make the layered Green's
  function of that source the exact exterior solution, so the scattered
  field and far field of the computed density must reproduce the source's
  (pins the reaction part and the trapezoidal sums across scatterers and
  layers as well as the logarithmic split).
"""

import numpy as np
import pytest
from scipy.special import hankel1, jv

from oracle.farfield import far_field, scattered_field
from oracle.green import LayeredGreen
from oracle.incident import boundary_data
from oracle.kress import Nodes, log_weights, matrix, spectral_derivative
from oracle.medium import Medium
from oracle.nystrom import Elements
from oracle.nystrom import matrix as midpoint_matrix
from oracle.solve import lu_solve
from paper_2511_12450_amd import workloads as wl

MED3 = Medium([0.0, 1.3], [2.0, 3.5, 2.5], [1.0, 2.0, 1.5])


@pytest.mark.parametrize("M", [6, 16, 40])
def test_log_weights_integrate_trigonometric_polynomials(M):
    n = M // 2
    R = log_weights(M)
    t = 2.0 * np.pi * np.arange(M) / M
    k = (np.arange(M)[:, None] - np.arange(M)[None, :]) % M
    W = R[k]  # W[i, j] = R_j(t_i)
    assert np.allclose(W @ np.ones(M), 0.0, atol=1e-12)
    for m in range(1, n):
        assert np.allclose(W @ np.cos(m * t), -2.0 * np.pi * np.cos(m * t) / m, atol=1e-12)
        assert np.allclose(W @ np.sin(m * t), -2.0 * np.pi * np.sin(m * t) / m, atol=1e-12)


def test_spectral_derivative_of_ellipse():
    M = 48
    t = 2.0 * np.pi * np.arange(M) / M
    P = wl.ellipse((0.3, -0.2), 0.7, 0.4, 0.5, M)
    a, b, rot = 0.7, 0.4, 0.5
    dx = -a * np.sin(t) * np.cos(rot) - b * np.cos(t) * np.sin(rot)
    dy = -a * np.sin(t) * np.sin(rot) + b * np.cos(t) * np.cos(rot)
    assert np.abs(spectral_derivative(P[:, 0]) - dx).max() < 1e-13
    assert np.abs(spectral_derivative(P[:, 1]) - dy).max() < 1e-13


def test_rejects_odd_counts_and_interface_crossing():
    with pytest.raises(ValueError):
        Nodes(MED3, [wl.circle((0.0, 0.6), 0.3, 15)])
    with pytest.raises(ValueError):
        Nodes(MED3, [wl.circle((0.0, -1.2), 0.3, 16)])


def _disk_case(M):
    k, a, cy, th = 2.0, 1.0, 2.0, np.radians(30.0)
    med = Medium([0.0], [k, k])
    P = [wl.circle((0.0, cy), a, M)]
    phi = np.linspace(0, 2 * np.pi, 12, endpoint=False)
    xr, yr = 2.5 * np.cos(phi), cy + 2.5 * np.sin(phi)
    n = np.arange(-50, 51)
    c = -(1j ** n) * jv(n, k * a) / hankel1(n, k * a)
    exact = np.sum(c[:, None] * hankel1(n[:, None], k * 2.5) * np.exp(1j * n[:, None] * (phi[None, :] + th)), axis=0)
    exact *= np.exp(-1j * k * np.sin(th) * cy)
    return med, P, th, xr, yr, exact


def test_disk_spectral_convergence_vs_bessel_series():
    errs = []
    for M in (16, 24, 32, 48):
        med, P, th, xr, yr, exact = _disk_case(M)
        nd = Nodes(med, P)
        ph = lu_solve(matrix(med, nd), boundary_data(med, th, nd.cx, nd.cy))
        us = scattered_field(med, nd, ph, xr, yr)
        errs.append(np.abs(us - exact).max() / np.abs(exact).max())
    print("disk, spectral rule", errs)
    assert errs[-1] < 1e-12
    assert errs[2] < 1e-9
    assert errs[1] < errs[0] / 30 and errs[2] < errs[1] / 30
    # the first-order rule at the largest N
    med, P, th, xr, yr, exact = _disk_case(48)
    el = Elements(med, P)
    ph = lu_solve(midpoint_matrix(med, el), boundary_data(med, th, el.cx, el.cy))
    e1 = np.abs(scattered_field(med, el, ph, xr, yr) - exact).max() / np.abs(exact).max()
    assert e1 > 1e-4 and errs[-1] < 1e-7 * e1


class _Point:
    """A unit point source seen as one quadrature node (for far_field)."""

    def __init__(self, med, x, y):
        self.cx, self.cy, self.w = np.array([x]), np.array([y]), np.array([1.0])
        self.layer = med.layer_of(self.cy)
        self.n = 1


def _three_layer_polys(M):
    # one scatterer in each layer (interfaces at y = 0 and y = -1.3)
    return [wl.ellipse((0.3, -0.65), 0.35, 0.2, 0.4, M), wl.circle((1.5, 1.0), 0.3, M),
            wl.star((-1.2, -2.1), 0.3, M, 0.3)]


@pytest.mark.parametrize("src", [(0.3, -0.65), (-1.2, -2.1)])
def test_layered_point_source_reproduced(src):
    G = LayeredGreen(MED3)
    ls = int(MED3.layer_of(np.array([src[1]]))[0])
    rec = np.array([[2.5, 0.4], [-2.0, 1.9], [0.0, -2.3], [1.2, -0.6], [-0.8, 0.9]])
    errs = []
    for M in (24, 48, 64):
        nd = Nodes(MED3, _three_layer_polys(M))
        f = np.array([G.green(nd.cx[i], nd.cy[i], [src[0]], [src[1]], lp=ls)[0] for i in range(nd.n)])
        ph = lu_solve(matrix(MED3, nd, G), f)
        us = scattered_field(MED3, nd, ph, rec[:, 0], rec[:, 1], G)
        ref = np.array([G.green(x, y, [src[0]], [src[1]], lp=ls)[0] for x, y in rec])
        obs = np.radians([20.0, 75.0, 140.0, 200.0, 290.0])
        ff = far_field(MED3, nd, ph, obs)
        ffr = far_field(MED3, _Point(MED3, *src), np.array([1.0]), obs)
        errs.append(max(np.abs(us - ref).max() / np.abs(ref).max(), np.abs(ff - ffr).max() / np.abs(ffr).max()))
    print("layered point source", src, errs)
    assert errs[-1] < 1e-9 and errs[0] > errs[1] > errs[2]
