"""Pins of the oracle's sound-hard and impedance scatterers (the Neumann and
Robin conditions of Sec. 2.1):

* the gradient of the layered Green's function in the target equals central
  differences of the oracle's own G (pinned elsewhere by the interface
  conditions), for sources in the target's layer and in the layers above and
  below, in a three-layer eta != 1 medium;
* the boundary data -(d_n + i beta)(u^inc + u^b) equals the normal
  derivative of the Dirichlet data taken by differences, in every layer;
* sound-hard and impedance disks in a homogeneous medium: the Bessel series
  u^s = sum c_n H_n(kr) e^{in(phi - alpha)},
  c_n = -i^n (k J_n'(ka) + i beta J_n(ka)) / (k H_n'(ka) + i beta H_n(ka)),
  reached at first order by the Nystrom solution.
"""

import numpy as np
import pytest
from scipy.special import h1vp, hankel1, jv, jvp

from oracle.farfield import scattered_field
from oracle.green import LayeredGreen
from oracle.incident import boundary_data, boundary_data_bc
from oracle.medium import Medium
from oracle.nystrom import Elements, matrix_bc
from oracle.solve import lu_solve
from paper_2511_12450_amd import workloads as wl

MED3 = Medium([0.0, 1.3], [2.0, 3.5, 2.5], [1.0, 2.0, 1.5])


@pytest.mark.parametrize("lp,src", [(1, ([-1.2, 0.9, 2.5], [-0.8, -1.0, -0.2])), (0, ([0.5, -1.0], [0.3, 1.2])),
                                    (2, ([0.5, -1.0], [-1.6, -2.4]))])
def test_green_gradient_equals_differences(lp, src):
    G = LayeredGreen(MED3)
    x, y = 0.37, -0.4  # layer 1
    xs, ys = np.array(src[0]), np.array(src[1])
    g, gx, gy = G.green_grad(x, y, xs, ys, 1, lp)
    h = 1e-5
    fx = (G.green(x + h, y, xs, ys, l=1, lp=lp) - G.green(x - h, y, xs, ys, l=1, lp=lp)) / (2 * h)
    fy = (G.green(x, y + h, xs, ys, l=1, lp=lp) - G.green(x, y - h, xs, ys, l=1, lp=lp)) / (2 * h)
    assert np.allclose(g, G.green(x, y, xs, ys, l=1, lp=lp), rtol=1e-13)
    assert np.abs(gx - fx).max() < 1e-7 * np.abs(gx).max()
    assert np.abs(gy - fy).max() < 1e-7 * np.abs(gy).max()


@pytest.mark.parametrize("theta_deg", [30.0, 110.0])
def test_boundary_data_equals_normal_difference(theta_deg):
    th = np.radians(theta_deg)
    pts = np.array([[0.3, 0.7], [-1.0, -0.5], [2.0, -2.2], [0.1, -1.25]])  # layers 0, 1, 2, 1
    nrm = np.array([[0.6, 0.8], [-1.0, 0.0], [0.0, -1.0], [0.28, -0.96]])
    h = 1e-6
    for beta in (None, 1.7):
        g = boundary_data_bc(MED3, th, pts[:, 0], pts[:, 1], nrm[:, 0], nrm[:, 1], beta)
        up = boundary_data(MED3, th, pts[:, 0] + h * nrm[:, 0], pts[:, 1] + h * nrm[:, 1])
        um = boundary_data(MED3, th, pts[:, 0] - h * nrm[:, 0], pts[:, 1] - h * nrm[:, 1])
        ref = (up - um) / (2 * h)  # d_n of -(u^inc + u^b)
        if beta is not None:
            ref = ref + 1j * beta * boundary_data(MED3, th, pts[:, 0], pts[:, 1])
        assert np.allclose(g, ref, rtol=1e-7, atol=1e-8)


def _disk_bc_exact(k, a, beta, alpha, r, phi, nmax=60):
    n = np.arange(-nmax, nmax + 1)
    b = 0.0 if beta is None else beta
    c = -(1j ** n) * (k * jvp(n, k * a) + 1j * b * jv(n, k * a)) / (k * h1vp(n, k * a) + 1j * b * hankel1(n, k * a))
    return np.sum(c[:, None] * hankel1(n[:, None], k * r[None, :]) * np.exp(1j * n[:, None] * (phi[None, :] - alpha)), axis=0)


@pytest.mark.parametrize("beta", [None, 1.5])
def test_disk_neumann_robin_bessel_series(beta):
    """Homogeneous two-layer medium (equal k, eta) with a disk above y = 0."""
    k, a, cy = 2.0, 1.0, 2.0
    med = Medium([0.0], [k, k])
    theta = np.radians(30.0)
    alpha = -theta  # propagation direction (cos t, -sin t)
    phi = np.linspace(0, 2 * np.pi, 16, endpoint=False)
    rr = np.full(phi.size, 2.5)
    xr, yr = rr * np.cos(phi), cy + rr * np.sin(phi)
    exact = _disk_bc_exact(k, a, beta, alpha, rr, phi) * np.exp(-1j * k * np.sin(theta) * cy)
    errs = []
    G = LayeredGreen(med)
    for n in (64, 128, 256):
        el = Elements(med, [wl.circle((0.0, cy), a, n)])
        A = matrix_bc(med, el, beta, G)
        g = boundary_data_bc(med, theta, el.cx, el.cy, el.nx, el.ny, beta)
        ph = lu_solve(A, g)
        us = scattered_field(med, el, ph, xr, yr, G)
        errs.append(np.max(np.abs(us - exact)) / np.max(np.abs(exact)))
    print("disk", beta, errs)
    assert errs[-1] < 1e-2
    r1, r2 = errs[0] / errs[1], errs[1] / errs[2]
    assert 1.6 < r1 < 4.5 and 1.6 < r2 < 4.5, errs
