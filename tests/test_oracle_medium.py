"""Pins of the oracle's spectral coefficients against independent mathematics.

Each check solves the interface conditions of the paper's model (Sec. 2.1:
[u] = 0, [eta du/dn] = 0) directly as a linear system, or uses a classical
closed form, so a dropped term, a wrong sign or a wrong index in the
recursions of Sec. 3.1 fails here.
"""

import numpy as np
import pytest

from oracle.incident import background, background_amplitudes, boundary_data, incident
from oracle.medium import Medium, nonzero_components

MEDIA = [
    Medium([0.0], [2.0, 3.0]),
    Medium([0.0], [2.0, 3.0], [1.0, 4.0]),
    Medium([0.0, 2.0], [5.0, 7.0, 4.0]),
    Medium([0.0, 1.3], [2.0, 3.5, 2.5], [1.0, 2.0, 1.5]),
    Medium([0.3, 1.0, 2.2], [3.2, 2.5, 5.1, 8.6], [1.0, 2.0, 3.0, 4.0]),
]
LAMS = [0.3, 1.7, 2.9, 4.5, 9.0, 2.0 - 0.3j, 6.0 - 0.2j]


def _stack_solve_from_above(med, lam):
    """Amplitudes of a downgoing wave e^{i(lam x - k_0y y)} hitting the stack,
    from the interface conditions solved as one linear system.  Unknowns:
    reflected up-amplitude in layer 0, (up, down) in layers 1..L-1, down in
    layer L; amplitudes multiply e^{+-i k_{l,y} y} (global reference)."""
    L = med.L
    ky = med.ky(np.array([lam]))[:, 0]
    eta = med.eta
    # unknown order: r0, (a1, b1), ..., (a_{L-1}, b_{L-1}), tL
    n = 2 * L
    M = np.zeros((n, n), dtype=complex)
    rhs = np.zeros(n, dtype=complex)

    def col_up(l):
        return 0 if l == 0 else 2 * l - 1

    def col_dn(l):
        return n - 1 if l == L else 2 * l

    for m in range(L):
        y = -med.d[m]
        # layer m above, layer m+1 below
        for side, l, sgn in ((0, m, 1.0), (1, m + 1, -1.0)):
            eu, ed = np.exp(1j * ky[l] * y), np.exp(-1j * ky[l] * y)
            # up component (absent in layer L), down component (layer 0: the incident wave)
            if l < L:
                M[2 * m, col_up(l)] += sgn * eu
                M[2 * m + 1, col_up(l)] += sgn * eta[l] * 1j * ky[l] * eu
            if l == 0:
                rhs[2 * m] -= sgn * ed
                rhs[2 * m + 1] -= sgn * eta[l] * (-1j * ky[l]) * ed
            else:
                M[2 * m, col_dn(l)] += sgn * ed
                M[2 * m + 1, col_dn(l)] += sgn * eta[l] * (-1j * ky[l]) * ed
    sol = np.linalg.solve(M, rhs)
    up = np.zeros(L + 1, dtype=complex)
    dn = np.zeros(L + 1, dtype=complex)
    up[0] = sol[0]
    dn[0] = 1.0
    for l in range(1, L):
        up[l], dn[l] = sol[col_up(l)], sol[col_dn(l)]
    dn[L] = sol[n - 1]
    return up, dn


@pytest.mark.parametrize("mi", range(len(MEDIA)))
@pytest.mark.parametrize("lam", LAMS)
def test_downward_coefficients_match_interface_solve(mi, lam):
    """R~_{l,l+1}, T~_{0l} and the background amplitudes of Sec. 2.2 equal the
    amplitudes obtained by solving all interface conditions at once."""
    med = MEDIA[mi]
    up, dn = _stack_solve_from_above(med, lam)
    C = med.coefficients(np.array([lam], dtype=complex))
    ky = med.ky(np.array([lam]))[:, 0]
    assert np.allclose(C["Rdn"][0][0] * np.exp(2j * ky[0] * med.d[0]), up[0], rtol=1e-11, atol=1e-13)
    for l in range(1, med.L + 1):
        T0l = med.gen_transmission(C, 0, l)[0]
        assert np.allclose(T0l, dn[l], rtol=1e-11, atol=1e-13)
        if l < med.L:
            A = C["Rdn"][l][0] * T0l * np.exp(2j * ky[l] * med.d[l])
            assert np.allclose(A, up[l], rtol=1e-11, atol=1e-13)


@pytest.mark.parametrize("mi", range(len(MEDIA)))
@pytest.mark.parametrize("lam", LAMS)
def test_upward_coefficients_match_mirrored_stack(mi, lam):
    """R~_{l+1,l} and T~_{L l} (upward recursion) equal the downward
    quantities of the mirror-image stack (y -> -y, layer order reversed)."""
    med = MEDIA[mi]
    L = med.L
    dm = -med.d[::-1]
    mir = Medium(dm - dm[0], med.k[::-1], med.eta[::-1])
    shift = dm[0]  # mirror coordinate y' = -y + shift puts its first interface at 0
    C = med.coefficients(np.array([lam], dtype=complex))
    Cm = mir.coefficients(np.array([lam], dtype=complex))
    for l in range(L + 1):
        # R~_{l,l-1} of the stack == R~_{L-l, L-l+1} of the mirror (local quantity)
        assert np.allclose(C["Rup"][l][0], Cm["Rdn"][L - l][0], rtol=1e-11, atol=1e-13)
    # transmission magnitudes from layer L to each layer (phases depend on the reference)
    kyv = med.ky(np.array([lam]))[:, 0]
    for l in range(L):
        T = med.gen_transmission(C, L, l)[0]
        Tm = mir.gen_transmission(Cm, 0, L - l)[0]
        # an up-wave e^{i k_L y} is a down-wave of the mirror (y' = -y + shift) with amplitude e^{i k_L shift}
        ph = np.exp(-1j * (kyv[l] - kyv[L]) * shift)
        assert np.allclose(T, Tm * ph, rtol=1e-10, atol=1e-13)


def test_single_interface_fresnel_closed_form():
    med = Medium([0.0], [2.0, 3.0], [1.0, 2.5])
    lam = np.array([0.5, 1.5, 2.5, 4.0])
    kk = med.ky(lam)
    C = med.coefficients(lam)
    a, b = kk[0], 2.5 * kk[1]
    assert np.allclose(C["Rdn"][0], (a - b) / (a + b), rtol=1e-14)
    assert np.allclose(med.gen_transmission(C, 0, 1), 2 * a / (a + b), rtol=1e-14)


def test_single_slab_airy_formula():
    """Three layers: R~_{01} = (R01 + R12 e^{2ik1h})/(1 + R01 R12 e^{2ik1h})."""
    med = Medium([0.0, 0.8], [2.0, 3.0, 1.5])
    lam = np.array([0.4, 1.2, 1.9, 2.6])
    kk = med.ky(lam)
    r01 = (kk[0] - kk[1]) / (kk[0] + kk[1])
    r12 = (kk[1] - kk[2]) / (kk[1] + kk[2])
    e = np.exp(2j * kk[1] * 0.8)
    C = med.coefficients(lam)
    assert np.allclose(C["Rdn"][0], (r01 + r12 * e) / (1 + r01 * r12 * e), rtol=1e-13)


@pytest.mark.parametrize("mi", range(len(MEDIA)))
def test_flux_conservation(mi):
    """Lossless stack: eta_0 k_0y (1 - |R~_01|^2) = eta_L Re(k_Ly) |T~_0L|^2."""
    med = MEDIA[mi]
    L = med.L
    lam = np.linspace(0.01, 0.999 * med.k[0], 40)
    C = med.coefficients(lam.astype(complex))
    kk = med.ky(lam)
    T = med.gen_transmission(C, 0, L)
    lhs = med.eta[0] * kk[0].real * (1 - np.abs(C["Rdn"][0]) ** 2)
    rhs = med.eta[L] * kk[L].real * np.abs(T) ** 2
    assert np.allclose(lhs, rhs, rtol=1e-12, atol=1e-14)


@pytest.mark.parametrize("L", [1, 2, 3, 4, 5])
def test_component_count_and_zeros(L):
    """Remark of Sec. 3.1: 4L^2 non-zero components; the others vanish."""
    rng = np.random.default_rng(L)
    med = Medium(np.cumsum(rng.uniform(0.5, 1.5, L)) - 0.5, rng.uniform(1, 5, L + 1))
    count = sum(len(nonzero_components(l, lp, L)) for l in range(L + 1) for lp in range(L + 1))
    assert count == 4 * L * L
    lam = np.array([0.7, 3.0 - 0.2j, 8.0])
    for l in range(L + 1):
        for lp in range(L + 1):
            sig = med.densities(lam, l, lp)
            nz = nonzero_components(l, lp, L)
            for c in ("ud", "uu", "dd", "du"):
                if c not in nz:
                    assert np.all(sig[c] == 0), (l, lp, c)


@pytest.mark.parametrize("mi", range(len(MEDIA)))
@pytest.mark.parametrize("theta_deg", [20.0, 60.0, 90.0, 135.0])
def test_background_field_transmission_conditions(mi, theta_deg):
    """u^inc + u^b and eta d/dy(u^inc + u^b) are continuous (eq. TLhelmholtztotallayer2)."""
    med = MEDIA[mi]
    th = np.radians(theta_deg)
    kx = med.k[0] * np.cos(th)
    k0y = med.k[0] * np.sin(th)
    kx_, ky, A, B = background_amplitudes(med, th)
    x = 0.37
    for m in range(med.L):
        y = -med.d[m]
        vals = []
        for l in (m, m + 1):
            ub = A[l] * np.exp(1j * (kx * x + ky[l] * y)) + B[l] * np.exp(1j * (kx * x - ky[l] * y))
            dub = 1j * ky[l] * (A[l] * np.exp(1j * (kx * x + ky[l] * y)) - B[l] * np.exp(1j * (kx * x - ky[l] * y)))
            if l == 0:
                ub += np.exp(1j * (kx * x - k0y * y))
                dub += -1j * k0y * np.exp(1j * (kx * x - k0y * y))
            vals.append((ub, med.eta[l] * dub))
        assert abs(vals[0][0] - vals[1][0]) < 1e-12 * max(1, abs(vals[0][0]))
        assert abs(vals[0][1] - vals[1][1]) < 1e-11 * max(1, abs(vals[0][1]))
    # the helpers agree with the amplitudes away from interfaces
    y0 = 0.5 - med.d[0]
    assert np.allclose(background(med, th, [x], [y0])[0], A[0] * np.exp(1j * (kx * x + ky[0] * y0)))
    assert np.allclose(incident(med, th, [x], [y0])[0], np.exp(1j * (kx * x - k0y * y0)))


def _d_dy(f, y, h, sgn):
    """One-sided fourth-order derivative of f at y from samples y + sgn j h,
    j = 0..4 (all on one side of an interface)."""
    c = np.array([-25.0, 48.0, -36.0, 16.0, -3.0]) / 12.0
    return sum(c[j] * f(y + sgn * j * h) for j in range(5)) / (sgn * h)


@pytest.mark.parametrize("mi", range(len(MEDIA)))
@pytest.mark.parametrize("theta_deg", [20.0, 75.0, 90.0, 135.0])
def test_field_helpers_in_every_layer(mi, theta_deg):
    """incident(), background() and boundary_data() themselves, in every layer
    (Sec. 2.2, eqs. incidentwave, TLhelmholtztotallayer2, homogeneousscattering):

    * at interior points of every layer, u^inc + u^b equals the field of the
      amplitudes obtained by solving all interface conditions at once
      (independent of the recursions), and u^inc vanishes below layer 0;
    * just above and just below every interface (+-1e-9), u^inc + u^b and
      eta d/dy(u^inc + u^b) agree, the derivatives taken by one-sided finite
      differences of the helpers' values inside each layer;
    * background(dy=True) equals the finite-difference derivative of
      background() inside each layer;
    * boundary_data = -(u^inc + u^b)."""
    med = MEDIA[mi]
    th = np.radians(theta_deg)
    kx = med.k[0] * np.cos(th)
    up, dn = _stack_solve_from_above(med, kx)
    ky = med.ky(np.array([kx], dtype=complex))[:, 0]
    xs = np.array([-1.3, 0.37, 2.9])

    def total(x, y):
        return incident(med, th, x, y) + background(med, th, x, y)

    # interior points of every layer (the outer layers sampled 0.2 and 1.1 away)
    tops = [None] + [-med.d[l] for l in range(med.L)]
    bots = [-med.d[l] for l in range(med.L)] + [None]
    for l in range(med.L + 1):
        if tops[l] is None:
            ys = [bots[l] + 0.2, bots[l] + 1.1]
        elif bots[l] is None:
            ys = [tops[l] - 0.2, tops[l] - 1.1]
        else:
            h = tops[l] - bots[l]
            ys = [bots[l] + 0.25 * h, bots[l] + 0.7 * h]
        for y in ys:
            yy = np.full(xs.shape, y)
            assert np.all(med.layer_of(yy) == l)
            ref = up[l] * np.exp(1j * (kx * xs + ky[l] * y)) + dn[l] * np.exp(1j * (kx * xs - ky[l] * y))
            got = total(xs, yy)
            assert np.allclose(got, ref, rtol=1e-11, atol=1e-12), (l, y)
            inc = incident(med, th, xs, yy)
            if l == 0:
                assert np.allclose(inc, np.exp(1j * (kx * xs - med.k[0] * np.sin(th) * y)), rtol=1e-14)
            else:
                assert np.all(inc == 0), (l, y)
            assert np.allclose(boundary_data(med, th, xs, yy), -got, rtol=1e-14, atol=0)
            hh = 1e-3
            for sgn in (1.0, -1.0):
                fd = _d_dy(lambda t: background(med, th, xs, np.full(xs.shape, t)), y, hh, sgn)
                _, dub = background(med, th, xs, yy, dy=True)
                assert np.allclose(dub, fd, rtol=1e-7, atol=1e-8 * med.k.max()), (l, y)

    # across every interface, from the helpers' values on each side
    eps, hh = 1e-9, 1e-3
    for m in range(med.L):
        yi = -med.d[m]
        ya, yb = yi + eps, yi - eps
        assert np.all(med.layer_of(np.full(xs.shape, ya)) == m)
        assert np.all(med.layer_of(np.full(xs.shape, yb)) == m + 1)
        ua, ub_ = total(xs, np.full(xs.shape, ya)), total(xs, np.full(xs.shape, yb))
        assert np.allclose(ua, ub_, rtol=1e-7, atol=1e-8), m
        da = _d_dy(lambda t: total(xs, np.full(xs.shape, t)), ya, hh, 1.0)
        db = _d_dy(lambda t: total(xs, np.full(xs.shape, t)), yb, hh, -1.0)
        scale = med.k.max() * max(1.0, np.abs(ua).max())
        assert np.allclose(med.eta[m] * da, med.eta[m + 1] * db, rtol=0, atol=1e-6 * scale * med.eta.max()), m
        if m == 0:
            assert np.all(incident(med, th, xs, np.full(xs.shape, yb)) == 0)
