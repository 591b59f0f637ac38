"""Incident plane wave, background field and boundary data.

Oracle (test infrastructure): see the package docstring.

Paper, Sec. 2: u^inc = exp(i(k_{0,x} x - k_{0,y} y)) in layer 0 and zero below
(eq. incidentwave); the background field u^b with amplitudes
A_0 = R~_{01} e^{2 i k_{0,y} d_0}, A_l = R~_{l,l+1} T~_{0l} e^{2 i k_{l,y} d_l},
B_l = T~_{0l}, B_L = T~_{0L} at lambda = k_{0,x}; and the data
g = -u^inc - u^b on Gamma_0, g = -u^b on the other Gamma_l
(eq. homogeneousscattering).

Reading: the incidence angle theta is measured from +x and the wave
propagates along (cos theta, -sin theta), so k_{0,x} = k_0 cos theta and
k_{0,y} = k_0 sin theta > 0 for 0 < theta < pi.
"""

import numpy as np


def background_amplitudes(med, theta):
    """(kx, ky[l], A[l], B[l]) of u^b for incidence angle theta."""
    kx = med.k[0] * np.cos(theta)
    C = med.coefficients(np.array([kx], dtype=complex))
    ky = np.array([C["ky"][l][0] for l in range(med.L + 1)])
    L = med.L
    A = np.zeros(L + 1, dtype=complex)
    B = np.zeros(L + 1, dtype=complex)
    A[0] = C["Rdn"][0][0] * np.exp(2j * ky[0] * med.d[0])
    for l in range(1, L + 1):
        T0l = med.gen_transmission(C, 0, l)[0]
        B[l] = T0l
        if l < L:
            A[l] = C["Rdn"][l][0] * T0l * np.exp(2j * ky[l] * med.d[l])
    return kx, ky, A, B


def incident(med, theta, x, y):
    x = np.asarray(x, dtype=float)
    y = np.asarray(y, dtype=float)
    kx = med.k[0] * np.cos(theta)
    k0y = med.k[0] * np.sin(theta)
    lay = med.layer_of(y)
    return np.where(lay == 0, np.exp(1j * (kx * x - k0y * y)), 0.0)


def background(med, theta, x, y, dy=False):
    x = np.asarray(x, dtype=float)
    y = np.asarray(y, dtype=float)
    kx, ky, A, B = background_amplitudes(med, theta)
    lay = med.layer_of(y)
    kyl = ky[lay]
    up = A[lay] * np.exp(1j * (kx * x + kyl * y))
    dn = B[lay] * np.exp(1j * (kx * x - kyl * y))
    u = up + dn
    if not dy:
        return u
    return u, 1j * kyl * (up - dn)


def boundary_data(med, theta, x, y):
    """g at collocation points (eq. homogeneousscattering)."""
    return -incident(med, theta, x, y) - background(med, theta, x, y)


def boundary_data_bc(med, theta, x, y, nx, ny, beta=None):
    """Data of the sound-hard (beta None) or impedance condition
    (d_n + i beta) u = 0 with u = u^inc + u^b + u^s: the right side
    -(d_n + i beta)(u^inc + u^b) at points with normals (nx, ny)."""
    x = np.asarray(x, dtype=float)
    y = np.asarray(y, dtype=float)
    kx = med.k[0] * np.cos(theta)
    k0y = med.k[0] * np.sin(theta)
    ui = incident(med, theta, x, y)
    ub, dub = background(med, theta, x, y, dy=True)
    u = ui + ub
    ux = 1j * kx * u
    uy = -1j * k0y * ui + dub
    g = -(np.asarray(nx) * ux + np.asarray(ny) * uy)
    if beta is not None:
        g = g - 1j * beta * u
    return g
