"""Layered medium: interfaces, Fresnel and generalized coefficients, densities.

Oracle (test infrastructure): see the package docstring.

Paper: Sec. 2.1 (layer strips), Sec. 3.1 (Fresnel coefficients, the two
generalized-reflection recursions Rellrecursionup / Rellrecursiondown, the
generalized transmission generaltransmission, and the reaction densities of
Cases I-III: densityinsourcelayer, disity1, disity2).

Readings:
* the round-trip factor printed as exp(-2 k_{l,y} h_l) is read as
  exp(+2i k_{l,y} h_l), the form the paper prints inside Cases II and III;
* the downward recursion starts from R~_{L,L+1} = 0 (the Remark after
  eq. planewavekernel) and runs l = L-1 .. 0;
* k_{l,y} = sqrt(k_l^2 - lambda^2) on the branch Im >= 0 (outgoing/decaying);
* the top and bottom layers have no thickness; it is only ever multiplied by
  R~_{0,-1} = R~_{L,L+1} = 0.
"""

import numpy as np

UP, DN = "u", "d"
COMPONENTS = ("ud", "uu", "dd", "du")  # (arrival direction at target, departure at source)


def nonzero_components(l, lp, L):
    """Reaction components (l, l', *star) that do not vanish identically.

    Remark after eq. planewavekernel: sigma^{dd}_{0l'} = sigma^{du}_{0l'} = 0,
    sigma^{uu}_{Ll'} = sigma^{ud}_{Ll'} = 0, sigma^{uu}_{l0} = sigma^{du}_{l0} = 0
    and sigma^{ud}_{lL} = sigma^{dd}_{lL} = 0, leaving 4 L^2 components.
    """
    out = []
    for c in COMPONENTS:
        at_t, at_s = c[0], c[1]
        if l == 0 and at_t == DN:
            continue
        if l == L and at_t == UP:
            continue
        if lp == 0 and at_s == UP:
            continue
        if lp == L and at_s == DN:
            continue
        out.append(c)
    return out


class Medium:
    """L+1 layers l = 0..L, interfaces y = -d_l (l = 0..L-1), wavenumbers k_l,
    and the coefficients eta_l that weight the normal derivative in the
    transmission condition [eta du/dn] = 0 (Sec. 2.1)."""

    def __init__(self, d, k, eta=None):
        d = np.atleast_1d(np.asarray(d, dtype=float))
        k = np.atleast_1d(np.asarray(k, dtype=float))
        L = d.size
        if k.size != L + 1:
            raise ValueError("need len(k) == len(d) + 1")
        if L > 1 and not np.all(np.diff(d) > 0):
            raise ValueError("interfaces must satisfy d_0 < d_1 < ...")
        if np.any(k <= 0):
            raise ValueError("wavenumbers must be positive")
        eta = np.ones(L + 1) if eta is None else np.asarray(eta, dtype=float)
        if eta.size != L + 1 or np.any(eta <= 0):
            raise ValueError("eta must have L+1 positive entries")
        self.L, self.d, self.k, self.eta = L, d, k, eta

    # -- geometry -------------------------------------------------------------
    def layer_of(self, y):
        """Layer index of points y (Sec. 2.1: -d_l < y < -d_{l-1}).  A point
        within 1e-12 of an interface is given to the upper layer (reading)."""
        y = np.asarray(y, dtype=float)
        lay = np.zeros(y.shape, dtype=int)
        for l in range(self.L):
            lay += (y < -self.d[l] - 1e-12).astype(int)
        return lay

    def thickness(self, l):
        if 1 <= l <= self.L - 1:
            return self.d[l] - self.d[l - 1]
        return 0.0

    def tau(self, m, a):
        """Reflection of a coordinate about the interface y = -d_m
        (eq. reflections): tau_m(a) = -2 d_m - a."""
        return -2.0 * self.d[m] - a

    # -- spectral quantities --------------------------------------------------
    def ky(self, lam):
        """k_{l,y}(lambda) for all layers, shape (L+1,) + lam.shape, Im >= 0."""
        lam = np.asarray(lam, dtype=complex)
        kk = self.k.reshape((-1,) + (1,) * lam.ndim)
        v = np.sqrt(kk * kk - lam * lam)
        return np.where(v.imag < 0, -v, v)

    def coefficients(self, lam):
        """All spectral coefficients at lam.  Returns a dict with
        ky[l], R[l] = R_{l,l+1}, Tdn[l] = T_{l,l+1}, Tup[l] = T_{l+1,l},
        Rup[l] = R~_{l,l-1} (l=0..L), Rdn[l] = R~_{l,l+1} (l=0..L),
        ph[l] = exp(2 i k_{l,y} h_l)."""
        lam = np.asarray(lam, dtype=complex)
        L, eta, d = self.L, self.eta, self.d
        ky = self.ky(lam)
        R, Tdn, Tup = [], [], []
        for l in range(L):
            a = eta[l] * ky[l]
            b = eta[l + 1] * ky[l + 1]
            R.append((a - b) / (a + b))
            Tdn.append(2.0 * a / (a + b))
            # T_{l+1,l} = (eta_{l+1} k_{l+1,y} / eta_l k_{l,y}) T_{l,l+1}
            Tup.append(2.0 * b / (a + b))
        ph = [np.exp(2j * ky[l] * self.thickness(l)) for l in range(L + 1)]
        zero = np.zeros(lam.shape, dtype=complex)
        # upward recursion: R~_{0,-1} = 0; R~_{l+1,l} from R~_{l,l-1}
        Rup = [zero]
        for l in range(L):
            Rloc = -R[l]  # R_{l+1,l} = -R_{l,l+1}
            t = Rup[l] * ph[l]
            Rup.append((Rloc + t) / (1.0 + Rloc * t))
        # downward recursion: R~_{L,L+1} = 0; R~_{l,l+1} from R~_{l+1,l+2}
        Rdn = [zero] * (L + 1)
        for l in range(L - 1, -1, -1):
            t = Rdn[l + 1] * ph[l + 1]
            Rdn[l] = (R[l] + t) / (1.0 + R[l] * t)
        return dict(ky=ky, R=R, Tdn=Tdn, Tup=Tup, Rup=Rup, Rdn=Rdn, ph=ph, d=d)

    def gen_transmission(self, C, lp, l):
        """T~_{l'l}: generalized transmission from layer l' to layer l
        (eq. generaltransmission), T~_{l'l'} = 1."""
        ky, R, Tdn, Tup, Rup, Rdn, ph, d = (C[s] for s in ("ky", "R", "Tdn", "Tup", "Rup", "Rdn", "ph", "d"))
        val = np.ones_like(ky[0])
        if l < lp:
            for m in range(lp - 1, l - 1, -1):
                num = Tup[m] * np.exp(1j * (ky[m] - ky[m + 1]) * d[m])
                den = 1.0 + (-R[m]) * Rup[m] * ph[m]
                val = num * val / den
        elif l > lp:
            for m in range(lp + 1, l + 1):
                num = Tdn[m - 1] * np.exp(1j * (ky[m - 1] - ky[m]) * d[m - 1])
                den = 1.0 + R[m - 1] * Rdn[m] * ph[m]
                val = num * val / den
        return val

    def densities(self, lam, l, lp, C=None):
        """sigma^{*star}_{l l'}(lam) for the four components, Cases I-III."""
        if C is None:
            C = self.coefficients(lam)
        Rup, Rdn, ph = C["Rup"], C["Rdn"], C["ph"]
        # source-layer (Case I) densities of layer l'
        D = 1.0 - Rdn[lp] * Rup[lp] * ph[lp]
        s_ud = Rdn[lp] / D
        s_du = Rup[lp] / D
        s_uu = Rup[lp] * s_ud
        s_dd = s_uu
        if l == lp:
            return {"ud": s_ud, "du": s_du, "uu": s_uu, "dd": s_dd}
        T = self.gen_transmission(C, lp, l)
        if l < lp:  # Case II
            ud = T * s_ud
            uu = T * (1.0 + s_uu * ph[lp])
            return {"ud": ud, "uu": uu, "dd": Rup[l] * ud, "du": Rup[l] * uu}
        # Case III
        du = T * s_du
        dd = T * (1.0 + s_dd * ph[lp])
        return {"du": du, "dd": dd, "uu": Rdn[l] * du, "ud": Rdn[l] * dd}

    # -- exponent of each reaction component ----------------------------------
    def theta_coeffs(self, comp, l, lp, y, yp):
        """Coefficients (A, B) with Theta = k_{l,y} A + k_{l',y} B, the phase of
        component comp in eq. fourreactions (target y in layer l, source y' in
        layer l').  The large-|lambda| decay distance is D = A + B >= 0."""
        tau = self.tau
        if comp == "ud":
            if l <= lp:
                return y, -tau(lp, yp)
            return -tau(l, y), yp
        if comp == "uu":
            if l < lp:
                return y, -yp
            return -tau(l, y), tau(lp - 1, yp)
        if comp == "dd":
            if l <= lp:
                return tau(l - 1, y), -tau(lp, yp)
            return -y, yp
        if comp == "du":
            if l < lp:
                return tau(l - 1, y), -yp
            return -y, tau(lp - 1, yp)
        raise ValueError(comp)
