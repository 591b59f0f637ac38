"""Seeded synthetic inputs: layered media, scatterer node polygons, angles.

This module only generates inputs (medium parameters, closed CCW node
polygons, incidence angles, seeded random vectors).  It holds none of the
method's arithmetic: elements, layer assignment and everything after them are
computed separately by the library and by the test oracle.

The workloads are shaped like the paper's examples (Sec. 5: a few to
thousands of scatterers, some crossing interfaces, layer thickness 1-2,
5-petal "flower" curves r = a sin k(theta - theta0) + b, eq. scattererpara).
Node placement: n nodes at uniform parameter t_j = 2 pi j / n, counter-
clockwise; each node-to-next-node chord is one element.
"""

from dataclasses import dataclass, field

import numpy as np


@dataclass
class Workload:
    name: str
    d: np.ndarray          # interface depths, interfaces at y = -d[l]
    k: np.ndarray          # wavenumbers per layer (top first)
    eta: np.ndarray        # transmission weights per layer
    polygons: list         # list of (n_j, 2) float64 arrays, CCW
    angles_deg: np.ndarray # incidence angles (from +x, wave travels (cos t, -sin t))
    p: int = 20            # expansion order for the fast method
    tol: float = 1e-8      # GMRES relative tolerance
    extra: dict = field(default_factory=dict)

    @property
    def n_elements(self):
        return int(sum(P.shape[0] for P in self.polygons))

    def flat_nodes(self):
        """(offsets int64[M+1], nodes float64[sum n_j, 2]) as the C-ABI takes them."""
        counts = [P.shape[0] for P in self.polygons]
        off = np.zeros(len(counts) + 1, dtype=np.int64)
        off[1:] = np.cumsum(counts)
        nodes = np.ascontiguousarray(np.concatenate(self.polygons, axis=0), dtype=np.float64)
        return off, nodes


# -- curves -------------------------------------------------------------------

def circle(c, R, n):
    t = 2.0 * np.pi * np.arange(n) / n
    return np.stack([c[0] + R * np.cos(t), c[1] + R * np.sin(t)], axis=1)


def star(c, R, n, t0, petals=5, amp=0.2):
    t = 2.0 * np.pi * np.arange(n) / n
    r = R * (1.0 + amp * np.cos(petals * (t - t0)))
    return np.stack([c[0] + r * np.cos(t), c[1] + r * np.sin(t)], axis=1)


def ellipse(c, a, b, rot, n):
    t = 2.0 * np.pi * np.arange(n) / n
    x, y = a * np.cos(t), b * np.sin(t)
    cr, sr = np.cos(rot), np.sin(rot)
    return np.stack([c[0] + cr * x - sr * y, c[1] + sr * x + cr * y], axis=1)


def flower(c, a, b, k, theta0, n):
    """eq. scattererpara: r = a sin k(theta - theta0) + b."""
    t = 2.0 * np.pi * np.arange(n) / n
    r = a * np.sin(k * (t - theta0)) + b
    return np.stack([c[0] + r * np.cos(t), c[1] + r * np.sin(t)], axis=1)


# -- random placement -----------------------------------------------------------

def _place(rng, n_scat, box, radius_fn, gap, d, straddle_frac=0.0, iface_clear=0.0,
           kinds=("circle",), max_tries=2000000):
    """Random sequential placement of n_scat shapes with circumradius from
    radius_fn; non-overlapping circumcircles with clearance `gap`; a fraction
    straddles an interface, the rest keep every point `iface_clear` away
    from every interface."""
    (x0, x1), (y0, y1) = box
    n_str = int(round(straddle_frac * n_scat))
    placed_c = np.zeros((0, 2))
    placed_r = np.zeros(0)
    out = []
    tries = 0
    while len(out) < n_scat:
        tries += 1
        if tries > max_tries:
            raise RuntimeError("placement did not converge; enlarge the box")
        j = len(out)
        kind = kinds[j % len(kinds)]
        R, Rc = radius_fn(rng, kind)
        x = rng.uniform(x0, x1)
        if j < n_str:
            m = rng.integers(0, len(d))
            y = -d[m] + rng.uniform(-0.5, 0.5) * R
        else:
            y = rng.uniform(y0, y1)
            if len(d) and np.min(np.abs(y + np.asarray(d))) < Rc + iface_clear:
                continue
        if placed_r.size:
            dist = np.hypot(placed_c[:, 0] - x, placed_c[:, 1] - y)
            if np.any(dist < placed_r + Rc + gap):
                continue
        placed_c = np.vstack([placed_c, [x, y]])
        placed_r = np.append(placed_r, Rc)
        out.append((kind, (x, y), R))
    return out


def _shapes(rng, placed, n_nodes):
    polys = []
    for kind, c, R in placed:
        if kind == "circle":
            polys.append(circle(c, R, n_nodes))
        elif kind == "star":
            polys.append(star(c, R, n_nodes, rng.uniform(0, 2 * np.pi)))
        elif kind == "ellipse":
            polys.append(ellipse(c, R, R * rng.uniform(0.5, 0.9), rng.uniform(0, np.pi), n_nodes))
        else:
            raise ValueError(kind)
    return polys


# -- the workloads --------------------------------------------------------------

def plain_small(seed=1):
    """Two layers (interface y=0, k=2 above, 3 below), 4 circles with radius
    U[0.3,0.6], two centres in [-3,3]x[1,4] and two in [-3,3]x[-4,-1], 64
    nodes each (N=256), incidence 30 deg, GMRES tol 1e-8."""
    rng = np.random.default_rng(seed)
    d = np.array([0.0])
    cents, rads = [], []
    for box in (((-3, 3), (1, 4)), ((-3, 3), (1, 4)), ((-3, 3), (-4, -1)), ((-3, 3), (-4, -1))):
        while True:
            c = (rng.uniform(*box[0]), rng.uniform(*box[1]))
            R = rng.uniform(0.3, 0.6)
            if all(np.hypot(c[0] - q[0], c[1] - q[1]) >= R + r + 0.1 for q, r in zip(cents, rads)):
                break
        cents.append(c)
        rads.append(R)
    polys = [circle(c, R, 64) for c, R in zip(cents, rads)]
    return Workload("plain_small_N256", d, np.array([2.0, 3.0]), np.ones(2), polys,
                    np.array([30.0]), p=20, tol=1e-8)


def three_layer(seed=2, n_scat=400, n_nodes=160, box=((-10.0, 10.0), (-5.0, 3.0)), angles=(30.0,)):
    """Three layers (interfaces y=0, y=-2; k=(5,7,4)); alternating circles and
    5-petal stars r = R(1 + 0.2 cos 5(t - t0)) with R ~ U[0.1,0.25]; 10%
    straddle an interface (centre y = -d_j + U[-0.5,0.5] R); the others keep
    0.02 from every interface; circumcircle gap >= 0.05; 160 nodes each."""
    rng = np.random.default_rng(seed)
    d = np.array([0.0, 2.0])

    def radius(rng_, kind):
        R = rng_.uniform(0.1, 0.25)
        return R, (1.2 * R if kind == "star" else R)

    placed = _place(rng, n_scat, box, radius, 0.05, d, straddle_frac=0.1, iface_clear=0.02,
                    kinds=("circle", "star"))
    polys = _shapes(rng, placed, n_nodes)
    N = n_scat * n_nodes
    return Workload(f"three_layer_N{N}", d, np.array([5.0, 7.0, 4.0]), np.ones(3), polys,
                    np.asarray(angles, dtype=float), p=20, tol=1e-6)


def three_layer_mini(seed=3, n_scat=25, n_nodes=160, angles=None):
    """The three-layer generator at 25 scatterers (N=4000) in a box scaled
    to keep the scatterer density of the 400-scatterer case."""
    s = np.sqrt(n_scat / 400.0)
    box = ((-10.0 * s, 10.0 * s), (-1.0 - 4.0 * s, -1.0 + 4.0 * s))
    if angles is None:
        angles = np.linspace(10.0, 170.0, 64)
    return three_layer(seed, n_scat, n_nodes, box, angles)


def three_layer_smooth(n_nodes=64, seed=4, n_scat=100, box=((-5.0, 5.0), (-4.0, 2.0))):
    """The three-layer medium (interfaces y=0, y=-2; k=(5,7,4)) with smooth
    scatterers only, none touching an interface (every point 0.05 away):
    circles, ellipses (axis ratio U[0.5,0.9]) and 5-petal stars in equal
    thirds, R ~ U[0.1,0.25], gap >= 0.05, n_nodes nodes each at equal
    parameter steps; a unit point source at the centre of scatterer 0 gives
    a manufactured solution."""
    rng = np.random.default_rng(seed)
    d = np.array([0.0, 2.0])

    def radius(rng_, kind):
        R = rng_.uniform(0.1, 0.25)
        return R, (1.2 * R if kind == "star" else R)

    placed = _place(rng, n_scat, box, radius, 0.05, d, straddle_frac=0.0, iface_clear=0.05,
                    kinds=("circle", "ellipse", "star"))
    polys = _shapes(rng, placed, n_nodes)
    w = Workload(f"three_layer_smooth_N{n_scat * n_nodes}", d, np.array([5.0, 7.0, 4.0]), np.ones(3), polys,
                 np.array([30.0]), p=20, tol=1e-8, extra={"source": np.array([placed[0][1]], dtype=float)})
    return w


def multi_rhs(seed=3):
    """The 400-scatterer three-layer geometry with 64 incidence angles in
    [10, 170] deg solved as one block."""
    return three_layer(seed=2, angles=np.linspace(10.0, 170.0, 64))


def five_layer(seed=5, n_scat=4000, n_nodes=250, box=((-30.0, 30.0), (-12.0, 6.0)), n_angles=8):
    """Five layers (interfaces 0, -1.5, -3, -4.5; k=(8,12,6,10,9)); circles,
    ellipses and stars in equal thirds, R ~ U[0.08,0.16]; 15% straddle an
    interface; gap >= 0.03; 250 nodes each (N=1,000,000)."""
    rng = np.random.default_rng(seed)
    d = np.array([0.0, 1.5, 3.0, 4.5])

    def radius(rng_, kind):
        R = rng_.uniform(0.08, 0.16)
        return R, (1.2 * R if kind == "star" else R)

    placed = _place(rng, n_scat, box, radius, 0.03, d, straddle_frac=0.15, iface_clear=0.02,
                    kinds=("circle", "ellipse", "star"))
    polys = _shapes(rng, placed, n_nodes)
    N = n_scat * n_nodes
    return Workload(f"five_layer_N{N}", d, np.array([8.0, 12.0, 6.0, 10.0, 9.0]), np.ones(5), polys,
                    np.linspace(10.0, 170.0, n_angles), p=24, tol=1e-6)


def stream_geometry(g):
    """One geometry of the serving pool (seed 4+g): 2-4 layers, thickness
    U[1,3], k ~ U[1,10], N ~ U[4000, 250000] in scatterers of 160 nodes,
    R ~ U[0.1,0.2], 10% straddlers, box for ~0.3 area fraction (enlarged by
    25% steps, same draws, when the placement does not fit)."""

    def radius(rng_, kind):
        R = rng_.uniform(0.1, 0.2)
        return R, (1.2 * R if kind == "star" else R)

    for attempt in range(8):
        rng = np.random.default_rng(4 + g)
        n_layers = int(rng.integers(2, 5))
        th = rng.uniform(1.0, 3.0, size=n_layers - 2)
        d = np.concatenate([[0.0], np.cumsum(th)]) if n_layers > 2 else np.array([0.0])
        k = rng.uniform(1.0, 10.0, size=n_layers)
        N = int(rng.uniform(4000, 250000))
        n_scat = max(1, N // 160)
        area = n_scat * np.pi * (0.15 * 1.2) ** 2 / 0.3
        side = np.sqrt(area) * 1.25 ** attempt
        ymid = -0.5 * d[-1]
        box = ((-side, side), (ymid - side / 4, ymid + side / 4))
        try:
            placed = _place(rng, n_scat, box, radius, 0.03, d, straddle_frac=0.1, iface_clear=0.02,
                            kinds=("circle", "star"), max_tries=200000)
            break
        except RuntimeError:
            if attempt == 7:
                raise
    polys = _shapes(rng, placed, 160)
    return Workload(f"stream_g{g}_N{n_scat * 160}", d, k, np.ones(n_layers), polys,
                    np.array([90.0]), p=20, tol=1e-6)


def paper_example1(n_per_side_unit=40):
    """Example 1 geometry (Sec. 5): L-shape crossing 4 of 5 layers,
    eta={1..5}, k={3.2,2.5,5.1,8.6,6.9}, interfaces y=0,-1,-2,-3; the
    manufactured solution is G_{l0}(r, (0, 0.375))."""
    V = np.array([(0.75, 0.75), (-0.75, 0.75), (-0.75, -2.5), (2.25, -2.5), (2.25, -1.5), (0.75, -1.5)])
    pts = []
    for a, b in zip(V, np.roll(V, -1, axis=0)):
        m = max(1, int(round(np.hypot(*(b - a)) * n_per_side_unit)))
        t = np.arange(m) / m
        pts.append(a[None, :] + t[:, None] * (b - a)[None, :])
    P = np.concatenate(pts, axis=0)
    return Workload("paper_example1", np.array([0.0, 1.0, 2.0, 3.0]), np.array([3.2, 2.5, 5.1, 8.6, 6.9]),
                    np.array([1.0, 2.0, 3.0, 4.0, 5.0]), [P], np.array([90.0]), extra={"source": (0.0, 0.375)})


def paper_example2(n_elements=12000):
    """Example 2 geometry (Sec. 5): six layers, interfaces y = 0, -1, -2, -3,
    -4, eta = (1.1, 2.3, 3.4, 4.6, 5.0, 6.6), k = (1.2, 2.3, 4.5, 6.1, 7.7,
    10.0); two "peanuts" of eq. scattererpara (a = 0.5, b = 1, petal number 2,
    theta0 = pi/4) centred at (0, -1) and (2, -3), n_elements / 2 nodes each;
    incident wave e^{i(-3 sqrt(2)/5)(x + y)}: k_0 = 1.2 travelling along
    (-1, -1)/sqrt(2), i.e. theta = 135 deg."""
    m = n_elements // 2
    polys = [flower((0.0, -1.0), 0.5, 1.0, 2, np.pi / 4, m), flower((2.0, -3.0), 0.5, 1.0, 2, np.pi / 4, m)]
    return Workload("paper_example2", np.array([0.0, 1.0, 2.0, 3.0, 4.0]),
                    np.array([1.2, 2.3, 4.5, 6.1, 7.7, 10.0]), np.array([1.1, 2.3, 3.4, 4.6, 5.0, 6.6]), polys,
                    np.array([135.0]))


def paper_example3(n_elements=12000):
    """Example 3 geometry (Sec. 5): six layers, interfaces y = 0, -1, -2, -3,
    -4, eta = (1, 2, 3, 4, 5, 6), k = (2, 3, 6, 5, 8, 10); five 5-petal
    flowers of eq. scattererpara (a = 0.2, b = 0.7, theta0 = 0) centred at
    (-1.5, 0), (1.5, 0), (0, -2), (-1.5, -4) and, as printed, (1.5, 4),
    n_elements / 5 nodes each; incident wave e^{-2iy}: theta = 90 deg."""
    m = n_elements // 5
    cs = [(-1.5, 0.0), (1.5, 0.0), (0.0, -2.0), (-1.5, -4.0), (1.5, 4.0)]
    polys = [flower(c, 0.2, 0.7, 5, 0.0, m) for c in cs]
    return Workload("paper_example3", np.array([0.0, 1.0, 2.0, 3.0, 4.0]), np.array([2.0, 3.0, 6.0, 5.0, 8.0, 10.0]),
                    np.array([1.0, 2.0, 3.0, 4.0, 5.0, 6.0]), polys, np.array([90.0]))


def random_vector(n, seed, n_rhs=1):
    """Seeded complex Gaussian vectors, shape (n_rhs, n)."""
    rng = np.random.default_rng(seed)
    return (rng.standard_normal((n_rhs, n)) + 1j * rng.standard_normal((n_rhs, n))) / np.sqrt(2.0)
