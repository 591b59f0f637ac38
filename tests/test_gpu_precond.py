"""Parity of the preconditioner (Sec. 4.2) with the oracle's dense
construction, through the C-ABI.

A three-layer eta != 1 medium with scatterers crossing both interfaces and
several leaf boxes per layer, for the leaf-box subdomains (precond = 1), one
level up (precond = 2) and the automatic level (precond = -1):

* the subdomains the library builds (lm_precond_subdomains: level, leaf
  level, each box's own elements and its neighbourhood) equal the oracle's,
  derived by the oracle from its own reading of the tree, as integer sets;
* lm_precond_apply in FP64 equals the oracle's sum of local solves entry by
  entry; the bar is 100 cond(P_B) eps, the backward-error bound of two LU
  solves of the same blocks in FP64 (the two factorisations pivot the same
  way only up to rounding);
* the served form (binary16 rows with power-of-two row scales, input split
  into two binary16 parts, FP32 accumulation) within 2e-3 of the oracle per
  entry: binary16 keeps 11 bits of each row entry (relative 2^-12) and the
  errors of a row's q entries add up in root-sum-square.
"""

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import precond as opre
from oracle.medium import Medium
from oracle.nystrom import Elements
from paper_2511_12450_amd import lmfmm
from paper_2511_12450_amd import workloads as wl
from tests.parity import check

pytestmark = pytest.mark.gpu

LEAF = 16


def _case():
    d, k, eta = np.array([0.0, 1.3]), np.array([2.0, 3.5, 2.5]), np.array([1.0, 2.0, 1.5])
    rng = np.random.default_rng(11)

    def radius(rng_, kind):
        R = rng_.uniform(0.2, 0.45)
        return R, (1.2 * R if kind == "star" else R)

    placed = wl._place(rng, 20, ((-7.0, 7.0), (-3.2, 2.0)), radius, 0.1, d, straddle_frac=0.3, iface_clear=0.02,
                       kinds=("circle", "star"))
    polys = wl._shapes(rng, placed, 40)
    return wl.Workload("precond3", d, k, eta, polys, np.array([60.0]))


@pytest.fixture(scope="module")
def case():
    w = _case()
    med = Medium(w.d, w.k, w.eta)
    el = Elements(med, w.polygons)
    crossing = sum(len(set(el.layer[el.scatterer == s].tolist())) > 1 for s in range(len(w.polygons)))
    assert crossing >= 4 and len(set(el.layer.tolist())) == 3
    return w, med, el


@pytest.mark.parametrize("pc", [1, 2, -1])
def test_precond_subdomains_and_apply(case, pc):
    w, med, el = case
    print(f"case: precond3 N={el.n} precond={pc} leaf_size={LEAF}", flush=True)
    geo = lmfmm.Geometry.from_workload(w, method=lmfmm.LM_FMM, precond=pc, leaf_size=LEAF)
    lev, lf, subs = geo.precond_subdomains()
    olev, olf = opre.level_for(med, el, pc, leaf_size=LEAF)
    osubs = opre.subdomains(med, el, olev, olf)
    print(f"library level {lev} leaf {lf} subdomains {len(subs)}; oracle level {olev} leaf {olf} "
          f"subdomains {len(osubs)}", flush=True)
    assert (lev, lf) == (olev, olf)
    assert len(subs) == len(osubs)
    for (own, J), (oown, oJ) in zip(subs, osubs):
        assert sorted(own.tolist()) == sorted(oown.tolist())
        assert sorted(J.tolist()) == sorted(oJ.tolist())
        assert sorted(J[: len(own)].tolist()) == sorted(own.tolist())
    if pc == 1:
        assert len(subs) >= 8
    cond = max(np.linalg.cond(opre.local_matrix(med, el, J)) for _, J in osubs)
    x = wl.random_vector(el.n, seed=21, n_rhs=3)
    ref = opre.apply(med, el, olev, olf, x)
    xd = torch.from_numpy(x).cuda()
    y64 = geo.precond_apply(xd, precision=lmfmm.LM_FP64).cpu().numpy()
    bar = 100.0 * cond * np.finfo(float).eps
    print(f"max cond(P_B) {cond:.3e}, FP64 bar {bar:.2e}", flush=True)
    check(y64, ref, bar, f"precond FP64 pc={pc}")
    y16 = geo.precond_apply(xd, precision=lmfmm.LM_MIXED).cpu().numpy()
    check(y16, ref, 2e-3, f"precond binary16 pc={pc}", bar_norm=1e-3)
