"""The stored full-size oracle rows (tests/golden/fullsize_rows_*.txt) are
well formed and still what the oracle computes: one stored row of the
64,000-element three-layer workload is recomputed here from the oracle (about
15 s) and compared with the file; the five-layer file (a row takes 20-30
minutes there) is checked for shape and for its rows being the ones the
writer draws."""

import importlib.util
import os
import re

import numpy as np
import pytest

from oracle.medium import Medium
from oracle.nystrom import Elements, matrix_rows
from paper_2511_12450_amd import workloads as wl

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _writer():
    spec = importlib.util.spec_from_file_location("make_fullsize_rows", os.path.join(GOLDEN, "make_fullsize_rows.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def _load(name):
    path = os.path.join(GOLDEN, f"fullsize_rows_{name}.txt")
    with open(path) as f:
        head = f.read(1024)
    m = re.search(r"random_vector\(N, seed=(\d+), n_rhs=(\d+)\)", head)
    a = np.loadtxt(path)
    return int(m.group(1)), int(m.group(2)), a


@pytest.mark.parametrize("name", ["three_layer", "five_layer"])
def test_golden_rows_shape_and_draw(name):
    seed, nrhs, a = _load(name)
    gen, vseed, n_rhs, n_near, n_any, rseed, keep = _writer().CASES[name]
    assert (seed, nrhs) == (vseed, n_rhs)
    rows = np.unique(a[:, 0].astype(np.int64))
    assert a.shape == (rows.size * nrhs, 4)
    assert np.all(np.isfinite(a[:, 2:]))
    w = gen()
    med = Medium(w.d, w.k, w.eta)
    el = Elements(med, w.polygons)
    drawn = _writer().sample_rows(med, el, n_near, n_any, rseed)[:keep]
    assert np.array_equal(np.sort(drawn), rows)


@pytest.mark.slow
def test_three_layer_row_recomputed():
    seed, nrhs, a = _load("three_layer")
    w = wl.three_layer()
    med = Medium(w.d, w.k, w.eta)
    el = Elements(med, w.polygons)
    X = wl.random_vector(el.n, seed=seed, n_rhs=nrhs)
    row = int(a[0, 0])
    stored = a[a[:, 0] == row]
    y = matrix_rows(med, el, [row])[0] @ X[:4].T
    ref = stored[:4, 2] + 1j * stored[:4, 3]
    assert np.allclose(y, ref, rtol=1e-12, atol=0.0)


def test_mini_far_fields_file():
    """The stored far fields of the 64-angle mini workload: every angle and
    observation direction the writer produces, finite."""
    spec = importlib.util.spec_from_file_location("make_mini_far_fields", os.path.join(GOLDEN, "make_mini_far_fields.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    a = np.loadtxt(os.path.join(GOLDEN, "mini_far_fields.txt"))
    n_obs = mod.obs_angles().size
    assert a.shape == (64 * n_obs, 4)
    assert np.array_equal(a[:, 0].astype(int), np.repeat(np.arange(64), n_obs))
    assert np.array_equal(a[:, 1].astype(int), np.tile(np.arange(n_obs), 64))
    assert np.all(np.isfinite(a[:, 2:])) and np.abs(a[:, 2:]).max() > 0
