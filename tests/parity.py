"""Element-wise parity checks shared by the GPU tests.

Every comparison is made per right-hand side r, both entry by entry,
|y_ri - ref_ri| <= bar * max_i |ref_ri|, and in the 2-norm,
||y_r - ref_r|| <= bar * ||ref_r||, so one bad entry (an element next to an
interface, say) is not diluted by the rest of the vector.
"""

import numpy as np


def check(y, ref, bar, label, bar_norm=None, idx=None):
    """Assert parity of y against ref (arrays of shape (R, n) or (n,)) and
    return (worst element-wise ratio, worst 2-norm ratio).  idx: optional
    labels of the n entries (element indices of sampled rows) for the
    message."""
    y = np.atleast_2d(np.asarray(y))
    ref = np.atleast_2d(np.asarray(ref))
    assert y.shape == ref.shape, (y.shape, ref.shape)
    bar_norm = bar if bar_norm is None else bar_norm
    worst_e, worst_n, where = 0.0, 0.0, None
    for r in range(ref.shape[0]):
        d = np.abs(y[r] - ref[r])
        sc = np.abs(ref[r]).max()
        e = float(d.max() / sc) if sc > 0 else float(d.max())
        nrm = float(np.linalg.norm(y[r] - ref[r]) / np.linalg.norm(ref[r]))
        if e >= worst_e:
            i = int(np.argmax(d))
            worst_e, where = e, (r, i if idx is None else int(idx[i]))
        worst_n = max(worst_n, nrm)
    print(f"{label}: worst element {worst_e:.3e} (rhs {where[0]}, entry {where[1]}), worst 2-norm {worst_n:.3e}",
          flush=True)
    assert np.all(np.isfinite(y)), label
    assert worst_e <= bar, f"{label}: element-wise {worst_e:.3e} > {bar:.1e} at rhs/entry {where}"
    assert worst_n <= bar_norm, f"{label}: 2-norm {worst_n:.3e} > {bar_norm:.1e}"
    return worst_e, worst_n
