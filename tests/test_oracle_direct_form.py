"""The block Gauss-Seidel step of Alg. 2 in its direct form.

The GPU colour phases compute the step as x_s = A_ss^-1 (b_s - A_{s,r} x_r),
r the unknowns outside the patch, and read only the coupling of each patch
cell's patch facets (faces) to its far facets (faces).  These checks pin
that reading on the oracle's own operators and patches, on the CPU:

* one sweep in the direct form equals the oracle's sweep in the correction
  form x_s += A_ss^-1 (b - A x)_s to rounding (triangles, vertex patches;
  tetrahedra, edge patches), from a non-zero iterate;
* on triangles the columns outside a vertex patch that its rows couple to
  are exactly unknowns of the far facets of the patch cells (the facet of
  each cell opposite the patch vertex).
"""
import numpy as np
import pytest

import synth
from oracle import mg, mg3d, solver, solver3d


def _direct_sweep(sm, x, b):
    """One forward sweep, x_s = A_ss^-1 (b_s - A_{s,r} x_r) patch by patch in
    the smoother's colour and patch order."""
    n = len(x)
    for pats in sm.colours:
        for d, rows, Ainv in pats:
            out = np.ones(n, dtype=bool)
            out[d] = False
            x[d] = Ainv @ (b[d] - rows[:, np.where(out)[0]] @ x[out])


@pytest.mark.parametrize("dim,k,gamma", [(2, 1, 1e2), (2, 2, 1e4), (3, 1, 1e2)])
def test_direct_form_sweep_equals_correction_form(dim, k, gamma):
    if dim == 2:
        S = solver.Setup(*synth.kuhn_square(2)[:2], 1, k, 1.0, 1.0, gamma)
        sm = mg.PatchGS(S.Aeps, S.lv, k + 1)
    else:
        S = solver3d.Setup3(*synth.kuhn_cube(1)[:2], 1, k, 1.0, 1.0, gamma)
        sm = mg3d.EdgePatchGS(S.Aeps, S.lv, (k + 1) * (k + 2) // 2)
    n = S.Aeps.shape[0]
    b = synth.uniform_pm1(31, 0, (n,))
    x0 = synth.uniform_pm1(31, 1, (n,))
    x_corr = x0.copy()
    sm.forward(x_corr, b)
    x_dir = x0.copy()
    _direct_sweep(sm, x_dir, b)
    scale = np.abs(x_corr).max()
    assert scale > 0.0
    # the two forms differ by rounding only, amplified by the patch
    # condition numbers (the AL term at gamma = 1e4 makes them large)
    assert np.abs(x_dir - x_corr).max() <= 1e-9 * scale
    # and both changed the iterate (the sweep is not the identity)
    assert np.abs(x_corr - x0).max() > 1e-3 * scale


def test_patch_rows_couple_outside_only_through_far_facets():
    k = 2
    S = solver.Setup(*synth.kuhn_square(2)[:2], 1, k, 1.0, 1.0, 1e2)
    lv, m = S.lv, k + 1
    A = S.Aeps.tocsr()
    vf = lv.vertex_facets()
    checked = 0
    for v in range(len(vf)):
        fs = vf[v]
        if not fs:
            continue
        d = {(lv.int_id[f] * 2 + cc) * m + j for f in fs for cc in range(2) for j in range(m)}
        # far facets: in each cell around v the facet opposite v
        far = set()
        for K in np.where((lv.cells == v).any(axis=1))[0]:
            i = int(np.where(lv.cells[K] == v)[0][0])
            f = lv.cell_facets[K, i]
            if lv.int_id[f] >= 0:
                far |= {(lv.int_id[f] * 2 + cc) * m + j for cc in range(2) for j in range(m)}
        rows = A[sorted(d)]
        outside = set(rows.indices[np.abs(rows.data) > 0.0]) - d
        assert outside <= far, (v, sorted(outside - far)[:6])
        checked += 1
    assert checked == int((np.asarray([len(f) for f in vf]) > 0).sum()) and checked > 0
