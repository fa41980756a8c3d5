"""Pins of the oracle's damped block Jacobi smoother (eq. bjac), of the
vertex-patch option on tetrahedra, and of the additive counterpart of MG_hp
(Remark 3.4), on triangles and tetrahedra.

The damping 1 / (number of colours) rests on one fact that is checked
directly: within one colour the patch projections P_s = E_s A_ss^-1 E_s^T A
sum to an A-orthogonal projection (the patches of a colour share no
unknown and no matrix coupling), so sum_s P_s <= n_colours and
I - damp sum_s P_s is a positive semidefinite contraction in the A-norm.
The additive preconditioner is a sum of two symmetric positive definite
operators; the paper reports that it degrades as eps -> 0 and k grows,
while the multiplicative one does not.
"""
import numpy as np
import pytest

import synth
from oracle import mg, mg3d, solver, solver3d


def _dense(op, n):
    """Matrix of the linear map b -> op(b)."""
    M = np.zeros((n, n))
    for i in range(n):
        e = np.zeros(n)
        e[i] = 1.0
        M[:, i] = op(e)
    return M


def _setup2(k, gamma, nr=1, **kw):
    c, t = synth.kuhn_square(2)
    return solver.Setup(c, t, nr, k, 1.0, 1.0, gamma, **kw)


def _setup3(k, gamma, **kw):
    c, t = synth.kuhn_cube(1)
    return solver3d.Setup3(c, t, 1, k, 1.0, 1.0, gamma, **kw)


def _projections(sm, A):
    out = []
    for pats in sm.colours:
        Q = np.zeros(A.shape)
        for d, rows, Ainv in pats:
            Q[d] += Ainv @ A[d]
        out.append(Q)
    return out


@pytest.mark.parametrize("dim,k,patch", [(2, 2, "vertex"), (2, 2, "edge"), (3, 1, "edge"), (3, 1, "vertex")])
def test_colour_projections_are_A_orthogonal_projections(dim, k, patch):
    S = _setup2(k, 1e2) if dim == 2 else _setup3(k, 1e2)
    A = S.Aeps.toarray()
    if dim == 2:
        sm = mg.PatchGS(S.Aeps, S.lv, k + 1, "jacobi", patch)
    else:
        sm = mg3d.EdgePatchGS(S.Aeps, S.lv, (k + 1) * (k + 2) // 2, "jacobi", patch)
    for Q in _projections(sm, A):
        assert np.abs(Q @ Q - Q).max() <= 1e-9 * max(1.0, np.abs(Q).max())
        # A-orthogonal: A Q symmetric
        AQ = A @ Q
        assert np.abs(AQ - AQ.T).max() <= 1e-9 * np.abs(AQ).max()


@pytest.mark.parametrize("dim,k", [(2, 1), (2, 3), (3, 1)])
def test_jacobi_step_is_a_symmetric_contraction(dim, k):
    S = _setup2(k, 1e4) if dim == 2 else _setup3(k, 1e4)
    A = S.Aeps.toarray()
    n = A.shape[0]
    sm = S.prec.relax
    sm.jacobi = True
    sm.damp = 1.0 / len(sm.colours)

    def step(b):
        x = np.zeros(n)
        sm.forward(x, b)
        return x

    R = _dense(step, n)
    assert np.abs(R - R.T).max() <= 1e-10 * np.abs(R).max()
    # eigenvalues of R A (similar to A^1/2 R A^1/2): in (0, 1]
    L = np.linalg.cholesky(A)
    ev = np.linalg.eigvalsh(L.T @ R @ L)
    assert ev.min() > 0.0
    assert ev.max() <= 1.0 + 1e-10
    # the backward sweep is the same operator
    x = np.zeros(n)
    b = synth.uniform_pm1(4, 0, (n,))
    sm.backward(x, b)
    assert np.abs(x - R @ b).max() <= 1e-12 * np.abs(x).max()


@pytest.mark.parametrize("smoother,additive", [("jacobi", False), ("gs", True), ("jacobi", True)])
def test_variants_are_symmetric_positive_definite(smoother, additive):
    S = _setup2(2, 1e2, smoother=smoother, additive=additive)
    n = S.Aeps.shape[0]
    B = _dense(S.prec, n)
    assert np.abs(B - B.T).max() <= 1e-10 * np.abs(B).max()
    assert np.linalg.eigvalsh(0.5 * (B + B.T)).min() > 0.0


def test_jacobi_mg_hp_converges_in_bounded_iterations():
    # damped Jacobi needs more sweeps' worth of iterations than Gauss-Seidel
    # but stays bounded over gamma on a fixed mesh, and within a small
    # factor of the Gauss-Seidel counts
    its = {}
    for sm in ("gs", "jacobi"):
        for gamma in (1.0, 1e2, 1e6):
            S = _setup2(2, gamma, nr=2, smoother=sm)
            b = synth.uniform_pm1(1, 0, (S.Aeps.shape[0],))
            x, n, _ = S.inner(b)
            assert np.linalg.norm(S.Aeps @ x - b) <= 1e-7 * np.linalg.norm(b)
            its[sm, gamma] = n
    for gamma in (1.0, 1e2, 1e6):
        assert its["jacobi", gamma] <= 3 * its["gs", gamma], its
    assert its["jacobi", 1e6] <= 1.3 * its["jacobi", 1e2] + 1, its


def test_additive_degrades_where_multiplicative_does_not():
    # Remark 3.4: the additive variant's counts grow as eps -> 0 and as k
    # grows; the multiplicative MG_hp stays flat over the same range
    its = {}
    for additive in (False, True):
        for k in (1, 3):
            for gamma in (1e2, 1e6):
                S = _setup2(k, gamma, nr=2, additive=additive)
                b = synth.uniform_pm1(1, 0, (S.Aeps.shape[0],))
                _, n, _ = S.inner(b)
                its[additive, k, gamma] = n
    for k in (1, 3):
        assert abs(its[False, k, 1e6] - its[False, k, 1e2]) <= 1, its
        assert its[True, k, 1e6] >= 1.15 * its[True, k, 1e2], its
    assert its[True, 3, 1e6] >= 1.5 * its[True, 1, 1e6], its
    assert its[False, 3, 1e6] <= its[False, 1, 1e6] + 3, its
    assert its[True, 3, 1e6] >= 4 * its[False, 3, 1e6], its


def test_additive_equals_multiplicative_at_k0():
    # at k = 0 both are MG_h on the finest level (Alg. 2, first case)
    Sm = _setup2(0, 1e2)
    Sa = _setup2(0, 1e2, additive=True)
    b = synth.uniform_pm1(2, 0, (Sm.Aeps.shape[0],))
    assert np.abs(Sm.prec(b) - Sa.prec(b)).max() <= 1e-14 * np.abs(Sm.prec(b)).max()


def test_vertex_patch_relaxation_on_tetrahedra():
    # vertex patches contain the edge patches of their edges' faces, so the
    # vertex-patch relaxation needs no more iterations than the edge-patch
    # one, and the preconditioner stays symmetric positive definite
    its = {}
    for pr in ("edge", "vertex"):
        S = _setup3(2, 1e3, patch_relax=pr, patch_smooth=pr)
        n = S.Aeps.shape[0]
        b = synth.uniform_pm1(1, 0, (n,))
        _, its[pr], _ = S.inner(b)
        if pr == "vertex":
            B = _dense(S.prec, n)
            assert np.abs(B - B.T).max() <= 1e-10 * np.abs(B).max()
            assert np.linalg.eigvalsh(0.5 * (B + B.T)).min() > 0.0
    assert its["vertex"] <= its["edge"], its


def test_facet_patches_of_triangles():
    # edge (facet) patches in two dimensions: every dof facet alone, facets
    # of one colour in no common cell; as a lowest-order smoother with
    # vertex-patch relaxation (the paper's step setting) MG_hp stays SPD
    from oracle import mesh
    c, t = synth.kuhn_square(4)
    lv = mesh.Level(c, t)
    pats, col = lv.facet_patches()
    assert sorted(p[0] for p in pats) == sorted(np.where(lv.dof)[0].tolist())
    for K in range(lv.n_cells):
        cs = [col[i] for i, p in enumerate(pats) if p[0] in lv.cell_facets[K]]
        assert len(cs) == len(set(cs))
    S = _setup2(2, 1e2, patch_relax="vertex", patch_smooth="edge")
    n = S.Aeps.shape[0]
    B = _dense(S.prec, n)
    assert np.abs(B - B.T).max() <= 1e-10 * np.abs(B).max()
    assert np.linalg.eigvalsh(0.5 * (B + B.T)).min() > 0.0
