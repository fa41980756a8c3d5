"""Convergence orders of the GPU solves (Sec. 5.1) and the flexible-CG
breakdown status, through the C ABI.

Generalized Stokes at k = 3 (the k = 1, 2 rates are covered with the
post-processing parity tests): ||u - u_h|| and ||p - p_h|| at order k+1,
||u - u*|| at order k+2.  Stationary Navier-Stokes (Sec. 5.1.2) through
hdgmg_picard_newton (Alg. 3 in the library): the same orders for u_h and
u*.  Breakdown: with m_relax = 0, MG_hp is the lowest-order correction
alone, which annihilates a residual without mode-0 components (z.r = 0); the
oracle's flexible CG raises and the library returns HDGMG_EBREAKDOWN.
"""
import numpy as np
import pytest

import synth
from oracle import krylov, solver, solver3d
from tests import manufactured as mf

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _note(msg):
    print(msg, flush=True)


def dev(a):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def _l2(W, e):
    return float(np.sqrt(np.sum(W[..., None] * e ** 2) if e.ndim == 3 else np.sum(W * e ** 2)))


def test_stokes_eoc_k3():
    import paper_2303_06762_amd as hd
    k = 3
    errs = []
    for nr in (0, 1, 2):
        c, t = synth.kuhn_square(2)
        _note(f"stokes eoc k=3 n_refine={nr}")
        s = hd.Solver(c, t, nr, k, 1.0, 1.0, 1e3, uzawa_tol=1e-13, uzawa_max=64, rtol=1e-12, atol=0.0)
        s.assemble()
        X = host(s.data_points())
        f = mf.source(X, 1.0, 1.0)
        u, p, state, info, st = s.solve(dev(f))
        assert st in (0, 1)
        us = host(s.postprocess(dev(f), state))
        W = host(s.data_weights())
        errs.append((_l2(W, host(u) - mf.velocity(X)), _l2(W, host(p) - mf.pressure(X)),
                     _l2(W, us - mf.velocity(X))))
        assert info["div_l2"] <= 1e-9
        s.close()
    rates = [np.log2(errs[1][i] / errs[2][i]) for i in range(3)]
    _note(f"  errors {errs} rates {rates}")
    assert rates[0] > k + 1 - 0.3 and rates[1] > k + 1 - 0.3, rates
    assert rates[2] > k + 2 - 0.4, rates


@pytest.mark.parametrize("k", [1, 2, 3])
def test_navier_stokes_eoc(k):
    import paper_2303_06762_amd as hd
    nu = 0.05
    nrs = (1, 2, 3) if k < 3 else (0, 1, 2)
    errs = []
    for nr in nrs:
        c, t = synth.kuhn_square(2)
        _note(f"navier-stokes eoc k={k} n_refine={nr}")
        s = hd.Solver(c, t, nr, k, 0.0, nu, 1e3, oseen=1, uzawa_tol=1e-13, uzawa_max=64, rtol=1e-12,
                      atol=0.0)
        X = host(s.data_points())
        f = mf.ns_source(X, nu)
        out = hd.picard_newton(s, dev(f), eps_picard=1e-3, newton_rtol=1e-12, newton_atol=1e-14, max_newton=8)
        assert out[-1]["kind"] == "newton"
        assert all(o["status"] in (0, 1) for o in out)
        last = out[-1]
        W = host(s.data_weights())
        # u* of the converged state: its local fields are those of the Picard
        # system with the converged velocity as the wind (the discrete
        # solution is a fixed point of the Picard map)
        s.set_newton(None)
        s.set_wind(last["u"])
        s.assemble()
        us = host(s.postprocess(dev(f), last["state"]))
        errs.append((_l2(W, host(last["u"]) - mf.velocity(X)), _l2(W, us - mf.velocity(X))))
        assert last["info"]["div_l2"] <= 1e-9
        s.close()
    rates = [np.log2(errs[1][i] / errs[2][i]) for i in range(2)]
    _note(f"  errors {errs} rates {rates}")
    assert rates[0] > k + 1 - 0.3, rates
    assert rates[1] > k + 2 - 0.4, rates


@pytest.mark.parametrize("dim", [2, 3])
def test_breakdown_status(dim):
    import paper_2303_06762_amd as hd
    k = 2
    if dim == 2:
        c, t = synth.kuhn_square(2)
        O = solver.Setup(c, t, 1, k, 1.0, 1.0, 1e2, m_p=0)
        s = hd.Solver(c, t, 1, k, 1.0, 1.0, 1e2, m_relax=0)
        m = k + 1
    else:
        c, t = synth.kuhn_cube(1)
        O = solver3d.Setup3(c, t, 1, k, 1.0, 1.0, 1e2, m_p=0)
        s = hd.Solver(c, t, 1, k, 1.0, 1.0, 1e2, m_relax=0, m_smooth=2)
        m = (k + 1) * (k + 2) // 2
    s.assemble()
    b = synth.uniform_pm1(3, 0, (s.n_skel,))
    b[::m] = 0.0  # no mode-0 component: MG_hp(b) = 0
    with pytest.raises(krylov.Breakdown):
        O.inner(b)
    with pytest.raises(hd.HdgmgError) as e:
        s.inner_solve(dev(b))
    assert e.value.status == -6
    # a residual with a mode-0 component does not break down at the start
    b2 = synth.uniform_pm1(4, 0, (s.n_skel,))
    z = host(s.precondition(dev(b2)))
    assert float(z @ b2) > 0.0
    s.close()
