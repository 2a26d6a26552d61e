"""Differentiation through the regularised Gauss-Newton step (Eq. 3) with
respect to the data, the sampling weights, the regularisation weight and the
references (the linearisation point held fixed): the GPU step and its
gradients (GaussNewtonStep, backward = nlinv_gn_step_vjp) against central
differences of the FP64 oracle's step solved to convergence.  The step is
linear in y and x_ref (their differences are exact); alpha and P enter
nonlinearly (differences with a small step).  One case keeps every
sensitivity component on the grid (n = 32), one keeps a band (n = 64: 32 of
64 per axis, the rest following N = alpha I)."""
import numpy as np
import pytest

from oracle import nlinv_oracle as O
from paper_1301_1215_amd import Plan
from tests.gpu_util import dev, host, rand_c, rel, soft_mask

pytestmark = pytest.mark.gpu

CG_GPU = 80       # CG iterations of the GPU step and of its backward
CG_ORACLE = 400   # the oracle's step, converged


def _oracle_step(y, P, alpha, rr, cr, rn, cn, d):
    res = O.irgnm(y, P, d, O.IRGNMParams(1, CG_ORACLE, alpha0=alpha, alpha_q=1.0, scale_norm=0.0),
                  rho0=rn, chat0=cn, rho_ref=rr, chat_ref=cr)
    return res.rho, res.chat


def _loss(h_r, h_c, r, c):
    return float(np.real(np.vdot(h_r, r) + np.vdot(h_c, c)))


@pytest.mark.parametrize("n,n_om,J", [(32, 32, 3), (64, 32, 2)])
def test_gradients_match_oracle_differences(n, n_om, J):
    import torch
    from paper_1301_1215_amd.autograd import gauss_newton_step
    rng = np.random.default_rng([61, n, J])
    d = O.Dims(n, n_om, J)
    y = rand_c((J, n, n), rng)
    P = soft_mask(n, rng)
    alpha = 0.5
    rn = (1.0 + 0.1 * rand_c((n_om, n_om), rng)).astype(np.complex64)
    cn = (0.05 * rand_c((J, n, n), rng)).astype(np.complex64)
    rr, cr = rand_c((n_om, n_om), rng, 0.5), rand_c((J, n, n), rng, 0.05)
    h_r, h_c = rand_c((n_om, n_om), rng), rand_c((J, n, n), rng)
    # directions for the differences
    v_y = rand_c((J, n, n), rng)
    q_P = rng.standard_normal((n, n)).astype(np.float32)
    v_r, v_c = rand_c((n_om, n_om), rng), rand_c((J, n, n), rng, 0.05)

    with Plan(n, n_om, J) as pl:
        ty = dev(y).requires_grad_()
        tP = dev(P).requires_grad_()
        ta = torch.tensor(alpha, dtype=torch.float64, device="cuda", requires_grad=True)
        tr, tc = dev(rr).requires_grad_(), dev(cr).requires_grad_()
        r1, c1 = gauss_newton_step(ty, tP, ta, tr, tc, dev(rn), dev(cn), pl, CG_GPU)
        L = (torch.conj(dev(h_r)) * r1).real.sum() + (torch.conj(dev(h_c)) * c1).real.sum()
        L.backward()
        g = {"y": host(ty.grad), "P": host(tP.grad), "alpha": float(ta.grad), "r": host(tr.grad),
             "c": host(tc.grad)}
        r1, c1 = host(r1), host(c1)

    ref_r, ref_c = _oracle_step(y, P, alpha, rr, cr, rn, cn, d)
    assert rel(r1, ref_r) < 1e-4 and rel(c1, ref_c) < 1e-4

    def L_of(y_=y, P_=P, a_=alpha, r_=rr, c_=cr):
        return _loss(h_r, h_c, *_oracle_step(y_, P_, a_, r_, c_, rn, cn, d))
    # linear in y and in x_ref: a unit difference is exact
    dy = (L_of(y_=y + v_y) - L_of(y_=y - v_y)) / 2
    assert abs(np.real(np.vdot(g["y"], v_y)) - dy) <= 2e-3 * abs(dy)
    dref = (L_of(r_=rr + v_r, c_=cr + v_c) - L_of(r_=rr - v_r, c_=cr - v_c)) / 2
    assert abs(np.real(np.vdot(g["r"], v_r) + np.vdot(g["c"], v_c)) - dref) <= 2e-3 * abs(dref)
    ea = 1e-4
    da = (L_of(a_=alpha + ea) - L_of(a_=alpha - ea)) / (2 * ea)
    assert abs(g["alpha"] - da) <= 2e-3 * abs(da)
    eP = 1e-4
    dP = (L_of(P_=P + eP * q_P) - L_of(P_=P - eP * q_P)) / (2 * eP)
    assert abs(float(np.sum(g["P"] * q_P)) - dP) <= 2e-3 * abs(dP)


def test_linearisation_point_must_not_require_grad():
    import torch
    from paper_1301_1215_amd.autograd import gauss_newton_step
    n, J = 16, 1
    z = torch.zeros((n, n), dtype=torch.complex64, device="cuda")
    zc = torch.zeros((J, n, n), dtype=torch.complex64, device="cuda")
    P = torch.ones((n, n), dtype=torch.float32, device="cuda")
    with Plan(n, n, J) as pl:
        with pytest.raises(ValueError):
            gauss_newton_step(zc, P, 1.0, z, zc, z.clone().requires_grad_(), zc, pl, 4)
