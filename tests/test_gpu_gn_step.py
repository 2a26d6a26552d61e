"""Differentiation through the regularised Gauss-Newton step (Eq. 3) with
respect to the data, the sampling weights, the regularisation weight, the
references and the linearisation point, and through a chain of such steps
(the Newton loop): the GPU step and its gradients (GaussNewtonStep, backward
= nlinv_gn_step_vjp) against central differences of the FP64 oracle's steps
solved to convergence.  The step is linear in y and x_ref (their differences
are exact); alpha, P and x_n enter nonlinearly (differences with a small
step).  One case keeps every sensitivity component on the grid (n = 32), one
keeps a band (n = 64: 32 of 64 per axis, the rest following N = alpha I)."""
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
    w_r, w_c = rand_c((n_om, n_om), rng, 0.1), rand_c((J, n, n), rng, 0.05)

    with Plan(n, n_om, J) as pl:
        ty = dev(y).requires_grad_()
        tP = dev(P).requires_grad_()
        ta = torch.tensor(alpha, dtype=torch.float64, device="cuda", requires_grad=True)
        tr, tc = dev(rr).requires_grad_(), dev(cr).requires_grad_()
        tn, tcn = dev(rn).requires_grad_(), dev(cn).requires_grad_()
        r1, c1 = gauss_newton_step(ty, tP, ta, tr, tc, tn, tcn, pl, CG_GPU)
        L = (torch.conj(dev(h_r)) * r1).real.sum() + (torch.conj(dev(h_c)) * c1).real.sum()
        L.backward()
        g = {"y": host(ty.grad), "P": host(tP.grad), "alpha": float(ta.grad), "r": host(tr.grad),
             "c": host(tc.grad), "rn": host(tn.grad), "cn": host(tcn.grad)}
        r1, c1 = host(r1), host(c1)

    ref_r, ref_c = _oracle_step(y, P, alpha, rr, cr, rn, cn, d)
    assert rel(r1, ref_r) < 1e-4 and rel(c1, ref_c) < 1e-4

    def L_of(y_=y, P_=P, a_=alpha, r_=rr, c_=cr, rn_=rn, cn_=cn):
        return _loss(h_r, h_c, *_oracle_step(y_, P_, a_, r_, c_, rn_, cn_, d))
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
    # the linearisation point: the step is nonlinear in x_n
    ex = 1e-3
    dx_n = (L_of(rn_=rn + ex * w_r, cn_=cn + ex * w_c) - L_of(rn_=rn - ex * w_r, cn_=cn - ex * w_c)) / (2 * ex)
    gx = float(np.real(np.vdot(g["rn"], w_r) + np.vdot(g["cn"], w_c)))
    assert abs(gx - dx_n) <= 2e-3 * abs(dx_n), (gx, dx_n)


NEWTON = 3


def _oracle_loop(y, P, a0, q, r0, c0, d):
    res = O.irgnm(y, P, d, O.IRGNMParams(NEWTON, CG_ORACLE, alpha0=a0, alpha_q=q, scale_norm=0.0),
                  rho0=r0, chat0=c0)
    return res.rho, res.chat


@pytest.mark.parametrize("n,n_om,J", [(32, 32, 3), (64, 32, 2)])
def test_unrolled_newton_loop_gradients(n, n_om, J):
    """Three Newton steps (alpha 1, 0.5, 0.25, x_ref = x0): the chained step
    derivatives against differences of the oracle's loop, with respect to
    y, P, alpha0 and the start x0 (which is also the reference)."""
    import torch
    from paper_1301_1215_amd.autograd import irgnm_unrolled
    rng = np.random.default_rng([67, n, J])
    d = O.Dims(n, n_om, J)
    y = rand_c((J, n, n), rng)
    P = soft_mask(n, rng)
    a0, q = 1.0, 0.5
    r0 = (1.0 + 0.1 * rand_c((n_om, n_om), rng)).astype(np.complex64)
    c0 = (0.05 * rand_c((J, n, n), rng)).astype(np.complex64)
    h_r, h_c = rand_c((n_om, n_om), rng), rand_c((J, n, n), rng)
    v_y = rand_c((J, n, n), rng)
    q_P = rng.standard_normal((n, n)).astype(np.float32)
    w_r, w_c = rand_c((n_om, n_om), rng, 0.1), rand_c((J, n, n), rng, 0.05)

    with Plan(n, n_om, J) as pl:
        ty, tP = dev(y).requires_grad_(), dev(P).requires_grad_()
        ta = torch.tensor(a0, dtype=torch.float64, device="cuda", requires_grad=True)
        tr, tc = dev(r0).requires_grad_(), dev(c0).requires_grad_()
        rN, cN = irgnm_unrolled(ty, tP, tr, tc, pl, NEWTON, CG_GPU, alpha0=ta, alpha_q=q)
        L = (torch.conj(dev(h_r)) * rN).real.sum() + (torch.conj(dev(h_c)) * cN).real.sum()
        L.backward()
        g = {"y": host(ty.grad), "P": host(tP.grad), "alpha": float(ta.grad), "r": host(tr.grad),
             "c": host(tc.grad)}
        rN, cN = host(rN), host(cN)

    ref_r, ref_c = _oracle_loop(y, P, a0, q, r0, c0, d)
    assert rel(rN, ref_r) < 2e-4 and rel(cN, ref_c) < 2e-4

    def L_of(y_=y, P_=P, a_=a0, r_=r0, c_=c0):
        return _loss(h_r, h_c, *_oracle_loop(y_, P_, a_, q, r_, c_, d))
    tol = 3e-3
    e = 1e-3
    dy = (L_of(y_=y + e * v_y) - L_of(y_=y - e * v_y)) / (2 * e)
    assert abs(np.real(np.vdot(g["y"], v_y)) - dy) <= tol * abs(dy), (np.real(np.vdot(g["y"], v_y)), dy)
    dP = (L_of(P_=P + 1e-4 * q_P) - L_of(P_=P - 1e-4 * q_P)) / 2e-4
    assert abs(float(np.sum(g["P"] * q_P)) - dP) <= tol * abs(dP), (float(np.sum(g["P"] * q_P)), dP)
    da = (L_of(a_=a0 + 1e-4) - L_of(a_=a0 - 1e-4)) / 2e-4
    assert abs(g["alpha"] - da) <= tol * abs(da), (g["alpha"], da)
    dx = (L_of(r_=r0 + e * w_r, c_=c0 + e * w_c) - L_of(r_=r0 - e * w_r, c_=c0 - e * w_c)) / (2 * e)
    gx = float(np.real(np.vdot(g["r"], w_r) + np.vdot(g["c"], w_c)))
    assert abs(gx - dx) <= tol * abs(dx), (gx, dx)
