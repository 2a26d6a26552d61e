"""Differentiation through F: torch.autograd.Function whose backward is the
DF^H kernel (and the mask-gradient kernel), checked against exact central
differences of F (F is bilinear, so they carry no truncation error), the
oracle adjoint, and the oracle mask gradient."""
import numpy as np
import pytest

from oracle import nlinv_oracle as O
from paper_1301_1215_amd import Plan, synth
from tests.gpu_util import dev, host, rel, rand_c

pytestmark = pytest.mark.gpu


def _setup(n, J, seed):
    fr, logits = synth.soft_mask_frame(n, J)
    rng = np.random.default_rng([3, n, seed])
    rho = rand_c((n, n), rng)
    chat = rand_c((J, n, n), rng)
    return fr, logits, rho, chat, rng


def test_torch_gradcheck_32x32_4_coils():
    import torch
    from paper_1301_1215_amd.autograd import nlinv_F
    n, J = 32, 4
    fr, logits, rho, chat, rng = _setup(n, J, 0)
    with Plan(n, n, J) as pl:
        r = dev(rho).requires_grad_()
        c = dev(chat).requires_grad_()
        P = dev(fr.P).requires_grad_()
        # eps = 1 is exact for a bilinear map; FP32 sets the tolerance
        assert torch.autograd.gradcheck(lambda a, b, p: nlinv_F(a, b, p, pl), (r, c, P), eps=1.0,
                                        atol=2e-3, rtol=2e-3, fast_mode=True, nondet_tol=0.0)


def test_backward_is_the_oracle_adjoint_and_central_differences():
    import torch
    from paper_1301_1215_amd.autograd import nlinv_F
    n, J = 32, 4
    fr, logits, rho, chat, rng = _setup(n, J, 1)
    g = rand_c((J, n, n), rng)
    h_rho, h_chat = rand_c((n, n), rng), rand_c((J, n, n), rng)
    d = O.Dims(n, n, J)
    with Plan(n, n, J) as pl:
        r = dev(rho).requires_grad_()
        c = dev(chat).requires_grad_()
        P = dev(fr.P).requires_grad_()
        y = nlinv_F(r, c, P, pl)
        L = (torch.conj(dev(g)) * y).real.sum()
        L.backward()
        gr, gc, gP = host(r.grad), host(c.grad), host(P.grad)
        # exact central difference of the GPU forward along h
        yp = host(pl.forward(dev(rho + h_rho), dev(chat + h_chat), dev(fr.P))).astype(np.complex128)
        ym = host(pl.forward(dev(rho - h_rho), dev(chat - h_chat), dev(fr.P))).astype(np.complex128)
    a_rho, a_chat = O.adjoint(rho, chat, fr.P, g, d)
    assert rel(gr, a_rho) < 1e-5
    assert rel(gc, a_chat) < 1e-5
    assert rel(gP, O.mask_gradient(rho, chat, fr.P, g, d)) < 1e-5
    dd = np.vdot(g.astype(np.complex128), (yp - ym) / 2).real
    dg = np.vdot(gr.astype(np.complex128), h_rho).real + np.vdot(gc.astype(np.complex128), h_chat).real
    assert abs(dd - dg) / abs(dd) < 1e-4


def test_mask_logits_gradient_256x256_8_coils():
    """Data-consistency loss of a soft mask P = sigmoid(logits):
    dL/dlogits against the oracle mask gradient chained through the sigmoid,
    and against an exact central difference in P (L is quadratic in P)."""
    import torch
    from paper_1301_1215_amd.autograd import nlinv_F
    n, J = 256, 8
    fr, logits, rho, chat, rng = _setup(n, J, 2)
    d = O.Dims(n, n, J)
    with Plan(n, n, J) as pl:
        lg = dev(logits).requires_grad_()
        P = torch.sigmoid(lg)
        y = nlinv_F(dev(rho), dev(chat), P, pl)
        L = 0.5 * (y - dev(fr.y)).abs().pow(2).sum()
        L.backward()
        got = host(lg.grad)
        Pf = host(P.detach())
    g = O.forward(rho, chat, Pf, d) - fr.y.astype(np.complex128)
    sig = 1.0 / (1.0 + np.exp(-logits.astype(np.float64)))
    ref = O.mask_gradient(rho, chat, Pf, g, d) * sig * (1.0 - sig)
    assert rel(got, ref) < 1e-4
    e = rng.standard_normal((n, n))
    Lf = lambda PP: 0.5 * np.linalg.norm(O.forward(rho, chat, PP, d) - fr.y) ** 2
    fd = (Lf(Pf + e) - Lf(Pf - e)) / 2.0
    gP = O.mask_gradient(rho, chat, Pf, g, d)
    assert abs(np.sum(gP * e) - fd) / abs(fd) < 1e-9
