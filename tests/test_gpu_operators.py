"""GPU parity of every operator call of the C ABI against the FP64 oracle.

Bar: relative L2 error <= 1e-5 per apply (FP32 on the GPU, FP64 oracle on
the same complex64 / float32 inputs)."""
import numpy as np
import pytest

from oracle import nlinv_oracle as O
from paper_1301_1215_amd import Plan
from tests.gpu_util import dev, host, rel, rand_c, soft_mask

pytestmark = pytest.mark.gpu

TOL = 1e-5
SIZES = [8, 12, 16, 24, 32, 48, 64, 96, 128, 192, 256, 384, 512, 768, 1024]


@pytest.mark.parametrize("n", SIZES)
def test_fft_engine_is_the_centred_unitary_dft(n):
    """One coil, chat = n * delta at DC (so c = 1), P = 1, Omega = grid:
    F(rho) is the centred DFT of rho, on every supported grid size."""
    rng = np.random.default_rng([10, n])
    rho = rand_c((n, n), rng)
    chat = np.zeros((1, n, n), np.complex64)
    chat[0, n // 2, n // 2] = n
    with Plan(n, n, 1) as pl:
        y = host(pl.forward(dev(rho), dev(chat), dev(np.ones((n, n), np.float32))))
    assert rel(y[0], O.dft2c(rho)) < TOL


@pytest.mark.parametrize("n", [8, 12, 48, 384, 1024])
def test_coil_maps_inverse_weighted_dft(n):
    rng = np.random.default_rng([11, n])
    n_om = n // 2
    d = O.Dims(n, n_om, 3)
    chat = rand_c((3, n, n), rng)
    with Plan(n, n_om, 3) as pl:
        c = host(pl.coil_maps(dev(chat)))
    assert rel(c, O.coil_maps(chat, d)) < TOL


SHAPES = [(64, 64, 8), (384, 192, 12), (96, 48, 3), (48, 24, 2), (128, 64, 5), (512, 256, 4),
          (32, 32, 1), (24, 12, 3), (1024, 512, 2), (8, 2, 1), (192, 96, 7), (768, 384, 1)]


def _point(n, n_om, J, seed):
    rng = np.random.default_rng([12, n, n_om, J, seed])
    rho = rand_c((n_om, n_om), rng)
    chat = rand_c((J, n, n), rng)
    P = soft_mask(n, rng)
    return rng, rho, chat, P


@pytest.mark.parametrize("n,n_om,J", SHAPES)
def test_operators_match_oracle(n, n_om, J):
    rng, rho, chat, P = _point(n, n_om, J, 0)
    drho, dchat = rand_c((n_om, n_om), rng), rand_c((J, n, n), rng)
    z = rand_c((J, n, n), rng)
    alpha = 0.3
    d = O.Dims(n, n_om, J)
    with Plan(n, n_om, J) as pl:
        g_rho, g_chat, gP, g_drho, g_dchat, gz = map(dev, (rho, chat, P, drho, dchat, z))
        y, c = pl.forward(g_rho, g_chat, gP, return_c=True)
        dy = pl.deriv(g_rho, g_chat, gP, g_drho, g_dchat, c=c)
        dy_nc = pl.deriv(g_rho, g_chat, gP, g_drho, g_dchat)
        ar, ac = pl.adjoint(g_rho, g_chat, gP, gz, c=c)
        nr, nc = pl.normal(g_rho, g_chat, gP, alpha, g_drho, g_dchat, c=c)
        img = pl.image(g_rho, c)
        y, c, dy, dy_nc, ar, ac, nr, nc, img = map(host, (y, c, dy, dy_nc, ar, ac, nr, nc, img))
    c_ref = O.coil_maps(chat, d)
    assert rel(c, c_ref) < TOL
    assert rel(y, O.forward(rho, chat, P, d)) < TOL
    dy_ref = O.deriv(rho, chat, P, drho, dchat, d)
    assert rel(dy, dy_ref) < TOL
    assert rel(dy_nc, dy_ref) < TOL
    a_ref = O.adjoint(rho, chat, P, z, d)
    assert rel(ar, a_ref[0]) < TOL
    assert rel(ac, a_ref[1]) < TOL
    n_ref = O.normal(rho, chat, P, alpha, drho, dchat, d)
    assert rel(nr, n_ref[0]) < TOL
    assert rel(nc, n_ref[1]) < TOL
    assert rel(img, O.combined_image(rho, chat, d)) < TOL


@pytest.mark.parametrize("n,n_om,J", [(64, 32, 4), (384, 192, 12), (48, 48, 2)])
def test_adjoint_identity_in_fp32(n, n_om, J):
    """<DF h, z> = <h, DF^H z> evaluated on the GPU outputs."""
    rng, rho, chat, P = _point(n, n_om, J, 1)
    h_rho, h_chat, z = rand_c((n_om, n_om), rng), rand_c((J, n, n), rng), rand_c((J, n, n), rng)
    with Plan(n, n_om, J) as pl:
        dy = host(pl.deriv(dev(rho), dev(chat), dev(P), dev(h_rho), dev(h_chat)))
        ar, ac = map(host, pl.adjoint(dev(rho), dev(chat), dev(P), dev(z)))
    lhs = np.vdot(dy.astype(np.complex128), z.astype(np.complex128))
    rhs = np.vdot(h_rho.astype(np.complex128), ar) + np.vdot(h_chat.astype(np.complex128), ac)
    assert abs(lhs - rhs) / abs(lhs) < TOL


@pytest.mark.parametrize("n,n_om,J", [(32, 32, 4), (256, 256, 8), (96, 48, 3)])
def test_mask_gradient_matches_oracle(n, n_om, J):
    rng, rho, chat, P = _point(n, n_om, J, 2)
    g = rand_c((J, n, n), rng)
    d = O.Dims(n, n_om, J)
    with Plan(n, n_om, J) as pl:
        gP = host(pl.mask_gradient(dev(rho), dev(chat), dev(g)))
    assert rel(gP, O.mask_gradient(rho, chat, P, g, d)) < TOL


@pytest.mark.parametrize("n,n_om,J", [(384, 192, 12), (64, 64, 8)])
def test_every_pass_variant_gives_the_same_operator(n, n_om, J):
    from paper_1301_1215_amd._native import NlinvError
    rng, rho, chat, P = _point(n, n_om, J, 3)
    drho, dchat = rand_c((n_om, n_om), rng), rand_c((J, n, n), rng)
    d = O.Dims(n, n_om, J)
    n_ref = O.normal(rho, chat, P, 0.5, drho, dchat, d)
    with Plan(n, n_om, J) as pl:
        tried = 0
        for cv in range(4):
            for rv in range(8):
                try:
                    pl.set_variant(n, cv, rv)
                except NlinvError:
                    continue
                tried += 1
                nr, nc = map(host, pl.normal(dev(rho), dev(chat), dev(P), 0.5, dev(drho), dev(dchat)))
                assert rel(nr, n_ref[0]) < TOL, (cv, rv)
                assert rel(nc, n_ref[1]) < TOL, (cv, rv)
        assert tried >= 4


def test_kernel_timing_counts_launches():
    n, n_om, J = 128, 64, 4
    rng, rho, chat, P = _point(n, n_om, J, 4)
    with Plan(n, n_om, J) as pl:
        pl.timing_enable("col_psf")
        args = tuple(map(dev, (rho, chat, P)))
        for _ in range(3):
            pl.normal(*args, 0.5, dev(rho), dev(chat))
        cnt, ms = pl.timing_read()
        assert cnt == 3 and ms > 0
        assert pl.timing_read()[0] == 0
        # every 2nd launch from the enable call: launches 0, 2, 4 of 5
        pl.timing_enable("col_psf", 2)
        for _ in range(5):
            pl.normal(*args, 0.5, dev(rho), dev(chat))
        assert pl.timing_read()[0] == 3
        from paper_1301_1215_amd._native import NlinvError
        with pytest.raises(NlinvError):
            pl.timing_enable("col_psf", -1)


# 1D transforms done by one launch of each pass class (per plane)
TRANSFORMS_1D = {"col_winv_ifft": 1, "col_p_ifft": 1, "col_fft_p": 1, "col_resid_p_ifft": 2, "col_psf": 2,
                 "col_fft_winv_add": 1, "col_fft_gprod": 1, "row_cache": 1, "row_fwd": 1, "row_deriv": 2,
                 "row_adj": 2}


def _launch_counts(pl, fn):
    from paper_1301_1215_amd import _native as NAT
    import torch
    counts = {}
    for k in NAT.nlinv_kernel_class_names():
        pl.timing_enable(k, True)
        fn()
        torch.cuda.synchronize()
        cnt, _ = pl.timing_read()
        pl.timing_enable(k, False)
        if cnt:
            counts[k] = cnt
    return counts


def test_transform_counts_match_table1():
    """Table 1: F, DF and DF^H each take two 2D transforms (F including the
    W^{-1} of the sensitivities; DF and DF^H with them cached), and DF^H one
    channel summation."""
    from tests.test_oracle_pins import _table1
    t1 = _table1()
    n, n_om, J = 64, 32, 3
    rng, rho, chat, P = _point(n, n_om, J, 5)
    with Plan(n, n_om, J) as pl:
        r, c_, Pd, z = dev(rho), dev(chat), dev(P), dev(rand_c((J, n, n), rng))
        c = pl.coil_maps(c_)
        ops = {"F": lambda: pl.forward(r, c_, Pd),
               "DF": lambda: pl.deriv(r, c_, Pd, r, c_, c=c),
               "DFH": lambda: pl.adjoint(r, c_, Pd, z, c=c)}
        for name, fn in ops.items():
            counts = _launch_counts(pl, fn)
            n1d = sum(TRANSFORMS_1D.get(k, 0) * v for k, v in counts.items())
            assert n1d == 2 * t1[name]["fft"], (name, counts)
            assert counts.get("coil_sum", 0) == t1[name]["sum_c"], (name, counts)


def test_autotune_picks_valid_variants_and_keeps_parity(tmp_path, monkeypatch):
    monkeypatch.setenv("NLINV_TUNE_CACHE", str(tmp_path / "tune.txt"))
    n, n_om, J = 192, 96, 6
    rng, rho, chat, P = _point(n, n_om, J, 6)
    drho, dchat = rand_c((n_om, n_om), rng), rand_c((J, n, n), rng)
    d = O.Dims(n, n_om, J)
    ref = O.normal(rho, chat, P, 0.5, drho, dchat, d)
    with Plan(n, n_om, J) as pl:
        pl.autotune()
        cv, rv = pl.variant(n)
        assert cv >= 0 and rv >= 0
        nr, nc = map(host, pl.normal(dev(rho), dev(chat), dev(P), 0.5, dev(drho), dev(dchat)))
        assert rel(nr, ref[0]) < TOL and rel(nc, ref[1]) < TOL
    line = (tmp_path / "tune.txt").read_text().split()
    # arch, n, planes, the side of the band the solve keeps (64 at n = 192), 9 + 4 variants,
    # the normal operator's and the CG iteration's forms (no whole-plane kernel at 192: the
    # axis passes), the intermediates' access policy
    assert line[1:4] == ["192", str(J), "64"] and len(line) == 4 + 9 + 4 + 3 and line[-3:-1] == ["0", "0"]
    assert line[-1] in ("0", "1")
    with Plan(n, n_om, J) as pl2:    # served from the cache file
        pl2.autotune()
        assert pl2.variant(n) == (cv, rv)
        assert pl2.streaming() == int(line[-1])


def test_streaming_policy_follows_the_intermediate_size():
    """The pass intermediates are streamed where one of them ([planes][m][n]
    complex) exceeds 30 MiB: 32 planes of 256 x 512 (32 MiB) yes, four
    12-coil frames of 192 x 384 (27 MiB) and small grids no."""
    with Plan(512, 256, 32) as pl:
        assert pl.streaming() == 1
    with Plan(frames=[(384, 192, 12)] * 4) as pl:
        assert pl.streaming(384) == 0
    with Plan(64, 32, 8) as pl:
        assert pl.streaming() == 0
        pl.set_streaming(1)
        assert pl.streaming() == 1


def test_kernel_timing_inside_a_replayed_graph():
    from paper_1301_1215_amd import synth
    fr = synth.make_frame(2, 9, 64, 32, 3, "radial", spokes=9)
    with Plan(64, 32, 3) as pl:
        pl.timing_enable("col_psf")
        prm = Plan.params(2, 4, use_graph=True)
        for _ in range(3):
            pl.solve(dev(fr.y), dev(fr.P), prm)
        cnt, ms = pl.timing_read()
        assert cnt == 2 * 4 and ms > 0     # one replay's launches
        cnt2, _ = pl.timing_read()         # graph-owned brackets stay readable
        assert cnt2 == cnt


@pytest.mark.parametrize("n,n_om,J", [(8, 4, 2), (12, 6, 2), (16, 16, 3), (24, 12, 3), (24, 10, 2),
                                      (32, 16, 4), (48, 24, 4), (64, 32, 8), (64, 64, 8)])
def test_whole_plane_normal_matches_oracle(n, n_om, J):
    """The whole-plane kernel (one workgroup per coil plane, the four centred
    2D transforms of DF and DF^H in LDS) against the FP64 oracle and against
    the axis passes, Omega the centred half, the grid, and an uneven crop."""
    rng, rho, chat, P = _point(n, n_om, J, 7)
    drho, dchat = rand_c((n_om, n_om), rng), rand_c((J, n, n), rng)
    d = O.Dims(n, n_om, J)
    ref = O.normal(rho, chat, P, 0.5, drho, dchat, d)
    with Plan(n, n_om, J) as pl:
        pl.set_normal_form(1)
        assert pl.normal_form() == 1
        args = (dev(rho), dev(chat), dev(P), 0.5, dev(drho), dev(dchat))
        wr, wc = map(host, pl.normal(*args))
        pl.set_normal_form(0)
        ar, ac = map(host, pl.normal(*args))
    assert rel(wr, ref[0]) < TOL and rel(wc, ref[1]) < TOL
    assert rel(wr, ar) < TOL and rel(wc, ac) < TOL


def test_whole_plane_form_only_where_it_exists():
    from paper_1301_1215_amd._native import NlinvError
    with Plan(96, 48, 2) as pl:
        assert pl.normal_form() == 0
        with pytest.raises(NlinvError):
            pl.set_normal_form(1)


def test_autotune_chooses_the_normal_form_and_keeps_parity(tmp_path, monkeypatch):
    """At 64 x 64 (8 coils) the autotuner times the axis passes against the
    whole-plane kernel for nlinv_normal; whichever it keeps, the operator
    keeps parity and the cache line records the choice."""
    monkeypatch.setenv("NLINV_TUNE_CACHE", str(tmp_path / "tune.txt"))
    n, n_om, J = 64, 64, 8
    rng, rho, chat, P = _point(n, n_om, J, 8)
    drho, dchat = rand_c((n_om, n_om), rng), rand_c((J, n, n), rng)
    ref = O.normal(rho, chat, P, 0.5, drho, dchat, O.Dims(n, n_om, J))
    with Plan(n, n_om, J) as pl:
        pl.autotune()
        form = pl.normal_form()
        assert form in (0, 1)
        nr, nc = map(host, pl.normal(dev(rho), dev(chat), dev(P), 0.5, dev(drho), dev(dchat)))
        assert rel(nr, ref[0]) < TOL and rel(nc, ref[1]) < TOL
    line = (tmp_path / "tune.txt").read_text().split()
    assert line[1:3] == ["64", str(J)] and line[-3] == str(form) and line[-2] in ("0", "1")
    with Plan(n, n_om, J) as pl2:    # served from the cache file
        pl2.autotune()
        assert pl2.normal_form() == form
