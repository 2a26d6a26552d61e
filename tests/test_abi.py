"""The C ABI library: it loads, exports every entry point include/nlinv.h
declares, and rejects bad arguments before touching a GPU."""
import ctypes
import os
import re

import pytest

from paper_1301_1215_amd import _native as N

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    src = open(os.path.join(ROOT, "include", "nlinv.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(nlinv_\w+)\s*\(", src)) - {"NLINV_STATS_LEN"})


def test_header_declares_the_five_operators_and_solves():
    names = declared_functions()
    for f in ("nlinv_forward", "nlinv_deriv", "nlinv_adjoint", "nlinv_normal", "nlinv_irgnm_solve",
              "nlinv_irgnm_solve_batch", "nlinv_irgnm_solve_series"):
        assert f in names


def test_library_exports_every_declared_symbol():
    lib = N.load()
    missing = [f for f in declared_functions() if not hasattr(lib, f)]
    assert not missing, missing
    assert sorted(N.EXPORTED) == declared_functions()


def _create(n, n_om, J, a=220.0, l=32.0):
    lib = N.load()
    h = ctypes.c_void_p()
    d = (N.nlinv_dims * 1)(N.nlinv_dims(n, n_om, J, a, l))
    st = lib.nlinv_plan_create(ctypes.byref(h), d, 1)
    if st == N.NLINV_OK:
        lib.nlinv_plan_destroy(h)
    return st


@pytest.mark.parametrize("n,n_om,J,code", [
    (100, 50, 4, N.NLINV_EUNSUPPORTED),    # 100 = 2^2 5^2
    (6, 6, 1, N.NLINV_EUNSUPPORTED),       # below the smallest grid
    (2048, 64, 1, N.NLINV_EUNSUPPORTED),   # above the largest grid
    (64, 33, 4, N.NLINV_EUNSUPPORTED),     # odd Omega side
    (64, 128, 4, N.NLINV_EUNSUPPORTED),    # Omega larger than the grid
    (64, 32, 65, N.NLINV_EUNSUPPORTED),    # too many coils
    (64, 32, 0, N.NLINV_EINVAL),
    (0, 0, 1, N.NLINV_EINVAL),
])
def test_plan_create_rejects_bad_dims(n, n_om, J, code):
    assert _create(n, n_om, J) == code


def test_null_arguments():
    lib = N.load()
    d = (N.nlinv_dims * 1)(N.nlinv_dims(64, 32, 4, 220.0, 32.0))
    assert lib.nlinv_plan_create(None, d, 1) == N.NLINV_EINVAL
    assert lib.nlinv_plan_destroy(None) == N.NLINV_OK
    assert lib.nlinv_forward(None, None, None, None, None, None, None) == N.NLINV_EINVAL
    assert lib.nlinv_irgnm_solve(None, None, None, None, None, None, None, None, None, None, None) == N.NLINV_EINVAL
    assert lib.nlinv_status_string(N.NLINV_EUNSUPPORTED) == b"unsupported size"
    assert lib.nlinv_kernel_class_name(-1) is None
    assert len(N.nlinv_kernel_class_names()) > 10


@pytest.mark.parametrize("n", [8, 12, 16, 24, 32, 48, 64, 96, 128, 192, 256, 384, 512, 768, 1024])
def test_every_supported_size_passes_the_host_checks(n):
    """Plan creation checks sizes and pass variants on the host before any
    HIP call; a supported size gets past them (to NLINV_OK on a GPU, or to a
    HIP error where there is none)."""
    assert _create(n, n // 2, 4) in (N.NLINV_OK, N.NLINV_EHIP)


# ---- the binding's shape checks (run before any library call, no GPU needed)

@pytest.fixture
def fake_plan():
    """A handle registered with frame shapes, as nlinv_plan_create would; the
    library is never called with it (every check below fails first)."""
    h = ctypes.c_void_p(0x1000)
    N._PLANS[h.value] = [(16, 8, 2)]
    yield h
    N._PLANS.pop(h.value, None)


def _t(*shape, dtype=None):
    import torch
    return torch.zeros(shape, dtype=dtype or torch.complex64)


def test_operator_shapes_are_checked_before_the_call(fake_plan):
    import torch
    good = dict(rho=_t(8, 8), chat=_t(2, 16, 16), c=_t(2, 8, 8), P=_t(16, 16, dtype=torch.float32))
    with pytest.raises(ValueError, match="drho"):
        N.nlinv_normal(fake_plan, good["rho"], good["chat"], good["c"], good["P"], 1.0, _t(16, 16),
                       _t(2, 16, 16), _t(8, 8), _t(2, 16, 16))
    with pytest.raises(ValueError, match="dchat_out"):
        N.nlinv_adjoint(fake_plan, good["rho"], good["chat"], None, good["P"], _t(2, 16, 16), _t(8, 8),
                        _t(3, 16, 16))
    with pytest.raises(ValueError, match="P"):
        N.nlinv_forward(fake_plan, good["rho"], good["chat"], _t(8, 8, dtype=torch.float32), _t(2, 16, 16))
    with pytest.raises(ValueError, match="c_out"):
        N.nlinv_coil_maps(fake_plan, good["chat"], _t(2, 16, 16))
    with pytest.raises(ValueError, match="gP_out"):
        N.nlinv_mask_gradient(fake_plan, good["rho"], good["chat"], None, _t(2, 16, 16), _t(8, 8))


def test_solve_shapes_and_frame_counts_are_checked(fake_plan):
    import torch
    prm = N.make_params(2, 3)
    f = dict(y=_t(2, 16, 16), P=_t(16, 16, dtype=torch.float32), rho=_t(8, 8), chat=_t(2, 16, 16),
             stats=torch.zeros(N.stats_len(2, 3), dtype=torch.float64))
    with pytest.raises(ValueError, match="2 frame descriptors for a plan of 1"):
        N.nlinv_irgnm_solve_batch(fake_plan, [f, f], prm)
    with pytest.raises(ValueError, match="stats"):
        N.nlinv_irgnm_solve_batch(fake_plan, [dict(f, stats=torch.zeros(3, dtype=torch.float64))], prm)
    with pytest.raises(ValueError, match="chat_ref"):
        N.nlinv_irgnm_solve(fake_plan, f["y"], f["P"], prm, f["rho"], f["chat"], _t(8, 8), _t(2, 8, 8))
    with pytest.raises(ValueError, match="frame 1 y"):
        N.nlinv_irgnm_solve_series(fake_plan, [f, dict(f, y=_t(2, 16, 8))], prm)
    with pytest.raises(ValueError, match="unknown plan"):
        N.nlinv_normal(ctypes.c_void_p(0x2000), *[None] * 9)


def test_noalloc_normal_refuses_before_touching_a_gpu():
    """NULL arguments, bad dims and frames larger than the static scratch are
    refused before any HIP call (the pointers here are never dereferenced)."""
    lib = N.load()
    fake = ctypes.c_void_p(1 << 20)     # aligned, never read: the call returns first
    def call(n, m, J, c=fake, rho=fake):
        d = N.nlinv_dims(n, m, J, 220.0, 32.0)
        return lib.nlinv_normal_noalloc(ctypes.byref(d), rho, fake, c, fake, 1.0, fake, fake, fake, fake, None)
    assert call(512, 256, 32, rho=None) == N.NLINV_EINVAL
    assert call(100, 50, 4) == N.NLINV_EUNSUPPORTED
    assert call(1024, 1024, 16) == N.NLINV_ESCRATCH
    # 512 x 512, Omega 256, 32 coils fits with and without a caller's c
    assert N.noalloc_scratch_need(512, 256, 32, with_c=False) <= N.NOALLOC_SCRATCH_BYTES
    assert N.noalloc_scratch_need(1024, 512, 16, with_c=False) > N.NOALLOC_SCRATCH_BYTES
    assert call(1024, 512, 16, c=None) == N.NLINV_ESCRATCH
    assert lib.nlinv_status_string(N.NLINV_ESCRATCH).decode().startswith("frame too large")


def test_gridding_refuses_bad_arguments_before_touching_a_gpu():
    lib = N.load()
    fake = ctypes.c_void_p(1 << 20)
    def call(n=64, J=2, S=3, R=64, width=4.0, beta=9.0, angles=fake, data=fake, dcf=None):
        return lib.nlinv_grid_radial(n, J, S, R, angles, dcf, width, beta, data, fake, None)
    assert call(width=64.0) == N.NLINV_EINVAL          # window as wide as the grid
    assert call(width=0.0) == N.NLINV_EINVAL
    assert call(beta=-1.0) == N.NLINV_EINVAL
    assert call(S=0) == N.NLINV_EINVAL
    assert call(S=1025) == N.NLINV_EINVAL
    assert call(angles=None) == N.NLINV_EINVAL
    assert call(data=ctypes.c_void_p((1 << 20) + 4)) == N.NLINV_EINVAL   # complex data 8-byte aligned
    assert lib.nlinv_degrid_radial(64, 2, 3, 64, fake, None, 4.0, 9.0, fake, None, None) == N.NLINV_EINVAL


def test_coil_compression_refuses_bad_arguments_before_touching_a_gpu():
    lib = N.load()
    fake = ctypes.c_void_p(1 << 20)
    assert lib.nlinv_coil_compress_workspace(0, 100) == 0
    assert lib.nlinv_coil_compress_workspace(65, 100) == 0
    need = lib.nlinv_coil_compress_workspace(8, 4096)
    assert need > 0
    def call(J=8, M=4096, K=3, ws=need, y=fake):
        return lib.nlinv_coil_compress(J, M, K, y, fake, None, None, fake, ws, None)
    assert call(K=0) == N.NLINV_EINVAL
    assert call(K=9) == N.NLINV_EINVAL
    assert call(ws=need - 1) == N.NLINV_EINVAL
    assert call(y=None) == N.NLINV_EINVAL
    assert call(J=65) == N.NLINV_EINVAL
