"""ctypes binding of libnlinv.so (include/nlinv.h): argument marshalling only.

Every function here has the name of the C entry point it calls and passes
torch tensors' device pointers and the current HIP stream through.  No step
of the computation runs in Python.  Loading fails loudly when the library is
missing: there is no fallback path.
"""
from __future__ import annotations

import ctypes as C
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libnlinv.so")

NLINV_OK, NLINV_EINVAL, NLINV_EUNSUPPORTED, NLINV_ENOMEM, NLINV_EHIP, NLINV_ESCRATCH = 0, -1, -2, -3, -4, -5
# bytes of the static device scratch of nlinv_normal_noalloc (NLINV_NOALLOC_SCRATCH_BYTES)
NOALLOC_SCRATCH_BYTES = 80 << 20
NLINV_USE_GRAPH, NLINV_WARM_START = 1, 2

EXPORTED = (
    "nlinv_plan_create", "nlinv_plan_create_branched", "nlinv_plan_destroy", "nlinv_coil_maps", "nlinv_forward", "nlinv_deriv",
    "nlinv_adjoint", "nlinv_normal", "nlinv_normal_noalloc", "nlinv_mask_gradient", "nlinv_image", "nlinv_irgnm_solve",
    "nlinv_irgnm_solve_batch", "nlinv_irgnm_solve_series", "nlinv_plan_autotune", "nlinv_plan_variant", "nlinv_plan_band",
    "nlinv_plan_normal_form", "nlinv_plan_set_normal_form", "nlinv_plan_cg_form", "nlinv_plan_set_cg_form",
    "nlinv_plan_streaming", "nlinv_plan_set_streaming",
    "nlinv_plan_set_variant", "nlinv_plan_timing_enable", "nlinv_plan_timing_read",
    "nlinv_plan_timing_read_class",
    "nlinv_kernel_class_name", "nlinv_status_string", "nlinv_last_hip_error", "nlinv_bandwidth_probe",
    "nlinv_grid_radial", "nlinv_degrid_radial", "nlinv_coil_compress_workspace", "nlinv_coil_compress",
    "nlinv_gn_step_vjp_workspace", "nlinv_gn_step_vjp", "nlinv_check_launch_args",
)


class nlinv_dims(C.Structure):
    _fields_ = [("n", C.c_int32), ("n_om", C.c_int32), ("ncoils", C.c_int32),
                ("sobolev_a", C.c_float), ("sobolev_l", C.c_float)]


class nlinv_irgnm_params(C.Structure):
    _fields_ = [("newton_steps", C.c_int32), ("cg_iters", C.c_int32), ("alpha0", C.c_float),
                ("alpha_q", C.c_float), ("alpha_min", C.c_float), ("scale_norm", C.c_float),
                ("flags", C.c_uint32)]


class nlinv_frame(C.Structure):
    _fields_ = [("y", C.c_void_p), ("P", C.c_void_p), ("rho", C.c_void_p), ("chat", C.c_void_p),
                ("rho_ref", C.c_void_p), ("chat_ref", C.c_void_p), ("image", C.c_void_p),
                ("stats", C.c_void_p)]


def stats_len(newton: int, cg: int) -> int:
    return 2 + newton + newton * cg


class NlinvError(RuntimeError):
    pass


_lib = None


def load(path: str | None = None):
    """Load the library (once).  Raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    p = path or LIB_PATH
    if not os.path.exists(p):
        raise NlinvError(f"{p} not found: build it with `python -m paper_1301_1215_amd.build`")
    lib = C.CDLL(p)
    vp, i32, f32 = C.c_void_p, C.c_int32, C.c_float
    sig = {
        "nlinv_plan_create": ([C.POINTER(vp), C.POINTER(nlinv_dims), i32], C.c_int),
        "nlinv_plan_create_branched": ([C.POINTER(vp), C.POINTER(nlinv_dims), i32, i32], C.c_int),
        "nlinv_plan_destroy": ([vp], C.c_int),
        "nlinv_coil_maps": ([vp, vp, vp, vp], C.c_int),
        "nlinv_forward": ([vp, vp, vp, vp, vp, vp, vp], C.c_int),
        "nlinv_deriv": ([vp, vp, vp, vp, vp, vp, vp, vp, vp], C.c_int),
        "nlinv_adjoint": ([vp, vp, vp, vp, vp, vp, vp, vp, vp], C.c_int),
        "nlinv_normal": ([vp, vp, vp, vp, vp, f32, vp, vp, vp, vp, vp], C.c_int),
        "nlinv_normal_noalloc": ([C.POINTER(nlinv_dims), vp, vp, vp, vp, f32, vp, vp, vp, vp, vp], C.c_int),
        "nlinv_mask_gradient": ([vp, vp, vp, vp, vp, vp, vp], C.c_int),
        "nlinv_image": ([vp, vp, vp, vp, vp], C.c_int),
        "nlinv_irgnm_solve": ([vp, vp, vp, C.POINTER(nlinv_irgnm_params), vp, vp, vp, vp, vp, vp, vp], C.c_int),
        "nlinv_irgnm_solve_batch": ([vp, C.POINTER(nlinv_frame), C.POINTER(nlinv_irgnm_params), vp], C.c_int),
        "nlinv_irgnm_solve_series": ([vp, i32, C.POINTER(nlinv_frame), C.POINTER(nlinv_irgnm_params), vp],
                                     C.c_int),
        "nlinv_plan_autotune": ([vp, vp], C.c_int),
        "nlinv_plan_variant": ([vp, i32, C.POINTER(i32), C.POINTER(i32)], C.c_int),
        "nlinv_plan_set_variant": ([vp, i32, i32, i32], C.c_int),
        "nlinv_plan_normal_form": ([vp, i32, C.POINTER(i32)], C.c_int),
        "nlinv_plan_set_normal_form": ([vp, i32, i32], C.c_int),
        "nlinv_plan_cg_form": ([vp, i32, C.POINTER(i32)], C.c_int),
        "nlinv_plan_set_cg_form": ([vp, i32, i32], C.c_int),
        "nlinv_plan_streaming": ([vp, i32, C.POINTER(i32)], C.c_int),
        "nlinv_plan_set_streaming": ([vp, i32, i32], C.c_int),
        "nlinv_plan_band": ([vp, i32, C.POINTER(i32), C.POINTER(i32)], C.c_int),
        "nlinv_plan_timing_enable": ([vp, i32, i32], C.c_int),
        "nlinv_plan_timing_read": ([vp, C.POINTER(i32), C.POINTER(C.c_double)], C.c_int),
        "nlinv_plan_timing_read_class": ([vp, i32, C.POINTER(i32), C.POINTER(C.c_double)], C.c_int),
        "nlinv_kernel_class_name": ([i32], C.c_char_p),
        "nlinv_status_string": ([C.c_int], C.c_char_p),
        "nlinv_bandwidth_probe": ([vp, vp, C.c_size_t, vp], C.c_int),
        "nlinv_grid_radial": ([i32, i32, i32, i32, vp, vp, f32, f32, vp, vp, vp], C.c_int),
        "nlinv_coil_compress_workspace": ([i32, C.c_int64], C.c_size_t),
        "nlinv_gn_step_vjp_workspace": ([vp], C.c_size_t),
        "nlinv_check_launch_args": ([i32, i32, i32, i32, i32, i32, i32, C.POINTER(C.c_int64), C.POINTER(i32)],
                                    C.c_int),
        "nlinv_gn_step_vjp": ([vp, vp, vp, vp, vp, f32, vp, vp, vp, vp, vp, vp, i32, vp, vp, vp, vp, vp, vp, vp,
                               vp, C.c_size_t, vp], C.c_int),
        "nlinv_coil_compress": ([i32, C.c_int64, i32, vp, vp, vp, vp, vp, C.c_size_t, vp], C.c_int),
        "nlinv_degrid_radial": ([i32, i32, i32, i32, vp, vp, f32, f32, vp, vp, vp], C.c_int),
        "nlinv_last_hip_error": ([], C.c_int),
    }
    for name, (args, res) in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = res
    _lib = lib
    return lib


def check(status: int, what: str = "") -> None:
    if status != NLINV_OK:
        lib = load()
        msg = lib.nlinv_status_string(status).decode()
        hip = lib.nlinv_last_hip_error() if status == NLINV_EHIP else 0
        raise NlinvError(f"{what}: {msg} (status {status}{', hip error %d' % hip if hip else ''})")


# ---------------------------------------------------------------------------
# pointer / stream marshalling
# ---------------------------------------------------------------------------

def _ptr(t, dtype=None, what="tensor"):
    """Device pointer of a contiguous CUDA (HIP) tensor, or None."""
    if t is None:
        return None
    import torch
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{what}: expected a torch.Tensor")
    if not t.is_cuda:
        raise ValueError(f"{what}: must be on the GPU")
    if dtype is not None and t.dtype != dtype:
        raise TypeError(f"{what}: expected {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{what}: must be contiguous")
    return t.data_ptr()


def _stream(stream=None):
    import torch
    s = torch.cuda.current_stream() if stream is None else stream
    return s.cuda_stream if hasattr(s, "cuda_stream") else int(s)


def _c64(t, what):
    import torch
    return _ptr(t, torch.complex64, what)


def _f32(t, what):
    import torch
    return _ptr(t, torch.float32, what)


# ---------------------------------------------------------------------------
# shape checks: every tensor is checked against the plan's frame shapes here,
# before the library is called, so that a wrong-sized array never reaches a
# kernel (the library only sees pointers)
# ---------------------------------------------------------------------------

_PLANS: dict = {}   # plan handle value -> [(n, n_om, ncoils)] per frame


def _plan_dims(plan):
    key = plan.value if isinstance(plan, C.c_void_p) else plan
    dims = _PLANS.get(key)
    if dims is None:
        raise ValueError("unknown plan handle (not created by nlinv_plan_create, or destroyed)")
    return dims


def _expect(t, shape, what):
    """Raise unless t (nullable) has exactly `shape`."""
    if t is None:
        return
    got = tuple(getattr(t, "shape", ()))
    if got != tuple(shape):
        raise ValueError(f"{what}: expected shape {tuple(shape)}, got {got}")


def _op_shapes(plan, **ts):
    """Check operator arguments against frame 0's shape: names ending in
    rho / image are Omega images, chat / y / dy / g k-space coil planes, c
    Omega coil planes, P and gP the grid."""
    n, m, J = _plan_dims(plan)[0]
    for what, t in ts.items():
        base = what.replace("_out", "").replace("_inout", "").replace("_ref", "").replace("_next", "")
        base = base.replace("_n", "") if base.endswith("_n") else base
        base = base.replace("_g", "") if base.endswith("_g") else base
        if base in ("rho", "drho", "image"):
            _expect(t, (m, m), what)
        elif base in ("chat", "dchat", "y", "dy", "g"):
            _expect(t, (J, n, n), what)
        elif base == "c":
            _expect(t, (J, m, m), what)
        elif base in ("P", "gP"):
            _expect(t, (n, n), what)
        else:
            raise KeyError(what)


def _frame_shapes(fd, f, prm, where):
    n, m, J = fd
    for k in ("y", "chat", "chat_ref"):
        _expect(f.get(k), (J, n, n), f"{where} {k}")
    for k in ("rho", "rho_ref", "image"):
        _expect(f.get(k), (m, m), f"{where} {k}")
    _expect(f.get("P"), (n, n), f"{where} P")
    st = f.get("stats")
    if st is not None:
        need = stats_len(prm.newton_steps, prm.cg_iters)
        if st.dim() != 1 or st.numel() < need:
            raise ValueError(f"{where} stats: expected a vector of at least {need} doubles, "
                             f"got shape {tuple(st.shape)}")


# ---------------------------------------------------------------------------
# entry points under their C names
# ---------------------------------------------------------------------------

def nlinv_plan_create(dims_list, nframes=None, branch_frames=0):
    """dims_list: sequence of (n, n_om, ncoils[, a, l]) or nlinv_dims;
    branch_frames > 0 calls nlinv_plan_create_branched."""
    lib = load()
    arr = (nlinv_dims * len(dims_list))()
    for i, d in enumerate(dims_list):
        if isinstance(d, nlinv_dims):
            arr[i] = d
        else:
            a = d[3] if len(d) > 3 else 220.0
            l = d[4] if len(d) > 4 else 32.0
            arr[i] = nlinv_dims(int(d[0]), int(d[1]), int(d[2]), float(a), float(l))
    h = C.c_void_p()
    nf = len(dims_list) if nframes is None else nframes
    if branch_frames:
        check(lib.nlinv_plan_create_branched(C.byref(h), arr, nf, int(branch_frames)),
              "nlinv_plan_create_branched")
    else:
        check(lib.nlinv_plan_create(C.byref(h), arr, nf), "nlinv_plan_create")
    _PLANS[h.value] = [(arr[i].n, arr[i].n_om, arr[i].ncoils) for i in range(nf)]
    return h


def nlinv_plan_destroy(plan):
    check(load().nlinv_plan_destroy(plan), "nlinv_plan_destroy")
    _PLANS.pop(plan.value if isinstance(plan, C.c_void_p) else plan, None)


def nlinv_coil_maps(plan, chat, c_out, stream=None):
    _op_shapes(plan, chat=chat, c_out=c_out)
    check(load().nlinv_coil_maps(plan, _c64(chat, "chat"), _c64(c_out, "c_out"), _stream(stream)),
          "nlinv_coil_maps")


def nlinv_forward(plan, rho, chat, P, y_out, c_out=None, stream=None):
    _op_shapes(plan, rho=rho, chat=chat, P=P, y_out=y_out, c_out=c_out)
    check(load().nlinv_forward(plan, _c64(rho, "rho"), _c64(chat, "chat"), _f32(P, "P"),
                               _c64(y_out, "y_out"), _c64(c_out, "c_out"), _stream(stream)), "nlinv_forward")


def nlinv_deriv(plan, rho, chat, c, P, drho, dchat, dy_out, stream=None):
    _op_shapes(plan, rho=rho, chat=chat, c=c, P=P, drho=drho, dchat=dchat, dy_out=dy_out)
    check(load().nlinv_deriv(plan, _c64(rho, "rho"), _c64(chat, "chat"), _c64(c, "c"), _f32(P, "P"),
                             _c64(drho, "drho"), _c64(dchat, "dchat"), _c64(dy_out, "dy_out"),
                             _stream(stream)), "nlinv_deriv")


def nlinv_adjoint(plan, rho, chat, c, P, dy, drho_out, dchat_out, stream=None):
    _op_shapes(plan, rho=rho, chat=chat, c=c, P=P, dy=dy, drho_out=drho_out, dchat_out=dchat_out)
    check(load().nlinv_adjoint(plan, _c64(rho, "rho"), _c64(chat, "chat"), _c64(c, "c"), _f32(P, "P"),
                               _c64(dy, "dy"), _c64(drho_out, "drho_out"), _c64(dchat_out, "dchat_out"),
                               _stream(stream)), "nlinv_adjoint")


def nlinv_normal(plan, rho, chat, c, P, alpha, drho, dchat, drho_out, dchat_out, stream=None):
    _op_shapes(plan, rho=rho, chat=chat, c=c, P=P, drho=drho, dchat=dchat, drho_out=drho_out,
               dchat_out=dchat_out)
    check(load().nlinv_normal(plan, _c64(rho, "rho"), _c64(chat, "chat"), _c64(c, "c"), _f32(P, "P"),
                              float(alpha), _c64(drho, "drho"), _c64(dchat, "dchat"),
                              _c64(drho_out, "drho_out"), _c64(dchat_out, "dchat_out"), _stream(stream)),
          "nlinv_normal")


def noalloc_scratch_need(n, n_om, ncoils, with_c):
    """Scratch bytes nlinv_normal_noalloc needs for a frame (its header's formula)."""
    r = lambda b: (b + 255) // 256 * 256
    om = r(8 * ncoils * n_om * n_om)
    return r(8 * n) + r(4 * n * n) + om + r(8 * ncoils * n_om * n) + (0 if with_c else om)


def nlinv_normal_noalloc(dims, rho, chat, c, P, alpha, drho, dchat, drho_out, dchat_out, stream=None):
    """dims: (n, n_om, ncoils[, a, l]) of the one frame; no plan."""
    n, m, J = int(dims[0]), int(dims[1]), int(dims[2])
    a = float(dims[3]) if len(dims) > 3 else 220.0
    l = float(dims[4]) if len(dims) > 4 else 32.0
    for what, t in dict(rho=rho, drho=drho, drho_out=drho_out).items():
        _expect(t, (m, m), what)
    for what, t in dict(chat=chat, dchat=dchat, dchat_out=dchat_out).items():
        _expect(t, (J, n, n), what)
    _expect(c, (J, m, m), "c")
    _expect(P, (n, n), "P")
    d = nlinv_dims(n, m, J, a, l)
    check(load().nlinv_normal_noalloc(C.byref(d), _c64(rho, "rho"), _c64(chat, "chat"), _c64(c, "c"),
                                      _f32(P, "P"), float(alpha), _c64(drho, "drho"), _c64(dchat, "dchat"),
                                      _c64(drho_out, "drho_out"), _c64(dchat_out, "dchat_out"),
                                      _stream(stream)), "nlinv_normal_noalloc")


def nlinv_mask_gradient(plan, rho, chat, c, g, gP_out, stream=None):
    _op_shapes(plan, rho=rho, chat=chat, c=c, g=g, gP_out=gP_out)
    check(load().nlinv_mask_gradient(plan, _c64(rho, "rho"), _c64(chat, "chat"), _c64(c, "c"),
                                     _c64(g, "g"), _f32(gP_out, "gP_out"), _stream(stream)),
          "nlinv_mask_gradient")


def nlinv_image(plan, rho, c, image_out, stream=None):
    _op_shapes(plan, rho=rho, c=c, image_out=image_out)
    check(load().nlinv_image(plan, _c64(rho, "rho"), _c64(c, "c"), _c64(image_out, "image_out"),
                             _stream(stream)), "nlinv_image")


def make_params(newton_steps=7, cg_iters=10, alpha0=1.0, alpha_q=0.5, alpha_min=0.0, scale_norm=100.0,
                flags=0):
    return nlinv_irgnm_params(int(newton_steps), int(cg_iters), float(alpha0), float(alpha_q),
                              float(alpha_min), float(scale_norm), int(flags))


def nlinv_irgnm_solve(plan, y, P, prm, rho_inout, chat_inout, rho_ref=None, chat_ref=None, image_out=None,
                      stats_out=None, stream=None):
    import torch
    dims = _plan_dims(plan)
    if len(dims) != 1:
        raise ValueError("nlinv_irgnm_solve: the plan holds more than one frame (use the batch call)")
    _frame_shapes(dims[0], dict(y=y, P=P, rho=rho_inout, chat=chat_inout, rho_ref=rho_ref, chat_ref=chat_ref,
                                image=image_out, stats=stats_out), prm, "nlinv_irgnm_solve")
    check(load().nlinv_irgnm_solve(plan, _c64(y, "y"), _f32(P, "P"), C.byref(prm),
                                   _c64(rho_inout, "rho_inout"), _c64(chat_inout, "chat_inout"),
                                   _c64(rho_ref, "rho_ref"), _c64(chat_ref, "chat_ref"),
                                   _c64(image_out, "image_out"), _ptr(stats_out, torch.float64, "stats_out"),
                                   _stream(stream)), "nlinv_irgnm_solve")


def _frames(frames):
    import torch
    arr = (nlinv_frame * len(frames))()
    for i, f in enumerate(frames):
        arr[i] = nlinv_frame(_c64(f["y"], "y"), _f32(f["P"], "P"), _c64(f["rho"], "rho"),
                             _c64(f["chat"], "chat"), _c64(f.get("rho_ref"), "rho_ref"),
                             _c64(f.get("chat_ref"), "chat_ref"), _c64(f.get("image"), "image"),
                             _ptr(f.get("stats"), torch.float64, "stats"))
    return arr


def nlinv_irgnm_solve_batch(plan, frames, prm, stream=None):
    dims = _plan_dims(plan)
    if len(frames) != len(dims):
        raise ValueError(f"nlinv_irgnm_solve_batch: {len(frames)} frame descriptors for a plan of "
                         f"{len(dims)} frames")
    for i, (fd, f) in enumerate(zip(dims, frames)):
        _frame_shapes(fd, f, prm, f"nlinv_irgnm_solve_batch frame {i}")
    arr = _frames(frames)
    check(load().nlinv_irgnm_solve_batch(plan, arr, C.byref(prm), _stream(stream)), "nlinv_irgnm_solve_batch")


def nlinv_irgnm_solve_series(plan, frames, prm, stream=None):
    dims = _plan_dims(plan)
    if len(dims) != 1:
        raise ValueError("nlinv_irgnm_solve_series: the plan must hold one frame shape")
    for i, f in enumerate(frames):
        _frame_shapes(dims[0], f, prm, f"nlinv_irgnm_solve_series frame {i}")
    arr = _frames(frames)
    check(load().nlinv_irgnm_solve_series(plan, len(frames), arr, C.byref(prm), _stream(stream)),
          "nlinv_irgnm_solve_series")


def nlinv_plan_autotune(plan, stream=None):
    check(load().nlinv_plan_autotune(plan, _stream(stream)), "nlinv_plan_autotune")


def nlinv_plan_variant(plan, n):
    cv, rv = C.c_int32(), C.c_int32()
    check(load().nlinv_plan_variant(plan, int(n), C.byref(cv), C.byref(rv)), "nlinv_plan_variant")
    return cv.value, rv.value


def nlinv_plan_band(plan, n):
    """(kb, kb_lo): the band of k-space the solves keep of the sensitivities."""
    kb, lo = C.c_int32(), C.c_int32()
    check(load().nlinv_plan_band(plan, int(n), C.byref(kb), C.byref(lo)), "nlinv_plan_band")
    return kb.value, lo.value


def nlinv_plan_normal_form(plan, n):
    f = C.c_int32()
    check(load().nlinv_plan_normal_form(plan, int(n), C.byref(f)), "nlinv_plan_normal_form")
    return f.value


def nlinv_plan_set_normal_form(plan, n, form):
    check(load().nlinv_plan_set_normal_form(plan, int(n), int(form)), "nlinv_plan_set_normal_form")


def nlinv_plan_cg_form(plan, n):
    f = C.c_int32()
    check(load().nlinv_plan_cg_form(plan, int(n), C.byref(f)), "nlinv_plan_cg_form")
    return f.value


def nlinv_plan_set_cg_form(plan, n, form):
    check(load().nlinv_plan_set_cg_form(plan, int(n), int(form)), "nlinv_plan_set_cg_form")


def nlinv_plan_streaming(plan, n):
    f = C.c_int32()
    check(load().nlinv_plan_streaming(plan, int(n), C.byref(f)), "nlinv_plan_streaming")
    return f.value


def nlinv_plan_set_streaming(plan, n, on):
    check(load().nlinv_plan_set_streaming(plan, int(n), int(on)), "nlinv_plan_set_streaming")


def nlinv_plan_set_variant(plan, n, col_variant, row_variant):
    check(load().nlinv_plan_set_variant(plan, int(n), int(col_variant), int(row_variant)),
          "nlinv_plan_set_variant")


def nlinv_kernel_class_names():
    lib = load()
    out = []
    k = 0
    while True:
        s = lib.nlinv_kernel_class_name(k)
        if s is None:
            return out
        out.append(s.decode())
        k += 1


def nlinv_plan_timing_enable(plan, kclass, enable=True):
    """enable: True / 1 brackets every launch of the class, an int k >= 1
    every k-th, False / 0 turns the brackets off."""
    if isinstance(kclass, str):
        kclass = nlinv_kernel_class_names().index(kclass)
    k = (1 if enable else 0) if isinstance(enable, bool) else int(enable)
    check(load().nlinv_plan_timing_enable(plan, int(kclass), k), "nlinv_plan_timing_enable")


def nlinv_plan_timing_read(plan):
    n, ms = C.c_int32(), C.c_double()
    check(load().nlinv_plan_timing_read(plan, C.byref(n), C.byref(ms)), "nlinv_plan_timing_read")
    return n.value, ms.value


def nlinv_plan_timing_read_class(plan, kclass):
    if isinstance(kclass, str):
        kclass = nlinv_kernel_class_names().index(kclass)
    n, ms = C.c_int32(), C.c_double()
    check(load().nlinv_plan_timing_read_class(plan, int(kclass), C.byref(n), C.byref(ms)),
          "nlinv_plan_timing_read_class")
    return n.value, ms.value


def nlinv_bandwidth_probe(src, dst, nbytes=None, stream=None):
    nbytes = src.numel() * src.element_size() if nbytes is None else int(nbytes)
    check(load().nlinv_bandwidth_probe(_ptr(src, None, "src"), _ptr(dst, None, "dst"), nbytes, _stream(stream)),
          "nlinv_bandwidth_probe")


def nlinv_grid_radial(n, angles, data, width, beta, dcf=None, grid_out=None, stream=None):
    """data [J, S, R] complex64, angles [S] float32 (radians), dcf [R] float32
    or None -> grid [J, n, n] complex64 (allocated when grid_out is None)."""
    import torch
    if data.dim() != 3:
        raise ValueError(f"data: expected [J, S, R], got shape {tuple(data.shape)}")
    J, S, R = data.shape
    _expect(angles, (S,), "angles")
    _expect(dcf, (R,), "dcf")
    if grid_out is None:
        grid_out = torch.empty((J, n, n), dtype=torch.complex64, device=data.device)
    _expect(grid_out, (J, n, n), "grid_out")
    check(load().nlinv_grid_radial(int(n), J, S, R, _f32(angles, "angles"), _f32(dcf, "dcf"), float(width),
                                   float(beta), _c64(data, "data"), _c64(grid_out, "grid_out"), _stream(stream)),
          "nlinv_grid_radial")
    return grid_out


def nlinv_degrid_radial(grid, angles, R, width, beta, dcf=None, data_out=None, stream=None):
    """grid [J, n, n] complex64 -> samples [J, S, R] complex64."""
    import torch
    if grid.dim() != 3 or grid.shape[1] != grid.shape[2]:
        raise ValueError(f"grid: expected [J, n, n], got shape {tuple(grid.shape)}")
    J, n = grid.shape[0], grid.shape[1]
    S = angles.shape[0]
    _expect(dcf, (R,), "dcf")
    if data_out is None:
        data_out = torch.empty((J, S, R), dtype=torch.complex64, device=grid.device)
    _expect(data_out, (J, S, R), "data_out")
    check(load().nlinv_degrid_radial(int(n), J, S, int(R), _f32(angles, "angles"), _f32(dcf, "dcf"), float(width),
                                     float(beta), _c64(grid, "grid"), _c64(data_out, "data_out"), _stream(stream)),
          "nlinv_degrid_radial")
    return data_out


def nlinv_coil_compress(y, K, stream=None):
    """y [J, ...] complex64 (each channel's samples) -> (y' [K, ...] complex64,
    eigenvalues [J] float64 descending, basis [J, K] complex64); the
    workspace is allocated here with torch (the caller side of the ABI)."""
    import torch
    J = y.shape[0]
    M = y.numel() // J
    ws_bytes = load().nlinv_coil_compress_workspace(int(J), int(M))
    if ws_bytes == 0:
        raise ValueError(f"nlinv_coil_compress: unsupported J = {J} or M = {M}")
    ws = torch.empty(ws_bytes, dtype=torch.uint8, device=y.device)
    out = torch.empty((int(K),) + tuple(y.shape[1:]), dtype=torch.complex64, device=y.device)
    lam = torch.empty(J, dtype=torch.float64, device=y.device)
    V = torch.empty((J, int(K)), dtype=torch.complex64, device=y.device)
    check(load().nlinv_coil_compress(int(J), int(M), int(K), _c64(y, "y"), _c64(out, "y_out"),
                                     _ptr(lam, torch.float64, "eigvals"), _c64(V, "basis"), ws.data_ptr(), ws_bytes,
                                     _stream(stream)), "nlinv_coil_compress")
    return out, lam, V


def nlinv_gn_step_vjp(plan, rho_n, chat_n, y, P, alpha, rho_next, chat_next, rho_ref, chat_ref, g_rho, g_chat,
                      cg_iters, want_y=True, want_ref=True, want_P=True, want_alpha=True, want_x_n=False,
                      stream=None):
    """Gradients of a loss of x_{n+1} = GN step(x_n; y, P, alpha, x_ref) given
    g = dL/dx_{n+1}: dict with 'y', 'rho_ref', 'chat_ref', 'P', 'alpha',
    'rho_n', 'chat_n' (the requested ones; the workspace allocated here with
    torch)."""
    import torch
    _op_shapes(plan, rho=rho_n, chat=chat_n, y=y, P=P, rho_next=rho_next, chat_next=chat_next, rho_ref=rho_ref,
               chat_ref=chat_ref, rho_g=g_rho, chat_g=g_chat)
    lib = load()
    dev = y.device
    ws_bytes = lib.nlinv_gn_step_vjp_workspace(plan)
    ws = torch.empty(ws_bytes, dtype=torch.uint8, device=dev)
    out = {}
    if want_y:
        out["y"] = torch.empty_like(y)
    if want_ref:
        out["rho_ref"], out["chat_ref"] = torch.empty_like(rho_ref), torch.empty_like(chat_ref)
    if want_P:
        out["P"] = torch.empty_like(P)
    if want_alpha:
        out["alpha"] = torch.zeros((), dtype=torch.float64, device=dev)
    if want_x_n:
        out["rho_n"], out["chat_n"] = torch.empty_like(rho_n), torch.empty_like(chat_n)
    check(lib.nlinv_gn_step_vjp(plan, _c64(rho_n, "rho_n"), _c64(chat_n, "chat_n"), _c64(y, "y"), _f32(P, "P"),
                                float(alpha), _c64(rho_next, "rho_next"), _c64(chat_next, "chat_next"),
                                _c64(rho_ref, "rho_ref"), _c64(chat_ref, "chat_ref"), _c64(g_rho, "g_rho"),
                                _c64(g_chat, "g_chat"), int(cg_iters), _c64(out.get("y"), "grad_y"),
                                _c64(out.get("rho_ref"), "grad_rho_ref"), _c64(out.get("chat_ref"), "grad_chat_ref"),
                                _f32(out.get("P"), "grad_P"), _ptr(out.get("alpha"), torch.float64, "grad_alpha"),
                                _c64(out.get("rho_n"), "grad_rho_n"), _c64(out.get("chat_n"), "grad_chat_n"),
                                ws.data_ptr(), ws_bytes, _stream(stream)), "nlinv_gn_step_vjp")
    return out


def nlinv_check_launch_args(n, n_om, ncoils, nframes=1, newton=2, cg=3, drop_mode=-1, lib=None):
    """(status, launches checked, kernel class of the first incomplete launch or -1)."""
    lib = lib or load()
    cnt, bad = C.c_int64(), C.c_int32()
    st = lib.nlinv_check_launch_args(int(n), int(n_om), int(ncoils), int(nframes), int(newton), int(cg),
                                     int(drop_mode), C.byref(cnt), C.byref(bad))
    return st, cnt.value, bad.value

