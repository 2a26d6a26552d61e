"""Torch-facing convenience layer over the C ABI.

`Plan` owns an nlinv_plan and allocates output tensors with torch (the
caller side of the ABI); every computation is one call of libnlinv.so.
"""
from __future__ import annotations

from dataclasses import dataclass

from . import _native as N


@dataclass(frozen=True)
class FrameDims:
    n: int
    n_om: int
    ncoils: int
    sobolev_a: float = 220.0
    sobolev_l: float = 32.0


class Plan:
    """Workspace for one frame shape, or for a batch of frames of uneven shapes.

    branch_frames > 0: frames of one shape are grouped in runs of at most
    that many, each group a concurrent branch of the solve (bitwise the same
    results, more frames/s on a batch)."""

    def __init__(self, n=None, n_om=None, ncoils=None, sobolev_a=220.0, sobolev_l=32.0, frames=None,
                 branch_frames=0):
        import torch
        if frames is None:
            frames = [FrameDims(n, n_om, ncoils, sobolev_a, sobolev_l)]
        self.frames = [f if isinstance(f, FrameDims) else FrameDims(*f) for f in frames]
        self.device = torch.device("cuda", torch.cuda.current_device())
        self.handle = N.nlinv_plan_create([(f.n, f.n_om, f.ncoils, f.sobolev_a, f.sobolev_l)
                                           for f in self.frames], branch_frames=branch_frames)

    # -- lifetime ----------------------------------------------------------
    def close(self):
        if getattr(self, "handle", None) is not None:
            N.nlinv_plan_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    # -- shapes --------------------------------------------------------------
    @property
    def dims(self) -> FrameDims:
        return self.frames[0]

    def _empty(self, *shape, dtype=None):
        import torch
        return torch.empty(shape, dtype=dtype or torch.complex64, device=self.device)

    # -- operators (frame 0's shape) --------------------------------------------
    def coil_maps(self, chat):
        d = self.dims
        c = self._empty(d.ncoils, d.n_om, d.n_om)
        N.nlinv_coil_maps(self.handle, chat, c)
        return c

    def forward(self, rho, chat, P, return_c=False):
        d = self.dims
        y = self._empty(d.ncoils, d.n, d.n)
        c = self._empty(d.ncoils, d.n_om, d.n_om) if return_c else None
        N.nlinv_forward(self.handle, rho, chat, P, y, c)
        return (y, c) if return_c else y

    def deriv(self, rho, chat, P, drho, dchat, c=None):
        d = self.dims
        dy = self._empty(d.ncoils, d.n, d.n)
        N.nlinv_deriv(self.handle, rho, chat, c, P, drho, dchat, dy)
        return dy

    def adjoint(self, rho, chat, P, dy, c=None):
        d = self.dims
        drho = self._empty(d.n_om, d.n_om)
        dchat = self._empty(d.ncoils, d.n, d.n)
        N.nlinv_adjoint(self.handle, rho, chat, c, P, dy, drho, dchat)
        return drho, dchat

    def normal(self, rho, chat, P, alpha, drho, dchat, c=None):
        d = self.dims
        orho = self._empty(d.n_om, d.n_om)
        ochat = self._empty(d.ncoils, d.n, d.n)
        N.nlinv_normal(self.handle, rho, chat, c, P, alpha, drho, dchat, orho, ochat)
        return orho, ochat

    def mask_gradient(self, rho, chat, g, c=None):
        import torch
        d = self.dims
        gP = self._empty(d.n, d.n, dtype=torch.float32)
        N.nlinv_mask_gradient(self.handle, rho, chat, c, g, gP)
        return gP

    def image(self, rho, c):
        d = self.dims
        img = self._empty(d.n_om, d.n_om)
        N.nlinv_image(self.handle, rho, c, img)
        return img

    # -- solves ------------------------------------------------------------------
    @staticmethod
    def params(newton_steps=7, cg_iters=10, alpha0=1.0, alpha_q=0.5, alpha_min=0.0, scale_norm=100.0,
               use_graph=False, warm_start=False):
        flags = (N.NLINV_USE_GRAPH if use_graph else 0) | (N.NLINV_WARM_START if warm_start else 0)
        return N.make_params(newton_steps, cg_iters, alpha0, alpha_q, alpha_min, scale_norm, flags)

    def _frame_out(self, fd: FrameDims, prm, rho0=None, chat0=None):
        import torch
        rho = rho0.clone() if rho0 is not None else self._empty(fd.n_om, fd.n_om)
        chat = chat0.clone() if chat0 is not None else self._empty(fd.ncoils, fd.n, fd.n)
        return dict(rho=rho, chat=chat, image=self._empty(fd.n_om, fd.n_om),
                    stats=torch.zeros(N.stats_len(prm.newton_steps, prm.cg_iters), dtype=torch.float64,
                                      device=self.device))

    def solve(self, y, P, prm, rho0=None, chat0=None, rho_ref=None, chat_ref=None):
        out = self._frame_out(self.dims, prm, rho0, chat0)
        N.nlinv_irgnm_solve(self.handle, y, P, prm, out["rho"], out["chat"], rho_ref, chat_ref, out["image"],
                            out["stats"])
        return out

    def solve_batch(self, data, prm, outs=None):
        """data: list of (y, P) per plan frame.  Returns one dict per frame."""
        if len(data) != len(self.frames):
            raise ValueError(f"solve_batch: {len(data)} (y, P) pairs for a plan of {len(self.frames)} frames")
        if outs is None:
            outs = [self._frame_out(fd, prm) for fd in self.frames]
        if len(outs) != len(data):
            raise ValueError(f"solve_batch: {len(outs)} outputs for {len(data)} frames")
        frames = [dict(y=y, P=P, **o) for (y, P), o in zip(data, outs)]
        N.nlinv_irgnm_solve_batch(self.handle, frames, prm)
        return outs

    def solve_series(self, data, prm, outs=None):
        """data: list of (y, P) frames of frame 0's shape, solved in order."""
        if outs is None:
            outs = [self._frame_out(self.dims, prm) for _ in data]
        if len(outs) != len(data):
            raise ValueError(f"solve_series: {len(outs)} outputs for {len(data)} frames")
        frames = [dict(y=y, P=P, **o) for (y, P), o in zip(data, outs)]
        N.nlinv_irgnm_solve_series(self.handle, frames, prm)
        return outs

    # -- tuning and timing -----------------------------------------------------------
    def autotune(self):
        N.nlinv_plan_autotune(self.handle)

    def variant(self, n):
        return N.nlinv_plan_variant(self.handle, n)

    def band(self, n=None):
        """(kb, kb_lo): rows and columns [kb_lo, kb_lo + kb) of k-space the
        solves keep of the sensitivities of grid size n (default frame 0's)."""
        return N.nlinv_plan_band(self.handle, self.dims.n if n is None else n)

    def set_variant(self, n, col_variant, row_variant):
        N.nlinv_plan_set_variant(self.handle, n, col_variant, row_variant)

    def normal_form(self, n=None):
        """0: nlinv_normal runs the axis passes; 1: the whole-plane kernel."""
        return N.nlinv_plan_normal_form(self.handle, self.dims.n if n is None else n)

    def set_normal_form(self, form, n=None):
        N.nlinv_plan_set_normal_form(self.handle, self.dims.n if n is None else n, form)

    def cg_form(self, n=None):
        """0: the solves' CG iteration is the five fused passes; 1: the two
        whole-plane launches."""
        return N.nlinv_plan_cg_form(self.handle, self.dims.n if n is None else n)

    def set_cg_form(self, form, n=None):
        N.nlinv_plan_set_cg_form(self.handle, self.dims.n if n is None else n, form)

    def streaming(self, n=None):
        """1: the passes access the intermediates T and T2 non-temporally."""
        return N.nlinv_plan_streaming(self.handle, self.dims.n if n is None else n)

    def set_streaming(self, on, n=None):
        N.nlinv_plan_set_streaming(self.handle, self.dims.n if n is None else n, 1 if on else 0)

    def timing_enable(self, kclass, enable=True):
        N.nlinv_plan_timing_enable(self.handle, kclass, enable)

    def timing_read(self, kclass=None):
        """(bracketed launches, total ms): of every class, or of one class."""
        if kclass is None:
            return N.nlinv_plan_timing_read(self.handle)
        return N.nlinv_plan_timing_read_class(self.handle, kclass)
