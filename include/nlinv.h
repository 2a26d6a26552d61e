/*
 * nlinv.h -- C ABI of the MI355X (gfx950) library for nonlinear-inverse MRI
 * reconstruction: the iteratively regularised Gauss-Newton method (IRGNM)
 * that estimates an image and the coil sensitivities together
 * (Schaetz & Uecker, Sec. 3.1, Eqs. 2-3).
 *
 * Model (Eq. 2).  For an unknown x = (rho, chat):
 *   F(x)_j = P . DTFT( E( rho . c_j ) ),   c_j = E^H W^{-1} chat_j,
 *   W^{-1} chat = DTFT^{-1}( chat / w ),   w(k) = (1 + a |k|^2)^(l/2),
 * where DTFT is the centred unitary 2D DFT on the n x n grid (DC at index
 * n/2, k_d = (kappa_d - n/2)/n), E zero-pads an n_om x n_om image into the
 * centre of the grid (the mask M_Omega of Eq. 2) and E^H crops it, and P is
 * the real k-space sampling array (the projection P_k; binary for measured /
 * not measured, or a soft weight).
 *
 * Conventions shared by every call:
 *   - Array arguments are DEVICE pointers to C-contiguous data owned by the
 *     caller; they must stay valid until `stream` has executed the call.
 *     nlinv_c32 has the layout of std::complex<float> / torch.complex64.
 *     Pointers must be 16-byte aligned.
 *   - Shapes: rho-like arrays [n_om][n_om]; chat-like and k-space arrays
 *     [J][n][n]; sensitivities c [J][n_om][n_om]; P [n][n] float32.
 *   - `stream` is a hipStream_t (NULL = the null stream).  Every compute call
 *     only enqueues work and returns; kernel faults surface at the caller's
 *     next synchronisation.  Compute calls never allocate device memory.
 *   - Return value: NLINV_OK (0) or a negative status.  NLINV_EINVAL for a
 *     NULL / misaligned pointer or bad argument, NLINV_EUNSUPPORTED for a
 *     grid size outside {8, 12, 16, 24, 32, 48, 64, 96, 128, 192, 256, 384,
 *     512, 768, 1024} (2^p and 3 * 2^p), Omega sides that are odd or larger
 *     than n, or more than 64 coils, NLINV_ENOMEM when plan creation cannot allocate,
 *     NLINV_EHIP for a HIP error (its code: nlinv_last_hip_error()).
 *     No C++ exception crosses this interface.
 *   - Outputs must not alias inputs except where a name ends in _inout.
 *   - A plan is not thread-safe; separate plans are independent.
 */
#ifndef NLINV_H
#define NLINV_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct { float re, im; } nlinv_c32;

typedef struct nlinv_plan_s* nlinv_plan;

/* Geometry of one frame.  sobolev_a = 220 and sobolev_l = 32 give the
 * weight (1 + 220 |k|^2)^16 on the coil sensitivities. */
typedef struct {
    int32_t n;          /* grid side (square grid): 2^p or 3 * 2^p, 8 <= n <= 1024 */
    int32_t n_om;       /* side of the centred image region Omega, even, <= n */
    int32_t ncoils;     /* J, 1..64 */
    float sobolev_a;
    float sobolev_l;
} nlinv_dims;

/* Gauss-Newton parameters (Eq. 3).  alpha_n = max(alpha0 * alpha_q^n, alpha_min),
 * n = 0..newton_steps-1; each step runs cg_iters conjugate-gradient iterations
 * from 0 (stopping early only when <r,r> = 0 or Re<p, N p> <= 0).
 * scale_norm > 0 scales the data to ||y|| = scale_norm before the solve and
 * undoes it on rho afterwards (exact: F is bilinear); 0 turns it off. */
typedef struct {
    int32_t newton_steps;
    int32_t cg_iters;
    float alpha0;
    float alpha_q;
    float alpha_min;
    float scale_norm;
    uint32_t flags;     /* NLINV_* flags below */
} nlinv_irgnm_params;

enum {
    NLINV_OK = 0,
    NLINV_EINVAL = -1,
    NLINV_EUNSUPPORTED = -2,
    NLINV_ENOMEM = -3,
    NLINV_EHIP = -4,
    NLINV_ESCRATCH = -5     /* nlinv_normal_noalloc: the frame needs more than its static scratch */
};

enum {
    NLINV_USE_GRAPH = 1u,   /* replay the solve from a captured hipGraph */
    NLINV_WARM_START = 2u   /* rho/chat hold the start x0 (data units); else rho = 1, chat = 0 */
};

/* Stats written per frame (device doubles), when a stats pointer is given:
 *   [0] data scale s, [1] flags (bit 0: CG breakdown in some step,
 *   bit 1: non-finite scalar met), [2 .. 2+N) ||y_s - F(x_n)|| per Newton
 *   step (scaled units), then N*K values <r,r> after each CG iteration
 *   (-1 where an iteration was skipped after a breakdown). */
#define NLINV_STATS_LEN(newton, cg) (2 + (newton) + (newton) * (cg))

/* One frame of a batched or serial solve (all pointers on the device). */
typedef struct {
    const nlinv_c32* y;         /* [J][n][n] measured k-space data */
    const float* P;             /* [n][n] sampling array */
    nlinv_c32* rho;             /* [n_om][n_om] out (in: x0 with NLINV_WARM_START) */
    nlinv_c32* chat;            /* [J][n][n]    out (in: x0 with NLINV_WARM_START) */
    const nlinv_c32* rho_ref;   /* nullable: x_ref (data units); NULL -> x_ref = x0 */
    const nlinv_c32* chat_ref;
    nlinv_c32* image;           /* nullable [n_om][n_om]: rho . sqrt(sum_j |c_j|^2) */
    double* stats;              /* nullable, NLINV_STATS_LEN doubles */
} nlinv_frame;

/* ---- plans --------------------------------------------------------------
 * A plan holds the workspace for `nframes` frames of the given shapes
 * (dims[0..nframes-1]; frames may differ in n, n_om and J).  It allocates all
 * device memory here, on the current HIP device; compute calls allocate none.
 * The single-frame operators and nlinv_irgnm_solve act on frame 0's shape. */
int nlinv_plan_create(nlinv_plan* out, const nlinv_dims* dims, int32_t nframes);
/* As nlinv_plan_create, but frames of one shape are grouped in runs of at
 * most `branch_frames` (<= 0: no limit, the same as nlinv_plan_create).  Each
 * group runs its Newton loop as a concurrent branch (on a default-priority
 * stream of the plan, forked from and joined into the caller's stream or
 * graph), so
 * groups overlap each other's memory- and VALU-bound passes: more frames/s
 * on a batch, while every kernel shares the GPU with the other branches.
 * At most 8 streams are used; groups beyond that share them in turn.
 * Results are bitwise those of nlinv_plan_create. */
int nlinv_plan_create_branched(nlinv_plan* out, const nlinv_dims* dims, int32_t nframes, int32_t branch_frames);
int nlinv_plan_destroy(nlinv_plan plan);                  /* NULL-safe */

/* c_j = E^H W^{-1} chat_j (Eq. 2: the weighted inverse transform of the
 * sensitivities, restricted to Omega): the linearisation cache that the
 * method computes once per Newton step.  c_out [J][n_om][n_om]. */
int nlinv_coil_maps(nlinv_plan plan, const nlinv_c32* chat, nlinv_c32* c_out, void* stream);

/* y = F(rho, chat) (Eq. 2).  y_out [J][n][n]; c_out (nullable) receives c. */
int nlinv_forward(nlinv_plan plan, const nlinv_c32* rho, const nlinv_c32* chat,
                  const float* P, nlinv_c32* y_out, nlinv_c32* c_out, void* stream);

/* dy = DF_x (drho, dchat): the Frechet derivative of F at x = (rho, chat)
 * (left factor of Eq. 3), dy_j = P . DTFT(E(drho . c_j + rho . E^H W^{-1} dchat_j)).
 * c = nlinv_coil_maps(chat); if c is NULL it is recomputed from chat. */
int nlinv_deriv(nlinv_plan plan, const nlinv_c32* rho, const nlinv_c32* chat,
                const nlinv_c32* c, const float* P, const nlinv_c32* drho,
                const nlinv_c32* dchat, nlinv_c32* dy_out, void* stream);

/* (drho, dchat) = DF_x^H dy (Eq. 3): u_j = E^H DTFT^{-1}(P . dy_j),
 * drho = sum_j conj(c_j) . u_j,  dchat_j = DTFT(E(conj(rho) . u_j)) / w. */
int nlinv_adjoint(nlinv_plan plan, const nlinv_c32* rho, const nlinv_c32* chat,
                  const nlinv_c32* c, const float* P, const nlinv_c32* dy,
                  nlinv_c32* drho_out, nlinv_c32* dchat_out, void* stream);

/* (DF_x^H DF_x + alpha I) h, the left-hand side of Eq. 3 (P enters squared). */
int nlinv_normal(nlinv_plan plan, const nlinv_c32* rho, const nlinv_c32* chat,
                 const nlinv_c32* c, const float* P, float alpha,
                 const nlinv_c32* drho, const nlinv_c32* dchat,
                 nlinv_c32* drho_out, nlinv_c32* dchat_out, void* stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the normal
 * operator of nlinv_normal for one frame of shape *dims, without a plan.  It
 * allocates nothing: its workspace is a static device array of
 * NLINV_NOALLOC_SCRATCH_BYTES per GPU (held until the process ends), which
 * must hold the twiddles (8 n B), the inverse weight table (4 n^2 B), the
 * coil products (8 J n_om^2 B), the pass intermediate (8 J n_om n B) and,
 * when c is NULL, the sensitivities (8 J n_om^2 B), each rounded up to
 * 256 B; larger frames are refused with NLINV_ESCRATCH before anything is
 * enqueued (512 x 512, n_om 256, 32 coils fits; every smaller shape does).
 * Arguments, layouts and the result are those of nlinv_normal (default pass
 * variants).  Every call on a GPU reuses that GPU's array and rebuilds what it
 * needs in it, so calls that overlap on one GPU (other streams or threads)
 * race and give wrong results; serialise them. */
#define NLINV_NOALLOC_SCRATCH_BYTES ((size_t)80 << 20)
int nlinv_normal_noalloc(const nlinv_dims* dims, const nlinv_c32* rho, const nlinv_c32* chat,
                         const nlinv_c32* c, const float* P, float alpha,
                         const nlinv_c32* drho, const nlinv_c32* dchat,
                         nlinv_c32* drho_out, nlinv_c32* dchat_out, void* stream);

/* Gradient with respect to P of a loss of y = F(x; P), given
 * g = dL/dRe(y) + i dL/dIm(y) [J][n][n]:  gP = Re sum_j conj(g_j) . DTFT(E(rho . c_j)).
 * gP_out [n][n] float32. c as in nlinv_deriv. */
int nlinv_mask_gradient(nlinv_plan plan, const nlinv_c32* rho, const nlinv_c32* chat,
                        const nlinv_c32* c, const nlinv_c32* g, float* gP_out, void* stream);

/* image = rho . sqrt(sum_j |c_j|^2) on Omega. */
int nlinv_image(nlinv_plan plan, const nlinv_c32* rho, const nlinv_c32* c,
                nlinv_c32* image_out, void* stream);

/* ---- solves ---------------------------------------------------------------
 * Eq. 3 iterated: x_{n+1} = x_n + dx with dx from cg_iters CG iterations on
 * (DF^H DF + alpha_n I) dx = DF^H (y - F x_n) - alpha_n (x_n - x_ref).
 * One frame of frame 0's shape; rho_inout / chat_inout give x0 when
 * NLINV_WARM_START is set and receive the result.  rho_ref / chat_ref:
 * nullable x_ref (NULL -> x_ref = x0).  image_out, stats_out nullable. */
int nlinv_irgnm_solve(nlinv_plan plan, const nlinv_c32* y, const float* P,
                      const nlinv_irgnm_params* prm, nlinv_c32* rho_inout,
                      nlinv_c32* chat_inout, const nlinv_c32* rho_ref,
                      const nlinv_c32* chat_ref, nlinv_c32* image_out,
                      double* stats_out, void* stream);

/* All nframes frames of the plan solved together (frame f has dims[f]);
 * `frames` is a HOST array of nframes descriptors.  Frames are independent:
 * each has its own data scale, CG scalars and breakdown guard. */
int nlinv_irgnm_solve_batch(nlinv_plan plan, const nlinv_frame* frames,
                            const nlinv_irgnm_params* prm, void* stream);

/* A temporal series (Sec. 3.2): `count` frames of frame 0's shape solved in
 * order; frame 0 starts as in nlinv_irgnm_solve (its rho_ref / chat_ref
 * honoured), frame t > 0 starts from and is regularised towards the result of
 * frame t-1 (x0 = x_ref = x(t-1), in data units).  `frames` is a HOST array;
 * the whole series is enqueued without host synchronisation. */
int nlinv_irgnm_solve_series(nlinv_plan plan, int32_t count, const nlinv_frame* frames,
                             const nlinv_irgnm_params* prm, void* stream);

/* ---- differentiation through a Gauss-Newton step --------------------------
 * The regularised Gauss-Newton step of Eq. 3 as a differentiable map:
 * x_{n+1} = x_n + dx with
 *   (DF^H DF + alpha I) dx = DF^H (y - F x_n) - alpha (x_n - x_ref)
 * (forward: nlinv_irgnm_solve with newton_steps = 1, alpha0 = alpha,
 * scale_norm = 0, NLINV_WARM_START, x0 = x_n, the references x_ref).  Given
 * g = dL/dx_{n+1} (g_rho [n_om][n_om], g_chat [J][n][n]; complex gradients
 * as dL/dRe + i dL/dIm), with lambda = (DF^H DF + alpha I)^{-1} g solved by
 * cg_iters CG iterations of the same solver:
 *   grad_y        = DF lambda                                  [J][n][n]
 *   grad_*_ref    = alpha lambda                               (both or neither)
 *   grad_alpha    = -Re<lambda, x_{n+1} - x_ref>               (one device double)
 *   grad_P        = Re sum_j conj(u_j) (y_j - 2 P w_j)         [n][n] float32
 *                   u = A lambda, w = A (x_{n+1} - x_n / 2), A = DF at x_n with P = 1
 * (F is bilinear, so F(x_n) + A dx = A (x_{n+1} - x_n / 2)), and for the
 * linearisation point itself (both or neither)
 *   grad_*_n      = DF_lambda^H (y - DF (x_{n+1} - x_n / 2)) - DF_dx^H (DF lambda)
 * where DF is the derivative at x_n, DF_v the derivative at the point v, and
 * dx = x_{n+1} - x_n (F bilinear: DF_h k = DF_k h;
 * the normal equations' N lambda = g cancel the direct terms), so that an
 * N-step solve can be differentiated step by step from its stored iterates.
 * rho_next, chat_next: the forward's result.  Every output is nullable.  The caller
 * provides `workspace` (device, 16-byte aligned) of at least
 * nlinv_gn_step_vjp_workspace(plan) bytes.  Plans of one frame only. */
size_t nlinv_gn_step_vjp_workspace(nlinv_plan plan);
int nlinv_gn_step_vjp(nlinv_plan plan, const nlinv_c32* rho_n, const nlinv_c32* chat_n, const nlinv_c32* y,
                      const float* P, float alpha, const nlinv_c32* rho_next, const nlinv_c32* chat_next,
                      const nlinv_c32* rho_ref, const nlinv_c32* chat_ref, const nlinv_c32* g_rho,
                      const nlinv_c32* g_chat, int32_t cg_iters, nlinv_c32* grad_y, nlinv_c32* grad_rho_ref,
                      nlinv_c32* grad_chat_ref, float* grad_P, double* grad_alpha, nlinv_c32* grad_rho_n,
                      nlinv_c32* grad_chat_n, void* workspace, size_t workspace_bytes, void* stream);

/* ---- autotuning -----------------------------------------------------------
 * Time the FFT pass variants (lines per workgroup) of every pass mode for
 * every shape class of the plan on `stream` (which must not be capturing),
 * and keep the fastest per mode; then refine the five passes of the CG loop
 * by timing whole CG iterations, captured and replayed as a graph as the
 * solves do, one pass mode at a time over all its variants.  It overwrites the
 * plan's workspace, so call it between solves.  It also chooses the form of the normal operator entry
 * point (nlinv_plan_normal_form) and of the solves' CG iteration
 * (nlinv_plan_cg_form).  Results are cached per (device
 * architecture, n, planes) in the text file named by NLINV_TUNE_CACHE, if
 * set; NLINV_TUNE_VERBOSE prints the timings to stderr.  Without this call a
 * fixed default is used. */
int nlinv_plan_autotune(nlinv_plan plan, void* stream);

/* Choice made for grid size n (NLINV_EINVAL if n is not in the plan): the
 * variant index of the PSF column pass and of the derivative row pass of the
 * CG loop. */
int nlinv_plan_variant(nlinv_plan plan, int32_t n, int32_t* col_variant, int32_t* row_variant);

/* Form of the normal operator entry point (nlinv_normal) for grid size n:
 * 0 = the axis passes (the five fused passes of the CG loop), 1 = the
 * whole-plane kernel: one workgroup per coil plane holds the n x n plane in
 * LDS and runs all four centred 2D transforms of DF and DF^H (Eq. 2) there,
 * then a fixed-order coil sum forms the image part; it exists for
 * 8 <= n <= 64.  nlinv_plan_autotune times both and keeps the faster (the
 * default is 0).  NLINV_EINVAL if n is not in the plan. */
int nlinv_plan_normal_form(nlinv_plan plan, int32_t n, int32_t* form);
/* Force the form for grid size n (for tests): NLINV_EINVAL for a form the
 * size does not have or an n not in the plan. */
int nlinv_plan_set_normal_form(nlinv_plan plan, int32_t n, int32_t form);

/* Form of the solves' CG iteration for grid size n: 0 = the five fused axis
 * passes, 1 = two launches (8 <= n <= 64): one workgroup per coil plane
 * updates the direction p = r + beta p and applies the normal operator of
 * Eq. 3 to it with the whole plane in LDS, then an update launch forms the
 * step a = <r, r> / Re<p, N p> and applies r -= a N p, x += a p (the image
 * part through a fixed-order coil sum).  The scalar steps (beta, a,
 * breakdown, statistics, the components outside the band) are the same in
 * both forms.  nlinv_plan_autotune times both (default 0).  NLINV_EINVAL if n
 * is not in the plan. */
int nlinv_plan_cg_form(nlinv_plan plan, int32_t n, int32_t* form);
/* Force the CG form for grid size n (for tests; drops a captured graph):
 * NLINV_EINVAL for a form the size does not have or an n not in the plan. */
int nlinv_plan_set_cg_form(nlinv_plan plan, int32_t n, int32_t form);

/* Access policy of the pass intermediates for grid size n (*on = 0 or 1):
 * with 1, every column and row pass loads its input T or T2 (the previous
 * pass's output, read once) non-temporally, and the column passes store
 * theirs so: they then do not displace the operands every CG iteration
 * re-reads (coil maps, P, 1/w) from the L2, which pays where the
 * intermediates exceed the L2s; where they fit, plain accesses are faster.
 * Results are identical either way.  The plan sets 1 where one intermediate
 * ([planes][m][n] complex) exceeds 30 MiB, just under the eight XCDs' L2s
 * together (32 MB).  NLINV_EINVAL if n is not in the plan. */
int nlinv_plan_streaming(nlinv_plan plan, int32_t n, int32_t* on);
/* Force the policy for grid size n (for tests; drops a captured graph):
 * NLINV_EINVAL for on outside {0, 1} or an n not in the plan. */
int nlinv_plan_set_streaming(nlinv_plan plan, int32_t n, int32_t on);

/* The band of k-space the solves keep of the sensitivities for grid size n:
 * rows and columns [*kb_lo, *kb_lo + *kb).  Outside it every Sobolev weight
 * has 1/w <= 2^-40, so those components of chat reach c = E^H W^{-1} chat
 * only far below single-precision rounding: the solves treat them as
 * untouched by DF (there the normal operator of Eq. 3 is alpha I, which CG
 * follows exactly through a few per-frame scalars) and write them once, at
 * the end.  *kb = n (the whole grid) for small grids, flat weights, or when
 * the environment variable NLINV_FULL_CHAT=1 was set at plan creation.  The
 * operator entry points always act on the whole grid.  NLINV_EINVAL if n is
 * not in the plan. */
int nlinv_plan_band(nlinv_plan plan, int32_t n, int32_t* kb, int32_t* kb_lo);

/* Force one variant on every column / row pass of grid size n (for tests):
 * returns NLINV_EINVAL for an index that is not valid for n.  Column
 * variants 0-3 are 16, 8, 32 and 4 columns per workgroup; row variants 0-3
 * are 8, 16, 4 and 2 rows per workgroup, 4-7 the same with the line FFT's
 * split N = N1 x N2 transposed in the derivative and adjoint row passes of
 * the CG loop (valid where N1 != N2). */
int nlinv_plan_set_variant(nlinv_plan plan, int32_t n, int32_t col_variant, int32_t row_variant);

/* ---- kernel timing --------------------------------------------------------
 * enable = k >= 1: every k-th launch of the kernel class `kclass` (see
 * nlinv_kernel_class_name) made by this plan is bracketed by HIP events on
 * its stream, counting launches from this call and from the start of each
 * graph capture (k = 1: every launch; each bracket costs the stream a few
 * microseconds between kernels).  enable = 0: off; negative: NLINV_EINVAL.
 * nlinv_plan_timing_read synchronises those events and returns the
 * bracketed launch count and the summed duration in milliseconds, then
 * resets. */
int nlinv_plan_timing_enable(nlinv_plan plan, int32_t kclass, int32_t enable);
int nlinv_plan_timing_read(nlinv_plan plan, int32_t* launches, double* total_ms);
/* As nlinv_plan_timing_read, but only the bracketed launches of kernel class
 * `kclass` (-1: every class, the same as nlinv_plan_timing_read); the other
 * classes' brackets are kept for their own reads.  Several classes can be
 * bracketed in one solve and read apart afterwards. */
int nlinv_plan_timing_read_class(nlinv_plan plan, int32_t kclass, int32_t* launches, double* total_ms);
/* Names of the kernel classes, by index; the class "cg_iteration" brackets a
 * whole CG iteration (its five launches) as one. */
const char* nlinv_kernel_class_name(int32_t kclass);   /* NULL past the last */

/* ---- gridding of radial samples -------------------------------------------
 * The step before the reconstruction (Sec. 3.1: the non-Cartesian samples
 * are interpolated to the grid; Sec. 3.2: on a grid doubled for the
 * interpolation's accuracy): convolution gridding with a separable
 * Kaiser-Bessel window, and its adjoint.  Spoke s (angle angles[s], radians)
 * carries R samples at radii r_i = i - floor(R/2) (grid units), at
 * k_si = (n/2 + r_i cos angles[s], n/2 + r_i sin angles[s]) (DC at n/2 along
 * both axes); the window is kb(d0) kb(d1) with
 * kb(d) = I0(beta sqrt(1 - (2d/width)^2)) / I0(beta) for |d| <= width/2, and
 * a window that crosses the grid's edge wraps around.  dcf [R] (nullable:
 * all 1) weights the samples by radius (density compensation).
 *   nlinv_grid_radial:   grid_out[j][u][v] = sum_{s,i} dcf[i] data[j][s][i] window(u, v; k_si)
 *   nlinv_degrid_radial: data_out[j][s][i] = dcf[i] sum_{u,v} window(u, v; k_si) grid[j][u][v]
 * data [J][S][R] and grids [J][n][n] complex; angles [S] and dcf [R] float32;
 * all device pointers (complex arrays 8-byte, float arrays 4-byte aligned).
 * Gridding all-ones data (J = 1) gives the sampling density, the k-space
 * weights P of the reconstruction.  Every output element is written by one
 * thread in a fixed order (deterministic); positions, window membership and
 * the window are evaluated in double precision, the sums in single.
 * NLINV_EINVAL for S outside 1..1024, width outside (0, n), negative beta,
 * NULL or misaligned pointers.  No plan, no allocation. */
int nlinv_grid_radial(int32_t n, int32_t J, int32_t S, int32_t R, const float* angles, const float* dcf,
                      float width, float beta, const nlinv_c32* data, nlinv_c32* grid_out, void* stream);
int nlinv_degrid_radial(int32_t n, int32_t J, int32_t S, int32_t R, const float* angles, const float* dcf,
                        float width, float beta, const nlinv_c32* grid, nlinv_c32* data_out, void* stream);

/* ---- PCA channel compression ---------------------------------------------
 * Sec. 3.2: the receive channels are compressed by a principal component
 * analysis before the reconstruction (32 to 8-12 in the paper).  y [J][M]
 * holds every channel's M samples (e.g. M = n*n k-space grid points; zeros
 * add nothing).  The channel covariance A[i][k] = sum_m y_i[m] conj(y_k[m])
 * (products of the single-precision samples summed in double precision) is
 * decomposed A = V diag(lambda) V^H (cyclic Jacobi in double precision on
 * the GPU), lambda descending, each eigenvector scaled so that its
 * largest-magnitude entry is real and positive (the first on a tie); then
 * y_out[k][m] = sum_j conj(V[j][k]) y[j][m] for the K kept virtual channels.
 * eigvals_out [J] (double) and basis_out [J][K] (complex64, column k the k-th
 * eigenvector) are nullable.  The caller provides `workspace` (device, 16-byte
 * aligned) of at least nlinv_coil_compress_workspace(J, M) bytes (0 for bad
 * J or M); the call allocates nothing.  NLINV_EINVAL for J outside 1..64, K
 * outside 1..J, M < 1, a small workspace, NULL or misaligned pointers. */
size_t nlinv_coil_compress_workspace(int32_t J, int64_t M);
int nlinv_coil_compress(int32_t J, int64_t M, int32_t K, const nlinv_c32* y, nlinv_c32* y_out,
                        double* eigvals_out, nlinv_c32* basis_out, void* workspace, size_t workspace_bytes,
                        void* stream);

/* ---- host-side check of the launch arguments ------------------------------
 * For callers' and the library's tests (no GPU needed, nothing allocated on a
 * device, no HIP call): builds the launch arguments of a solve's whole Newton
 * loop (newton x cg iterations, nframes frames of the shape n, n_om, ncoils
 * with the default weight) and of the autotuner's trial launch of every pass
 * mode, exactly as a solve would, with placeholder device pointers, and
 * checks each launch's operands the way a real launch is checked before it
 * is enqueued.  drop_mode >= 0 plants an omission in the tuner's launch of
 * that column mode (its operands are cleared, as a dropped argument line
 * would leave them).  *launches: the number of launches checked;
 * *first_bad: the kernel class (nlinv_kernel_class_name) of the first
 * launch with a missing operand, or -1.  NLINV_OK when every launch is
 * complete, NLINV_EINVAL otherwise (or for bad arguments). */
int nlinv_check_launch_args(int32_t n, int32_t n_om, int32_t ncoils, int32_t nframes, int32_t newton,
                            int32_t cg, int32_t drop_mode, int64_t* launches, int32_t* first_bad);

/* ---- measurement ----------------------------------------------------------
 * Bandwidth probe: copy `bytes` (a multiple of 16) from src to dst (device,
 * 16-byte aligned, not overlapping) with a plain streaming kernel.  It gives
 * the practical HBM ceiling next to the 8 TB/s specification, and is the
 * copy of known size that calibrates hardware traffic counters. */
int nlinv_bandwidth_probe(const void* src, void* dst, size_t bytes, void* stream);

const char* nlinv_status_string(int status);
int nlinv_last_hip_error(void);

#ifdef __cplusplus
}
#endif

#endif /* NLINV_H */
