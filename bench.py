"""Benchmark of the IRGNM hot path on one MI355X.

Default workload (the largest single-GPU configuration): the temporal series,
512x512 grid (2x oversampled, Omega = central 256x256), 32 coils, 13 radial
spokes per frame rotating by the golden angle, ellipses moving sinusoidally,
noise sigma 1e-3, 7 Newton steps x 10 CG iterations per frame, each frame
warm-started from and regularised towards the previous frame's result.  One
step = 8 consecutive frames solved in order by one series call: all frames
enqueued without host synchronisation, each frame's Newton loop replayed from
a captured hipGraph (inputs resident in HBM).  value = frames/s of the job.

The line also carries:
  roofline      the CG iteration (five pass kernels) against the HBM
                roofline: compulsory bytes per iteration and frame (B_cg)
                over the sum of the five kernels' average durations, all
                measured live with HIP events on every 7th launch of each
                class inside the timed graph replays;
  cpu_baseline  the FP64 oracle on a bounded sample (2 of 7 Newton steps of
                frame 0) on the host cores, scaled to frames/s;
  nrmse_vs_oracle  the GPU image of that same 2-Newton-step solve of frame 0
                against the oracle's;
  plain_*       the plain path: one eager solve call per frame, the
                warm-start chain driven from the host;
  other_workloads  frames/s of the 64-frame ragged batch and of 4 batched
                384x384 12-coil frames.
"""
from __future__ import annotations

import argparse
import glob
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBPS = 8000.0
NEWTON, CG = 7, 10
# Every 7th launch of a timed kernel class is bracketed with HIP events (an
# event record holds the stream about a microsecond); 7 is coprime with the 10
# CG iterations of a Newton step, so the brackets cycle through every
# iteration index.
TIMING_STRIDE = 7
# the five kernel classes of one CG iteration (q = N_alpha p with p = r + beta p
# in the first and r -= a q, x += a p in the last)
CG_CLASSES = ("col_pupd_winv_ifft", "row_deriv", "col_psf", "row_adj", "col_fft_winv_cg_update")
MAX_WORKERS = 16   # host threads for the oracle's FFTs (at most one GPU's share of a 16-threads-per-GPU host)

WORKLOADS = {
    # name: (n, n_om, J, description)
    "series_512": (512, 256, 32, "series_512: 512x512 grid, Omega 256x256, 32 coils, 13 golden-angle radial "
                                 "spokes per frame, moving phantom, 7 Newton x 10 CG per frame, each frame "
                                 "warm-started from the previous; 8 sequential frames per step"),
    "realtime_384": (384, 192, 12, "realtime_384: 384x384 grid, Omega 192x192, 12 coils, 15 radial spokes, "
                                   "7 Newton x 10 CG; independent frames batched"),
}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


# ---------------------------------------------------------------------------
# byte models
# ---------------------------------------------------------------------------

def normal_bytes(n, m, J, kb=None):
    """B_normal: compulsory bytes of one (DF^H DF + alpha) apply on one frame:
    read h (its sensitivity part and its image part), the linearisation point
    (c on Omega, rho) and P; write N h.  complex64 = 8 B, P float32 = 4 B.
    The sensitivity part counts the kb x kb band of k-space the solve keeps
    (kb = n: every component, the dense count)."""
    N_, NO, K = n * n, m * m, (kb or n) ** 2
    return 8 * (J * K + NO) + 8 * (J * NO + NO) + 4 * N_ + 8 * (J * K + NO)


def cg_bytes(n, m, J, kb=None):
    """B_cg = B_normal + 7 V: one CG iteration with the apply fused with the
    vector updates (read r, q / write r; read x, p, r / write x, p; the read
    of p shared with the apply), V = 8 (J kb^2 + m^2) bytes per vector."""
    V = 8 * (J * (kb or n) ** 2 + m * m)
    return normal_bytes(n, m, J, kb) + 7 * V


def fft_flops(n, m, J, kb):
    """Line-FFT work of one CG iteration on one frame, 5 L log2 L flops per
    transform of length L = n: the first column pass transforms the kb band
    columns, each row pass 2 transforms of the m Omega rows, the PSF column
    pass 2 transforms of all n columns, the last column pass the kb band
    columns; per coil plane."""
    import math
    t = 5.0 * n * math.log2(n)
    return J * t * (kb + 2 * m + 2 * n + 2 * m + kb)


def schedule_bytes(kc: str, n: int, m: int, planes: int, frames: int, kb: int) -> float:
    """Bytes one launch of pass class `kc` moves in the build's pass schedule
    inside a solve (its operands and results, the intermediates between the
    two axes included: T [m][n], and [m][kb] on the band side), for `planes`
    coil planes of `frames` frames, with the sensitivity vectors on the
    kb x kb band; the 1/w table (shared by every plane, L2-resident) is not
    counted."""
    c, mn, mm, nn, mk, kk = 8.0, float(m * n), float(m * m), float(n * n), float(m * kb), float(kb * kb)
    per = {
        "col_winv_ifft": planes * c * (kk + mk),
        "col_pupd_winv_ifft": planes * c * (3 * kk + mk) + frames * 3 * c * mm,   # read r, p; write p, T
        "col_p_ifft": planes * c * (nn + mn) + frames * 4 * nn,
        "col_fft_p": planes * c * (mn + nn) + frames * 4 * nn,
        "col_resid_p_ifft": planes * c * (2 * mn + nn) + frames * 4 * nn,
        "col_psf": planes * c * (2 * mn) + frames * 4 * nn,
        "col_fft_winv_add": planes * c * (mk + 3 * kk),
        # read T, p, r, x (chat) and the coil products; write r, x; rho parts: read p, r, dx; write r, dx
        "col_fft_winv_cg_update": planes * c * (mk + 5 * kk + mm) + frames * 5 * c * mm,
        "row_cache": planes * c * (mk + mm),
        "row_fwd": planes * c * (mm + mn) + frames * c * mm,
        "row_deriv": planes * c * (mk + mn + mm) + frames * 2 * c * mm,
        "row_adj": planes * c * (mn + mk + 2 * mm) + frames * c * mm,
        "coil_sum": planes * c * mm + frames * 3 * c * mm,
        "vec_dot": (planes * nn + frames * mm) * 2 * c,
    }
    return per.get(kc, float("nan"))


def kernel_source_hash():
    csrc = os.path.join(ROOT, "paper_1301_1215_amd", "csrc")
    h = hashlib.sha256()
    for pth in sorted(glob.glob(os.path.join(csrc, "*.hpp")) + glob.glob(os.path.join(csrc, "*.hip"))):
        h.update(open(pth, "rb").read())
    return h.hexdigest()


def pmc_traffic(workload: str):
    """HBM bytes per launch of each kernel class from the committed
    FETCH_SIZE / WRITE_SIZE summary of this workload, or None when the kernel
    sources changed since the counters were taken."""
    path = os.path.join(ROOT, "profiles", f"pmc_traffic__{workload}.txt")
    if not os.path.exists(path):
        return None
    meta, traffic = {}, {}
    for line in open(path):
        f = line.split()
        if not f or f[0].startswith("#"):
            continue
        if f[0] == "traffic" and len(f) == 7:
            # one line per kernel variant; the solve's is the one with the most
            # dispatches (others are the autotuner's trial launches)
            if f[1] not in traffic or int(f[3]) > traffic[f[1]][0]:
                traffic[f[1]] = (int(f[3]), int(f[6]))
        elif len(f) == 2:
            meta[f[0]] = f[1]
    if meta.get("source_sha256") != kernel_source_hash():
        return None
    return {k: v[1] for k, v in traffic.items()}


# ---------------------------------------------------------------------------
# host side: the oracle baseline
# ---------------------------------------------------------------------------

def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    import platform
    return platform.processor() or "unknown"


def cpu_baseline(frame, newton_sample: int):
    """The FP64 oracle on `newton_sample` Newton steps (x10 CG) of `frame`,
    scaled to frames/s of the full 7 x 10 solve; returns (record, image)."""
    from oracle import nlinv_oracle as O
    workers = min(os.cpu_count() or 1, MAX_WORKERS)
    O.set_workers(workers)
    d = O.Dims(frame.n, frame.n_om, frame.ncoils)
    t0 = time.perf_counter()
    res = O.irgnm(frame.y, frame.P, d, O.IRGNMParams(newton_steps=newton_sample, cg_iters=CG))
    dt = time.perf_counter() - t0
    per_frame = dt * NEWTON / newton_sample
    rec = {"value": 1.0 / per_frame, "unit": "frames/s", "cores": workers, "kind": "oracle",
           "sample": f"{newton_sample} of {NEWTON} Newton steps (x{CG} CG) of frame 0 "
                     f"({frame.n}x{frame.n}, {frame.ncoils} coils), FP64 numpy with scipy.fft on {workers} "
                     f"worker threads (elementwise work on 1); {dt:.1f} s measured, scaled to a frame",
           "cpu_model": cpu_model(), "host_cores": os.cpu_count()}
    return rec, res.image


def stream_probe(nbytes=1 << 30, reps=20):
    """Read + write GB/s of the library's streaming copy kernel over `nbytes`."""
    import torch
    from paper_1301_1215_amd import _native as NAT
    src = torch.empty(nbytes // 4, dtype=torch.float32, device="cuda").fill_(1.0)
    dst = torch.empty_like(src)
    for _ in range(3):
        NAT.nlinv_bandwidth_probe(src, dst, nbytes)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        NAT.nlinv_bandwidth_probe(src, dst, nbytes)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    del src, dst
    return 2 * nbytes / (ms * 1e-3) / 1e9


# ---------------------------------------------------------------------------
# GPU measurements
# ---------------------------------------------------------------------------

def class_totals(pl, run, names):
    """Summed duration and launch count of every kernel class in one step
    (every launch bracketed)."""
    import torch
    for k in names:
        pl.timing_enable(k, True)
    run()
    torch.cuda.synchronize()
    totals = {}
    for k in names:
        cnt, ms = pl.timing_read(k)
        if cnt:
            totals[k] = (ms, cnt)
    for k in names:
        pl.timing_enable(k, False)
    log("bench: kernel-class totals per step (ms, launches): " +
        ", ".join(f"{k}={v[0]:.3f}/{v[1]}" for k, v in sorted(totals.items(), key=lambda kv: -kv[1][0])))
    return totals


def timed_steps(pl, run, steps, classes):
    """Time `steps` calls of run() with every TIMING_STRIDE-th launch of each
    class in `classes` bracketed; returns (seconds, {class: (launches, ms)})."""
    import torch
    for k in classes:
        pl.timing_enable(k, TIMING_STRIDE)
    run()                      # captures the graphs with the brackets
    torch.cuda.synchronize()
    for k in classes:
        pl.timing_read(k)      # discard
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        run()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    # graph-owned brackets hold the latest replay of each captured graph
    per = {k: pl.timing_read(k) for k in classes}
    for k in classes:
        pl.timing_enable(k, False)
    return dt, per


def roofline_record(workload, n, m, J, kb, frames_per_launch, iter_ms, per, traffic):
    """The CG iteration against the HBM roofline: B_cg (with the sensitivity
    vectors on the kb x kb band the solve keeps) x frames per launch over the
    average duration of one CG iteration (its five launches, bracketed as one
    inside the timed graph replays); the per-class averages (from brackets of
    each launch, in a separate run) are the breakdown."""
    avg = {k: (ms / cnt if cnt else float("nan")) for k, (cnt, ms) in per.items()}
    sum_ms = iter_ms
    B = cg_bytes(n, m, J, kb) * frames_per_launch
    B_dense = cg_bytes(n, m, J) * frames_per_launch
    sched = {k: schedule_bytes(k, n, m, J * frames_per_launch, frames_per_launch, kb) for k in CG_CLASSES}
    achieved = B / (sum_ms * 1e-3) / 1e9
    flops = fft_flops(n, m, J, kb) * frames_per_launch
    rec = {"bound": "hbm",
           "kernel": "CG iteration = " + " + ".join(CG_CLASSES),
           "achieved": achieved, "peak": HBM_PEAK_GBPS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBPS,
           "traffic": None,
           "algorithmic_bytes_per_launch": B,
           "algorithmic_bytes_note": f"B_cg = B_normal + 7V per frame x {frames_per_launch} frame(s) per launch, "
                                     f"sensitivity vectors on the {kb}x{kb} band of the {n}x{n} grid that the "
                                     f"solve keeps (1/w > 2^-40 inside)",
           "band": kb,
           "dense_chat_bytes_per_launch": B_dense,
           "dense_chat_GBps": B_dense / (sum_ms * 1e-3) / 1e9,
           "fft_flops_per_launch": flops,
           "fft_TFLOPs": flops / (sum_ms * 1e-3) / 1e12,
           "cg_iteration_ms": iter_ms,
           "avg_launch_ms": {k: avg[k] for k in CG_CLASSES},
           "sum_avg_launch_ms": sum(avg[k] for k in CG_CLASSES),
           "launches_timed": {k: per[k][0] for k in CG_CLASSES},
           "schedule_bytes_per_launch": {k: sched[k] for k in CG_CLASSES},
           "schedule_GBps": sum(sched.values()) / (sum_ms * 1e-3) / 1e9,
           "timing_stride": TIMING_STRIDE, "event_timing_on": "graph",
           "timing_note": "achieved uses cg_iteration_ms (every 7th CG iteration bracketed whole in the timed "
                          "replays); avg_launch_ms brackets each launch of the five classes in a separate run "
                          "(each bracket adds a few microseconds of dispatch)"}
    if traffic and all(k in traffic for k in CG_CLASSES):
        rec["traffic"] = sum(traffic[k] for k in CG_CLASSES)
        rec["traffic_per_kernel"] = {k: traffic[k] for k in CG_CLASSES}
        rec["traffic_GBps"] = rec["traffic"] / (sum_ms * 1e-3) / 1e9
    rec["normal_applies_per_s"] = frames_per_launch / (sum_ms * 1e-3)
    rec["normal_algorithmic_GBps"] = normal_bytes(n, m, J) * frames_per_launch / (sum_ms * 1e-3) / 1e9
    return rec


def series_bench(a, NAT, torch):
    from paper_1301_1215_amd import Plan, synth
    n, m, J, desc = WORKLOADS["series_512"]
    F = a.frames or 8
    log(f"bench: generating {F} frames of the {n}x{n}, {J}-coil series")
    ph = synth.temporal_phantom()
    frames = [synth.temporal_frame(t, ph) for t in range(F)]
    data = [(torch.from_numpy(f.y).cuda(), torch.from_numpy(f.P).cuda()) for f in frames]
    prm = Plan.params(NEWTON, CG, use_graph=True)
    pl = Plan(n, m, J)
    if not a.no_autotune:
        os.environ.setdefault("NLINV_TUNE_VERBOSE", "1")
        pl.autotune()
    outs = [pl._frame_out(pl.dims, prm) for _ in range(F)]
    run = lambda: pl.solve_series(data, prm, outs)
    for _ in range(max(1, a.warmup)):
        run()
    torch.cuda.synchronize()
    names = [k for k in NAT.nlinv_kernel_class_names() if k != "cg_iteration"]
    totals = class_totals(pl, run, names)
    log(f"bench: timing {a.steps} steps of {F} sequential frames")
    dt, it = timed_steps(pl, run, a.steps, ("cg_iteration",))
    ms_step = 1e3 * dt / a.steps
    fps = F * a.steps / dt
    log(f"bench: {ms_step:.2f} ms/step, {fps:.2f} frames/s")
    _, per = timed_steps(pl, run, 1, CG_CLASSES)
    iter_ms = it["cg_iteration"][1] / it["cg_iteration"][0]
    roof = roofline_record("series_512", n, m, J, pl.band()[0], 1, iter_ms, per, pmc_traffic("series_512"))
    extras = {"kernel_class_ms_per_step": {k: v[0] for k, v in totals.items()}}
    img_last = outs[-1]["image"].clone()

    # plain path: one eager solve call per frame, warm start driven from the host
    if not a.no_compare:
        pprm0 = Plan.params(NEWTON, CG, use_graph=False)
        pprm = Plan.params(NEWTON, CG, use_graph=False, warm_start=True)

        def plain():
            prev = None
            for y, P in data:
                if prev is None:
                    prev = pl.solve(y, P, pprm0)
                else:
                    prev = pl.solve(y, P, pprm, rho0=prev["rho"], chat0=prev["chat"], rho_ref=prev["rho"],
                                    chat_ref=prev["chat"])
            return prev
        plain()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        last = plain()
        torch.cuda.synchronize()
        pdt = time.perf_counter() - t0
        extras["plain_frames_per_s"] = F / pdt
        extras["plain_path"] = "one eager solve call per frame (no graph), warm start chained from the host"
        extras["series_vs_plain_last_image_rel"] = float(
            (last["image"] - img_last).abs().pow(2).sum().sqrt() / img_last.abs().pow(2).sum().sqrt())

    # FP64 oracle sample and the GPU solve of the same sample
    cpu, nrmse = None, None
    if a.cpu_newton > 0:
        cpu, ref_img = cpu_baseline(frames[0], a.cpu_newton)
        g = pl.solve(data[0][0], data[0][1], Plan.params(a.cpu_newton, CG, use_graph=True))
        gi = g["image"].cpu().numpy()
        import numpy as np
        nrmse = float(np.linalg.norm(gi - ref_img) / np.linalg.norm(ref_img))
        extras["nrmse_vs_oracle"] = nrmse
        extras["nrmse_sample"] = (f"image of frame 0 after {a.cpu_newton} Newton steps x {CG} CG, GPU (graph) "
                                  f"vs the FP64 oracle's cpu_baseline solve")
    pl.close()
    del outs, data
    torch.cuda.empty_cache()
    return dict(value=fps, ms_per_step=ms_step, workload=desc, frames_per_step=F, path="series+hipGraph",
                roofline=roof, cpu=cpu, extras=extras)


def realtime_bench(a, NAT, torch, steps=None, quiet=False):
    """Independent 384x384 12-coil frames batched in one graph-replayed solve."""
    from paper_1301_1215_amd import Plan, synth
    n, m, J, desc = WORKLOADS["realtime_384"]
    F = a.frames or 4
    frames = [synth.make_frame(2, t, n, m, J, "radial", spokes=15, mask_frame=t + 1) for t in range(F)]
    data = [(torch.from_numpy(f.y).cuda(), torch.from_numpy(f.P).cuda()) for f in frames]
    prm = Plan.params(NEWTON, CG, use_graph=True)
    pl = Plan(frames=[(n, m, J)] * F)
    if not a.no_autotune:
        pl.autotune()
    outs = [pl._frame_out(pl.frames[i], prm) for i in range(F)]
    run = lambda: pl.solve_batch(data, prm, outs)
    for _ in range(max(1, a.warmup)):
        run()
    torch.cuda.synchronize()
    dt, it = timed_steps(pl, run, steps or a.steps, ("cg_iteration",))
    k = steps or a.steps
    _, per = timed_steps(pl, run, 1, CG_CLASSES)
    roof = roofline_record("realtime_384", n, m, J, pl.band()[0], F, it["cg_iteration"][1] / it["cg_iteration"][0],
                           per, None)
    pl.close()
    del outs, data
    torch.cuda.empty_cache()
    return dict(value=F * k / dt, ms_per_step=1e3 * dt / k, workload=desc + f"; {F} frames per step",
                frames_per_step=F, path="batched+hipGraph", roofline=roof, cpu=None, extras={})


def ragged_bench(a, torch, steps):
    from paper_1301_1215_amd import Plan, synth
    frames = synth.ragged_batch(64)
    data = [(torch.from_numpy(f.y).cuda(), torch.from_numpy(f.P).cuda()) for f in frames]
    prm = Plan.params(NEWTON, CG, use_graph=True)
    pl = Plan(frames=[(f.n, f.n_om, f.ncoils) for f in frames])
    if not a.no_autotune:
        pl.autotune()
    outs = [pl._frame_out(fd, prm) for fd in pl.frames]
    run = lambda: pl.solve_batch(data, prm, outs)
    run()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        run()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    pl.close()
    del outs, data
    torch.cuda.empty_cache()
    return {"frames_per_s": 64 * steps / dt, "ms_per_step": 1e3 * dt / steps,
            "workload": "ragged_64: 64 independent frames, n in {128,192,256,384} (Omega half), J in "
                        "{8,12,16,32}, spokes in {11,15,21}, 7 Newton x 10 CG, one batched graph-replayed solve"}


def single_64_bench(a, torch, steps=20, applies=200):
    """The single 64 x 64 frame (8 coils, Cartesian, 6 Newton x 10 CG): frames/s
    of a graph-replayed solve with each CG form (the five fused passes, the two
    whole-plane launches) and nlinv_normal applies/s with each normal form."""
    from paper_1301_1215_amd import Plan, synth
    fr = synth.single_frame_64()
    y, P = torch.from_numpy(fr.y).cuda(), torch.from_numpy(fr.P).cuda()
    prm = Plan.params(6, 10, use_graph=True)
    rec = {"workload": "single_64: 64x64 grid, Omega = grid, 8 coils, Cartesian 16 central + 25% outer lines, "
                       "6 Newton x 10 CG, one frame per graph-replayed solve"}
    with Plan(64, 64, 8) as pl:
        if not a.no_autotune:
            pl.autotune()
        rec["cg_form_chosen"], rec["normal_form_chosen"] = pl.cg_form(), pl.normal_form()
        outs = [pl._frame_out(pl.dims, prm)]
        for form, name in ((0, "axis_passes"), (1, "whole_plane")):
            pl.set_cg_form(form)
            for _ in range(2):
                pl.solve_batch([(y, P)], prm, outs)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(steps):
                pl.solve_batch([(y, P)], prm, outs)
            torch.cuda.synchronize()
            rec[f"frames_per_s_{name}"] = steps / (time.perf_counter() - t0)
        rho, chat = outs[0]["rho"], outs[0]["chat"]
        c = pl.coil_maps(chat)   # the linearisation's cache, as inside a solve
        for form, name in ((0, "axis_passes"), (1, "whole_plane")):
            pl.set_normal_form(form)
            pl.normal(rho, chat, P, 0.5, rho, chat, c=c)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(applies):
                pl.normal(rho, chat, P, 0.5, rho, chat, c=c)
            torch.cuda.synchronize()
            rec[f"normal_applies_per_s_{name}"] = applies / (time.perf_counter() - t0)
    return rec


# ---------------------------------------------------------------------------
# profile summaries (host only): rocprofv3 CSV output -> profiles/*.{md,txt}
# ---------------------------------------------------------------------------

COL_MODE_CLASS = ("col_winv_ifft", "col_p_ifft", "col_fft_p", "col_resid_p_ifft", "col_psf", "col_fft_winv_add",
                  "col_fft_gprod", "col_pupd_winv_ifft", "col_fft_winv_cg_update")
ROW_MODE_CLASS = ("row_cache", "row_fwd", "row_deriv", "row_adj")


def kernel_class_of(name: str):
    """(class, n) of a pass kernel's demangled name, e.g.
    'void nlinv::k_col<512, 8, 4, true, true>(nlinv::ColArgs)' -> ('col_psf', 512)."""
    import re
    m = re.search(r"k_(col|row)<(\d+), (\d+), (\d+)", name)
    if m:
        table = COL_MODE_CLASS if m.group(1) == "col" else ROW_MODE_CLASS
        return table[int(m.group(4))], int(m.group(2))
    for key, kc in (("k_coil_sum", "coil_sum"), ("k_vec<0>", "vec_dot"), ("k_image", "image"),
                    ("k_stream_copy", "stream_copy")):
        if key in name:
            return kc, 0
    return None, 0


def summarize_trace(prof_dir: str, line_json: str, out_md: str, command: str):
    import csv
    rows = list(csv.DictReader(open(os.path.join(prof_dir, "bench_kernel_stats.csv"))))
    line = json.loads(open(line_json).read().strip().splitlines()[-1])
    roof = line["roofline"]
    n = WORKLOADS["series_512"][0] if "series_512" in line["config"]["workload"] else 384
    out = ["# Kernel trace: " + line["config"]["workload"], "", "Command (repo root, MI355X, ROCm 7.2):", "",
           "    " + command, "",
           "Kernel statistics (`bench_kernel_stats.csv`, top 16 by total time; durations in microseconds).",
           "The command also runs the warm-up, the per-class totals, the autotuner, the plain path, the",
           "oracle sample's GPU solve and the other workloads, so the call counts cover all of them.", "",
           "| kernel | calls | avg us | min us | max us | % time |", "|---|---|---|---|---|---|"]
    for r in rows[:16]:
        out.append(f"| `{r['Name'][:100]}` | {r['Calls']} | {float(r['AverageNs']) / 1e3:.2f} | "
                   f"{float(r['MinNs']) / 1e3:.2f} | {float(r['MaxNs']) / 1e3:.2f} | {float(r['Percentage']):.2f} |")
    out += ["", f"bench.py line printed by the same command: value {line['value']:.1f} frames/s, "
                f"{line['ms_per_step']:.2f} ms/step.", "",
            "The CG iteration's five kernel classes: HIP-event average inside the timed graph replays (the",
            "bench line) against the trace's average of the same kernel (the variant with the most calls):", "",
            "| class | events us | trace us | trace kernel |", "|---|---|---|---|"]
    best = {}
    for r in rows:
        kc, kn = kernel_class_of(r["Name"])
        if kc in CG_CLASSES and kn == n and (kc not in best or int(r["Calls"]) > int(best[kc]["Calls"])):
            best[kc] = r
    tsum = 0.0
    for kc in CG_CLASSES:
        ev = 1e3 * roof["avg_launch_ms"][kc]
        tr = float(best[kc]["AverageNs"]) / 1e3 if kc in best else float("nan")
        tsum += tr
        out.append(f"| {kc} | {ev:.2f} | {tr:.2f} | `{best[kc]['Name'][:60] if kc in best else '-'}` |")
    B = roof["algorithmic_bytes_per_launch"]
    it = 1e3 * roof["cg_iteration_ms"]
    out += ["", f"Sum of the five: per-launch events {1e3 * roof['sum_avg_launch_ms']:.1f} us, trace {tsum:.1f} us; "
                f"one whole CG iteration bracketed as one (the roofline's duration): {it:.1f} us (the trace's sum "
                f"plus the four gaps between the launches).",
            f"Algorithmic bytes per CG iteration (B_cg on the {roof.get('band')}-wide band): {B / 1e6:.1f} MB "
            f"-> {B / (it * 1e-6) / 1e9:.0f} GB/s on the iteration = {B / (it * 1e-6) / 1e12 / 8:.3f} of 8 TB/s "
            f"({B / (tsum * 1e-6) / 1e9:.0f} GB/s on the trace's sum)."]
    open(out_md, "w").write("\n".join(out) + "\n")
    print(out_md)


def summarize_pmc(fetch_dir: str, write_dir: str, out_txt: str, workload: str, commands):
    """Average FETCH_SIZE / WRITE_SIZE (KiB) per dispatch of every kernel, the
    calibration factors from the 1 GiB bandwidth-probe copy, and HBM-side
    traffic per launch of each kernel class."""
    import csv
    from collections import defaultdict

    def load(d, counter):
        acc = defaultdict(lambda: [0, 0.0])
        for r in csv.DictReader(open(os.path.join(d, "run_counter_collection.csv"))):
            if r["Counter_Name"] != counter:
                continue
            k = (r["Kernel_Name"], int(r["Grid_Size"]))
            acc[k][0] += 1
            acc[k][1] += float(r["Counter_Value"])
        return {k: (v[0], v[1] / v[0]) for k, v in acc.items()}
    fe, wr = load(fetch_dir, "FETCH_SIZE"), load(write_dir, "WRITE_SIZE")
    probe = [(k, v) for k, v in fe.items() if "k_stream_copy" in k[0]]
    probe_w = [(k, v) for k, v in wr.items() if "k_stream_copy" in k[0]]
    kib = float(1 << 20)            # the probe copies 1 GiB each way
    ff = kib / probe[0][1][1] if probe else 1.0
    wf = kib / probe_w[0][1][1] if probe_w else 1.0
    lines = [f"# HBM-side traffic per launch from FETCH_SIZE / WRITE_SIZE -- {workload}",
             "# Two counter runs (repo root, MI355X, ROCm 7.2):"] + ["#   " + c for c in commands] + [
             "# Counters are KiB per dispatch averaged over the dispatches of one kernel and grid size; they count",
             "# what leaves the L2s (the 256 MB Infinity Cache sits behind them, in front of HBM).",
             f"# Calibration: the 1 GiB bandwidth-probe copy reads FETCH {probe[0][1][1] if probe else 0:.1f} KiB "
             f"(factor {ff:.4f}) and WRITE {probe_w[0][1][1] if probe_w else 0:.1f} KiB (factor {wf:.4f}).",
             "# traffic_bytes = (FETCH x fetch_factor + WRITE x write_factor) x 1024",
             "# traffic  class  kernel  dispatches  fetch_KiB  write_KiB  traffic_bytes",
             f"source_sha256 {kernel_source_hash()}", f"fetch_factor {ff:.6f}", f"write_factor {wf:.6f}"]
    recs = []
    for (name, grid), (cnt, fkib) in fe.items():
        kc, _ = kernel_class_of(name)
        if kc is None or (name, grid) not in wr:
            continue
        wkib = wr[(name, grid)][1]
        short = name.replace("void nlinv::", "").split("(")[0].replace(" ", "")
        recs.append((kc, short, cnt, fkib, wkib, int((fkib * ff + wkib * wf) * 1024)))
    recs.sort(key=lambda r: -r[2] * r[5])
    for kc, short, cnt, fkib, wkib, tb in recs:
        lines.append(f"traffic {kc} {short} {cnt} {fkib:.1f} {wkib:.1f} {tb}")
    open(out_txt, "w").write("\n".join(lines) + "\n")
    print(out_txt)


def summarize_sq(dir_a: str, dir_b: str, out_txt: str, workload: str, commands):
    """Per-wave instruction counts and wait / VALU-issue shares of the
    workload's grid-size passes from two SQ counter runs (dir_a: SQ_WAVES,
    SQ_WAVE_CYCLES, SQ_INSTS_VALU, SQ_INSTS_LDS, SQ_ACTIVE_INST_VALU,
    SQ_LDS_BANK_CONFLICT; dir_b: SQ_WAIT_ANY, SQ_INSTS_VMEM), averaged over
    the dispatches of each kernel."""
    import csv
    from collections import defaultdict

    def load(d):
        acc, disp = defaultdict(lambda: defaultdict(float)), defaultdict(set)
        for r in csv.DictReader(open(os.path.join(d, "run_counter_collection.csv"))):
            acc[r["Kernel_Name"]][r["Counter_Name"]] += float(r["Counter_Value"])
            disp[r["Kernel_Name"]].add(r["Dispatch_Id"])
        return {k: {c: v / len(disp[k]) for c, v in cs.items()} for k, cs in acc.items()}, disp
    a, da = load(dir_a)
    b, _ = load(dir_b)
    n = WORKLOADS[workload][0]
    lines = [f"# SQ counters of the {n}x{n} passes -- {workload}",
             "# Commands (repo root, MI355X, ROCm 7.2; the first run autotunes and saves the pass variants):"] + [
             "#   " + c for c in commands] + [
             "# Per dispatch, averaged over the dispatches of each kernel (counter values summed over the chip):",
             "#   VALU, LDS, VMEM = SQ_INSTS_VALU, SQ_INSTS_LDS, SQ_INSTS_VMEM per wave (SQ_WAVES);",
             "#   wait = SQ_WAIT_ANY / SQ_WAVE_CYCLES (share of the waves' resident cycles spent waiting on anything);",
             "#   valu_busy = SQ_ACTIVE_INST_VALU / SQ_WAVE_CYCLES (share of those cycles issuing VALU work);",
             "#   bank = SQ_LDS_BANK_CONFLICT per dispatch.",
             "# class  kernel  dispatches  waves  VALU  LDS  VMEM  wait  valu_busy  bank"]
    recs = []
    for name, A in a.items():
        kc, _ = kernel_class_of(name)
        if kc is None or f"<{n}," not in name.replace(" ", "") or not A.get("SQ_WAVES"):
            continue
        B = b.get(name, {})
        w, cyc = A["SQ_WAVES"], max(A.get("SQ_WAVE_CYCLES", 0.0), 1.0)
        short = name.replace("void nlinv::", "").split("(")[0].replace(" ", "")
        recs.append((len(da[name]), f"{kc}  {short}  {len(da[name])}  {w:.0f}  {A.get('SQ_INSTS_VALU', 0) / w:.0f}  "
                     f"{A.get('SQ_INSTS_LDS', 0) / w:.0f}  {B.get('SQ_INSTS_VMEM', 0) / w:.0f}  "
                     f"{B.get('SQ_WAIT_ANY', 0) / cyc:.3f}  {A.get('SQ_ACTIVE_INST_VALU', 0) / cyc:.3f}  "
                     f"{A.get('SQ_LDS_BANK_CONFLICT', 0):.0f}"))
    recs.sort(key=lambda r: -r[0])
    lines += [r[1] for r in recs]
    open(out_txt, "w").write("\n".join(lines) + "\n")
    print(out_txt)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=8)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="series_512", choices=["series_512", "realtime_384"],
                    help="series_512 (the benchmark line) or realtime_384 (independent frames batched)")
    ap.add_argument("--frames", type=int, default=0, help="frames per step (default 8 series / 4 batched)")
    ap.add_argument("--cpu-newton", type=int, default=2, help="Newton steps of the CPU oracle sample (0: skip)")
    ap.add_argument("--no-compare", action="store_true", help="skip the plain-path comparison")
    ap.add_argument("--no-other", action="store_true", help="skip the other workloads' frames/s")
    ap.add_argument("--no-autotune", action="store_true", help="keep the default pass variants")
    ap.add_argument("--stream-probe", action="store_true",
                    help="also measure a 1 GiB device-to-device copy with the library's probe kernel")
    ap.add_argument("--summarize-trace", nargs=3, metavar=("PROF_DIR", "LINE_JSON", "OUT_MD"),
                    help="write a kernel-trace summary (no GPU needed) and exit")
    ap.add_argument("--summarize-pmc", nargs=3, metavar=("FETCH_DIR", "WRITE_DIR", "OUT_TXT"),
                    help="write a FETCH_SIZE / WRITE_SIZE traffic summary (no GPU needed) and exit")
    ap.add_argument("--summarize-sq", nargs=3, metavar=("DIR_A", "DIR_B", "OUT_TXT"),
                    help="write an SQ counter summary (no GPU needed) and exit")
    ap.add_argument("--command", action="append", default=[], help="command lines to record in a summary")
    a = ap.parse_args()

    if a.summarize_trace:
        summarize_trace(*a.summarize_trace, command=" ".join(a.command) or "python3 bench.py")
        return
    if a.summarize_pmc:
        summarize_pmc(*a.summarize_pmc, workload=a.workload, commands=a.command)
        return
    if a.summarize_sq:
        summarize_sq(*a.summarize_sq, workload=a.workload, commands=a.command)
        return

    if a.gpus != 1:
        print(f"bench.py: the benchmark runs on one GPU; --gpus {a.gpus} is not supported (how the path "
              f"would shard across GPUs is a design, not built)", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1301_1215_amd import _native as NAT

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    NAT.load()
    if a.workload == "series_512":
        r = series_bench(a, NAT, torch)
    else:
        r = realtime_bench(a, NAT, torch)
    extras = r["extras"]
    if not a.no_other and a.workload == "series_512":
        log("bench: other workloads (frames/s only)")
        other = {"ragged_64": ragged_bench(a, torch, 2)}
        rt = realtime_bench(a, NAT, torch, steps=5)
        other["realtime_384_x4"] = {"frames_per_s": rt["value"], "ms_per_step": rt["ms_per_step"],
                                    "workload": rt["workload"], "cg_iteration_frac": rt["roofline"]["frac"]}
        other["single_64"] = single_64_bench(a, torch)
        extras["other_workloads"] = other
    if a.stream_probe:
        extras["stream_copy_GBps"] = stream_probe()
    out = {
        "metric": "IRGNM frames/sec and DF^H.DF applies/sec (HBM GB/s) at <=1e-3 NRMSE vs FP64",
        "value": r["value"], "unit": "frames/s", "n_gpus": 1, "steps": a.steps, "warmup": a.warmup,
        "ms_per_step": r["ms_per_step"], "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "c64 (fp32), fp64 CG dots/scalars", "data": "synthetic",
        "config": {"workload": r["workload"], "frames_per_step": r["frames_per_step"], "path": r["path"]},
        **extras,
        "roofline": r["roofline"],
        "cpu_baseline": r["cpu"],
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
