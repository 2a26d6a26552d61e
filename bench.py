"""Benchmark of the IRGNM hot path on one MI355X.

Workload (the real-time shape): 384x384 grid (2x oversampled 192x192 FOV,
Omega = central 192x192), 12 coils, 15 golden-angle radial spokes, noise
sigma 1e-3, 7 Newton steps x 10 CG iterations.  One step = one batched,
graph-replayed IRGNM solve of `--frames` independent frames of that shape
(inputs resident in HBM).  value = frames/s of the whole job.

Also measured: the plain path (one frame per solve call, eager launches),
DF^H DF applies/s with their algorithmic GB/s, the average duration of the
dominant kernel class from HIP events over the timed region, and the FP64
CPU oracle on a bounded sample.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBPS = 8000.0
N, N_OM, J, SPOKES, NEWTON, CG = 384, 192, 12, 15, 7, 10
# The timed steps bracket every 7th launch of the roofline's kernel class
# with HIP events (each event record holds the stream a few microseconds);
# 7 is coprime with the 10 CG iterations per Newton step, so the bracketed
# launches cycle through every iteration index.
TIMING_STRIDE = 7


def log(*a):
    print(*a, file=sys.stderr, flush=True)


# algorithmic bytes per launch of each kernel class, for `planes` coil planes
# of `frames` frames (n x n grid, m x m Omega); complex64 = 8 B, P float32 = 4 B
def kernel_bytes(kc: str, n: int, m: int, planes: int, frames: int) -> float:
    c, mn, mm, nn = 8.0, float(m * n), float(m * m), float(n * n)
    # the 1/w table (4 n^2 B per class) is shared by all planes and L2-resident: not counted
    per = {
        "col_winv_ifft": planes * c * (nn + mn),                               # read chat, write T
        "col_pupd_winv_ifft": planes * c * (3 * nn + mn) + frames * 3 * c * mm,  # read r, p; write p, T
        "col_p_ifft": planes * c * (nn + mn) + frames * 4 * nn,
        "col_fft_p": planes * c * (mn + nn) + frames * 4 * nn,
        "col_resid_p_ifft": planes * c * (2 * mn + nn) + frames * 4 * nn,       # read T, y, P; write T
        "col_psf": planes * c * (2 * mn) + frames * 4 * nn,
        "col_fft_winv_add": planes * c * (mn + 3 * nn),                        # read T, x, x_ref; write
        # read T, p, r, x (chat) and the coil products; write r, x; rho parts: read p, r, dx; write r, dx
        "col_fft_winv_cg_update": planes * c * (mn + 5 * nn + mm) + frames * 5 * c * mm,
        "row_cache": planes * c * (mn + mm),
        "row_fwd": planes * c * (mm + mn) + frames * c * mm,
        "row_deriv": planes * c * (2 * mn + mm) + frames * 2 * c * mm,
        "row_adj": planes * c * (2 * mn + 2 * mm) + frames * c * mm,
        "coil_sum": planes * c * mm + frames * 3 * c * mm,                     # right-hand side: read x, x_ref; write
        "vec_dot": (planes * nn + frames * mm) * 2 * c,
    }
    return per.get(kc, float("nan"))


def kernel_source_hash():
    import glob
    import hashlib
    csrc = os.path.join(ROOT, "paper_1301_1215_amd", "csrc")
    h = hashlib.sha256()
    for pth in sorted(glob.glob(os.path.join(csrc, "*.hpp")) + glob.glob(os.path.join(csrc, "*.hip"))):
        h.update(open(pth, "rb").read())
    return h.hexdigest()


def pmc_traffic(kc: str, frames: int):
    """HBM bytes per launch of kernel class `kc` from the committed
    FETCH_SIZE / WRITE_SIZE summary, or None when the kernels changed since
    the counters were taken or the batch differs."""
    path = os.path.join(ROOT, "profiles", "pmc_traffic__realtime_384_b4.txt")
    if not os.path.exists(path):
        return None
    meta, traffic = {}, {}
    for line in open(path):
        f = line.split()
        if not f or f[0].startswith("#"):
            continue
        if f[0] == "traffic" and len(f) == 7:
            # one line per kernel variant; the solve's is the one with the
            # most dispatches (the others are the autotuner's trial launches)
            if f[1] not in traffic or int(f[3]) > traffic[f[1]][0]:
                traffic[f[1]] = (int(f[3]), int(f[6]))
        elif len(f) == 2:
            meta[f[0]] = f[1]
    if meta.get("source_sha256") != kernel_source_hash() or int(meta.get("frames_per_step", -1)) != frames:
        return None
    return traffic[kc][1] if kc in traffic else None


def normal_bytes(n, m, J, frames=1):
    """Compulsory bytes of one (DF^H DF + alpha) apply: read h, c|Omega, rho, P; write N h."""
    N_, NO = n * n, m * m
    return frames * (8 * (J * N_ + NO) + 8 * (J * NO + NO) + 4 * N_ + 8 * (J * N_ + NO))


def cpu_baseline(newton_sample: int):
    """FP64 oracle on `newton_sample` Newton steps of one frame; scaled to frames/s."""
    import numpy as np
    from oracle import nlinv_oracle as O
    from paper_1301_1215_amd import synth
    cores = min(os.cpu_count() or 1, 16)
    O.set_workers(cores)
    fr = synth.realtime_384()
    d = O.Dims(fr.n, fr.n_om, fr.ncoils)
    t0 = time.perf_counter()
    O.irgnm(fr.y, fr.P, d, O.IRGNMParams(newton_steps=newton_sample, cg_iters=CG))
    dt = time.perf_counter() - t0
    per_frame = dt * NEWTON / newton_sample
    return {"value": 1.0 / per_frame, "unit": "frames/s", "cores": cores, "kind": "oracle",
            "sample": f"{newton_sample} of {NEWTON} Newton steps (x{CG} CG) of one 384x384, 12-coil frame, "
                      f"FP64 numpy/scipy.fft with {cores} FFT workers; {dt:.1f} s measured, scaled to a frame"}


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
    return 2 * nbytes / (ms * 1e-3) / 1e9


def dominant_class(pl, data, prm, outs, names):
    """Kernel class with the largest summed duration in one step."""
    import torch
    totals = {}
    for k in names:
        pl.timing_enable(k, True)
        pl.solve_batch(data, prm, outs)
        torch.cuda.synchronize()
        cnt, ms = pl.timing_read()
        pl.timing_enable(k, False)
        if cnt:
            totals[k] = (ms, cnt)
    kc = max(totals, key=lambda k: totals[k][0])
    log("bench: kernel-class totals per step (ms, launches): " +
        ", ".join(f"{k}={v[0]:.3f}/{v[1]}" for k, v in sorted(totals.items(), key=lambda kv: -kv[1][0])))
    dominant_class.totals = totals
    return kc


# kernel classes of one (DF^H DF + alpha) apply inside CG; the first also does
# p = r + beta p, the last r -= a q and x += a p with the rho parts fused in (one CG iteration but its scalars)
APPLY_CLASSES = ("col_pupd_winv_ifft", "row_deriv", "col_psf", "row_adj", "col_fft_winv_cg_update")


def apply_rates(totals, B):
    """N_alpha applies/s and GB/s from the per-class totals of one step:
    algorithmic = compulsory bytes B_normal per frame-apply; schedule = the
    bytes the pass schedule moves (the byte model, which the traffic
    counters reproduce)."""
    K = NEWTON * CG
    ms = 0.0
    sched = 0.0
    for k in APPLY_CLASSES:
        if k not in totals:
            return {}
        t, cnt = totals[k]
        ms += t * (K / cnt)                     # the coil sum and row_adj also run for the right-hand sides
        sched += kernel_bytes(k, N, N_OM, J * B, B) * K
    per_s = B * K / (ms * 1e-3)
    return {"normal_applies_per_s": per_s,
            "normal_apply_us": 1e3 * ms / K,
            "normal_algorithmic_GBps": normal_bytes(N, N_OM, J, B) * K / (ms * 1e-3) / 1e9,
            "normal_schedule_GBps": sched / (ms * 1e-3) / 1e9}


def compare_paths(a, data, outs, B):
    """Plain path (one frame per solve call, eager launches) and back-to-back
    DF^H DF applies on one frame."""
    import numpy as np
    import torch
    from paper_1301_1215_amd import Plan, synth
    from paper_1301_1215_amd import _native as NAT
    img0 = outs[0]["image"].clone()
    plain = Plan(N, N_OM, J)
    pprm = Plan.params(NEWTON, CG, use_graph=False)
    pout = plain.solve(*data[0], pprm)
    torch.cuda.synchronize()
    spot = float((pout["image"] - img0).abs().pow(2).sum().sqrt() / img0.abs().pow(2).sum().sqrt())
    t0 = time.perf_counter()
    for i in range(a.plain_frames):
        plain.solve(*data[i % B], pprm)
    torch.cuda.synchronize()
    plain_fps = a.plain_frames / (time.perf_counter() - t0)
    rng = np.random.default_rng([2, 0, 3])
    rho = torch.from_numpy(synth.random_complex((N_OM, N_OM), rng)).cuda()
    chat = torch.from_numpy(synth.random_complex((J, N, N), rng)).cuda()
    c = plain.coil_maps(chat)
    h_r = torch.from_numpy(synth.random_complex((N_OM, N_OM), rng)).cuda()
    h_c = torch.from_numpy(synth.random_complex((J, N, N), rng)).cuda()
    o_r, o_c = torch.empty_like(h_r), torch.empty_like(h_c)
    P0 = data[0][1]
    for _ in range(10):
        NAT.nlinv_normal(plain.handle, rho, chat, c, P0, 0.5, h_r, h_c, o_r, o_c)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(a.applies):
        NAT.nlinv_normal(plain.handle, rho, chat, c, P0, 0.5, h_r, h_c, o_r, o_c)
    torch.cuda.synchronize()
    ap_s = a.applies / (time.perf_counter() - t0)
    nb = normal_bytes(N, N_OM, J)
    plain.close()
    return {"plain_frames_per_s": plain_fps, "plain_normal_applies_per_s": ap_s,
            "plain_normal_algorithmic_GBps": nb * ap_s / 1e9, "batched_vs_plain_image_rel": spot}


def other_workload(a):
    """Frames/s of the other workloads (no roofline line): 64x64 8-coil
    Cartesian frames batched (6 x 10), the 64-frame ragged batch (7 x 10),
    or the 512x512 32-coil series, 8 sequential warm-started frames per step."""
    import torch
    from paper_1301_1215_amd import Plan, synth
    if a.workload == "single_64":
        B = a.frames
        frames = [synth.make_frame(1, t, 64, 64, 8, "cartesian", newton=6) for t in range(B)]
        newton, desc = 6, f"single_64: {B} frames of 64x64, 8 coils, Cartesian 28/64 rows, 6 Newton x 10 CG"
    elif a.workload == "ragged_64":
        frames = synth.ragged_batch(64)
        B, newton = 64, 7
        desc = "ragged_64: 64 frames, n in {128,192,256,384}, J in {8,12,16,32}, spokes in {11,15,21}, 7x10"
    else:
        ph = synth.temporal_phantom()
        frames = [synth.temporal_frame(t, ph) for t in range(8)]
        B, newton = 8, 7
        desc = "series_512: 8 sequential frames of 512x512, 32 coils, 13 spokes, warm-started, 7x10"
    data = [(torch.from_numpy(f.y).cuda(), torch.from_numpy(f.P).cuda()) for f in frames]
    prm = Plan.params(newton, CG, use_graph=not a.no_graph)
    if a.workload == "series_512":
        pl = Plan(512, 256, 32)
        run = lambda outs: pl.solve_series(data, prm, outs)
        outs = [pl._frame_out(pl.dims, prm) for _ in range(B)]
    else:
        pl = Plan(frames=[(f.n, f.n_om, f.ncoils) for f in frames], branch_frames=a.branch_frames)
        run = lambda outs: pl.solve_batch(data, prm, outs)
        outs = [pl._frame_out(fd, prm) for fd in pl.frames]
    if not a.no_autotune:
        pl.autotune()
    for _ in range(max(1, a.warmup)):
        run(outs)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(a.steps):
        run(outs)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    out = {"metric": "IRGNM frames/sec", "value": B * a.steps / dt, "unit": "frames/s", "n_gpus": 1,
           "steps": a.steps, "warmup": a.warmup, "ms_per_step": 1e3 * dt / a.steps, "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "c64 (fp32), fp64 CG dots/scalars",
           "data": "synthetic", "config": {"workload": desc, "frames_per_step": B,
                                           "path": ("series" if a.workload == "series_512" else "batched")
                                           + ("" if a.no_graph else "+hipGraph")
                                           + (f", branches of {a.branch_frames} frames" if a.branch_frames
                                              else "")},
           "roofline": None, "cpu_baseline": None}
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--frames", type=int, default=4, help="frames per batched step")
    ap.add_argument("--compare", action="store_true",
                    help="also time the plain path (one frame per solve, eager) and DF^H DF applies; "
                         "their launches share kernels with the timed path, so keep this off for the "
                         "rocprofv3 run that backs the roofline")
    ap.add_argument("--plain-frames", type=int, default=4)
    ap.add_argument("--applies", type=int, default=200)
    ap.add_argument("--cpu-newton", type=int, default=2, help="Newton steps of the CPU oracle sample (0: skip)")
    ap.add_argument("--no-graph", action="store_true")
    ap.add_argument("--branch-frames", type=int, default=0,
                    help="frames of one shape per concurrent branch (0: one branch per shape); the "
                         "roofline kernel's launches then share the GPU with the other branches")
    ap.add_argument("--no-autotune", action="store_true", help="keep the default pass variants")
    ap.add_argument("--kernel-class", default=None, help="kernel class for the roofline (default: dominant)")
    ap.add_argument("--stream-probe", action="store_true",
                    help="also measure a 1 GiB device-to-device copy (the practical HBM ceiling)")
    ap.add_argument("--workload", default="realtime_384",
                    choices=["realtime_384", "single_64", "ragged_64", "series_512"],
                    help="realtime_384 (the benchmark line); the others report frames/s only")
    a = ap.parse_args()

    if a.gpus != 1:
        print(f"bench.py: this benchmark runs on one GPU; --gpus {a.gpus} is not supported "
              f"(the coil-split multi-GPU decomposition is designed, not built)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    from paper_1301_1215_amd import Plan, synth
    from paper_1301_1215_amd import _native as NAT

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    NAT.load()
    if a.workload != "realtime_384":
        return other_workload(a)
    B = a.frames
    log(f"bench: generating {B} frames of {N}x{N}, {J} coils, {SPOKES} spokes")
    frames = [synth.make_frame(2, t, N, N_OM, J, "radial", spokes=SPOKES, newton=NEWTON, cg=CG,
                               mask_frame=t + 1) for t in range(B)]
    data = [(torch.from_numpy(f.y).cuda(), torch.from_numpy(f.P).cuda()) for f in frames]
    prm = Plan.params(NEWTON, CG, use_graph=not a.no_graph)
    pl = Plan(frames=[(N, N_OM, J)] * B, branch_frames=a.branch_frames)
    if not a.no_autotune:
        os.environ.setdefault("NLINV_TUNE_VERBOSE", "1")
        pl.autotune()
        log(f"bench: autotuned pass variants for n={N}: (column, row) = {pl.variant(N)}")
    outs = [pl._frame_out(pl.frames[i], prm) for i in range(B)]
    stream = torch.cuda.current_stream()

    # warm-up (captures the graph); then find the dominant kernel class
    for _ in range(max(1, a.warmup)):
        pl.solve_batch(data, prm, outs)
    torch.cuda.synchronize()
    names = NAT.nlinv_kernel_class_names()
    kc = a.kernel_class
    timing_path = "graph" if not a.no_graph else "eager"
    try:
        if kc is None:
            kc = dominant_class(pl, data, prm, outs, names)
        pl.timing_enable(kc, TIMING_STRIDE)
        pl.solve_batch(data, prm, outs)       # recapture with the brackets of this class
        torch.cuda.synchronize()
        pl.timing_read()
    except NAT.NlinvError as e:
        # event brackets inside the captured graph unavailable: time this class on eager launches
        log(f"bench: graph-side kernel timing failed ({e}); timing kernels on eager launches")
        timing_path = "eager"
        for k in names:
            pl.timing_enable(k, False)
        eprm = Plan.params(NEWTON, CG, use_graph=False)
        if kc is None:
            kc = dominant_class(pl, data, eprm, outs, names)

    # timed region
    log(f"bench: timing {a.steps} steps of {B} frames")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    launches, kms = 0, 0.0
    for _ in range(a.steps):
        pl.solve_batch(data, prm, outs)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    if timing_path == "graph" or a.no_graph:
        # graph-owned brackets hold the last replay; eager ones every launch
        launches, kms = pl.timing_read()
    else:
        # the same steps again on eager launches, with this class bracketed
        pl.timing_enable(kc, TIMING_STRIDE)
        for _ in range(a.steps):
            pl.solve_batch(data, eprm, outs)
        torch.cuda.synchronize()
        launches, kms = pl.timing_read()
    pl.timing_enable(kc, False)
    ms_step = 1e3 * dt / a.steps
    fps = B * a.steps / dt
    log(f"bench: {ms_step:.2f} ms/step, {fps:.1f} frames/s; {kc}: {launches} launches, {kms:.3f} ms")

    extras = {}
    if getattr(dominant_class, "totals", None) and not a.branch_frames:
        extras.update(apply_rates(dominant_class.totals, B))
    if a.compare:
        extras.update(compare_paths(a, data, outs, B))

    # roofline of the dominant kernel class
    # with concurrent branches each launch covers one branch's frames
    nbranch = -(-B // a.branch_frames) if a.branch_frames > 0 else 1
    per_launch = kernel_bytes(kc, N, N_OM, J * B, B) / nbranch
    avg_ms = kms / max(launches, 1)
    achieved = per_launch / (avg_ms * 1e-3) / 1e9 if launches else None
    roof = {"bound": "hbm", "kernel": kc, "achieved": achieved, "peak": HBM_PEAK_GBPS, "unit": "GB/s",
            "frac": (achieved / HBM_PEAK_GBPS) if achieved else None,
            # the counters were taken on launches that cover all B frames
            "traffic": None if a.branch_frames else pmc_traffic(kc, B),
            "bytes_per_launch": per_launch, "avg_launch_ms": avg_ms, "launches_timed": launches,
            "timing_stride": TIMING_STRIDE, "event_timing_on": timing_path}

    if a.stream_probe:
        extras["stream_copy_GBps"] = stream_probe()
    cpu = cpu_baseline(a.cpu_newton) if a.cpu_newton > 0 else None
    out = {
        "metric": "IRGNM frames/sec and DF^H.DF applies/sec (HBM GB/s) at <=1e-3 NRMSE vs FP64",
        "value": fps, "unit": "frames/s", "n_gpus": 1, "steps": a.steps, "warmup": a.warmup,
        "ms_per_step": ms_step, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "c64 (fp32), fp64 CG dots/scalars", "data": "synthetic",
        "config": {"workload": "realtime_384: 384x384 grid, Omega 192x192, 12 coils, 15 radial spokes, "
                               "7 Newton x 10 CG",
                   "frames_per_step": B, "path": "batched" + ("" if a.no_graph else "+hipGraph")
                   + (f", branches of {a.branch_frames} frames" if a.branch_frames else "")},
        **extras,
        "roofline": roof,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
