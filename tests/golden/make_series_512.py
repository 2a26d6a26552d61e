"""Writes series_512_oracle.npz: the FP64 oracle's temporal series on the
512x512, 32-coil, 13-spoke workload (frames 0..7, 7 Newton x 10 CG, each
frame warm-started from and regularised towards the previous one, Sec. 3.2).

Only the oracle and the seeded input generator are called.  Stored per frame:
the image on every second pixel of Omega along both axes (complex64), the
oracle's residual norms per Newton step, and a SHA-256 of the frame's inputs
(y and P as handed to both sides) so that a test can tell whether the inputs
it generates are the ones this file was made from.

Usage: python -m tests.golden.make_series_512   (about 5-10 min on 8 cores)
"""
from __future__ import annotations

import hashlib
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

from oracle import nlinv_oracle as O          # noqa: E402
from paper_1301_1215_amd import synth         # noqa: E402

FRAMES = 8
NEWTON, CG = 7, 10
STRIDE = 2
OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "series_512_oracle.npz")


def input_digest(y: np.ndarray, P: np.ndarray) -> str:
    h = hashlib.sha256()
    h.update(np.ascontiguousarray(y).tobytes())
    h.update(np.ascontiguousarray(P).tobytes())
    return h.hexdigest()


def main():
    O.set_workers(os.cpu_count() or 1)
    ph = synth.temporal_phantom()
    frames = [synth.temporal_frame(t, ph) for t in range(FRAMES)]
    d = O.Dims(frames[0].n, frames[0].n_om, frames[0].ncoils)
    prm = O.IRGNMParams(NEWTON, CG)
    imgs, r0, dig = [], [], []
    prev = None
    for t, f in enumerate(frames):
        t0 = time.perf_counter()
        if prev is None:
            res = O.irgnm(f.y, f.P, d, prm)
        else:
            res = O.irgnm(f.y, f.P, d, prm, rho0=prev.rho, chat0=prev.chat, rho_ref=prev.rho, chat_ref=prev.chat)
        prev = res
        imgs.append(res.image[::STRIDE, ::STRIDE].astype(np.complex64))
        r0.append(np.array(res.r0_norms))
        dig.append(input_digest(f.y, f.P))
        print(f"frame {t}: {time.perf_counter() - t0:.1f} s", flush=True)
    np.savez_compressed(OUT, image_sampled=np.stack(imgs), r0_norms=np.stack(r0), stride=STRIDE,
                        newton=NEWTON, cg=CG, input_sha256=np.array(dig))
    print("wrote", OUT)


if __name__ == "__main__":
    main()
