"""Write the oracle reference for the full-length 512^3 order-16 forward test.

Runs the CPU oracle (and nothing else) on the seeded 512^3 order-16 workload
for all 2000 steps and stores, in fullsize_3d-512-o16.npz (values rounded to
float32; that rounding, about 6e-8 relative, is far below every tolerance):
  rec_full   receiver indices sampled at every step
  d_full     FP64-oracle traces at rec_full [2000][len(rec_full)]
  t_sub      every 20th step
  rec_sub    a second set of receivers, sampled at t_sub
  d_sub      FP64-oracle traces [len(t_sub)][len(rec_sub)]
  pts        flat grid indices of sampled points of u^2000: whole lines along
             x, y and z through planes next to tile and x-chunk edges (so any
             blocking plan has sampled points on both sides of its edges),
             plus random points
  u          FP64-oracle u^2000 at pts
and, after the second pass (--precision f32), the error of the FP32 build of
the oracle against the FP64 values at the same samples:
  f32_rel_d, f32_rel_u        relative L2
  f32_maxrel_d, f32_maxrel_u  max |f32 - f64| / max |f64|

Usage (in this order; each pass takes about 2 hours on 8 cores and 5-9 GB):
  python tests/golden/make_fullsize_512.py --precision f64
  python tests/golden/make_fullsize_512.py --precision f32
"""
import argparse
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_1609_03361_amd import synth  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "fullsize_3d-512-o16.npz")

# (second, third) coordinates of whole sampled lines; each pair straddles a
# multiple of 16, 32, 64 or 128 (tile edges in y and z) or the x-chunk edges
# of 3-chunk and 4-chunk plans (170/171, 341/342, 127/128, 255/256, 383/384)
X_LINES = [(255, 2), (256, 25), (15, 63), (16, 64), (31, 127), (32, 128), (127, 255), (128, 256),
           (200, 300), (383, 447), (384, 448), (511, 511), (0, 0), (255, 160), (256, 31), (100, 32)]
Y_LINES = [(170, 2), (171, 25), (341, 63), (342, 64), (255, 127), (256, 128), (127, 255),
           (128, 256), (85, 300), (86, 448), (0, 0), (511, 511), (400, 31), (401, 32), (255, 100),
           (256, 200)]
Z_LINES = [(170, 15), (171, 16), (341, 31), (342, 32), (255, 255), (256, 256), (127, 128),
           (128, 127), (0, 0), (511, 511), (300, 200), (42, 470), (170, 255), (171, 256),
           (341, 100), (342, 101)]


def sample_indices(p):
    n = p.shape[0]
    nrec = p.rec.shape[0]
    rng = np.random.default_rng(512)
    side = int(round(np.sqrt(nrec)))
    corners = [0, side - 1, nrec - side, nrec - 1]      # the last row/column hit the edge clamp
    rec_full = np.unique(np.concatenate([corners, rng.choice(nrec, 60, replace=False)]))
    rec_sub = np.sort(rng.choice(nrec, 1024, replace=False))
    t_sub = np.arange(0, p.nt, 20)
    ax = np.arange(n)
    pts = []
    for (y, z) in X_LINES:
        pts.append(np.ravel_multi_index((ax, np.full(n, y), np.full(n, z)), p.shape))
    for (x, z) in Y_LINES:
        pts.append(np.ravel_multi_index((np.full(n, x), ax, np.full(n, z)), p.shape))
    for (x, y) in Z_LINES:
        pts.append(np.ravel_multi_index((np.full(n, x), np.full(n, y), ax), p.shape))
    rnd = rng.integers(0, n, size=(4096, 3))
    pts.append(np.ravel_multi_index(tuple(rnd.T), p.shape))
    return rec_full, rec_sub, t_sub, np.concatenate(pts).astype(np.int64)


def run(p, precision):
    t0 = time.time()
    r = oracle.forward(p.shape, p.spacing, p.order, p.dt, p.nt, p.m, p.eta, p.src, p.q, p.rec,
                       precision=precision)
    print(f"oracle {precision}: {p.nt} steps in {time.time() - t0:.0f} s", flush=True)
    return r


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def maxrel(a, b):
    return float(np.max(np.abs(a - b)) / np.max(np.abs(b)))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--precision", choices=("f64", "f32"), required=True)
    args = ap.parse_args()
    p = synth.config_3d_o16()
    rec_full, rec_sub, t_sub, pts = sample_indices(p)
    r = run(p, args.precision)
    d_full = r["d"][:, rec_full]
    d_sub = r["d"][np.ix_(t_sub, rec_sub)]
    u = r["u"].ravel()[pts]
    if args.precision == "f64":
        np.savez_compressed(OUT, rec_full=rec_full, d_full=d_full.astype(np.float32),
                            t_sub=t_sub, rec_sub=rec_sub, d_sub=d_sub.astype(np.float32),
                            pts=pts, u=u.astype(np.float32))
    else:
        g = dict(np.load(OUT))
        assert np.array_equal(g["pts"], pts) and np.array_equal(g["rec_full"], rec_full)
        d_ref = np.concatenate([g["d_full"].ravel(), g["d_sub"].ravel()]).astype(np.float64)
        d_got = np.concatenate([d_full.ravel(), d_sub.ravel()])
        g["f32_rel_d"] = rel(d_got, d_ref)
        g["f32_maxrel_d"] = maxrel(d_got, d_ref)
        g["f32_rel_u"] = rel(u, g["u"].astype(np.float64))
        g["f32_maxrel_u"] = maxrel(u, g["u"].astype(np.float64))
        print({k: float(g[k]) for k in g if k.startswith("f32_")}, flush=True)
        np.savez_compressed(OUT, **g)
    print("wrote", OUT, flush=True)


if __name__ == "__main__":
    main()
