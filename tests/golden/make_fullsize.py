"""Write the oracle reference for the full-size 256^3 order-8 forward test.

Runs the FP64 oracle (and nothing else) on the seeded 256^3 workload for all
1000 steps and stores, in fullsize_3d-256-o8.npz:
  rec_idx  the sampled receiver indices
  d        oracle traces at those receivers [1000][len(rec_idx)]
  pts      sampled flat grid indices
  u        oracle u^1000 at those points
and, after a second pass with --precision f32, the error of the FP32 build of
the oracle against those values (f32_rel_d, f32_rel_u, f32_maxrel_d,
f32_maxrel_u): the FP32 round-off floor of the plain scheme.
Usage: python tests/golden/make_fullsize.py [--precision f32]
(about 5 minutes per pass on 8 cores)
"""
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_1609_03361_amd import synth  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "fullsize_3d-256-o8.npz")


def sample_indices(p):
    rng = np.random.default_rng(256)
    rec_idx = np.sort(rng.choice(p.rec.shape[0], 48, replace=False))
    # points: near the source (where the field is large) and random elsewhere
    n = p.shape[0]
    near = [(i, j, k) for i in (120, 127, 128, 135) for j in (110, 127, 140) for k in (2, 3, 10, 40)]
    far = rng.integers(0, n, size=(400, 3))
    pts = np.array([np.ravel_multi_index(t, p.shape) for t in near] +
                   [np.ravel_multi_index(tuple(t), p.shape) for t in far], dtype=np.int64)
    return rec_idx, pts


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def maxrel(a, b):
    return float(np.max(np.abs(a - b)) / np.max(np.abs(b)))


def main():
    import argparse
    ap = argparse.ArgumentParser()
    ap.add_argument("--precision", choices=("f64", "f32"), default="f64",
                    help="f64 writes the reference; f32 then adds the error of the FP32 build "
                         "of the oracle at the same samples (f32_rel_d, f32_rel_u, "
                         "f32_maxrel_d, f32_maxrel_u)")
    args = ap.parse_args()
    p = synth.config_3d_o8()
    rec_idx, pts = sample_indices(p)
    r = oracle.forward(p.shape, p.spacing, p.order, p.dt, p.nt, p.m, p.eta, p.src, p.q, p.rec,
                       precision=args.precision)
    d, u = r["d"][:, rec_idx], r["u"].ravel()[pts]
    if args.precision == "f64":
        np.savez_compressed(OUT, rec_idx=rec_idx, d=d, pts=pts, u=u)
    else:
        g = dict(np.load(OUT))
        assert np.array_equal(g["pts"], pts) and np.array_equal(g["rec_idx"], rec_idx)
        g["f32_rel_d"], g["f32_maxrel_d"] = rel(d, g["d"]), maxrel(d, g["d"])
        g["f32_rel_u"], g["f32_maxrel_u"] = rel(u, g["u"]), maxrel(u, g["u"])
        print({k: float(g[k]) for k in g if k.startswith("f32_")}, flush=True)
        np.savez_compressed(OUT, **g)
    print("wrote", OUT)


if __name__ == "__main__":
    main()
