"""Write the oracle reference for the full-size 256^3 order-8 forward test.

Runs the FP64 oracle (and nothing else) on the seeded 256^3 workload for all
1000 steps and stores, in fullsize_3d-256-o8.npz:
  rec_idx  the sampled receiver indices
  d        oracle traces at those receivers [1000][len(rec_idx)]
  pts      sampled flat grid indices
  u        oracle u^1000 at those points
Usage: python tests/golden/make_fullsize.py   (about 5 minutes on 8 cores)
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


def main():
    p = synth.config_3d_o8()
    rec_idx, pts = sample_indices(p)
    r = oracle.forward(p.shape, p.spacing, p.order, p.dt, p.nt, p.m, p.eta, p.src, p.q, p.rec)
    np.savez_compressed(OUT, rec_idx=rec_idx, d=r["d"][:, rec_idx], pts=pts,
                        u=r["u"].ravel()[pts])
    print("wrote", OUT)


if __name__ == "__main__":
    main()
