"""Write the oracle reference for the full-size batched 2D test.

Runs the FP64 oracle (and nothing else) on three of the 48 seeded shots of
the batched workload (2001 x 801 model, order 8, 2000 steps): the first, the
narrowest and the widest.  Stores, in fullsize_batch2d-o8.npz:
  shots    the shot indices
  rec_idx  sampled receiver indices (the same for every shot)
  t_idx    sampled time steps
  d        oracle traces [shot][t_idx][rec_idx] (float32)
and, after a second pass with --precision f32, the per-shot error of the FP32
build of the oracle at the same samples (f32_rel, f32_maxrel).
Usage: python tests/golden/make_batch_golden.py [--precision f32]
(a few minutes per pass on 8 cores)
"""
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_1609_03361_amd import synth  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "fullsize_batch2d-o8.npz")


def pick(probs):
    widths = [p.shape[0] for p in probs]
    return sorted({0, int(np.argmin(widths)), int(np.argmax(widths))})


def main():
    import argparse
    ap = argparse.ArgumentParser()
    ap.add_argument("--precision", choices=("f64", "f32"), default="f64",
                    help="f64 writes the reference; f32 then adds, per shot, the error of the "
                         "FP32 build of the oracle at the same samples (f32_rel, f32_maxrel)")
    args = ap.parse_args()
    probs = synth.config_batched_2d()
    shots = pick(probs)
    rec_idx = np.arange(0, 400, 13)
    t_idx = np.arange(0, probs[0].nt, 4)
    out = []
    for s in shots:
        p = probs[s]
        r = oracle.forward(p.shape, p.spacing, p.order, p.dt, p.nt, p.m, p.eta, p.src, p.q, p.rec,
                           want_final=False, precision=args.precision)
        out.append(r["d"][np.ix_(t_idx, rec_idx)])
        print(f"shot {s} ({p.name}) done", flush=True)
    if args.precision == "f64":
        np.savez_compressed(OUT, shots=np.array(shots), rec_idx=rec_idx, t_idx=t_idx,
                            d=np.array(out, dtype=np.float32))
    else:
        g = dict(np.load(OUT))
        assert np.array_equal(g["shots"], shots)
        ref = g["d"].astype(np.float64)
        got = np.array(out)
        g["f32_rel"] = np.array([np.linalg.norm(got[k] - ref[k]) / np.linalg.norm(ref[k])
                                 for k in range(len(shots))])
        g["f32_maxrel"] = np.array([np.max(np.abs(got[k] - ref[k])) / np.max(np.abs(ref[k]))
                                    for k in range(len(shots))])
        print("f32_rel", g["f32_rel"], "f32_maxrel", g["f32_maxrel"], flush=True)
        np.savez_compressed(OUT, **g)
    print("wrote", OUT)


if __name__ == "__main__":
    main()
