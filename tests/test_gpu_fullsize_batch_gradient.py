"""Full-size checks of the batched-shot and gradient workloads in the
launch configuration the benchmark times.

* 48 batched 2D shots (2001 x 801 model, order 8, 2000 steps), one hipGraph
  replay: sampled traces of three shots against oracle values stored by
  tests/golden/make_batch_golden.py (which calls only the oracle).
* FWI gradient on 200^3, order 8, 1500 steps, checkpoints every 20: the
  oracle's full-storage gradient does not fit this size, so the check is a
  property that holds at any size -- the directional derivative <g, dm>
  matches the central difference of the misfit, with the O(h^2) error of
  the difference falling as h halves.
"""
import os

import numpy as np
import pytest

from gpu_util import assert_close, rel_l2
from paper_1609_03361_amd import synth

pytestmark = pytest.mark.gpu
GOLD = os.path.join(os.path.dirname(__file__), "golden", "fullsize_batch2d-o8.npz")


@pytest.fixture(scope="module")
def dev():
    import torch
    assert torch.cuda.is_available()
    return torch.device("cuda:0")


def test_48_batched_shots_full_size_sampled(dev):
    """Three of the shots (the first, the narrowest, the widest) at sampled
    times and receivers: relative L2 and max-abs / max-ref <= 1e-5, and within
    twice the error of the FP32 build of the oracle on the same samples (stored
    with the reference).  Over 2000 steps the FP32 rounding of each update adds
    up; the results are bitwise reproducible and do not depend on the tile."""
    import torch
    from paper_1609_03361_amd import api
    ref = np.load(GOLD)
    probs = synth.config_batched_2d()
    shots = [(api.Geometry(p.shape, p.spacing, p.order, p.dt, p.nt, p.src, p.rec),
              torch.from_numpy(p.m).to(dev), torch.from_numpy(p.eta).to(dev),
              torch.from_numpy(p.q).to(dev)) for p in probs]
    d = api.forward_batch(shots)
    torch.cuda.synchronize()
    for k, s in enumerate(ref["shots"]):
        got = d[int(s)].cpu().numpy()[np.ix_(ref["t_idx"], ref["rec_idx"])]
        floor = float(ref["f32_rel"][k])
        e, _ = assert_close(got, ref["d"][k], f"batched shot {int(s)} ({probs[int(s)].name}) "
                            f"sampled traces", fp32_oracle=floor)
        print(f"  FP32 oracle at the same samples: {floor:.3e}", flush=True)
        assert e <= 2 * floor


@pytest.mark.parametrize("ckpt_dtype", ["fp32", "bf16"])
def test_gradient_200cube_directional_derivative(dev, ckpt_dtype):
    import torch
    from paper_1609_03361_amd import api
    m0, mt, eta, shots = synth.config_gradient_3d()
    p = shots[0]
    geom = api.Geometry(p.shape, p.spacing, p.order, p.dt, p.nt, p.src, p.rec)
    M0 = torch.from_numpy(m0).to(dev)
    MT = torch.from_numpy(mt).to(dev)
    E = torch.from_numpy(eta).to(dev)
    q = torch.from_numpy(p.q).to(dev)
    dobs = api.forward(geom, MT, E, q)
    J, g = api.gradient(geom, M0, E, q, dobs, ckpt_every=20, ckpt_dtype=ckpt_dtype)
    dm = MT - M0
    gd = float((g.double() * dm.double()).sum())

    def misfit(mm):
        d = api.forward(geom, mm.contiguous(), E, q)
        return 0.5 * float(((d - dobs).double() ** 2).sum())

    errs = []
    for h in (0.2, 0.1):
        cd = (misfit(M0 + h * dm) - misfit(M0 - h * dm)) / (2 * h)
        errs.append(abs(cd / gd - 1.0))
        print(f"{ckpt_dtype} h={h}: central difference / <g, dm> - 1 = {cd / gd - 1:.2e}", flush=True)
    # measured: 1.7e-3 at h = 0.2 and 4.3e-4 at h = 0.1 (ratio 3.96), the same to
    # 1e-6 with BF16 checkpoints; an error in g of relative size e would leave
    # a floor of about e here instead of the fall by 4
    assert errs[1] < 1e-3
    assert 3.0 < errs[0] / errs[1] < 5.0
