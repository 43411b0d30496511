"""Full-size parity in the launch configuration the benchmark times.

* 256^3, order 8, all 1000 steps (the bench workload): sampled traces and
  sampled points of u^1000 against oracle values stored by
  tests/golden/make_fullsize.py (which calls only the oracle);
* 512^3, order 16, all 2000 steps (the roofline benchmark): whole traces of 64
  receivers, every 20th step of 1024 more, and u^2000 along whole lines in
  x, y and z through planes next to tile and x-chunk edges, against oracle
  values stored by tests/golden/make_fullsize_512.py (oracle only).
Each check is relative L2 and max-abs / max-ref <= 1e-5, and within twice
the error of the FP32 build of the oracle at the same samples (the FP32
round-off floor of the plain scheme, stored with the reference).
"""
import os

import numpy as np
import pytest

from gpu_util import assert_close, device_inputs
from paper_1609_03361_amd import synth

pytestmark = pytest.mark.gpu
GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


@pytest.fixture(scope="module")
def dev():
    import torch
    assert torch.cuda.is_available()
    return torch.device("cuda:0")


def test_256cube_order8_1000_steps_sampled(dev):
    """The planned tile, then the tile the autotuner picks on this grid (the
    one the benchmark's headline leg times)."""
    import torch
    from paper_1609_03361_amd import api
    ref = np.load(os.path.join(GOLDEN, "fullsize_3d-256-o8.npz"))
    p = synth.config_3d_o8()
    geom, m, eta, q = device_inputs(p, dev)
    for which in ("planned", "tuned"):
        tile = 0
        if which == "tuned":
            tile, us = api.tune(geom, steps=10)
            print(f"tuned tile {tile >> 16}/{tile & 0xffff}: {us:.2f} us/step", flush=True)
        d, u = api.forward(geom, m, eta, q, return_final=True, tile=tile)
        torch.cuda.synchronize()
        d = d.cpu().numpy()[:, ref["rec_idx"]]
        u = u.cpu().numpy().ravel()[ref["pts"]]
        ed, _ = assert_close(d, ref["d"], f"3d-256-o8 x 1000 sampled traces ({which} tile)",
                             fp32_oracle=float(ref["f32_rel_d"]))
        eu, _ = assert_close(u, ref["u"], f"3d-256-o8 x 1000 sampled u^1000 ({which} tile)",
                             fp32_oracle=float(ref["f32_rel_u"]))
        assert ed <= 2 * float(ref["f32_rel_d"]) and eu <= 2 * float(ref["f32_rel_u"])
    print(f"FP32 oracle at the same samples: traces {float(ref['f32_rel_d']):.3e}, "
          f"u {float(ref['f32_rel_u']):.3e}", flush=True)


def test_512cube_order16_2000_steps_sampled(dev):
    import torch
    from paper_1609_03361_amd import api
    path = os.path.join(GOLDEN, "fullsize_3d-512-o16.npz")
    ref = np.load(path)
    p = synth.config_3d_o16()
    geom, m, eta, q = device_inputs(p, dev)
    d, u = api.forward(geom, m, eta, q, return_final=True)
    torch.cuda.synchronize()
    d = d.cpu().numpy()
    d_got = np.concatenate([d[:, ref["rec_full"]].ravel(),
                            d[np.ix_(ref["t_sub"], ref["rec_sub"])].ravel()])
    d_ref = np.concatenate([ref["d_full"].ravel(), ref["d_sub"].ravel()])
    del d
    u = u.cpu().numpy().ravel()[ref["pts"]]
    extra = {}
    if "f32_rel_d" in ref:
        extra = dict(fp32_oracle_d=float(ref["f32_rel_d"]), fp32_oracle_u=float(ref["f32_rel_u"]))
    ed, _ = assert_close(d_got, d_ref, "3d-512-o16 x 2000 sampled traces", **extra)
    eu, _ = assert_close(u, ref["u"], "3d-512-o16 x 2000 u^2000 on lines through tile and "
                         "chunk edges", **extra)
    if extra:
        print(f"FP32 oracle at the same samples: traces {extra['fp32_oracle_d']:.3e}, "
              f"u {extra['fp32_oracle_u']:.3e}", flush=True)
        assert ed <= 2 * extra["fp32_oracle_d"] and eu <= 2 * extra["fp32_oracle_u"]
