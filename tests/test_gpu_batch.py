"""Batched shots and tiles: every shot of a batch (one launch per step over
all shots, captured in a hipGraph) must equal the same shot run alone, bit
for bit; explicit and tuned tiles must not change any result; a couple of
shots are also checked against the oracle."""
import numpy as np
import pytest

from gpu_util import device_inputs, oracle_forward, rel_l2
from paper_1609_03361_amd import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dev():
    import torch
    assert torch.cuda.is_available()
    return torch.device("cuda:0")


def _shots(dev, n=5, nt=120):
    import torch
    from paper_1609_03361_amd import api
    probs = synth.config_batched_2d(nshots=n, nx=301, nz=81, nt=nt, wmin=60, nrec=37)
    out = []
    for p in probs:
        geom, m, eta, q = device_inputs(p, dev)
        out.append((geom, m, eta, q))
    return probs, out


@pytest.mark.parametrize("graph", [True, False])
def test_batch_equals_single_shots_bitwise(dev, graph):
    import torch
    from paper_1609_03361_amd import api
    probs, shots = _shots(dev)
    print("widths", [p.shape[0] for p in probs], flush=True)
    d, u = api.forward_batch(shots, return_final=True, graph=graph)
    for i, (geom, m, eta, q) in enumerate(shots):
        ds, us = api.forward(geom, m, eta, q, return_final=True)
        torch.cuda.synchronize()
        assert torch.equal(ds, d[i]), i
        assert torch.equal(us, u[i]), i


def test_batch_graph_replay_is_reused_and_stable(dev):
    import torch
    from paper_1609_03361_amd import api
    probs, shots = _shots(dev, n=3, nt=60)
    a = api.forward_batch(shots, return_final=True)
    b = api.forward_batch(shots, return_final=True)
    torch.cuda.synchronize()
    for x, y in zip(a[0] + a[1], b[0] + b[1]):
        assert torch.equal(x, y)


def test_batch_shots_match_oracle(dev):
    import torch
    from paper_1609_03361_amd import api
    probs, shots = _shots(dev, n=3, nt=150)
    d, u = api.forward_batch(shots, return_final=True)
    torch.cuda.synchronize()
    for i in (0, 2):
        ref = oracle_forward(probs[i])
        assert rel_l2(d[i].cpu().numpy(), ref["d"]) < 1e-5
        assert rel_l2(u[i].cpu().numpy(), ref["u"]) < 1e-5


def test_3d_batch_equals_single(dev):
    import torch
    from paper_1609_03361_amd import api
    shots = []
    for k, shape in enumerate([(20, 18, 24), (31, 22, 24), (17, 26, 24)]):
        p = synth.random_problem(shape, 8, 30, seed=40 + k, nsrc=2, nrec=6)
        p.dt = 0.0004
        shots.append(device_inputs(p, dev))
    d, u = api.forward_batch(shots, return_final=True)
    for i, (geom, m, eta, q) in enumerate(shots):
        ds, us = api.forward(geom, m, eta, q, return_final=True)
        torch.cuda.synchronize()
        assert torch.equal(ds, d[i]) and torch.equal(us, u[i])


@pytest.mark.parametrize("shape,order", [((33, 29, 40), 8), ((60, 70), 8), ((25, 23, 31), 4),
                                         ((45, 33), 6), ((21, 17, 13), 16)])
def test_tiles_do_not_change_results(dev, shape, order):
    import torch
    from paper_1609_03361_amd import api
    p = synth.random_problem(shape, order, 16, seed=5, nsrc=3, nrec=8)
    geom, m, eta, q = device_inputs(p, dev)
    ref = api.forward(geom, m, eta, q, return_final=True)
    # block shapes: 4 in 2D, 11 in 3D (rows are padded to 4 points inside the library)
    for v in range(4 if len(shape) == 2 else 11):
        for x in (1, order // 2, 7, 64):
            got = api.forward(geom, m, eta, q, return_final=True, tile=api.tile_id(v, x))
            torch.cuda.synchronize()
            assert torch.equal(got[0], ref[0]) and torch.equal(got[1], ref[1]), (v, x)


def test_tuner_picks_a_tile_and_results_stay_bitwise(dev):
    import torch
    from paper_1609_03361_amd import api
    p = synth.random_problem((48, 44, 64), 8, 12, seed=6, nsrc=2, nrec=5)
    geom, m, eta, q = device_inputs(p, dev)
    ref = api.forward(geom, m, eta, q, return_final=True)
    tile, us = api.tune(geom, steps=5)
    print(f"tuned tile variant {tile >> 16} x-chunk {tile & 0xffff}: {us:.2f} us/step", flush=True)
    assert tile > 0 and us > 0
    got = api.forward(geom, m, eta, q, return_final=True)      # tile 0 -> cached tile
    torch.cuda.synchronize()
    assert torch.equal(got[0], ref[0]) and torch.equal(got[1], ref[1])
    probs, shots = _shots(dev, n=3, nt=20)
    bt, bus = api.tune_batch(shots, steps=3)
    print(f"batch tile variant {bt >> 16} x-chunk {bt & 0xffff}: {bus:.2f} us/step", flush=True)
    assert bt > 0


@pytest.mark.parametrize("graph", [True, False])
def test_persistent_batch_equals_per_step_batch_bitwise(dev, graph):
    """All steps of all shots in one persistent co-resident launch with a
    device-wide barrier per step, as the cooperative node of a hipGraph (mode
    3) or launched directly (mode 2): bitwise the per-step result, also when
    the graph is replayed a second time."""
    import torch
    from paper_1609_03361_amd import api
    probs, shots = _shots(dev, n=5, nt=90)
    a = api.forward_batch(shots, return_final=True)
    for rep in range(2):
        print(f"persistent batch, graph={graph}, call {rep}", flush=True)
        b = api.forward_batch(shots, return_final=True, persistent=True, graph=graph)
        mode = api.last_batch_mode()
        torch.cuda.synchronize()
        print(f"persistent batch ran in mode {mode}", flush=True)
        assert mode == (3 if graph else 2)
        for x, y in zip(a[0] + a[1], b[0] + b[1]):
            assert torch.equal(x, y)


def test_persistent_3d_batch_equals_single(dev):
    import torch
    from paper_1609_03361_amd import api
    shots = []
    for k, shape in enumerate([(20, 18, 24), (31, 22, 24), (17, 26, 24)]):
        p = synth.random_problem(shape, 8, 30, seed=40 + k, nsrc=2, nrec=6)
        p.dt = 0.0004
        shots.append(device_inputs(p, dev))
    d, u = api.forward_batch(shots, return_final=True, persistent=True)
    for i, (geom, m, eta, q) in enumerate(shots):
        ds, us = api.forward(geom, m, eta, q, return_final=True)
        torch.cuda.synchronize()
        assert torch.equal(ds, d[i]) and torch.equal(us, u[i])


def test_imaging_tile_tuned_separately_and_gradient_unchanged(dev):
    """wave_tune with the imaging flag times the adjoint step with the fused
    imaging condition; its winner is cached under its own key, and the
    gradient does not change by a bit."""
    import torch
    from paper_1609_03361_amd import api
    p = synth.random_problem((30, 28, 36), 8, 40, seed=8, nsrc=2, nrec=9)
    geom, m, eta, q = device_inputs(p, dev)
    d_obs = api.forward(geom, m * 1.01, eta, q)
    J0, g0 = api.gradient(geom, m, eta, q, d_obs, ckpt_every=10)
    t_img, us_img = api.tune(geom, steps=3, imaging=True)
    t_fwd, us_fwd = api.tune(geom, steps=3)
    print(f"imaging tile {t_img >> 16}/{t_img & 0xffff} {us_img:.2f} us; "
          f"plain tile {t_fwd >> 16}/{t_fwd & 0xffff} {us_fwd:.2f} us", flush=True)
    J1, g1 = api.gradient(geom, m, eta, q, d_obs, ckpt_every=10)
    torch.cuda.synchronize()
    assert torch.equal(g0, g1) and torch.equal(J0, J1)


def test_tune_shot_times_the_shot_and_results_stay_bitwise(dev):
    """wave_tune_shot times the step with the shot's own points (forward:
    sources injected, receivers sampled; imaging adjoint: 300 receivers, a
    dense set gathered a step ahead, injected and the sources sampled); its
    winners are cached for tile 0 and change no result."""
    import torch
    from paper_1609_03361_amd import api
    p = synth.random_problem((30, 28, 36), 8, 40, seed=18, nsrc=2, nrec=300)
    geom, m, eta, q = device_inputs(p, dev)
    d_obs = api.forward(geom, m * 1.01, eta, q)
    d0 = api.forward(geom, m, eta, q)
    J0, g0 = api.gradient(geom, m, eta, q, d_obs, ckpt_every=10)
    t_f, us_f = api.tune(geom, steps=3, m=m, eta=eta)
    t_i, us_i = api.tune(geom, steps=3, imaging=True, m=m, eta=eta)
    print(f"shot-tuned step {t_f >> 16}/{t_f & 0xffff} {us_f:.2f} us; "
          f"imaging {t_i >> 16}/{t_i & 0xffff} {us_i:.2f} us", flush=True)
    assert us_f > 0 and us_i > 0
    d1 = api.forward(geom, m, eta, q)
    J1, g1 = api.gradient(geom, m, eta, q, d_obs, ckpt_every=10)
    torch.cuda.synchronize()
    assert torch.equal(d0, d1) and torch.equal(g0, g1) and torch.equal(J0, J1)


def test_dense_sources_gathered_path_equals_direct_bitwise(dev):
    """Point sets of 256 entries or more have their values gathered into entry
    order a step ahead (single-shot launches); the batch kernel reads them
    directly.  Both must give the same bits."""
    import torch
    from paper_1609_03361_amd import api
    shots = []
    for k, shape in enumerate([(24, 22, 28), (30, 26, 20)]):
        p = synth.random_problem(shape, 8, 25, seed=60 + k, nsrc=40, nrec=50)   # 320 entries
        p.dt = 0.0004
        shots.append(device_inputs(p, dev))
    d, u = api.forward_batch(shots, return_final=True)
    for i, (geom, m, eta, q) in enumerate(shots):
        ds, us = api.forward(geom, m, eta, q, return_final=True)
        torch.cuda.synchronize()
        assert torch.equal(ds, d[i]) and torch.equal(us, u[i]), i
