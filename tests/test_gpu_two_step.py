"""Temporal blocking: the two-step 2D body (tile variant 4 of the batched
forward and of the single-shot forward without checkpoints) computes levels
n+1 and n+2 in one pass.  Every point's arithmetic
is that of a single step, so the traces and final wavefields must equal the
one-step slab's bit for bit, for even and odd step counts (an odd count
starts with one step), with and without the graph; and the oracle must agree
to the usual FP32 bar."""
import numpy as np
import pytest

from gpu_util import assert_close, device_inputs, oracle_forward
from paper_1609_03361_amd import synth

pytestmark = pytest.mark.gpu

ONE_STEP = 3
TWO_STEP = 4


@pytest.fixture(scope="module")
def dev():
    import torch
    assert torch.cuda.is_available()
    return torch.device("cuda:0")


def _random_shots(dev, order, nt, seed):
    """Shots of several sizes sharing order, nt and dt: z spans of one to
    three tiles of the two-step slab (256 - 2 RZ owned points) with ragged
    tails, x extents that leave a short last chunk, sources and receivers at
    random spots, on the grid corners and on a shared spot (so injected rows
    fall inside the widened rows of neighbouring chunks and tiles)."""
    shapes = [(70, 530), (45, 260), (33, 301), (19, 77)]
    probs = [synth.random_problem(s, order, nt, seed=seed + k, nsrc=6, nrec=9)
             for k, s in enumerate(shapes)]
    dt = min(p.dt for p in probs)
    for p in probs:
        p.dt = dt
    return probs, [device_inputs(p, dev) for p in probs]


def _equal(a, b):
    import torch
    return all(torch.equal(x, y) for x, y in zip(a, b))


@pytest.mark.parametrize("order,nt", [(8, 40), (8, 41), (2, 17), (4, 30), (12, 23), (16, 26)])
def test_two_step_equals_one_step_bitwise(dev, order, nt):
    import torch
    from paper_1609_03361_amd import api
    probs, shots = _random_shots(dev, order, nt, seed=100 + order)
    print(f"order {order} nt {nt}: shapes {[p.shape for p in probs]}", flush=True)
    d1, u1 = api.forward_batch(shots, return_final=True, tile=api.tile_id(ONE_STEP, 0))
    for graph in (True, False):
        for x in (0, 7, 16):
            d2, u2 = api.forward_batch(shots, return_final=True, graph=graph,
                                       tile=api.tile_id(TWO_STEP, x))
            torch.cuda.synchronize()
            assert _equal(d1, d2), (graph, x, "traces")
            assert _equal(u1, u2), (graph, x, "u^nt")


def test_two_step_single_step_run(dev):
    """nt = 1: the run is the one-step start alone (no pass, no final sampling)."""
    import torch
    from paper_1609_03361_amd import api
    probs, shots = _random_shots(dev, 8, 1, seed=7)
    a = api.forward_batch(shots, return_final=True, tile=api.tile_id(ONE_STEP, 0))
    b = api.forward_batch(shots, return_final=True, tile=api.tile_id(TWO_STEP, 0))
    torch.cuda.synchronize()
    assert _equal(a[0], b[0]) and _equal(a[1], b[1])


def test_two_step_batched_shots_equal_single_shots_and_oracle(dev):
    """The batched-shot workload's geometry at reduced size: two-step batch
    against each shot run alone (bitwise) and against the oracle."""
    import torch
    from paper_1609_03361_amd import api
    probs = synth.config_batched_2d(nshots=4, nx=401, nz=301, nt=151, wmin=90, nrec=41)
    shots = [device_inputs(p, dev) for p in probs]
    d, u = api.forward_batch(shots, return_final=True, tile=api.tile_id(TWO_STEP, 0))
    torch.cuda.synchronize()
    for i, (geom, m, eta, q) in enumerate(shots):
        ds, us = api.forward(geom, m, eta, q, return_final=True)
        torch.cuda.synchronize()
        assert torch.equal(ds, d[i]) and torch.equal(us, u[i]), i
    for i in (0, 3):
        ref = oracle_forward(probs[i])
        assert_close(d[i].cpu().numpy(), ref["d"], f"two-step {probs[i].name} traces")
        assert_close(u[i].cpu().numpy(), ref["u"], f"two-step {probs[i].name} u^nt")


def test_two_step_rejected_where_a_step_at_a_time_is_needed(dev):
    """The checkpointed forward, the adjoint and the gradient take one step
    per launch: the two-step tile is an argument error there."""
    import torch
    from paper_1609_03361_amd import api, _lib
    p = synth.random_problem((30, 40), 8, 4, seed=2)
    geom, m, eta, q = device_inputs(p, dev)
    d = api.forward(geom, m, eta, q)
    tile = api.tile_id(TWO_STEP, 0)
    ck = torch.empty(api.checkpoint_bytes(geom, 2), dtype=torch.uint8, device=dev)
    calls = [lambda: api.forward(geom, m, eta, q, checkpoint=ck, ckpt_every=2, tile=tile),
             lambda: api.adjoint(geom, m, eta, d, tile=tile),
             lambda: api.gradient(geom, m, eta, q, d, ckpt_every=2, tile=tile)]
    for call in calls:
        with pytest.raises(_lib.WaveError) as e:
            call()
        assert e.value.code == _lib.WAVE_EINVAL


def test_persistent_batch_maps_the_two_step_tile_to_single_steps(dev):
    import torch
    from paper_1609_03361_amd import api
    probs, shots = _random_shots(dev, 8, 20, seed=11)
    a = api.forward_batch(shots, return_final=True, tile=api.tile_id(ONE_STEP, 0))
    b = api.forward_batch(shots, return_final=True, persistent=True, tile=api.tile_id(TWO_STEP, 0))
    torch.cuda.synchronize()
    assert _equal(a[0], b[0]) and _equal(a[1], b[1])


def test_tuner_times_the_two_step_slab(dev):
    """The batch tuner's candidates include the two-step slab; whatever it
    picks, results are bitwise those of the one-step slab."""
    import os
    import torch
    from paper_1609_03361_amd import api
    probs, shots = _random_shots(dev, 8, 12, seed=21)
    ref = api.forward_batch(shots, return_final=True, tile=api.tile_id(ONE_STEP, 0))
    os.environ["WAVE_TUNE_VERBOSE"] = "1"
    try:
        tile, us = api.tune_batch(shots, steps=4)
    finally:
        del os.environ["WAVE_TUNE_VERBOSE"]
    print(f"batch tile variant {tile >> 16} x-chunk {tile & 0xffff}: {us:.2f} us/step", flush=True)
    got = api.forward_batch(shots, return_final=True)
    torch.cuda.synchronize()
    assert _equal(ref[0], got[0]) and _equal(ref[1], got[1])


@pytest.mark.parametrize("order,nt,nsrc", [(8, 40, 3), (8, 33, 70), (4, 21, 5), (16, 24, 4)])
def test_single_shot_forward_two_step_equals_one_step(dev, order, nt, nsrc):
    """wave_forward without checkpoints on a 2D grid with tile variant 4 runs
    as a batch of one shot on the two-step body: traces and u^nt bitwise those
    of the one-step path (70 sources: a dense set, whose one-step run gathers
    the injection values a step ahead)."""
    import torch
    from paper_1609_03361_amd import api
    p = synth.random_problem((83, 530), order, nt, seed=300 + order + nsrc, nsrc=nsrc, nrec=17)
    geom, m, eta, q = device_inputs(p, dev)
    a = api.forward(geom, m, eta, q, return_final=True, tile=api.tile_id(ONE_STEP, 0))
    for x in (0, 24):
        b = api.forward(geom, m, eta, q, return_final=True, tile=api.tile_id(TWO_STEP, x))
        torch.cuda.synchronize()
        assert torch.equal(a[0], b[0]) and torch.equal(a[1], b[1]), x
