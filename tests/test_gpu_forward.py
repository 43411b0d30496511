"""Forward parity: the HIP path (through the C ABI) against the FP64 oracle
on the same seeded inputs.  Tolerance: relative L2 <= 1e-5 and max-abs /
max-ref <= 1e-5 on the traces and on the final wavefield.  On the 101^2
order-4 workload the FP32 build of the oracle is run too: the GPU error must
stay within twice that FP32 round-off floor."""
import numpy as np
import pytest

from gpu_util import assert_close, device_inputs, oracle_forward, record, rel_l2
from paper_1609_03361_amd import synth

pytestmark = pytest.mark.gpu
TOL = 1e-5


@pytest.fixture(scope="module")
def dev():
    import torch
    assert torch.cuda.is_available()
    return torch.device("cuda:0")


def _run(p, dev):
    import torch
    from paper_1609_03361_amd import api
    geom, m, eta, q = device_inputs(p, dev)
    d, u = api.forward(geom, m, eta, q, return_final=True)
    torch.cuda.synchronize()
    return d.cpu().numpy(), u.cpu().numpy()


def test_2d_101_order4_full(dev):
    p = synth.config_2d_small()
    print(f"case {p.name} nt={p.nt}", flush=True)
    d, u = _run(p, dev)
    ref = oracle_forward(p)
    r32 = oracle_forward(p, precision="f32")
    floor_d, floor_u = rel_l2(r32["d"], ref["d"]), rel_l2(r32["u"], ref["u"])
    ed, _ = assert_close(d, ref["d"], f"{p.name} traces", fp32_oracle=floor_d)
    eu, _ = assert_close(u, ref["u"], f"{p.name} u^nt", fp32_oracle=floor_u)
    print(f"FP32 oracle floor: traces {floor_d:.3e}, u {floor_u:.3e}", flush=True)
    assert ed <= 2 * floor_d and eu <= 2 * floor_u


SWEEP = [((37, 29), 2, 40), ((61, 70), 4, 50), ((45, 131), 6, 40), ((33, 65), 8, 60),
         ((70, 47), 10, 40), ((41, 52), 12, 40), ((39, 44), 14, 40), ((50, 67), 16, 50),
         ((13, 17, 19), 2, 30), ((21, 18, 33), 4, 30), ((17, 23, 70), 6, 25),
         ((24, 26, 65), 8, 30), ((19, 31, 22), 10, 20), ((25, 20, 29), 12, 20),
         ((18, 27, 33), 14, 20), ((33, 29, 37), 16, 25)]


@pytest.mark.parametrize("shape,order,nt", SWEEP)
def test_random_sweep(dev, shape, order, nt):
    p = synth.random_problem(shape, order, nt, seed=order + len(shape), nsrc=4, nrec=11)
    print(f"case {p.name}", flush=True)
    d, u = _run(p, dev)
    ref = oracle_forward(p)
    assert_close(d, ref["d"], f"{p.name} traces")
    assert_close(u, ref["u"], f"{p.name} u^nt")


def test_3d_64_order8_200_steps(dev):
    p = synth.config_3d_o8(n=64, nt=200, nrec_side=16, width=10)
    print(f"case {p.name}", flush=True)
    d, u = _run(p, dev)
    ref = oracle_forward(p)
    assert_close(d, ref["d"], f"{p.name} traces")
    assert_close(u, ref["u"], f"{p.name} u^nt")


def test_no_sources_no_receivers_and_zero_field(dev):
    import torch
    from paper_1609_03361_amd import api
    p = synth.random_problem((20, 24), 4, 5, seed=3)
    geom, m, eta, q = device_inputs(p, dev)
    geom.src = None
    d, u = api.forward(geom, m, eta, None, return_final=True)
    torch.cuda.synchronize()
    assert d.shape == (5, p.rec.shape[0]) and float(d.abs().max()) == 0.0
    assert float(u.abs().max()) == 0.0


def test_deterministic_bitwise(dev):
    import torch
    from paper_1609_03361_amd import api
    p = synth.random_problem((30, 31, 29), 8, 20, seed=9, nsrc=5, nrec=20)
    geom, m, eta, q = device_inputs(p, dev)
    a = api.forward(geom, m, eta, q, return_final=True)
    b = api.forward(geom, m, eta, q, return_final=True)
    torch.cuda.synchronize()
    assert torch.equal(a[0], b[0]) and torch.equal(a[1], b[1])


def test_cfl_and_field_errors(dev):
    import torch
    from paper_1609_03361_amd import api, _lib
    p = synth.random_problem((20, 22), 8, 5, seed=4)
    geom, m, eta, q = device_inputs(p, dev)
    geom.dt = p.dt * 2.0          # CFL 0.8 > the order-8 2D bound 0.5546
    with pytest.raises(_lib.WaveError) as e:
        api.forward(geom, m, eta, q)
    assert e.value.code == _lib.WAVE_ECFL
    geom.dt = p.dt
    bad = m.clone()
    bad[3, 4] = float("nan")
    with pytest.raises(_lib.WaveError) as e:
        api.forward(geom, bad, eta, q)
    assert e.value.code == _lib.WAVE_EINVAL
    neg = eta.clone()
    neg[1, 1] = -1.0
    with pytest.raises(_lib.WaveError) as e:
        api.forward(geom, m, neg, q)
    assert e.value.code == _lib.WAVE_EINVAL
