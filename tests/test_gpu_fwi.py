"""FWI iterations around the gradient: the misfit decreases at every
accepted step and the model moves towards the true one."""
import numpy as np
import pytest
from scipy.ndimage import gaussian_filter

from paper_1609_03361_amd import synth

pytestmark = pytest.mark.gpu


def test_three_iterations_reduce_misfit_and_model_error():
    import torch
    from paper_1609_03361_amd import api, fwi
    dev = torch.device("cuda:0")
    n, nz, h = 120, 80, 10.0
    v0 = np.full((n, nz), 2000.0)
    v0 += np.linspace(0, 800, nz)[None, :]
    xx, zz = np.meshgrid(np.arange(n), np.arange(nz), indexing="ij")
    blob = np.exp(-((xx - 60) ** 2 + (zz - 40) ** 2) / (2 * 8.0 ** 2))
    v_true = v0 * (1 + 0.08 * blob)
    m0 = (1 / v0 ** 2).astype(np.float32)
    mt = (1 / v_true ** 2).astype(np.float32)
    vmax = float(v_true.max())
    eta = synth.sponge(m0, h, 20, vmax)
    dt = synth.cfl_dt(h, vmax)
    nt = 700
    q = synth.ricker(15.0, nt, dt).reshape(nt, 1)
    rec = synth.line_receivers(60, (n - 1) * h, 20.0)
    shots = []
    e = torch.from_numpy(eta).to(dev)
    for sx in (200.0, 600.0, 1000.0):
        geom = api.Geometry((n, nz), (h, h), 8, dt, nt, np.array([[sx, 20.0]]), rec)
        qq = torch.from_numpy(q).to(dev)
        d_obs = api.forward(geom, torch.from_numpy(mt).to(dev), e, qq)
        shots.append((geom, qq, d_obs))
    mask = torch.zeros((n, nz), dtype=torch.float32, device=dev)
    mask[25:n - 25, 10:nz - 25] = 1.0
    # velocity bounds keep every update inside the time step's stability limit
    state = fwi.FWIState(shots, e, vmin=1500.0, vmax=1.15 * vmax, mask=mask)
    m = torch.from_numpy(m0).to(dev)
    mt_d = torch.from_numpy(mt).to(dev)
    err0 = float((m - mt_d).norm())
    Js = []
    for it in range(3):
        m, J, a = fwi.fwi_iteration(state, m)
        Js.append(J)
        print(f"iteration {it}: J0 {state.history[-1]['J0']:.4e} -> J {J:.4e} (step {a})", flush=True)
        assert a > 0
    assert Js[0] < state.history[0]["J0"] and Js[1] < Js[0] and Js[2] < Js[1]
    assert float((m - mt_d).norm()) < err0
