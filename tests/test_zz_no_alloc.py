"""wave_forward_noalloc (the entry point for callers that cannot allocate)
against wave_forward through the C ABI: bitwise equal outputs on two calls in
a row, the second on a smaller grid (so the shared device array still holds
the first call's larger contents), no torch allocation during the calls, and
a clear WAVE_EWORKSPACE for a grid whose workspace exceeds the array."""
import ctypes as C

import numpy as np
import pytest

from gpu_util import device_inputs, oracle_forward, rel_l2
from paper_1609_03361_amd import synth

pytestmark = pytest.mark.gpu


def _noalloc(p, geom, m, eta, q, dev):
    import torch
    from paper_1609_03361_amd import _lib as L
    sp, rp = geom.points()
    d = torch.empty((p.nt, rp.npts), dtype=torch.float32, device=dev)
    u = torch.empty(p.shape, dtype=torch.float32, device=dev)
    before = torch.cuda.memory_allocated(dev)
    stream = C.c_void_p(torch.cuda.current_stream(dev).cuda_stream)
    rc = L.lib().wave_forward_noalloc(C.byref(geom.grid()), m.data_ptr(), eta.data_ptr(),
                                      C.byref(sp.s), q.data_ptr(), C.byref(rp.s), d.data_ptr(),
                                      u.data_ptr(), stream)
    L.check(rc, "wave_forward_noalloc")
    assert torch.cuda.memory_allocated(dev) == before
    return d, u


def test_noalloc_forward_equals_forward_on_two_calls():
    import torch
    from paper_1609_03361_amd import api
    dev = torch.device("cuda:0")
    cases = [synth.random_problem((61, 47, 70), 8, 50, seed=11, nsrc=3, nrec=20),
             synth.random_problem((37, 41), 4, 80, seed=12, nsrc=2, nrec=9)]
    for p in cases:
        print(f"case {p.name}", flush=True)
        geom, m, eta, q = device_inputs(p, dev)
        d0, u0 = api.forward(geom, m, eta, q, return_final=True)
        d1, u1 = _noalloc(p, geom, m, eta, q, dev)
        torch.cuda.synchronize()
        assert torch.equal(d0, d1) and torch.equal(u0, u1)
        ref = oracle_forward(p)
        assert rel_l2(d1.cpu().numpy(), ref["d"]) < 1e-5
        assert rel_l2(u1.cpu().numpy(), ref["u"]) < 1e-5


def test_noalloc_rejects_a_grid_beyond_its_array():
    import torch
    from paper_1609_03361_amd import _lib as L
    from paper_1609_03361_amd import api
    dev = torch.device("cuda:0")
    shape = (200, 200, 120)            # 4 fields x 19.2 MB: above 64 MiB
    p = synth.random_problem((8, 8, 8), 4, 3, seed=1, nsrc=1, nrec=1)
    geom = api.Geometry(shape, (10.0,) * 3, 4, 1e-4, 3, p.src, p.rec)
    m = torch.full(shape, 1 / 1500.0 ** 2, device=dev)
    eta = torch.zeros(shape, device=dev)
    q = torch.zeros((3, 1), device=dev)
    with pytest.raises(L.WaveError) as e:
        _noalloc(p, geom, m, eta, q, dev)
    assert e.value.code == L.WAVE_EWORKSPACE
    assert "no-allocation" in str(e.value)
