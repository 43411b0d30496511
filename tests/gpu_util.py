"""Helpers shared by the GPU tests: move a synthetic problem to the device,
run the HIP path through the C ABI and the oracle on the same inputs."""
import numpy as np

import oracle


def rel_l2(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    nb = np.linalg.norm(b)
    return float(np.linalg.norm(a - b) / nb) if nb > 0 else float(np.linalg.norm(a))


def device_inputs(p, dev):
    import torch
    from paper_1609_03361_amd import api
    geom = api.Geometry(p.shape, p.spacing, p.order, p.dt, p.nt, p.src, p.rec)
    m = torch.from_numpy(np.ascontiguousarray(p.m)).to(dev)
    eta = None if p.eta is None else torch.from_numpy(np.ascontiguousarray(p.eta)).to(dev)
    q = torch.from_numpy(np.ascontiguousarray(p.q)).to(dev)
    return geom, m, eta, q


def oracle_forward(p, **kw):
    return oracle.forward(p.shape, p.spacing, p.order, p.dt, p.nt, p.m, p.eta, p.src, p.q, p.rec,
                          **kw)
