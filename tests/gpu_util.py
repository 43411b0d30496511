"""Helpers shared by the GPU tests: move a synthetic problem to the device,
run the HIP path through the C ABI and the oracle on the same inputs, and
compare them.

Parity is judged by two numbers: the relative L2 error over the whole array
(the benchmark spec's tolerance, 1e-5 for FP32 results) and the largest pointwise
error relative to the largest reference magnitude, which a localized error
at one tile or chunk edge cannot hide under.  With WAVE_ACCURACY_LOG set,
every comparison is appended to that file as one JSON line."""
import json
import os

import numpy as np

import oracle

# max |got - ref| / max |ref|: pointwise FP32 rounding of a wavefield is of the
# order of the field's own relative error, so the same 1e-5 bound applies to
# the largest pointwise deviation as to the L2 norm
MAX_TOL = 1e-5


def rel_l2(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    nb = np.linalg.norm(b)
    return float(np.linalg.norm(a - b) / nb) if nb > 0 else float(np.linalg.norm(a))


def max_rel(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    mb = float(np.max(np.abs(b))) if b.size else 0.0
    if b.size == 0:
        return 0.0
    return float(np.max(np.abs(a - b)) / mb) if mb > 0 else float(np.max(np.abs(a)))


def record(label, **values):
    """Append one measurement to the accuracy log (if WAVE_ACCURACY_LOG is set)."""
    path = os.environ.get("WAVE_ACCURACY_LOG")
    if not path:
        return
    os.makedirs(os.path.dirname(os.path.abspath(path)), exist_ok=True)
    with open(path, "a") as f:
        f.write(json.dumps({"label": label, **values}) + "\n")


def assert_close(got, ref, label, tol=1e-5, tol_max=MAX_TOL, **extra):
    """Relative L2 <= tol and max-abs / max-ref <= tol_max; both printed and logged."""
    e2, em = rel_l2(got, ref), max_rel(got, ref)
    print(f"{label}: rel L2 {e2:.3e} (tol {tol:.0e}), max {em:.3e} (tol {tol_max:.0e})", flush=True)
    record(label, rel_l2=e2, max_rel=em, tol=tol, tol_max=tol_max, **extra)
    assert e2 <= tol, (label, e2)
    assert em <= tol_max, (label, em)
    return e2, em


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
