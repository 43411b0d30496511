"""C-ABI checks that need no GPU: the library loads, exports every entry
point declared in include/wave.h, and rejects bad arguments with the
documented codes before touching the device."""
import ctypes as C
import os
import re

import numpy as np
import pytest

from paper_1609_03361_amd import _lib as L

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    text = open(os.path.join(ROOT, "include", "wave.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(wave_[a-z_]+)\s*\(", text)))


def test_library_exports_every_declared_function():
    names = declared_functions()
    assert set(names) == set(L.EXPORTS), names
    lib = L.lib()
    for n in names:
        assert hasattr(lib, n), n
    assert b"gfx950" in lib.wave_version()


def _size(op, shape=(20, 30), spacing=(10.0, 10.0), order=8, dt=1e-3, nt=10, src=None, rec=None,
          **kw):
    g = L.make_grid(shape, spacing, order, dt, nt)
    sp = L.HostPoints(src, len(shape))
    rp = L.HostPoints(rec, len(shape))
    o = L.make_opts(**kw)
    n = C.c_size_t(0)
    rc = L.lib().wave_workspace_size(op, C.byref(g), C.byref(sp.s), C.byref(rp.s), C.byref(o),
                                     C.byref(n))
    return rc, n.value


def test_workspace_size_grows_with_op_and_points():
    rc, f = _size(L.WAVE_OP_FORWARD)
    assert rc == 0 and f >= 4 * 20 * 30 * 4
    rc, a = _size(L.WAVE_OP_ADJOINT)
    assert rc == 0
    rc, g = _size(L.WAVE_OP_GRADIENT)
    assert rc == 0 and g > f
    rc, f2 = _size(L.WAVE_OP_FORWARD, rec=np.zeros((1000, 2)))
    assert rc == 0 and f2 > f


@pytest.mark.parametrize("kw,code", [
    (dict(order=3), L.WAVE_EINVAL), (dict(order=18), L.WAVE_EINVAL), (dict(order=0), L.WAVE_EINVAL),
    (dict(nt=0), L.WAVE_EINVAL), (dict(dt=0.0), L.WAVE_EINVAL), (dict(dt=float("nan")), L.WAVE_EINVAL),
    (dict(shape=(1, 30)), L.WAVE_EINVAL), (dict(spacing=(0.0, 1.0)), L.WAVE_EINVAL),
    (dict(shape=(4, 4, 4, 4), spacing=(1, 1, 1, 1)), L.WAVE_EINVAL),
])
def test_workspace_size_rejects_bad_grids(kw, code):
    rc, _ = _size(L.WAVE_OP_FORWARD, **kw)
    assert rc == code
    assert L.lib().wave_last_error()


def _forward_rc(shape=(20, 30), src=((50.0, 50.0),), rec=((10.0, 20.0),), ws=True, ws_bytes=None,
                q=True, d=True, m=True, tile=0):
    nd = len(shape)
    g = L.make_grid(shape, (10.0,) * nd, 4, 1e-3, 5)
    sp = L.HostPoints(src, nd)
    rp = L.HostPoints(rec, nd)
    fake = 1 << 20          # never dereferenced: every case fails validation first
    o = L.make_opts(fake if ws else 0, ws_bytes if ws_bytes is not None else 1 << 40, tile=tile)
    rc = L.lib().wave_forward(C.byref(g), fake if m else None, None, C.byref(sp.s),
                              fake if q else None, C.byref(rp.s), fake if d else None, None, None,
                              C.byref(o), None)
    return rc


def _gpu_visible():
    try:
        import torch
        return torch.cuda.device_count() > 0
    except Exception:
        return False


@pytest.mark.skipif(_gpu_visible(), reason="uses placeholder device pointers; CPU-only check")
def test_forward_argument_errors_return_before_any_device_work():
    assert _forward_rc(m=False) == L.WAVE_EINVAL
    assert _forward_rc(q=False) == L.WAVE_EINVAL
    assert _forward_rc(d=False) == L.WAVE_EINVAL
    assert _forward_rc(src=((-1.0, 5.0),)) == L.WAVE_ERANGE
    assert _forward_rc(rec=((190.0, 290.0 + 1e-6),)) == L.WAVE_ERANGE
    assert _forward_rc(ws=False) == L.WAVE_EWORKSPACE
    assert _forward_rc(ws_bytes=1024) == L.WAVE_EWORKSPACE
    assert b"workspace" in L.lib().wave_last_error()
    # block shapes: 4 in 2D (ids 0..3, and 4 = two steps per pass), 11 in 3D (ids 0..10)
    assert _forward_rc(tile=(5 << 16) | 8) == L.WAVE_EINVAL
    assert b"variant 5" in L.lib().wave_last_error()
    assert _forward_rc(tile=-1) == L.WAVE_EINVAL
    assert _forward_rc(shape=(20, 30, 40), src=((50.0, 50.0, 50.0),), rec=((10.0, 20.0, 30.0),),
                       tile=(11 << 16) | 8) == L.WAVE_EINVAL


def test_library_fields_use_rows_padded_to_four_points():
    """Rows inside the workspace and the checkpoints hold nz rounded up to a
    multiple of 4: nz = 801..804 need the same bytes, nz = 805 more."""
    sizes = [_size(L.WAVE_OP_GRADIENT, shape=(40, nz))[1] for nz in (801, 802, 803, 804, 805)]
    assert len(set(sizes[:4])) == 1 and sizes[4] > sizes[3]
    ck = []
    for nz in (801, 804, 805):
        g = L.make_grid((40, nz), (10.0, 10.0), 8, 1e-3, 100)
        n = C.c_size_t(0)
        assert L.lib().wave_checkpoint_size(C.byref(g), C.byref(L.make_opts()), C.byref(n)) == 0
        ck.append(n.value)
    assert ck[0] == ck[1] < ck[2]


def test_checkpoint_size_scales_with_dtype_and_interval():
    g = L.make_grid((30, 40, 50), (10.0,) * 3, 8, 1e-3, 100)
    sizes = {}
    for dt_, every in (("fp32", 20), ("bf16", 20), ("fp16", 20), ("fp32", 10)):
        n = C.c_size_t(0)
        o = L.make_opts(ckpt_every=every, ckpt_dtype=dt_)
        assert L.lib().wave_checkpoint_size(C.byref(g), C.byref(o), C.byref(n)) == 0
        sizes[(dt_, every)] = n.value
    N = 30 * 40 * 50
    assert sizes[("fp32", 20)] >= 5 * 2 * N * 4
    assert sizes[("bf16", 20)] < 0.6 * sizes[("fp32", 20)]
    assert sizes[("fp16", 20)] == sizes[("bf16", 20)]
    assert sizes[("fp32", 10)] > 1.9 * sizes[("fp32", 20)]


def test_python_api_imports_without_gpu():
    from paper_1609_03361_amd import api
    import paper_1609_03361_amd as pkg
    assert pkg.Geometry is api.Geometry and callable(pkg.wave_apply)
    g = api.Geometry((10, 12), (5.0, 5.0), 4, 1e-3, 7)
    assert g.grid().nt == 7


def test_batch_rejects_mismatched_shots_before_device_work():
    g1 = L.make_grid((20, 30), (10.0, 10.0), 8, 1e-3, 10)
    g2 = L.make_grid((25, 30), (10.0, 10.0), 8, 1e-3, 11)
    arr = (L.Shot * 2)()
    for s, g in zip(arr, (g1, g2)):
        s.grid = g
        s.m = 1 << 20
    n = C.c_size_t(0)
    assert L.lib().wave_batch_workspace_size(2, arr, None, C.byref(n)) == L.WAVE_EINVAL
    assert b"same ndim" in L.lib().wave_last_error()
    arr[1].grid = L.make_grid((25, 30), (10.0, 10.0), 8, 1e-3, 10)
    assert L.lib().wave_batch_workspace_size(2, arr, None, C.byref(n)) == 0 and n.value > 0


def test_workspace_of_each_op_holds_only_what_it_touches():
    rec = np.zeros((50, 2))
    src = np.zeros((2, 2))
    sizes = {op: _size(op, src=src, rec=rec, nt=100)[1]
             for op in (L.WAVE_OP_FORWARD, L.WAVE_OP_ADJOINT, L.WAVE_OP_GRADIENT,
                        L.WAVE_OP_FORWARD_CKPT, L.WAVE_OP_BACKWARD)}
    # forward with caller-owned checkpoints: the forward plus 4 KiB of reduction
    # scratch (the codec's maxima), no ring, no adjoint fields
    assert sizes[L.WAVE_OP_FORWARD] < sizes[L.WAVE_OP_FORWARD_CKPT] <= sizes[L.WAVE_OP_FORWARD] + 4096 + 256
    # backward: ring of ckpt_every + 1 fields, adjoint pair and accumulator, no checkpoints
    assert sizes[L.WAVE_OP_BACKWARD] < sizes[L.WAVE_OP_GRADIENT]
    rc, ck = 0, C.c_size_t(0)
    g = L.make_grid((20, 30), (10.0, 10.0), 8, 1e-3, 100)
    assert L.lib().wave_checkpoint_size(C.byref(g), C.byref(L.make_opts()), C.byref(ck)) == 0
    assert sizes[L.WAVE_OP_GRADIENT] >= sizes[L.WAVE_OP_BACKWARD] + ck.value
    rc, bad = _size(5)
    assert rc == L.WAVE_EINVAL


@pytest.mark.parametrize("shape", [(2001, 801), (101, 101), (5, 9), (256, 256, 256), (48, 48, 48)])
@pytest.mark.parametrize("order", [4, 8, 16])
def test_tile_candidates_are_distinct_launches(shape, order):
    from paper_1609_03361_amd import api
    geom = api.Geometry(shape, (10.0,) * len(shape), order, 1e-3, 10)
    ids = api.tile_candidates(geom)
    assert len(ids) == len(set(ids)) > 0
    for t in ids:
        variant, xc = t >> 16, t & 0xFFFF
        assert 1 <= xc <= shape[0]
        if len(shape) == 2 and variant == 3:
            assert xc <= 16                  # the slab holds at most 16 rows
        # the tile the launch uses is the candidate itself
        assert api.resolve_tile(geom, t) == t


def test_tile_candidates_include_every_split_into_2_to_32_chunks():
    """The tuner's x-chunks include every split of the grid into 2..32 chunks
    of at least 2R planes (on 200^3 order 8 the best plain step sits at 17
    planes, between the fixed lengths), besides the fixed lengths 2R, 4R,
    8 .. 128."""
    from paper_1609_03361_amd import api
    geom = api.Geometry((200, 200, 200), (10.0,) * 3, 8, 1e-3, 10)
    ids = set(api.tile_candidates(geom))
    for k in range(2, 33):
        x = -(-200 // k)
        assert x < 8 or ((3 << 16) | x) in ids, x
    assert ((3 << 16) | 7) not in ids             # shorter than 2R
    for x in (8, 16, 32, 64, 128):
        assert (3 << 16) | x in ids, x


def test_resolve_tile_clamps_requests():
    from paper_1609_03361_amd import api
    geom = api.Geometry((2001, 801), (10.0, 10.0), 8, 1e-3, 10)
    assert api.resolve_tile(geom, (3 << 16) | 64) == (3 << 16) | 16
    assert api.resolve_tile(geom, (0 << 16) | 5000) == (0 << 16) | 2001
    with pytest.raises(L.WaveError):
        api.resolve_tile(geom, 9 << 16)


def test_two_step_variant_scope_and_workspace():
    """2D tile variant 4 (two steps per pass) is accepted by the batched
    forward and by the single-shot forward without checkpoints (as a batch of
    one shot), resolves to columns of 64 rows when planned, and is not among
    the single-shot tuner's candidates; a 2D batch workspace holds the second
    wavefield pair its passes write (3D batches keep one pair), and the 2D
    forward workspace covers the one-shot batch."""
    from paper_1609_03361_amd import api
    geom = api.Geometry((2001, 801), (10.0, 10.0), 8, 1e-3, 10)
    assert all(t >> 16 != 4 for t in api.tile_candidates(geom))
    assert api.resolve_tile(geom, 4 << 16) == (4 << 16) | 64
    assert api.resolve_tile(geom, (4 << 16) | 40) == (4 << 16) | 40
    g = L.make_grid((2001, 801), (10.0, 10.0), 8, 1e-3, 10)
    sp = L.HostPoints(((5000.0, 25.0),), 2)
    rp = L.HostPoints(((100.0, 20.0), (200.0, 20.0)), 2)
    fwd = C.c_size_t(0)
    assert L.lib().wave_workspace_size(L.WAVE_OP_FORWARD, C.byref(g), C.byref(sp.s), C.byref(rp.s),
                                       None, C.byref(fwd)) == 0
    arr = (L.Shot * 1)()
    arr[0].grid = g
    arr[0].m = 1 << 20
    arr[0].src.npts, arr[0].rec.npts = 1, 2
    arr[0].q, arr[0].d = 1 << 20, 1 << 20
    one = C.c_size_t(0)
    assert L.lib().wave_batch_workspace_size(1, arr, None, C.byref(one)) == 0
    assert fwd.value >= one.value

    def batch_bytes(shape):
        arr = (L.Shot * 1)()
        arr[0].grid = L.make_grid(shape, (10.0,) * len(shape), 8, 1e-3, 10)
        arr[0].m = 1 << 20
        n = C.c_size_t(0)
        assert L.lib().wave_batch_workspace_size(1, arr, None, C.byref(n)) == 0
        return n.value

    # fields use rows padded to 4 points; growing nx by one adds one row of each
    # per-point array: alpha, beta and the wavefields
    r2 = batch_bytes((41, 64)) - batch_bytes((40, 64))
    assert abs(r2 - 6 * 64 * 4) < 64 * 4
    r3 = batch_bytes((11, 8, 64)) - batch_bytes((10, 8, 64))
    assert abs(r3 - 4 * 8 * 64 * 4) < 8 * 64 * 4
