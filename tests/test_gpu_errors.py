"""Error and warning codes of the C ABI, forced on the device through dp.h's entry points,
plus two handles computing on two streams at once.

Each device-detected condition is made by an input the library's own checks turn into a
status flag (a type out of range, a NaN coordinate, two atoms at one position, more than
DP_MAX_CANDIDATES atoms within rc of an atom, a type block fuller than sel); every kernel
still runs to completion on clamped or zeroed values, and dp_status reports the code.
Host-detected conditions (a singular box, a short workspace or weight buffer, calls
before dp_upload, NULL arguments) return before anything is launched.
"""
import ctypes as C

import numpy as np
import pytest

from paper_2004_11658_amd import inputs as I
from oracle.oracle import Oracle, set_threads
from conftest import TINY, tiny_water

pytestmark = pytest.mark.gpu
set_threads(8)

DP_WARN_SEL_OVERFLOW, DP_ERR_ARG, DP_ERR_BOX, DP_ERR_TYPE = 1, -1, -3, -4
DP_ERR_CAPACITY, DP_ERR_WORKSPACE, DP_ERR_NONFINITE, DP_ERR_OVERLAP = -5, -6, -8, -9


@pytest.fixture(scope="module")
def dp():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2004_11658_amd import dp as D
    return D


def _code(dp, fn):
    try:
        fn()
    except dp.DPError as e:
        return e.code
    return 0


def test_err_box_singular(dp, tiny_model):
    c, t, b = tiny_water(11, 2, 6.3)
    m = dp.DPModel(tiny_model)
    bad = np.array(b, dtype=np.float64).copy()
    bad[2] = bad[0] + bad[1]           # c = a + b: zero volume
    print("case singular box", flush=True)
    assert _code(dp, lambda: m.compute(c, t, bad)) == DP_ERR_BOX
    left = np.array(b, dtype=np.float64)[[1, 0, 2]]   # left-handed
    assert _code(dp, lambda: m.compute(c, t, left)) == DP_ERR_BOX


def test_err_type_out_of_range(dp, tiny_model):
    c, t, b = tiny_water(11, 2, 6.3)
    t = np.array(t, dtype=np.int32)
    t[3] = 7
    m = dp.DPModel(tiny_model)
    print("case bad type", flush=True)
    assert _code(dp, lambda: m.compute(c, t, b)) == DP_ERR_TYPE


def test_err_nonfinite_coordinate(dp, tiny_model):
    c, t, b = tiny_water(11, 2, 6.3)
    c = np.array(c, dtype=np.float64)
    c[5, 1] = np.nan
    m = dp.DPModel(tiny_model)
    print("case NaN coordinate", flush=True)
    assert _code(dp, lambda: m.compute(c, t, b)) == DP_ERR_NONFINITE


def test_err_overlap(dp, tiny_model):
    c, t, b = tiny_water(11, 2, 6.3)
    c = np.array(c, dtype=np.float64)
    c[9] = c[8]
    m = dp.DPModel(tiny_model)
    print("case coincident atoms", flush=True)
    assert _code(dp, lambda: m.compute(c, t, b)) == DP_ERR_OVERLAP


def test_err_capacity_too_many_candidates(dp, water_model):
    # 11^3 atoms on a 0.5 A grid (max distance from the centre 4.3 A < rc = 6 A) in a
    # 40 A box: the centre atom has 1,330 atoms within rc, above DP_MAX_CANDIDATES = 1024
    g = np.arange(11) * 0.5
    c = np.stack(np.meshgrid(g, g, g, indexing="ij"), -1).reshape(-1, 3) + 17.5
    t = (np.arange(len(c)) % 2).astype(np.int32)
    b = np.eye(3) * 40.0
    m = dp.DPModel(water_model)
    print("case capacity", len(c), flush=True)
    assert _code(dp, lambda: m.compute(c, t, b)) == DP_ERR_CAPACITY


def test_warn_sel_overflow_keeps_nearest(dp, tiny_model):
    # tiny model: sel 12 / 24 within rc = 4 A; a 4x4x4 grid of alternating species at
    # 1.2 A spacing gives inner atoms more than 12 species-0 neighbours: the warning,
    # with the nearest 12 kept on both sides (oracle and library), so results still agree
    g = np.arange(4) * 1.2
    c = np.stack(np.meshgrid(g, g, g, indexing="ij"), -1).reshape(-1, 3) + 4.0
    c = c + np.random.default_rng(3).uniform(-0.05, 0.05, c.shape)
    t = (np.arange(len(c)) % 2).astype(np.int32)
    b = np.eye(3) * 12.0
    m = dp.DPModel(tiny_model)
    print("case sel overflow", flush=True)
    E, F, W = m.compute(c, t, b, check=False)
    assert m.status() == DP_WARN_SEL_OVERFLOW
    r = Oracle(tiny_model).eval(c, t, b)
    assert r["overflow"]
    assert abs(float(E.cpu()[0]) - r["E"]) <= 1e-10 * abs(r["E"])
    Fo = r["F"]
    assert np.linalg.norm(F.cpu().numpy() - Fo, axis=1).max() <= 1e-9 * np.linalg.norm(Fo, axis=1).max()


def test_err_workspace_and_weight_buffer(dp, tiny_model):
    import torch
    L = dp.lib()
    c, t, b = tiny_water(11, 2, 6.3)
    m = dp.DPModel(tiny_model)
    x = torch.as_tensor(c, device="cuda")
    ty = torch.as_tensor(t, dtype=torch.int32, device="cuda")
    b9 = np.ascontiguousarray(np.asarray(b, dtype=np.float64).reshape(9))
    E = torch.empty(1, dtype=torch.float64, device="cuda")
    F = torch.empty(len(t), 3, dtype=torch.float64, device="cuda")
    ws = torch.empty(4096, dtype=torch.uint8, device="cuda")
    print("case short workspace", flush=True)
    rc = L.dp_compute(m.h, len(t), C.c_void_p(x.data_ptr()), C.c_void_p(ty.data_ptr()),
                      b9.ctypes.data_as(C.c_void_p), C.c_void_p(E.data_ptr()), C.c_void_p(F.data_ptr()),
                      None, None, C.c_void_p(ws.data_ptr()), ws.numel(), None)
    assert rc == DP_ERR_WORKSPACE
    assert b"workspace" in L.dp_last_error(m.h)
    # a weight buffer one byte short, and a misaligned one
    nb = C.c_size_t()
    assert L.dp_device_bytes(m.h, C.byref(nb)) == 0
    buf = torch.empty(nb.value + 512, dtype=torch.uint8, device="cuda")
    assert L.dp_upload(m.h, C.c_void_p(buf.data_ptr()), nb.value - 1, None) == DP_ERR_WORKSPACE
    assert L.dp_upload(m.h, C.c_void_p(buf.data_ptr() + 8), nb.value, None) == DP_ERR_ARG
    # the handle's own region is still bound: results unchanged
    E1, F1, _ = m.compute(c, t, b)
    r = Oracle(tiny_model).eval(c, t, b)
    assert abs(float(E1.cpu()[0]) - r["E"]) <= 1e-10 * abs(r["E"])


def test_err_arg_before_upload_and_nulls(dp, tiny_model):
    import torch
    L = dp.lib()
    h = C.c_void_p()
    assert L.dp_init(tiny_model.encode(), None, C.byref(h)) == 0
    try:
        c, t, b = tiny_water(11, 2, 6.3)
        x = torch.as_tensor(c, device="cuda")
        ty = torch.as_tensor(t, dtype=torch.int32, device="cuda")
        b9 = np.ascontiguousarray(np.asarray(b, dtype=np.float64).reshape(9))
        E = torch.empty(1, dtype=torch.float64, device="cuda")
        F = torch.empty(len(t), 3, dtype=torch.float64, device="cuda")
        ws = torch.empty(1 << 24, dtype=torch.uint8, device="cuda")
        args = (h, len(t), C.c_void_p(x.data_ptr()), C.c_void_p(ty.data_ptr()), b9.ctypes.data_as(C.c_void_p),
                C.c_void_p(E.data_ptr()), C.c_void_p(F.data_ptr()), None, None, C.c_void_p(ws.data_ptr()),
                ws.numel(), None)
        print("case no upload", flush=True)
        assert L.dp_compute(*args) == DP_ERR_ARG
        assert b"dp_upload" in L.dp_last_error(h)
        nb = C.c_size_t()
        L.dp_device_bytes(h, C.byref(nb))
        wbuf = torch.empty(nb.value, dtype=torch.uint8, device="cuda")
        assert L.dp_upload(h, C.c_void_p(wbuf.data_ptr()), wbuf.numel(), None) == 0
        # NULL outputs and coordinates
        bad = list(args)
        bad[5] = None
        assert L.dp_compute(*bad) == DP_ERR_ARG
        bad = list(args)
        bad[2] = None
        assert L.dp_compute(*bad) == DP_ERR_ARG
        assert L.dp_compute(*args) == 0
        torch.cuda.synchronize()
        r = Oracle(tiny_model).eval(c, t, b)
        assert abs(float(E.cpu()[0]) - r["E"]) <= 1e-10 * abs(r["E"])
    finally:
        L.dp_free(h)


def test_err_arg_atom_counts(dp, tiny_model):
    """An empty frame (alone or inside a ragged batch) and a batch above 2^26 atoms are
    rejected on the host with DP_ERR_ARG, before anything is launched."""
    import torch
    L = dp.lib()
    m = dp.DPModel(tiny_model, "fp64")
    c, t, b = tiny_water(11, 2, 6.3)
    n = len(t)
    b9 = np.ascontiguousarray(np.tile(np.asarray(b, dtype=np.float64).reshape(9), 3))
    nb = C.c_size_t()
    for case, off in (("empty frame", [0, 0]), ("empty middle frame", [0, n, n, 2 * n]),
                      ("decreasing offsets", [0, n, n - 1, 2 * n]), ("above 2^26 atoms", [0, (1 << 26) + 1])):
        print("case", case, flush=True)
        o = np.asarray(off, dtype=np.int64)
        nf = len(off) - 1
        assert L.dp_workspace_size(m.h, nf, o.ctypes.data_as(C.c_void_p), b9.ctypes.data_as(C.c_void_p),
                                   C.byref(nb)) == DP_ERR_ARG
        assert L.dp_last_error(m.h)
    # the evaluations themselves: nothing launched, outputs untouched
    x = torch.as_tensor(np.vstack([c, c]), device="cuda")
    ty = torch.as_tensor(np.concatenate([t, t]), dtype=torch.int32, device="cuda")
    E = torch.full((3,), 7.0, dtype=torch.float64, device="cuda")
    F = torch.full((2 * n, 3), 7.0, dtype=torch.float64, device="cuda")
    ws = torch.empty(1 << 24, dtype=torch.uint8, device="cuda")
    print("case dp_compute natoms 0", flush=True)
    assert L.dp_compute(m.h, 0, C.c_void_p(x.data_ptr()), C.c_void_p(ty.data_ptr()),
                        b9.ctypes.data_as(C.c_void_p), C.c_void_p(E.data_ptr()), C.c_void_p(F.data_ptr()),
                        None, None, C.c_void_p(ws.data_ptr()), ws.numel(), None) == DP_ERR_ARG
    print("case dp_compute_batch empty middle frame", flush=True)
    o = np.asarray([0, n, n, 2 * n], dtype=np.int64)
    assert L.dp_compute_batch(m.h, 3, o.ctypes.data_as(C.c_void_p), C.c_void_p(x.data_ptr()),
                              C.c_void_p(ty.data_ptr()), b9.ctypes.data_as(C.c_void_p), C.c_void_p(E.data_ptr()),
                              C.c_void_p(F.data_ptr()), None, None, C.c_void_p(ws.data_ptr()), ws.numel(),
                              None) == DP_ERR_ARG
    torch.cuda.synchronize()
    assert bool((E == 7.0).all()) and bool((F == 7.0).all())
    # the handle still works after the rejected calls
    En, Fn, _ = m.compute(torch.as_tensor(c, device="cuda"), torch.as_tensor(t, dtype=torch.int32, device="cuda"), b)
    r = Oracle(tiny_model).eval(c, t, b)
    assert abs(float(En.cpu()[0]) - r["E"]) <= 1e-10 * abs(r["E"])


def test_two_handles_on_two_streams(dp, tiny_model, water_model, water192):
    """Two handles, each with its own workspace, launched on two streams back to back
    without a synchronisation between them: both results equal the serial ones."""
    import torch
    c1, t1, b1 = tiny_water(11, 2, 6.3)
    c2, t2, b2 = water192
    m1 = dp.DPModel(tiny_model, deterministic=True)
    m2 = dp.DPModel(water_model, deterministic=True)
    ref1 = [v.clone() for v in m1.compute(c1, t1, b1)]
    ref2 = [v.clone() for v in m2.compute(c2, t2, b2)]
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    x1 = torch.as_tensor(c1, device="cuda")
    x2 = torch.as_tensor(c2, device="cuda")
    torch.cuda.synchronize()
    print("case two streams", flush=True)
    outs = []
    for _ in range(3):
        with torch.cuda.stream(s1):
            o1 = m1.compute(x1, t1, b1, check=False)
        with torch.cuda.stream(s2):
            o2 = m2.compute(x2, t2, b2, check=False)
        outs.append((o1, o2))
    torch.cuda.synchronize()
    for o1, o2 in outs:
        for a, r in zip(o1, ref1):
            assert torch.equal(a, r)
        for a, r in zip(o2, ref2):
            assert torch.equal(a, r)
