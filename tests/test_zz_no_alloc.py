"""dp_compute_noalloc (workspace in the library's built-in scratch array) against
dp_compute (caller workspace), through the C ABI: two calls in a row, the second on a
smaller frame, on a deterministic handle (results must be bit-identical: same kernels,
same summation order) and on an atomics handle (E, virial within 1e-12 and F within
1e-12 of the largest force, the size of FP64 atomic reordering); plus the host-side
rejection of a frame whose workspace exceeds the array."""
import ctypes as C

import numpy as np
import pytest

from paper_2004_11658_amd import inputs as I

pytestmark = pytest.mark.gpu

DP_ERR_WORKSPACE = -6


@pytest.fixture(scope="module")
def dp():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2004_11658_amd import dp as D
    L = D.lib()
    L.dp_compute_noalloc.argtypes = [C.c_void_p, C.c_int64] + [C.c_void_p] * 7 + [C.c_void_p]
    L.dp_compute_noalloc.restype = C.c_int
    return D


def _noalloc(dp, m, coords, types, box):
    import torch
    x = torch.as_tensor(np.ascontiguousarray(coords, dtype=np.float64), device="cuda")
    t = torch.as_tensor(np.ascontiguousarray(types, dtype=np.int32), device="cuda")
    b9 = np.ascontiguousarray(np.asarray(box, dtype=np.float64).reshape(9))
    n = len(types)
    E = torch.full((1,), np.nan, dtype=torch.float64, device="cuda")
    F = torch.full((n, 3), np.nan, dtype=torch.float64, device="cuda")
    W = torch.full((9,), np.nan, dtype=torch.float64, device="cuda")
    Ei = torch.full((n,), np.nan, dtype=torch.float64, device="cuda")
    st = C.c_void_p(torch.cuda.current_stream().cuda_stream)
    rc = dp.lib().dp_compute_noalloc(m.h, n, C.c_void_p(x.data_ptr()), C.c_void_p(t.data_ptr()),
                                     b9.ctypes.data_as(C.c_void_p), C.c_void_p(E.data_ptr()),
                                     C.c_void_p(F.data_ptr()), C.c_void_p(W.data_ptr()),
                                     C.c_void_p(Ei.data_ptr()), st)
    torch.cuda.synchronize()
    return rc, E, F, W.view(3, 3), Ei


def _frames():
    big = I.config_water192()                       # 192 atoms, 12.42 A cube
    small = I.water_lattice(3, 9.3, 31)             # 81 atoms, 9.3 A cube (images within rc)
    return [big, small]


@pytest.mark.parametrize("deterministic", [True, False])
def test_noalloc_matches_compute_two_calls(dp, water_model, deterministic):
    m = dp.DPModel(water_model, deterministic=deterministic)
    for k, (c, t, b) in enumerate(_frames()):
        print("noalloc call", k, "atoms", len(t), "deterministic", deterministic, flush=True)
        rc, E, F, W, Ei = _noalloc(dp, m, c, t, b)
        assert rc == 0, dp.lib().dp_last_error(m.h)
        Er, Fr, Wr, Eir = m.compute(c, t, b, atom_energy=True)
        assert np.isfinite(F.cpu().numpy()).all()
        if deterministic:
            assert np.array_equal(E.cpu().numpy(), Er.cpu().numpy())
            assert np.array_equal(F.cpu().numpy(), Fr.cpu().numpy())
            assert np.array_equal(W.cpu().numpy(), Wr.cpu().numpy())
            assert np.array_equal(Ei.cpu().numpy(), Eir.cpu().numpy())
        else:
            e, er = float(E.cpu()[0]), float(Er.cpu()[0])
            assert abs(e - er) <= 1e-12 * abs(er)
            Fn, Frn = F.cpu().numpy(), Fr.cpu().numpy()
            assert np.abs(Fn - Frn).max() <= 1e-12 * np.abs(Frn).max()
            Wn, Wrn = W.cpu().numpy(), Wr.cpu().numpy()
            assert np.abs(Wn - Wrn).max() <= 1e-12 * np.abs(Wrn).max()
            assert np.abs(Ei.cpu().numpy() - Eir.cpu().numpy()).max() <= 1e-12 * np.abs(Eir.cpu().numpy()).max()


def test_noalloc_rejects_frames_beyond_the_array(dp, water_model):
    m = dp.DPModel(water_model)
    c, t, b = I.config_water12k(202)
    print("noalloc oversize", len(t), flush=True)
    rc, E, F, W, Ei = _noalloc(dp, m, c, t, b)
    assert rc == DP_ERR_WORKSPACE
    assert b"scratch array" in dp.lib().dp_last_error(m.h)
    assert np.isnan(E.cpu().numpy()).all()          # nothing was launched


def test_noalloc_capacity_report(dp, water_model):
    """Prints the workspace of water frames of growing size (FP64) against the array's
    64 MiB; the largest lattice that fits must run through the entry point."""
    import ctypes as C
    m = dp.DPModel(water_model, deterministic=True)
    L = dp.lib()
    fit = None
    for k in (4, 5, 6, 7, 8, 9):
        c, t, b = I.water_lattice(k, 12.42 * k / 4, 40 + k)
        off = np.array([0, len(t)], dtype=np.int64)
        b9 = np.ascontiguousarray(np.asarray(b, dtype=np.float64).reshape(9))
        nb = C.c_size_t()
        assert L.dp_workspace_size(m.h, 1, off.ctypes.data_as(C.c_void_p), b9.ctypes.data_as(C.c_void_p),
                                   C.byref(nb)) == 0
        print("water atoms", len(t), "workspace MiB", nb.value / 2 ** 20, flush=True)
        if nb.value <= 64 << 20:
            fit = (c, t, b)
    assert fit is not None
    c, t, b = fit
    rc, E, F, W, Ei = _noalloc(dp, m, c, t, b)
    assert rc == 0
    Er, Fr, Wr = m.compute(c, t, b)
    assert np.array_equal(F.cpu().numpy(), Fr.cpu().numpy())
