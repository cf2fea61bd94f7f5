"""GPU parity: the HIP library (through its C ABI) against the FP64 CPU oracle.

Bars: neighbour lists bit-exact (integer work); FP64 energies within 1e-10 relative and
forces within 1e-9 relative (normwise: max_i |dF_i| / max_i |F_i|), virial 1e-9 relative;
descriptor intermediates T and dE/dT within 1e-12 relative (normwise) - these are sums of
O(100) FP64 terms, so the expected error is ~100 ulp of the largest entry.
"""
import numpy as np
import pytest

from paper_2004_11658_amd import inputs as I
from oracle.oracle import Oracle, set_threads
from conftest import TINY, model_file, tiny_water

pytestmark = pytest.mark.gpu
set_threads(8)


@pytest.fixture(scope="module")
def dp():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2004_11658_amd import dp as D
    return D


def _cases():
    c1, t1, b1 = tiny_water(11, 2, 6.3)
    c2, t2, b2 = I.water_lattice(1, 3.2, 5)
    c3, t3, b3 = tiny_water(12, 2, 6.6)
    tric = np.array([[6.6, 0.0, 0.0], [1.3, 6.4, 0.0], [-0.9, 0.7, 6.5]])
    c3 = c3 @ np.linalg.inv(b3) @ tric
    return {"two_images": (c1, t1, b1), "self_images": (c2, t2, b2), "triclinic": (c3, t3, tric)}


def _rel(a, b):
    a, b = np.asarray(a), np.asarray(b)
    return np.abs(a - b).max() / max(np.abs(b).max(), 1e-300)


def _frel(F, Fo):
    return np.linalg.norm(F - Fo, axis=1).max() / np.linalg.norm(Fo, axis=1).max()


@pytest.mark.parametrize("case", ["two_images", "self_images", "triclinic"])
def test_nlist_small_boxes_bit_exact(dp, tiny_model, case):
    c, t, b = _cases()[case]
    print("case", case, len(t), flush=True)
    m = dp.DPModel(tiny_model)
    nl, img, nn, rc = m.nlist(c, t, b)
    o = Oracle(tiny_model)
    onl, oimg, onn, ovf = o.nlist(c, t, b)
    assert np.array_equal(nl.cpu().numpy(), onl)
    assert np.array_equal(img.cpu().numpy(), oimg)
    assert np.array_equal(nn.cpu().numpy(), onn)
    assert (rc == 1) == ovf


def test_nlist_dense_second_pass_bit_exact(dp, copper_model):
    """Compressed copper (a = 3.0 A, ~320 neighbours within rc = 8 A): every atom has more
    candidates than the first formatting pass stages, so the whole list comes from the
    second pass; bit-exact against the oracle, and E / F as well."""
    c, t, b = I.copper_fcc(6, 3.0, 17)
    m = dp.DPModel(copper_model)
    nl, img, nn, rc = m.nlist(c, t, b)
    o = Oracle(copper_model)
    onl, oimg, onn, ovf = o.nlist(c, t, b)
    assert onn.min() > 256
    assert np.array_equal(nl.cpu().numpy(), onl)
    assert np.array_equal(img.cpu().numpy(), oimg)
    assert np.array_equal(nn.cpu().numpy(), onn)
    E, F, W = m.compute(c, t, b)
    r = o.eval(c, t, b)
    assert abs(float(E.cpu()[0]) - r["E"]) <= 1e-10 * abs(r["E"])
    assert _frel(F.cpu().numpy(), r["F"]) < 1e-9


def test_nlist_perfect_lattice_ties_bit_exact(dp, copper_model):
    """Unjittered FCC copper: whole neighbour shells share one r^2, so the formatting's
    fast ranking by quantised r^2 sees ties and must fall back to the exact key
    (species, r^2, owner, image); the list is still bit-exact against the oracle."""
    c, t, b = I.copper_fcc(4, 3.634, 1, sigma=0.0)
    m = dp.DPModel(copper_model)
    nl, img, nn, rc = m.nlist(c, t, b)
    onl, oimg, onn, _ = Oracle(copper_model).nlist(c, t, b)
    assert onn.max() <= 256
    assert np.array_equal(nl.cpu().numpy(), onl)
    assert np.array_equal(img.cpu().numpy(), oimg)
    assert np.array_equal(nn.cpu().numpy(), onn)


def test_nlist_water192_bit_exact(dp, water_model, water192):
    c, t, b = water192
    m = dp.DPModel(water_model)
    nl, img, nn, rc = m.nlist(c, t, b)
    onl, oimg, onn, _ = Oracle(water_model).nlist(c, t, b)
    assert rc == 0
    assert np.array_equal(nl.cpu().numpy(), onl)
    assert np.array_equal(img.cpu().numpy(), oimg)
    assert np.array_equal(nn.cpu().numpy(), onn)


def test_descriptor_water192(dp, water_model, water192):
    c, t, b = water192
    m = dp.DPModel(water_model)
    T, gT = m.descriptor(c, t, b)
    r = Oracle(water_model).eval(c, t, b, dumps=True)
    assert _rel(T.cpu().numpy(), r["T"]) < 1e-12
    assert _rel(gT.cpu().numpy(), r["gT"]) < 1e-11


@pytest.mark.parametrize("which", ["water192", "tiny_two_images", "tiny_self_images", "tiny_triclinic"])
def test_energy_forces_virial_fp64(dp, water_model, tiny_model, water192, which):
    if which == "water192":
        path, (c, t, b) = water_model, water192
    else:
        path, (c, t, b) = tiny_model, _cases()[which[5:]]
    print("case", which, flush=True)
    m = dp.DPModel(path)
    E, F, W, Ei = m.compute(c, t, b, atom_energy=True)
    r = Oracle(path).eval(c, t, b)
    E = float(E.cpu()[0])
    assert abs(E - r["E"]) <= 1e-10 * abs(r["E"])
    assert _frel(F.cpu().numpy(), r["F"]) < 1e-9
    assert _rel(W.cpu().numpy(), r["W"]) < 1e-9
    assert _rel(Ei.cpu().numpy(), r["Ei"]) < 1e-10


def test_md_water192_fp64_matches_oracle(dp, water_model, water192):
    """20 velocity-Verlet steps: positions, velocities and thermo rows (Section 4)."""
    import torch
    c, t, b = water192
    masses = [I.MASS["O"], I.MASS["H"]]
    v = I.maxwell_velocities(t, masses, 300.0, 302)
    m = dp.DPModel(water_model)
    x_d = torch.as_tensor(c, device="cuda").clone()
    v_d = torch.as_tensor(v, device="cuda").clone()
    th = m.md_run(x_d, v_d, t, masses, b, 0.5, 20, 5).cpu().numpy()
    xo, vo, tho = Oracle(water_model).md(c, v, t, masses, b, 0.5, 20, 5)
    assert np.abs(x_d.cpu().numpy() - xo).max() < 1e-10
    assert _rel(v_d.cpu().numpy(), vo) < 1e-8
    assert np.abs(th[:, 0] - tho[:, 0]).max() == 0
    assert _rel(th[:, 1:], tho[:, 1:]) < 1e-10


def test_water12k_full_frame_fp64(dp, water_model):
    """The benchmark's 12,288-atom frame, every atom against the oracle."""
    c, t, b = I.config_water12k(202)
    m = dp.DPModel(water_model)
    nl, img, nn, rc = m.nlist(c, t, b)
    assert rc == 0
    o = Oracle(water_model)
    onl, oimg, onn, _ = o.nlist(c, t, b)
    assert np.array_equal(nl.cpu().numpy(), onl) and np.array_equal(img.cpu().numpy(), oimg)
    E, F, W, Ei = m.compute(c, t, b, atom_energy=True)
    r = o.eval(c, t, b)
    assert abs(float(E.cpu()[0]) - r["E"]) <= 1e-10 * abs(r["E"])
    assert _frel(F.cpu().numpy(), r["F"]) < 1e-9
    assert _rel(W.cpu().numpy(), r["W"]) < 1e-9
    assert _rel(Ei.cpu().numpy(), r["Ei"]) < 1e-10


def test_copper131k_sampled_fp64(dp, copper_model):
    """131,072-atom copper (one GPU's share of the paper's weak-scaling run): E_i and F_i of
    sampled atoms, each computed exactly by the oracle from the centres that see it."""
    c, t, b = I.config_copper131k(203)
    m = dp.DPModel(copper_model)
    E, F, W, Ei = m.compute(c, t, b, atom_energy=True)
    idx = np.random.default_rng(7).choice(len(t), 24, replace=False)
    oEi, oF = Oracle(copper_model).eval_sampled(c, t, b, idx)
    Fg = F.cpu().numpy()[idx]
    assert _rel(Ei.cpu().numpy()[idx], oEi) < 1e-10
    assert np.linalg.norm(Fg - oF, axis=1).max() <= 1e-9 * np.linalg.norm(oF, axis=1).max()
    # momentum: sum of all forces vanishes
    Fa = F.cpu().numpy()
    assert np.abs(Fa.sum(0)).max() <= 1e-9 * np.abs(Fa).max()


def test_ragged_batch_fp64(dp, water_model):
    """All 64 frames of uneven size (96..3,072 atoms, 102k atoms, small boxes down to
    9.9 A) in one call, every frame against the oracle."""
    import os
    set_threads(min(16, len(os.sched_getaffinity(0))))
    frames = I.ragged_water_batch(64, 204)
    sel = frames
    coords = np.concatenate([f[0] for f in sel])
    types = np.concatenate([f[1] for f in sel])
    boxes = np.stack([f[2] for f in sel])
    off = np.concatenate([[0], np.cumsum([len(f[1]) for f in sel])])
    m = dp.DPModel(water_model)
    E, F, W = m.compute_batch(coords, types, off, boxes)
    E, F, W = E.cpu().numpy(), F.cpu().numpy(), W.cpu().numpy()
    o = Oracle(water_model)
    for k, (c, t, b) in enumerate(sel):
        r = o.eval(c, t, b)
        assert abs(E[k] - r["E"]) <= 1e-10 * abs(r["E"])
        assert _frel(F[off[k]:off[k + 1]], r["F"]) < 1e-9
        assert _rel(W[k], r["W"]) < 1e-9


@pytest.mark.parametrize("skin", [0.05, 2.0])
def test_md_verlet_skin_matches_oracle(dp, water_model, water192, skin):
    """Velocity Verlet with neighbour reuse (a8: rebuild when some atom moved more than
    skin / 2; skin 0.05 A rebuilds many times in 20 steps, 2 A never): the same
    trajectory as the oracle, which builds a fresh list at every step."""
    import torch
    c, t, b = water192
    print("skin", skin, flush=True)
    masses = [I.MASS["O"], I.MASS["H"]]
    v = I.maxwell_velocities(t, masses, 300.0, 302)
    m = dp.DPModel(water_model, skin=skin)
    x_d = torch.as_tensor(c, device="cuda").clone()
    v_d = torch.as_tensor(v, device="cuda").clone()
    th = m.md_run(x_d, v_d, t, masses, b, 0.5, 20, 5).cpu().numpy()
    xo, vo, tho = Oracle(water_model).md(c, v, t, masses, b, 0.5, 20, 5)
    assert np.abs(x_d.cpu().numpy() - xo).max() < 1e-10
    assert _rel(v_d.cpu().numpy(), vo) < 1e-8
    assert _rel(th[:, 1:], tho[:, 1:]) < 1e-10


@pytest.mark.parametrize("mode", ["fp64", "bf16x3"])
def test_md_verlet_forces_equal_fresh_list(dp, water_model, mode):
    """After 60 steps of the 12,288-atom water MD with a 0.3 A skin (several rebuilds),
    the forces of the last step (reused list) equal a fresh evaluation at the same
    coordinates."""
    import torch
    c, t, b = I.config_water12k(202)
    masses = [I.MASS["O"], I.MASS["H"]]
    v = I.maxwell_velocities(t, masses, 300.0, 302)
    m = dp.DPModel(water_model, mode, skin=0.3)
    x_d = torch.as_tensor(c, device="cuda").clone()
    v_d = torch.as_tensor(v, device="cuda").clone()
    F_md = torch.empty_like(x_d)
    m.md_run(x_d, v_d, t, masses, b, 0.5, 60, 0, forces=F_md)
    E, F, W = dp.DPModel(water_model, mode).compute(x_d, t, b)
    F_md, F = F_md.cpu().numpy(), F.cpu().numpy()
    tol = 1e-12 if mode == "fp64" else 1e-6
    assert np.abs(F_md - F).max() <= tol * np.abs(F).max()


@pytest.mark.parametrize("mode", ["fp64", "bf16x3"])
def test_deterministic_forces(dp, water_model, mode):
    """Deterministic mode (pair forces stored per list slot and gathered per atom in slot
    order) gives bit-identical forces on repeated calls, and the atomic mode's forces
    up to summation order; FP64 also against the oracle on the 12,288-atom frame."""
    c, t, b = I.config_water12k(202)
    md = dp.DPModel(water_model, mode, deterministic=True)
    E1, F1, W1 = md.compute(c, t, b)
    E2, F2, W2 = md.compute(c, t, b)
    F1, F2 = F1.cpu().numpy(), F2.cpu().numpy()
    assert np.array_equal(F1, F2)
    assert np.array_equal(W1.cpu().numpy(), W2.cpu().numpy())
    Ea, Fa, Wa = dp.DPModel(water_model, mode).compute(c, t, b)
    Fa = Fa.cpu().numpy()
    assert np.abs(F1 - Fa).max() <= 1e-12 * np.abs(Fa).max()
    assert float(E1.cpu()[0]) == float(Ea.cpu()[0])
    if mode == "fp64":
        r = Oracle(water_model).eval(c, t, b)
        assert _frel(F1, r["F"]) < 1e-9


def test_deterministic_small_box_self_images(dp, tiny_model):
    """Self-images (box < 2 rc): the gather sees several slots of one owner per centre."""
    c, t, b = _cases()["self_images"]
    md = dp.DPModel(tiny_model, deterministic=True)
    E, F, W = md.compute(c, t, b)
    r = Oracle(tiny_model).eval(c, t, b)
    assert _frel(F.cpu().numpy(), r["F"]) < 1e-9
    assert abs(float(E.cpu()[0]) - r["E"]) <= 1e-10 * abs(r["E"])


def test_deterministic_rejects_student(dp, water_model):
    import torch
    md = dp.DPModel(water_model, deterministic=True)
    th = torch.zeros(4 * dp.student_size(32, 100), dtype=torch.float64, device="cuda")
    with pytest.raises(Exception):
        md.set_student(32, th, np.zeros(4), np.ones(4))
