"""Three species: the species-generic paths of the HIP library against the FP64 oracle.

The other GPU tests use models with one or two species.  Here a third species (a second
oxygen-like label drawn at random for half of the O atoms, the atom order shuffled so
that the species interleave) runs the code that loops over an arbitrary species count:
the list filter of the Verlet list, the (species, distance, index) ordering with three
sel blocks of odd widths, three centre-species row groups in the fitting kernels and in
the parameter gradient, nine embedding nets and nine student nets.

Bars as in the two-species tests: neighbour lists bit-exact; FP64 energy 1e-10, forces
1e-9 (normwise), virial 1e-9; FP32 and split-BF16 force RMSE 1e-3 against FP64; MD
positions 1e-10 A after 20 steps; parameter gradient 1e-9 of its largest entry.
"""
import dataclasses

import numpy as np
import pytest

from paper_2004_11658_amd import inputs as I
from oracle.oracle import Oracle, set_threads
from oracle import torch_ref as TR
from conftest import model_file, tiny_water

pytestmark = pytest.mark.gpu
set_threads(8)

# small nets, sel widths that are not multiples of 4 or of a tile
TRI = I.ModelSpec(ntypes=3, emb_width=(4, 8, 16), fit_width=(12, 12, 12), m2=4,
                  sel=(9, 27, 7), rc=4.0, rcs=0.5)
# the water model's nets and cut-off, its oxygen block split in two
WATER3 = dataclasses.replace(I.WATER, ntypes=3, sel=(29, 92, 27))
MASSES = [I.MASS["O"], I.MASS["H"], 18.998]


@pytest.fixture(scope="module")
def dp():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2004_11658_amd import dp as D
    return D


@pytest.fixture(scope="module")
def tri_model():
    return model_file("tri", TRI, 9)


@pytest.fixture(scope="module")
def water3_model():
    return model_file("water3", WATER3, 105)


def three_species(frame, seed):
    """Half of the O atoms (at random) become species 2; then the atoms are shuffled."""
    c, t, b = frame
    rng = np.random.Generator(np.random.PCG64(seed))
    t = t.copy()
    t[(t == 0) & (rng.random(len(t)) < 0.5)] = 2
    p = rng.permutation(len(t))
    return np.ascontiguousarray(c[p]), np.ascontiguousarray(t[p], dtype=np.int32), b


def _small_frames():
    c1, t1, b1 = tiny_water(11, 2, 6.3)
    c2, t2, b2 = tiny_water(12, 2, 6.6)
    tric = np.array([[6.6, 0.0, 0.0], [1.3, 6.4, 0.0], [-0.9, 0.7, 6.5]])
    c2 = c2 @ np.linalg.inv(b2) @ tric
    return {"tiny_cubic": three_species((c1, t1, b1), 21),
            "tiny_triclinic": three_species((c2, t2, tric), 22),
            "water192": three_species(I.config_water192(), 23)}


def _rel(a, b):
    a, b = np.asarray(a), np.asarray(b)
    return np.abs(a - b).max() / max(np.abs(b).max(), 1e-300)


def _frel(F, Fo):
    return np.linalg.norm(F - Fo, axis=1).max() / np.linalg.norm(Fo, axis=1).max()


def _case(which, tri_model, water3_model):
    frame = _small_frames()[which]
    return (water3_model if which == "water192" else tri_model), frame


@pytest.mark.parametrize("which", ["tiny_cubic", "tiny_triclinic", "water192"])
def test_three_species_nlist_bit_exact(dp, tri_model, water3_model, which):
    path, (c, t, b) = _case(which, tri_model, water3_model)
    print("nlist three species", which, np.bincount(t), flush=True)
    nl, img, nn, rc = dp.DPModel(path).nlist(c, t, b)
    onl, oimg, onn, ovf = Oracle(path).nlist(c, t, b)
    assert np.array_equal(nl.cpu().numpy(), onl)
    assert np.array_equal(img.cpu().numpy(), oimg)
    assert np.array_equal(nn.cpu().numpy(), onn)
    assert (rc == 1) == ovf


@pytest.mark.parametrize("which", ["tiny_cubic", "tiny_triclinic", "water192"])
def test_three_species_energy_forces_virial_fp64(dp, tri_model, water3_model, which):
    path, (c, t, b) = _case(which, tri_model, water3_model)
    print("fp64 three species", which, flush=True)
    E, F, W, Ei = dp.DPModel(path).compute(c, t, b, atom_energy=True)
    r = Oracle(path).eval(c, t, b)
    assert abs(float(E.cpu()[0]) - r["E"]) <= 1e-10 * abs(r["E"])
    assert _frel(F.cpu().numpy(), r["F"]) < 1e-9
    assert _rel(W.cpu().numpy(), r["W"]) < 1e-9
    assert _rel(Ei.cpu().numpy(), r["Ei"]) < 1e-10


@pytest.mark.parametrize("mode", ["fp32", "bf16x3"])
def test_three_species_precision_modes(dp, water3_model, mode):
    """1536 atoms (512 molecules): several row tiles of every species in the fitting
    kernels, with ragged tails."""
    c, t, b = three_species(I.water_lattice(8, 24.84, 24), 25)
    print("mode", mode, "three species", np.bincount(t), flush=True)
    r = Oracle(water3_model).eval(c, t, b)
    E, F, W = dp.DPModel(water3_model, mode).compute(c, t, b)
    F = F.cpu().numpy()
    err = float(np.sqrt(((F - r["F"]) ** 2).mean()) / np.sqrt((r["F"] ** 2).mean()))
    eE = abs(float(E.cpu()[0]) - r["E"]) / np.abs(r["Ei"]).sum()
    print("mode %s force rmse %.3e energy %.3e" % (mode, err, eE), flush=True)
    assert np.isfinite(F).all()
    assert err < 1e-3 and eE < 1e-3


@pytest.mark.parametrize("skin", [0.05, 2.0])
def test_three_species_md_verlet_matches_oracle(dp, water3_model, skin):
    """20 steps of velocity Verlet with the Verlet list (skin 0.05 A rebuilds often, 2 A
    never) against the oracle's fresh list at every step."""
    import torch
    c, t, b = _small_frames()["water192"]
    print("md three species skin", skin, flush=True)
    v = I.maxwell_velocities(t, MASSES, 300.0, 303)
    m = dp.DPModel(water3_model, skin=skin)
    x_d = torch.as_tensor(c, device="cuda").clone()
    v_d = torch.as_tensor(v, device="cuda").clone()
    th = m.md_run(x_d, v_d, t, MASSES, b, 0.5, 20, 5).cpu().numpy()
    xo, vo, tho = Oracle(water3_model).md(c, v, t, MASSES, b, 0.5, 20, 5)
    assert np.abs(x_d.cpu().numpy() - xo).max() < 1e-10
    assert _rel(v_d.cpu().numpy(), vo) < 1e-8
    assert _rel(th[:, 1:], tho[:, 1:]) < 1e-10


def test_three_species_param_grad_matches_oracle(dp, tri_model):
    import torch
    fr = _small_frames()
    frames = [fr["tiny_cubic"], fr["tiny_triclinic"], three_species(I.water_lattice(1, 3.2, 31), 26)]
    print("param grad three species", [len(f[1]) for f in frames], flush=True)
    o = Oracle(tri_model)
    rng = np.random.default_rng(6)
    tg = []
    for (c, t, b) in frames:
        r = o.eval(c, t, b)
        tg.append((r["E"] + rng.normal(0, 0.5), r["F"] + rng.normal(0, 0.02, r["F"].shape)))
    arch = TR.Arch(tri_model)
    ofr = []
    for (c, t, b), (Et, Ft) in zip(frames, tg):
        nl, img, _, _ = o.nlist(c, t, b)
        ofr.append((c, t, b, nl, img, Et, Ft))
    L_ref, g_ref = TR.loss_and_grad(arch, arch.params, ofr, 1.0)
    m = dp.DPModel(tri_model)
    coords = np.concatenate([f[0] for f in frames])
    types = np.concatenate([f[1] for f in frames])
    boxes = np.stack([f[2] for f in frames])
    off = np.concatenate([[0], np.cumsum([len(f[1]) for f in frames])])
    theta = torch.as_tensor(arch.params, device="cuda").clone().requires_grad_(True)
    E, F = dp.DPEnergyForce.apply(theta, m, coords, types, off, boxes)
    Et = torch.as_tensor([x[0] for x in tg], device="cuda")
    Ft = torch.as_tensor(np.concatenate([x[1] for x in tg]), device="cuda")
    nat = torch.as_tensor(np.diff(off), device="cuda", dtype=torch.float64)
    L = (((E - Et) ** 2) / nat).sum() + ((F - Ft) ** 2).sum()
    L.backward()
    g = theta.grad.cpu().numpy()
    assert abs(float(L) - L_ref) <= 1e-10 * abs(L_ref)
    err = np.abs(g - g_ref).max() / np.abs(g_ref).max()
    print("grad rel err", err, flush=True)
    assert err < 1e-9


@pytest.mark.parametrize("prec", ["fp64", "bf16x3"])
def test_three_species_student_inference_matches_oracle(dp, water3_model, prec):
    """Nine random students with narrow ranges (part of the neighbours fall back to the
    full net): E and F against the oracle's substituted model."""
    import torch
    c, t, b = _small_frames()["water192"]
    H, M, nt = 32, 100, 3
    rng = np.random.default_rng(7)
    ths = [rng.normal(0, 0.3, dp.student_size(H, M)) for _ in range(nt * nt)]
    lo = rng.uniform(0.05, 0.1, nt * nt)
    hi = rng.uniform(0.5, 0.7, nt * nt)
    m = dp.DPModel(water3_model, prec)
    m.set_student(H, torch.as_tensor(np.concatenate(ths), device="cuda"), lo, hi)
    E, F, W = m.compute(c, t, b)
    arch = TR.Arch(water3_model)
    nl, img, _, _ = Oracle(water3_model).nlist(c, t, b)
    st = {(a, bb): (ths[nt * a + bb], H, lo[nt * a + bb], hi[nt * a + bb])
          for a in range(nt) for bb in range(nt)}
    Er, Fr, _ = TR.energy_forces(arch, torch.as_tensor(arch.params), c, t, b, nl, img, student=st)
    Er, Fr = float(Er.detach()), Fr.numpy()
    tolE, tolF = {"fp64": (1e-10, 1e-9), "bf16x3": (6.1e-5, 1e-3)}[prec]
    dE = abs(float(E.cpu()[0]) - Er) / abs(Er)
    dF = np.linalg.norm(F.cpu().numpy() - Fr, axis=1).max() / np.linalg.norm(Fr, axis=1).max()
    print(prec, "three species student dE", dE, "dF", dF, flush=True)
    assert dE < tolE and dF < tolF
