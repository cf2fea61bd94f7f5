"""Pins of the FP64 CPU oracle against what the paper and the mathematics fix.

Each test targets a place where a plausible mistake (dropped term, wrong sign or index,
transposed operand) would show.  No value here comes from the GPU path.
"""
import itertools
import math

import numpy as np
import pytest

from paper_2004_11658_amd import inputs as I
from oracle.oracle import Oracle, set_threads
from oracle import torch_ref as TR
from conftest import TINY, TINY1, model_file, tiny_water

set_threads(4)


# ---------------------------------------------------------------------------------------
# switch function s(r) = w(r)/r  (Section 2, Eq. 5: w decays smoothly from 1 to 0 at rc)
# ---------------------------------------------------------------------------------------

def test_switch_boundary_conditions_fix_the_quintic(tiny_model):
    """w = 1 below rcs, 0 at and beyond rc; w', w'' vanish at both ends; w(mid) = 1/2.
    Six boundary conditions determine a quintic uniquely, so a wrong coefficient fails."""
    o = Oracle(tiny_model)
    rcs, rc = TINY.rcs, TINY.rc
    r = np.array([0.1, 0.3, rcs - 1e-9, rc + 1e-9, rc, 5.0, 9.0])
    s, _ = o.smooth(r)
    np.testing.assert_allclose(s[:3] * r[:3], 1.0, rtol=0, atol=1e-12)
    assert np.all(s[3:] == 0.0)
    mid = 0.5 * (rcs + rc)
    sm, _ = o.smooth(np.array([mid]))
    assert abs(sm[0] * mid - 0.5) < 1e-14

    def w(x):
        return o.smooth(np.atleast_1d(x))[0] * x

    h = 1e-4
    for x0, side in [(rcs, +1), (rc, -1)]:
        x1, x2 = x0 + side * h, x0 + side * 2 * h
        # one-sided first and second differences of w vanish like h^3 (w' = w'' = 0)
        d1 = (w(x1) - w(x0 + side * 1e-13)) / h
        d2 = (w(x2) - 2 * w(x1) + w(x0 + side * 1e-13)) / (h * h)
        assert abs(d1) < 1e-6 and abs(d2) < 1e-3
    # monotone decreasing in between
    xs = np.linspace(rcs, rc, 201)
    ws = w(xs)
    assert np.all(np.diff(ws) <= 1e-15)


def test_switch_derivative_matches_finite_difference(tiny_model):
    o = Oracle(tiny_model)
    r = np.linspace(0.2, 4.5, 77)
    _, ds = o.smooth(r)
    h = 1e-6
    fd = (o.smooth(r + h)[0] - o.smooth(r - h)[0]) / (2 * h)
    np.testing.assert_allclose(ds, fd, rtol=1e-6, atol=1e-8)


def test_environment_row_and_derivative(tiny_model):
    """R = s(r)(1, x/r, y/r, z/r) (Eq. 5) and dR/dd by central differences."""
    o = Oracle(tiny_model)
    rng = np.random.default_rng(0)
    for _ in range(20):
        d = rng.normal(size=3)
        d *= rng.uniform(0.3, 3.9) / np.linalg.norm(d)
        R, dR = o.env_row(d)
        r = np.linalg.norm(d)
        s, _ = o.smooth(np.array([r]))
        np.testing.assert_allclose(R, s[0] * np.concatenate([[1.0], d / r]), rtol=1e-14)
        h = 1e-6
        for b in range(3):
            e = np.zeros(3)
            e[b] = h
            fd = (o.env_row(d + e)[0] - o.env_row(d - e)[0]) / (2 * h)
            np.testing.assert_allclose(dR[:, b], fd, rtol=1e-6, atol=1e-9)


# ---------------------------------------------------------------------------------------
# neighbour list (Alg. 1; sorted by type, distance, index; padded per type)
# ---------------------------------------------------------------------------------------

def numpy_neighbours(coords, types, box, rc):
    """Independent enumeration: every atom j and every image n in a generous cube of
    images, kept when |x_j + n B - x_i| < rc (minimum over nothing: all images)."""
    Bi = np.linalg.inv(box)
    width = 1.0 / np.sqrt((Bi * Bi).sum(0))
    K = [int(math.ceil(rc / w)) for w in width]
    f = coords @ Bi
    xw = coords - np.floor(f) @ box
    rng_ = [range(-k - 2, k + 3) for k in K]
    out = []
    for i in range(len(types)):
        row = []
        for j in range(len(types)):
            for n in itertools.product(*rng_):
                if j == i and n == (0, 0, 0):
                    continue
                d = xw[j] + np.array(n, float) @ box - xw[i]
                r2 = float(d @ d)
                if r2 < rc * rc:
                    code = ((n[0] + K[0]) * (2 * K[1] + 1) + (n[1] + K[1])) * (2 * K[2] + 1) + n[2] + K[2]
                    row.append((int(types[j]), r2, j, code))
        out.append(sorted(row))
    return out


def _tiny_boxes():
    c1, t1, b1 = tiny_water(11, 2, 6.3)                    # box < 2 rc: several images of j
    c2, t2, b2 = I.water_lattice(1, 3.2, 5)                # box < rc: self images
    c3, t3, b3 = tiny_water(12, 2, 6.6)
    tric = np.array([[6.6, 0.0, 0.0], [1.3, 6.4, 0.0], [-0.9, 0.7, 6.5]])
    c3 = c3 @ np.linalg.inv(b3) @ tric                     # triclinic, same fractional coords
    return [(c1, t1, b1), (c2, t2, b2), (c3, t3, tric)]


@pytest.mark.parametrize("case", range(3))
def test_nlist_matches_independent_enumeration(tiny_model, case):
    o = Oracle(tiny_model)
    coords, types, box = _tiny_boxes()[case]
    nl, img, nnei, ovf = o.nlist(coords, types, box)
    ref = numpy_neighbours(coords, types, box, TINY.rc)
    off = np.concatenate([[0], np.cumsum(TINY.sel)])
    for i, row in enumerate(ref):
        for t in range(TINY.ntypes):
            blk = [(e[2], e[3]) for e in row if e[0] == t][:TINY.sel[t]]
            got_j = nl[i, off[t]:off[t + 1]]
            got_c = img[i, off[t]:off[t + 1]]
            assert nnei[i, t] == len(blk)
            assert [(int(a), int(b)) for a, b in zip(got_j[:len(blk)], got_c[:len(blk)])] == blk
            assert np.all(got_j[len(blk):] == -1)
    if case == 1:   # a 3.2 A box with rc 4 A: every atom sees images of itself
        assert any(i in nl[i] for i in range(len(types)))


def test_nlist_overflow_keeps_nearest(tmp_path):
    spec = I.ModelSpec(ntypes=2, emb_width=(4, 8, 16), fit_width=(12,), m2=4, sel=(3, 5),
                       rc=4.0, rcs=0.5)
    path = model_file("ovf", spec, 3)
    o = Oracle(path)
    coords, types, box = tiny_water(11, 2, 6.3)
    nl, img, nnei, ovf = o.nlist(coords, types, box)
    assert ovf
    ref = numpy_neighbours(coords, types, box, spec.rc)
    for i, row in enumerate(ref):
        o_only = [e[2] for e in row if e[0] == 0][:3]
        assert list(nl[i, :len(o_only)]) == o_only


def test_paper_layout_numbers():
    """O-H embedding rows of the 12,288-atom benchmark (Section 3.2.3) follow from the
    per-type-pair slot layout: 4,096 O centres x 92 H slots."""
    import json, os
    g = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_numbers.json")))
    oh = g["oh_embedding_rows"]
    c, t, b = I.config_water12k()
    n_o = int((t == 0).sum())
    assert n_o == oh["n_oxygen"] and I.WATER.sel[1] == oh["hydrogen_slots"]
    assert n_o * I.WATER.sel[1] == oh["rows"]
    assert I.WATER.emb_width[1] == oh["K"] and I.WATER.emb_width[2] == oh["N"]
    mem = g["memory_eq13"]
    gb = mem["copies"] * mem["N_l"] * mem["N_m"] * mem["M"] * mem["sizeof"] / 1e9
    assert abs(gb - mem["GB"]) < 0.005
    ws = g["water_system"]
    assert ws["cell_atoms"] * np.prod(ws["replicas"]) == ws["atoms"] == 3 * ws["molecules"]
    cu = g["copper_system"]
    assert 4 * np.prod(cu["replicas"]) == cu["atoms"]
    assert len(t) == g["water_benchmark"]["atoms"] == 3 * g["water_benchmark"]["molecules"]
    ms = g["model_shapes"]
    assert list(I.WATER.emb_width) == ms["embedding"] and list(I.WATER.fit_width) == ms["fitting"]
    assert I.WATER.rc == ms["rc_water"] and I.COPPER.rc == ms["rc_copper"]
    assert I.WATER.nm == ms["nm_water"]
    sp = g["multi_species_nets"]
    spec3 = I.ModelSpec(ntypes=sp["species"], emb_width=(4, 8), fit_width=(6,), m2=2,
                        sel=(2, 2, 2), rc=3.0, rcs=1.0)
    kinds = [k for (k, a, b, _i, _o) in spec3.layer_shapes()]
    nets_emb = len({(a, b) for (k, a, b, _i, _o) in spec3.layer_shapes() if k == "emb"})
    nets_fit = len({a for (k, a, b, _i, _o) in spec3.layer_shapes() if k == "out"})
    assert nets_emb == sp["embedding_nets"] and nets_fit == sp["fitting_nets"] and "fit" in kinds


# ---------------------------------------------------------------------------------------
# special cases with closed forms
# ---------------------------------------------------------------------------------------

def _zeroed(spec, seed, keep=()):
    """Random params with every weight block zeroed except the kinds/layers in keep."""
    p = I.random_params(spec, seed)
    off = 0
    out = p.copy()
    idx_emb = 0
    for kind, a, b, ni, no in spec.layer_shapes():
        tag = (kind, idx_emb % len(spec.emb_width)) if kind == "emb" else (kind,)
        if kind == "emb":
            idx_emb += 1
        if tag not in keep:
            out[off:off + ni * no] = 0.0
        off += ni * no + no
    return out


def test_constant_embedding_gives_closed_form_T():
    """All embedding weights zero: G = c from the biases alone, with the concat
    pattern h1 = (h0, h0) + tanh(b1), G = (h1, h1) + tanh(b2) (Eq. 8-9);
    then T = c (x) sum_j R_j / N_m (Eq. 4)."""
    spec = TINY
    p = _zeroed(spec, 21, keep={("fit",), ("out",)})
    o = Oracle(model_file("constemb", spec, 21, p))
    coords, types, box = tiny_water(11, 2, 6.3)
    r = o.eval(coords, types, box, dumps=True)
    nl, img, nnei, _ = o.nlist(coords, types, box)
    arch = TR.Arch(model_file("constemb", spec, 21, p))
    for i in [0, 3, 9, 17]:
        Rsum = np.zeros(4)
        for k in range(spec.nm):
            if nl[i, k] < 0:
                continue
        # G depends on the pair of types only; sum R per neighbour type
        for t in range(spec.ntypes):
            layers = arch.emb[(int(types[i]), t)]
            b0 = p[layers[0][2]:layers[0][2] + spec.emb_width[0]]
            b1 = p[layers[1][2]:layers[1][2] + spec.emb_width[1]]
            b2 = p[layers[2][2]:layers[2][2] + spec.emb_width[2]]
            h0 = np.tanh(b0)
            h1 = np.concatenate([h0, h0]) + np.tanh(b1)
            c = np.concatenate([h1, h1]) + np.tanh(b2)
            off = sum(spec.sel[:t])
            Rs = np.zeros(4)
            for k in range(off, off + spec.sel[t]):
                j = nl[i, k]
                if j < 0:
                    continue
                K = TR.box_K(arch, box)
                n = TR.decode_img(np.array([img[i, k]]), K)[0]
                wrapf = np.floor(coords @ np.linalg.inv(box))
                d = coords[j] - coords[i] + (n - wrapf[j] + wrapf[i]) @ box
                rr = np.linalg.norm(d)
                s, _ = o.smooth(np.array([rr]))
                Rs += s[0] * np.concatenate([[1.0], d / rr])
            Rsum += 0.0
            if t == 0:
                Texp = np.outer(c, Rs)
            else:
                Texp += np.outer(c, Rs)
        np.testing.assert_allclose(r["T"][i], Texp / spec.nm, rtol=1e-12, atol=1e-15)


def test_zero_fitting_weights_give_constant_energy():
    """All fitting weights zero: E_i = x(b) . w_o + b_o is geometry independent, F = 0, W = 0."""
    spec = TINY
    p = _zeroed(spec, 22, keep={("emb", 0), ("emb", 1), ("emb", 2), ("out",)})
    o = Oracle(model_file("zerofit", spec, 22, p))
    coords, types, box = tiny_water(11, 2, 6.3)
    r = o.eval(coords, types, box)
    assert np.abs(r["F"]).max() == 0.0 and np.abs(r["W"]).max() == 0.0
    r2 = o.eval(coords + np.random.default_rng(1).normal(0, 0.05, coords.shape), types, box)
    assert abs(r2["E"] - r["E"]) < 1e-12


def test_dimer_closed_form():
    """Two atoms far from their images.  For a single neighbour, Eq. 4-5 give
    D = (2 s^2 / N_m^2) G G<^T (since |(1, d/r)|^2 = 2), so with fitting hidden layers 2..
    zeroed, E_i = tanh(D . W1 + b1) . w_o + b_o; forces are equal and opposite along d and
    the virial is -d (x) g, rank one and symmetric."""
    spec = TINY1
    p = _zeroed(spec, 23, keep={("emb", 0), ("emb", 1), ("emb", 2), ("fit",), ("out",)})
    # zero the second fitting layer's weights and bias so that it passes x through
    arch_tmp = TR.Arch(model_file("dimer", spec, 23, p))
    W2off, (ni, no), b2off = arch_tmp.fit[0][1]
    p[W2off:W2off + ni * no] = 0.0
    p[b2off:b2off + no] = 0.0
    path = model_file("dimer", spec, 23, p)
    o = Oracle(path)
    arch = TR.Arch(path)
    box = np.diag([30.0, 30.0, 30.0])
    for rr in [0.7, 1.5, 2.4, 3.3]:
        u = np.array([0.3, -0.5, 0.8]) / np.linalg.norm([0.3, -0.5, 0.8])
        coords = np.array([[10.0, 11.0, 12.0], [10.0, 11.0, 12.0] + rr * u])
        types = np.array([0, 0], np.int32)
        r = o.eval(coords, types, box, dumps=True)
        s, _ = o.smooth(np.array([rr]))
        import torch
        G = TR.embed(arch, torch.as_tensor(p), 0, 0, torch.as_tensor(s)).numpy()[0]
        D = 2 * s[0] ** 2 / spec.nm ** 2 * np.outer(G, G[:spec.m2])
        np.testing.assert_allclose(r["D"][0], D, rtol=1e-12, atol=1e-18)
        W1off, (a1, b1n), b1off = arch.fit[0][0]
        W1 = p[W1off:W1off + a1 * b1n].reshape(a1, b1n)
        bb1 = p[b1off:b1off + b1n]
        Woff, (a3, _), boff = arch.fit[0][-1]
        wo = p[Woff:Woff + a3]
        bo = p[boff]
        Ei = np.tanh(D.reshape(-1) @ W1 + bb1) @ wo + bo
        np.testing.assert_allclose(r["E"], 2 * Ei, rtol=1e-13)
        F = r["F"]
        np.testing.assert_allclose(F[0], -F[1], rtol=1e-12, atol=1e-18)
        assert np.linalg.norm(np.cross(F[0], u)) <= 1e-10 * max(np.linalg.norm(F[0]), 1e-300)
        d = coords[1] - coords[0]
        np.testing.assert_allclose(r["W"], -np.outer(d, -F[1]) * 1.0, rtol=1e-10, atol=1e-16)
        np.testing.assert_allclose(r["W"], r["W"].T, rtol=0, atol=1e-12 * np.abs(r["W"]).max())


# ---------------------------------------------------------------------------------------
# symmetries of the descriptor (Section 2: translation, rotation, permutation)
# ---------------------------------------------------------------------------------------

def _rel(a, b):
    return np.abs(np.asarray(a) - np.asarray(b)).max() / max(np.abs(np.asarray(b)).max(), 1e-300)


def test_translation_and_lattice_shift(water_model, water192):
    o = Oracle(water_model)
    c, t, b = water192
    r0 = o.eval(c, t, b)
    r1 = o.eval(c + np.array([0.37, -1.2, 2.9]), t, b)
    assert _rel(r1["E"], r0["E"]) < 1e-12 and _rel(r1["F"], r0["F"]) < 1e-10
    c2 = c.copy()
    c2[5] += b[1] - 2 * b[2]
    r2 = o.eval(c2, t, b)
    assert _rel(r2["E"], r0["E"]) < 1e-12 and _rel(r2["F"], r0["F"]) < 1e-10


def test_rotation_cluster_in_vacuum(tiny_model):
    o = Oracle(tiny_model)
    c, t, _ = tiny_water(13, 2, 6.3)
    box = np.diag([60.0, 60.0, 60.0])
    c = c + 20.0
    r0 = o.eval(c, t, box)
    rng = np.random.default_rng(5)
    for _ in range(3):
        Q = I._rand_rotation(rng)
        cen = c.mean(0)
        cr = (c - cen) @ Q.T + cen
        r1 = o.eval(cr, t, box)
        assert _rel(r1["E"], r0["E"]) < 1e-12
        assert _rel(r1["F"], r0["F"] @ Q.T) < 1e-10
        assert _rel(r1["W"], Q @ r0["W"] @ Q.T) < 1e-10


def test_cubic_rotations_periodic(water_model, water192):
    o = Oracle(water_model)
    c, t, b = water192
    r0 = o.eval(c, t, b)
    perms = list(itertools.permutations(range(3)))
    rng = np.random.default_rng(9)
    mats = []
    for p in perms:
        for sg in itertools.product([1, -1], repeat=3):
            Q = np.zeros((3, 3))
            for i in range(3):
                Q[i, p[i]] = sg[i]
            if np.linalg.det(Q) > 0:
                mats.append(Q)
    assert len(mats) == 24
    for k in rng.choice(24, 4, replace=False):
        Q = mats[k]
        r1 = o.eval(c @ Q.T, t, b)
        assert _rel(r1["E"], r0["E"]) < 1e-12
        assert _rel(r1["F"], r0["F"] @ Q.T) < 1e-10


def test_permutation_of_same_species(water_model, water192):
    o = Oracle(water_model)
    c, t, b = water192
    r0 = o.eval(c, t, b)
    rng = np.random.default_rng(3)
    perm = np.concatenate([rng.permutation(64), 64 + rng.permutation(128)])
    perm = rng.permutation(192)          # types move with their atoms
    r1 = o.eval(c[perm], t[perm], b)
    assert _rel(r1["E"], r0["E"]) < 1e-12
    assert _rel(r1["F"], r0["F"][perm]) < 1e-10


def test_momentum_conservation(water_model, water192):
    o = Oracle(water_model)
    c, t, b = water192
    F = o.eval(c, t, b)["F"]
    assert np.abs(F.sum(0)).max() <= 1e-12 * math.sqrt(len(t)) * np.abs(F).max()


# ---------------------------------------------------------------------------------------
# derivatives: forces (Eq. 10) and virial by finite differences
# ---------------------------------------------------------------------------------------

@pytest.mark.parametrize("which", ["water", "tiny_small_box"])
def test_forces_are_minus_gradient(which, water_model, tiny_model, water192):
    if which == "water":
        o = Oracle(water_model)
        c, t, b = water192
    else:
        o = Oracle(tiny_model)
        c, t, b = I.water_lattice(1, 3.2, 5)
    F = o.eval(c, t, b)["F"]
    rng = np.random.default_rng(2)
    picks = [(int(i), int(k)) for i, k in zip(rng.integers(0, len(t), 12), rng.integers(0, 3, 12))]
    h = 1e-5
    for i, k in picks:
        cp, cm = c.copy(), c.copy()
        cp[i, k] += h
        cm[i, k] -= h
        fd = -(o.eval(cp, t, b)["E"] - o.eval(cm, t, b)["E"]) / (2 * h)
        assert abs(fd - F[i, k]) <= 1e-6 * np.abs(F).max() + 1e-6 * abs(F[i, k])


@pytest.mark.parametrize("tric", [False, True])
def test_virial_is_minus_strain_derivative(tiny_model, tric):
    o = Oracle(tiny_model)
    c, t, b = tiny_water(12, 2, 6.6)
    if tric:
        B2 = np.array([[6.6, 0.0, 0.0], [1.3, 6.4, 0.0], [-0.9, 0.7, 6.5]])
        c = c @ np.linalg.inv(b) @ B2
        b = B2
    W = o.eval(c, t, b)["W"]
    h = 1e-6
    for a in range(3):
        for bb in range(3):
            eps = np.zeros((3, 3))
            eps[a, bb] = h
            Ep = o.eval(c @ (np.eye(3) + eps), t, b @ (np.eye(3) + eps))["E"]
            Em = o.eval(c @ (np.eye(3) - eps), t, b @ (np.eye(3) - eps))["E"]
            fd = -(Ep - Em) / (2 * h)
            assert abs(fd - W[a, bb]) <= 1e-6 * np.abs(W).max()
    assert np.abs(W - W.T).max() <= 1e-12 * np.abs(W).max()


def test_hand_adjoint_equals_autograd(water_model, water192, tiny_model):
    """The C oracle's hand-written back propagation and torch autograd on an
    independently written forward agree (two derivations of Eq. 10)."""
    import torch
    for path, (c, t, b) in [(water_model, water192), (tiny_model, I.water_lattice(1, 3.2, 5))]:
        o = Oracle(path)
        r = o.eval(c, t, b)
        nl, img, _, _ = o.nlist(c, t, b)
        arch = TR.Arch(path)
        E, F, Ei = TR.energy_forces(arch, torch.as_tensor(arch.params), c, t, b, nl, img)
        assert abs(float(E.detach()) - r["E"]) <= 1e-13 * abs(r["E"])
        assert _rel(F.numpy(), r["F"]) < 1e-12
        assert _rel(Ei.detach().numpy(), r["Ei"]) < 1e-12


def test_sampled_evaluation_equals_full(water_model, water192, tiny_model):
    for path, (c, t, b) in [(water_model, water192), (tiny_model, tiny_water(11, 2, 6.3))]:
        o = Oracle(path)
        r = o.eval(c, t, b)
        idx = np.array([0, 1, 7, len(t) - 1])
        Ei, F = o.eval_sampled(c, t, b, idx)
        assert _rel(Ei, r["Ei"][idx]) < 1e-13
        assert np.abs(F - r["F"][idx]).max() < 1e-12 * np.abs(r["F"]).max()


# ---------------------------------------------------------------------------------------
# velocity Verlet (Section 4)
# ---------------------------------------------------------------------------------------

def test_md_free_flight_with_zero_forces():
    spec = TINY
    p = _zeroed(spec, 22, keep={("emb", 0), ("emb", 1), ("emb", 2), ("out",)})
    o = Oracle(model_file("zerofit", spec, 22, p))
    c, t, b = tiny_water(11, 2, 6.3)
    v = I.maxwell_velocities(t, [15.9994, 1.00794], 300.0, 3)
    x, v2, th = o.md(c, v, t, [15.9994, 1.00794], b, 0.5, 10, 5)
    np.testing.assert_allclose(x, c + 10 * 0.5 * v, rtol=0, atol=1e-12)
    np.testing.assert_allclose(v2, v, rtol=0, atol=0)
    m = np.array([15.9994, 1.00794])[t]
    ke = 0.5 * (m[:, None] * v * v).sum() * I.AMU_A2_FS2_IN_EV
    assert abs(th[0, 2] - ke) < 1e-12 * ke
    assert abs(th[0, 3] - 300.0) < 1e-9


def test_md_energy_error_scales_as_dt_squared():
    """Velocity Verlet is second order: the total-energy error falls 4x when dt halves
    (sel wide enough that no type block is ever truncated, so E is smooth)."""
    spec = I.ModelSpec(ntypes=2, emb_width=(4, 8, 16), fit_width=(12, 12, 12), m2=4,
                       sel=(30, 60), rc=4.0, rcs=0.5)
    o = Oracle(model_file("tinywide", spec, 7))
    c, t, b = tiny_water(11, 2, 6.3)
    masses = [15.9994, 1.00794]
    v = I.maxwell_velocities(t, masses, 300.0, 4)
    errs = []
    for dt, n in [(1.0, 40), (0.5, 80)]:
        _, _, th = o.md(c, v, t, masses, b, dt, n, 1)
        errs.append(np.abs(th[:, 4] - th[0, 4]).max())
    ratio = errs[0] / errs[1]
    assert 3.5 < ratio < 4.5, (errs, ratio)


# ---------------------------------------------------------------------------------------
# parameter gradient of the E + F loss, and the student net
# ---------------------------------------------------------------------------------------

def test_parameter_gradient_matches_finite_differences(tiny_model):
    """torch double back propagation vs central differences of the C oracle's loss."""
    arch = TR.Arch(tiny_model)
    o = Oracle(tiny_model)
    frames = []
    rng = np.random.default_rng(4)
    for seed, (ns, L) in [(31, (1, 3.2)), (32, (2, 6.3))]:
        c, t, b = I.water_lattice(ns, L, seed)
        nl, img, _, _ = o.nlist(c, t, b)
        r = o.eval(c, t, b)
        frames.append((c, t, b, nl, img, r["E"] + rng.normal(0, 0.3),
                       r["F"] + rng.normal(0, 0.02, r["F"].shape)))
    lam = 1.0
    th0 = arch.params.copy()
    L0, g = TR.loss_and_grad(arch, th0, frames, lam)

    def loss(th):
        o.set_params(th)
        tot = 0.0
        for (c, t, b, _nl, _img, Et, Ft) in frames:
            r = o.eval(c, t, b)
            tot += (r["E"] - Et) ** 2 / len(t) + lam * ((r["F"] - Ft) ** 2).sum()
        return tot

    assert abs(loss(th0) - L0) < 1e-12 * abs(L0)
    # every tensor: a few entries of each weight block and each bias
    picks = []
    for lay in list(arch.emb.values()) + list(arch.fit.values()):
        for (woff, (ni, no), boff) in lay:
            picks += [woff + int(rng.integers(0, ni * no)), boff + int(rng.integers(0, no))]
    h = 1e-6
    for q in picks:
        tp, tm = th0.copy(), th0.copy()
        tp[q] += h
        tm[q] -= h
        fd = (loss(tp) - loss(tm)) / (2 * h)
        assert abs(fd - g[q]) <= 1e-5 * max(abs(g[q]), 1e-3 * np.abs(g).max()), (q, fd, g[q])
    o.set_params(th0)


def test_student_gradient_and_adam():
    import torch
    H, M = 5, 7
    rng = np.random.default_rng(6)
    th = rng.normal(0, 0.5, TR.student_layout(H, M)["size"])
    s = rng.uniform(0, 1.2, 40)
    tgt = rng.normal(0, 1, (40, M))
    L, g = TR.student_loss_grad(th, H, M, s, tgt)
    h = 1e-6
    for q in range(len(th)):
        tp, tm = th.copy(), th.copy()
        tp[q] += h
        tm[q] -= h
        fd = (TR.student_loss_grad(tp, H, M, s, tgt)[0] - TR.student_loss_grad(tm, H, M, s, tgt)[0]) / (2 * h)
        assert abs(fd - g[q]) < 1e-7
    # a teacher of the student's own shape is learnable to ~0 loss
    teacher = rng.normal(0, 0.5, len(th))
    tgt = TR.student_forward(torch.as_tensor(teacher), H, M, torch.as_tensor(s)).numpy()
    m = np.zeros_like(th)
    v = np.zeros_like(th)
    cur = th.copy()
    for step in range(1, 4001):
        L, g = TR.student_loss_grad(cur, H, M, s, tgt)
        cur, m, v = TR.adam_step(cur, m, v, g, step, 1e-2 if step < 3000 else 1e-3)
    assert L < 1e-5


# ---------------------------------------------------------------------------------------
# Adam (Kingma & Ba 2015, Algorithm 1) by hand, thermo pressure, student substitution,
# thread-count independence
# ---------------------------------------------------------------------------------------

def test_adam_two_steps_by_hand():
    """Two Adam steps worked out by hand from the published definition (beta1 0.9,
    beta2 0.999, eps 1e-8, lr 0.1).  Step 1: m = 0.1 g, v = 0.001 g^2; the bias
    corrections divide by 0.1 and 0.001, so the step is lr g / (|g| + eps): 0.1 for
    g = 0.5 (up to eps) and exactly 0.05 for g = 1e-8 (where eps outside the root
    matters).  Step 2 with g = -0.25 after 0.5: m = 0.09*0.5 - 0.1*0.25 = 0.02,
    v = 0.000999*0.25 + 0.001*0.0625 = 0.00031225, corrections 1 - 0.81 = 0.19 and
    1 - 0.998001 = 0.001999.  A dropped correction or eps under the root fails."""
    lr = 0.1
    th0 = np.array([1.0, 1.0])
    g1 = np.array([0.5, 1e-8])
    g2 = np.array([-0.25, 1e-8])
    z = np.zeros(2)
    th1, m1, v1 = TR.adam_step(th0, z, z, g1, 1, lr)
    np.testing.assert_allclose(m1, [0.05, 1e-9], rtol=1e-15)
    np.testing.assert_allclose(v1, [0.00025, 1e-19], rtol=1e-15)
    step1 = np.array([0.1 * 0.5 / (0.5 + 1e-8), 0.05])
    np.testing.assert_allclose(th0 - th1, step1, rtol=1e-13)
    th2, m2, v2 = TR.adam_step(th1, m1, v1, g2, 2, lr)
    np.testing.assert_allclose(m2[0], 0.02, rtol=1e-14)
    np.testing.assert_allclose(v2[0], 0.00031225, rtol=1e-14)
    mh, vh = 0.02 / 0.19, 0.00031225 / 0.001999
    np.testing.assert_allclose(th1[0] - th2[0], 0.1 * mh / (math.sqrt(vh) + 1e-8), rtol=1e-13)
    # the second component keeps g = 1e-8: m_hat = 1e-8, v_hat = 1e-16, step lr / 2 again
    np.testing.assert_allclose(th1[1] - th2[1], 0.05, rtol=1e-12)


EV_A3_IN_BAR = 1.602176634e6      # 1 eV/A^3 = 160.2176634 GPa (exact SI definitions)


def test_thermo_ideal_gas_pressure():
    """Zero fitting weights: F = 0 and W = 0, so the thermo pressure is the kinetic one,
    P V = 2 KE / 3 = (N - 1) k_B T with T over 3N - 3 degrees of freedom.  Two atoms of
    1 amu at 1 A/fs carry KE = 1/9.64853321e-3 = 103.6427 eV (1 amu A^2/fs^2 in eV)."""
    spec = TINY
    p = _zeroed(spec, 22, keep={("emb", 0), ("emb", 1), ("emb", 2), ("out",)})
    o = Oracle(model_file("zerofit", spec, 22, p))
    c, t, b = tiny_water(11, 2, 6.3)
    V = abs(np.linalg.det(b))
    v = np.zeros_like(c)
    v[0] = [1.0, 0.0, 0.0]
    v[1] = [-1.0, 0.0, 0.0]
    masses = [1.0, 1.0]
    _, _, th = o.md(c, v, t, masses, b, 0.5, 0, 1)
    ke = 103.6426965
    assert abs(th[0, 2] - ke) < 1e-6
    assert abs(th[0, 5] - 2.0 * ke / (3.0 * V) * EV_A3_IN_BAR) < 1e-9 * abs(th[0, 5])
    kB = 8.617333262e-5
    n = len(t)
    assert abs(th[0, 5] - (n - 1) * kB * th[0, 3] / V * EV_A3_IN_BAR) < 1e-9 * abs(th[0, 5])


@pytest.mark.parametrize("tric", [False, True])
def test_thermo_pressure_is_minus_volume_derivative(tiny_model, tric):
    """At rest the thermo pressure is tr W / (3 V) (Section 4 reports pressure from the
    virial); under the isotropic scaling x -> l x, B -> l B this must equal -dE/dV,
    checked by central differences of the energy (V(l) = l^3 V)."""
    o = Oracle(tiny_model)
    c, t, b = tiny_water(11, 2, 6.3)
    if tric:
        b = b.copy()
        b[1, 0] += 0.7
        b[2, 1] -= 0.4
        b[2, 0] += 0.3
    V = np.linalg.det(b)
    _, _, th = o.md(c, np.zeros_like(c), t, [15.9994, 1.00794], b, 0.5, 0, 1)
    h = 1e-6
    Ep = o.eval(c * (1 + h), t, b * (1 + h))["E"]
    Em = o.eval(c * (1 - h), t, b * (1 - h))["E"]
    dEdl = (Ep - Em) / (2 * h)
    P_fd = -dEdl / (3.0 * V) * EV_A3_IN_BAR
    assert abs(th[0, 5] - P_fd) < 1e-6 * abs(P_fd), (th[0, 5], P_fd)
    assert th[0, 2] == 0.0


def test_student_substitution_empty_range_and_constant_student(tiny_model):
    """The student substitution of the torch reference: an s range that holds no
    neighbour leaves E bit-identical to the full net; a constant student (W2 = 0,
    b2 = c) over the whole range gives the closed form T = c (x) sum_j R_j / N_m
    (Eq. 4 with G = c) for every centre."""
    import torch
    arch = TR.Arch(tiny_model)
    o = Oracle(tiny_model)
    c, t, b = tiny_water(11, 2, 6.3)
    nl, img, _, _ = o.nlist(c, t, b)
    theta = torch.as_tensor(arch.params)
    x = torch.as_tensor(c)
    E_full, _ = TR.energy(arch, theta, x, t, b, nl, img)
    H, M = 4, arch.M
    rng = np.random.default_rng(3)
    ths = rng.normal(0, 0.5, TR.student_layout(H, M)["size"])
    empty = {(a, bb): (ths, H, -2.0, -1.0) for a in range(2) for bb in range(2)}
    E_empty, _ = TR.energy(arch, theta, x, t, b, nl, img, student=empty)
    assert float(E_empty) == float(E_full)
    cvec = rng.normal(0, 1, M)
    const = np.zeros_like(ths)
    const[2 * H + H * M:] = cvec
    full_range = {(a, bb): (const, H, 0.0, 1e9) for a in range(2) for bb in range(2)}
    out = {}
    TR.energy(arch, theta, x, t, b, nl, img, student=full_range, out=out)
    T = out["T"].numpy()
    K = TR.box_K(arch, b)
    wrapf = np.floor(c @ np.linalg.inv(b))
    for i in range(len(t)):
        Rs = np.zeros(4)
        for k in range(arch.nm):
            j = nl[i, k]
            if j < 0:
                continue
            n = TR.decode_img(np.array([img[i, k]]), K)[0]
            d = c[j] - c[i] + (n - wrapf[j] + wrapf[i]) @ b
            R, _ = o.env_row(d)
            Rs += R
        np.testing.assert_allclose(T[i], np.outer(cvec, Rs) / arch.nm, rtol=1e-12, atol=1e-15)


def test_oracle_results_independent_of_thread_count(water_model, water192):
    """Per-thread partial sums: a team wider than the old fixed 64-slot arrays gives the
    one-thread result (up to summation order)."""
    c, t, b = water192
    o = Oracle(water_model)
    set_threads(1)
    r1 = o.eval(c, t, b)
    set_threads(80)
    r2 = o.eval(c, t, b)
    set_threads(4)
    assert abs(r2["E"] - r1["E"]) < 1e-12 * abs(r1["E"])
    assert np.abs(r2["F"] - r1["F"]).max() < 1e-12 * np.abs(r1["F"]).max()
    assert np.abs(r2["W"] - r1["W"]).max() < 1e-12 * np.abs(r1["W"]).max()


# ---------------------------------------------------------------------------------------
# isobaric MD (Martyna-Tobias-Klein barostat driven by the virial pressure, optional
# Nose-Hoover thermostat), the oracle's or_md_npt
# ---------------------------------------------------------------------------------------

KB_EV = 8.617333262e-5


def _ideal_gas_oracle():
    spec = TINY
    p = _zeroed(spec, 22, keep={("emb", 0), ("emb", 1), ("emb", 2), ("out",)})
    return Oracle(model_file("zerofit", spec, 22, p))


def test_npt_ideal_gas_adiabatic_invariant():
    """With F = 0 and W = 0 the isoenthalpic equations reduce to dv/dt = -alpha v_eps v,
    dV/dt = 3 V v_eps, so KE V^(2 alpha / 3) is invariant (alpha = 1 + 3 / N_f); the
    splitting solves both exactly at constant v_eps, so the invariant holds to rounding at
    any step size while the gas is compressed far from its start (here it oscillates
    between 250 and 10 A^3 with a period of 60 fs)."""
    o = _ideal_gas_oracle()
    c, t, b = tiny_water(11, 2, 6.3)
    masses = [15.9994, 1.00794]
    v = I.maxwell_velocities(t, masses, 300.0, 3)
    n = len(t)
    alpha = 1.0 + 3.0 / (3.0 * n - 3.0)
    x, v2, box, th, st = o.md_npt(c, v, t, masses, b, 5.0e4, 40.0, 300.0, 0.0, 2.0, 60, 5)
    inv = th[:, 2] * th[:, 6] ** (2.0 * alpha / 3.0)
    assert th[:, 6].min() < 0.1 * th[0, 6]        # the box really moved
    np.testing.assert_allclose(inv, inv[0], rtol=1e-12)
    # the wrong exponent (alpha = 1, the non-MTK form) would not be invariant
    inv1 = th[:, 2] * th[:, 6] ** (2.0 / 3.0)
    assert np.abs(inv1 / inv1[0] - 1.0).max() > 1e-4
    assert abs(np.linalg.det(box) - th[-1, 6]) < 1e-9 * th[-1, 6]


def test_npt_ideal_gas_barostat_at_equilibrium():
    """P_ext equal to the ideal gas's alpha-weighted kinetic pressure alpha 2 KE / (3 V):
    the barostat force vanishes, so the box stays put and the atoms fly freely."""
    o = _ideal_gas_oracle()
    c, t, b = tiny_water(11, 2, 6.3)
    masses = [15.9994, 1.00794]
    v = I.maxwell_velocities(t, masses, 300.0, 3)
    n = len(t)
    alpha = 1.0 + 3.0 / (3.0 * n - 3.0)
    m = np.array(masses)[t]
    ke = 0.5 * (m[:, None] * v * v).sum() * I.AMU_A2_FS2_IN_EV
    V = np.linalg.det(b)
    pext = alpha * 2.0 * ke / (3.0 * V) * EV_A3_IN_BAR
    x, v2, box, th, st = o.md_npt(c, v, t, masses, b, pext, 40.0, 300.0, 0.0, 1.0, 10, 5)
    np.testing.assert_allclose(box, b, rtol=0, atol=1e-12)
    np.testing.assert_allclose(v2, v, rtol=1e-12, atol=0)
    np.testing.assert_allclose(x, c + 10 * 1.0 * v, rtol=0, atol=1e-10)
    assert abs(st[0]) < 1e-9


def test_npt_infinite_barostat_mass_is_velocity_verlet(tiny_model):
    """A barostat of huge mass (tau_p = 1e9 fs) and no thermostat leave the box fixed and
    reduce every part of the splitting to velocity Verlet: the trajectory equals or_md's."""
    o = Oracle(tiny_model)
    c, t, b = tiny_water(11, 2, 6.3)
    masses = [15.9994, 1.00794]
    v = I.maxwell_velocities(t, masses, 300.0, 4)
    x1, v1, box, th, _ = o.md_npt(c, v, t, masses, b, 1.0, 1e9, 300.0, 0.0, 0.5, 20, 5)
    x0, v0, th0 = o.md(c, v, t, masses, b, 0.5, 20, 5)
    np.testing.assert_allclose(x1, x0, rtol=0, atol=1e-10)
    np.testing.assert_allclose(v1, v0, rtol=0, atol=1e-10)
    np.testing.assert_allclose(th[:, :6], th0, rtol=1e-9, atol=1e-9)
    np.testing.assert_allclose(box, b, rtol=0, atol=1e-12)


@pytest.mark.parametrize("tau_t", [0.0, 25.0])
def test_npt_conserved_quantity_error_scales_as_dt_squared(tau_t):
    """The splitting is second order: the drift of H = E_pot + KE + p_eps^2 / 2W + P_ext V
    (+ p_xi^2 / 2Q + N_f kT xi with the thermostat) falls about 4x when dt halves."""
    spec = I.ModelSpec(ntypes=2, emb_width=(4, 8, 16), fit_width=(12, 12, 12), m2=4,
                       sel=(30, 60), rc=4.0, rcs=0.5)
    o = Oracle(model_file("tinywide", spec, 7))
    c, t, b = tiny_water(11, 2, 6.3)
    masses = [15.9994, 1.00794]
    v = I.maxwell_velocities(t, masses, 300.0, 4)
    errs = []
    for dt, n in [(1.0, 40), (0.5, 80)]:
        _, _, box, th, _ = o.md_npt(c, v, t, masses, b, 2000.0, 30.0, 300.0, tau_t, dt, n, 1)
        errs.append(np.abs(th[:, 7] - th[0, 7]).max())
        assert abs(th[-1, 6] / th[0, 6] - 1.0) > 1e-3     # the box moved
    ratio = errs[0] / errs[1]
    assert 3.5 < ratio < 4.5, (errs, ratio)


# ---------------------------------------------------------------------------------------
# per-atom outputs (the engine-facing interface): E_i and the per-centre virial W_i
# ---------------------------------------------------------------------------------------

@pytest.mark.parametrize("tric", [False, True])
def test_per_centre_virial_is_minus_strain_derivative_of_atomic_energy(tiny_model, tric):
    """E_i depends only on the relative vectors d_ij of centre i's environment (Eq. 1-5),
    so W_i = -sum_j d_ij (x) dE_i/dd_ij equals -dE_i/d(eps) under x -> x (I + eps), checked
    per atom and component by central differences; sum_i W_i = W, sum_i E_i = E.  A pair
    term assigned to the neighbour instead of the centre fails the per-atom check while
    the sums still agree; a sign error fails the sum.  (W_i is symmetric, by the
    rotational invariance of E_i, so a transposed outer product gives the same matrix.)"""
    o = Oracle(tiny_model)
    c, t, b = tiny_water(12, 2, 6.6)
    if tric:
        B2 = np.array([[6.6, 0.0, 0.0], [1.3, 6.4, 0.0], [-0.9, 0.7, 6.5]])
        c = c @ np.linalg.inv(b) @ B2
        b = B2
    r = o.eval_atomic(c, t, b)
    Wi = r["Wi"]
    np.testing.assert_allclose(Wi.sum(axis=0), r["W"], rtol=0, atol=1e-12 * np.abs(r["W"]).max())
    assert abs(r["Ei"].sum() - r["E"]) <= 1e-12 * abs(r["E"])
    h = 1e-6
    scale = np.abs(Wi).max()
    for a in range(3):
        for bb in range(3):
            eps = np.zeros((3, 3))
            eps[a, bb] = h
            Ep = o.eval_atomic(c @ (np.eye(3) + eps), t, b @ (np.eye(3) + eps))["Ei"]
            Em = o.eval_atomic(c @ (np.eye(3) - eps), t, b @ (np.eye(3) - eps))["Ei"]
            fd = -(Ep - Em) / (2 * h)
            assert np.abs(fd - Wi[:, a, bb]).max() <= 1e-6 * scale, (a, bb)
