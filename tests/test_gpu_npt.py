"""Isobaric MD and triclinic production MD on the GPU against the oracle.

dp_md_run_npt (isotropic Martyna-Tobias-Klein barostat on the virial pressure, optional
Nose-Hoover thermostat, Verlet list with skin checked against the scaled reference
positions) follows or_md_npt, which rebuilds its list from scratch at every step:
positions to 1e-10 A, velocities 1e-8 and box, volume, pressure and conserved quantity
to 1e-10 relative after 20 steps.  dp_md_run (velocity Verlet) in a triclinic cell
follows or_md the same way."""
import numpy as np
import pytest

from paper_2004_11658_amd import inputs as I
from oracle.oracle import Oracle, set_threads

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dp():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2004_11658_amd import dp as D
    return D


def _triclinic_water192():
    c, t, b = I.config_water192()
    tric = np.array([[12.42, 0.0, 0.0], [2.1, 12.1, 0.0], [-1.6, 1.3, 12.6]])
    return c @ np.linalg.inv(b) @ tric, t, tric


def _rel(a, b):
    return np.abs(np.asarray(a) - np.asarray(b)).max() / max(np.abs(np.asarray(b)).max(), 1e-300)


@pytest.mark.parametrize("case", ["npt_triclinic", "nph_cubic", "npt_small_skin"])
def test_npt_matches_oracle(dp, water_model, case):
    import torch
    set_threads(8)
    masses = [I.MASS["O"], I.MASS["H"]]
    if case == "nph_cubic":
        c, t, b = I.config_water192()
    else:
        c, t, b = _triclinic_water192()
    v = I.maxwell_velocities(t, masses, 300.0, 302)
    skin = 0.3 if case == "npt_small_skin" else 2.0
    tau_t = 0.0 if case == "nph_cubic" else 25.0
    # the random-weight water starts near 2e4 bar: 4e4 bar compresses the cell by about
    # 7 % in volume over the 10 fs, 1e4 bar expands it by about 4 %
    pbar, tau_p = (1.0e4 if case == "nph_cubic" else 4.0e4), 100.0
    print("npt case", case, flush=True)
    m = dp.DPModel(water_model, skin=skin)
    x_d = torch.as_tensor(c, device="cuda").clone()
    v_d = torch.as_tensor(v, device="cuda").clone()
    th, box, st = m.md_run_npt(x_d, v_d, t, masses, b, pbar, tau_p, 300.0, tau_t, 0.5, 20, 5, min_scale=0.85)
    th, box, st = th.cpu().numpy(), box.cpu().numpy(), st.cpu().numpy()
    xo, vo, boxo, tho, sto = Oracle(water_model).md_npt(c, v, t, masses, b, pbar, tau_p, 300.0, tau_t, 0.5, 20, 5)
    print(case, "V", tho[0, 6], "->", tho[-1, 6], "H drift", np.abs(tho[:, 7] - tho[0, 7]).max(), flush=True)
    assert abs(tho[-1, 6] / tho[0, 6] - 1.0) > 0.02          # the box moved
    assert np.abs(x_d.cpu().numpy() - xo).max() < 1e-10
    assert _rel(v_d.cpu().numpy(), vo) < 1e-8
    assert _rel(box, boxo) < 1e-12
    assert _rel(th[:, 1:], tho[:, 1:]) < 1e-10
    assert _rel(st, sto) < 1e-9


def test_nve_md_triclinic_matches_oracle(dp, water_model):
    """Velocity Verlet with the 2 A skin in a triclinic cell (production MD)."""
    import torch
    set_threads(8)
    masses = [I.MASS["O"], I.MASS["H"]]
    c, t, b = _triclinic_water192()
    v = I.maxwell_velocities(t, masses, 300.0, 302)
    m = dp.DPModel(water_model, skin=2.0)
    x_d = torch.as_tensor(c, device="cuda").clone()
    v_d = torch.as_tensor(v, device="cuda").clone()
    th = m.md_run(x_d, v_d, t, masses, b, 0.5, 20, 5).cpu().numpy()
    xo, vo, tho = Oracle(water_model).md(c, v, t, masses, b, 0.5, 20, 5)
    assert np.abs(x_d.cpu().numpy() - xo).max() < 1e-10
    assert _rel(v_d.cpu().numpy(), vo) < 1e-8
    assert _rel(th[:, 1:], tho[:, 1:]) < 1e-10


def test_npt_rejects_bad_options(dp, water_model):
    import torch
    masses = [I.MASS["O"], I.MASS["H"]]
    c, t, b = I.config_water192()
    x_d = torch.as_tensor(c, device="cuda").clone()
    v_d = torch.zeros_like(x_d)
    no_skin = dp.DPModel(water_model)
    with pytest.raises(dp.DPError) as e:
        no_skin.md_run_npt(x_d, v_d, t, masses, b, 1.0, 50.0, 300.0, 0.0, 0.5, 2, 1)
    assert e.value.code == -1
    m = dp.DPModel(water_model, skin=1.0)
    for bad in [dict(tau_p=0.0), dict(temperature=-1.0), dict(min_scale=0.3)]:
        kw = dict(pressure_bar=1.0, tau_p=50.0, temperature=300.0, tau_t=0.0, min_scale=0.9)
        kw.update(bad)
        with pytest.raises(dp.DPError) as e:
            m.md_run_npt(x_d, v_d, t, masses, b, kw["pressure_bar"], kw["tau_p"], kw["temperature"], kw["tau_t"],
                         0.5, 2, 1, min_scale=kw["min_scale"])
        assert e.value.code == -1
