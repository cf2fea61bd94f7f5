"""Checkpoint and resume of the MD driver.

The whole MD state between dp_md_run calls is the caller's positions and velocities (with
the box and the species): every call rebuilds its neighbour list and evaluates the forces
at its starting positions.  So N + N steps through a checkpoint written to disk and read
back give the trajectory of one 2N-step run: bit for bit in deterministic mode with a list
built at every step (the split run then repeats exactly the arithmetic of the continuous
one: the same lists, the same fixed-order force sums, the two half kicks of the velocity
Verlet step applied one after the other in both), and to rounding with the Verlet list,
whose rebuild points differ between the two runs.
"""
import numpy as np
import pytest

from paper_2004_11658_amd import inputs as I

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dp():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2004_11658_amd import dp as D
    return D


@pytest.mark.parametrize("skin,deterministic", [(0.0, True), (2.0, False)])
def test_md_resume_from_checkpoint(dp, water_model, water192, tmp_path, skin, deterministic):
    import torch
    c, t, b = water192
    masses = [I.MASS["O"], I.MASS["H"]]
    v = I.maxwell_velocities(t, masses, 300.0, 302)
    print("resume skin", skin, "deterministic", deterministic, flush=True)
    m = dp.DPModel(water_model, skin=skin, deterministic=deterministic)
    # one run of 20 steps
    x1 = torch.as_tensor(c, device="cuda").clone()
    v1 = torch.as_tensor(v, device="cuda").clone()
    m.md_run(x1, v1, t, masses, b, 0.5, 20, 0)
    # 10 steps, a checkpoint on disk, 10 more from it
    x2 = torch.as_tensor(c, device="cuda").clone()
    v2 = torch.as_tensor(v, device="cuda").clone()
    m.md_run(x2, v2, t, masses, b, 0.5, 10, 0)
    ck = tmp_path / "md_step10.npz"
    np.savez(ck, x=x2.cpu().numpy(), v=v2.cpu().numpy(), box=np.asarray(b), types=np.asarray(t), step=10)
    del x2, v2
    st = np.load(ck)
    assert int(st["step"]) == 10
    x3 = torch.as_tensor(st["x"], device="cuda").clone()
    v3 = torch.as_tensor(st["v"], device="cuda").clone()
    m.md_run(x3, v3, st["types"], masses, st["box"], 0.5, 10, 0)
    x1, v1, x3, v3 = x1.cpu().numpy(), v1.cpu().numpy(), x3.cpu().numpy(), v3.cpu().numpy()
    if deterministic:
        assert np.array_equal(x1, x3)
        assert np.array_equal(v1, v3)
    else:
        assert np.abs(x1 - x3).max() < 1e-10
        assert np.abs(v1 - v3).max() < 1e-8 * np.abs(v1).max()
