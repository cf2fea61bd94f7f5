import os
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

from paper_2004_11658_amd import inputs as I  # noqa: E402

MODEL_DIR = os.path.join(ROOT, "tests", "_models")


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs through the HIP library)")
    config.addinivalue_line("markers", "slow: long CPU oracle runs")


# a small model with the same structure as the water model (2 species, doubling
# embedding layers, square hidden fitting layers), cheap enough for finite differences
TINY = I.ModelSpec(ntypes=2, emb_width=(4, 8, 16), fit_width=(12, 12, 12), m2=4,
                   sel=(12, 24), rc=4.0, rcs=0.5)
TINY1 = I.ModelSpec(ntypes=1, emb_width=(4, 8, 16), fit_width=(12, 12), m2=4,
                    sel=(40,), rc=4.0, rcs=1.0)


def model_file(name, spec, seed, params=None):
    os.makedirs(MODEL_DIR, exist_ok=True)
    path = os.path.join(MODEL_DIR, "%s_%d.bin" % (name, seed))
    if params is None:
        params = I.random_params(spec, seed)
    I.write_model(path, spec, params)
    return path


@pytest.fixture(scope="session")
def water_model():
    return model_file("water", I.WATER, 101)


@pytest.fixture(scope="session")
def water_model_b():
    return model_file("water", I.WATER, 104)


@pytest.fixture(scope="session")
def copper_model():
    return model_file("copper", I.COPPER, 103)


@pytest.fixture(scope="session")
def tiny_model():
    return model_file("tiny", TINY, 7)


@pytest.fixture(scope="session")
def tiny1_model():
    return model_file("tiny1", TINY1, 8)


@pytest.fixture(scope="session")
def water192():
    return I.config_water192()


def tiny_water(seed=11, n_side=2, L=6.3):
    """8 water molecules in a 6.3 A cube (box < 2 rc of the tiny model: self images)."""
    return I.water_lattice(n_side, L, seed)
