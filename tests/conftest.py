import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")


@pytest.fixture(scope="session")
def glat():
    from mlmc_inputs import graphene
    return graphene()


@pytest.fixture(scope="session")
def mlat():
    from mlmc_inputs import mos2_shaped
    return mos2_shaped()


@pytest.fixture(scope="session")
def plat():
    from mlmc_inputs import mos2_shaped
    return mos2_shaped(s_pairs=True)
