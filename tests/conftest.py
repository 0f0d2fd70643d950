"""Shared fixtures. GPU tests carry the ``gpu`` marker; everything else runs
on the CPU."""
import os
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import synthnet  # noqa: E402

YEAR_S = 3.15576e7   # Julian year in seconds


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs through the HIP library)")
    config.addinivalue_line("markers", "slow: long CPU-side oracle runs")


@pytest.fixture(scope="session")
def oracle_mod():
    import oracle
    oracle.lib()
    oracle.set_threads(min(8, os.cpu_count() or 1))
    return oracle


@pytest.fixture(scope="session")
def tiny():
    return synthnet.workload("tiny", n_cells=4)


@pytest.fixture(scope="session")
def medium_net():
    net, _ = synthnet.workload("medium", n_cells=1)
    return net


@pytest.fixture(scope="session")
def medium(medium_net):
    cells = synthnet.make_cells(medium_net, 64, synthnet.SEED_BASE + 1)
    return medium_net, cells


def network_from(reactions, alpha, n_species, beta=None, gamma=None, composition=None):
    return synthnet.network_from_lists(n_species, reactions, alpha, beta, gamma, composition)
