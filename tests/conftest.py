import json
import os
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

GOLDEN = os.path.join(ROOT, "tests", "golden")


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) and the built HIP library")
    config.addinivalue_line("markers", "slow: oracle work that takes more than a few seconds")


def golden(name):
    with open(os.path.join(GOLDEN, name)) as f:
        return json.load(f)


@pytest.fixture(scope="session")
def spec64():
    from oracle import tables
    return tables.TableSpec.default(64)


@pytest.fixture(scope="session")
def tables64(spec64):
    from oracle import tables
    return tables.build_tables(spec64)


@pytest.fixture(scope="session")
def ts64(spec64, tables64):
    from oracle import step
    return step.TableSet(spec64, tables64)


@pytest.fixture(scope="session")
def cells0_small():
    from paper_2505_08855_amd import workloads
    return workloads.workload(0, n=2048)


def rel_err(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return np.abs(a - b) / np.maximum(np.abs(b), 1e-300)
