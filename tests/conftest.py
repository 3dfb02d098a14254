import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

GOLDEN = os.path.join(ROOT, "tests", "golden")


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs through the HIP library's C ABI)")
    config.addinivalue_line("markers", "slow: long CPU test (oracle at full parameters)")


def golden(name):
    import json
    with open(os.path.join(GOLDEN, name)) as f:
        return json.load(f)


def oracle_vectors(name):
    """The oracle's stored expected values of a full-size workload
    (tests/golden/oracle_<name>.json).  They take hours of host time to
    write; a test whose vectors are not written yet is skipped with the
    command that writes them."""
    path = os.path.join(GOLDEN, f"oracle_{name}.json")
    if not os.path.exists(path):
        pytest.skip(f"oracle vectors not written: python tests/golden/make_oracle_vectors.py {name}")
    return golden(f"oracle_{name}.json")


@pytest.fixture(scope="session")
def oracle_toy_keys():
    from oracle import tfhe as T
    return T.Keys(T.toy_params(), seed=11)


@pytest.fixture(scope="session")
def oracle_keys():
    from oracle import tfhe as T
    return T.Keys(T.default_params(), seed=1)
