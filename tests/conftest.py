import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs the HIP library)")
    config.addinivalue_line("markers", "slow: long CPU test")


def oracle_config(params: dict, **kw):
    import oracle
    keys = {f for f in oracle.Config.__dataclass_fields__}
    p = {k: v for k, v in params.items() if k in keys}
    p.update(kw)
    return oracle.Config(**p)


@pytest.fixture(scope="session")
def ora():
    import oracle
    oracle.lib()
    return oracle
