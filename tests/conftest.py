import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU")
    config.addinivalue_line("markers", "slow: long-running CPU test")


@pytest.fixture(scope="session")
def oracle_mod():
    import oracle
    oracle.build()
    return oracle


def _gpu_available():
    try:
        import torch
        return torch.cuda.is_available()
    except Exception:
        return False


@pytest.fixture(scope="session")
def ea_gpu():
    """The product package, on a machine with a GPU (the library must load)."""
    if not _gpu_available():
        pytest.skip("no GPU")
    import paper_1411_5512_amd as ea
    ea.abi.lib()  # raises if libea.so is missing: there is no fallback
    return ea


GOLDEN = os.path.join(ROOT, "tests", "golden")


def golden_values(name: str) -> dict:
    """A tests/golden fixture of "name value  # citation" lines as a dict."""
    out = {}
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.split("#", 1)[0].strip()
            if line:
                key, value = line.split()
                out[key] = float(value)
    return out


@pytest.fixture(scope="session")
def paper():
    """The results the paper prints (tests/golden/paper_values.txt)."""
    return golden_values("paper_values.txt")
