import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

GOLDEN = os.path.join(ROOT, "tests", "golden")


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU; calls the HIP library through its C ABI")


def read_golden(name):
    """Non-comment lines of a golden fixture."""
    with open(os.path.join(GOLDEN, name)) as f:
        return [ln.rstrip("\n") for ln in f if ln.strip() and not ln.startswith("#")]


@pytest.fixture(scope="session")
def oracle_mod():
    import oracle

    oracle.build(force=False)
    return oracle


@pytest.fixture(scope="session")
def gpu():
    """Skip unless a GPU is present; never falls back to a CPU path."""
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1104_1824_amd import snp

    snp.lib()  # raises if libsnp.so is not built
    return torch.device("cuda:0")
