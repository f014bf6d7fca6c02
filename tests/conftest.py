import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU")


@pytest.fixture(scope="session", autouse=True)
def _built_helpers():
    """Build the CPU-side helper libraries if they are not there yet."""
    import oracle
    from paper_2309_09131_amd import build as pbuild
    oracle.build(force=False)
    pbuild.build_synth(force=False)
