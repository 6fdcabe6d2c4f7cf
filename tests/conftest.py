import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: full-size workload (seconds to minutes)")


@pytest.fixture(autouse=True)
def _tuned_configurations():
    """After a test, put the shipped tuning table back in effect: tests that
    force configurations reset them to the compiled defaults, and the tests
    after them should run the tuned ones, as the library does."""
    yield
    mod = sys.modules.get("paper_2305_03448_amd")
    if mod is not None and getattr(mod, "_lib", None) is not None and os.path.exists(mod.TUNE_FILE):
        mod._lib.desc_config_load(mod.TUNE_FILE.encode())
