import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU")
    config.addinivalue_line("markers", "slow: long-running CPU test")


_HEADLINE_REPORT = []


@pytest.fixture(scope="session")
def headline_report():
    """Summary lines of the headline-precision tests, printed at the end of
    the session."""
    return _HEADLINE_REPORT


def pytest_terminal_summary(terminalreporter, exitstatus, config):
    if _HEADLINE_REPORT:
        terminalreporter.write_sep("-", "headline precision against the FP64 oracle")
        for line in _HEADLINE_REPORT:
            terminalreporter.write_line(line)
