import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: longer CPU test")


# Lines of the form "[err] ..." that passing tests print (measured errors
# next to their bars) are collected and repeated in the terminal summary,
# so that the margins show in a quiet run too.
_ERR_LINES = []


def pytest_runtest_logreport(report):
    if report.when == "call" and report.passed:
        for line in report.capstdout.splitlines():
            if line.startswith("[err]"):
                _ERR_LINES.append(line)


def pytest_terminal_summary(terminalreporter):
    if _ERR_LINES:
        terminalreporter.section("measured errors and their bars")
        for line in _ERR_LINES:
            terminalreporter.write_line(line)
