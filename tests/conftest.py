import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs through the HIP library)")
    config.addinivalue_line("markers", "slow: long-running CPU test")


def pytest_terminal_summary(terminalreporter):
    """Achieved errors of the GPU parity tests (largest per-variable
    relative L2 or maximum, per test), so that the run's output records
    them next to the pass count."""
    mod = sys.modules.get("gpu_common")
    rows = getattr(mod, "ACHIEVED", None) if mod else None
    if not rows:
        return
    terminalreporter.write_sep("-", "achieved parity errors (largest per test)")
    line = ""
    for name, worst, _ in rows:
        item = f"{name}={worst:.1e}"
        if len(line) + len(item) + 2 > 118:
            terminalreporter.write_line(line)
            line = ""
        line = f"{line}  {item}" if line else item
    if line:
        terminalreporter.write_line(line)
