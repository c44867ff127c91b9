import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: long CPU test")


def pytest_terminal_summary(terminalreporter):
    """Worst parity errors per configuration and precision (GPU runs)."""
    try:
        from tests.gpu_common import WORST
    except Exception:
        return
    if not WORST:
        return
    tr = terminalreporter
    tr.write_sep("-", "worst parity error per configuration (e_x, e_phi, e_res; largest error/bar; frames)")
    for (cfg, dt), (e, ratio, n) in sorted(WORST.items()):
        tr.write_line(f"{cfg:14s} {dt:8s} e_x {e[0]:.2e} e_phi {e[1]:.2e} e_res {e[2]:.2e} "
                      f"err/bar {ratio:.2f} frames {n}")
