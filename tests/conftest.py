import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU")


def pytest_terminal_summary(terminalreporter):
    """Report the largest GPU - oracle relative difference of the walk's FP64 scores and W/B figures seen."""
    mod = sys.modules.get("test_gpu_walk") or sys.modules.get("tests.test_gpu_walk")
    diff = getattr(mod, "SCORE_DIFF", None) if mod else None
    if diff and (diff["score"] > 0 or diff["wb"] > 0):
        terminalreporter.write_line(f"walk FP64 GPU-oracle max relative difference: scores {diff['score']:.3e}, "
                                    f"W/B {diff['wb']:.3e}")
