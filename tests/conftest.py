import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HERE = os.path.dirname(os.path.abspath(__file__))
for p in (ROOT, HERE):
    if p not in sys.path:
        sys.path.insert(0, p)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs the HIP library)")
    config.addinivalue_line("markers", "slow: long CPU test")


@pytest.fixture(scope="session")
def oracle_mod():
    import oracle
    oracle.build(force=False)
    return oracle


# Small games used across the CPU suite ------------------------------------

def tiny_games():
    import gamegen as gg
    return {
        "cfg1": gg.cfg1(),
        # S=2, depth 3, binary: brute force over pure strategies is cheap
        "s2d3": gg.public_game(7, S=2, max_depth=3, branch_lo=2, branch_hi=2, p_stop=0.0),
        # terminals at several depths, including children of the root
        # (payoff entries in player 2's empty-sequence column)
        "stops": gg.public_game(2, S=2, max_depth=4, branch_lo=2, branch_hi=3, p_stop=0.3),
        # perfect information
        "perfect": gg.public_game(11, S=1, max_depth=6, branch_lo=2, branch_hi=3, p_stop=0.2),
    }


@pytest.fixture(scope="session")
def games():
    return tiny_games()


def pytest_terminal_summary(terminalreporter):
    from helpers import SESSION_REPORT
    if SESSION_REPORT:
        terminalreporter.write_sep("-", "errors against the FP64 oracle (FP32 modes)")
        for line in SESSION_REPORT:
            terminalreporter.write_line(line)
