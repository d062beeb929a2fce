import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: full-size case (minutes of CPU)")


@pytest.fixture(scope="session")
def orc():
    import oracle

    oracle.lib()
    return oracle


class _Level1Problem:
    """The paper's 100^3 Laplace problem with level-1 ILU factors (Sec. 4),
    and its SAIT factor pairs, each built once per session."""

    def __init__(self):
        import numpy as np

        import oracle
        from workloads import poisson3d

        self.A = poisson3d(100)
        self.L, self.U = oracle.iluk(self.A, 1)
        self.f = np.random.default_rng(0).uniform(0.0, 1.0, self.A.n)
        self._pairs = {}

    def sait(self, kind, param):
        import oracle

        key = (kind, param)
        if key not in self._pairs:
            kw = {"tau": param} if kind == "thr" else {"p": param}
            self._pairs[key] = oracle.sait_factors(self.L, self.U, 10, **kw)
        return self._pairs[key]


@pytest.fixture(scope="session")
def paper_level1():
    return _Level1Problem()
