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
    config.addinivalue_line("markers", "workloads(*names): full-size synthetic inputs the "
                                       "test reads, drawn before any test touches the GPU")


def pytest_collection_finish(session):
    """Draw the full-size inputs of the selected tests now, while no test has
    initialised the GPU (the generator forks worker processes)."""
    names = []
    for item in session.items:
        m = item.get_closest_marker("workloads")
        if m:
            names += [n for n in m.args if n not in names]
    if names:
        import inputs

        inputs.pregenerate(names, log=lambda msg: print(msg, flush=True))


@pytest.fixture(scope="session")
def O():
    import oracle
    if not os.path.exists(oracle.LIB):
        oracle.build()
    return oracle.get()
