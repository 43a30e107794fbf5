import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (HIP device) to run")
    config.addinivalue_line("markers", "slow: large CPU case")


@pytest.fixture(scope="session")
def oracle():
    from oracle import oracle as O
    O.build(force=False)
    return O


def read_golden(name):
    """Parse a golden text fixture: '#' comments, '[section]' headers, rows."""
    path = os.path.join(ROOT, "tests", "golden", name)
    sections, cur = {}, None
    with open(path) as fh:
        for line in fh:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            if line.startswith("["):
                cur = line.strip("[]")
                sections[cur] = []
                continue
            sections.setdefault(cur, []).append([float(v) for v in line.split()])
    return sections
