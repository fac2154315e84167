import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

# Parallel test workers (pytest -n) split the cores among the C oracle's
# OpenMP loops: more spinning threads than cores slow those loops down by
# orders of magnitude.
if os.environ.get("PYTEST_XDIST_WORKER_COUNT"):
    os.environ.setdefault("OMP_NUM_THREADS",
                          str(max(1, (os.cpu_count() or 1) // int(os.environ["PYTEST_XDIST_WORKER_COUNT"]))))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: longer CPU test")


def golden(name):
    return os.path.join(ROOT, "tests", "golden", name)


def paper_constants():
    out = {}
    with open(golden("paper_constants.txt")) as fh:
        for line in fh:
            if line.startswith("#") or not line.strip():
                continue
            parts = line.split()
            out[parts[0]] = float(parts[1])
    return out


def appendix_table():
    ks, cs = [], []
    with open(golden("oucs3_equivalent_explicit_interior.txt")) as fh:
        for line in fh:
            if line.startswith("#") or not line.strip():
                continue
            k, c = line.split()
            ks.append(int(k))
            cs.append(float(c))
    return ks, cs
