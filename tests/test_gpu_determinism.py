"""Results do not depend on the process: every output of tests/det_child.py
(binning, assembly, the mass assignment with the resident, Chebyshev and
tile-streaming solvers, three fluid steps) is bit-identical in two fresh processes and in this one.
The binning order, the scatter sums and every reduction have a fixed order; nothing
depends on atomics' arrival order, launch timing or allocation addresses."""
import json
import os
import subprocess
import sys

import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_outputs_identical_across_processes():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    runs = []
    for k in range(2):
        r = subprocess.run([sys.executable, os.path.join(ROOT, "tests", "det_child.py")],
                           capture_output=True, text=True, timeout=240)
        assert r.returncode == 0, r.stderr[-2000:]
        runs.append(json.loads(r.stdout.strip().splitlines()[-1]))
    sys.path.insert(0, os.path.join(ROOT, "tests"))
    import det_child
    runs.append(det_child.digests())
    for k, other in enumerate(runs[1:], 1):
        diff = sorted(key for key in runs[0] if runs[0][key] != other.get(key))
        print(f"run {k}: {len(runs[0])} outputs, differing from run 0: {diff}", flush=True)
        assert not diff
