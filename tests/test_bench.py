"""Host logic of bench.py (CPU): the one-GPU guard and the candidate count
that the neighbour-list roofline is priced on."""
import json
import os
import subprocess
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in json.loads(r.stdout.strip().splitlines()[-1])["error"]


def test_list_candidates_equals_brute_force():
    """Every ordered pair (i, j != i) whose cells are neighbours (periodic,
    27-cell stencil) is one candidate."""
    rng = np.random.default_rng(0)
    box = (5.0, 6.3, 4.0)
    x = rng.random((400, 3)) * box
    nc = [int(np.floor(L / 1.0)) for L in box]
    c = np.stack([np.minimum((x[:, a] * nc[a] / box[a]).astype(int), nc[a] - 1) for a in range(3)], axis=1)
    d = np.abs(c[:, None, :] - c[None, :, :])
    d = np.minimum(d, np.array(nc) - d)
    near = np.all(d <= 1, axis=2)
    np.fill_diagonal(near, False)
    assert bench.list_candidates(x, box, 1.0) == int(near.sum())
