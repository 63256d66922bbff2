"""Host-side logic of the benchmark (no GPU): how bodies are grouped into
batches, each below the 2^31 - 1 entries of A a batch holds."""
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402

LIMIT = 2**31 - 1


def test_eight_stiff_copies_run_as_six_and_two():
    """eight copies of the 328,877,342-entry ellipsoid: six fit one batch"""
    g = bench.batch_groups([328_877_342] * 8)
    assert g == [[0, 1, 2, 3, 4, 5], [6, 7]]
    assert all(sum(328_877_342 for _ in grp) < LIMIT for grp in g)


def test_groups_cover_every_body_once_and_stay_below_the_limit():
    import numpy as np
    rng = np.random.default_rng(5)
    sizes = [int(v) for v in rng.integers(1, 900_000_000, 40)]
    g = bench.batch_groups(sizes)
    assert [k for grp in g for k in grp] == list(range(len(sizes)))
    for grp in g:
        assert len(grp) == 1 or sum(sizes[k] for k in grp) < LIMIT


def test_boundaries():
    assert bench.batch_groups([]) == []
    assert bench.batch_groups([5, 7, 11]) == [[0, 1, 2]]
    assert bench.batch_groups([LIMIT - 1, 1]) == [[0], [1]]      # LIMIT would not fit
    assert bench.batch_groups([LIMIT - 2, 1]) == [[0, 1]]        # LIMIT - 1 fits
    assert bench.batch_groups([LIMIT + 5, 3]) == [[0], [1]]      # oversize alone


def test_more_than_one_gpu_is_refused_before_any_gpu_work():
    """the benchmark measures one GPU; --gpus 2 exits with a message and
    status 2 without touching a device"""
    import subprocess
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in (r.stdout + r.stderr)
