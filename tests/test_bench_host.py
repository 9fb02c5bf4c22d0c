"""Host-side checks of bench.py: the one-GPU contract and the flop count's census keys."""
import subprocess
import sys
from pathlib import Path

import bench
import paper_1407_3444_amd as lib

ROOT = Path(__file__).resolve().parents[1]


def test_flop_count_reads_every_census_key():
    """The roofline's flop count takes the census as the binding returns it (chi0_census's counts
    in CENSUS_KEYS order); a key missing on either side fails here rather than on the GPU."""
    census = dict.fromkeys(lib.CENSUS_KEYS, 1)
    assert bench.census_flops(census) > 0
    assert bench.census_flops(census, mixed=True) > 0
    for k in lib.CENSUS_KEYS:
        c = dict(census)
        c[k] = 2
        assert bench.census_flops(c) >= bench.census_flops(census)


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, str(ROOT / "bench.py"), "--gpus", "2"], capture_output=True, text=True,
                       timeout=120, cwd=ROOT)
    assert r.returncode != 0
    assert "one GPU" in (r.stdout + r.stderr) or "1 GPU" in (r.stdout + r.stderr)
