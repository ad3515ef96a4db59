"""bench.py's contract on the CPU: more than one GPU is refused with a
message before anything touches a device, and the per-sweep algorithmic
bytes that the roofline uses reproduce the figures the committed profile
summaries quote for the 128^3 workload's level-0 and level-1 sweeps."""
import os
import re
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=300, cwd=ROOT,
                       env=dict(os.environ, CUDA_VISIBLE_DEVICES="", HIP_VISIBLE_DEVICES=""))
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout.strip() == ""


def _quoted_bytes(name):
    with open(os.path.join(ROOT, "profiles", name)) as fh:
        text = fh.read()
    m = re.search(r"w = 8: ([0-9,]+) B", text)
    assert m, name
    return int(m.group(1).replace(",", ""))


@pytest.mark.parametrize("name,li", [
    ("k_schwarz_l0_hex128_patch.md",
     dict(star_row_nnz=401718018, star_rows=12290298, nblocks=2048383, fac_entries=43016043,
          n=6193536)),
    ("k_schwarz_pipe_l1_hex128_patch.md",
     dict(star_row_nnz=401122081, star_rows=1500282, nblocks=250047, fac_entries=5250987,
          n=762048)),
])
def test_sweep_bytes_match_the_profile_summaries(name, li):
    assert bench.sweep_bytes(li, 8) == _quoted_bytes(name)
