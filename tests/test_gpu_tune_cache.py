"""The autotuner's results persist in a text file keyed by device and build:
a second process reads the shape back instead of timing candidates."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

CHILD = r"""
import json, sys
sys.path.insert(0, {root!r})
import torch
torch.cuda.init()
import nsworkloads as W
from paper_1201_2118_amd.solver import Solver
prm = dict(W.cavity(128, dt=5e-4), precision="mixed")
s = Solver(prm)
print(json.dumps(list(s.timing().sor_tile)), flush=True)
"""


def _child(cache):
    env = dict(os.environ, NS_TUNE_CACHE=str(cache))
    r = subprocess.run([sys.executable, "-c", CHILD.format(root=ROOT)], env=env, capture_output=True, text=True,
                       timeout=300)
    assert r.returncode == 0, r.stderr[-2000:]
    return [int(x) for x in r.stdout.strip().splitlines()[-1].strip("[]").split(",")]


@pytest.mark.gpu
def test_tuned_shape_persists_across_processes(tmp_path):
    cache = tmp_path / "sub" / "tune.txt"
    first = _child(cache)
    lines = cache.read_text().splitlines()
    assert len(lines) == 1, lines
    f = lines[0].split()
    # arch, compute units, build, nx ny nz esz per, rows, chunk
    assert len(f) == 10 and f[0].startswith("gfx"), f
    assert f[3:8] == ["128", "128", "128", "4", "0"], f
    assert [int(f[8]), int(f[9])] == first
    # a stored shape is taken as it stands: replace it by another valid one
    other = [8, 32] if first != [8, 32] else [4, 32]
    cache.write_text(" ".join(f[:8] + [str(other[0]), str(other[1])]) + "\n")
    assert _child(cache) == other
    assert len(cache.read_text().splitlines()) == 1  # nothing re-tuned or appended
    # a line for another build is ignored: tuning runs and appends its own
    cache.write_text(" ".join(f[:2] + ["other-build"] + f[3:8] + [str(other[0]), str(other[1])]) + "\n")
    third = _child(cache)
    lines = cache.read_text().splitlines()
    assert len(lines) == 2 and lines[1].split()[2] == f[2], lines
    assert [int(x) for x in lines[1].split()[8:]] == third
