"""The cache policies of streamed levels (non-temporal coefficient and
right-hand-side loads) change no arithmetic: with every level streamed and
with none streamed, the preconditioner output and a full solve are bitwise
the same.  MFMG_STREAM_BYTES is read once per process, so each setting runs
in a child process of its own."""

import os
import subprocess
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)

CHILD = r'''
import sys
import numpy as np
sys.path.insert(0, {root!r})
sys.path.insert(0, {tests!r})
from gpu_fixtures import small_cases
from paper_2604_18886_amd import mfmg
case = small_cases()["cut_sphere_5_7"]()
out = {{}}
for prec in (0, 1):
    h = case.gpu_hierarchy(precision=prec)
    rng = np.random.default_rng(97)
    r = np.where(case.disc.active, rng.uniform(-1, 1, case.T.n), 0.0)
    out["z%d" % prec] = mfmg.apply_precond(h, case.device(r)).cpu().numpy()
    p = case.device(np.zeros(case.T.n))
    _, st = mfmg.pcg_solve(h, case.device(case.rhs), p, rtol=1e-10)
    out["p%d" % prec] = p.cpu().numpy()
    out["it%d" % prec] = np.array([st["iters"]])
np.savez({path!r}, **out)
'''


def _run(tmp_path, stream_bytes, tag):
    path = str(tmp_path / f"{tag}.npz")
    env = dict(os.environ, MFMG_STREAM_BYTES=str(stream_bytes))
    code = CHILD.format(root=ROOT, tests=HERE, path=path)
    print(f"  child MFMG_STREAM_BYTES={stream_bytes}", flush=True)
    r = subprocess.run([sys.executable, "-c", code], env=env, capture_output=True, text=True,
                       timeout=240)
    assert r.returncode == 0, r.stderr[-2000:]
    return dict(np.load(path))


def test_streamed_levels_compute_the_same_values(tmp_path):
    every = _run(tmp_path, 0, "every_level_streamed")
    none = _run(tmp_path, 1 << 50, "no_level_streamed")
    for prec in (0, 1):
        assert np.abs(none[f"z{prec}"]).max() > 0.0
        assert np.array_equal(every[f"z{prec}"], none[f"z{prec}"]), prec
        assert np.array_equal(every[f"it{prec}"], none[f"it{prec}"]), prec
        assert np.array_equal(every[f"p{prec}"], none[f"p{prec}"]), prec
