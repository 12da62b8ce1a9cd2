"""The autotuner's on-disk cache (KPME_TUNE_CACHE): an autotuned plan
appends its stage-2 term split, stage-2 stream count and stage-1 split,
keyed by the shape class, as "key value" lines; a plan of the same class
created in a fresh process with the same cache file starts from those values
(no tuning run) and computes the same operator."""
import os
import subprocess
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SHAPE = ((30.0, 36.0, 40.0), (30, 36, 40), 4, 0.5, 14)


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


CHILD = r"""
import sys, json
sys.path.insert(0, sys.argv[1])
import numpy as np, torch
from paper_2601_18838_amd import kpme
box, grid, p, beta, rank = json.loads(sys.argv[2])
pl = kpme.Plan(box, grid, p, beta, rank=rank, precision="fp16x3", max_particles=16)
q = torch.tensor(np.random.default_rng(3).standard_normal(grid), dtype=torch.float32, device="cuda")
phi = pl.skp_apply(q).cpu().double().numpy()
np.save(sys.argv[3], phi)
print(json.dumps([pl.stage2_parts(), pl.stage2_streams(), pl.stage1_split()]), flush=True)
"""


def test_tuned_shape_is_cached_on_disk_and_reused(tmp_path, monkeypatch):
    import json
    from paper_2601_18838_amd import kpme
    print("[tune cache] autotune and reuse", flush=True)
    cache = tmp_path / "tune.txt"
    monkeypatch.setenv("KPME_TUNE_CACHE", str(cache))
    box, grid, p, beta, rank = SHAPE
    pl = kpme.Plan(box, grid, p, beta, rank=rank, precision="fp16x3", max_particles=16)
    parts = pl.autotune()
    tuned = [parts, pl.stage2_streams(), pl.stage1_split()]
    assert 1 <= tuned[0] <= 8 and tuned[1] in (1, 2) and tuned[2] >= 1
    lines = [l.split() for l in cache.read_text().splitlines() if l.strip()]
    keys = {k.split("_")[0]: int(v) for k, v in lines}
    assert keys == {"s2parts": tuned[0], "s2streams": tuned[1], "s1split": tuned[2]}
    q = torch.tensor(np.random.default_rng(3).standard_normal(grid), dtype=torch.float32,
                     device="cuda")
    ref = pl.skp_apply(q).cpu().double().numpy()
    out = tmp_path / "phi.npy"
    env = dict(os.environ, KPME_TUNE_CACHE=str(cache))
    r = subprocess.run([sys.executable, "-c", CHILD, ROOT, json.dumps(SHAPE), str(out)],
                       capture_output=True, text=True, env=env, timeout=300)
    assert r.returncode == 0, r.stderr[-3000:]
    assert json.loads(r.stdout.strip().splitlines()[-1]) == tuned
    phi = np.load(out)
    assert np.abs(phi - ref).max() <= 1e-5 * np.abs(ref).max()
