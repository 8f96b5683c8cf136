"""The tuning table persisted through SGWLS_TUNE_CACHE: a process that
autotunes writes it, a fresh process loads it at its first filter call and
uses the same variants; a stale file (another library version) is ignored."""
import os
import subprocess
import sys

import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

SCRIPT = r"""
import sys, json
sys.path.insert(0, sys.argv[1])
import numpy as np, torch
torch.zeros(1, device="cuda")
from paper_1705_01674_amd import ops
rng = np.random.default_rng(3)
f = torch.from_numpy(rng.uniform(0, 1, (3, 200, 300)).astype(np.float32)).cuda()
g = torch.from_numpy(rng.uniform(0, 1, (200, 300)).astype(np.float32)).cuda()
p = ops.Params(lam=4.0, r=1, iters=1)
out = {}
if sys.argv[2] == "tune":
    out["chosen"] = {f"{d}_{cb}": v for (d, cb), v in ops.autotune(f, g, p, reps=2).items()}
else:
    ops.sgwls_filter(f, g, p)
    torch.cuda.synchronize()
out["size"] = ops.nat.lib.sgwls_tune_size()
out["query"] = {f"0_3": ops.tune_query(0, 3, 200, 300, p), "1_3": ops.tune_query(1, 3, 200, 300, p)}
print(json.dumps(out))
"""


def run(mode, path):
    env = dict(os.environ, SGWLS_TUNE_CACHE=path)
    res = subprocess.run([sys.executable, "-c", SCRIPT, ROOT, mode], env=env, capture_output=True,
                         text=True, timeout=180)
    assert res.returncode == 0, res.stderr[-2000:]
    import json
    return json.loads(res.stdout.strip().splitlines()[-1])


def test_tuning_table_persists_across_processes(tmp_path):
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    path = str(tmp_path / "tune.txt")
    first = run("tune", path)
    assert os.path.exists(path)
    assert open(path).readline().startswith("sgwls-tune ")
    second = run("use", path)
    assert second["size"] >= first["size"] > 0
    assert second["query"] == first["query"]
    # a stale file is ignored (the table stays empty, no error)
    with open(path, "w") as fh:
        fh.write("sgwls-tune 1 gfx950\n1 3 0 0 0 30 1\n")
    stale = run("use", path)
    assert stale["size"] == 0
