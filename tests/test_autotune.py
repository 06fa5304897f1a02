"""Autotuner table logic (CPU) and a short tuning run (GPU)."""
import json

import numpy as np
import pytest

from paper_2606_18463_amd import autotune as at


def test_key_buckets_are_powers_of_two():
    assert at.key(1000, 300, 1, 64) == "1:64:512:1024"
    assert at.key(1024, 512, 1, 64) == "1:64:512:1024"
    assert at.key(1025, 513, 0, 16) == "0:16:1024:2048"


def test_table_round_trip(tmp_path):
    p = tmp_path / "t.json"
    t = at.Table(str(p))
    t.entries[at.key(5000, 200, 1, 64)] = dict(s=16, exec_mode=0, variant=1, grid_blocks=0,
                                               updates_per_s=1e4)
    t.save()
    t2 = at.Table(str(p))
    c = t2.get(6000, 250, 1, 64)
    assert c is not None and c.s == 16 and c.variant == 1 and c.gram_tile == 0
    assert t2.get(6000, 250, 1, 32) is None
    t2.entries[at.key(5000, 200, 1, 32)] = dict(s=8, exec_mode=0, variant=3, grid_blocks=0,
                                                updates_per_s=2e4, gram_tile=128)
    assert t2.get(5000, 200, 1, 32).gram_tile == 128
    assert json.loads(p.read_text())


@pytest.mark.gpu
def test_tune_small_problem(tmp_path):
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("needs a GPU")
    import paper_2606_18463_amd as cg
    g = np.random.default_rng(0)
    X = torch.from_numpy((g.standard_normal((8192, 256)) / 16).astype(np.float32)).cuda()
    y = torch.from_numpy(np.where(g.random(8192) < 0.5, -1.0, 1.0).astype(np.float32)).cuda()
    Xm = cg.dense_matrix(X)
    t = at.Table(str(tmp_path / "t.json"))
    res = []
    c = t.lookup_or_tune(Xm, y, 32, s_grid=(1, 4, 16), budget_s=0.003, results=res)
    assert c.s in (1, 4, 16) and c.updates_per_s > 0
    assert {r.gram_tile for r in res if r.s > 1} == {64, 128}
    assert t.get(8192, 256, cg.F32, 32) == c
