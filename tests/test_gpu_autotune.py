"""GPU check of the sweep-shape autotuner: it times only shapes that hold the
class's rows, installs the fastest one, and solves still match the oracle
with the tuned shapes."""
import numpy as np
import pytest
import torch

from oracle import boxls as ob
from tests.gpu_helpers import parity_vs_oracle, to_dev
from tests.test_gpu_parity import planted

pytestmark = pytest.mark.gpu


def test_autotune_installs_valid_shapes_and_keeps_parity():
    import paper_2202_07258_amd as bx
    from paper_2202_07258_amd import native as N
    variants = N.sweep_variants()
    before = {c: N.variant_for_rows(variants[c]["capacity"]) for c in (1, 3)}
    scale_before = {c: N.group_scale(c) for c in (1, 3)}
    table = bx.autotune.tune(classes=[1, 3], iters=20, reps=1)
    try:
        for c in (1, 3):
            row = table["classes"][c]
            m = variants[c]["capacity"]
            assert all(variants[v]["capacity"] >= m for v in row["us"])
            assert row["best"] == min(row["us"], key=row["us"].get)
            assert N.variant_for_rows(m) == row["best"]
            assert all(t > 0 for t in row["us"].values())
            assert row["scale"] in row["scale_us"] and N.group_scale(c) == row["scale"]
        # a solve with the tuned shapes (class 3: 257..512 rows) matches the oracle
        P = planted(77, 400, 900, dtype=np.float32, box=(-1.0, 1.0))
        eta = 1.0 / (1.05 * ob.lipschitz(P.A64()))
        A, y, l, u = to_dev(P)
        kw = dict(screen_every=10, eps_gap=1e-8, max_iter=5000, step=eta)
        x, s, info = bx.solve_bvls(A, y, l, u, **kw)
        torch.cuda.synchronize()
        parity_vs_oracle(P, x.cpu().numpy(), s.cpu().numpy(), info, **kw)
    finally:
        for c, v in before.items():
            N.set_sweep_variant(c, v)
            N.set_group_scale(c, scale_before[c])


def test_tuning_table_is_stored_and_reused(tmp_path):
    """The persistent table: a class tuned once under this GPU's key (arch,
    HIP runtime, library version, setting) is reused by the next call without
    timing anything, and re-applied."""
    import paper_2202_07258_amd as bx
    from paper_2202_07258_amd import native as N
    path = str(tmp_path / "tune.json")
    before = (N.variant_for_rows(128), N.group_scale(1))
    try:
        t1 = bx.autotune.tuned(classes=[1], path=path, iters=10, reps=1)
        assert t1["tuned"] == [1] and t1["cached"] == []
        assert "gfx950" in t1["key"]
        N.set_sweep_variant(1, -1)
        t2 = bx.autotune.tuned(classes=[1], path=path)
        assert t2["tuned"] == [] and t2["cached"] == [1] and t2["key"] == t1["key"]
        assert N.variant_for_rows(128) == int(t1["classes"][1]["best"])
        assert bx.autotune.load(path)[t1["key"]]["1"]["best"] == t1["classes"][1]["best"]
    finally:
        N.set_sweep_variant(1, before[0])
        N.set_group_scale(1, before[1])
