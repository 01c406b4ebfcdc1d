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
