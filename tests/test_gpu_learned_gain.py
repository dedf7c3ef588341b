"""What the trained warm start gains over plain Gauss-Newton-Krylov (committed weights).

Two held-out phantom pairs at the 128^3 / 32^3 image-transport configuration, registered
plain (v0 = 0) and from the network's prediction.  The warm-started run must reach the
plain run's final objective with fewer Gauss-Newton iterations and at most half the
Hessian matvecs (the held-out mean over 200 pairs is 2.5x and 4.1x fewer).
"""
import os

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

WEIGHTS = os.path.join(os.path.dirname(__file__), "..", "paper_2006_06823_amd", "weights", "warmstart_v1_128.npz")


def test_warm_start_reaches_plain_objective_faster():
    from paper_2006_06823_amd import learned as LW
    seeds = [20000, 20001]
    pairs = [LW.render_pair(s) for s in seeds]

    class Pairs:
        def pairs(self, sds):
            for s, (a, b) in zip(sds, pairs):
                yield s, a, b

    reg = LW.Registrar(variant=1)
    net = LW.load_weights(WEIGHTS, device=reg.device)
    rows = LW.compare(net, reg, seeds, Pairs(), LW.SolveOpts(), log=lambda *a, **k: None, with_Z=False)
    for r in rows:
        assert not r["fallback"]
        assert r["pred_vnorm_rel"] < 0.5
        assert r["learned_E"]["E"] <= r["plain"]["E"]
        assert r["learned_E"]["gn_iters"] < r["plain"]["gn_iters"]
        assert r["learned_E"]["hess_matvecs"] <= 0.5 * r["plain"]["hess_matvecs"]
        # the warm-started run with the plain stopping rule ends at least as low as plain
        assert r["learned"]["E"] <= r["plain"]["E"] * (1 + 1e-6)
