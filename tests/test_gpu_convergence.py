"""Micro convergence (Sec. 6, micro-convergence studies; the elasticity-tensor
estimate of Sec. 4): Pbar and Abar of an RVE with a square inclusion resolved
exactly at n = 4 ... 64, for the fully linear case, geometrically nonlinear
linear elasticity (St. Venant-Kirchhoff) and the neo-Hookean law.  What the
paper reports, and what is checked here: the orders of successive differences
stay at or below the full order 2q = 2 (the inclusion's corners lower the
regularity), and they are nearly the same for the three laws.  The points
n = 4, 8 are also solved by the oracle (same law) at the parity bar."""
import numpy as np
import pytest

import oracle
from paper_1908_08292_amd import api, rve

pytestmark = pytest.mark.gpu
LAWS = [("linear", rve.LAW_LINEAR, oracle.LAW_LINEAR), ("svk", rve.LAW_SVK, oracle.LAW_SVK),
        ("neo-Hookean", rve.LAW_NEOHOOKE, oracle.LAW_NEOHOOKE)]


def test_micro_convergence_orders():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    F = np.array([[1.08, 0.05], [-0.03, 0.94]])
    orders = {}
    for name, glaw, olaw in LAWS:
        print(f"case micro convergence {name}", flush=True)
        res, od = api.micro_convergence(glaw, F=F)
        orders[name] = od
        print(f"  orders P {np.round(od['P'], 3)}, A {np.round(od['A'], 3)}", flush=True)
        lame = oracle.two_phase_lame(10.0)
        with oracle.law(olaw):
            for n in (4, 8):
                ref = oracle.rve_solve(2, n, api.square_inclusion_phase(n), lame, F)
                assert ref["status"] == 0
                P, A = res[n]
                assert np.linalg.norm(P - ref["P"]) <= 1e-8 * np.linalg.norm(ref["P"])
                assert np.linalg.norm(A - ref["A"]) <= 1e-6 * np.linalg.norm(ref["A"])
        # differences shrink under refinement at an order no better than 2q = 2
        for key in ("P", "A"):
            d = od[key + "_diffs"]
            assert all(d[k + 1] < d[k] for k in range(len(d) - 1))
            assert max(od[key]) <= 2.2
            assert min(od[key]) >= 0.5
    # nonlinearity barely changes the observed order (the paper's observation)
    lin = np.array(orders["linear"]["A"])
    for name in ("svk", "neo-Hookean"):
        assert np.abs(np.array(orders[name]["A"]) - lin).max() <= 0.3, (name, orders[name]["A"], lin)
