"""What the trained network gains (Section 3.3's prediction step, stood in for by the MLP):
on fresh 3-D systems outside the training family, solve_auto with the committed weights (the
default (0.5, 0.5) judging each prediction) against plain default-parameter GADI-IR, both to
RES 1e-10 in half precision.  Device time includes the guard's probes."""
import math

import numpy as np
import pytest

import gadi_inputs as gi
import oracle

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover - CPU container
    pytest.skip("no GPU", allow_module_level=True)

import paper_2501_04229_amd as gadi  # noqa: E402
from paper_2501_04229_amd import predictor as pr  # noqa: E402

# eight systems of the evaluation family's kind at n in [64, 96], seeded apart from it
SUBSET = dict(count=8, seed=5, nmin=64, nmax=96)


def gain_records(p, subset=SUBSET, tol=1e-10):
    """Per system: device seconds and sweeps of the default solve and of solve_auto."""
    rows = []
    for n, dim, beta, seed in gi.test_family(**subset):
        A = gi.convdiff(n, dim, beta)
        xs, b = gi.rhs_for(A, "uniform", seed)
        g = gadi.System(A)
        bd = torch.from_numpy(b).cuda()
        g.solve(bd, 0.5, 0.5, tol=tol, maxit_outer=3)  # launch-shape tuning, not timed
        xd, idf = g.solve(bd, 0.5, 0.5, tol=tol)
        # the default's measured work is the judge of the prediction
        xa, iau, used = pr.solve_auto(g, A, bd, p, tol=tol, judge=pr.work(idf))
        torch.cuda.synchronize()
        rows.append({"n": n, "beta": beta, "A": A, "b": b, "x": xa.cpu().numpy(), "used": used,
                     "default": idf, "auto": iau,
                     "t_default": idf["seconds"], "t_auto": iau["seconds"] + iau["guard_seconds"]})
        g.close()
    return rows


def test_trained_network_gains_over_the_default():
    rows = gain_records(pr.load())
    for r in rows:
        print(f"# n={r['n']} beta={r['beta']:.3g}: default {r['t_default']:.4f}s "
              f"({r['default']['outer_sweeps']} sweeps), auto {r['t_auto']:.4f}s "
              f"({r['auto']['outer_sweeps']} sweeps, used {r['used']})", flush=True)
        assert r["default"]["status"] == gadi.OK and r["auto"]["status"] == gadi.OK, r
        o = oracle.OracleSystem(r["A"])
        rel = np.linalg.norm(r["b"] - o.spmv("A", r["x"])) / np.linalg.norm(r["b"])
        assert rel <= 1.0000001e-10, rel
    gain = math.exp(np.mean([math.log(r["t_default"] / r["t_auto"]) for r in rows]))
    print(f"# geometric-mean device-time gain {gain:.3f}", flush=True)
    assert gain > 1.0
