"""The continuous-batching solve server.

Each request's alpha computed in the mix (batched matvecs with other requests, admitted
and retired while others run) must be bitwise equal to solving it alone with
dwfmm_fmm_solve (FP64, same CG, same reduction order); its residual is re-measured by
the CPU oracle.  Admission under a tiny memory budget serialises requests; a request
with invalid data is finished with an error while the others complete.
"""
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_2402_09531_amd as dw  # noqa: E402
from paper_2402_09531_amd import workloads as W  # noqa: E402


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def requests(count=7, seed=3):
    rng = np.random.default_rng(seed)
    out = []
    for i in range(count):
        n = int(rng.integers(1500, 9000))
        d = int(rng.integers(3, 9))
        X = W.points(n, d, 2.0, 500 + i)
        f = np.sin(X.sum(1))
        out.append(dict(X=X, b=W.dim_weights(d, 2.0), f=f, kernel="matern32", ell=1.0, q=4, lam=1.0,
                        rtol=1e-10, max_iter=400, leaf=64, eta=0.8))
    return out


def alone(r):
    tree = dw.build_tree(torch.from_numpy(r["X"]).cuda(), r["b"], r["leaf"], r["eta"])
    op = dw.fmm_create(tree, r["kernel"], r["ell"], r["q"])
    fd = torch.from_numpy(r["f"][:, None]).cuda()
    ad = torch.zeros_like(fd)
    info = dw.fmm_solve(op, r["lam"], fd, ad, r["rtol"], r["max_iter"])[0]
    return ad.cpu().numpy()[:, 0], info


def run_server(reqs, budget, stagger=2):
    srv = dw.Server(budget, max_active=16, check_every=1)
    ids, results, pending = [], {}, list(range(len(reqs)))
    ticks = 0
    while pending or len(results) < len(ids):
        # requests arrive while others are running
        for _ in range(min(stagger, len(pending))):
            k = pending.pop(0)
            r = reqs[k]
            ids.append(srv.submit(r["X"], r["b"], r["f"], r["leaf"], r["eta"], r["kernel"], r["ell"], r["q"],
                                  r["lam"], r["rtol"], r["max_iter"]))
        srv.tick()
        ticks += 1
        for k, rid in enumerate(ids):
            if k in results:
                continue
            out = srv.result(rid)
            if out is not None:
                results[k] = out
        assert ticks < 100000
    assert srv.bytes_held() == 0
    return results


def test_server_results_equal_alone(orc):
    reqs = requests()
    results = run_server(reqs, budget=1 << 40)
    for k, r in enumerate(reqs):
        a_mix, info_mix = results[k]
        a_alone, info_alone = alone(r)
        say(f"[server] request {k}: n={len(r['f'])} iters {info_mix['iters']} status {info_mix['status']} "
            f"alone iters {info_alone['iters']}")
        assert info_mix["status"] == 0 and info_alone["status"] == 0
        assert info_mix["iters"] == info_alone["iters"]
        assert np.array_equal(a_mix, a_alone)
    r = reqs[0]
    P = orc.Plan(r["X"], r["b"], r["leaf"], r["eta"], r["kernel"], r["ell"], r["q"])
    a = results[0][0]
    res = np.linalg.norm(r["f"] - (P.matvec(a) + r["lam"] * a)) / np.linalg.norm(r["f"])
    assert res <= 1.05 * r["rtol"]


def test_server_tiny_budget_and_failed_request():
    reqs = requests(count=4, seed=9)
    bad = dict(reqs[1])
    bad["X"] = bad["X"].copy()
    bad["X"][5, 0] = np.nan
    reqs.insert(2, bad)
    results = run_server(reqs, budget=1, stagger=5)   # one request at a time
    for k in range(len(reqs)):
        status = results[k][1]["status"]
        assert status == (dw.E_NONFINITE if k == 2 else 0), (k, status)


def test_server_reduced_precision_request_status(orc):
    """An FP32 request runs CG on its FP32 operator without refinement: at a tolerance that operator
    reaches, OK with the FP64 residual within it; at 1e-9, below the FP32 operator's accuracy, its
    recursive residual may still get there, but the FP64 residual does not and the status says so."""
    r = requests(count=1, seed=21)[0]
    srv = dw.Server(1 << 40, max_active=4, check_every=1)
    ids = [srv.submit(r["X"], r["b"], r["f"], r["leaf"], r["eta"], r["kernel"], r["ell"], r["q"], r["lam"], rtol,
                      r["max_iter"], precision="fp32") for rtol in (1e-3, 1e-9)]
    done, ticks = {}, 0
    while len(done) < 2:
        srv.tick()
        ticks += 1
        assert ticks < 100000
        for rid in ids:
            if rid not in done:
                out = srv.result(rid)
                if out is not None:
                    done[rid] = out
    (a1, i1), (a2, i2) = done[ids[0]], done[ids[1]]
    say(f"[server fp32] rtol 1e-3: status {i1['status']} true {i1['rel_res_true']:.2e}; "
        f"rtol 1e-9: status {i2['status']} recursive {i2['rel_res_recursive']:.2e} true {i2['rel_res_true']:.2e}")
    assert i1["status"] == 0 and i1["rel_res_true"] <= 1e-3
    assert i2["rel_res_true"] > 1e-9 and i2["status"] == dw.E_NOT_CONVERGED
    # the reported FP64 residual is the oracle's
    P = orc.Plan(r["X"], r["b"], r["leaf"], r["eta"], r["kernel"], r["ell"], r["q"])
    res = np.linalg.norm(r["f"] - (P.matvec(a2) + r["lam"] * a2)) / np.linalg.norm(r["f"])
    assert abs(res - i2["rel_res_true"]) <= 1e-3 * res
