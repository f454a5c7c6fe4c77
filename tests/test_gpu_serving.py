"""The serving loop (dao_server_*): requests admitted as slots and memory
free up, rounds of all live solves advanced together, each result the plan
its solo dao_solve gives (same round beams and reduced costs; F within 1e-9
in FP64, 1e-5 in FP32, as for dao_solve_batch), and served plans against
the oracle directly (its solve in FP64, its stored trajectory in FP32)."""
import time

import numpy as np
import pytest

import paper_1003_5402_amd as dao
from gpu_util import ctx_for, torch_cuda
from phantom import make_phantom

pytestmark = pytest.mark.gpu

REQS = [("mini", 0, "f64", 5), ("tiny", 0, "f32", 6), ("tiny", 1, "f32", 4), ("mini", 1, "f32", 6),
        ("tiny", 2, "f64", 5)]


def _alone(ph, dtype, n_ap):
    ctx = ctx_for(ph, dtype=dtype)
    try:
        return ctx.solve(n_ap), ctx.info()["device_bytes"]
    finally:
        ctx.close()


def _drain(server, tickets, limit_s=120.0):
    """Step until every ticket is done (the admission thread may still be
    building contexts when a step finds nothing live)."""
    results, max_live, max_used = {}, 0, 0
    t0 = time.time()
    while len(results) < len(tickets):
        assert time.time() - t0 < limit_s, "serving loop made no progress"
        live, _done = server.step()
        info = server.info()
        max_live, max_used = max(max_live, live), max(max_used, info["used_bytes"])
        for t in tickets:
            if t not in results:
                state, plan = server.poll(t)
                if state == 2:
                    results[t] = plan
        if live == 0:
            time.sleep(0.001)
    return [results[t] for t in tickets], max_live, max_used


def _run(server, reqs, phs):
    tickets = [server.submit(ph, n, dtype=dt) for (_, _, dt, n), ph in zip(reqs, phs)]
    return _drain(server, tickets)


@pytest.mark.parametrize("batch_masters,workers", [(True, 4), (False, 1)])
def test_serving_results_equal_solo_solves(batch_masters, workers):
    """With one admission thread, and with four building contexts at once
    (requests may then be admitted out of arrival order)."""
    torch = torch_cuda()
    phs = [make_phantom(n, s) for n, s, _, _ in REQS]
    solo = [_alone(ph, dt, n) for ph, (_, _, dt, n) in zip(phs, REQS)]
    server = dao.Server(max_live=3, stream=torch.cuda.current_stream().cuda_stream, batch_masters=batch_masters,
                        workers=workers)
    try:
        res, max_live, _ = _run(server, REQS, phs)
        assert max_live <= 3
        for (name, seed, dt, n), r, (ref, _) in zip(REQS, res, solo):
            tol = 1e-9 if dt == "f64" else 1e-5
            print(f"[serve] {name}/{seed} {dt}: rounds {r['rounds']} F {r['F']:.10e} solo {ref['F']:.10e}", flush=True)
            assert r["status"] == ref["status"] and r["rounds"] == ref["rounds"]
            assert np.array_equal(r["round_beam"], ref["round_beam"])
            assert abs(r["F"] - ref["F"]) <= tol * ref["F"]
            np.testing.assert_allclose(r["round_rc"], ref["round_rc"], rtol=100 * tol)
    finally:
        server.close()


def test_admission_respects_the_memory_cap():
    torch = torch_cuda()
    reqs = [("tiny", s, "f32", 3) for s in range(4)]
    phs = [make_phantom(n, s) for n, s, _, _ in reqs]
    sizes = [_alone(ph, "f32", 3)[1] for ph in phs]
    cap = int(max(sizes) * 2.5)                      # room for two contexts at a time
    server = dao.Server(max_live=8, hbm_cap_bytes=cap, stream=torch.cuda.current_stream().cuda_stream)
    try:
        res, max_live, max_used = _run(server, reqs, phs)
        assert max_used <= cap and max_live <= 2
        assert all(r["rounds"] == 3 for r in res)
    finally:
        server.close()
    # a request that cannot fit even alone ends with DAO_ENOMEM, the others run
    server = dao.Server(max_live=4, hbm_cap_bytes=min(sizes) // 4, stream=torch.cuda.current_stream().cuda_stream)
    try:
        t = server.submit(phs[0], 3, dtype="f32")
        (plan,), _, _ = _drain(server, [t])
        assert plan["status"] == dao.DAO_ENOMEM
    finally:
        server.close()


def test_served_plans_against_the_oracle():
    """Plans served in a mix (the prostate-shaped 50-aperture plan in FP32 next
    to 32^3 plans in FP64 and FP32) against the oracle directly: the FP64
    plan takes the oracle's aperture wherever the decision gap exceeds 1e-9
    (objective after every round within 1e-9); the prostate-shaped plan
    matches the oracle's stored trajectory round by round up to its first
    decision within the master's tolerance (objective within 1e-5)."""
    import json
    import os

    import oracle
    from conftest import oracle_problem
    torch = torch_cuda()
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "prostate_seed0_r50.json")
    if not os.path.exists(path):
        pytest.skip("no stored trajectory")
    with open(path) as f:
        doc = json.load(f)
    reqs = [("prostate", 0, "f32", 50), ("tiny", 0, "f64", 10), ("tiny", 1, "f32", 6)]
    phs = [make_phantom(n, s) for n, s, _, _ in reqs]
    server = dao.Server(max_live=3, stream=torch.cuda.current_stream().cuda_stream)
    try:
        res, _, _ = _run(server, reqs, phs)
    finally:
        server.close()
    # the FP64 32^3 plan against the oracle's solve
    P = oracle_problem(phs[1])
    ref = oracle.solve(P, 10, eps=1e-6)
    r = res[1]
    assert r["rounds"] == len(ref["log"])
    for k, rec in enumerate(ref["log"]):
        if rec["gap"] > 1e-9:
            assert r["round_beam"][k] == rec["beam"], k
        assert abs(r["round_F"][k] - rec["F"]) <= 1e-9 * rec["F"], k
    # the prostate-shaped plan against the stored trajectory
    r = res[0]
    assert r["rounds"] == 50
    rc1 = doc["rc1"]
    matched = 0
    for k, rec in enumerate(doc["rounds"]):
        # the plan records each round's beam, reduced cost and objective, not
        # the leaves: another aperture of the same beam with a reduced cost
        # within the master's tolerance shows in the objective after the round
        if (r["round_beam"][k] != rec["beam"] or abs(r["round_rc"][k] - rec["rc"]) > 1e-6 * abs(rc1)
                or abs(r["round_F"][k] - rec["F"]) > 1e-5 * rec["F"]):
            assert rec["gap"] <= 1e-6 * abs(rc1), (k, rec["gap"])
            break
        matched += 1
    print(f"[serve] prostate served plan: {matched} of 50 rounds match the oracle's, F {r['F']:.10e} "
          f"oracle {doc['F']:.10e}", flush=True)
