"""Batched solves and the continuous-batching server through the C ABI.

Every instance's arithmetic (work lists, reduction orders, Krylov control) is
independent of the rest of its batch, so a result must equal the solo
result bit for bit, in a batch and when admitted mid-flight by the server.
Solo results themselves are checked against the oracle.
"""
import time

import numpy as np
import pytest

import oracle
import pbgen

pytestmark = pytest.mark.gpu

SPECS = [
    dict(n=4, a=4.0, c=4.0, bump=False, t=4.0, L=6, helix=0, partials=0, kappa=0.125, center_charge=1.0),
    dict(n=3, a=6.0, c=9.0, bump=True, t=3.0, L=3, helix=3, partials=5, kappa=0.2, seed=(9, 1)),
    dict(n=1, a=4.0, c=4.0, bump=False, t=3.0, L=2, helix=0, partials=0, kappa=0.3, center_charge=-2.0),
    dict(n=6, a=8.0, c=14.0, bump=True, t=5.0, L=5, helix=6, partials=20, kappa=0.05, seed=(9, 2)),
    dict(n=5, a=5.0, c=5.0, bump=False, t=4.0, L=4, helix=0, partials=0, kappa=0.33, center_charge=3.0),
]
OPTS = dict(tol_nl=1e-9, tol_gr=1e-11, tol_gr0=1e-11, tol_omega=1e-8, l_e=0.0, max_gmres=20000)


@pytest.fixture(scope="module")
def setup():
    import paper_2511_21713_amd as pb
    ctx = pb.Context(0)
    probs = [pbgen.make_problem(**s) for s in SPECS]
    solo = []
    for prob in probs:
        g = pb.Problem.from_inputs(ctx, prob)
        solo.append(g.solve(**OPTS))
        g.close()
    return pb, ctx, probs, solo


def test_solo_matches_oracle(setup):
    pb, ctx, probs, solo = setup
    for prob, r in zip(probs[:3], solo[:3]):
        ro, _, _ = oracle.Oracle.from_problem(prob).solve(**OPTS)
        assert abs(r["total"] - ro["total"]) < 1e-10 * abs(ro["total"])


@pytest.mark.parametrize("precision", [0, 1])
def test_batch_equals_solo_bitwise(setup, precision):
    pb, ctx, probs, solo = setup
    if precision == 1:
        solo = []
        for prob in probs:
            g = pb.Problem.from_inputs(ctx, prob, precision=1)
            solo.append(g.solve(**OPTS))
            g.close()
    gs = [pb.Problem.from_inputs(ctx, prob, precision=precision) for prob in probs]
    code, res = pb.solve_batch(ctx, gs, **OPTS)
    assert code == 0
    for r, s in zip(res, solo):
        print(f"  batch {r['total']!r} solo {s['total']!r} newton {r['newton_iters']} gmres {r['gmres_iters_total']}",
              flush=True)
        assert r["status"] == 0
        assert r["total"] == s["total"] and r["lc"] == s["lc"] and r["nc"] == s["nc"]
        assert r["newton_iters"] == s["newton_iters"] and r["gmres_iters"] == s["gmres_iters"]


def test_graph_replay_equals_eager_launches(setup):
    """The Krylov step replayed from a captured HIP graph gives the same
    results bit for bit as launching its kernels one by one, solo and in a
    batch, across repeated solves (every replay reuses the capture)."""
    pb, ctx, probs, solo = setup
    for prec in (pb.FP64, pb.MIXED):
        eager, graph = [], []
        for prob in probs[:3]:
            g = pb.Problem.from_inputs(ctx, prob, precision=prec)
            eager.append(g.solve(hip_graph=0, **OPTS))
            for _ in range(2):
                r = g.solve(hip_graph=1, **OPTS)
                assert r["total"] == eager[-1]["total"] and r["gmres_iters"] == eager[-1]["gmres_iters"]
            graph.append(r)
            g.close()
        gs = [pb.Problem.from_inputs(ctx, prob, precision=prec) for prob in probs[:3]]
        for rep in range(2):
            code, res = pb.solve_batch(ctx, gs, hip_graph=1, **OPTS)
            assert code == 0
            for r, e in zip(res, eager):
                assert r["total"] == e["total"] and r["gmres_iters"] == e["gmres_iters"]
        for g in gs:
            g.close()


def test_batch_isolates_a_failing_instance(setup):
    pb, ctx, probs, solo = setup
    gs = [pb.Problem.from_inputs(ctx, prob) for prob in probs[:3]]
    gs[1].set_charges(np.array([[0.0, 0.0, 100.0]]), np.array([1.0]))  # outside the solute
    code, res = pb.solve_batch(ctx, gs, **OPTS)
    assert code == pb.ECHARGE
    assert res[1]["status"] == pb.ECHARGE
    assert res[0]["status"] == 0 and res[0]["total"] == solo[0]["total"]
    assert res[2]["status"] == 0 and res[2]["total"] == solo[2]["total"]


def test_server_results_equal_solo(setup):
    pb, ctx, probs, solo = setup
    srv = pb.Server(ctx, hbm_budget_bytes=8 << 30, max_slots=2)
    tickets = []
    gs = []
    for i, prob in enumerate(probs):
        g = pb.Problem.from_inputs(ctx, prob)
        gs.append(g)
        tickets.append(srv.submit(g, **OPTS))
        time.sleep(0.01 * i)  # staggered arrivals join a running batch
    out = {}
    t0 = time.time()
    while len(out) < len(tickets) and time.time() - t0 < 120:
        for t in tickets:
            if t not in out:
                r = srv.poll(t)
                if r is not None:
                    out[t] = r
        time.sleep(0.005)
    srv.close()
    assert len(out) == len(tickets)
    for t, s in zip(tickets, solo):
        assert out[t]["status"] == 0
        assert out[t]["total"] == s["total"], (out[t]["total"], s["total"])


def test_server_rejects_oversized_request(setup):
    pb, ctx, probs, solo = setup
    srv = pb.Server(ctx, hbm_budget_bytes=1 << 20, max_slots=1)
    g = pb.Problem.from_inputs(ctx, probs[0])
    with pytest.raises(pb.PbfbError) as e:
        srv.submit(g)
    assert e.value.code == pb.ENOMEM
    srv.close()


def test_server_budget_binds_requests_wait(setup):
    """An HBM budget that holds one request at a time: later requests wait for
    admission (t_wait_s > 0) instead of failing, the device memory in use
    (hipMemGetInfo, sampled while serving) stays within the budget, every
    completed request has released its device memory, and each result equals
    its solo result bit for bit."""
    import threading

    import torch
    pb, ctx, probs, solo = setup
    gs = [pb.Problem.from_inputs(ctx, prob) for prob in probs]
    fp = [g.footprint(**OPTS) for g in gs]
    budget = int(1.2 * max(a + b for a, b in fp))
    assert min(a for a, _ in fp) * 2 > budget  # no two requests fit together
    low, free0 = [0], 0
    stop = threading.Event()
    th = None
    out, tickets = {}, []
    srv = pb.Server(ctx, hbm_budget_bytes=budget, max_slots=4)
    gw = pb.Problem.from_inputs(ctx, probs[0])
    try:
        # one request first, so that the runtime's own lazy allocations (code
        # objects, queues, graph resources) are in place before the baseline
        tw = srv.submit(gw, **OPTS)
        t0 = time.time()
        while srv.poll(tw) is None and time.time() - t0 < 60:
            time.sleep(0.002)
        torch.cuda.synchronize()
        free0 = torch.cuda.mem_get_info()[0]
        low[0] = free0

        def sample():
            while not stop.is_set():
                low[0] = min(low[0], torch.cuda.mem_get_info()[0])
                time.sleep(0.0005)

        th = threading.Thread(target=sample, daemon=True)
        th.start()
        tickets = [srv.submit(g, **OPTS) for g in gs]
        t0 = time.time()
        while len(out) < len(tickets) and time.time() - t0 < 120:
            for t in tickets:
                if t not in out:
                    r = srv.poll(t)
                    if r is not None:
                        out[t] = r
            time.sleep(0.002)
    finally:
        srv.close()
        stop.set()
        if th is not None:
            th.join()
    assert len(out) == len(tickets)
    waits = [out[t]["t_wait_s"] for t in tickets]
    print(f"  budget {budget / 2**20:.0f} MiB (footprints {[(round(a / 2**20), round(b / 2**20)) for a, b in fp]} "
          f"MiB), admission waits {['%.3f' % w for w in waits]} s, peak device use "
          f"{(free0 - low[0]) / 2**20:.1f} MiB", flush=True)
    assert sum(w > 1e-3 for w in waits) >= len(tickets) - 2
    assert free0 - low[0] <= budget
    for g in gs + [gw]:
        assert g.hbm() == 0  # released at completion
    for t, s in zip(tickets, solo):
        assert out[t]["status"] == 0
        assert out[t]["total"] == s["total"], (out[t]["total"], s["total"])
    for g in gs + [gw]:
        g.close()
