"""Pins for the per-iteration scheme schedule of the oracle's Newton solve.

Sec. 3.3.1 raises the reaction term over the first iterations: the cubic
Taylor polynomial of sinh, then the 5th and 7th orders, then sinh itself
(T3-HS, T3-T5-HS, T3-T5-T7-T7-HS).  Each scheduled step is a Newton step
(eq. NR_main) with that step's N and J, so two steps at a fixed relaxation
factor are rebuilt here from the oracle's residual, Jacobian and GMRES
pieces; any schedule that ends in sinh reaches the sinh solution.
"""
import numpy as np

import oracle
import pbgen

SPEC = dict(n=3, a=6.0, c=9.0, bump=True, t=3.0, L=3, helix=3, partials=5, kappa=0.2, seed=(9, 1))
GM = dict(tol=1e-13, maxit=20000, precond=oracle.PC_CHEB_SPAI)


def _oracle():
    return oracle.Oracle.from_problem(pbgen.make_problem(**SPEC))


def manual_steps(o, schemes, omega=1.0):
    """Phi_L from (A + J_LIN) Phi_L = b, then per scheme s: d = -F_s(Phi),
    J_s(Phi) Delta = d, Phi_NL += omega Delta."""
    b = o.rhs()
    phil, st, _ = o.gmres(oracle.LIN, b, b, **GM)
    assert st == 0
    phinl = np.zeros(o.n)
    es = []
    for s in schemes:
        phi = phil + phinl
        D, st, _ = o.gmres(s, phi, -o.residual(s, phi), **GM)
        assert st == 0
        phinl = phinl + omega * D
        es.append(omega * np.linalg.norm(D))
    return phil, phinl, es


def test_scheduled_steps_use_the_listed_schemes():
    o = _oracle()
    kw = dict(omega_auto=0, omega_fixed=1.0, max_newton=2, tol_nl=0.0, tol_gr=1e-13, tol_gr0=1e-13, l_e=0.0,
              max_gmres=20000)
    seconds = {}
    for sched in ([oracle.T3, oracle.T5], [oracle.T3, oracle.T7], [oracle.T5, oracle.HS]):
        r, pl, pn = o.solve(schedule=sched, **kw)
        assert r["newton_iters"] == 2
        ml, mn, es = manual_steps(o, sched)
        assert np.linalg.norm(pn - mn) < 1e-9 * np.linalg.norm(mn)
        assert np.allclose(r["e_k"], es, rtol=1e-9, atol=0)
        seconds[tuple(sched)] = r["e_k"][1]
    # the second step differs between T5 and T7, so a swapped scheme is seen
    a, b = seconds[(oracle.T3, oracle.T5)], seconds[(oracle.T3, oracle.T7)]
    assert abs(a - b) > 1e-6 * abs(a)


def test_one_entry_schedule_is_the_cubic_start():
    o = _oracle()
    r0, _, _ = o.solve()
    r1, _, _ = o.solve(schedule=[oracle.T3])
    assert r0["total"] == r1["total"] and r0["omega"] == r1["omega"]
    r2, _, _ = o.solve(scheme_first=oracle.HS)
    r3, _, _ = o.solve(schedule=[oracle.HS])
    assert r2["total"] == r3["total"] and r2["omega"] == r3["omega"]


def test_schedules_reach_the_sinh_solution():
    o = _oracle()
    kw = dict(tol_nl=1e-9, tol_gr=1e-12, tol_gr0=1e-12, tol_omega=1e-9, l_e=0.0, max_gmres=20000)
    ref, _, _ = o.solve(**kw)
    assert ref["status"] == 0
    for sched in ([oracle.T3, oracle.T5], [oracle.T3, oracle.T5, oracle.T7, oracle.T7]):
        r, _, _ = o.solve(schedule=sched, **kw)
        assert r["status"] == 0 and r["newton_iters"] > len(sched)
        assert abs(r["total"] - ref["total"]) < 1e-10 * abs(ref["total"])
