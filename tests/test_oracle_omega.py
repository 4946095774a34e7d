"""Pins for the oracle's root finders of f_d (the relaxation-factor search).

The paper compares Newton-Raphson, bisection, secant and bisection-then-
secant searches for the root of f_d, and starts the first Newton iteration
of its most charged case from three bisection midpoints in [2, 3] followed by
secant steps.  The finders are pinned on closed-form functions whose roots
and iterate sequences follow from the definitions (a secant step is exact on
a linear function, a Newton step too, bisection visits dyadic midpoints),
then on the method's own f_d, where every finder must reach the same root and
the same solution.
"""
import math

import numpy as np
import pytest

import oracle
import pbgen


def recorder(f):
    seen = []

    def g(w):
        seen.append(w)
        return f(w)
    return g, seen


def linear(root, slope=-1.0):
    return lambda w: (slope * (w - root), slope)


def test_newton_is_exact_on_a_linear_function():
    g, seen = recorder(linear(1.37))
    w, ev, fb = oracle.root_find(oracle.OMEGA_NEWTON, 2, 1.0, g, tol_omega=1e-12)
    assert fb == 0 and abs(w - 1.37) < 1e-15 and ev == 2 and seen == [1.0, w]


def test_secant_is_exact_on_a_linear_function():
    g, seen = recorder(linear(1.37, slope=-0.8))
    w, ev, fb = oracle.root_find(oracle.OMEGA_SECANT, 2, 1.0, g, tol_omega=1e-12)
    assert fb == 0 and abs(w - 1.37) < 1e-14 and ev == 3
    assert seen[:2] == [1.0, 1.125]


def test_bisection_visits_dyadic_midpoints():
    g, seen = recorder(linear(0.7))
    w, ev, fb = oracle.root_find(oracle.OMEGA_BISECT, 1, 1.0, g, tol_omega=1e-9, max_omega_it=200)
    assert fb == 0 and abs(w - 0.7) < 1e-9
    assert seen[:6] == [0.0, 4.0, 2.0, 1.0, 0.5, 0.75]
    # each midpoint halves the bracket around the root
    lo, hi = 0.0, 4.0
    for x in seen[2:]:
        assert x == 0.5 * (lo + hi)
        if x < 0.7:
            lo = x
        else:
            hi = x


def test_bisection_without_a_sign_change_continues_with_newton():
    # root at 5, outside [0, 4]: no bracket; Newton from the start value is clamped at 4
    g, seen = recorder(linear(5.0))
    w, ev, fb = oracle.root_find(oracle.OMEGA_BISECT, 1, 1.0, g, max_omega_it=10)
    assert seen[:3] == [0.0, 4.0, 1.0] and w == 4.0 and ev == 10 and fb == 0


def test_bisect_then_secant_switches_after_the_first_iteration():
    g, seen = recorder(linear(1.3))
    oracle.root_find(oracle.OMEGA_BSEC, 1, 2.0, g, tol_omega=1e-10, max_omega_it=200)
    assert seen[:3] == [0.0, 4.0, 2.0]
    g, seen = recorder(linear(1.3))
    w, ev, fb = oracle.root_find(oracle.OMEGA_BSEC, 2, 1.0, g, tol_omega=1e-10)
    assert seen[:2] == [1.0, 1.125] and ev == 3 and abs(w - 1.3) < 1e-12


def test_first_iteration_start_from_bisection_and_secant():
    # f_d = 2.3 - w: midpoints 2.5 (f < 0), 2.25 (f > 0), 2.375 (f < 0); the secant
    # through (2.25, 2.375) gives 2.3, 0.075 from 2.375, so f is taken there and the
    # next secant returns 2.3 again (< 0.05 away): Newton starts at 2.3 and stops
    g, seen = recorder(linear(2.3))
    w, ev, fb = oracle.root_find(oracle.OMEGA_NEWTON_BS, 1, 2.0, g, tol_omega=1e-10)
    assert np.allclose(seen, [2.5, 2.25, 2.375, 2.3, 2.3], rtol=0, atol=1e-14)
    assert ev == 5 and abs(w - 2.3) < 1e-14 and fb == 0
    # later iterations: plain Newton from the start value
    g, seen = recorder(linear(1.1))
    oracle.root_find(oracle.OMEGA_NEWTON_BS, 2, 1.0, g, tol_omega=1e-10)
    assert seen[0] == 1.0


def test_nonlinear_closed_form_roots():
    # f = (1 - w/2) e^{w/3}: single root at 2 in [0, 4]
    f = lambda w: ((1 - w / 2) * math.exp(w / 3), (-0.5 + (1 - w / 2) / 3) * math.exp(w / 3))
    for m in (oracle.OMEGA_NEWTON, oracle.OMEGA_BISECT, oracle.OMEGA_SECANT, oracle.OMEGA_BSEC,
              oracle.OMEGA_NEWTON_BS):
        w, ev, fb = oracle.root_find(m, 1, 1.0, f, tol_omega=1e-11, max_omega_it=200)
        assert fb == 0 and abs(w - 2.0) < 1e-9, (m, w)


def test_undefined_value_falls_back_to_one():
    for m in range(5):
        w, ev, fb = oracle.root_find(m, 1, 1.5, lambda w: None)
        assert w == 1.0 and fb == 1 and ev == 1


SPEC = dict(n=3, a=6.0, c=9.0, bump=True, t=3.0, L=3, helix=3, partials=5, kappa=0.2, seed=(9, 1))


def test_every_finder_reaches_the_same_solution():
    """On the method's own f_d with a tight search tolerance, every finder
    lands on the same root at every Newton step, so the iterates, the step
    sizes and the energy agree; only the number of f_d evaluations differs.
    At the last step the residual is at rounding level and f_d is rounding
    noise, so its root is not compared."""
    prob = pbgen.make_problem(**SPEC)
    o = oracle.Oracle.from_problem(prob)
    kw = dict(tol_nl=1e-8, tol_gr=1e-12, tol_gr0=1e-12, tol_omega=1e-9, l_e=0.0, max_gmres=20000,
              max_omega_it=200)
    ref, _, _ = o.solve(omega_method=oracle.OMEGA_NEWTON, **kw)
    assert ref["status"] == 0
    for m in (oracle.OMEGA_BISECT, oracle.OMEGA_SECANT, oracle.OMEGA_BSEC, oracle.OMEGA_NEWTON_BS):
        r, _, _ = o.solve(omega_method=m, **kw)
        assert r["status"] == 0 and r["omega_fallback"] == 0
        assert r["newton_iters"] == ref["newton_iters"], m
        assert np.allclose(r["omega"][:-1], ref["omega"][:-1], rtol=0, atol=1e-7), (m, r["omega"], ref["omega"])
        assert abs(r["total"] - ref["total"]) < 1e-9 * abs(ref["total"])


# ---------------------------------------------------------------------------
# Picard iteration (Sec. 2.4.2): A Delta = d, the same f_d, the R_e reuse rule
# ---------------------------------------------------------------------------
def test_direct_secant_formula():
    # f_d(0) = 1 in a Picard step; on a linear f_d through (0, 1) the direct
    # formula w0 / (1 - f_d(w0)) from w0 = 1/8 is the root, after one evaluation
    g, seen = recorder(lambda w: (1.0 - w / 0.37, -1.0 / 0.37))
    w, ev, fb = oracle.root_find(oracle.OMEGA_BSEC_DF, 2, 1.0, g)
    assert seen == [0.125] and ev == 1 and fb == 0 and abs(w - 0.37) < 1e-15
    g, seen = recorder(lambda w: (1.0 - w / 0.37, -1.0 / 0.37))
    oracle.root_find(oracle.OMEGA_BSEC_DF, 1, 1.0, g, omega_max=1.0, tol_omega=1e-9, max_omega_it=200)
    assert seen[:3] == [0.0, 1.0, 0.5]  # bisection of [0, 1] in the first iteration


def test_picard_fd_at_zero_is_one():
    """With Delta solving A Delta = d (the Picard step), p = -A Delta = -r(0),
    so f_d(0) = -(p + r').r / ((p + r').p) = 1 exactly (derived from eq. fd=0)."""
    prob = pbgen.make_problem(**SPEC)
    o = oracle.Oracle.from_problem(prob)
    rng = np.random.default_rng(5)
    phi = 0.3 * rng.standard_normal(o.n)
    d = -o.residual(oracle.HS, phi)
    D, st, it = o.gmres(oracle.NONE, phi, d, tol=1e-13, maxit=20000, precond=oracle.PC_CHEB_SPAI)
    assert st == 0
    f0, _, st = o.fd(oracle.HS, phi, D, 0.0)
    assert st == 0 and abs(f0 - 1.0) < 1e-9, f0
    # Newton's step does not have this property
    Dn, st, it = o.gmres(oracle.HS, phi, d, tol=1e-13, maxit=20000, precond=oracle.PC_CHEB_SPAI)
    fn, _, _ = o.fd(oracle.HS, phi, Dn, 0.0)
    assert abs(fn - 1.0) > 1e-3


def test_picard_reaches_the_newton_solution_in_more_steps():
    prob = pbgen.make_problem(**SPEC)
    o = oracle.Oracle.from_problem(prob)
    kw = dict(tol_nl=1e-9, tol_gr=1e-12, tol_gr0=1e-12, tol_omega=1e-9, l_e=0.0, max_gmres=20000, max_newton=200,
              max_omega_it=200)
    rn, _, _ = o.solve(**kw)
    rp, _, _ = o.solve(nonlinear_method=oracle.PICARD, omega_method=oracle.OMEGA_BISECT, omega_max=1.0, **kw)
    assert rn["status"] == 0 and rp["status"] == 0
    assert abs(rp["total"] - rn["total"]) < 1e-10 * abs(rn["total"])
    assert rp["newton_iters"] > 2 * rn["newton_iters"]
    assert all(0.0 <= w <= 1.0 for w in rp["omega"])


def test_picard_norm_ratio_rule():
    """The relaxation factor is reused exactly when e_{k-2} / e_{k-1} >= R_e."""
    prob = pbgen.make_problem(**SPEC)
    o = oracle.Oracle.from_problem(prob)
    r, _, _ = o.solve(nonlinear_method=oracle.PICARD, omega_method=oracle.OMEGA_BSEC_DF, omega_max=1.0, l_e=0.0,
                      r_e=1.4)
    assert r["status"] == 0
    e, w = r["e_k"], r["omega"]
    reused = 0
    for k in range(2, len(w)):
        if e[k - 2] >= 1.4 * e[k - 1]:
            assert w[k] == w[k - 1]
            reused += 1
        else:
            assert w[k] != w[k - 1]
    assert reused > 0
    # R_e = 0: a search at every step
    r0, _, _ = o.solve(nonlinear_method=oracle.PICARD, omega_method=oracle.OMEGA_BSEC_DF, omega_max=1.0, l_e=0.0,
                       r_e=0.0)
    assert all(r0["omega"][k] != r0["omega"][k - 1] for k in range(1, len(r0["omega"])))


@pytest.mark.parametrize("r_e", [1.4, 3.0, 4.5])
def test_picard_first_reuse_from_a_run_without_the_rule(r_e):
    """The norm-ratio rule (the section on reducing omega searches: search
    again only when the ratio of the two latest step norms falls below R_e),
    checked against a run that never applies it.  Until the rule first
    reuses a factor, a run with R_e and one with R_e = 0 take identical steps,
    so the step norms e_1, e_2, ... of the R_e = 0 run, which the rule played
    no part in producing, fix the first reuse: the smallest k >= 3 with
    e_{k-2} >= R_e e_{k-1}.  The three thresholds put it at three different
    steps of the same sequence, so using other step norms (e_{k-3}/e_{k-2},
    the inverse ratio), another first step or the opposite comparison moves
    it and fails."""
    prob = pbgen.make_problem(**SPEC)
    o = oracle.Oracle.from_problem(prob)
    kw = dict(nonlinear_method=oracle.PICARD, omega_method=oracle.OMEGA_BSEC_DF, omega_max=1.0, l_e=0.0)
    r0, _, _ = o.solve(r_e=0.0, **kw)
    e0, w0 = r0["e_k"], r0["omega"]
    kstar = next(k for k in range(3, len(e0) + 1) if e0[k - 3] >= r_e * e0[k - 2])
    assert all(w0[j] != w0[j - 1] for j in range(1, len(w0)))  # R_e = 0: a new factor at every step
    r, _, _ = o.solve(r_e=r_e, **kw)
    assert r["status"] == 0
    e, w = r["e_k"], r["omega"]
    for j in range(kstar - 1):  # steps 1 .. k* - 1 as without the rule
        assert w[j] == pytest.approx(w0[j], rel=1e-12, abs=0.0)
        assert e[j] == pytest.approx(e0[j], rel=1e-12, abs=0.0)
    assert w[kstar - 1] == w[kstar - 2]  # step k* reuses the factor of step k* - 1
    assert w0[kstar - 1] != pytest.approx(w0[kstar - 2], rel=1e-6)
