"""Matrix-free boundary-element mode through the C ABI.

Nothing dense is stored: every apply evaluates the regular quadrature-point
pairs on the fly and adds the touching-pair blocks and 1/2 M kept from setup.
The integrals are those of the dense operator, summed in another order, so
the residual and Jacobian products must match the oracle at the FP64 bar,
full solves reach the oracle's energy, mixed precision stays within its bar,
and a matrix-free instance gives the same result solo and in a batch.
"""
import sys

import numpy as np
import pytest

import oracle
import pbgen

pytestmark = pytest.mark.gpu

CASES = {
    "sphere_n4": dict(n=4, a=4.0, c=4.0, bump=False, t=4.0, L=6, helix=0, partials=0, kappa=0.125,
                      center_charge=1.0),
    "bumpy_n3": dict(n=3, a=6.0, c=9.0, bump=True, t=3.0, L=3, helix=3, partials=5, kappa=0.2, seed=(9, 1)),
    "icosahedron": dict(n=1, a=4.0, c=4.0, bump=False, t=3.0, L=2, helix=0, partials=0, kappa=0.3,
                        center_charge=-2.0),
}
TIGHT = dict(tol_nl=1e-10, tol_gr=1e-12, tol_gr0=1e-12, tol_omega=1e-9, l_e=0.0, max_gmres=20000)


def log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def rel(a, b):
    return np.abs(np.asarray(a) - np.asarray(b)).max() / max(np.abs(np.asarray(b)).max(), 1e-300)


@pytest.fixture(scope="module")
def ctx():
    import paper_2511_21713_amd as pb
    return pb.Context(0)


@pytest.fixture(scope="module", params=sorted(CASES))
def case(request, ctx):
    import paper_2511_21713_amd as pb
    name = request.param
    log(f"[gpu matrix-free] case {name}")
    prob = pbgen.make_problem(**CASES[name])
    o = oracle.Oracle.from_problem(prob)
    g = pb.Problem.from_inputs(ctx, prob)
    g.set_bem_mode(pb.BEM_MATRIX_FREE)
    return name, prob, o, g


@pytest.mark.parametrize("scheme", [oracle.LIN, oracle.HS])
def test_matrix_free_products_match_oracle(case, scheme):
    name, prob, o, g = case
    rng = np.random.default_rng(21 + scheme)
    phi = rng.standard_normal(o.n)
    v = rng.standard_normal(o.n)
    eF = rel(g.residual(scheme, phi), o.residual(scheme, phi))
    eJ = rel(g.apply_jacobian(scheme, phi, v), o.apply_jacobian(scheme, phi, v))
    log(f"  {name} scheme {scheme}: F {eF:.2e} Jv {eJ:.2e}")
    assert eF < 1e-12 and eJ < 1e-12


def test_matrix_free_tight_solve_matches_oracle(case):
    """The approximate inverse from the near field of V' preconditions about
    as well as the one from full rows: the Krylov count stays close to the
    dense path's (the oracle uses full rows), and far below the count with
    the inverse diagonal."""
    name, prob, o, g = case
    rg = g.solve(**TIGHT)
    ro, _, _ = o.solve(**TIGHT)
    rd = g.solve(precond=0, **TIGHT)
    log(f"  {name}: total {rg['total']!r} vs {ro['total']!r}, gmres {rg['gmres_iters_total']} "
        f"(oracle {ro['gmres_iters_total']}, inverse diagonal {rd['gmres_iters_total']})")
    assert rg["status"] == 0 and rd["status"] == 0
    assert abs(rg["total"] - ro["total"]) < 1e-10 * abs(ro["total"])
    assert abs(rd["total"] - ro["total"]) < 1e-10 * abs(ro["total"])
    assert rg["gmres_iters_total"] <= 1.25 * ro["gmres_iters_total"]


def test_matrix_free_mixed_precision(case, ctx):
    """FP32 evaluation rounds the source strengths of every apply, so the
    apply is linear only to ~1e-7 and GMRES is run to 1e-7 (a dense FP32
    operator is exactly linear); the energy bar is the mixed one."""
    import paper_2511_21713_amd as pb
    name, prob, o, _ = case
    gm = pb.Problem.from_inputs(ctx, prob, precision=pb.MIXED)
    gm.set_bem_mode(pb.BEM_MATRIX_FREE)
    rng = np.random.default_rng(5)
    phi = rng.standard_normal(o.n)
    v = rng.standard_normal(o.n)
    eJ = rel(gm.apply_jacobian(oracle.HS, phi, v), o.apply_jacobian(oracle.HS, phi, v))
    rm = gm.solve(**dict(TIGHT, tol_nl=1e-6, tol_gr=1e-7, tol_gr0=1e-7, tol_omega=1e-6))
    ro, _, _ = o.solve(**TIGHT)
    eE = abs(rm["total"] - ro["total"]) / abs(ro["total"])
    log(f"  {name} mixed matrix-free: Jv {eJ:.2e}, energy {eE:.2e}")
    assert eJ < 1e-5 and rm["status"] == 0 and eE < 1e-5
    gm.close()


def test_matrix_free_same_in_a_batch_and_beside_dense(ctx):
    import paper_2511_21713_amd as pb
    probs = [pbgen.make_problem(**CASES[k]) for k in sorted(CASES)]
    solo = []
    for prob in probs:
        g = pb.Problem.from_inputs(ctx, prob)
        g.set_bem_mode(pb.BEM_MATRIX_FREE)
        solo.append(g.solve(**TIGHT))
        g.close()
    gs = []
    for i, prob in enumerate(probs):
        g = pb.Problem.from_inputs(ctx, prob)
        if i != 1:
            g.set_bem_mode(pb.BEM_MATRIX_FREE)
        gs.append(g)
    code, res = pb.solve_batch(ctx, gs, **TIGHT)
    assert code == 0
    for i, (r, s) in enumerate(zip(res, solo)):
        if i == 1:  # the dense instance: same energy to rounding
            assert abs(r["total"] - s["total"]) < 1e-10 * abs(s["total"])
        else:
            assert r["total"] == s["total"] and r["gmres_iters"] == s["gmres_iters"]
    for g in gs:
        g.close()


def test_export_refused_in_matrix_free_mode(case):
    import paper_2511_21713_amd as pb
    name, prob, o, g = case
    with pytest.raises(pb.PbfbError):
        g.export_bem(0)
