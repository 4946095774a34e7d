"""The two-field form (Sec. 2.3, eq. fembem_matrix) through the C ABI.

FEM on the solute and the shell with the point charges as load, Yukawa BEM
on Gamma_s, lambda_m recovered after the solve from the trace of u with the
Laplace operators of Gamma_m (Sec. 2.3.1).  The load, the residual and
Jacobian products must match the oracle at the FP64 bar, full solves its
energy (the oracle recovers lambda_m by a dense solve, the library by
conjugate gradients), mixed precision stays within its bar, and a two-field
instance gives the same result solo and in a batch beside a shell-only one.
"""
import sys

import numpy as np
import pytest

import oracle
import pbgen

pytestmark = pytest.mark.gpu

CASES = {
    "bumpy_n3": dict(n=3, a=6.0, c=9.0, bump=True, t=3.0, L=3, helix=3, partials=5, kappa=0.2, seed=(9, 1),
                     solute_layers=3),
    "sphere_n8": dict(n=8, a=4.0, c=4.0, bump=False, t=4.0, L=6, helix=0, partials=0, kappa=0.125,
                      center_charge=6.0, solute_layers=4),
    "bumpy_n16": dict(n=16, a=8.0, c=12.0, bump=True, t=4.0, L=4, helix=8, partials=40, kappa=0.125, seed=(3, 2),
                      solute_layers=3),
}
TIGHT = dict(tol_nl=1e-10, tol_gr=1e-12, tol_gr0=1e-12, tol_omega=1e-9, l_e=0.0, max_gmres=20000)


_ORACLE = {}


def oracle_solve(name, o):
    if name not in _ORACLE:
        _ORACLE[name] = o.solve(**TIGHT)
    return _ORACLE[name]


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
    log(f"[gpu two-field] case {name}")
    prob = pbgen.make_problem(**CASES[name])
    o = oracle.Oracle.from_problem(prob)
    g = pb.Problem.from_inputs(ctx, prob)
    return name, prob, o, g


def test_two_field_load_matches_oracle(case):
    name, prob, o, g = case
    b, bo = g.export_rhs(), o.rhs()
    log(f"  {name}: load {rel(b, bo):.2e}")
    assert rel(b, bo) < 1e-13
    assert np.all(b[o.n_nodes:] == 0.0)


@pytest.mark.parametrize("scheme", [oracle.LIN, oracle.T3, oracle.HS])
def test_two_field_products_match_oracle(case, scheme):
    name, prob, o, g = case
    rng = np.random.default_rng(31 + scheme)
    phi = rng.standard_normal(o.n)
    v = rng.standard_normal(o.n)
    eF = rel(g.residual(scheme, phi), o.residual(scheme, phi))
    eJ = rel(g.apply_jacobian(scheme, phi, v), o.apply_jacobian(scheme, phi, v))
    log(f"  {name} scheme {scheme}: F {eF:.2e} Jv {eJ:.2e}")
    assert eF < 1e-12 and eJ < 1e-12
    # the lambda_m rows are the identity
    Jv = g.apply_jacobian(scheme, phi, v)
    assert np.array_equal(Jv[o.n_nodes:o.n_nodes + o.n_m], v[o.n_nodes:o.n_nodes + o.n_m])


def test_two_field_tight_solve_matches_oracle(case):
    name, prob, o, g = case
    phi = np.zeros(2 * o.n)
    rg = g.solve(phi_out=phi, **TIGHT)
    ro, pl, pn = oracle_solve(name, o)
    log(f"  {name}: total {rg['total']!r} vs {ro['total']!r} (lc {rg['lc']:.6f} nc {rg['nc']:.6f} "
        f"dG {rg['dg_omega_i']:.6f}), newton {rg['newton_iters']}/{ro['newton_iters']}, "
        f"gmres {rg['gmres_iters_total']}/{ro['gmres_iters_total']}")
    assert rg["status"] == 0 and rg["newton_iters"] == ro["newton_iters"]
    for k in ("total", "lc", "nc", "dg_omega_i"):
        assert abs(rg[k] - ro[k]) <= 1e-10 * abs(ro["total"]), k
    nn, nm = o.n_nodes, o.n_m
    assert np.all(phi[nn:nn + nm] == 0.0) and np.all(phi[o.n + nn:o.n + nn + nm] == 0.0)
    assert rel(phi[:o.n], pl) < 1e-9 and rel(phi[o.n:], pn) < 1e-8
    # the energy entry point recovers lambda_m the same way
    e = g.energy(phi[:o.n], phi[o.n:])
    assert abs(e["total"] - rg["total"]) <= 1e-12 * abs(rg["total"])


def test_two_field_mixed_precision(case, ctx):
    import paper_2511_21713_amd as pb
    name, prob, o, _ = case
    gm = pb.Problem.from_inputs(ctx, prob, precision=pb.MIXED)
    rm = gm.solve(**dict(TIGHT, tol_nl=1e-7, tol_gr=1e-9, tol_gr0=1e-9, tol_omega=1e-7))
    ro, _, _ = oracle_solve(name, o)
    eE = abs(rm["total"] - ro["total"]) / abs(ro["total"])
    log(f"  {name} mixed: energy {eE:.2e}")
    assert rm["status"] == 0 and eE < 1e-5
    gm.close()


def test_two_field_same_in_a_batch_beside_shell_only(ctx):
    import paper_2511_21713_amd as pb
    specs = [CASES["bumpy_n3"], {k: v for k, v in CASES["bumpy_n3"].items() if k != "solute_layers"},
             CASES["sphere_n8"]]
    probs = [pbgen.make_problem(**sp) for sp in specs]
    solo = []
    for prob in probs:
        g = pb.Problem.from_inputs(ctx, prob)
        solo.append(g.solve(**TIGHT))
        g.close()
    gs = [pb.Problem.from_inputs(ctx, prob) for prob in probs]
    code, res = pb.solve_batch(ctx, gs, **TIGHT)
    assert code == 0
    for r, s in zip(res, solo):
        assert r["total"] == s["total"] and r["gmres_iters"] == s["gmres_iters"]
    # the two forms differ by the discretisation only
    assert abs(solo[0]["total"] - solo[1]["total"]) < 0.05 * abs(solo[1]["total"])
    for g in gs:
        g.close()


def test_two_field_errors(ctx):
    import paper_2511_21713_amd as pb
    prob = pbgen.make_problem(**CASES["bumpy_n3"])
    g = pb.Problem.from_inputs(ctx, prob)
    for bad in (-1, len(prob.tets)):
        with pytest.raises(pb.PbfbError):
            g.set_two_field(bad)
    with pytest.raises(pb.PbfbError):
        g.set_bem_mode(pb.BEM_MATRIX_FREE)
    # back to the shell-only form: the same mesh with the solute tets is then
    # not a valid shell (its Gamma_m is inside the FEM domain), so only the
    # switch itself is checked
    g.set_two_field(0)
    g.set_bem_mode(pb.BEM_MATRIX_FREE)
    with pytest.raises(pb.PbfbError):
        g.set_two_field(prob.n_tets_m)
    g.close()


# ---------------------------------------------------------------------------
# Gamma_m given as its own surface mesh, finer than the volume mesh's
# interface and not a face set of it (Sec. 2.3.1: the trace of the volume
# solution on it by interpolation between the two meshes)
# ---------------------------------------------------------------------------
RS_CASES = {
    "bumpy_n3_rs7": dict(CASES["bumpy_n3"], reaction_n=7),
    "sphere_n8_rs12": dict(CASES["sphere_n8"], reaction_n=12),
}
_RS_ORACLE = {}


@pytest.fixture(scope="module", params=sorted(RS_CASES))
def rs_case(request, ctx):
    import paper_2511_21713_amd as pb
    name = request.param
    log(f"[gpu two-field, independent Gamma_m] case {name}")
    prob = pbgen.make_problem(**RS_CASES[name])
    o = oracle.Oracle.from_problem(prob)
    g = pb.Problem.from_inputs(ctx, prob)
    return name, prob, o, g


def rs_oracle_solve(name, o):
    if name not in _RS_ORACLE:
        _RS_ORACLE[name] = o.solve(**TIGHT)
    return _RS_ORACLE[name]


def test_independent_gamma_m_solve_matches_oracle(rs_case, ctx):
    import paper_2511_21713_amd as pb
    name, prob, o, g = rs_case
    phi = np.zeros(2 * o.n)
    rg = g.solve(phi_out=phi, **TIGHT)
    ro, pl, pn = rs_oracle_solve(name, o)
    log(f"  {name}: total {rg['total']!r} vs {ro['total']!r} (lc {rg['lc']:.6f} nc {rg['nc']:.6f}), "
        f"newton {rg['newton_iters']}/{ro['newton_iters']}")
    assert rg["status"] == 0 and rg["newton_iters"] == ro["newton_iters"]
    for k in ("total", "lc", "nc", "dg_omega_i"):
        assert abs(rg[k] - ro[k]) <= 1e-10 * abs(ro["total"]), k
    assert rel(phi[:o.n], pl) < 1e-9 and rel(phi[o.n:], pn) < 1e-8
    e = g.energy(phi[:o.n], phi[o.n:])
    assert abs(e["total"] - rg["total"]) <= 1e-12 * abs(rg["total"])
    # the same volume mesh with the interface faces as Gamma_m: the volume
    # solution is the same, the energy differs by the surface discretisation
    base = {k: v for k, v in RS_CASES[name].items() if k != "reaction_n"}
    g0 = pb.Problem.from_inputs(ctx, pbgen.make_problem(**base))
    e0 = g0.energy(phi[:o.n], phi[o.n:])
    d = abs(e0["total"] - rg["total"]) / abs(rg["total"])
    log(f"  {name}: conforming-Gamma_m energy differs by {d:.2e}")
    assert 1e-8 < d < 0.05
    g0.close()


def test_independent_gamma_m_mixed_precision(rs_case, ctx):
    import paper_2511_21713_amd as pb
    name, prob, o, _ = rs_case
    gm = pb.Problem.from_inputs(ctx, prob, precision=pb.MIXED)
    rm = gm.solve(**dict(TIGHT, tol_nl=1e-7, tol_gr=1e-9, tol_gr0=1e-9, tol_omega=1e-7))
    ro, _, _ = rs_oracle_solve(name, o)
    eE = abs(rm["total"] - ro["total"]) / abs(ro["total"])
    log(f"  {name} mixed: energy {eE:.2e}")
    assert rm["status"] == 0 and eE < 1e-5
    gm.close()


def test_independent_gamma_m_batch_equals_solo(ctx):
    import paper_2511_21713_amd as pb
    probs = [pbgen.make_problem(**RS_CASES["bumpy_n3_rs7"]), pbgen.make_problem(**CASES["bumpy_n3"])]
    solo = []
    for prob in probs:
        g = pb.Problem.from_inputs(ctx, prob)
        solo.append(g.solve(**TIGHT))
        g.close()
    gs = [pb.Problem.from_inputs(ctx, prob) for prob in probs]
    code, res = pb.solve_batch(ctx, gs, **TIGHT)
    assert code == 0
    for r, s in zip(res, solo):
        assert r["total"] == s["total"] and r["gmres_iters"] == s["gmres_iters"]
    for g in gs:
        g.close()


def test_independent_gamma_m_errors(ctx):
    import paper_2511_21713_amd as pb
    prob = pbgen.make_problem(**RS_CASES["bumpy_n3_rs7"])
    v, t = prob.rs_verts, prob.rs_tris
    g = pb.Problem.from_inputs(ctx, prob)
    with pytest.raises(pb.PbfbError):          # vertex id out of range
        g.set_reaction_surface(v, np.where(t == 0, len(v), t))
    with pytest.raises(pb.PbfbError):          # not closed
        g.set_reaction_surface(v, t[1:])
    # oriented inward: refused at setup
    g.set_reaction_surface(v, t[:, ::-1].copy())
    with pytest.raises(pb.PbfbError):
        g.solve(**TIGHT)
    # a surface outside the FEM mesh: refused at setup
    g.set_reaction_surface(v + np.array([0.0, 0.0, 100.0]), t)
    with pytest.raises(pb.PbfbError):
        g.solve(**TIGHT)
    # removed: the conforming two-field form again (bitwise the plain one)
    g.set_reaction_surface(None, None)
    r = g.solve(**TIGHT)
    g2 = pb.Problem.from_inputs(ctx, pbgen.make_problem(**CASES["bumpy_n3"]))
    assert r["total"] == g2.solve(**TIGHT)["total"]
    g.close()
    g2.close()
