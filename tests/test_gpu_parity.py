"""GPU parity: the HIP library (through its C ABI) against the CPU oracle.

FP64 bar: 1e-12 relative on assembled operators, residuals and Jacobian
products (tighter than the 1e-10 the method's parity target asks for), and
1e-10 relative on energies and surface potentials of full solves.
"""
import os
import sys

import numpy as np
import pytest

import oracle
import pbgen
from conftest import cached_config

pytestmark = pytest.mark.gpu


def log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ctx():
    import paper_2511_21713_amd as pb
    return pb.Context(0)


def gpu_problem(ctx, prob, precision=0):
    import paper_2511_21713_amd as pb
    return pb.Problem.from_inputs(ctx, prob, precision=precision)


def rel(a, b):
    return np.abs(np.asarray(a) - np.asarray(b)).max() / max(np.abs(np.asarray(b)).max(), 1e-300)


CASES = {
    "sphere_n4": dict(n=4, a=4.0, c=4.0, bump=False, t=4.0, L=6, helix=0, partials=0, kappa=0.125,
                      center_charge=1.0),
    # ragged block tails: 20 n^2 triangles not a multiple of 16 or 32
    "bumpy_n3": dict(n=3, a=6.0, c=9.0, bump=True, t=3.0, L=3, helix=3, partials=5, kappa=0.2, seed=(9, 1)),
    "icosahedron": dict(n=1, a=4.0, c=4.0, bump=False, t=3.0, L=2, helix=0, partials=0, kappa=0.3,
                        center_charge=-2.0),
}


@pytest.fixture(scope="module", params=sorted(CASES))
def case(request, ctx):
    name = request.param
    log(f"[gpu parity] case {name}")
    prob = pbgen.make_problem(**CASES[name])
    o = oracle.Oracle.from_problem(prob)
    g = gpu_problem(ctx, prob)
    return name, prob, o, g


def test_bem_blocks_match_oracle(case):
    name, prob, o, g = case
    for surf in (0, 1):
        V, K = o.bem_dense(surf)
        nv = V.shape[0]
        M = np.stack([o.surface_mass_apply(surf, e) for e in np.eye(nv)], 1)
        Kp_ref = 0.5 * M + (K if surf == 0 else -K)
        Vp_ref = -V if surf == 0 else V
        Vp, Kp = g.export_bem(surf)
        for A, B in ((Vp, Vp_ref), (Kp, Kp_ref)):
            rowmax = np.abs(B).max(1, keepdims=True)
            err = (np.abs(A - B) / rowmax).max()
            log(f"  {name} surf {surf} entrywise rel err {err:.2e}")
            assert err < 1e-12


def test_rhs_matches_oracle(case):
    name, prob, o, g = case
    b = g.export_rhs()
    assert rel(b, o.rhs()) < 1e-12


@pytest.mark.parametrize("scheme", [oracle.LIN, oracle.T3, oracle.T5, oracle.T7, oracle.HS])
def test_residual_and_jacobian_match_oracle(case, scheme):
    name, prob, o, g = case
    rng = np.random.default_rng(11 + scheme)
    phi = rng.standard_normal(o.n)
    v = rng.standard_normal(o.n)
    F = g.residual(scheme, phi)
    Jv = g.apply_jacobian(scheme, phi, v)
    eF, eJ = rel(F, o.residual(scheme, phi)), rel(Jv, o.apply_jacobian(scheme, phi, v))
    log(f"  {name} scheme {scheme}: F {eF:.2e} Jv {eJ:.2e}")
    assert eF < 1e-12 and eJ < 1e-12


def test_device_tensors_path(case):
    torch = pytest.importorskip("torch")
    name, prob, o, g = case
    rng = np.random.default_rng(3)
    phi = rng.standard_normal(o.n)
    v = rng.standard_normal(o.n)
    tphi = torch.tensor(phi, device="cuda:0")
    tv = torch.tensor(v, device="cuda:0")
    out = g.apply_jacobian(oracle.HS, tphi, tv, stream=torch.cuda.current_stream())
    torch.cuda.synchronize()
    assert rel(out.cpu().numpy(), o.apply_jacobian(oracle.HS, phi, v)) < 1e-12


@pytest.mark.parametrize("pc", [0, 1])
def test_tight_solve_matches_oracle(case, pc):
    # pc 0: inverse diagonal; 1: Chebyshev terms on the FEM block + approximate inverse of the single layers
    name, prob, o, g = case
    kw = dict(tol_nl=1e-10, tol_gr=1e-12, tol_gr0=1e-12, tol_omega=1e-9, l_e=0.0, max_gmres=20000, precond=pc)
    rg = g.solve(**kw)
    ro, pl, pnl = o.solve(**kw)
    log(f"  {name} pc {pc}: gpu {rg['total']:.12f} ({rg['newton_iters']} it, gmres {rg['gmres_iters_total']}) "
        f"oracle {ro['total']:.12f} ({ro['newton_iters']} it, gmres {ro['gmres_iters_total']})")
    assert rg["status"] == 0 and ro["status"] == 0
    assert abs(rg["total"] - ro["total"]) < 1e-10 * abs(ro["total"])
    phi = np.zeros(2 * o.n)
    g.solve(phi_out=phi, **kw)
    gs = o.surface_nodes(0)
    u_gpu = (phi[:o.n] + phi[o.n:])[gs]
    u_ora = (pl + pnl)[gs]
    assert np.linalg.norm(u_gpu - u_ora) < 1e-10 * np.linalg.norm(u_ora)


@pytest.mark.parametrize("pc", [0, 1])
def test_paper_tolerance_solve_iterates_like_oracle(case, pc):
    # Tol_NL = 1e-3, Tol_GR = 1e-6, adaptive Tol_GR0 = 1e-3, Tol_omega = 0.1, L_e = 0.35 (App. B settings)
    name, prob, o, g = case
    rg = g.solve(precond=pc)
    ro, _, _ = o.solve(precond=pc)
    log(f"  {name}: gpu it {rg['newton_iters']} omega {rg['omega']} gmres {rg['gmres_iters']}; "
        f"oracle it {ro['newton_iters']} omega {ro['omega']} gmres {ro['gmres_iters']}")
    assert rg["newton_iters"] == ro["newton_iters"]
    assert np.allclose(rg["omega"], ro["omega"], atol=1e-6)
    assert abs(rg["total"] - ro["total"]) < 1e-6 * abs(ro["total"])


@pytest.mark.parametrize("method", [1, 2, 3, 4])
def test_omega_root_finders_iterate_like_oracle(case, method):
    """Bisection, secant, bisection-then-secant and the bisection/secant start
    of the first Newton search for the relaxation factor, at the App. B
    settings: the same Newton steps, the same number of f_d evaluations per
    step and the same factors as the oracle."""
    name, prob, o, g = case
    rg = g.solve(omega_method=method)
    ro, _, _ = o.solve(omega_method=method)
    log(f"  {name} method {method}: gpu it {rg['newton_iters']} omega {rg['omega']} evals {rg['omega_iters']}; "
        f"oracle omega {ro['omega']} evals {ro['omega_iters']}")
    assert rg["status"] == 0 and ro["status"] == 0
    assert rg["newton_iters"] == ro["newton_iters"]
    assert rg["omega_iters"] == ro["omega_iters"]
    assert np.allclose(rg["omega"], ro["omega"], atol=1e-6)
    assert abs(rg["total"] - ro["total"]) < 1e-6 * abs(ro["total"])


def test_picard_iterates_like_oracle(case):
    """Picard iteration (A Delta = d) with the direct-secant relaxation search
    and the norm-ratio reuse rule, omega in [0, 1]: the same steps and factors
    as the oracle at the App. B tolerances, and the same energy as Newton at
    tight ones."""
    name, prob, o, g = case
    kw = dict(nonlinear_method=1, omega_method=5, omega_max=1.0, l_e=0.0, max_newton=200)
    rg = g.solve(**kw)
    ro, _, _ = o.solve(**kw)
    log(f"  {name} picard: gpu it {rg['newton_iters']} omega {np.round(rg['omega'], 4)}; oracle it {ro['newton_iters']}")
    assert rg["status"] == 0 and ro["status"] == 0
    assert rg["newton_iters"] == ro["newton_iters"] and rg["omega_iters"] == ro["omega_iters"]
    assert np.allclose(rg["omega"], ro["omega"], atol=1e-6)
    tight = dict(kw, omega_method=1, tol_nl=1e-9, tol_gr=1e-12, tol_gr0=1e-12, tol_omega=1e-9, max_omega_it=200,
                 max_gmres=20000)
    rg = g.solve(**tight)
    ro, _, _ = o.solve(**tight)
    assert rg["status"] == 0
    assert abs(rg["total"] - ro["total"]) < 1e-10 * abs(ro["total"])


@pytest.mark.parametrize("sched", [(1, 3), (1, 3, 4, 4)])
def test_scheme_schedule_iterates_like_oracle(case, sched):
    """T3-T5-HS and T3-T5-T7-T7-HS (Sec. 3.3.1) at the App. B settings: the
    same steps and relaxation factors as the oracle, and at tight tolerances
    the same energy as T3-HS."""
    name, prob, o, g = case
    rg = g.solve(schedule=sched)
    ro, _, _ = o.solve(schedule=sched)
    log(f"  {name} schedule {sched}: gpu it {rg['newton_iters']} omega {np.round(rg['omega'], 4)}; "
        f"oracle it {ro['newton_iters']}")
    assert rg["status"] == 0 and ro["status"] == 0
    assert rg["newton_iters"] == ro["newton_iters"] and rg["omega_iters"] == ro["omega_iters"]
    assert np.allclose(rg["omega"], ro["omega"], atol=1e-6)
    tight = dict(tol_nl=1e-10, tol_gr=1e-12, tol_gr0=1e-12, tol_omega=1e-9, l_e=0.0, max_gmres=20000)
    rg = g.solve(schedule=sched, **tight)
    ro, _, _ = o.solve(**tight)
    assert rg["status"] == 0
    assert abs(rg["total"] - ro["total"]) < 1e-10 * abs(ro["total"])


def test_mixed_precision_matches_oracle(case, ctx):
    """Mixed precision: regular panel pairs evaluated in FP32 (FP64 pair
    blocks and gathers), operators stored in FP32, FP32 Krylov basis inside
    FP64 restarts.  Bars: stored blocks within 1e-6 of the row maximum (FP32
    rounding of kernel values and of the stored entry), energy and surface
    potential of a tight solve within 1e-5 of the FP64 oracle."""
    import paper_2511_21713_amd as pb
    name, prob, o, g64 = case
    gm = gpu_problem(ctx, prob, precision=pb.MIXED)
    for surf in (0, 1):
        V, K = o.bem_dense(surf)
        nv = V.shape[0]
        M = np.stack([o.surface_mass_apply(surf, e) for e in np.eye(nv)], 1)
        Kp_ref = 0.5 * M + (K if surf == 0 else -K)
        Vp_ref = -V if surf == 0 else V
        Vp, Kp = gm.export_bem(surf)
        for A, B in ((Vp, Vp_ref), (Kp, Kp_ref)):
            err = (np.abs(A - B) / np.abs(B).max(1, keepdims=True)).max()
            log(f"  {name} mixed surf {surf} entrywise rel err {err:.2e}")
            assert err < 1e-6
    kw = dict(tol_nl=1e-10, tol_gr=1e-12, tol_gr0=1e-12, tol_omega=1e-9, l_e=0.0, max_gmres=20000)
    ro, pl, pnl = o.solve(**kw)
    gs = o.surface_nodes(0)
    u_ora = (pl + pnl)[gs]
    for basis32 in (0, 1):
        phi = np.zeros(2 * o.n)
        rm = gm.solve(phi_out=phi, krylov_fp32=basis32, **kw)
        u_mix = (phi[:o.n] + phi[o.n:])[gs]
        eE = abs(rm["total"] - ro["total"]) / abs(ro["total"])
        eU = np.linalg.norm(u_mix - u_ora) / np.linalg.norm(u_ora)
        log(f"  {name} mixed (FP32 basis {basis32}): total {rm['total']:.10f} vs {ro['total']:.10f}: "
            f"energy {eE:.2e}, potential {eU:.2e}, gmres {rm['gmres_iters_total']}")
        assert rm["status"] == 0
        assert eE < 1e-5 and eU < 1e-5
    gm.close()


def test_timed_solves_repeat(ctx):
    """Event timing on across several solves: the timer's event pool fills
    and is folded while timed ranges are open; every solve must still end
    normally with the same result."""
    prob = pbgen.make_problem(**CASES["sphere_n4"])
    g = gpu_problem(ctx, prob)
    kw = dict(tol_nl=1e-10, tol_gr=1e-12, tol_gr0=1e-12, tol_omega=1e-9, l_e=0.0, max_gmres=20000, precond=0)
    g.timing_enable(True)
    g.timing(0, reset=True)
    totals = []
    for k in range(6):
        g.reset_operators()
        r = g.solve(**kw)
        assert r["status"] == 0
        totals.append(r["total"])
    ms, cnt = g.timing(0)
    log(f"  timed solves: {len(totals)} solves, {cnt} timed applies, {ms:.4f} ms each")
    # four timed ranges per Krylov step (preconditioner, apply, GEMV, SpMV): the 4096-pair pool fills
    assert 4 * cnt > 2 * 4096 and ms > 0
    assert all(t == totals[0] for t in totals)
    g.close()


def test_fixed_relaxation_sphere_config():
    # the charged-sphere workload: plain FP64 Newton with omega = 0.5
    import paper_2511_21713_amd as pb
    prob = cached_config(0)
    o = oracle.Oracle.from_problem(prob)
    g = pb.Problem.from_inputs(pb.Context(0), prob)
    kw = dict(omega_auto=0, omega_fixed=0.5, tol_nl=1e-8, tol_gr=1e-12, tol_gr0=1e-12)
    rg, (ro, _, _) = g.solve(**kw), o.solve(**kw)
    assert rg["newton_iters"] == ro["newton_iters"]
    assert abs(rg["total"] - ro["total"]) < 1e-10 * abs(ro["total"])


def test_energy_entry_point(case):
    name, prob, o, g = case
    rng = np.random.default_rng(5)
    pl, pn = rng.standard_normal(o.n), 0.3 * rng.standard_normal(o.n)
    eg, eo = g.energy(pl, pn), o.energy(pl, pn)
    for k in ("lc", "nc", "dg_omega_i"):
        assert abs(eg[k] - eo[k]) < 1e-11 * max(abs(eo[k]), 1e-300), (k, eg[k], eo[k])


def test_deterministic(case):
    name, prob, o, g = case
    rng = np.random.default_rng(8)
    phi = rng.standard_normal(o.n)
    v = rng.standard_normal(o.n)
    a = g.apply_jacobian(oracle.HS, phi, v)
    b = g.apply_jacobian(oracle.HS, phi, v)
    assert np.array_equal(a, b)


# ---------------------------------------------------------------------------
# error paths
# ---------------------------------------------------------------------------
def test_error_codes(ctx):
    import paper_2511_21713_amd as pb
    prob = cached_config(0)
    g = pb.Problem(ctx)
    with pytest.raises(pb.PbfbError) as e:
        g.setup()
    assert e.value.code in (pb.ESTATE, pb.EINVAL)
    g.set_mesh(prob.nodes, prob.tets, prob.tri_m, prob.tri_s)
    with pytest.raises(pb.PbfbError) as e:
        g.set_params(-1.0, 80.0, 0.125)
    assert e.value.code == pb.EINVAL
    g.set_params(4.0, 80.0, 0.125)
    g.set_charges(np.array([[0.0, 0.0, 3.6]]), np.array([1.0]))  # 0.4 A from Gamma_m
    with pytest.raises(pb.PbfbError) as e:
        g.solve()
    assert e.value.code == pb.ECHARGE
    g.set_charges(np.array([[0.0, 0.0, 20.0]]), np.array([1.0]))  # outside
    with pytest.raises(pb.PbfbError) as e:
        g.solve()
    assert e.value.code == pb.ECHARGE
    for bad_opts in (dict(schedule=[0]), dict(schedule=[1, 7]), dict(n_schedule=9), dict(scheme_first=0)):
        with pytest.raises(pb.PbfbError) as e:
            g.solve(**bad_opts)
        assert e.value.code == pb.EINVAL
    bad = prob.tri_m[1:]  # open surface
    g2 = pb.Problem(ctx)
    with pytest.raises(pb.PbfbError) as e:
        g2.set_mesh(prob.nodes, prob.tets, bad, prob.tri_s)
    assert e.value.code == pb.EMESH
    flat = prob.tets.copy()
    flat[0, 3] = flat[0, 2]
    g3 = pb.Problem.from_inputs(ctx, prob)
    g3.set_mesh(prob.nodes, flat, prob.tri_m, prob.tri_s)
    with pytest.raises(pb.PbfbError) as e:
        g3.setup()
    assert e.value.code == pb.EMESH


def test_inward_oriented_surfaces_are_refused(ctx):
    """A surface oriented consistently but towards the solute (every
    triangle flipped) is closed and manifold, yet flips the sign of its double
    layer: setup refuses it with PBFB_EMESH from the negative enclosed volume,
    for Gamma_m and for Gamma_s, with and without charges."""
    import paper_2511_21713_amd as pb
    prob = cached_config(0)
    for which in ("m", "s"):
        for charged in (True, False):
            tm = prob.tri_m[:, [0, 2, 1]].copy() if which == "m" else prob.tri_m
            ts = prob.tri_s[:, [0, 2, 1]].copy() if which == "s" else prob.tri_s
            g = pb.Problem(ctx)
            g.set_mesh(prob.nodes, prob.tets, tm, ts)
            g.set_params(prob.eps_in, prob.eps_out, prob.kappa)
            if charged:
                g.set_charges(prob.q_xyz, prob.q_z)
            else:
                g.set_charges(np.zeros((0, 3)), np.zeros(0))
            with pytest.raises(pb.PbfbError) as e:
                g.setup()
            log(f"  flipped Gamma_{which}, charges {charged}: {pb.last_error()}")
            assert e.value.code == pb.EMESH
            g.close()
    g = pb.Problem.from_inputs(ctx, prob)  # the outward-oriented mesh is accepted
    g.setup()
    g.close()


def test_problem_outliving_its_context():
    """A context destroyed before its problems detaches them: calls on them
    fail with PBFB_ESTATE, destroying them still works, and a new context is
    unaffected (finalizers of garbage cycles may run in any order)."""
    import paper_2511_21713_amd as pb
    prob = cached_config(0)
    c2 = pb.Context(0)
    g = pb.Problem.from_inputs(c2, prob)
    g.setup()
    c2.close()
    with pytest.raises(pb.PbfbError) as e:
        g.residual(oracle.HS, np.zeros(g.n))
    assert e.value.code == pb.ESTATE
    g.close()
    c3 = pb.Context(0)
    g3 = pb.Problem.from_inputs(c3, prob)
    g3.setup()
    g3.close()
    c3.close()


def test_parameter_changes_recompute_what_depends_on_them(ctx):
    """After a setup, new permittivities recompute the FEM values and the
    load (not the boundary operators, which do not depend on them) and a new
    kappa the Yukawa operators: the products then match an oracle built with
    the new values, and the Laplace operators are left as they were."""
    import dataclasses

    import paper_2511_21713_amd as pb
    prob = cached_config(0)
    g = pb.Problem.from_inputs(ctx, prob)
    g.setup()
    Vm0, Km0 = g.export_bem(0)
    rng = np.random.default_rng(41)
    phi = 0.5 * rng.standard_normal(g.n)
    v = rng.standard_normal(g.n)
    for eps_in, eps_out, kappa in ((2.0, 80.0, prob.kappa), (2.0, 60.0, prob.kappa), (2.0, 60.0, 0.3)):
        g.set_params(eps_in, eps_out, kappa)
        q = dataclasses.replace(prob, eps_in=eps_in, eps_out=eps_out, kappa=kappa)
        o = oracle.Oracle.from_problem(q)
        eF = rel(g.residual(oracle.HS, phi), o.residual(oracle.HS, phi))
        eJ = rel(g.apply_jacobian(oracle.HS, phi, v), o.apply_jacobian(oracle.HS, phi, v))
        log(f"  eps {eps_in}/{eps_out} kappa {kappa}: F {eF:.2e} Jv {eJ:.2e}")
        assert eF < 1e-12 and eJ < 1e-12
        Vm, Km = g.export_bem(0)
        assert np.array_equal(Vm, Vm0) and np.array_equal(Km, Km0)
    g.close()


def test_iteration_limit_returns_the_last_iterate(case):
    """Stopped by max_newton: PBFB_ENOTCONV, with the result and phi_out
    holding the last iterate, which equals the oracle's after the same
    steps."""
    import paper_2511_21713_amd as pb
    name, prob, o, g = case
    kw = dict(max_newton=2, tol_nl=1e-14, tol_gr=1e-12, tol_gr0=1e-12, tol_omega=1e-9, l_e=0.0, max_gmres=20000)
    phi = np.zeros(2 * o.n)
    rg = g.solve(phi_out=phi, check=False, **kw)
    ro, pl, pnl = o.solve(**kw)
    log(f"  {name}: status {rg['status']} (oracle {ro['status']}), newton {rg['newton_iters']}, "
        f"total {rg['total']:.10f} vs {ro['total']:.10f}")
    assert rg["status"] == pb.ENOTCONV and ro["status"] == pb.ENOTCONV
    assert rg["newton_iters"] == 2 and len(rg["omega"]) == 2
    assert abs(rg["total"] - ro["total"]) < 1e-10 * abs(ro["total"])
    assert np.linalg.norm(phi[o.n:] - pnl) < 1e-9 * np.linalg.norm(pnl)
    with pytest.raises(pb.PbfbError) as e:
        g.solve(**kw)
    assert e.value.code == pb.ENOTCONV


def test_degenerate_inputs(ctx):
    """Edge cases of the method: no charges (b = 0: the solve returns at
    once with Phi = 0 and zero energy), kappa = 0 (no ions: the shell
    equation is linear, Gamma_s carries the Laplace kernel, and the
    nonlinear part vanishes), and an empty batch."""
    import dataclasses

    import paper_2511_21713_amd as pb
    prob = cached_config(0)
    # no charges
    g = pb.Problem.from_inputs(ctx, prob)
    g.set_charges(np.zeros((0, 3)), np.zeros(0))
    phi = np.ones(2 * g.n)
    r = g.solve(phi_out=phi)
    log(f"  no charges: status {r['status']}, total {r['total']!r}, newton {r['newton_iters']}")
    assert r["status"] == 0 and r["total"] == 0.0 and not np.any(phi)
    g.close()
    # kappa = 0
    q = dataclasses.replace(prob, kappa=0.0)
    o = oracle.Oracle.from_problem(q)
    g = pb.Problem.from_inputs(ctx, q)
    kw = dict(tol_nl=1e-10, tol_gr=1e-12, tol_gr0=1e-12, tol_omega=1e-9, l_e=0.0, max_gmres=20000)
    rg = g.solve(**kw)
    ro, _, _ = o.solve(**kw)
    log(f"  kappa 0: total {rg['total']!r} vs {ro['total']!r}, nc {rg['nc']:.3e}")
    assert rg["status"] == 0 and abs(rg["total"] - ro["total"]) < 1e-10 * abs(ro["total"])
    assert rg["nc"] == 0.0 or abs(rg["nc"]) < 1e-12 * abs(rg["total"])
    rng = np.random.default_rng(4)
    x = rng.standard_normal(o.n)
    assert rel(g.residual(oracle.HS, x), o.residual(oracle.HS, x)) < 1e-12
    g.close()
    # an empty batch
    code, res = pb.solve_batch(ctx, [])
    assert code == 0 and res == []

