"""Parity at the benchmark's full size (RNA-like workload, 20480 triangles per
interface, 133146 unknowns), in the launch configuration bench.py times.

The oracle cannot assemble the full dense operators in test time, so it
computes sampled rows one by one (Galerkin rows of V and K, rows of F(Phi) and
of J(Phi) v) and checks properties of the converged solution that hold at any
size: the oracle's residual at the GPU's Phi* is small, the energy split adds
up, and the mixed-precision solve agrees with FP64 within 1e-5.
"""
import numpy as np
import pytest

import oracle
from conftest import cached_config

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def big():
    import paper_2511_21713_amd as pb
    print("[gpu fullsize] generating the 20k-triangle workload", flush=True)
    prob = cached_config(1)
    ctx = pb.Context(0)
    g = pb.Problem.from_inputs(ctx, prob)
    g.setup()
    o = oracle.Oracle.from_problem(prob)
    return prob, ctx, g, o


def sample_rows(n, k, seed):
    rng = np.random.default_rng(seed)
    r = set(rng.choice(n, size=k, replace=False).tolist()) | {0, n - 1}
    return np.array(sorted(r), dtype=np.int64)


def test_bem_rows_full_size(big):
    prob, ctx, g, o = big
    for surf in (0, 1):
        nv = o.n_m if surf == 0 else o.n_s
        rows = sample_rows(nv, 24, 100 + surf)
        V, K = o.bem_rows(surf, rows)
        Vp, Kp = g.export_bem(surf)
        sV = -1.0 if surf == 0 else 1.0
        errV = np.abs(Vp[rows] - sV * V).max() / np.abs(V).max()
        # K' = 1/2 M +- K: compare K' - 1/2 M through a product with random vectors
        x = np.random.default_rng(3).standard_normal(nv)
        Mx = o.surface_mass_apply(surf, x)[rows]
        sK = 1.0 if surf == 0 else -1.0
        errK = np.abs(Kp[rows] @ x - (0.5 * Mx + sK * (K @ x))).max() / np.abs(K @ x).max()
        print(f"  surface {surf}: V rows {errV:.2e}, K rows (products) {errK:.2e}", flush=True)
        assert errV < 1e-12 and errK < 1e-11


@pytest.mark.parametrize("scheme", [oracle.LIN, oracle.T3, oracle.HS])
def test_operator_rows_full_size(big, scheme):
    prob, ctx, g, o = big
    rng = np.random.default_rng(20 + scheme)
    phi = 0.5 * rng.standard_normal(o.n)
    v = rng.standard_normal(o.n)
    rows = np.concatenate([sample_rows(o.n_nodes, 40, 1), o.n_nodes + sample_rows(o.n_m, 12, 2),
                           o.n_nodes + o.n_m + sample_rows(o.n_s, 12, 3)])
    F = g.residual(scheme, phi)
    Jv = g.apply_jacobian(scheme, phi, v)
    Fr = o.residual_rows(scheme, phi, rows)
    Jr = o.jacobian_rows(scheme, phi, v, rows)
    eF = np.abs(F[rows] - Fr).max() / np.abs(Fr).max()
    eJ = np.abs(Jv[rows] - Jr).max() / np.abs(Jr).max()
    print(f"  scheme {scheme}: F rows {eF:.2e}, Jv rows {eJ:.2e}", flush=True)
    assert eF < 1e-12 and eJ < 1e-12


def test_solve_full_size_properties(big):
    import paper_2511_21713_amd as pb
    prob, ctx, g, o = big
    n = g.n
    phi = np.zeros(2 * n)
    r = g.solve(phi_out=phi, tol_nl=1e-8, tol_gr=1e-9, tol_gr0=1e-9, tol_omega=1e-6, l_e=0.0, max_gmres=20000)
    print(f"  fp64: total {r['total']:.10f}, newton {r['newton_iters']}, gmres {r['gmres_iters_total']}", flush=True)
    assert r["status"] == 0
    assert abs(r["total"] - (r["lc"] + r["nc"] + r["dg_omega_i"])) < 1e-12 * abs(r["total"])
    assert r["nc"] < 0 < r["dg_omega_i"]  # net-negative solute
    star = phi[:n] + phi[n:]
    rows = np.concatenate([sample_rows(o.n_nodes, 40, 7), o.n_nodes + sample_rows(o.n_m, 10, 8),
                           o.n_nodes + o.n_m + sample_rows(o.n_s, 10, 9)])
    Fr = o.residual_rows(oracle.HS, star, rows)
    b = g.export_rhs()
    scale = np.abs(b).max()
    print(f"  oracle residual at Phi*: max {np.abs(Fr).max() / scale:.2e} of max|b|", flush=True)
    assert np.abs(Fr).max() < 1e-7 * scale
    # energy of the GPU's Phi_L, Phi_NL recomputed by the oracle
    e = o.energy(phi[:n], phi[n:])
    assert abs(e["total"] - r["total"]) < 1e-10 * abs(r["total"])
    # mixed precision against FP64: energy and surface potential within 1e-5
    gm = pb.Problem.from_inputs(ctx, prob, precision=pb.MIXED)
    phim = np.zeros(2 * n)
    rm = gm.solve(phi_out=phim, tol_nl=1e-8, tol_gr=1e-9, tol_gr0=1e-9, tol_omega=1e-6, l_e=0.0, max_gmres=20000)
    gs = o.surface_nodes(0)
    um, u64 = (phim[:n] + phim[n:])[gs], star[gs]
    eE = abs(rm["total"] - r["total"]) / abs(r["total"])
    eU = np.linalg.norm(um - u64) / np.linalg.norm(u64)
    print(f"  mixed: total {rm['total']:.10f}, rel energy err {eE:.2e}, surface potential err {eU:.2e}", flush=True)
    assert eE <= 1e-5 and eU <= 1e-5
