"""Parity at the benchmark sizes, in the launch configuration bench.py times:
the RNA-like workload (20480 triangles per interface, 133146 unknowns) and its
large form (81920 triangles per interface, 614430 unknowns; each stored
interface operator then holds 40962 x 81920 entries, beyond 2^31, and the
mixed-precision form is the benchmark's headline).

The oracle cannot assemble the full dense operators in test time, so it
computes sampled rows one by one (Galerkin rows of V and K, rows of F(Phi) and
of J(Phi) v), compared with rows exported from the device, and checks
properties of the converged solution that hold at any size: the oracle's
residual at the GPU's Phi* is small, the energy split adds up, the oracle's
energy of the GPU's Phi_L, Phi_NL is the GPU's, and the mixed-precision solve
(FP32 Krylov basis inside FP64 refinement, as benchmarked) agrees with FP64
within 1e-5.
"""
import numpy as np
import pytest

import oracle
from conftest import cached_config

pytestmark = pytest.mark.gpu

# per workload: sampled BEM rows per surface, FEM / Gamma_m / Gamma_s rows of F and Jv
SAMPLES = {1: dict(bem=24, fem=40, surf=12), 2: dict(bem=12, fem=24, surf=6)}


@pytest.fixture(scope="module", params=[1, 2], ids=["rna20k", "rna80k"])
def big(request):
    import paper_2511_21713_amd as pb
    cfg = request.param
    print(f"[gpu fullsize] generating workload {cfg}", flush=True)
    prob = cached_config(cfg)
    ctx = pb.Context(0)
    g = pb.Problem.from_inputs(ctx, prob)
    print(f"[gpu fullsize] workload {cfg}: setup ({prob.tri_m.shape[0]} triangles per interface)", flush=True)
    g.setup()
    o = oracle.Oracle.from_problem(prob)
    yield cfg, prob, ctx, g, o
    g.close()
    ctx.close()


def sample_rows(n, k, seed):
    rng = np.random.default_rng(seed)
    r = set(rng.choice(n, size=k, replace=False).tolist()) | {0, n - 1}
    return np.array(sorted(r), dtype=np.int64)


def test_bem_rows_full_size(big):
    """Sampled Galerkin rows of both stored operators against the oracle's:
    FP64 storage at 1e-12, and the mixed-precision assembly (FP32 evaluation,
    symmetric completion and storage) at the FP32 bar of the tile tests."""
    import paper_2511_21713_amd as pb
    cfg, prob, ctx, g, o = big
    gm = pb.Problem.from_inputs(ctx, prob, precision=pb.MIXED)
    gm.setup()
    for surf in (0, 1):
        nv = o.n_m if surf == 0 else o.n_s
        rows = sample_rows(nv, SAMPLES[cfg]["bem"], 100 + surf)
        V, K = o.bem_rows(surf, rows)
        sV = -1.0 if surf == 0 else 1.0
        sK = 1.0 if surf == 0 else -1.0
        # K' = 1/2 M +- K: compare K' - 1/2 M through a product with random vectors
        x = np.random.default_rng(3).standard_normal(nv)
        Mx = o.surface_mass_apply(surf, x)[rows]
        for name, gg in (("fp64", g), ("mixed", gm)):
            Vp, Kp = gg.export_bem_rows(surf, rows)
            errV = np.abs(Vp - sV * V).max() / np.abs(V).max()
            dK = np.abs(Kp @ x - (0.5 * Mx + sK * (K @ x))).max()
            if name == "fp64":
                errK, barV, barK = dK / np.abs(K @ x).max(), 1e-12, 1e-11
            else:  # FP32 entries: against the size of the product's terms, not of its (cancelling) sum
                errK, barV, barK = dK / (np.abs(Kp) @ np.abs(x)).max(), 1e-6, 1e-6
            print(f"  workload {cfg}, surface {surf}, {name}: V rows {errV:.2e}, K rows (products) {errK:.2e}",
                  flush=True)
            assert errV < barV and errK < barK
    gm.close()


@pytest.mark.parametrize("scheme", [oracle.LIN, oracle.T3, oracle.HS])
def test_operator_rows_full_size(big, scheme):
    cfg, prob, ctx, g, o = big
    rng = np.random.default_rng(20 + scheme)
    phi = 0.5 * rng.standard_normal(o.n)
    v = rng.standard_normal(o.n)
    k = SAMPLES[cfg]
    rows = np.concatenate([sample_rows(o.n_nodes, k["fem"], 1), o.n_nodes + sample_rows(o.n_m, k["surf"], 2),
                           o.n_nodes + o.n_m + sample_rows(o.n_s, k["surf"], 3)])
    F = g.residual(scheme, phi)
    Jv = g.apply_jacobian(scheme, phi, v)
    Fr = o.residual_rows(scheme, phi, rows)
    Jr = o.jacobian_rows(scheme, phi, v, rows)
    eF = np.abs(F[rows] - Fr).max() / np.abs(Fr).max()
    eJ = np.abs(Jv[rows] - Jr).max() / np.abs(Jr).max()
    print(f"  workload {cfg}, scheme {scheme}: F rows {eF:.2e}, Jv rows {eJ:.2e}", flush=True)
    assert eF < 1e-12 and eJ < 1e-12


def test_solve_full_size_properties(big):
    import paper_2511_21713_amd as pb
    cfg, prob, ctx, g, o = big
    n = g.n
    phi = np.zeros(2 * n)
    kw = dict(tol_nl=1e-8, tol_gr=1e-9, tol_gr0=1e-9, tol_omega=1e-6, l_e=0.0, max_gmres=20000)
    r = g.solve(phi_out=phi, **kw)
    print(f"  workload {cfg} fp64: total {r['total']:.10f}, newton {r['newton_iters']}, "
          f"gmres {r['gmres_iters_total']}", flush=True)
    assert r["status"] == 0
    assert abs(r["total"] - (r["lc"] + r["nc"] + r["dg_omega_i"])) < 1e-12 * abs(r["total"])
    assert r["nc"] < 0 < r["dg_omega_i"]  # net-negative solute
    star = phi[:n] + phi[n:]
    k = SAMPLES[cfg]
    rows = np.concatenate([sample_rows(o.n_nodes, k["fem"], 7), o.n_nodes + sample_rows(o.n_m, k["surf"], 8),
                           o.n_nodes + o.n_m + sample_rows(o.n_s, k["surf"], 9)])
    Fr = o.residual_rows(oracle.HS, star, rows)
    b = g.export_rhs()
    scale = np.abs(b).max()
    print(f"  oracle residual at Phi*: max {np.abs(Fr).max() / scale:.2e} of max|b|", flush=True)
    assert np.abs(Fr).max() < 1e-7 * scale
    # energy of the GPU's Phi_L, Phi_NL recomputed by the oracle
    e = o.energy(phi[:n], phi[n:])
    assert abs(e["total"] - r["total"]) < 1e-10 * abs(r["total"])
    # mixed precision against FP64: energy and surface potential within 1e-5,
    # with the FP64 Krylov basis and with the FP32 basis inside FP64 refinement
    gs = o.surface_nodes(0)
    u64 = star[gs]
    gm = pb.Problem.from_inputs(ctx, prob, precision=pb.MIXED)
    for k32 in (0, 1):
        phim = np.zeros(2 * n)
        rm = gm.solve(phi_out=phim, krylov_fp32=k32, **kw)
        um = (phim[:n] + phim[n:])[gs]
        eE = abs(rm["total"] - r["total"]) / abs(r["total"])
        eU = np.linalg.norm(um - u64) / np.linalg.norm(u64)
        print(f"  mixed (krylov_fp32 {k32}): total {rm['total']:.10f}, rel energy err {eE:.2e}, "
              f"surface potential err {eU:.2e}, gmres {rm['gmres_iters_total']}", flush=True)
        assert rm["status"] == 0 and eE <= 1e-5 and eU <= 1e-5
    gm.close()
