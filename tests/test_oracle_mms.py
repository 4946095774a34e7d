"""Manufactured-solution convergence of the oracle's coupled system.

Smooth fields are chosen in every region: u* in the shell (a quadratic),
phi_m* harmonic inside Gamma_m, phi_s* = C exp(-kappa r)/r (a Yukawa
solution centred inside) outside Gamma_s.  They do not satisfy the
interface conditions or the shell equation, so the differences enter the
right-hand side: the volume source f = -eps_s Lap u* + eps_s kappa^2 sinh(u*)
and the flux jumps in the FEM rows, the Dirichlet jumps through the boundary
rows ((1/2 M + K0) g on Gamma_m, (1/2 M - Kk) g on Gamma_s).  The discrete
solution must then converge to (u*, dn phi_m*, dn phi_s*) as the mesh is
refined: nodal u at second order, the Neumann traces at first order (P1 on a
polyhedral surface, whose normal jumps across edges).  A wrong sign, term or
index anywhere in the coupled operator, the Coulomb-free right-hand side or
the Newton iteration stops the convergence.
"""
import numpy as np

import oracle
import pbgen

KAP, EPS_M, EPS_S = 0.125, 4.0, 80.0
X0 = np.array([0.5, -0.3, 0.2])
C = 6.0


def u_ex(x):
    return 0.6 + 0.08 * x[..., 2] + 0.004 * (x ** 2).sum(-1)


def grad_u(x):
    g = 0.008 * x.copy()
    g[..., 2] += 0.08
    return g


LAP_U = 0.024


def phim(x):
    return 0.9 + 0.05 * x[..., 0] + 0.01 * (x[..., 0] ** 2 - x[..., 1] ** 2)


def grad_phim(x):
    g = np.zeros_like(x)
    g[..., 0] = 0.05 + 0.02 * x[..., 0]
    g[..., 1] = -0.02 * x[..., 1]
    return g


def phis(x):
    r = np.linalg.norm(x - X0, axis=-1)
    return C * np.exp(-KAP * r) / r


def grad_phis(x):
    d = x - X0
    r = np.linalg.norm(d, axis=-1)
    return (C * np.exp(-KAP * r) * (-(1 + KAP * r) / r ** 3))[..., None] * d


def mms_errors(n, L):
    """Max nodal errors of u, lambda_m, lambda_s on the (n, L) sphere shell, and the solve result."""
    prob = pbgen.make_problem(n=n, a=4.0, c=4.0, bump=False, t=4.0, L=L, helix=0, partials=0, kappa=KAP,
                              center_charge=0.0)
    o = oracle.Oracle.from_problem(prob)
    x = prob.nodes
    nn = x.shape[0]
    gm, gs = o.surface_nodes(0), o.surface_nodes(1)
    nm = len(gm)
    e = np.zeros(o.n)
    # volume source f = -eps_s Lap u* + eps_s kappa^2 sinh(u*)
    tb, tw = oracle.rule_tet27()
    T = prob.tets
    P = x[T]  # (n_tets, 4, 3)
    vol = np.abs(np.einsum('ij,ij->i', np.cross(P[:, 1] - P[:, 0], P[:, 2] - P[:, 0]), P[:, 3] - P[:, 0])) / 6
    xq = np.einsum('qk,tkd->tqd', tb, P)
    f = -EPS_S * LAP_U + EPS_S * KAP ** 2 * np.sinh(u_ex(xq))
    contrib = vol[:, None] * np.einsum('q,tq,qk->tk', tw, f, tb)
    np.add.at(e, T.ravel(), contrib.ravel())
    # interface flux jumps (n outward from the inner region on both surfaces):
    # the FEM rows gain + int_Gm g_m v - int_Gs g_s v
    def jump_m(xq, nq):
        return EPS_M * (grad_phim(xq) * nq).sum(-1) - EPS_S * (grad_u(xq) * nq).sum(-1)

    def jump_s(xq, nq):
        return EPS_S * (grad_phis(xq) * nq).sum(-1) - EPS_S * (grad_u(xq) * nq).sum(-1)

    sb, sw = oracle.rule_tri6()
    for tri, sign, gnfun in ((prob.tri_m, +1, jump_m), (prob.tri_s, -1, jump_s)):
        Q = x[tri]
        cr = np.cross(Q[:, 1] - Q[:, 0], Q[:, 2] - Q[:, 0])
        ar = np.linalg.norm(cr, axis=1) / 2
        nq = cr / (2 * ar[:, None])
        xq = np.einsum('qk,tkd->tqd', sb, Q)
        g = gnfun(xq, nq[:, None, :])
        contrib = sign * ar[:, None] * np.einsum('q,tq,qk->tk', sw, g, sb)
        np.add.at(e, tri.ravel(), contrib.ravel())
    # Dirichlet jumps through the boundary rows
    _, Km = o.bem_dense(0)
    _, Ks = o.bem_dense(1)
    gDm = phim(x[gm]) - u_ex(x[gm])
    gDs = phis(x[gs]) - u_ex(x[gs])
    e[nn:nn + nm] = -(0.5 * o.surface_mass_apply(0, gDm) + Km @ gDm)
    e[nn + nm:] = -(0.5 * o.surface_mass_apply(1, gDs) - Ks @ gDs)
    o.set_rhs_extra(e)
    r, pl, pnl = o.solve(tol_nl=1e-11, tol_gr=1e-12, tol_gr0=1e-12, tol_omega=1e-10, l_e=0.0, max_gmres=20000)
    phi = pl + pnl
    eu = np.abs(phi[:nn] - u_ex(x)).max()
    # lambda vs the exact normal derivative at vertices (area-weighted vertex normals)
    def vnormals(tri, g):
        loc = {int(v): i for i, v in enumerate(g)}
        Q = x[tri]
        cr = np.cross(Q[:, 1] - Q[:, 0], Q[:, 2] - Q[:, 0])
        nv = np.zeros((len(g), 3))
        for k in range(3):
            np.add.at(nv, np.vectorize(loc.get)(tri[:, k]), cr)
        return nv / np.linalg.norm(nv, axis=1)[:, None]
    lm_ex = (grad_phim(x[gm]) * vnormals(prob.tri_m, gm)).sum(-1)
    ls_ex = (grad_phis(x[gs]) * vnormals(prob.tri_s, gs)).sum(-1)
    elm = np.abs(phi[nn:nn + nm] - lm_ex).max()
    els = np.abs(phi[nn + nm:] - ls_ex).max()
    return eu, elm, els, r


def test_laplace_yukawa_fields_solve_the_exterior_and_interior_equations():
    # the chosen fields are exact: harmonic inside, Yukawa outside
    x = np.random.default_rng(0).normal(size=(5, 3)) * 3.0 + 9.0
    h = 1e-3
    for f, k2 in ((phim, 0.0), (phis, KAP ** 2)):
        lap = sum((f(x + h * e) - 2 * f(x) + f(x - h * e)) / h ** 2 for e in np.eye(3))
        assert np.abs(-lap + k2 * f(x)).max() < 1e-6 * np.abs(f(x)).max()


def test_manufactured_solution_convergence():
    errs = [mms_errors(n, L) for n, L in ((2, 2), (4, 4), (8, 8))]
    for e in errs:
        assert e[3]["status"] == 0
    eu = [e[0] for e in errs]
    el = [max(e[1], e[2]) for e in errs]
    # second order in u, first order in the Neumann traces
    assert eu[1] / eu[2] > 3.5 and eu[0] / eu[1] > 3.0
    assert el[1] / el[2] > 1.8 and el[0] / el[1] > 1.8
    assert eu[2] < 4e-3 and el[2] < 3e-3
