"""Pins for the oracle's coupled solve, relaxation-factor search and energy.

Closed forms used (all derived in the test, none taken from the oracle):
* Born / Debye-Hueckel: a central charge in a sphere of radius a, linear
  solvent with screening kappa outside: u_r = (l_B z / a)(1/(eps_s (1 + kappa a)) - 1/eps_m).
* Kirkwood (1934): off-centre charges, per-multipole 2x2 matching at r = a.
* The spherically symmetric nonlinear problem reduces to the radial ODE
  u'' + 2u'/r = kappa^2 sinh u on the shell, solved here by scipy.
The solvation energy is 1/2 kT sum_k z_k u_r(x_k) + dG_Omega_i
(eq. Esolv; eq. Esolv_Lineal in the linear case).
"""
import csv
import json
import os

import numpy as np
import pytest
from scipy import integrate, optimize, special

import oracle
import pbgen

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def sphere_problem(n, a=4.0, t=4.0, L=6, z=1.0, kappa=0.125):
    p = pbgen.make_problem(n=n, a=a, c=a, bump=False, t=t, L=L, helix=0, partials=0, kappa=kappa,
                           center_charge=z)
    return p


def born_energy(o, a, z, eps_m, eps_s, kappa):
    ur = o.l_bjerrum * z / a * (1.0 / (eps_s * (1.0 + kappa * a)) - 1.0 / eps_m)
    return 0.5 * o.kT * z * ur, ur


def lin_solve(o, tol=1e-11):
    x, st, it = o.gmres(oracle.LIN, np.zeros(o.n), o.rhs(), tol=tol, maxit=20000)
    assert st == 0
    return x


# ---------------------------------------------------------------------------
# P6: Born / Debye-Hueckel, linear scheme
# ---------------------------------------------------------------------------
def test_born_debye_hueckel_second_order():
    res = {}
    for n in (4, 8):
        p = sphere_problem(n)
        o = oracle.Oracle.from_problem(p)
        x = lin_solve(o)
        res[n] = (o.energy(x)["total"], x[o.n_nodes:o.n_nodes + o.n_m].mean(), x[o.surface_nodes(0)].mean())
    E_ex, ur = born_energy(o, 4.0, 1.0, 4.0, 80.0, 0.125)
    e4, e8 = abs(res[4][0] - E_ex), abs(res[8][0] - E_ex)
    assert e8 / abs(E_ex) < 5e-3
    assert 3.2 < e4 / e8 < 4.8
    rich = (4 * res[8][0] - res[4][0]) / 3
    assert abs(rich - E_ex) / abs(E_ex) < 5e-4
    # surface potential and flux: u|_Gm = l_B z/(eps_m a) + u_r, lambda_m = -l_B z/(eps_m a^2)
    u_ex = o.l_bjerrum / (4.0 * 4.0) + ur
    lam_ex = -o.l_bjerrum / (4.0 * 16.0)
    assert abs(res[8][2] - u_ex) / u_ex < 5e-3
    assert abs(res[8][1] - lam_ex) / abs(lam_ex) < 1e-2


# ---------------------------------------------------------------------------
# P7: Kirkwood, the paper's validation sphere (Sec. 3.1), linear scheme
# ---------------------------------------------------------------------------
def kirkwood_reaction(a, eps_m, eps_s, kappa, lB, qx, qz, lmax=40):
    x = kappa * a
    r = np.linalg.norm(qx, axis=1)
    out = np.zeros(len(qz))
    for l in range(lmax):
        k = special.spherical_kn(l, x)
        dk = special.spherical_kn(l, x, derivative=True)
        # inside: E r^{-l-1} + A r^l; outside: B k_l(kappa r); per unit E
        M = np.array([[a ** l, -k], [eps_m * l * a ** (l - 1) if l else 0.0, -eps_s * kappa * dk]])
        rhs = np.array([-a ** (-l - 1), eps_m * (l + 1) * a ** (-l - 2)])
        A = np.linalg.solve(M, rhs)[0]
        for j in range(len(qz)):
            for kk in range(len(qz)):
                E = lB * qz[kk] * r[kk] ** l / eps_m
                if r[j] == 0 or r[kk] == 0:
                    cg = 1.0
                else:
                    cg = qx[j] @ qx[kk] / (r[j] * r[kk])
                out[j] += E * A * r[j] ** l * special.eval_legendre(l, cg)
    return out


def test_kirkwood_reduces_to_born():
    lB = 560.0
    ur = kirkwood_reaction(3.0, 4.0, 80.0, 0.2, lB, np.zeros((1, 3)), np.array([1.0]))
    assert abs(ur[0] - lB / 3.0 * (1 / (80 * 1.6) - 0.25)) < 1e-12 * lB


def test_kirkwood_paper_sphere():
    g = json.load(open(os.path.join(GOLD, "paper_sphere_case.json")))
    qx = np.array(g["charges_xyz"])
    qz = np.array(g["charges_z"])
    res = []
    for n in (4, 8):
        p = pbgen.make_problem(n=n, a=g["r_m"], c=g["r_m"], bump=False, t=g["r_s"] - g["r_m"], L=6, helix=0,
                               partials=0, kappa=g["kappa"])
        p.q_xyz, p.q_z = qx, qz
        o = oracle.Oracle.from_problem(p)
        res.append(o.energy(lin_solve(o))["total"])
    ur = kirkwood_reaction(g["r_m"], g["eps_m"], g["eps_s"], g["kappa"], o.l_bjerrum, qx, qz)
    E_ex = 0.5 * o.kT * np.sum(qz * ur)
    e = [abs(v - E_ex) / abs(E_ex) for v in res]
    assert e[1] < 5e-3
    assert 3.0 < e[0] / e[1] < 5.0
    assert abs((4 * res[1] - res[0]) / 3 - E_ex) / abs(E_ex) < 1e-3


# ---------------------------------------------------------------------------
# P8: nonlinear radial reference
# ---------------------------------------------------------------------------
def radial_reference(a, b, z, kappa, eps_m, eps_s, lB, kT, nonlinear=True):
    f = np.sinh if nonlinear else (lambda u: u)

    def ode(r, y):
        return np.vstack([y[1], kappa ** 2 * f(y[0]) - 2 * y[1] / r])

    def bc(ya, yb):
        return np.array([ya[1] + lB * z / (eps_s * a * a), yb[1] + (kappa + 1.0 / b) * yb[0]])

    r = np.linspace(a, b, 400)
    y0 = np.vstack([np.ones_like(r), np.zeros_like(r)])
    sol = integrate.solve_bvp(ode, bc, r, y0, tol=1e-10, max_nodes=200000)
    assert sol.success
    ua = sol.sol(a)[0]
    ur = ua - lB * z / (eps_m * a)
    w = lambda s: (lambda u: u * np.sinh(u) - 2 * np.cosh(u) + 2)(sol.sol(s)[0]) * 4 * np.pi * s * s
    integral = integrate.quad(w, a, b, epsabs=1e-14, epsrel=1e-12)[0]
    dg = kT / (4 * np.pi * lB) * 0.5 * eps_s * kappa ** 2 * integral if nonlinear else 0.0
    return 0.5 * kT * z * ur + dg, dg


@pytest.mark.parametrize("z", [1.0, 6.0])
def test_nonlinear_radial_reference(z):
    tot, dg = [], []
    for n in (4, 8):
        p = sphere_problem(n, z=z)
        o = oracle.Oracle.from_problem(p)
        r, _, _ = o.solve(tol_nl=1e-9, tol_gr=1e-11, tol_gr0=1e-11, l_e=0.0, tol_omega=1e-8)
        assert r["status"] == 0
        tot.append(r["total"])
        dg.append(r["dg_omega_i"])
        assert abs(r["total"] - (r["lc"] + r["nc"] + r["dg_omega_i"])) < 1e-12 * abs(r["total"])
    E_ex, dg_ex = radial_reference(4.0, 8.0, z, 0.125, 4.0, 80.0, o.l_bjerrum, o.kT)
    e = [abs(v - E_ex) / abs(E_ex) for v in tot]
    assert e[1] < 5e-3 and 3.0 < e[0] / e[1] < 5.0
    assert abs((4 * tot[1] - tot[0]) / 3 - E_ex) / abs(E_ex) < 5e-4
    ed = [abs(v - dg_ex) / dg_ex for v in dg]
    assert ed[1] < 0.02 and ed[1] < ed[0]
    # the linear variant of the radial ODE reproduces Born / Debye-Hueckel
    E_lin, _ = radial_reference(4.0, 8.0, z, 0.125, 4.0, 80.0, o.l_bjerrum, o.kT, nonlinear=False)
    assert abs(E_lin - born_energy(o, 4.0, z, 4.0, 80.0, 0.125)[0]) < 1e-8 * abs(E_lin)


# ---------------------------------------------------------------------------
# P10: brute-force Newton with dense LU on a tiny mesh
# ---------------------------------------------------------------------------
def dense_jacobian(o, scheme, phi):
    return np.stack([o.apply_jacobian(scheme, phi, e) for e in np.eye(o.n)], 1)


def test_bruteforce_newton_tiny_mesh():
    p = pbgen.make_problem(n=1, a=4.0, c=4.0, bump=False, t=3.0, L=2, helix=0, partials=0, kappa=0.2,
                           center_charge=8.0)
    o = oracle.Oracle.from_problem(p)
    # linear start then full Newton steps with LU
    x = np.linalg.solve(dense_jacobian(o, oracle.LIN, np.zeros(o.n)), o.rhs())
    for _ in range(60):
        F = o.residual(oracle.HS, x)
        if np.linalg.norm(F) < 1e-12 * np.linalg.norm(o.rhs()):
            break
        x -= np.linalg.solve(dense_jacobian(o, oracle.HS, x), F)
    assert np.linalg.norm(o.residual(oracle.HS, x)) < 1e-11 * np.linalg.norm(o.rhs())
    r, pl, pnl = o.solve(tol_nl=1e-12, tol_gr=1e-13, tol_gr0=1e-13, tol_omega=1e-10, l_e=0.0)
    assert r["status"] == 0
    assert np.abs(pl + pnl - x).max() < 1e-9 * np.abs(x).max()
    ref = o.energy(pl, pnl)
    assert abs(ref["total"] - r["total"]) < 1e-12 * abs(r["total"])
    # first step used the cubic start, the rest the full sinh (T3-HS)
    assert r["newton_iters"] >= 3
    assert 1.0 < r["omega"][0] <= 4.0


# ---------------------------------------------------------------------------
# relaxation factor: f_d' by differences, omega_opt vs. a direct minimisation
# ---------------------------------------------------------------------------
@pytest.fixture(scope="module")
def step_case():
    p = sphere_problem(4, z=6.0)
    o = oracle.Oracle.from_problem(p)
    phi = lin_solve(o)
    out = {}
    for s in (oracle.T3, oracle.HS):
        d = -o.residual(s, phi)
        D, st, _ = o.gmres(s, phi, d, tol=1e-12)
        assert st == 0
        out[s] = D
    return o, phi, out


@pytest.mark.parametrize("scheme", [oracle.T3, oracle.HS])
def test_fd_derivative_by_differences(step_case, scheme):
    o, phi, D = step_case
    for w in (0.4, 1.3, 2.2):
        fd, dfd, st = o.fd(scheme, phi, D[scheme], w)
        h = 1e-4
        fp = o.fd(scheme, phi, D[scheme], w + h)[0]
        fm = o.fd(scheme, phi, D[scheme], w - h)[0]
        assert st == 0
        assert abs((fp - fm) / (2 * h) - dfd) < 1e-6 * max(1.0, abs(dfd))


@pytest.mark.parametrize("scheme,w0", [(oracle.T3, 2.0), (oracle.HS, 1.0)])
def test_omega_opt_minimises_residual_norm(step_case, scheme, w0):
    o, phi, D = step_case
    w, it, fb = o.omega_search(scheme, phi, D[scheme], w0, tol_omega=1e-10)
    assert fb == 0 and it < 50

    def dnorm2(om):
        r = o.residual(scheme, phi + om * D[scheme])
        return r @ r

    best = optimize.minimize_scalar(dnorm2, bounds=(0.0, 4.0), method="bounded",
                                    options={"xatol": 1e-9})
    assert abs(best.x - w) < 1e-5
    assert abs(o.fd(scheme, phi, D[scheme], w)[0]) < 1e-9
    # d||d||^2/dw = 2 g_d, which vanishes where f_d does
    h = 1e-5
    assert abs(dnorm2(w + h) - dnorm2(w - h)) / (2 * h) < 1e-6 * dnorm2(w)


# ---------------------------------------------------------------------------
# P11-P13: invariants
# ---------------------------------------------------------------------------
def test_paper_energy_split_rows():
    rows = [r for r in csv.reader(open(os.path.join(GOLD, "paper_energy_split.csv"))) if r and r[0][0] != "#"]
    assert len(rows) == 8
    for _, _, tot, lc, nc, dg in rows:
        tot, lc, nc, dg = map(float, (tot, lc, nc, dg))
        assert abs(lc + nc + dg - tot) <= 1.5e-3  # three printed decimals
        assert nc < 0 < dg  # net-negative solute (-17 e)


def test_total_independent_of_path():
    p = sphere_problem(4, z=-6.0)
    o = oracle.Oracle.from_problem(p)
    common = dict(tol_nl=1e-9, tol_gr=1e-11, tol_omega=1e-6, max_newton=200)
    runs = [o.solve(**common, tol_gr0=1e-11, l_e=0.0)[0],
            o.solve(**common, tol_gr0=1e-3)[0],
            o.solve(**common, tol_gr0=1e-11, omega_auto=0, omega_fixed=1.0)[0],
            o.solve(**common, tol_gr0=1e-11, omega_auto=0, omega_fixed=0.5, scheme_first=oracle.HS)[0]]
    tot = [r["total"] for r in runs]
    assert all(r["status"] == 0 for r in runs)
    assert max(tot) - min(tot) < 1e-7 * abs(tot[0])
    # the adaptive GMRES tolerance moves LC and NC but not the total
    assert abs(runs[1]["lc"] - runs[0]["lc"]) > 1e-9 * abs(tot[0])
    # a net-negative solute: NC < 0 and dG_Omega_i > 0
    assert runs[0]["nc"] < 0 < runs[0]["dg_omega_i"]
    # self-adjusted omega needs fewer iterations than omega = 0.5
    assert runs[0]["newton_iters"] < runs[3]["newton_iters"]


def test_small_charge_scaling():
    vals = []
    for s in (0.05, 0.1):
        o = oracle.Oracle.from_problem(sphere_problem(4, z=s))
        r, _, _ = o.solve(tol_nl=1e-11, tol_gr=1e-13, tol_gr0=1e-13, l_e=0.0, tol_omega=1e-10)
        assert r["status"] == 0
        vals.append(r)
    assert abs(vals[1]["lc"] / vals[0]["lc"] - 4.0) < 1e-8
    # NC / LC = O(s^2) and dG = O(s^4): doubling s multiplies both by 16
    assert abs(vals[1]["nc"] / vals[0]["nc"] - 16.0) < 0.05
    assert abs(vals[1]["dg_omega_i"] / vals[0]["dg_omega_i"] - 16.0) < 0.05


def test_rigid_rotation_invariance():
    p = sphere_problem(4, z=3.0)
    p.q_xyz = np.array([[0.5, -0.3, 0.8]])
    o1 = oracle.Oracle.from_problem(p)
    Q, _ = np.linalg.qr(np.random.default_rng(5).standard_normal((3, 3)))
    if np.linalg.det(Q) < 0:
        Q[:, 0] = -Q[:, 0]
    o2 = oracle.Oracle(p.nodes @ Q.T, p.tets, p.tri_m, p.tri_s, p.q_xyz @ Q.T, p.q_z, 4.0, 80.0, 0.125)
    kw = dict(tol_nl=1e-10, tol_gr=1e-12, tol_gr0=1e-12, l_e=0.0, tol_omega=1e-8)
    r1, r2 = o1.solve(**kw)[0], o2.solve(**kw)[0]
    assert abs(r1["total"] - r2["total"]) < 1e-9 * abs(r1["total"])
