"""Pins for the oracle's Galerkin boundary operators.

V_ij = int int zeta_i(x) g(x,y) zeta_j(y),  K_ij = int int zeta_i(x) dg/dn_y zeta_j(y)
with g = exp(-kappa r)/(4 pi r) (Sec. 2.2, Yukawa kernel; kappa = 0 gives the
Laplace kernel of Sec. 2.3).  Touching triangle pairs use Sauter-Schwab rules.
"""
import numpy as np
import pytest
from scipy import special

import oracle
import pbgen
from conftest import cached_config


# ---------------------------------------------------------------------------
# Gauss identity: K0 applied to a constant density is -1/2 on a closed surface
# ---------------------------------------------------------------------------
def gauss_error(o):
    V, K = o.bem_dense(0)
    M1 = o.surface_mass_apply(0, np.ones(o.n_m))
    return np.abs(K.sum(1) + 0.5 * M1).max() / M1.max()


def test_gauss_identity_production_rules():
    p = cached_config(0)
    o = oracle.Oracle.from_problem(p)
    assert gauss_error(o) < 1e-5


def test_gauss_identity_converges_with_quadrature_order():
    # on the faceted surface the identity is exact, so the error must fall to
    # rounding level as the regular and singular orders rise; a sign or a
    # missing singular correction would leave an O(1) error.
    p = pbgen.make_problem(n=2, a=4.0, c=4.0, bump=False, t=4.0, L=1, helix=0, partials=0, kappa=0.125,
                           center_charge=1.0)
    errs = [gauss_error(oracle.Oracle.from_problem(p, reg_order=ro, n_ss=ns))
            for ro, ns in ((0, 4), (6, 6), (12, 10))]
    assert errs[0] < 1e-4
    assert errs[1] < errs[0] / 10
    assert errs[2] < 1e-10


def test_single_layer_symmetric():
    p = cached_config(0)
    o = oracle.Oracle.from_problem(p, n_ss=8)
    for s in (0, 1):
        V, _ = o.bem_dense(s)
        assert np.abs(V - V.T).max() < 1e-10 * np.abs(V).max()


# ---------------------------------------------------------------------------
# Sauter-Schwab panels vs. an independent semi-analytic integration
# ---------------------------------------------------------------------------
def _bary(Y, P):
    T = np.stack([P[1] - P[0], P[2] - P[0]], 1)
    c = np.linalg.lstsq(T, (Y - P[0]).T, rcond=None)[0]
    return np.stack([1 - c[0] - c[1], c[0], c[1]], 1)


def _inner_semi_analytic(X, P, b):
    """int_sig phi_b(y) / (4 pi |x - y|) dy for points X in the plane of sig.

    The triangle is split into the signed fan of triangles (x, Q1, Q2) over
    its edges; in Duffy coordinates from the apex the 1/r cancels and, phi_b
    being linear, the radial integral is exact, leaving
    int_0^1 (alpha + beta t) / |e1 + t e2| dt, integrated in closed form."""
    nrm = np.cross(P[1] - P[0], P[2] - P[0])
    nh = nrm / np.linalg.norm(nrm)
    fx = _bary(X, P)[:, b]
    fv = _bary(P, P)[:, b]
    tot = np.zeros(X.shape[0])
    for k in range(3):
        Q1, Q2 = P[k], P[(k + 1) % 3]
        e1 = Q1[None, :] - X
        e2 = Q2 - Q1
        cr = np.cross(e1, e2[None, :])
        J = np.linalg.norm(cr, axis=1)
        sg = np.sign(cr @ nh)
        a = e2 @ e2
        bb = 2 * e1 @ e2
        c = np.einsum("ij,ij->i", e1, e1)

        def F(t):
            return np.log(2 * np.sqrt(a * (a * t * t + bb * t + c)) + 2 * a * t + bb) / np.sqrt(a)

        def R(t):
            return np.sqrt(a * t * t + bb * t + c)

        I0 = F(1.0) - F(0.0)
        I1 = (R(1.0) - R(0.0)) / a - bb / (2 * a) * I0
        f1, f2 = fv[k], fv[(k + 1) % 3]
        tot += np.where(J > 1e-15, sg * J * 0.5 * ((fx + f1) * I0 + (f2 - f1) * I1), 0.0)
    return tot / (4 * np.pi)


def _outer(Pa, Pb, a, b, m):
    s, ws = np.polynomial.legendre.leggauss(m)
    s, ws = (s + 1) / 2, ws / 2
    S, T = np.meshgrid(s, s, indexing="ij")
    W = np.outer(ws, ws) * S
    c = Pa.mean(0)
    tot = 0.0
    for k in range(3):
        Q1, Q2 = Pa[k], Pa[(k + 1) % 3]
        J = np.linalg.norm(np.cross(Q1 - c, Q2 - Q1))
        X = c + S.reshape(-1, 1) * ((Q1 - c)[None, :] + T.reshape(-1, 1) * (Q2 - Q1)[None, :])
        tot += np.sum(W.ravel() * J * _bary(X, Pa)[:, a] * _inner_semi_analytic(X, Pb, b))
    return tot


def test_sauter_schwab_matches_semi_analytic_coplanar_panels():
    nodes = np.array([[0, 0, 0], [1, 0, 0], [0.3, 0.9, 0], [1.2, 0.8, 0], [-0.8, -0.5, 0], [0, -1.0, 0],
                      [0.5, 0.5, -1]], float)
    tri = np.array([[0, 1, 2], [1, 3, 2], [0, 4, 5]], np.int32)  # 0-1 share an edge, 0-2 a vertex
    tets = np.array([[0, 1, 2, 6]], np.int32)
    o10 = oracle.Oracle(nodes, tets, tri, tri, np.zeros((0, 3)), np.zeros(0), 4.0, 80.0, 0.0, n_ss=10)
    o4 = oracle.Oracle(nodes, tets, tri, tri, np.zeros((0, 3)), np.zeros(0), 4.0, 80.0, 0.0, n_ss=4)
    # the semi-analytic reference converges algebraically in the outer rule
    # (about 2e-7 at 40x40 points per sub-triangle); Sauter-Schwab converges
    # exponentially in n_ss
    for sig, tol in ((0, 4e-7), (1, 4e-7), (2, 1e-8)):
        ref = np.array([[_outer(nodes[tri[0]], nodes[tri[sig]], a, b, 40) for b in range(3)] for a in range(3)])
        V10, K10 = o10.pair_integral(0, 0, sig)
        V4, _ = o4.pair_integral(0, 0, sig)
        assert np.abs(V10 - ref).max() < tol * np.abs(ref).max(), (sig, V10, ref)
        assert np.abs(V4 - ref).max() < 1e-4 * np.abs(ref).max()
        assert np.abs(K10).max() < 1e-15  # coplanar panels: (x-y).n_y = 0


def test_sauter_schwab_exponential_convergence_nonplanar():
    p = cached_config(0)
    vals = []
    for ns in (3, 5, 7, 12):
        o = oracle.Oracle.from_problem(p, n_ss=ns)
        # triangle 0 against itself and its neighbours
        tri = p.tri_m
        nb = [j for j in range(tri.shape[0]) if len(set(tri[0]) & set(tri[j])) in (1, 2)][:4]
        vals.append(np.concatenate([np.concatenate([o.pair_integral(1, 0, j)[0].ravel(),
                                                    o.pair_integral(1, 0, j)[1].ravel()]) for j in [0] + nb]))
    d = [np.abs(vals[i] - vals[-1]).max() / np.abs(vals[-1]).max() for i in range(3)]
    # about one digit per extra point in each direction
    assert d[0] < 1e-3 and d[1] < 1e-5 and d[2] < 1e-7


# ---------------------------------------------------------------------------
# sphere eigenvalues: spherical harmonics diagonalise V and K on a sphere
# ---------------------------------------------------------------------------
def sphere_eigs(kind, R, kappa, l):
    if kind == "laplace":
        return R / (2 * l + 1), -1.0 / (2 * (2 * l + 1))
    # scipy's k_l carries a factor pi/2 (k_0(x) = pi e^{-x} / (2x))
    x = kappa * R
    i, k = special.spherical_in(l, x), special.spherical_kn(l, x) * 2 / np.pi
    di, dk = special.spherical_in(l, x, derivative=True), special.spherical_kn(l, x, derivative=True) * 2 / np.pi
    return kappa * R * R * i * k, 0.5 * x * x * (i * dk + di * k)


def rayleigh(o, surf, f):
    V, K = o.bem_dense(surf)
    Mf = o.surface_mass_apply(surf, f)
    return (f @ V @ f) / (f @ Mf), (f @ K @ f) / (f @ Mf)


def test_closed_forms_l0_yukawa_values():
    # P5 spot values: R = 8, kappa = 0.125 gives V[1] = (1 - e^{-2kR})/(2k)
    v, k = sphere_eigs("yukawa", 8.0, 0.125, 0)
    assert abs(v - (1 - np.exp(-2.0)) / 0.25) < 1e-12
    assert abs(k + (1 - np.exp(-2.0) * 2.0) / 2.0) < 1e-12


@pytest.mark.parametrize("surf,kind", [(0, "laplace"), (1, "yukawa")])
def test_sphere_rayleigh_quotients_converge(surf, kind):
    R_in, t, kappa = 4.0, 4.0, 0.125
    errs = []
    for n in (4, 8):
        p = pbgen.make_problem(n=n, a=R_in, c=R_in, bump=False, t=t, L=1, helix=0, partials=0, kappa=kappa,
                               center_charge=1.0)
        o = oracle.Oracle.from_problem(p)
        g = o.surface_nodes(surf)
        xyz = p.nodes[g]
        R = R_in if surf == 0 else R_in + t
        e = []
        for l, f in ((0, np.ones(g.size)), (1, xyz[:, 2] / R)):
            v_ex, k_ex = sphere_eigs(kind, R, kappa, l)
            v, k = rayleigh(o, surf, f)
            e += [abs(v - v_ex) / abs(v_ex), abs(k - k_ex) / abs(k_ex)]
        errs.append(np.array(e))
    assert np.all(errs[1] < 0.01)
    if kind == "laplace":
        # K0[1] = -1/2 holds exactly on the faceted surface (Gauss identity):
        # only the quadrature error is left, no h^2 discretisation error
        assert errs[0][1] < 1e-5 and errs[1][1] < 1e-5
        errs = [np.delete(e, 1) for e in errs]
    # O(h^2) for a flat-panel P1 discretisation; quotients already within
    # 1e-4 (the Yukawa l = 0 single layer, whose error changes sign between
    # these meshes) are only bounded
    big = errs[0] > 1e-4
    assert np.all(errs[1][~big] < 1e-4)
    ratio = errs[0][big] / errs[1][big]
    assert big.sum() >= 2 and np.all(ratio > 2.5), ratio


def test_yukawa_tends_to_laplace_as_kappa_vanishes():
    p = cached_config(0)
    # the same triangulation on both surfaces: surface 0 Laplace, surface 1 Yukawa
    o = oracle.Oracle(p.nodes, p.tets, p.tri_m, p.tri_m, p.q_xyz, p.q_z, 4.0, 80.0, 1e-6)
    V0, K0 = o.bem_dense(0)
    V1, K1 = o.bem_dense(1)
    assert np.abs(V1 - V0).max() < 2e-6 * np.abs(V0).max()
    assert np.abs(V1 - V0).max() > 0
    assert np.abs(K1 - K0).max() < 1e-10 * np.abs(K0).max()


def test_coulomb_load_converges():
    # sum_i f_i = int_{Gamma_m} phi_coul -> 4 pi a l_B z / eps_m for a central charge
    vals = []
    for n in (4, 8):
        p = pbgen.make_problem(n=n, a=4.0, c=4.0, bump=False, t=4.0, L=1, helix=0, partials=0,
                               kappa=0.125, center_charge=1.0)
        o = oracle.Oracle.from_problem(p)
        vals.append(o.coulomb_load().sum())
    ex = 4 * np.pi * 4.0 * o.l_bjerrum / 4.0
    e = [abs(v - ex) / ex for v in vals]
    assert e[1] < 5e-3 and 3.0 < e[0] / e[1] < 5.0
