"""Pins for the oracle's GMRES preconditioners.

The paper leaves the preconditioner open; the preconditioner only changes
the Krylov path, never the discrete solution.  Pinned here:
* the Chebyshev terms against the closed form of the Chebyshev residual
  polynomial, 1 - lam p(lam) = T_k((theta - lam)/delta) / T_k(theta/delta);
* the sparse approximate inverse is exact when the inverse lives on the
  pattern (B = T^-1 with T supported on the pattern gives M = T);
* the 1-ring pattern against a set computation from the triangles;
* the Gershgorin bound against element-entry assembly and the spectrum;
* solves with either preconditioner reach the same solution, and a
  preconditioned GMRES solve matches a dense direct solve.
"""
import numpy as np
import pytest

import oracle
import pbgen
from conftest import cached_problem

SPHERE = dict(n=4, a=4.0, c=4.0, bump=False, t=4.0, L=6, helix=0, partials=0, kappa=0.125, center_charge=1.0)
BUMPY = dict(n=3, a=6.0, c=9.0, bump=True, t=3.0, L=3, helix=3, partials=5, kappa=0.2, seed=(9, 1))


def cheb_T(k, x):
    x = np.asarray(x, dtype=float)
    out = np.empty_like(x)
    inside = np.abs(x) <= 1
    out[inside] = np.cos(k * np.arccos(x[inside]))
    xo = x[~inside]
    out[~inside] = np.sign(xo) ** k * np.cosh(k * np.arccosh(np.abs(xo)))
    return out


@pytest.mark.parametrize("k", [1, 2, 3, 5, 8, 12])
@pytest.mark.parametrize("ratio", [4.0, 30.0])
def test_chebyshev_terms_closed_form(k, ratio):
    rng = np.random.default_rng(k)
    lmax = 2.7
    lam = np.concatenate([rng.uniform(lmax / ratio, lmax, 40), rng.uniform(0.01 * lmax / ratio, lmax / ratio, 5)])
    dinv = rng.uniform(0.5, 2.0, lam.size)
    fdiag = lam / dinv  # D^-1 F = diag(lam)
    r = rng.standard_normal(lam.size)
    z = oracle.cheb_diag(fdiag, dinv, lmax, ratio, k, r)
    lo = lmax / ratio
    theta, delta = (lmax + lo) / 2, (lmax - lo) / 2
    p = (1.0 - cheb_T(k, (theta - lam) / delta) / cheb_T(k, np.array([theta / delta]))[0]) / lam
    np.testing.assert_allclose(z, p * dinv * r, rtol=1e-11, atol=1e-14)


def ring_by_sets(tri, nv):
    ring = [{i} for i in range(nv)]
    for t in tri:
        for a in t:
            ring[a].update(int(b) for b in t)
    return [sorted(s) for s in ring]


@pytest.mark.parametrize("spec", [SPHERE, BUMPY])
def test_ring_pattern(spec):
    prob = cached_problem(**spec)
    o = oracle.Oracle.from_problem(prob)
    for surf, tri in ((0, prob.tri_m), (1, prob.tri_s)):
        g = o.surface_nodes(surf)
        loc = {int(v): i for i, v in enumerate(g)}
        tl = np.vectorize(loc.get)(tri)
        ptr, col = o.surface_ring(surf)
        ref = ring_by_sets(tl, len(g))
        for i in range(len(g)):
            assert list(col[ptr[i]:ptr[i + 1]]) == ref[i]


def test_spai_exact_when_inverse_is_on_the_pattern():
    prob = cached_problem(**SPHERE)
    o = oracle.Oracle.from_problem(prob)
    ptr, col = o.surface_ring(0)
    nv = ptr.size - 1
    rng = np.random.default_rng(4)
    T = np.zeros((nv, nv))
    for i in range(nv):
        for e in range(ptr[i], ptr[i + 1]):
            j = col[e]
            if j < i:
                T[i, j] = T[j, i] = rng.uniform(-1, 1)
    T += np.diag(np.abs(T).sum(1) + rng.uniform(0.5, 1.5, nv))
    B = np.linalg.inv(T)
    val, st = oracle.spai_rows(B, ptr, col)
    assert st == 0
    M = np.zeros((nv, nv))
    for i in range(nv):
        M[i, col[ptr[i]:ptr[i + 1]]] = val[ptr[i]:ptr[i + 1]]
    np.testing.assert_allclose(M, T, atol=1e-9 * np.abs(T).max())
    # a diagonal matrix: the diagonal inverse
    d = rng.uniform(1, 3, nv)
    val, st = oracle.spai_rows(np.diag(d), ptr, col)
    M = np.zeros((nv, nv))
    for i in range(nv):
        M[i, col[ptr[i]:ptr[i + 1]]] = val[ptr[i]:ptr[i + 1]]
    np.testing.assert_allclose(M, np.diag(1 / d), atol=1e-14)


def test_gershgorin_bound():
    import scipy.sparse as sp
    prob = cached_problem(**BUMPY)
    o = oracle.Oracle.from_problem(prob)
    nn = prob.nodes.shape[0]
    ne = prob.tets.shape[0]
    rA, cA, vA = o.stiffness_entries(ne)
    rM, cM, vM = o.mass_entries(ne)
    c = prob.eps_out * prob.kappa ** 2
    F = (sp.coo_matrix((vA, (rA, cA)), shape=(nn, nn)) + c * sp.coo_matrix((vM, (rM, cM)), shape=(nn, nn))).tocsr()
    dg = F.diagonal()
    bound = (abs(F).sum(1).A1 / dg).max()
    got = o.fem_gershgorin(oracle.LIN, np.zeros(o.n))
    assert abs(got - bound) < 1e-12 * bound
    ev = np.linalg.eigvals((F / dg[:, None]).toarray()).real
    assert ev.max() <= got * (1 + 1e-12)


def test_preconditioned_gmres_matches_direct_solve():
    prob = pbgen.make_problem(n=1, a=4.0, c=4.0, bump=False, t=3.0, L=2, helix=0, partials=0, kappa=0.3,
                              center_charge=-2.0)
    o = oracle.Oracle.from_problem(prob)
    rng = np.random.default_rng(2)
    phi = 0.5 * rng.standard_normal(o.n)
    J = np.stack([o.apply_jacobian(oracle.HS, phi, e) for e in np.eye(o.n)], 1)
    b = rng.standard_normal(o.n)
    x_ref = np.linalg.solve(J, b)
    for pc in (oracle.PC_DIAG, oracle.PC_CHEB_SPAI):
        x, st, it = o.gmres(oracle.HS, phi, b, tol=1e-13, precond=pc)
        assert st == 0
        assert np.linalg.norm(x - x_ref) < 1e-10 * np.linalg.norm(x_ref)


def test_solution_independent_of_preconditioner():
    prob = cached_problem(**BUMPY)
    o = oracle.Oracle.from_problem(prob)
    kw = dict(tol_nl=1e-10, tol_gr=1e-12, tol_gr0=1e-12, tol_omega=1e-9, l_e=0.0, max_gmres=20000)
    rd, pld, pnd = o.solve(precond=oracle.PC_DIAG, **kw)
    rc, plc, pnc = o.solve(precond=oracle.PC_CHEB_SPAI, **kw)
    assert rd["status"] == 0 and rc["status"] == 0
    assert abs(rc["total"] - rd["total"]) < 1e-10 * abs(rd["total"])
    assert np.linalg.norm((plc + pnc) - (pld + pnd)) < 1e-9 * np.linalg.norm(pld + pnd)
    # the block preconditioner needs far fewer Krylov steps
    assert rc["gmres_iters_total"] < 0.6 * rd["gmres_iters_total"]
