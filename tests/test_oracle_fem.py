"""Pins for the oracle's FEM pieces on the shell (stiffness, mass, N, J, H).

Weak form of the shell equation (Sec. 2.2, tested with v rather than grad v,
which is how a reaction term is tested):
  A_ab = eps_s sum_T |T| grad phi_a . grad phi_b
  N(u)_a = eps_s kappa^2 int calN(u_h) phi_a,  J(u) v = eps_s kappa^2 int calN'(u_h) v_h phi_a,
  H(u)[v]_a = eps_s kappa^2 int calN''(u_h) v_h^2 phi_a
"""
import math

import numpy as np
import pytest
import scipy.sparse as sp

import oracle
import pbgen
from conftest import cached_config


@pytest.fixture(scope="module")
def cfg0():
    p = cached_config(0)
    return p, oracle.Oracle.from_problem(p)


def tet_volumes(p):
    x = p.nodes[p.tets]
    return np.abs(np.linalg.det(np.stack([x[:, 1] - x[:, 0], x[:, 2] - x[:, 0], x[:, 3] - x[:, 0]], 1))) / 6


def coo(p, entries):
    r, c, v = entries
    n = p.n_nodes
    return sp.coo_matrix((v, (r, c)), shape=(n, n)).tocsr()


def test_stiffness_row_sums_symmetry_psd(cfg0):
    p, o = cfg0
    A = coo(p, o.stiffness_entries(p.tets.shape[0]))
    amax = np.abs(A).max()
    assert np.abs(A @ np.ones(p.n_nodes)).max() <= 1e-13 * amax
    assert abs(A - A.T).max() <= 1e-14 * amax
    ev = np.linalg.eigvalsh(A.toarray())
    assert ev.min() > -1e-12 * ev.max()
    assert np.sum(ev < 1e-10 * ev.max()) == 1  # only constants in the kernel


def test_stiffness_energy_of_linear_field(cfg0):
    # P1 reproduces linear fields, so u^T A u = eps_s |g|^2 vol exactly
    p, o = cfg0
    A = coo(p, o.stiffness_entries(p.tets.shape[0]))
    g = np.array([0.3, -1.1, 0.7])
    u = p.nodes @ g
    vol = tet_volumes(p).sum()
    assert abs(u @ (A @ u) - p.eps_out * (g @ g) * vol) <= 1e-12 * p.eps_out * (g @ g) * vol


def test_single_tet_stiffness_closed_form():
    nodes = np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0], [0, 0, 1]], float)
    tets = np.array([[0, 1, 2, 3]], np.int32)
    tri = np.array([[0, 2, 1]], np.int32)
    o = oracle.Oracle(nodes, tets, tri, tri, np.zeros((0, 3)), np.zeros(0), 4.0, 80.0, 0.0)
    r, c, v = o.stiffness_entries(1)
    A = np.zeros((4, 4))
    np.add.at(A, (r, c), v)
    ref = np.array([[3, -1, -1, -1], [-1, 1, 0, 0], [-1, 0, 1, 0], [-1, 0, 0, 1]]) / 6.0 * 80.0
    assert np.allclose(A, ref, atol=1e-13)


def test_mass_closed_form_and_volume(cfg0):
    p, o = cfg0
    r, c, v = o.mass_entries(p.tets.shape[0])
    vol = tet_volumes(p)
    # P1 mass on a tet: |T| (1 + delta_ab) / 20
    ref = (np.repeat(vol, 16) * np.where(r == c, 2.0, 1.0) / 20.0)
    assert np.allclose(v, ref, rtol=1e-13, atol=0)
    M = coo(p, (r, c, v))
    one = np.ones(p.n_nodes)
    assert abs(one @ (M @ one) - vol.sum()) <= 1e-13 * vol.sum()


@pytest.mark.parametrize("scheme", [oracle.LIN, oracle.T3, oracle.T5, oracle.T7, oracle.HS])
def test_jacobian_at_zero_is_scaled_mass(cfg0, scheme):
    p, o = cfg0
    M = coo(p, o.mass_entries(p.tets.shape[0]))
    v = np.random.default_rng(1).standard_normal(p.n_nodes)
    J0v = o.fem_jacobian(scheme, np.zeros(p.n_nodes), v)
    ref = p.eps_out * p.kappa ** 2 * (M @ v)
    assert np.allclose(J0v, ref, rtol=1e-12, atol=1e-14 * np.abs(ref).max())


def test_nonlinear_on_constant_field(cfg0):
    p, o = cfg0
    c = 0.8
    u = np.full(p.n_nodes, c)
    vol = tet_volumes(p)
    lumped = np.zeros(p.n_nodes)
    np.add.at(lumped, p.tets.ravel(), np.repeat(vol / 4.0, 4))
    k2 = p.eps_out * p.kappa ** 2
    assert np.allclose(o.fem_nonlinear(oracle.HS, u), k2 * np.sinh(c) * lumped, rtol=1e-13)
    assert np.allclose(o.fem_nonlinear(oracle.T3, u), k2 * (c + c ** 3 / 6) * lumped, rtol=1e-13)
    assert np.allclose(o.fem_nonlinear(oracle.LIN, u), k2 * c * lumped, rtol=1e-13)
    # the Taylor schemes of Sec. 3.3.1: sinh cut after the 5th and 7th powers
    assert np.allclose(o.fem_nonlinear(oracle.T5, u), k2 * (c + c ** 3 / 6 + c ** 5 / 120) * lumped, rtol=1e-13)
    assert np.allclose(o.fem_nonlinear(oracle.T7, u),
                       k2 * (c + c ** 3 / 6 + c ** 5 / 120 + c ** 7 / 5040) * lumped, rtol=1e-13)
    # and their derivatives, the cosh and sinh series cut one and two orders lower
    one = np.ones(p.n_nodes)
    for s_, d1, d2 in ((oracle.T5, 1 + c ** 2 / 2 + c ** 4 / 24, c + c ** 3 / 6),
                       (oracle.T7, 1 + c ** 2 / 2 + c ** 4 / 24 + c ** 6 / 720, c + c ** 3 / 6 + c ** 5 / 120)):
        assert np.allclose(o.fem_jacobian(s_, u, one), k2 * d1 * lumped, rtol=1e-13)
        assert np.allclose(o.fem_hessian(s_, u, one), k2 * d2 * lumped, rtol=1e-13)


def test_taylor_schemes_approach_sinh():
    """On a constant field the gap between a Taylor scheme and sinh is the
    series remainder, bounded by cosh(c) c^(o+2) / (o+2)!; each order closes
    most of the gap of the one before."""
    p = cached_config(0)
    o = oracle.Oracle.from_problem(p)
    for c in (0.5, 1.5, 3.0):
        u = np.full(p.n_nodes, c)
        hs = o.fem_nonlinear(oracle.HS, u)
        gaps = []
        for s_, order in ((oracle.T3, 3), (oracle.T5, 5), (oracle.T7, 7)):
            gap = np.abs(o.fem_nonlinear(s_, u) - hs).max() / np.abs(hs).max()
            bound = np.cosh(c) * c ** (order + 2) / math.factorial(order + 2) / np.sinh(c)
            assert 0 < gap <= bound * (1 + 1e-9)
            gaps.append(gap)
        assert gaps[0] > gaps[1] > gaps[2]


@pytest.mark.parametrize("scheme", [oracle.T3, oracle.T5, oracle.T7, oracle.HS])
def test_jacobian_and_hessian_by_central_differences(cfg0, scheme):
    p, o = cfg0
    rng = np.random.default_rng(2)
    u = rng.standard_normal(p.n_nodes)
    v = rng.standard_normal(p.n_nodes)
    J = o.fem_jacobian(scheme, u, v)
    H = o.fem_hessian(scheme, u, v)
    errs_j, errs_h = [], []
    for h in (1e-2, 5e-3):
        fdJ = (o.fem_nonlinear(scheme, u + h * v) - o.fem_nonlinear(scheme, u - h * v)) / (2 * h)
        fdH = (o.fem_jacobian(scheme, u + h * v, v) - o.fem_jacobian(scheme, u - h * v, v)) / (2 * h)
        errs_j.append(np.abs(fdJ - J).max() / np.abs(J).max())
        errs_h.append(np.abs(fdH - H).max() / np.abs(H).max())
    assert errs_j[0] < 1e-3 and errs_h[0] < 1e-3
    # second-order decay (a sign or factor slip would give O(1) or O(h))
    assert 3.0 < errs_j[0] / errs_j[1] < 5.0
    assert 3.0 < errs_h[0] / errs_h[1] < 5.0 or errs_h[0] < 1e-12


def test_generator_meshes_valid():
    for cfg in (0,):
        p = cached_config(cfg)
        pbgen.validate(p)
        n = p.info["n"]
        assert p.tri_m.shape[0] == 20 * n * n
        assert p.nodes.shape[0] == (p.info["L"] + 1) * (10 * n * n + 2)
        assert p.tets.shape[0] == 3 * p.info["L"] * 20 * n * n
