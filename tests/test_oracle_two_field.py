"""Pins for the oracle's two-field form (Sec. 2.3, eq. fembem_matrix).

FEM covers the solute and the shell (Omega_m u Omega_i): permittivity eps_m
in the solute tets and eps_s in the shell, reaction term in the shell only,
the point charges as the FEM load, and Yukawa BEM on Gamma_s.  lam_m is not
an unknown of the solve: Sec. 2.3.1 recovers it afterwards from the trace of
u on Gamma_m with the Laplace single layer, and the energy follows.

Checks, each against something fixed independently of the oracle's code:
* the load reproduces the charges' total and first moments (a P1 basis
  reproduces constants and linear functions exactly);
* the stiffness of a linear field is the permittivity jump times the normal
  flux through the interfaces (divergence theorem, exact for P1 on flat
  faces), so a swapped permittivity shows;
* the reaction term of u = 1 integrates to eps_s kappa^2 sinh(1) |Omega_i|
  with |Omega_i| from the coordinates;
* the lam_m row is the identity and the FEM rows carry no lam_m column;
* recovering lam_m from the three-field solution's trace returns its lam_m
  (the recovery equation is that solution's Gamma_m row);
* Born / Debye-Hueckel sphere: the energy converges to the closed form.

Gamma_m as its own surface mesh (the trace by interpolation, Sec. 2.3.1):
* the interpolated trace reproduces linear fields at every vertex of a finer
  surface (and not quadratic ones);
* the interface faces given as an independent, renumbered mesh give the
  conforming form's lam_m and energy;
* Born sphere with a finer Gamma_m mesh: second-order convergence;
* a surface outside the FEM mesh is refused.
"""
import numpy as np

import oracle
import pbgen
from test_oracle_solve import born_energy, lin_solve, radial_reference

SPEC = dict(n=3, a=6.0, c=9.0, bump=True, t=3.0, L=3, helix=3, partials=5, kappa=0.2, seed=(9, 1))


def two_field(**kw):
    p = pbgen.make_problem(solute_layers=3, **dict(SPEC, **kw))
    return p, oracle.Oracle.from_problem(p)


def tet_volumes(p, tets):
    P = p.nodes[tets]
    return np.einsum("ij,ij->i", np.cross(P[:, 1] - P[:, 0], P[:, 2] - P[:, 0]), P[:, 3] - P[:, 0]) / 6.0


def face_flux(p, tris, c):
    """out_a = sum over triangles at node a of |tau| / 3 (c . n_tau)"""
    P = p.nodes[tris]
    cr = np.cross(P[:, 1] - P[:, 0], P[:, 2] - P[:, 0])  # 2 |tau| n
    f = (cr @ c) / 6.0
    out = np.zeros(p.n_nodes)
    for k in range(3):
        np.add.at(out, tris[:, k], f)
    return out


def test_point_load_moments():
    p, o = two_field()
    b = o.rhs()
    Q = 4.0 * np.pi * o.l_bjerrum * p.q_z
    nn = o.n_nodes
    assert abs(b[:nn].sum() - Q.sum()) < 1e-12 * np.abs(Q).sum()
    m1 = p.nodes.T @ b[:nn]
    assert np.allclose(m1, Q @ p.q_xyz, rtol=0, atol=1e-11 * np.abs(Q).sum() * 10)
    assert np.all(b[nn:] == 0.0)


def test_stiffness_of_a_linear_field_is_the_interface_flux():
    p, o = two_field()
    c = np.array([0.3, -1.1, 0.7])
    u = p.nodes @ c
    y = o.apply_A(np.concatenate([u, np.zeros(o.n_m + o.n_s)]))[:o.n_nodes]
    expect = (p.eps_in - p.eps_out) * face_flux(p, p.tri_m, c) + p.eps_out * face_flux(p, p.tri_s, c)
    assert np.abs(y - expect).max() < 1e-11 * np.abs(expect).max()
    # the same field in the three-field form sees eps_s on the shell only
    p3 = pbgen.make_problem(**SPEC)
    o3 = oracle.Oracle.from_problem(p3)
    y3 = o3.apply_A(np.concatenate([p3.nodes @ c, np.zeros(o3.n_m + o3.n_s)]))[:o3.n_nodes]
    e3 = -p3.eps_out * face_flux(p3, p3.tri_m, c) + p3.eps_out * face_flux(p3, p3.tri_s, c)
    assert np.abs(y3 - e3).max() < 1e-11 * np.abs(e3).max()


def test_reaction_only_in_the_shell():
    p, o = two_field()
    ones = np.ones(o.n_nodes)
    vol_i = tet_volumes(p, p.tets[: len(p.tets) - p.n_tets_m]).sum()
    N = o.fem_nonlinear(oracle.HS, ones)
    expect = p.eps_out * p.kappa ** 2 * np.sinh(1.0) * vol_i
    assert abs(N.sum() - expect) < 1e-12 * expect
    inner = np.setdiff1d(np.arange(o.n_nodes), np.unique(p.tets[: len(p.tets) - p.n_tets_m]))
    assert inner.size > 0 and np.all(N[inner] == 0.0)


def test_lambda_m_row_is_identity_and_decoupled():
    p, o = two_field()
    rng = np.random.default_rng(3)
    lam = rng.standard_normal(o.n_m)
    x = np.zeros(o.n)
    x[o.n_nodes:o.n_nodes + o.n_m] = lam
    y = o.apply_A(x)
    assert np.all(y[:o.n_nodes] == 0.0) and np.all(y[o.n_nodes + o.n_m:] == 0.0)
    assert np.array_equal(y[o.n_nodes:o.n_nodes + o.n_m], lam)
    # the row-sampled residual agrees with the full one
    phi = rng.standard_normal(o.n)
    F = o.residual(oracle.HS, phi)
    rows = np.array([0, 7, o.n_nodes - 1, o.n_nodes, o.n_nodes + o.n_m - 1, o.n_nodes + o.n_m, o.n - 1])
    assert np.allclose(o.residual_rows(oracle.HS, phi, rows), F[rows], rtol=1e-12, atol=1e-12 * np.abs(F).max())


def test_lambda_m_recovery_returns_the_three_field_flux():
    p3 = pbgen.make_problem(**SPEC)
    o3 = oracle.Oracle.from_problem(p3)
    x = lin_solve(o3, tol=1e-13)
    nn, nm = o3.n_nodes, o3.n_m
    lam = o3.lambda_m(x[:nn], with_load=True)
    assert np.abs(lam - x[nn:nn + nm]).max() < 1e-9 * np.abs(x[nn:nn + nm]).max()
    # without the load: the homogeneous row (the correction part Phi_NL)
    V, K = o3.bem_dense(0)
    um = x[o3.surface_nodes(0)]
    lam0 = o3.lambda_m(x[:nn], with_load=False)
    r = 0.5 * o3.surface_mass_apply(0, um) + K @ um - V @ lam0
    assert np.abs(r).max() < 1e-12 * np.abs(K @ um).max()


def test_born_sphere_two_field():
    res = {}
    for n, lay in ((4, 3), (8, 6)):
        p = pbgen.make_problem(n=n, a=4.0, c=4.0, bump=False, t=4.0, L=6, helix=0, partials=0, kappa=0.125,
                               center_charge=1.0, solute_layers=lay)
        o = oracle.Oracle.from_problem(p)
        x = lin_solve(o)
        assert np.all(x[o.n_nodes:o.n_nodes + o.n_m] == 0.0)
        res[n] = o.energy(x)["total"]
    E_ex, _ = born_energy(o, 4.0, 1.0, 4.0, 80.0, 0.125)
    e4, e8 = abs(res[4] - E_ex) / abs(E_ex), abs(res[8] - E_ex) / abs(E_ex)
    assert e8 < 5e-3 and 3.0 < e4 / e8 < 5.0


def test_nonlinear_sphere_two_field_matches_radial_reference():
    """Strongly nonlinear central charge: the sinh solve of the two-field
    form converges to the radial ODE's energy at second order, and its
    lam_m stays zero through the Newton steps."""
    tot = []
    for n, lay in ((4, 3), (8, 6)):
        p = pbgen.make_problem(n=n, a=4.0, c=4.0, bump=False, t=4.0, L=6, helix=0, partials=0, kappa=0.125,
                               center_charge=8.0, solute_layers=lay)
        o = oracle.Oracle.from_problem(p)
        r, pl, pn = o.solve(tol_nl=1e-9, tol_gr=1e-11, tol_gr0=1e-11, l_e=0.0, tol_omega=1e-8)
        assert r["status"] == 0 and r["newton_iters"] > 2
        assert np.all(pn[o.n_nodes:o.n_nodes + o.n_m] == 0.0)
        tot.append(r["total"])
    E_ex, _ = radial_reference(4.0, 8.0, 8.0, 0.125, 4.0, 80.0, o.l_bjerrum, o.kT)
    e = [abs(v - E_ex) / abs(E_ex) for v in tot]
    assert e[1] < 5e-3 and 3.0 < e[0] / e[1] < 5.0


# ---------------------------------------------------------------------------
# Gamma_m given as its own surface mesh (Sec. 2.3.1: the trace of the volume
# solution on it by interpolation between the two meshes)
# ---------------------------------------------------------------------------
def test_independent_gamma_m_trace_reproduces_linear_fields():
    """The P1 interpolant of a linear field is the field itself, at every
    vertex of a finer surface that is not a face set of the volume mesh."""
    p = pbgen.make_problem(solute_layers=3, reaction_n=2 * SPEC["n"] + 1, **SPEC)
    o = oracle.Oracle.from_problem(p)
    assert p.rs_verts.shape[0] == 10 * (2 * SPEC["n"] + 1) ** 2 + 2
    c, c0 = np.array([0.3, -1.1, 0.7]), 0.25
    tr = o.gamma_m_trace(p.nodes @ c + c0)
    expect = p.rs_verts @ c + c0
    assert np.abs(tr - expect).max() < 1e-12 * np.abs(expect).max()
    # a quadratic field is not reproduced (the interpolation is P1, not node selection)
    q = o.gamma_m_trace((p.nodes ** 2).sum(1))
    assert np.abs(q - (p.rs_verts ** 2).sum(1)).max() > 1e-4


def test_independent_gamma_m_on_the_interface_matches_the_conforming_form():
    """The interface faces of the volume mesh given as an independent mesh
    (own vertex array, renumbered): every vertex is a tet vertex, so the
    interpolated trace is the nodal value (to the rounding of the barycentric
    coordinates) and lam_m and the energy equal the conforming two-field
    form's."""
    p, o = two_field()
    x = lin_solve(o, tol=1e-12)
    nodes_m = np.unique(p.tri_m)
    perm = np.random.default_rng(5).permutation(nodes_m.size)   # independent numbering
    new_id = np.empty(p.n_nodes, np.int64)
    new_id[nodes_m[perm]] = np.arange(nodes_m.size)
    verts = np.empty((nodes_m.size, 3))
    verts[new_id[nodes_m]] = p.nodes[nodes_m]
    tris = new_id[p.tri_m].astype(np.int32)
    e0 = o.energy(x)
    lam0 = o.lambda_m(x[:o.n_nodes])
    o.set_reaction_surface(verts, tris)
    tr = o.gamma_m_trace(x[:o.n_nodes])[new_id[nodes_m]]
    assert np.abs(tr - x[nodes_m]).max() < 1e-13 * np.abs(x[nodes_m]).max()
    lam1 = o.lambda_m(x[:o.n_nodes])
    assert np.abs(lam1[new_id[nodes_m]] - lam0).max() < 1e-11 * np.abs(lam0).max()
    e1 = o.energy(x)
    assert abs(e1["total"] - e0["total"]) < 1e-11 * abs(e0["total"])


def test_born_sphere_with_a_finer_independent_gamma_m():
    """Born / Debye-Hueckel with lam_m and the reaction potential on a sphere
    mesh finer than the volume's interface (its vertices on the exact
    sphere): the energy converges to the closed form at second order as both
    meshes are refined."""
    res = {}
    for n, lay, nr in ((4, 3, 6), (8, 6, 12)):
        p = pbgen.make_problem(n=n, a=4.0, c=4.0, bump=False, t=4.0, L=6, helix=0, partials=0, kappa=0.125,
                               center_charge=1.0, solute_layers=lay, reaction_n=nr)
        assert np.allclose(np.linalg.norm(p.rs_verts, axis=1), 4.0, rtol=0, atol=1e-12)
        o = oracle.Oracle.from_problem(p)
        x = lin_solve(o)
        res[n] = o.energy(x)["total"]
        assert o.lambda_m(x[:o.n_nodes]).shape == (10 * nr * nr + 2,)  # lam_m lives on the finer mesh
    E_ex, _ = born_energy(o, 4.0, 1.0, 4.0, 80.0, 0.125)
    e4, e8 = abs(res[4] - E_ex) / abs(E_ex), abs(res[8] - E_ex) / abs(E_ex)
    assert e8 < 5e-3 and 3.0 < e4 / e8 < 5.0


def test_independent_gamma_m_outside_the_mesh_is_refused():
    p, o = two_field()
    bad = np.array([[0.0, 0.0, 100.0], [1.0, 0.0, 100.0], [0.0, 1.0, 100.0], [0.0, 0.0, 101.0]])
    tris = np.array([[0, 2, 1], [0, 1, 3], [1, 2, 3], [0, 3, 2]], np.int32)
    try:
        o.set_reaction_surface(bad, tris)
    except ValueError as e:
        assert "outside" in str(e)
    else:
        raise AssertionError("a surface outside the FEM mesh was accepted")
