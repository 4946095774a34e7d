"""Regular-assembly tile shapes and the autotuner, through the C ABI.

Every candidate shape (ta target x tb source triangles per workgroup) must
assemble the same Galerkin blocks as the oracle: the shape changes only the
order of the floating-point sums.  The surface here (720 triangles, 362
vertices) is not a multiple of any block size, so every shape has a ragged
last block on both sides, and the Yukawa surface takes the kappa > 0 kernel.
"""
import sys

import numpy as np
import pytest

import oracle
import pbgen

pytestmark = pytest.mark.gpu

SHAPES = [(16, 32), (8, 32), (8, 64), (16, 16), (8, 16)]
SPEC = dict(n=6, a=5.0, c=8.0, bump=True, t=3.0, L=2, helix=2, partials=4, kappa=0.15, seed=(9, 3))


def log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def tiles():
    import paper_2511_21713_amd as pb
    ctx = pb.Context(0)
    prob = pbgen.make_problem(**SPEC)
    o = oracle.Oracle.from_problem(prob)
    refs = []
    for surf in (0, 1):
        V, K = o.bem_dense(surf)
        nv = V.shape[0]
        M = np.stack([o.surface_mass_apply(surf, e) for e in np.eye(nv)], 1)
        refs.append((-V if surf == 0 else V, 0.5 * M + (K if surf == 0 else -K)))
    return pb, ctx, prob, refs


def rowrel(A, B):
    return (np.abs(A - B) / np.abs(B).max(1, keepdims=True)).max()


@pytest.mark.parametrize("precision", [0, 1])
@pytest.mark.parametrize("shape", SHAPES)
def test_each_tile_shape_matches_oracle(tiles, shape, precision):
    pb, ctx, prob, refs = tiles
    g = pb.Problem.from_inputs(ctx, prob, precision=precision)
    g.set_tile_shape(*shape)
    bar = 1e-12 if precision == 0 else 1e-6
    for surf in (0, 1):
        Vp, Kp = g.export_bem(surf)
        assert g.tile_shape(surf) == shape
        eV, eK = rowrel(Vp, refs[surf][0]), rowrel(Kp, refs[surf][1])
        log(f"  shape {shape} precision {precision} surf {surf}: V {eV:.2e} K {eK:.2e}")
        assert eV < bar and eK < bar
    g.close()


def test_tuned_shape_is_a_candidate_and_sticks(tiles):
    """Default mode: the autotuner picks a candidate; a second problem of the
    same size class in the same context reuses the choice, and the operators
    equal those of that shape pinned explicitly, bit for bit."""
    pb, ctx, prob, refs = tiles
    g = pb.Problem.from_inputs(ctx, prob)
    Vt, Kt = g.export_bem(1)
    shape = g.tile_shape(1)
    log(f"  tuned shape (Yukawa, FP64, 720 triangles): {shape}")
    assert shape in SHAPES
    assert rowrel(Vt, refs[1][0]) < 1e-12 and rowrel(Kt, refs[1][1]) < 1e-12
    g2 = pb.Problem.from_inputs(ctx, prob)
    V2, K2 = g2.export_bem(1)
    assert g2.tile_shape(1) == shape
    assert np.array_equal(V2, Vt) and np.array_equal(K2, Kt)
    g2.set_tile_shape(*shape)
    V3, K3 = g2.export_bem(1)
    assert np.array_equal(V3, Vt) and np.array_equal(K3, Kt)
    g2.set_tile_shape(0, 0)
    assert g2.tile_shape(1) == shape  # last assembly until the next one
    g.close()
    g2.close()


def test_solve_with_pinned_shapes_agrees(tiles):
    """Full solves with two different pinned shapes agree to rounding."""
    pb, ctx, prob, refs = tiles
    kw = dict(tol_nl=1e-10, tol_gr=1e-12, tol_gr0=1e-12, tol_omega=1e-9, l_e=0.0, max_gmres=20000)
    tot = []
    for shape in ((8, 32), (16, 16)):
        g = pb.Problem.from_inputs(ctx, prob)
        g.set_tile_shape(*shape)
        r = g.solve(**kw)
        assert r["status"] == 0
        tot.append(r["total"])
        g.close()
    log(f"  totals {tot[0]!r} {tot[1]!r}")
    assert abs(tot[0] - tot[1]) < 1e-11 * abs(tot[0])


@pytest.mark.parametrize("precision", [0, 1])
def test_symmetric_apply_matches_full_rows(tiles, precision):
    """A square shape stores the regular single layer bitwise symmetric and
    the apply reads K' and only the lower triangle of V' (plus the two-ring
    difference left by the touching blocks); a rectangular shape applies
    full rows.  The residual and Jacobian products of the two agree to
    rounding, and (FP64) match the oracle's."""
    pb, ctx, prob, refs = tiles
    o = oracle.Oracle.from_problem(prob)
    rng = np.random.default_rng(31 + precision)
    phi = rng.standard_normal(o.n)
    v = rng.standard_normal(o.n)
    out = {}
    for shape in ((16, 32), (16, 16)):
        g = pb.Problem.from_inputs(ctx, prob, precision=precision)
        g.set_tile_shape(*shape)
        out[shape] = (g.residual(oracle.HS, phi), g.apply_jacobian(oracle.HS, phi, v))
        assert g.tile_shape(0) == shape
        g.close()
    (Ff, Jf), (Fs, Js) = out[(16, 32)], out[(16, 16)]
    eF, eJ = rowrel(Fs[None, :], Ff[None, :]), rowrel(Js[None, :], Jf[None, :])
    log(f"  precision {precision}: symmetric vs full rows F {eF:.2e} Jv {eJ:.2e}")
    bar = 1e-13 if precision == 0 else 1e-6
    assert eF < bar and eJ < bar
    if precision == 0:
        assert rowrel(Js[None, :], o.apply_jacobian(oracle.HS, phi, v)[None, :]) < 1e-12


@pytest.mark.parametrize("shape", [(16, 16), (16, 32)])
def test_mixed_apply_accumulates_in_fp64(tiles, shape):
    """Mixed precision stores the boundary blocks in FP32 but forms every
    product in FP64: the device's Gamma_m and Gamma_s rows of J v equal a host
    FP64 product of the exported (widened) stored rows to 1e-13 of the sum of
    the products' magnitudes, far below the FP32 rounding of a partial sum."""
    pb, ctx, prob, refs = tiles
    g = pb.Problem.from_inputs(ctx, prob, precision=pb.MIXED)
    g.set_tile_shape(*shape)
    rng = np.random.default_rng(5)
    phi = rng.standard_normal(g.n)
    v = rng.standard_normal(g.n)
    Jv = g.apply_jacobian(oracle.LIN, phi, v)
    o = oracle.Oracle.from_problem(prob)
    off = g.n_nodes
    for surf, nv in ((0, g.n_m), (1, g.n_s)):
        Vp, Kp = g.export_bem(surf)
        u = v[o.surface_nodes(surf)]
        lam = v[off:off + nv]
        host = Kp @ u + Vp @ lam
        scale = np.abs(Kp) @ np.abs(u) + np.abs(Vp) @ np.abs(lam)
        err = (np.abs(Jv[off:off + nv] - host) / scale).max()
        log(f"  shape {shape} surf {surf}: mixed device rows vs host FP64 product {err:.2e}")
        assert err < 1e-13
        off += nv
    g.close()


def test_assembly_is_reproducible_and_launch_order_fixed(tiles):
    """The tiles of one launch add into disjoint operator entries (coloured
    blocks) and the launches follow each other, so the stored operators are
    bitwise the same on every assembly, for a square and a rectangular
    shape and both precisions."""
    pb, ctx, prob, refs = tiles
    for precision in (0, 1):
        for shape in ((16, 16), (16, 32)):
            g = pb.Problem.from_inputs(ctx, prob, precision=precision)
            g.set_tile_shape(*shape)
            first = [g.export_bem(s) for s in (0, 1)]
            for _ in range(2):
                g.reset_operators()
                again = [g.export_bem(s) for s in (0, 1)]
                for s in (0, 1):
                    assert np.array_equal(again[s][0], first[s][0]) and np.array_equal(again[s][1], first[s][1])
            g.close()


def test_bad_tile_shape_rejected(tiles):
    pb, ctx, prob, refs = tiles
    g = pb.Problem.from_inputs(ctx, prob)
    with pytest.raises(pb.PbfbError):
        g.set_tile_shape(12, 32)
    with pytest.raises(pb.PbfbError):
        g.set_tile_shape(16, 0)
    g.close()


def uv_sphere(nlon=9, nlat=6):
    """Unit sphere triangulated by latitude rings: the two poles have valence
    nlon (> 6), so some assembly block holds a vertex with more than 6 of its
    triangles and the fold takes its full corner lists."""
    verts = [(0.0, 0.0, 1.0)]
    for i in range(1, nlat):
        th = np.pi * i / nlat
        for j in range(nlon):
            ph = 2 * np.pi * (j + 0.5 * (i % 2)) / nlon
            verts.append((np.sin(th) * np.cos(ph), np.sin(th) * np.sin(ph), np.cos(th)))
    verts.append((0.0, 0.0, -1.0))
    verts = np.array(verts)
    ring = lambda i, j: 1 + (i - 1) * nlon + (j % nlon)
    south = len(verts) - 1
    tris = []
    for j in range(nlon):
        tris.append((0, ring(1, j), ring(1, j + 1)))
        tris.append((south, ring(nlat - 1, j + 1), ring(nlat - 1, j)))
    for i in range(1, nlat - 1):
        for j in range(nlon):
            a, b = ring(i, j), ring(i, j + 1)
            c, d = ring(i + 1, j), ring(i + 1, j + 1)
            if i % 2:
                tris += [(a, c, d), (a, d, b)]
            else:
                tris += [(a, c, b), (b, c, d)]
    tris = np.array(tris)
    # outward orientation (normal along the position)
    p = verts[tris]
    n = np.cross(p[:, 1] - p[:, 0], p[:, 2] - p[:, 0])
    flip = np.einsum("ij,ij->i", n, p.sum(1)) < 0
    tris[flip] = tris[flip][:, [0, 2, 1]]
    return verts, tris


def valence_problem(nlon, nlat=7):
    unit, tris = uv_sphere(nlon=nlon, nlat=nlat)
    nodes, tets, tri_m, tri_s = pbgen.shell_mesh(unit, tris, 4.0 * np.ones(unit.shape[0]), 3.0, 2)
    return pbgen.Problem(nodes=nodes, tets=tets, tri_m=tri_m, tri_s=tri_s, q_xyz=np.array([[0.0, 0.0, 0.5]]),
                         q_z=np.array([1.0]), eps_in=4.0, eps_out=80.0, kappa=0.2, info={})


@pytest.mark.parametrize("nlon", [9, 16, 24])
def test_high_valence_mesh_matches_oracle(tiles, nlon):
    """Poles of valence 9, 16 and 24 (the corner lists of the fold then take
    12 and 24 slots): every tile shape assembles the oracle's blocks."""
    pb, ctx, _, _ = tiles
    prob = valence_problem(nlon)
    o = oracle.Oracle.from_problem(prob)
    ref = []
    for surf in (0, 1):
        V, K = o.bem_dense(surf)
        nv = V.shape[0]
        M = np.stack([o.surface_mass_apply(surf, e) for e in np.eye(nv)], 1)
        ref.append((-V if surf == 0 else V, 0.5 * M + (K if surf == 0 else -K)))
    for shape in SHAPES:
        g = pb.Problem.from_inputs(ctx, prob)
        g.set_tile_shape(*shape)
        for surf in (0, 1):
            Vp, Kp = g.export_bem(surf)
            eV, eK = rowrel(Vp, ref[surf][0]), rowrel(Kp, ref[surf][1])
            log(f"  valence-{nlon} mesh, shape {shape}, surf {surf}: V {eV:.2e} K {eK:.2e}")
            assert eV < 1e-12 and eK < 1e-12
        g.close()


@pytest.mark.parametrize("precision", [0, 1])
def test_odd_vertex_count_matches_oracle(tiles, precision):
    """A surface with an odd number of vertices (47: the symmetric completion
    of FP32 storage then moves single entries instead of aligned pairs)
    assembles the oracle's blocks with every tile shape."""
    pb, ctx, _, _ = tiles
    prob = valence_problem(9, nlat=6)
    o = oracle.Oracle.from_problem(prob)
    bar = 1e-12 if precision == 0 else 1e-6
    ref = []
    for surf in (0, 1):
        V, K = o.bem_dense(surf)
        nv = V.shape[0]
        assert nv % 2 == 1
        M = np.stack([o.surface_mass_apply(surf, e) for e in np.eye(nv)], 1)
        ref.append((-V if surf == 0 else V, 0.5 * M + (K if surf == 0 else -K)))
    for shape in SHAPES:
        g = pb.Problem.from_inputs(ctx, prob, precision=precision)
        g.set_tile_shape(*shape)
        for surf in (0, 1):
            Vp, Kp = g.export_bem(surf)
            eV, eK = rowrel(Vp, ref[surf][0]), rowrel(Kp, ref[surf][1])
            log(f"  {Vp.shape[0]}-vertex mesh, shape {shape}, precision {precision}, surf {surf}: "
                f"V {eV:.2e} K {eK:.2e}")
            assert eV < bar and eK < bar
        g.close()


def test_high_valence_solve_matches_oracle(tiles):
    """A tight nonlinear solve on the valence-16 mesh (tuned shape) equals the
    oracle's energy and surface potential to 1e-10."""
    pb, ctx, _, _ = tiles
    prob = valence_problem(16)
    o = oracle.Oracle.from_problem(prob)
    kw = dict(tol_nl=1e-10, tol_gr=1e-12, tol_gr0=1e-12, tol_omega=1e-9, l_e=0.0, max_gmres=20000)
    g = pb.Problem.from_inputs(ctx, prob)
    phi = np.zeros(2 * g.n)
    r = g.solve(phi_out=phi, **kw)
    ro, pl, pnl = o.solve(**kw)
    gs = o.surface_nodes(0)
    u, uo = (phi[:g.n] + phi[g.n:])[gs], (pl + pnl)[gs]
    eE = abs(r["total"] - ro["total"]) / abs(ro["total"])
    eU = np.linalg.norm(u - uo) / np.linalg.norm(uo)
    log(f"  valence-16 solve: total {r['total']:.12f} vs {ro['total']:.12f} ({eE:.1e}), potential {eU:.1e}")
    assert r["status"] == 0 and eE < 1e-10 and eU < 1e-10
    g.close()
