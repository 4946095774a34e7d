"""Seeded synthetic inputs for the three-region FEM-BEM Poisson-Boltzmann problem.

This module only builds meshes, charges and physical parameters.  It holds
none of the method's arithmetic (no quadrature, no operators, no solver), so
both the CPU oracle and the HIP library can be fed from it.

Geometry recipe (the paper meshes molecular SES surfaces with NanoShaper and
fills the shell with TetMesh; those inputs are replaced here by synthetic
star-shaped solutes of the same size class):

* Gamma_m: class-I geodesic icosphere of frequency n (20 n^2 triangles,
  10 n^2 + 2 vertices), mapped radially by r(x) = spheroid radius plus a seeded
  real spherical-harmonic bump (l = 1..8) rescaled to amplitude A in [0.5, 1.5] A.
* Gamma_s: the radial copy r(x) + t.
* Shell Omega_i: L uniform radial layers of prisms, each prism split into three
  tetrahedra with the diagonal rule "lower-id bottom vertex to higher-id top
  vertex", which is conforming across neighbouring prisms.
* Charges: a double helix of unit negative charges (two strands half a turn
  apart, 11 charges per turn, 28 A pitch, radius 9 A, centred at z = 0) plus
  partial charges N(0, 0.3) drawn uniformly inside Gamma_m.  Helix charges that
  would sit outside Gamma_m or closer than ``clearance`` to it are pulled
  towards the origin until they keep that clearance.

Node numbering: FEM node (layer l, surface vertex v) has id l*Nv + v, so the
Gamma_m nodes are 0..Nv-1 and the Gamma_s nodes are L*Nv..(L+1)*Nv-1.
"""
from __future__ import annotations

import dataclasses
import functools
import math

import numpy as np

__all__ = ["Problem", "icosphere", "make_problem", "make_config", "config_params",
           "point_mesh_distance", "validate", "batch_instance", "serve_instance"]


@dataclasses.dataclass
class Problem:
    nodes: np.ndarray      # (n_nodes, 3) float64, Angstrom
    tets: np.ndarray       # (n_tets, 4) int32, positive orientation
    tri_m: np.ndarray      # (Nt, 3) int32 FEM node ids, outward (into the shell)
    tri_s: np.ndarray      # (Nt, 3) int32 FEM node ids, outward (into the far solvent)
    q_xyz: np.ndarray      # (Nq, 3) float64
    q_z: np.ndarray        # (Nq,) float64, valence in units of e
    eps_in: float
    eps_out: float
    kappa: float
    info: dict
    n_tets_m: int = 0      # > 0: the last n_tets_m tets fill the solute (two-field form)
    # two-field form: an independent Gamma_m surface mesh (own vertices on the
    # smooth solute surface, outward triangles), or None
    rs_verts: np.ndarray = None
    rs_tris: np.ndarray = None

    @property
    def n_nodes(self):
        return int(self.nodes.shape[0])


# ----------------------------------------------------------------------------
# surfaces
# ----------------------------------------------------------------------------
def _icosahedron():
    p = (1.0 + math.sqrt(5.0)) / 2.0
    v = np.array([[-1, p, 0], [1, p, 0], [-1, -p, 0], [1, -p, 0],
                  [0, -1, p], [0, 1, p], [0, -1, -p], [0, 1, -p],
                  [p, 0, -1], [p, 0, 1], [-p, 0, -1], [-p, 0, 1]], dtype=np.float64)
    f = np.array([[0, 11, 5], [0, 5, 1], [0, 1, 7], [0, 7, 10], [0, 10, 11],
                  [1, 5, 9], [5, 11, 4], [11, 10, 2], [10, 7, 6], [7, 1, 8],
                  [3, 9, 4], [3, 4, 2], [3, 2, 6], [3, 6, 8], [3, 8, 9],
                  [4, 9, 5], [2, 4, 11], [6, 2, 10], [8, 6, 7], [9, 8, 1]], dtype=np.int64)
    v /= np.linalg.norm(v, axis=1)[:, None]
    return v, f


def _icosphere_keyed(n: int):
    """icosphere(n) plus each vertex's key: its integer barycentric weights on
    the icosahedron corners, as a sorted tuple of (corner, weight)."""
    v, t, k = _icosphere_keyed_cached(int(n))
    return v.copy(), t.copy(), list(k)


@functools.lru_cache(maxsize=None)
def _icosphere_keyed_cached(n: int):
    if n < 1:
        raise ValueError("frequency must be >= 1")
    V, F = _icosahedron()
    key_to_id = {}
    pts = []

    def vid(face, i, j):
        a, b, c = (int(x) for x in F[face])
        w = {}
        for corner, weight in ((a, n - i - j), (b, i), (c, j)):
            if weight:
                w[corner] = w.get(corner, 0) + weight
        key = tuple(sorted(w.items()))
        if key not in key_to_id:
            key_to_id[key] = len(pts)
            p = sum(V[k] * (wt / n) for k, wt in key)
            pts.append(p / np.linalg.norm(p))
        return key_to_id[key]

    tris = []
    for face in range(20):
        for i in range(n):
            for j in range(n - i):
                tris.append((vid(face, i, j), vid(face, i + 1, j), vid(face, i, j + 1)))
                if i + j < n - 1:
                    tris.append((vid(face, i + 1, j), vid(face, i + 1, j + 1), vid(face, i, j + 1)))
    verts = np.array(pts)
    tris = np.array(tris, dtype=np.int64)
    # outward orientation
    a, b, c = verts[tris[:, 0]], verts[tris[:, 1]], verts[tris[:, 2]]
    nrm = np.cross(b - a, c - a)
    flip = np.einsum("ij,ij->i", nrm, a + b + c) < 0
    tris[flip] = tris[flip][:, [0, 2, 1]]
    assert verts.shape[0] == 10 * n * n + 2 and tris.shape[0] == 20 * n * n
    keys = [None] * len(pts)
    for k, i in key_to_id.items():
        keys[i] = k
    return verts, tris.astype(np.int32), keys


def icosphere(n: int):
    """Class-I geodesic subdivision of frequency n, projected to the unit sphere.

    Returns (verts (10n^2+2, 3), tris (20n^2, 3) int32, outward oriented).
    Grid points are keyed exactly by their integer barycentric weights on the
    icosahedron corners, so points on shared edges are merged exactly.
    """
    v, t, _ = _icosphere_keyed(n)
    return v, t


_SPH_CACHE = {}


def _real_sph_harm(lmax, xyz):
    """Real spherical harmonics Y_lm for l = 1..lmax (m = -l..l) at unit vectors
    (tables of the point sets seen before are reused)."""
    import hashlib
    key = (int(lmax), xyz.shape, hashlib.sha1(np.ascontiguousarray(xyz).tobytes()).hexdigest())
    if key not in _SPH_CACHE:
        if len(_SPH_CACHE) > 64:
            _SPH_CACHE.clear()
        _SPH_CACHE[key] = _real_sph_harm_eval(lmax, xyz)
    return _SPH_CACHE[key]


def _real_sph_harm_eval(lmax, xyz):
    from scipy import special
    theta = np.arccos(np.clip(xyz[:, 2], -1.0, 1.0))
    phi = np.arctan2(xyz[:, 1], xyz[:, 0])
    cols = []
    for l in range(1, lmax + 1):
        for m in range(-l, l + 1):
            y = special.sph_harm_y(l, abs(m), theta, phi)
            if m > 0:
                cols.append(math.sqrt(2.0) * (-1) ** m * y.real)
            elif m < 0:
                cols.append(math.sqrt(2.0) * (-1) ** m * y.imag)
            else:
                cols.append(y.real)
    return np.stack(cols, axis=1)


def radial_surface(unit, a, c, rng=None, lmax=8, amp_range=(0.5, 1.5), with_fn=False):
    """Radius r(x) of the star-shaped solute along each unit direction.

    Spheroid with semi-axes (a, a, c) plus, if rng is given, a seeded real
    spherical-harmonic bump sum_{l,m} c_lm Y_lm with c_lm ~ N(0,1)/(l+1)^2,
    rescaled so that max |bump| over the given directions equals A ~ U(amp_range).
    with_fn: also return the radius as a function of any unit directions
    (the same spheroid, coefficients and scale).
    """
    def spheroid(u):
        return 1.0 / np.sqrt((u[:, 0] ** 2 + u[:, 1] ** 2) / a ** 2 + u[:, 2] ** 2 / c ** 2)

    r = spheroid(unit)
    amp, coef, scale = 0.0, None, 0.0
    if rng is not None:
        amp = float(rng.uniform(*amp_range))
        ls = np.concatenate([[l] * (2 * l + 1) for l in range(1, lmax + 1)])
        coef = rng.standard_normal(ls.size) / (ls + 1.0) ** 2
        bump = _real_sph_harm(lmax, unit) @ coef
        scale = amp / np.max(np.abs(bump))
        bump *= scale
        r = r + bump
    if not with_fn:
        return r, amp

    def fn(u):
        out = spheroid(u)
        if coef is not None:
            out = out + (_real_sph_harm(lmax, u) @ coef) * scale
        return out

    return r, amp, fn


def shell_mesh(unit, tris, r_in, thickness, layers):
    """Prism shell between r_in(x) x and (r_in(x)+thickness) x, split into tets."""
    nv = unit.shape[0]
    L = int(layers)
    nodes = np.concatenate([(r_in + thickness * l / L)[:, None] * unit for l in range(L + 1)])
    t = np.sort(tris.astype(np.int64), axis=1)  # a < b < c by global id
    a, b, c = t[:, 0], t[:, 1], t[:, 2]
    tets = []
    for l in range(L):
        lo, hi = l * nv, (l + 1) * nv
        A, B, C = a + lo, b + lo, c + lo
        A2, B2, C2 = a + hi, b + hi, c + hi
        tets.append(np.stack([A, B, C, C2], 1))
        tets.append(np.stack([A, B, B2, C2], 1))
        tets.append(np.stack([A, A2, B2, C2], 1))
    tets = np.concatenate(tets)
    p = nodes[tets]
    vol = np.einsum("ij,ij->i", np.cross(p[:, 1] - p[:, 0], p[:, 2] - p[:, 0]), p[:, 3] - p[:, 0])
    neg = vol < 0
    tets[neg] = tets[neg][:, [0, 2, 1, 3]]
    tri_m = tris.astype(np.int64)
    tri_s = tris.astype(np.int64) + L * nv
    return nodes, tets.astype(np.int32), tri_m.astype(np.int32), tri_s.astype(np.int32)


def solute_mesh(n, radial, layers, first_id):
    """Tets filling the star-shaped solute inside Gamma_m = radial(unit) unit
    (Gamma_m: the frequency-n icosphere, node ids 0..10n^2+1).

    From Gamma_m inwards: `layers` scaled copies of Gamma_m joined by prisms
    split into 3 tets (as in the shell); then, while the frequency is even,
    a transition to the frequency-f/2 sphere, whose points are every other
    lattice point of the frequency-f one: each coarse triangle's slab (the 4
    fine triangles above it, the coarse one below, each side split at the
    fine edge midpoint) is coned to a point inside it, 14 tets; finally a cone
    from the coarsest sphere to the centre.  Every node then has a bounded
    number of neighbours (a cone from the fine sphere would join the centre
    to all of its vertices).  Copies sit at equal radial steps.  New nodes
    are numbered from first_id, so the shell part of the mesh is unchanged."""
    freqs = [n]
    while freqs[-1] % 2 == 0:
        freqs.append(freqs[-1] // 2)
    L, T = int(layers), len(freqs) - 1
    steps = L + T + 1
    nodes, tets = [], []
    next_id = [first_id]

    def add(x):
        i0 = next_id[0]
        nodes.append(x)
        next_id[0] += x.shape[0]
        return i0

    unit, tris, keys = _icosphere_keyed(n)
    r = radial(unit)
    gm_x = r[:, None] * unit  # Gamma_m, node ids 0..nv-1
    cur = np.arange(unit.shape[0])  # ids of the current (outermost remaining) copy
    k = 0
    t = np.sort(tris.astype(np.int64), axis=1)
    for _ in range(L):
        k += 1
        base = add((r * (1.0 - k / steps))[:, None] * unit)
        inner = base + np.arange(unit.shape[0])
        A, B, C = cur[t[:, 0]], cur[t[:, 1]], cur[t[:, 2]]
        A2, B2, C2 = inner[t[:, 0]], inner[t[:, 1]], inner[t[:, 2]]
        tets += [np.stack([A, B, C, C2], 1), np.stack([A, B, B2, C2], 1), np.stack([A, A2, B2, C2], 1)]
        cur = inner
    f = n
    for _ in range(T):
        k += 1
        fine_id = {kk: i for i, kk in enumerate(keys)}
        cu, ct, ck = _icosphere_keyed(f // 2)
        cr = radial(cu)
        base = add((cr * (1.0 - k / steps))[:, None] * cu)
        cids = base + np.arange(cu.shape[0])

        def fine_of(*ks):  # fine vertex id of a sum of coarse keys (weights double on the finer lattice)
            w = {}
            for kk in ks:
                for c, v in kk:
                    w[c] = w.get(c, 0) + v
            return int(cur[fine_id[tuple(sorted(w.items()))]])

        faces = []
        for (ia, ib, ic) in ct:
            X = [int(cids[ia]), int(cids[ib]), int(cids[ic])]
            kx = [ck[ia], ck[ib], ck[ic]]
            corner = [fine_of(kx[0], kx[0]), fine_of(kx[1], kx[1]), fine_of(kx[2], kx[2])]
            mid = {(0, 1): fine_of(kx[0], kx[1]), (1, 2): fine_of(kx[1], kx[2]), (0, 2): fine_of(kx[0], kx[2])}
            m01, m12, m02 = mid[(0, 1)], mid[(1, 2)], mid[(0, 2)]
            fc = [(corner[0], m01, m02), (corner[1], m12, m01), (corner[2], m02, m12), (m01, m12, m02),
                  (X[0], X[1], X[2])]
            for (i, j) in ((0, 1), (1, 2), (0, 2)):
                m = mid[(i, j)]
                fc += [(X[i], corner[i], m), (X[i], m, X[j]), (X[j], m, corner[j])]
            faces.append(fc)
        faces = np.array(faces, dtype=np.int64)  # (n_coarse_tri, 14, 3)
        # Steiner point: centroid of the slab's 9 vertices
        newx = np.concatenate(nodes)

        def pos(ids):
            return np.where((ids < first_id)[:, None], gm_x[np.minimum(ids, gm_x.shape[0] - 1)],
                            newx[np.maximum(ids - first_id, 0)])

        cen = np.stack([pos(np.unique(fc.ravel())).mean(0) for fc in faces])
        sb = add(cen)
        sid = sb + np.arange(faces.shape[0])
        tets.append(np.concatenate([np.concatenate([np.full((14, 1), sid[q]), faces[q]], 1)
                                    for q in range(faces.shape[0])]))
        cur, keys, f = cids, ck, f // 2
    # cone from the coarsest copy to the centre
    centre = add(np.zeros((1, 3)))
    ct = np.sort(_icosphere_keyed(f)[1].astype(np.int64), axis=1)
    tets.append(np.stack([cur[ct[:, 0]], cur[ct[:, 1]], cur[ct[:, 2]], np.full(ct.shape[0], centre)], 1))
    return np.concatenate(nodes), np.concatenate(tets)


def _radial_eval(u, unit, r):
    """r at the unit vectors u, each of which is one of `unit` (exact match
    of the lattice point's coordinates)."""
    idx = {tuple(x): i for i, x in enumerate(unit)}
    return np.array([r[idx[tuple(x)]] for x in u])


def _orient(nodes, tets):
    p = nodes[tets]
    vol = np.einsum("ij,ij->i", np.cross(p[:, 1] - p[:, 0], p[:, 2] - p[:, 0]), p[:, 3] - p[:, 0])
    neg = vol < 0
    tets[neg] = tets[neg][:, [0, 2, 1, 3]]
    return tets


# ----------------------------------------------------------------------------
# geometry queries used for charge placement and validation
# ----------------------------------------------------------------------------
def point_mesh_distance(p, verts, tris):
    """Exact Euclidean distance from each point p (k,3) to a triangle mesh."""
    return MeshQuery(verts, tris).distance(p)


class MeshQuery:
    """Exact distance and star-shaped inside queries against one triangle mesh.

    Both restrict the exact per-triangle tests to candidate sets that provably
    hold every triangle that can matter:
    * distance: with c_t the centroid and rho_t the largest centroid-to-vertex
      distance of triangle t, dist(x, t) >= |x - c_t| - rho_t, and dist(x,
      mesh) <= |x - v| for the nearest vertex v, so only triangles with
      |x - c_t| <= |x - v| + max rho need the exact test;
    * inside (ray from the origin): the directions of a triangle's points form
      the spherical triangle of its vertex directions, inside the cap around
      its normalised centroid that reaches the farthest vertex direction; the
      ray's direction must lie in that cap (with a margin for the hit test's
      tolerance)."""

    def __init__(self, verts, tris):
        from scipy.spatial import cKDTree
        self.A = verts[tris[:, 0]]
        self.B = verts[tris[:, 1]]
        self.C = verts[tris[:, 2]]
        self.E1 = self.B - self.A
        self.E2 = self.C - self.A
        self.small = tris.shape[0] <= 512
        if self.small:
            return
        cen = (self.A + self.B + self.C) / 3.0
        rho = np.max(np.stack([np.linalg.norm(V - cen, axis=1) for V in (self.A, self.B, self.C)]), axis=0)
        self.vtree = cKDTree(verts[np.unique(tris)])
        self.ctree = cKDTree(cen)
        self.slack = float(rho.max()) * (1.0 + 1e-9) + 1e-9
        cd = cen / np.linalg.norm(cen, axis=1)[:, None]
        chord = np.max(np.stack([np.linalg.norm(V / np.linalg.norm(V, axis=1)[:, None] - cd, axis=1)
                                 for V in (self.A, self.B, self.C)]), axis=0)
        self.dtree = cKDTree(cd)
        self.reach = float(chord.max()) * 1.01 + 1e-6

    def _pairs(self, tree, q, radii):
        """Flattened (point, candidate triangle) pairs of the ball queries."""
        lists = tree.query_ball_point(q, radii)
        cnt = np.fromiter((len(c) for c in lists), dtype=np.int64, count=len(lists))
        tri = np.fromiter((t for c in lists for t in c), dtype=np.int64, count=int(cnt.sum()))
        pt = np.repeat(np.arange(len(lists)), cnt)
        return pt, tri, cnt

    def distance(self, p):
        p = np.atleast_2d(np.asarray(p, dtype=np.float64))
        out = np.empty(p.shape[0])
        if p.shape[0] == 0:
            return out
        if self.small:
            for i, x in enumerate(p):
                out[i] = np.sqrt(np.min(_pt_tri_dist2(x, self.A, self.B, self.C)))
            return out
        dv, _ = self.vtree.query(p)
        pt, tri, cnt = self._pairs(self.ctree, p, dv * (1.0 + 1e-9) + self.slack)
        d2 = _pt_tri_dist2(p[pt], self.A[tri], self.B[tri], self.C[tri])
        start = np.concatenate([[0], np.cumsum(cnt)[:-1]])
        return np.sqrt(np.minimum.reduceat(d2, start))

    def inside(self, p):
        p = np.atleast_2d(np.asarray(p, dtype=np.float64))
        res = np.zeros(p.shape[0], dtype=bool)
        if p.shape[0] == 0:
            return res
        rn = np.linalg.norm(p, axis=1)
        zero = rn == 0
        res[zero] = True
        idx = np.nonzero(~zero)[0]
        if idx.size == 0:
            return res
        d = p[idx] / rn[idx][:, None]
        if self.small:
            pt = np.repeat(np.arange(idx.size), self.A.shape[0])
            tri = np.tile(np.arange(self.A.shape[0]), idx.size)
            cnt = np.full(idx.size, self.A.shape[0])
        else:
            pt, tri, cnt = self._pairs(self.dtree, d, self.reach)
        dd = d[pt]
        a, e1, e2 = self.A[tri], self.E1[tri], self.E2[tri]
        h = np.cross(dd, e2)
        det = np.einsum("ij,ij->i", e1, h)
        ok = np.abs(det) > 1e-14
        inv = np.where(ok, 1.0 / np.where(ok, det, 1.0), 0.0)
        s = -a
        u = np.einsum("ij,ij->i", s, h) * inv
        qv = np.cross(s, e1)
        v = np.einsum("ij,ij->i", qv, dd) * inv
        t = np.einsum("ij,ij->i", e2, qv) * inv
        hit = ok & (u >= -1e-12) & (v >= -1e-12) & (u + v <= 1 + 1e-12) & (t > 0)
        tmin = np.where(hit, t, np.inf)
        start = np.concatenate([[0], np.cumsum(cnt)[:-1]])
        has = cnt > 0
        first = np.full(idx.size, np.inf)
        first[has] = np.minimum.reduceat(tmin, start[has])
        res[idx] = np.isfinite(first) & (rn[idx] < first)
        return res


def _pt_tri_dist2(x, A, B, C):
    # closest point on triangle (Ericson, Real-Time Collision Detection, 5.1.5)
    ab, ac, ap = B - A, C - A, x - A
    d1 = np.einsum("ij,ij->i", ab, ap)
    d2 = np.einsum("ij,ij->i", ac, ap)
    bp = x - B
    d3 = np.einsum("ij,ij->i", ab, bp)
    d4 = np.einsum("ij,ij->i", ac, bp)
    cp = x - C
    d5 = np.einsum("ij,ij->i", ab, cp)
    d6 = np.einsum("ij,ij->i", ac, cp)
    va = d3 * d6 - d5 * d4
    vb = d5 * d2 - d1 * d6
    vc = d1 * d4 - d3 * d2
    denom = va + vb + vc
    with np.errstate(divide="ignore", invalid="ignore"):
        v = vb / denom
        w = vc / denom
    q = A + ab * v[:, None] + ac * w[:, None]
    # region tests, later assignments take priority in reverse order of checks
    m = (d1 <= 0) & (d2 <= 0)
    q[m] = A[m]
    m2 = (d3 >= 0) & (d4 <= d3)
    q[m2 & ~m] = B[m2 & ~m]
    done = m | m2
    m3 = (d6 >= 0) & (d5 <= d6) & ~done
    q[m3] = C[m3]
    done |= m3
    m4 = (vc <= 0) & (d1 >= 0) & (d3 <= 0) & ~done
    with np.errstate(divide="ignore", invalid="ignore"):
        t4 = d1 / (d1 - d3)
    q[m4] = A[m4] + t4[m4, None] * ab[m4]
    done |= m4
    m5 = (vb <= 0) & (d2 >= 0) & (d6 <= 0) & ~done
    with np.errstate(divide="ignore", invalid="ignore"):
        t5 = d2 / (d2 - d6)
    q[m5] = A[m5] + t5[m5, None] * ac[m5]
    done |= m5
    m6 = (va <= 0) & ((d4 - d3) >= 0) & ((d5 - d6) >= 0) & ~done
    with np.errstate(divide="ignore", invalid="ignore"):
        t6 = (d4 - d3) / ((d4 - d3) + (d5 - d6))
    q[m6] = B[m6] + t6[m6, None] * (C[m6] - B[m6])
    d = x - q
    return np.einsum("ij,ij->i", d, d)


def inside_star(p, verts, tris):
    """Inside test for a surface star-shaped about the origin (ray from origin)."""
    return MeshQuery(verts, tris).inside(p)


def _place_helix(n_per_strand, radius, verts, tris, clearance, log):
    pts = []
    rise = 28.0 / 11.0
    for s in range(2):
        for k in range(n_per_strand):
            th = 2.0 * math.pi * k / 11.0 + math.pi * s
            z = (k - (n_per_strand - 1) / 2.0) * rise
            pts.append([radius * math.cos(th), radius * math.sin(th), z])
    pts = np.array(pts)
    mq = MeshQuery(verts, tris)

    def ok(x, sc):  # every point x[i] scaled by sc[i] inside, with the clearance
        y = x * sc[:, None]
        good = mq.inside(y)
        if np.any(good):
            good[good] = mq.distance(y[good]) >= clearance
        return good

    # charges that violate the clearance move towards the origin: scale factors
    # 0.95, 0.90, ... until one is feasible (0 ends the search), then 16
    # bisections between it and the last infeasible one
    bad = ~ok(pts, np.ones(len(pts)))
    idx = np.nonzero(bad)[0]
    x = pts[idx]
    s_hi = np.ones(idx.size)
    step = np.ones(idx.size)
    active = np.ones(idx.size, dtype=bool)
    while np.any(active):
        step[active] = np.maximum(0.0, step[active] - 0.05)
        a_idx = np.nonzero(active)[0]
        zero = step[a_idx] == 0.0
        done = zero.copy()
        rest = a_idx[~zero]
        if rest.size:
            done[~zero] = ok(x[rest], step[rest])
        for j, dn in zip(a_idx, done):
            if not dn:
                s_hi[j] = step[j]
        active[a_idx[done]] = False
    s_lo = step.copy()
    for _ in range(16):
        mid = 0.5 * (s_lo + s_hi)
        g = ok(x, mid) if idx.size else np.zeros(0, dtype=bool)
        s_lo = np.where(g, mid, s_lo)
        s_hi = np.where(g, s_hi, mid)
    out = pts.copy()
    out[idx] = x * s_lo[:, None]
    log["helix_tapered"] = int(idx.size)
    return out


def _place_partials(count, sigma, rng, verts, tris, clearance):
    lo = verts.min(0)
    hi = verts.max(0)
    acc = []
    mq = MeshQuery(verts, tris)
    while len(acc) < count:
        cand = rng.uniform(lo, hi, size=(max(64, 2 * (count - len(acc))), 3))
        ins = mq.inside(cand)
        cand = cand[ins]
        if cand.size:
            d = mq.distance(cand)
            cand = cand[d >= clearance]
        for c in cand:
            if len(acc) < count:
                acc.append(c)
    z = rng.normal(0.0, sigma, size=count)
    return np.array(acc).reshape(-1, 3), z


# ----------------------------------------------------------------------------
# configurations
# ----------------------------------------------------------------------------
def config_params(cfg: int):
    """Geometry/charge recipe for the named workloads."""
    if cfg == 0:
        return dict(n=4, a=4.0, c=4.0, bump=False, t=4.0, L=6, helix=0, partials=0, kappa=0.125)
    if cfg == 1:
        return dict(n=32, a=10.0, c=30.0, bump=True, t=6.0, L=10, helix=24, partials=400, kappa=0.125)
    if cfg == 2:
        return dict(n=64, a=12.0, c=70.0, bump=True, t=6.0, L=12, helix=60, partials=400, kappa=0.125)
    raise ValueError(f"unknown config {cfg}")


def make_problem(n, a, c, bump, t, L, helix, partials, kappa, seed=(0, 0),
                 eps_in=4.0, eps_out=80.0, clearance=1.5, center_charge=None, solute_layers=0, reaction_n=None):
    """solute_layers > 0 adds the tets of the solute (Sec. 2.3's FEM domain
    Omega_m u Omega_i): they follow the shell tets, their new nodes follow the
    shell nodes, and Problem.n_tets_m counts them.  reaction_n (with
    solute_layers): an independent Gamma_m surface mesh, the icosphere of
    frequency reaction_n with its vertices on the smooth solute surface
    (Problem.rs_verts, rs_tris), not a face set of the volume mesh."""
    rng = np.random.default_rng(list(seed))
    unit, tris = icosphere(n)
    r, amp, rfn = radial_surface(unit, a, c, rng if bump else None, with_fn=True)
    nodes, tets, tri_m, tri_s = shell_mesh(unit, tris, r, t, L)
    n_tets_m = 0
    if solute_layers:
        inodes, itets = solute_mesh(n, lambda u: _radial_eval(u, unit, r), solute_layers, nodes.shape[0])
        nodes = np.concatenate([nodes, inodes])
        itets = _orient(nodes, itets)
        n_tets_m = int(itets.shape[0])
        tets = np.concatenate([tets, itets.astype(np.int32)])
    log = dict(n=n, a=a, c=c, amp=amp, t=t, L=L, seed=list(seed), solute_layers=int(solute_layers))
    rs_verts = rs_tris = None
    if reaction_n:
        if not solute_layers:
            raise ValueError("an independent Gamma_m mesh needs the two-field form (solute_layers > 0)")
        uf, rs_tris = icosphere(int(reaction_n))
        rs_verts = np.ascontiguousarray(rfn(uf)[:, None] * uf)
        rs_tris = np.ascontiguousarray(rs_tris, dtype=np.int32)
        log["reaction_n"] = int(reaction_n)
    gm = nodes[: unit.shape[0]]
    qx, qz = [], []
    if center_charge is not None:
        qx.append(np.zeros((1, 3)))
        qz.append(np.array([float(center_charge)]))
    if helix:
        hx = _place_helix(helix, 9.0, gm, tris, clearance, log)
        qx.append(hx)
        qz.append(-np.ones(hx.shape[0]))
    if partials:
        px, pz = _place_partials(partials, 0.3, rng, gm, tris, clearance)
        qx.append(px)
        qz.append(pz)
    q_xyz = np.concatenate(qx) if qx else np.zeros((0, 3))
    q_z = np.concatenate(qz) if qz else np.zeros(0)
    return Problem(nodes=np.ascontiguousarray(nodes), tets=np.ascontiguousarray(tets),
                   tri_m=np.ascontiguousarray(tri_m), tri_s=np.ascontiguousarray(tri_s),
                   q_xyz=np.ascontiguousarray(q_xyz, dtype=np.float64),
                   q_z=np.ascontiguousarray(q_z, dtype=np.float64),
                   eps_in=eps_in, eps_out=eps_out, kappa=kappa, info=log, n_tets_m=n_tets_m,
                   rs_verts=rs_verts, rs_tris=rs_tris)


def make_config(cfg: int, instance: int = 0, **override):
    """Workload `cfg` (0: charged sphere, 1: RNA-like 20k-triangle solute,
    2: RNA-like 80k-triangle solute), seeded by default_rng([cfg, instance])."""
    p = config_params(cfg)
    p.update(override)
    center = 1.0 if cfg == 0 else None
    return make_problem(seed=(cfg, instance), center_charge=center, **p)


def batch_instance(cfg: int, instance: int, n_lo=4, n_hi=44):
    """One instance of the batched workload: triangle count log-uniform over
    frequencies [n_lo, n_hi], kappa ~ U(0.03, 0.33), half sphere-type (the
    charged-sphere generator: central +1 charge) and half RNA-type (the
    RNA-like generator: helix of 4..60 charges plus its 400 partial charges)."""
    rng = np.random.default_rng([cfg, instance, 7])
    n = int(round(math.exp(rng.uniform(math.log(n_lo), math.log(n_hi)))))
    kappa = float(rng.uniform(0.03, 0.33))
    if instance % 2 == 0:
        return make_problem(n=n, a=4.0, c=4.0, bump=False, t=4.0, L=6, helix=0, partials=0,
                            kappa=kappa, seed=(cfg, instance), center_charge=1.0)
    h = int(rng.integers(4, 61))
    per = (h + 1) // 2
    span = (per - 1) * 28.0 / 11.0
    c = max(15.0, span / 2.0 + 8.0)
    L = 10
    return make_problem(n=n, a=10.0, c=c, bump=True, t=6.0, L=L, helix=per, partials=400,
                        kappa=kappa, seed=(cfg, instance))


def serve_instance(instance: int, n_lo=4, n_hi=64, cfg=4):
    """One request of the serving workload: an RNA-like solute of the
    RNA-like generator with a triangle count log-uniform over frequencies
    [n_lo, n_hi], a helix of 4..60 charges, its 400 partial charges and
    kappa ~ U(0.03, 0.33)."""
    rng = np.random.default_rng([cfg, instance, 11])
    n = int(round(math.exp(rng.uniform(math.log(n_lo), math.log(n_hi)))))
    kappa = float(rng.uniform(0.03, 0.33))
    h = int(rng.integers(4, 61))
    per = (h + 1) // 2
    c = max(15.0, (per - 1) * 28.0 / 11.0 / 2.0 + 8.0)
    return make_problem(n=n, a=10.0, c=c, bump=True, t=6.0, L=10, helix=per, partials=400, kappa=kappa,
                        seed=(cfg, instance))


# ----------------------------------------------------------------------------
# validation (mesh sanity; no method arithmetic)
# ----------------------------------------------------------------------------
def validate(p: Problem, clearance=1.0):
    nodes, tets = p.nodes, p.tets
    x = nodes[tets]
    vol = np.einsum("ij,ij->i", np.cross(x[:, 1] - x[:, 0], x[:, 2] - x[:, 0]), x[:, 3] - x[:, 0]) / 6
    assert np.all(vol > 0), "non-positive tet volume"
    for tri in (p.tri_m, p.tri_s):
        e = np.concatenate([tri[:, [0, 1]], tri[:, [1, 2]], tri[:, [2, 0]]])
        directed = set(map(tuple, e.tolist()))
        assert len(directed) == e.shape[0], "directed edge repeated"
        assert all((b, a) in directed for a, b in directed), "surface not closed"
        nv = np.unique(tri).size
        ne = e.shape[0] // 2
        assert nv - ne + tri.shape[0] == 2, "Euler characteristic != 2"
        v = nodes[tri]
        sv = np.einsum("ij,ij->i", v[:, 0], np.cross(v[:, 1], v[:, 2])).sum() / 6
        assert sv > 0, "surface not outward"
    if p.q_xyz.shape[0]:
        vm = np.unique(p.tri_m)
        d = point_mesh_distance(p.q_xyz, nodes, p.tri_m)
        assert np.all(d >= clearance), "charge too close to Gamma_m"
        assert np.all(inside_star(p.q_xyz, nodes, p.tri_m)), "charge outside Gamma_m"
    return True
