"""ctypes shim for the plain FP64 CPU oracle (oracle/pbref.c).

TEST INFRASTRUCTURE: only the tests, the smoke check and the CPU-baseline leg
of the benchmark may import this package.  The product path never calls it.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libpbref.so")

LIN, T3, HS, T5, T7 = 0, 1, 2, 3, 4

_lib = None


class Opts(C.Structure):
    _fields_ = [("scheme_first", C.c_int), ("omega_auto", C.c_int), ("omega_fixed", C.c_double),
                ("tol_nl", C.c_double), ("tol_gr", C.c_double), ("tol_gr0", C.c_double),
                ("tol_omega", C.c_double), ("l_e", C.c_double), ("omega0_first", C.c_double),
                ("omega0_next", C.c_double), ("omega_min", C.c_double), ("omega_max", C.c_double),
                ("max_newton", C.c_int), ("max_omega_it", C.c_int), ("gmres_restart", C.c_int),
                ("max_gmres", C.c_int), ("precond", C.c_int), ("cheb_degree", C.c_int),
                ("cheb_ratio", C.c_double), ("omega_method", C.c_int), ("nonlinear_method", C.c_int),
                ("r_e", C.c_double), ("n_schedule", C.c_int), ("schedule", C.c_int * 8)]


PC_DIAG, PC_CHEB_SPAI = 0, 1
OMEGA_NEWTON, OMEGA_BISECT, OMEGA_SECANT, OMEGA_BSEC, OMEGA_NEWTON_BS, OMEGA_BSEC_DF = 0, 1, 2, 3, 4, 5
NEWTON, PICARD = 0, 1
NONE = 7  # scheme without reaction term (the Picard linear operator)
FD_FN = C.CFUNCTYPE(C.c_int, C.c_void_p, C.c_double, C.POINTER(C.c_double), C.POINTER(C.c_double))


class Result(C.Structure):
    _fields_ = [("status", C.c_int), ("total", C.c_double), ("lc", C.c_double), ("nc", C.c_double),
                ("dg_omega_i", C.c_double), ("newton_iters", C.c_int), ("gmres_iters_total", C.c_int),
                ("gmres_lin", C.c_int), ("gmres_iters", C.c_int * 64), ("omega", C.c_double * 64),
                ("e_k", C.c_double * 64), ("omega_iters", C.c_int * 64), ("omega_fallback", C.c_int)]

    def as_dict(self):
        k = self.newton_iters
        return dict(status=self.status, total=self.total, lc=self.lc, nc=self.nc,
                    dg_omega_i=self.dg_omega_i, newton_iters=k, gmres_iters_total=self.gmres_iters_total,
                    gmres_lin=self.gmres_lin, gmres_iters=list(self.gmres_iters[:k]),
                    omega=list(self.omega[:k]), e_k=list(self.e_k[:k]),
                    omega_iters=list(self.omega_iters[:k]), omega_fallback=self.omega_fallback)


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            from . import build as _b
            _b.build()
        L = C.CDLL(LIB_PATH)
        P = C.c_void_p
        dp = C.POINTER(C.c_double)
        ip = C.POINTER(C.c_int32)
        lp = C.POINTER(C.c_int64)
        L.pbref_create.restype = P
        L.pbref_create.argtypes = [C.c_int64, dp, C.c_int64, ip, C.c_int64, ip, C.c_int64, ip, C.c_int64, dp, dp,
                                   C.c_double, C.c_double, C.c_double, C.c_double, C.c_int, C.c_int]
        L.pbref_destroy.argtypes = [P]
        L.pbref_sizes.argtypes = [P, lp]
        L.pbref_constants.argtypes = [P, dp]
        L.pbref_surface_nodes.argtypes = [P, C.c_int, ip]
        L.pbref_bem_dense.argtypes = [P, C.c_int]
        L.pbref_bem_get.argtypes = [P, C.c_int, dp, dp]
        L.pbref_bem_rows.argtypes = [P, C.c_int, C.c_int64, lp, dp, dp]
        L.pbref_pair_integral.argtypes = [P, C.c_int, C.c_int64, C.c_int64, dp, dp]
        L.pbref_surface_mass_apply.argtypes = [P, C.c_int, dp, dp]
        L.pbref_coulomb_load.argtypes = [P, dp]
        L.pbref_stiffness_entries.argtypes = [P, ip, ip, dp]
        L.pbref_mass_entries.argtypes = [P, ip, ip, dp]
        for f in ("pbref_fem_nonlinear",):
            getattr(L, f).argtypes = [P, C.c_int, dp, dp]
        for f in ("pbref_fem_jacobian", "pbref_fem_hessian"):
            getattr(L, f).argtypes = [P, C.c_int, dp, dp, dp]
        L.pbref_apply_A.argtypes = [P, dp, dp]
        L.pbref_dense_rows_apply.argtypes = [P, C.c_int, C.c_int64, dp, dp, dp, dp]
        L.pbref_rhs.argtypes = [P, dp]
        L.pbref_set_rhs_extra.argtypes = [P, dp]
        L.pbref_set_rhs_extra.restype = None
        L.pbref_residual.argtypes = [P, C.c_int, dp, dp]
        L.pbref_apply_jacobian.argtypes = [P, C.c_int, dp, dp, dp]
        L.pbref_residual_rows.argtypes = [P, C.c_int, dp, C.c_int64, lp, dp]
        L.pbref_jacobian_rows.argtypes = [P, C.c_int, dp, dp, C.c_int64, lp, dp]
        L.pbref_opts_default.argtypes = [C.POINTER(Opts)]
        L.pbref_gmres.argtypes = [P, C.c_int, dp, dp, dp, C.c_double, C.c_int, C.c_int, C.POINTER(C.c_int)]
        L.pbref_gmres_pc.argtypes = [P, C.c_int, dp, dp, dp, C.c_double, C.c_int, C.c_int, C.c_int, C.c_int,
                                     C.c_double, C.POINTER(C.c_int)]
        L.pbref_surface_ring.restype = C.c_int64
        L.pbref_surface_ring.argtypes = [P, C.c_int, ip, ip]
        L.pbref_spai_rows.argtypes = [C.c_int64, dp, ip, ip, dp]
        L.pbref_fem_gershgorin.restype = C.c_double
        L.pbref_fem_gershgorin.argtypes = [P, C.c_int, dp]
        L.pbref_cheb_diag.argtypes = [C.c_int64, dp, dp, C.c_double, C.c_double, C.c_int, dp, dp]
        L.pbref_solve.argtypes = [P, C.POINTER(Opts), C.POINTER(Result), dp, dp]
        L.pbref_energy.argtypes = [P, dp, dp, dp]
        L.pbref_fd.argtypes = [P, C.c_int, dp, dp, C.c_double, dp]
        L.pbref_root_find.argtypes = [C.c_int, C.c_int, C.c_double, FD_FN, P, C.POINTER(Opts),
                                      C.POINTER(C.c_int), C.POINTER(C.c_int)]
        L.pbref_root_find.restype = C.c_double
        L.pbref_omega_search.argtypes = [P, C.c_int, dp, dp, C.POINTER(Opts), dp, C.POINTER(C.c_int)]
        L.pbref_reaction_potential.argtypes = [P, dp, C.c_int64, dp, dp]
        L.pbref_set_two_field.argtypes = [P, C.c_int64]
        L.pbref_lambda_m.argtypes = [P, dp, C.c_int, dp]
        L.pbref_set_reaction_surface.argtypes = [P, C.c_int64, dp, C.c_int64, ip]
        L.pbref_gamma_m_vertices.argtypes = [P]
        L.pbref_gamma_m_vertices.restype = C.c_int64
        L.pbref_gamma_m_trace.argtypes = [P, dp, dp]
        L.pbref_rule_tri6.argtypes = [dp, dp]
        L.pbref_rule_tet27.argtypes = [dp, dp]
        L.pbref_rule_gauss01.argtypes = [C.c_int, dp, dp]
        L.pbref_rule_tri_collapsed.argtypes = [C.c_int, dp, dp]
        _lib = L
    return _lib


def set_threads(n):
    """OpenMP threads of the oracle's parallel loops in this process (the
    calling thread's setting, which every later oracle call inherits)."""
    lib()
    C.CDLL("libgomp.so.1").omp_set_num_threads(int(n))


def get_threads():
    lib()
    return int(C.CDLL("libgomp.so.1").omp_get_max_threads())


def _d(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _i(a):
    return a.ctypes.data_as(C.POINTER(C.c_int32))


def _l(a):
    return a.ctypes.data_as(C.POINTER(C.c_int64))


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def rule_tri6():
    b = np.zeros((6, 3)); w = np.zeros(6)
    lib().pbref_rule_tri6(_d(b), _d(w))
    return b, w


def rule_tet27():
    b = np.zeros((27, 4)); w = np.zeros(27)
    lib().pbref_rule_tet27(_d(b), _d(w))
    return b, w


def rule_gauss01(n):
    x = np.zeros(n); w = np.zeros(n)
    lib().pbref_rule_gauss01(n, _d(x), _d(w))
    return x, w


def rule_tri_collapsed(m):
    b = np.zeros((m * m, 3)); w = np.zeros(m * m)
    lib().pbref_rule_tri_collapsed(m, _d(b), _d(w))
    return b, w


def spai_rows(B, ptr, col):
    """Rows of the sparse approximate inverse of the dense matrix B on the pattern (ptr, col)."""
    B = _f64(B); ptr = np.ascontiguousarray(ptr, np.int32); col = np.ascontiguousarray(col, np.int32)
    val = np.zeros(col.size)
    st = lib().pbref_spai_rows(B.shape[0], _d(B), _i(ptr), _i(col), _d(val))
    return val, st


def cheb_diag(fdiag, dinv, lmax, ratio, k, r):
    """The Chebyshev terms of the FEM-block preconditioner for a diagonal F."""
    fdiag = _f64(fdiag); dinv = _f64(dinv); r = _f64(r); z = np.zeros(r.size)
    lib().pbref_cheb_diag(r.size, _d(fdiag), _d(dinv), lmax, ratio, k, _d(r), _d(z))
    return z


def default_opts(**kw):
    """Options with the defaults of pbref_opts_default; schedule=[T3, T5, ...]
    sets the per-iteration schemes (n_schedule and schedule)."""
    o = Opts()
    lib().pbref_opts_default(C.byref(o))
    for k, v in kw.items():
        if k == "schedule":
            v = list(v)
            assert len(v) <= 8
            o.n_schedule = len(v)
            for i, x in enumerate(v):
                o.schedule[i] = x
            continue
        setattr(o, k, v)
    return o


def root_find(method, k, omega0, f, **opts):
    """One root search of the oracle's f_d root finders on a Python function
    f(omega) -> (f_d, f_d') (None for an undefined value).  Returns (omega,
    evaluations, fallback)."""
    def cb(_ctx, w, fd, dfd):
        v = f(w)
        if v is None:
            return 1
        fd[0], dfd[0] = float(v[0]), float(v[1])
        return 0
    fn = FD_FN(cb)
    o = default_opts(**opts)
    ev, fb = C.c_int(0), C.c_int(0)
    w = lib().pbref_root_find(method, k, omega0, fn, None, C.byref(o), C.byref(ev), C.byref(fb))
    return w, ev.value, fb.value


class Oracle:
    """One oracle problem instance built from mesh, charges and parameters."""

    def __init__(self, nodes, tets, tri_m, tri_s, q_xyz, q_z, eps_in, eps_out, kappa,
                 temperature=298.15, reg_order=0, n_ss=4, n_tets_m=0, reaction_surface=None):
        L = lib()
        self._keep = [_f64(nodes), np.ascontiguousarray(tets, np.int32), np.ascontiguousarray(tri_m, np.int32),
                      np.ascontiguousarray(tri_s, np.int32), _f64(np.reshape(q_xyz, (-1, 3))), _f64(q_z)]
        x, t, tm, ts, qx, qz = self._keep
        self.h = L.pbref_create(x.shape[0], _d(x), t.shape[0], _i(t), tm.shape[0], _i(tm), ts.shape[0], _i(ts),
                                qz.shape[0], _d(qx), _d(qz), eps_in, eps_out, kappa, temperature,
                                reg_order, n_ss)
        if not self.h:
            raise ValueError("oracle rejected the mesh")
        self.two_field = n_tets_m > 0
        if self.two_field and L.pbref_set_two_field(self.h, int(n_tets_m)) != 0:
            raise ValueError("bad solute tet count")
        if reaction_surface is not None:
            self.set_reaction_surface(*reaction_surface)
        s = np.zeros(4, np.int64)
        L.pbref_sizes(self.h, _l(s))
        self.n_nodes, self.n_m, self.n_s, self.n = (int(v) for v in s)
        c = np.zeros(2)
        L.pbref_constants(self.h, _d(c))
        self.l_bjerrum, self.kT = float(c[0]), float(c[1])

    @classmethod
    def from_problem(cls, p, **kw):
        kw.setdefault("n_tets_m", getattr(p, "n_tets_m", 0))
        if getattr(p, "rs_verts", None) is not None:
            kw.setdefault("reaction_surface", (p.rs_verts, p.rs_tris))
        return cls(p.nodes, p.tets, p.tri_m, p.tri_s, p.q_xyz, p.q_z, p.eps_in, p.eps_out, p.kappa, **kw)

    def __del__(self):
        if getattr(self, "h", None):
            lib().pbref_destroy(self.h)
            self.h = None

    # surface data -----------------------------------------------------------
    def surface_nodes(self, surf):
        n = self.n_m if surf == 0 else self.n_s
        out = np.zeros(n, np.int32)
        lib().pbref_surface_nodes(self.h, surf, _i(out))
        return out

    def bem_dense(self, surf):
        n = self.n_m if surf == 0 else self.n_s
        r = lib().pbref_bem_dense(self.h, surf)
        if r:
            raise MemoryError(r)
        V = np.zeros((n, n)); K = np.zeros((n, n))
        lib().pbref_bem_get(self.h, surf, _d(V), _d(K))
        return V, K

    def bem_rows(self, surf, rows):
        n = self.n_m if surf == 0 else self.n_s
        rows = np.ascontiguousarray(rows, np.int64)
        V = np.zeros((rows.size, n)); K = np.zeros((rows.size, n))
        lib().pbref_bem_rows(self.h, surf, rows.size, _l(rows), _d(V), _d(K))
        return V, K

    def pair_integral(self, surf, tau, sig):
        V = np.zeros(9); K = np.zeros(9)
        lib().pbref_pair_integral(self.h, surf, tau, sig, _d(V), _d(K))
        return V.reshape(3, 3), K.reshape(3, 3)

    def surface_mass_apply(self, surf, x):
        x = _f64(x); y = np.zeros_like(x)
        lib().pbref_surface_mass_apply(self.h, surf, _d(x), _d(y))
        return y

    def coulomb_load(self):
        f = np.zeros(self.n_m)
        lib().pbref_coulomb_load(self.h, _d(f))
        return f

    # FEM -------------------------------------------------------------------
    def _entries(self, fn, nt):
        r = np.zeros(16 * nt, np.int32); c = np.zeros(16 * nt, np.int32); v = np.zeros(16 * nt)
        fn(self.h, _i(r), _i(c), _d(v))
        return r, c, v

    def stiffness_entries(self, n_tets):
        return self._entries(lib().pbref_stiffness_entries, n_tets)

    def mass_entries(self, n_tets):
        return self._entries(lib().pbref_mass_entries, n_tets)

    def fem_nonlinear(self, scheme, u):
        u = _f64(u); out = np.zeros(self.n_nodes)
        lib().pbref_fem_nonlinear(self.h, scheme, _d(u), _d(out))
        return out

    def fem_jacobian(self, scheme, u, v):
        u = _f64(u); v = _f64(v); out = np.zeros(self.n_nodes)
        lib().pbref_fem_jacobian(self.h, scheme, _d(u), _d(v), _d(out))
        return out

    def fem_hessian(self, scheme, u, v):
        u = _f64(u); v = _f64(v); out = np.zeros(self.n_nodes)
        lib().pbref_fem_hessian(self.h, scheme, _d(u), _d(v), _d(out))
        return out

    # coupled ---------------------------------------------------------------
    def apply_A(self, phi):
        phi = _f64(phi); y = np.zeros(self.n)
        r = lib().pbref_apply_A(self.h, _d(phi), _d(y))
        if r:
            raise RuntimeError(r)
        return y

    def dense_rows_apply(self, surf, V, K, x):
        V = _f64(V); K = _f64(K); x = _f64(x); out = np.zeros(V.shape[0])
        lib().pbref_dense_rows_apply(self.h, surf, V.shape[0], _d(V), _d(K), _d(x), _d(out))
        return out

    def rhs(self):
        b = np.zeros(self.n)
        lib().pbref_rhs(self.h, _d(b))
        return b

    def set_rhs_extra(self, e):
        """Add e to the right-hand side of every later residual and solve (None clears)."""
        if e is None:
            lib().pbref_set_rhs_extra(self.h, None)
        else:
            self._extra = _f64(e)
            lib().pbref_set_rhs_extra(self.h, _d(self._extra))

    def residual(self, scheme, phi):
        phi = _f64(phi); F = np.zeros(self.n)
        lib().pbref_residual(self.h, scheme, _d(phi), _d(F))
        return F

    def apply_jacobian(self, scheme, phi, v):
        phi = _f64(phi); v = _f64(v); y = np.zeros(self.n)
        lib().pbref_apply_jacobian(self.h, scheme, _d(phi), _d(v), _d(y))
        return y

    def residual_rows(self, scheme, phi, rows):
        phi = _f64(phi); rows = np.ascontiguousarray(rows, np.int64); out = np.zeros(rows.size)
        lib().pbref_residual_rows(self.h, scheme, _d(phi), rows.size, _l(rows), _d(out))
        return out

    def jacobian_rows(self, scheme, phi, v, rows):
        phi = _f64(phi); v = _f64(v); rows = np.ascontiguousarray(rows, np.int64); out = np.zeros(rows.size)
        lib().pbref_jacobian_rows(self.h, scheme, _d(phi), _d(v), rows.size, _l(rows), _d(out))
        return out

    def gmres(self, scheme, phi, b, tol=1e-10, restart=200, maxit=5000, precond=PC_DIAG, cheb_degree=16,
              cheb_ratio=200.0):
        phi = _f64(phi); b = _f64(b); x = np.zeros(self.n); it = C.c_int(0)
        st = lib().pbref_gmres_pc(self.h, scheme, _d(phi), _d(b), _d(x), tol, restart, maxit, precond,
                                  cheb_degree, cheb_ratio, C.byref(it))
        return x, st, it.value

    def surface_ring(self, surf):
        nnz = lib().pbref_surface_ring(self.h, surf, None, None)
        nv = len(self.surface_nodes(surf))
        ptr = np.zeros(nv + 1, np.int32); col = np.zeros(nnz, np.int32)
        lib().pbref_surface_ring(self.h, surf, _i(ptr), _i(col))
        return ptr, col

    def fem_gershgorin(self, scheme, u):
        return lib().pbref_fem_gershgorin(self.h, scheme, _d(_f64(u)))

    def solve(self, **opts):
        o = default_opts(**opts)
        res = Result()
        phil = np.zeros(self.n); phinl = np.zeros(self.n)
        lib().pbref_solve(self.h, C.byref(o), C.byref(res), _d(phil), _d(phinl))
        return res.as_dict(), phil, phinl

    def fd(self, scheme, phi, D, omega):
        phi = _f64(phi); D = _f64(D); out = np.zeros(2)
        st = lib().pbref_fd(self.h, scheme, _d(phi), _d(D), omega, _d(out))
        return float(out[0]), float(out[1]), st

    def omega_search(self, scheme, phi, D, omega0, **opts):
        o = default_opts(**opts)
        phi = _f64(phi); D = _f64(D); w = np.array([omega0], dtype=np.float64); it = C.c_int(0)
        fb = lib().pbref_omega_search(self.h, scheme, _d(phi), _d(D), C.byref(o), _d(w), C.byref(it))
        return float(w[0]), it.value, fb

    def energy(self, phi_lin, phi_nl=None):
        out = np.zeros(4)
        pl = _f64(phi_lin)
        pn = _f64(phi_nl) if phi_nl is not None else None
        lib().pbref_energy(self.h, _d(pl), _d(pn) if pn is not None else None, _d(out))
        return dict(total=out[0], lc=out[1], nc=out[2], dg_omega_i=out[3])

    def set_reaction_surface(self, verts, tris):
        """Two-field form: the Gamma_m mesh independent of the volume mesh
        (lam_m and the reaction potential live on it; the trace of u is its P1
        interpolant at the vertices).  verts = None removes it."""
        if verts is None:
            lib().pbref_set_reaction_surface(self.h, 0, None, 0, None)
            self._rs = None
            return
        v = _f64(np.reshape(verts, (-1, 3)))
        t = np.ascontiguousarray(tris, np.int32)
        r = lib().pbref_set_reaction_surface(self.h, v.shape[0], _d(v), t.shape[0], _i(t))
        if r == -3:
            raise ValueError("a Gamma_m vertex lies outside the FEM mesh")
        if r != 0:
            raise ValueError("bad Gamma_m surface")
        self._rs = (v, t)

    def gamma_m_trace(self, u):
        """u on the vertices of the surface that carries lam_m."""
        u = _f64(u)
        out = np.zeros(int(lib().pbref_gamma_m_vertices(self.h)))
        lib().pbref_gamma_m_trace(self.h, _d(u), _d(out))
        return out

    def lambda_m(self, u, with_load=True):
        """lam_m from the trace of u on Gamma_m (Sec. 2.3.1), by a dense solve."""
        u = _f64(u)
        out = np.zeros(int(lib().pbref_gamma_m_vertices(self.h)))
        if lib().pbref_lambda_m(self.h, _d(u), int(bool(with_load)), _d(out)) != 0:
            raise RuntimeError("singular single layer")
        return out

    def reaction_potential(self, phi, pts):
        phi = _f64(phi); pts = _f64(np.reshape(pts, (-1, 3))); out = np.zeros(pts.shape[0])
        lib().pbref_reaction_potential(self.h, _d(phi), pts.shape[0], _d(pts), _d(out))
        return out
