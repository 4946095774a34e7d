"""Python binding of libpbfb (the MI355X FEM-BEM nonlinear Poisson-Boltzmann
library).  Argument marshalling only: every step of the computation runs in
the library's HIP kernels.  PyTorch is used, when given, for device tensors
and the current stream.  The binding refuses to work without the compiled
library (there is no fallback path).
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libpbfb.so")

OK, EINVAL, EMESH, ECHARGE, ENOMEM, EDEVICE, ENOTCONV, ENAN, ESTATE = 0, -1, -2, -3, -4, -5, -6, -7, -8
FP64, MIXED = 0, 1
LIN, T3, HS, T5, T7 = 0, 1, 2, 3, 4
MEM_HOST, MEM_DEVICE = 0, 1
OMEGA_NEWTON, OMEGA_BISECT, OMEGA_SECANT, OMEGA_BSEC, OMEGA_NEWTON_BS, OMEGA_BSEC_DF = 0, 1, 2, 3, 4, 5
NEWTON, PICARD = 0, 1
BEM_DENSE, BEM_MATRIX_FREE = 0, 1
T_APPLY, T_GEMV, T_SPMV, T_ASM, T_SING = 0, 1, 2, 3, 4

EXPORTS = ["pbfb_ctx_create", "pbfb_ctx_destroy", "pbfb_last_error", "pbfb_problem_create", "pbfb_problem_destroy",
           "pbfb_set_mesh", "pbfb_set_charges", "pbfb_set_params", "pbfb_get_sizes", "pbfb_setup",
           "pbfb_reset_operators", "pbfb_residual", "pbfb_residual_noalloc",
           "pbfb_apply_jacobian", "pbfb_solve_opts_default", "pbfb_solve", "pbfb_solve_batch", "pbfb_server_create",
           "pbfb_server_submit", "pbfb_server_poll", "pbfb_request_footprint", "pbfb_server_destroy", "pbfb_energy", "pbfb_export_bem",
           "pbfb_export_bem_rows", "pbfb_export_rhs", "pbfb_set_bem_mode", "pbfb_set_two_field", "pbfb_set_reaction_surface", "pbfb_set_tile_shape", "pbfb_get_tile_shape", "pbfb_timing_enable", "pbfb_timing"]


class PbfbError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"pbfb error {code}: {msg}")
        self.code = code


class SolveOpts(C.Structure):
    _fields_ = [("scheme_first", C.c_int), ("omega_auto", C.c_int), ("omega_fixed", C.c_double),
                ("tol_nl", C.c_double), ("tol_gr", C.c_double), ("tol_gr0", C.c_double),
                ("tol_omega", C.c_double), ("l_e", C.c_double), ("omega0_first", C.c_double),
                ("omega0_next", C.c_double), ("omega_min", C.c_double), ("omega_max", C.c_double),
                ("max_newton", C.c_int), ("max_omega_it", C.c_int), ("gmres_restart", C.c_int),
                ("max_gmres", C.c_int), ("krylov_fp32", C.c_int), ("precond", C.c_int), ("cheb_degree", C.c_int),
                ("cheb_ratio", C.c_double), ("hip_graph", C.c_int), ("omega_method", C.c_int),
                ("nonlinear_method", C.c_int), ("r_e", C.c_double), ("n_schedule", C.c_int),
                ("schedule", C.c_int * 8)]


class Result(C.Structure):
    _fields_ = [("status", C.c_int), ("total", C.c_double), ("lc", C.c_double), ("nc", C.c_double),
                ("dg_omega_i", C.c_double), ("newton_iters", C.c_int), ("gmres_iters_total", C.c_int),
                ("gmres_lin", C.c_int), ("gmres_iters", C.c_int * 64), ("omega", C.c_double * 64),
                ("e_k", C.c_double * 64), ("omega_iters", C.c_int * 64), ("t_setup_s", C.c_double),
                ("t_solve_s", C.c_double), ("applies", C.c_int), ("t_wait_s", C.c_double)]

    def as_dict(self):
        k = min(self.newton_iters, 64)
        return dict(status=self.status, total=self.total, lc=self.lc, nc=self.nc, dg_omega_i=self.dg_omega_i,
                    newton_iters=self.newton_iters, gmres_iters_total=self.gmres_iters_total,
                    gmres_lin=self.gmres_lin, gmres_iters=list(self.gmres_iters[:k]), omega=list(self.omega[:k]),
                    e_k=list(self.e_k[:k]), omega_iters=list(self.omega_iters[:k]), t_setup_s=self.t_setup_s,
                    t_solve_s=self.t_solve_s, applies=self.applies, t_wait_s=self.t_wait_s)


_lib = None


def lib():
    """Load libpbfb.so; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with __graft_entry__.build() or "
                              "python paper_2511_21713_amd/build.py")
        # One HIP runtime per process: when PyTorch is installed its bundled
        # runtime (same soname) is loaded first, so the library binds to it
        # instead of pulling in a second copy that would fight over the device.
        try:
            import torch  # noqa: F401
        except ImportError:
            pass
        L = C.CDLL(LIB_PATH)
        P = C.c_void_p
        PP = C.POINTER(C.c_void_p)
        I64 = C.c_int64
        I64P = C.POINTER(C.c_int64)
        L.pbfb_ctx_create.argtypes = [C.c_int, PP]
        L.pbfb_ctx_destroy.argtypes = [P]
        L.pbfb_ctx_destroy.restype = None
        L.pbfb_last_error.restype = C.c_char_p
        L.pbfb_problem_create.argtypes = [P, C.c_int, PP]
        L.pbfb_problem_destroy.argtypes = [P]
        L.pbfb_problem_destroy.restype = None
        L.pbfb_set_mesh.argtypes = [P, I64, P, I64, P, I64, P, I64, P]
        L.pbfb_set_charges.argtypes = [P, I64, P, P]
        L.pbfb_set_params.argtypes = [P, C.c_double, C.c_double, C.c_double, C.c_double]
        L.pbfb_get_sizes.argtypes = [P, I64P, I64P, I64P, I64P, I64P]
        L.pbfb_setup.argtypes = [P, P]
        L.pbfb_reset_operators.argtypes = [P]
        L.pbfb_residual.argtypes = [P, C.c_int, P, P, C.c_int, P]
        L.pbfb_residual_noalloc.argtypes = [P, C.c_int, P, P, P]
        L.pbfb_apply_jacobian.argtypes = [P, C.c_int, P, P, P, C.c_int, P]
        L.pbfb_solve_opts_default.argtypes = [C.POINTER(SolveOpts)]
        L.pbfb_solve_opts_default.restype = None
        L.pbfb_solve.argtypes = [P, C.POINTER(SolveOpts), C.POINTER(Result), P, C.c_int, P]
        L.pbfb_energy.argtypes = [P, P, P, C.POINTER(C.c_double), C.c_int, P]
        L.pbfb_solve_batch.argtypes = [P, C.c_int, C.POINTER(C.c_void_p), C.POINTER(SolveOpts), C.POINTER(Result), P]
        L.pbfb_server_create.argtypes = [P, C.c_size_t, C.c_int, PP]
        L.pbfb_server_submit.argtypes = [P, P, C.POINTER(SolveOpts), C.POINTER(C.c_uint64)]
        L.pbfb_server_poll.argtypes = [P, C.c_uint64, C.POINTER(C.c_int), C.POINTER(Result)]
        L.pbfb_request_footprint.argtypes = [P, C.POINTER(SolveOpts), C.POINTER(C.c_size_t), C.POINTER(C.c_size_t)]
        L.pbfb_server_destroy.argtypes = [P]
        L.pbfb_export_bem.argtypes = [P, C.c_int, P, P]
        L.pbfb_export_bem_rows.argtypes = [P, C.c_int, I64, P, P, P]
        L.pbfb_export_rhs.argtypes = [P, P]
        L.pbfb_set_tile_shape.argtypes = [P, C.c_int, C.c_int]
        L.pbfb_set_bem_mode.argtypes = [P, C.c_int]
        L.pbfb_set_two_field.argtypes = [P, C.c_int64]
        L.pbfb_set_reaction_surface.argtypes = [P, C.c_int64, C.c_void_p, C.c_int64, C.c_void_p]
        L.pbfb_get_tile_shape.argtypes = [P, C.c_int, C.POINTER(C.c_int), C.POINTER(C.c_int)]
        L.pbfb_timing_enable.argtypes = [P, C.c_int]
        L.pbfb_timing.argtypes = [P, C.c_int, C.POINTER(C.c_double), I64P, C.c_int]
        _lib = L
    return _lib


def last_error():
    """Message of the last failing library call on this thread."""
    return lib().pbfb_last_error().decode()


def _check(code):
    if code != OK:
        raise PbfbError(code, lib().pbfb_last_error().decode())


def default_opts(**kw):
    """pbfb_solve_opts with the library defaults; schedule=[T3, T5, ...] sets
    n_schedule and the schedule entries."""
    o = SolveOpts()
    lib().pbfb_solve_opts_default(C.byref(o))
    for k, v in kw.items():
        if not hasattr(o, k):
            raise KeyError(k)
        if k == "schedule":
            v = list(v)
            if len(v) > 8:
                raise ValueError("at most 8 scheduled iterations")
            o.n_schedule = len(v)
            for i, x in enumerate(v):
                o.schedule[i] = x
            continue
        setattr(o, k, v)
    return o


def _is_torch(x):
    return type(x).__module__.startswith("torch")


def _vec(x, n, where):
    """(pointer, mem flag, keep-alive) for an FP64 vector argument."""
    if _is_torch(x):
        import torch
        assert x.dtype == torch.float64 and x.is_contiguous() and x.numel() == n
        return C.c_void_p(x.data_ptr()), (MEM_DEVICE if x.is_cuda else MEM_HOST), x
    a = np.ascontiguousarray(x, dtype=np.float64)
    assert a.size == n, (a.size, n)
    return C.c_void_p(a.ctypes.data), MEM_HOST, a


def _stream(stream):
    if stream is None:
        return None
    if _is_torch(stream):
        return C.c_void_p(stream.cuda_stream)
    return C.c_void_p(int(stream))


class Context:
    def __init__(self, device=0):
        h = C.c_void_p()
        _check(lib().pbfb_ctx_create(device, C.byref(h)))
        self.h = h
        self.device = device

    def close(self):
        if getattr(self, "h", None):
            lib().pbfb_ctx_destroy(self.h)
            self.h = None

    def __del__(self):
        self.close()


def solve_batch(ctx, problems, stream=None, **opts):
    """Solve several problems of one context together; returns a list of result dicts."""
    n = len(problems)
    arr = (C.c_void_p * max(n, 1))(*[p.h.value for p in problems])
    res = (Result * max(n, 1))()
    o = default_opts(**opts)
    code = lib().pbfb_solve_batch(ctx.h, n, arr, C.byref(o), res, _stream(stream))
    out = [res[i].as_dict() for i in range(n)]
    return code, out


class Server:
    """Continuous-batching server: submit problems, poll tickets."""

    def __init__(self, ctx, hbm_budget_bytes, max_slots):
        h = C.c_void_p()
        _check(lib().pbfb_server_create(ctx.h, int(hbm_budget_bytes), int(max_slots), C.byref(h)))
        self.h = h
        self.ctx = ctx
        self._keep = {}

    def submit(self, problem, **opts):
        o = default_opts(**opts)
        t = C.c_uint64()
        _check(lib().pbfb_server_submit(self.h, problem.h, C.byref(o), C.byref(t)))
        self._keep[t.value] = problem
        return t.value

    def poll(self, ticket):
        done = C.c_int()
        res = Result()
        _check(lib().pbfb_server_poll(self.h, ticket, C.byref(done), C.byref(res)))
        return (res.as_dict() if done.value else None)

    def close(self):
        if getattr(self, "h", None):
            code = lib().pbfb_server_destroy(self.h)
            self.h = None
            _check(code)

    def __del__(self):
        if getattr(self, "h", None):
            lib().pbfb_server_destroy(self.h)
            self.h = None


class Problem:
    """One Poisson-Boltzmann instance on the device (mesh, charges, parameters)."""

    def __init__(self, ctx, precision=FP64):
        h = C.c_void_p()
        _check(lib().pbfb_problem_create(ctx.h, precision, C.byref(h)))
        self.h = h
        self.ctx = ctx
        self.precision = precision

    @classmethod
    def from_inputs(cls, ctx, prob, precision=FP64, temperature=298.15):
        """Build from an object with nodes, tets, tri_m, tri_s, q_xyz, q_z, eps_in, eps_out, kappa."""
        self = cls(ctx, precision)
        self.set_mesh(prob.nodes, prob.tets, prob.tri_m, prob.tri_s)
        self.set_charges(prob.q_xyz, prob.q_z)
        self.set_params(prob.eps_in, prob.eps_out, prob.kappa, temperature)
        if getattr(prob, "n_tets_m", 0):
            self.set_two_field(prob.n_tets_m)
            if getattr(prob, "rs_verts", None) is not None:
                self.set_reaction_surface(prob.rs_verts, prob.rs_tris)
        return self

    def close(self):
        if getattr(self, "h", None):
            lib().pbfb_problem_destroy(self.h)
            self.h = None

    def __del__(self):
        self.close()

    # ---- inputs ---------------------------------------------------------------
    def set_mesh(self, nodes, tets, tri_m, tri_s):
        x = np.ascontiguousarray(nodes, np.float64)
        t = np.ascontiguousarray(tets, np.int32)
        a = np.ascontiguousarray(tri_m, np.int32)
        b = np.ascontiguousarray(tri_s, np.int32)
        _check(lib().pbfb_set_mesh(self.h, x.shape[0], x.ctypes.data, t.shape[0], t.ctypes.data, a.shape[0],
                                   a.ctypes.data, b.shape[0], b.ctypes.data))
        self._sizes()

    def set_charges(self, xyz, z):
        x = np.ascontiguousarray(np.reshape(xyz, (-1, 3)), np.float64)
        q = np.ascontiguousarray(z, np.float64)
        _check(lib().pbfb_set_charges(self.h, q.size, x.ctypes.data if q.size else None,
                                      q.ctypes.data if q.size else None))

    def set_params(self, eps_in, eps_out, kappa, temperature=298.15):
        _check(lib().pbfb_set_params(self.h, eps_in, eps_out, kappa, temperature))

    def _sizes(self):
        v = [C.c_int64() for _ in range(5)]
        _check(lib().pbfb_get_sizes(self.h, *[C.byref(x) for x in v]))
        self.n_nodes, self.n_m, self.n_s, self.n, self.hbm_bytes = (int(x.value) for x in v)
        return self.n

    def hbm(self):
        self._sizes()
        return self.hbm_bytes

    def setup(self, stream=None):
        _check(lib().pbfb_setup(self.h, _stream(stream)))

    def reset_operators(self):
        _check(lib().pbfb_reset_operators(self.h))

    # ---- operators ------------------------------------------------------------
    def residual(self, scheme, phi, out=None, stream=None):
        p, mem, keep = _vec(phi, self.n, "phi")
        if out is None:
            out = np.zeros(self.n) if mem == MEM_HOST else phi.new_zeros(self.n)
        o, mem2, keep2 = _vec(out, self.n, "out")
        assert mem == mem2
        _check(lib().pbfb_residual(self.h, scheme, p, o, mem, _stream(stream)))
        return out

    def residual_noalloc(self, scheme, phi, out, stream=None):
        """pbfb_residual_noalloc: phi and out are device tensors; nothing is allocated."""
        p, mem, keep = _vec(phi, self.n, "phi")
        o, mem2, keep2 = _vec(out, self.n, "out")
        if mem != MEM_DEVICE or mem2 != MEM_DEVICE:
            raise PbfbError(EINVAL, "residual_noalloc takes device tensors")
        _check(lib().pbfb_residual_noalloc(self.h, scheme, p, o, _stream(stream)))
        return out

    def apply_jacobian(self, scheme, phi, v, out=None, stream=None):
        p, mem, k1 = _vec(phi, self.n, "phi")
        q, mem2, k2 = _vec(v, self.n, "v")
        assert mem == mem2
        if out is None:
            out = np.zeros(self.n) if mem == MEM_HOST else v.new_zeros(self.n)
        o, mem3, k3 = _vec(out, self.n, "out")
        assert mem == mem3
        _check(lib().pbfb_apply_jacobian(self.h, scheme, p, q, o, mem, _stream(stream)))
        return out

    def solve(self, phi_out=None, stream=None, check=True, **opts):
        o = default_opts(**opts)
        res = Result()
        ptr, mem = None, MEM_HOST
        if phi_out is not None:
            ptr, mem, keep = _vec(phi_out, 2 * self.n, "phi_out")
        code = lib().pbfb_solve(self.h, C.byref(o), C.byref(res), ptr, mem, _stream(stream))
        if check and code not in (OK,):
            _check(code)
        return res.as_dict()

    def energy(self, phi_lin, phi_nl=None, stream=None):
        a, mem, k1 = _vec(phi_lin, self.n, "phi_lin")
        b = None
        if phi_nl is not None:
            b, mem2, k2 = _vec(phi_nl, self.n, "phi_nl")
            assert mem == mem2
        out = (C.c_double * 4)()
        _check(lib().pbfb_energy(self.h, a, b, out, mem, _stream(stream)))
        return dict(total=out[0], lc=out[1], nc=out[2], dg_omega_i=out[3])

    # ---- inspection -----------------------------------------------------------
    def export_bem(self, surf):
        nv = self.n_m if surf == 0 else self.n_s
        Vp = np.zeros((nv, nv))
        Kp = np.zeros((nv, nv))
        _check(lib().pbfb_export_bem(self.h, surf, Vp.ctypes.data, Kp.ctypes.data))
        return Vp, Kp

    def footprint(self, **opts):
        """(steady, setup) device bytes a server charges for solving this problem."""
        o = default_opts(**opts)
        a, b = C.c_size_t(), C.c_size_t()
        _check(lib().pbfb_request_footprint(self.h, C.byref(o), C.byref(a), C.byref(b)))
        return a.value, b.value

    def export_bem_rows(self, surf, rows):
        """Rows `rows` of the stored blocks (V', K') of surface `surf`."""
        nv = self.n_m if surf == 0 else self.n_s
        rows = np.ascontiguousarray(rows, dtype=np.int64)
        Vp = np.zeros((rows.size, nv))
        Kp = np.zeros((rows.size, nv))
        _check(lib().pbfb_export_bem_rows(self.h, surf, rows.size, rows.ctypes.data, Vp.ctypes.data, Kp.ctypes.data))
        return Vp, Kp

    def export_rhs(self):
        b = np.zeros(self.n)
        _check(lib().pbfb_export_rhs(self.h, b.ctypes.data))
        return b

    def set_bem_mode(self, mode):
        """BEM_DENSE (stored Galerkin blocks) or BEM_MATRIX_FREE (evaluated at every apply)."""
        _check(lib().pbfb_set_bem_mode(self.h, mode))

    def set_two_field(self, n_tets_m):
        """Two-field form: the last n_tets_m tets fill the solute (0: shell-only form)."""
        _check(lib().pbfb_set_two_field(self.h, int(n_tets_m)))

    def set_reaction_surface(self, verts, tris):
        """Two-field form: a Gamma_m surface mesh independent of the volume mesh
        (lambda_m, the reaction potential and the energy on it; the trace of u
        by P1 interpolation at its vertices).  verts = None removes it."""
        if verts is None:
            _check(lib().pbfb_set_reaction_surface(self.h, 0, None, 0, None))
            return
        v = np.ascontiguousarray(np.reshape(verts, (-1, 3)), dtype=np.float64)
        t = np.ascontiguousarray(tris, dtype=np.int32)
        _check(lib().pbfb_set_reaction_surface(self.h, v.shape[0], v.ctypes.data, t.shape[0], t.ctypes.data))

    def set_tile_shape(self, ta=0, tb=0):
        """Pin the regular-assembly tile shape (ta x tb triangles); 0, 0 = tuned."""
        _check(lib().pbfb_set_tile_shape(self.h, ta, tb))

    def tile_shape(self, surf):
        """Tile shape (ta, tb) of the last assembly of surface `surf`."""
        ta, tb = C.c_int(), C.c_int()
        _check(lib().pbfb_get_tile_shape(self.h, surf, C.byref(ta), C.byref(tb)))
        return ta.value, tb.value

    def timing_enable(self, on=True):
        _check(lib().pbfb_timing_enable(self.h, 1 if on else 0))

    def timing(self, which, reset=False):
        ms = C.c_double()
        cnt = C.c_int64()
        _check(lib().pbfb_timing(self.h, which, C.byref(ms), C.byref(cnt), 1 if reset else 0))
        return ms.value, cnt.value
