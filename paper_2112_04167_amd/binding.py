"""ctypes binding of the SIP-DG C-ABI (include/dg_sipdg.h).

Argument marshalling only: every step of the apply and the solves runs in the
HIP library.  PyTorch supplies device memory and streams.  If the library has
not been built the import fails loudly; there is no CPU fallback.
"""
import atexit
import ctypes
import os
import weakref

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "_lib", "libdgsipdg.so")

DG_OK, DG_NOT_CONVERGED, DG_PENDING = 0, 1, 2
DG_ERR_ARG, DG_ERR_OOM, DG_ERR_DEVICE, DG_ERR_NOT_SPD, DG_ERR_NONFINITE, DG_ERR_BUDGET = \
    -1, -2, -3, -4, -5, -6
DG_BC_PERIODIC, DG_BC_DIRICHLET, DG_BC_NEUMANN = 0, 1, 2
DG_FP64, DG_FP32, DG_MIXED = 0, 1, 1
DG_BATCH_HANDOFF = 1
DG_BATCH_CONCURRENT = 2
DG_PC_JACOBI, DG_PC_FDM = 0, 1

STATUS_NAMES = {0: "OK", 1: "NOT_CONVERGED", 2: "PENDING", -1: "ERR_ARG", -2: "ERR_OOM",
                -3: "ERR_DEVICE", -4: "ERR_NOT_SPD", -5: "ERR_NONFINITE", -6: "ERR_BUDGET"}


class DGError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__("%s (%d): %s" % (STATUS_NAMES.get(status, "?"), status, msg))
        self.status = status


class dg_solve_opts(ctypes.Structure):
    _fields_ = [("tol", ctypes.c_double), ("maxit", ctypes.c_int), ("precision", ctypes.c_int),
                ("inner_tol", ctypes.c_double), ("inner_maxit", ctypes.c_int),
                ("rhs_is_weak", ctypes.c_int), ("fixed_iters", ctypes.c_int),
                ("precond", ctypes.c_int)]


class dg_solve_info(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int), ("outer_iters", ctypes.c_int), ("status", ctypes.c_int),
                ("rel_res", ctypes.c_double), ("true_rel_res", ctypes.c_double),
                ("seconds", ctypes.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class dg_request(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int), ("P", ctypes.c_int), ("is_poisson", ctypes.c_int),
                ("lam", ctypes.c_double), ("rhs", ctypes.POINTER(ctypes.c_double)),
                ("rhs_seed", ctypes.c_uint64), ("tol", ctypes.c_double),
                ("precision", ctypes.c_int), ("keep_result", ctypes.c_int),
                ("precond", ctypes.c_int)]


DG_RK_MAX_STAGES = 8
DG_RK_TR, DG_RK_CB2, DG_RK_CB3C, DG_RK_CB3E, DG_RK_CB4, DG_RK_ARS3 = range(6)
RK_METHODS = {"RK-TR": DG_RK_TR, "RK-CB2": DG_RK_CB2, "RK-CB3c": DG_RK_CB3C, "RK-CB3e": DG_RK_CB3E,
              "RK-CB4": DG_RK_CB4, "RK-ARS3": DG_RK_ARS3}


class dg_tableau(ctypes.Structure):
    _S = DG_RK_MAX_STAGES
    _fields_ = [("s", ctypes.c_int), ("c", ctypes.c_double * _S), ("aI", ctypes.c_double * (_S * _S)),
                ("bI", ctypes.c_double * _S), ("aE", ctypes.c_double * (_S * _S)), ("bE", ctypes.c_double * _S)]


class dg_step_info(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int), ("solves", ctypes.c_int), ("pressure_iters", ctypes.c_int),
                ("velocity_iters", ctypes.c_int), ("seconds", ctypes.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class dg_server_stats(ctypes.Structure):
    _fields_ = [("completed", ctypes.c_int64), ("p50", ctypes.c_double), ("p99", ctypes.c_double),
                ("mean", ctypes.c_double), ("max", ctypes.c_double), ("makespan", ctypes.c_double),
                ("peak_bytes", ctypes.c_double), ("peak_active", ctypes.c_int)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


_lib = None

_VP = ctypes.c_void_p
_SIGS = {
    "dg_last_error": ([], ctypes.c_char_p),
    "dg_default_opts": ([ctypes.POINTER(dg_solve_opts)], None),
    "dg_mesh_create": ([ctypes.c_int] * 4 + [ctypes.POINTER(ctypes.c_double)] * 3 +
                       [ctypes.POINTER(ctypes.c_int), _VP, ctypes.POINTER(_VP)], ctypes.c_int),
    "dg_mesh_destroy": ([_VP], ctypes.c_int),
    "dg_mesh_ndof": ([_VP], ctypes.c_int64),
    "dg_solve_footprint": ([_VP, ctypes.c_int, ctypes.c_int], ctypes.c_size_t),
    "dg_mesh_coordinates": ([_VP, _VP, _VP, _VP, _VP], ctypes.c_int),
    "helmholtz_apply": ([_VP, ctypes.c_double, _VP, ctypes.c_double, _VP, _VP, ctypes.c_int, _VP],
                        ctypes.c_int),
    "helmholtz_fdm_apply": ([_VP, ctypes.c_double, ctypes.c_double, ctypes.c_int, _VP, _VP, _VP],
                            ctypes.c_int),
    "helmholtz_diag": ([_VP, ctypes.c_double, _VP, ctypes.c_double, _VP, ctypes.c_int, _VP],
                       ctypes.c_int),
    "helmholtz_solve": ([_VP, ctypes.c_double, _VP, ctypes.c_double, _VP, _VP,
                         ctypes.POINTER(dg_solve_opts), ctypes.POINTER(dg_solve_info)], ctypes.c_int),
    "helmholtz_solve_noalloc": ([_VP, ctypes.c_double, _VP, ctypes.c_double, _VP, _VP,
                                 ctypes.POINTER(dg_solve_opts), ctypes.POINTER(dg_solve_info)],
                                ctypes.c_int),
    "dg_divergence": ([_VP] * 10, ctypes.c_int),
    "dg_gradient": ([_VP] * 7, ctypes.c_int),
    "dg_project": ([_VP] * 9 + [ctypes.POINTER(dg_solve_opts), ctypes.POINTER(dg_solve_info)],
                   ctypes.c_int),
    "dg_viscosity": ([_VP] * 4 + [ctypes.c_double] * 3 + [_VP, _VP], ctypes.c_int),
    "dg_viscous_terms": ([_VP] * 15, ctypes.c_int),
    "dg_lincomb": ([ctypes.c_int64, _VP, ctypes.c_int, ctypes.POINTER(ctypes.c_double),
                    ctypes.POINTER(_VP), _VP, _VP], ctypes.c_int),
    "poisson_solve": ([_VP, _VP, _VP, ctypes.POINTER(dg_solve_opts), ctypes.POINTER(dg_solve_info)],
                      ctypes.c_int),
    "dg_imex_tableau": ([ctypes.c_int, ctypes.POINTER(dg_tableau)], ctypes.c_int),
    "dg_convection": ([_VP] * 7 + [ctypes.c_double, ctypes.c_int] + [_VP] * 4, ctypes.c_int),
    "dg_viscous_fd2": ([_VP] * 9, ctypes.c_int),
    "dg_imex_step": ([_VP, _VP, ctypes.POINTER(dg_tableau)] + [ctypes.c_double] * 4 + [_VP] * 3 +
                     [ctypes.POINTER(_VP), ctypes.POINTER(_VP), ctypes.c_int, ctypes.POINTER(dg_solve_opts),
                      ctypes.POINTER(dg_step_info)], ctypes.c_int),
    "dg_dirichlet_load": ([_VP, _VP, ctypes.c_double, _VP, ctypes.c_double, _VP, _VP], ctypes.c_int),
    "helmholtz_solve_batched": ([_VP, ctypes.c_int, ctypes.POINTER(ctypes.c_double),
                                 ctypes.POINTER(_VP), ctypes.POINTER(ctypes.c_int),
                                 ctypes.POINTER(_VP), ctypes.POINTER(_VP),
                                 ctypes.POINTER(dg_solve_opts), ctypes.POINTER(dg_solve_info)],
                                ctypes.c_int),
    "helmholtz_solve_batched_ex": ([_VP, ctypes.c_int, ctypes.POINTER(ctypes.c_double),
                                    ctypes.POINTER(_VP), ctypes.POINTER(ctypes.c_int),
                                    ctypes.POINTER(_VP), ctypes.POINTER(_VP),
                                    ctypes.POINTER(dg_solve_opts), ctypes.POINTER(dg_solve_info),
                                    ctypes.c_int], ctypes.c_int),
    "dg_server_create": ([ctypes.c_size_t, ctypes.c_int, ctypes.POINTER(_VP)], ctypes.c_int),
    "dg_server_submit": ([_VP, ctypes.POINTER(dg_request), ctypes.POINTER(ctypes.c_int64)],
                         ctypes.c_int),
    "dg_server_poll": ([_VP, ctypes.c_int64, ctypes.POINTER(dg_solve_info)], ctypes.c_int),
    "dg_server_fetch": ([_VP, ctypes.c_int64, ctypes.POINTER(ctypes.c_double)], ctypes.c_int),
    "dg_server_drain": ([_VP], ctypes.c_int),
    "dg_server_get_stats": ([_VP, ctypes.POINTER(dg_server_stats)], ctypes.c_int),
    "dg_server_destroy": ([_VP], ctypes.c_int),
}


def lib():
    """The loaded C-ABI library (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError("HIP library %s not built: run python -c 'import __graft_entry__ as g; "
                              "g.build()'" % LIB_PATH)
        L = ctypes.CDLL(LIB_PATH)
        for name, (args, res) in _SIGS.items():
            f = getattr(L, name, None)
            if f is None:
                continue
            f.argtypes = args
            f.restype = res
        _lib = L
    return _lib


def exported_symbols():
    return [n for n in _SIGS if hasattr(lib(), n)]


def last_error():
    return lib().dg_last_error().decode()


def _check(rc, allow_warning=False):
    if rc < 0 or (rc > 0 and not allow_warning):
        raise DGError(rc, last_error())
    return rc


def _dptr(t, dtype=None, n=None):
    """Device pointer of a contiguous CUDA tensor (None -> NULL)."""
    if t is None:
        return None
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError("expected a device tensor")
    if not t.is_contiguous():
        raise ValueError("tensor must be contiguous")
    if dtype is not None and t.dtype != dtype:
        raise TypeError("expected dtype %s, got %s" % (dtype, t.dtype))
    if n is not None and t.numel() != n:
        raise ValueError("expected %d values, got %d" % (n, t.numel()))
    return ctypes.c_void_p(t.data_ptr())


def _stream_ptr(stream):
    if stream is None:
        return None
    return ctypes.c_void_p(stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream))


def default_opts(**kw):
    o = dg_solve_opts()
    lib().dg_default_opts(ctypes.byref(o))
    for k, v in kw.items():
        if not hasattr(o, k):
            raise KeyError(k)
        setattr(o, k, v)
    return o


# Meshes and servers still alive when the interpreter exits are destroyed by
# an atexit hook, while the HIP runtime (and any profiler wrapped around it)
# is certainly still up, rather than by __del__ during interpreter teardown,
# whose order relative to the runtime's own exit handlers is not defined.
_live = weakref.WeakSet()


@atexit.register
def _destroy_live():
    for obj in list(_live):
        try:
            obj.destroy()
        except Exception:
            pass


class Mesh:
    """Owner of a dg_mesh handle."""

    def __init__(self, handle, nx, ny, nz, P, bc):
        _live.add(self)
        self.handle = handle
        self.nx, self.ny, self.nz, self.P, self.bc = nx, ny, nz, P, tuple(bc)
        self.ndof = int(lib().dg_mesh_ndof(handle))

    def destroy(self):
        if self.handle:
            lib().dg_mesh_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass

    def footprint(self, precision=DG_FP64, nrhs=1):
        return int(lib().dg_solve_footprint(self.handle, precision, nrhs))


def dg_mesh_create(nx, ny, nz, P, xv, yv, zv, bc, stream=None):
    arrs = [np.ascontiguousarray(v, dtype=np.float64) for v in (xv, yv, zv)]
    for a, n in zip(arrs, (nx, ny, nz)):
        if a.shape != (n + 1,):
            raise ValueError("vertex array must have n+1 entries")
    bca = (ctypes.c_int * 3)(*bc)
    h = ctypes.c_void_p()
    p = [a.ctypes.data_as(ctypes.POINTER(ctypes.c_double)) for a in arrs]
    _check(lib().dg_mesh_create(nx, ny, nz, P, p[0], p[1], p[2], bca, _stream_ptr(stream),
                                ctypes.byref(h)))
    return Mesh(h, nx, ny, nz, P, bc)


def mesh_from_spec(spec, stream=None):
    return dg_mesh_create(spec["nx"], spec["ny"], spec["nz"], spec["P"], spec["xv"], spec["yv"],
                          spec["zv"], spec["bc"], stream)


def mesh_coordinates(mesh, stream=None):
    """(X, Y, Z) nodal coordinates as device tensors (ABI layout)."""
    import torch
    out = [torch.empty(mesh.ndof, dtype=torch.float64, device="cuda") for _ in range(3)]
    _check(lib().dg_mesh_coordinates(mesh.handle, *[_dptr(t) for t in out], _stream_ptr(stream)))
    return out


def _dtype(precision):
    import torch
    return torch.float64 if precision == DG_FP64 else torch.float32


def helmholtz_apply(mesh, lam, nu_field, nu_const, x, y, precision=DG_FP64, stream=None):
    dt = _dtype(precision)
    _check(lib().helmholtz_apply(mesh.handle, float(lam), _dptr(nu_field, dt, mesh.ndof),
                                 float(nu_const), _dptr(x, dt, mesh.ndof), _dptr(y, dt, mesh.ndof),
                                 precision, _stream_ptr(stream)))


def helmholtz_fdm_apply(mesh, lam, nu_const, b, x, is_poisson=False, stream=None):
    """x = A^-1 b for a constant nu by fast diagonalisation (b: weak load)."""
    import torch
    _check(lib().helmholtz_fdm_apply(mesh.handle, float(lam), float(nu_const), int(is_poisson),
                                     _dptr(b, torch.float64, mesh.ndof), _dptr(x, torch.float64, mesh.ndof),
                                     _stream_ptr(stream)))


def helmholtz_diag(mesh, lam, nu_field, nu_const, d, precision=DG_FP64, stream=None):
    dt = _dtype(precision)
    _check(lib().helmholtz_diag(mesh.handle, float(lam), _dptr(nu_field, dt, mesh.ndof),
                                float(nu_const), _dptr(d, dt, mesh.ndof), precision,
                                _stream_ptr(stream)))


def helmholtz_solve(mesh, lam, nu_field, nu_const, rhs, x, opts=None, raise_on_error=True):
    import torch
    info = dg_solve_info()
    rc = lib().helmholtz_solve(mesh.handle, float(lam), _dptr(nu_field, torch.float64, mesh.ndof),
                               float(nu_const), _dptr(rhs, torch.float64, mesh.ndof),
                               _dptr(x, torch.float64, mesh.ndof),
                               ctypes.byref(opts) if opts is not None else None, ctypes.byref(info))
    if raise_on_error:
        _check(rc, allow_warning=True)
    d = info.as_dict()
    d["rc"] = rc
    return d


def helmholtz_solve_noalloc(mesh, lam, nu_field, nu_const, rhs, x, opts=None,
                            raise_on_error=True):
    """helmholtz_solve (FP64) with its workspace in the library's static
    device scratch array: allocates no device memory."""
    import torch
    info = dg_solve_info()
    rc = lib().helmholtz_solve_noalloc(mesh.handle, float(lam),
                                       _dptr(nu_field, torch.float64, mesh.ndof), float(nu_const),
                                       _dptr(rhs, torch.float64, mesh.ndof),
                                       _dptr(x, torch.float64, mesh.ndof),
                                       ctypes.byref(opts) if opts is not None else None,
                                       ctypes.byref(info))
    if raise_on_error:
        _check(rc, allow_warning=True)
    d = info.as_dict()
    d["rc"] = rc
    return d


def dg_divergence(mv, mp, v, b, vb=None, stream=None):
    """b = D(v; v_b) on the pressure mesh mp (degree P-1): weak divergence."""
    import torch
    vv = [_dptr(c, torch.float64, mv.ndof) for c in v]
    bb = [None, None, None] if vb is None else [_dptr(c, torch.float64, mv.ndof) for c in vb]
    _check(lib().dg_divergence(mv.handle, mp.handle, *vv, *bb, _dptr(b, torch.float64, mp.ndof),
                               _stream_ptr(stream)))


def dg_gradient(mv, mp, psi, g, stream=None):
    """g = G psi at the velocity nodes (three tensors)."""
    import torch
    _check(lib().dg_gradient(mv.handle, mp.handle, _dptr(psi, torch.float64, mp.ndof),
                             *[_dptr(c, torch.float64, mv.ndof) for c in g], _stream_ptr(stream)))


def dg_project(mv, mp, v, psi, vb=None, opts=None, raise_on_error=True):
    """The projection substep: v <- v - G psi with psi the pressure (in: guess)."""
    import torch
    info = dg_solve_info()
    vv = [_dptr(c, torch.float64, mv.ndof) for c in v]
    bb = [None, None, None] if vb is None else [_dptr(c, torch.float64, mv.ndof) for c in vb]
    rc = lib().dg_project(mv.handle, mp.handle, *vv, *bb, _dptr(psi, torch.float64, mp.ndof),
                          ctypes.byref(opts) if opts is not None else None, ctypes.byref(info))
    if raise_on_error:
        _check(rc, allow_warning=True)
    d = info.as_dict()
    d["rc"] = rc
    return d


def dg_viscosity(mesh, v, nu0, nu1, vref, nu, stream=None):
    """nu = nu0 + nu1 (|v|/vref)^2 at every node."""
    import torch
    _check(lib().dg_viscosity(mesh.handle, *[_dptr(c, torch.float64, mesh.ndof) for c in v], float(nu0),
                              float(nu1), float(vref), _dptr(nu, torch.float64, mesh.ndof),
                              _stream_ptr(stream)))


def dg_viscous_terms(mesh, nu, v, fd1=None, fd3=None, vb=None, stream=None):
    """F_d1 = div(nu grad v) and F_d3 = -grad(nu div v) into the given tensors."""
    import torch
    p = lambda t: _dptr(t, torch.float64, mesh.ndof)
    trip = lambda ts: [None] * 3 if ts is None else [p(t) for t in ts]
    _check(lib().dg_viscous_terms(mesh.handle, p(nu), *[p(c) for c in v], *trip(vb), *trip(fd1), *trip(fd3),
                                  _stream_ptr(stream)))


def dg_lincomb(y, x0, coefs, xs, stream=None):
    """y = x0 + sum coef_j xs_j (device tensors of equal length; x0 may be None)."""
    n = y.numel()
    k = len(xs)
    c = (ctypes.c_double * max(k, 1))(*[float(v) for v in coefs])
    pp = (ctypes.c_void_p * max(k, 1))(*[_dptr(t, None, n) for t in xs])
    _check(lib().dg_lincomb(n, _dptr(x0, None, n) if x0 is not None else None, k, c, pp, _dptr(y, None, n),
                            _stream_ptr(stream)))


def imex_tableau(method):
    """The App. A tableau `method` (DG_RK_* or its name, e.g. "RK-ARS3")."""
    if isinstance(method, str):
        method = RK_METHODS[method]
    t = dg_tableau()
    _check(lib().dg_imex_tableau(int(method), ctypes.byref(t)))
    return t


def dg_convection(mesh, v, out, vb=None, scale=1.0, accumulate=False, stream=None):
    """out = scale F_c(v) (or += with accumulate): -div(v v), LLF fluxes."""
    import torch
    p = lambda t: _dptr(t, torch.float64, mesh.ndof)
    bb = [None] * 3 if vb is None else [p(c) for c in vb]
    _check(lib().dg_convection(mesh.handle, *[p(c) for c in v], *bb, float(scale), int(bool(accumulate)),
                               *[p(c) for c in out], _stream_ptr(stream)))


def dg_viscous_fd2(mesh, nu, v, out, stream=None):
    """out = F_d2(v) = div(nu (grad v)^T) with the nodal viscosity nu."""
    import torch
    p = lambda t: _dptr(t, torch.float64, mesh.ndof)
    _check(lib().dg_viscous_fd2(mesh.handle, p(nu), *[p(c) for c in v], *[p(c) for c in out],
                                _stream_ptr(stream)))


def dg_dirichlet_load(mesh, nu, g, b, nu_const=1.0, scale=1.0, stream=None):
    """b += scale L(g): the Nitsche load of Dirichlet data g (nodal field)."""
    import torch
    p = lambda t: _dptr(t, torch.float64, mesh.ndof)
    _check(lib().dg_dirichlet_load(mesh.handle, p(nu) if nu is not None else None, float(nu_const), p(g),
                                   float(scale), p(b), _stream_ptr(stream)))


def dg_imex_step(mv, mp, tableau, dt, nu0, nu1, vref, v, forcing=None, final_projection=False, opts=None,
                 raise_on_error=True, wall=None):
    """One IMEX-RK step (Alg. 3) in place on the three velocity tensors v.
    tableau: a dg_tableau or a method (see imex_tableau); forcing, wall: None
    or a list over the stages of three tensors (or None) each (the forcing
    and the wall velocity at t + c_j dt)."""
    import torch
    tab = tableau if isinstance(tableau, dg_tableau) else imex_tableau(tableau)

    def per_stage(fields):
        if fields is None:
            return None
        flat = []
        for j in range(tab.s):
            fj = fields[j] if j < len(fields) else None
            for d in range(3):
                flat.append(None if fj is None or fj[d] is None else _dptr(fj[d], torch.float64, mv.ndof))
        return (ctypes.c_void_p * len(flat))(*flat)

    fp, wp = per_stage(forcing), per_stage(wall)
    info = dg_step_info()
    rc = lib().dg_imex_step(mv.handle, mp.handle, ctypes.byref(tab), float(dt), float(nu0), float(nu1),
                            float(vref), *[_dptr(c, torch.float64, mv.ndof) for c in v], fp, wp,
                            int(bool(final_projection)), ctypes.byref(opts) if opts is not None else None,
                            ctypes.byref(info))
    if raise_on_error:
        _check(rc, allow_warning=True)
    d = info.as_dict()
    d["rc"] = rc
    return d


def poisson_solve(mesh, rhs, x, opts=None, raise_on_error=True):
    import torch
    info = dg_solve_info()
    rc = lib().poisson_solve(mesh.handle, _dptr(rhs, torch.float64, mesh.ndof),
                             _dptr(x, torch.float64, mesh.ndof),
                             ctypes.byref(opts) if opts is not None else None, ctypes.byref(info))
    if raise_on_error:
        _check(rc, allow_warning=True)
    d = info.as_dict()
    d["rc"] = rc
    return d


def helmholtz_solve_batched(mesh, lambdas, nu_fields, is_poisson, rhs, xs, opts=None,
                            raise_on_error=True, handoff=False, concurrent=False):
    import torch
    n = len(rhs)
    lam = (ctypes.c_double * n)(*[float(v) for v in lambdas])
    nus = (ctypes.c_void_p * n)(*[_dptr(v, torch.float64, mesh.ndof) if v is not None else None
                                  for v in nu_fields])
    pois = (ctypes.c_int * n)(*[int(v) for v in is_poisson])
    rr = (ctypes.c_void_p * n)(*[_dptr(v, torch.float64, mesh.ndof) for v in rhs])
    xx = (ctypes.c_void_p * n)(*[_dptr(v, torch.float64, mesh.ndof) for v in xs])
    infos = (dg_solve_info * n)()
    rc = lib().helmholtz_solve_batched_ex(mesh.handle, n, lam, nus, pois, rr, xx,
                                          ctypes.byref(opts) if opts is not None else None, infos,
                                          (DG_BATCH_HANDOFF if handoff else 0) |
                                          (DG_BATCH_CONCURRENT if concurrent else 0))
    if raise_on_error:
        _check(rc, allow_warning=True)
    return rc, [i.as_dict() for i in infos]


class Server:
    """Continuous-batching request server (dg_server_*)."""

    def __init__(self, hbm_budget_bytes, max_slots):
        h = ctypes.c_void_p()
        _check(lib().dg_server_create(int(hbm_budget_bytes), int(max_slots), ctypes.byref(h)))
        _live.add(self)
        self.handle = h
        self._keep = {}

    def submit(self, n, P, lam, rhs_host=None, is_poisson=False, tol=1e-10, precision=DG_FP64,
               rhs_seed=0, keep_result=False, precond=DG_PC_JACOBI):
        """Queue one solve; rhs_host None -> f generated on the device from rhs_seed."""
        req = dg_request(n=n, P=P, is_poisson=int(is_poisson), lam=float(lam), rhs_seed=int(rhs_seed),
                         tol=tol, precision=precision, keep_result=int(keep_result),
                         precond=int(precond))
        if rhs_host is not None:
            rhs = np.ascontiguousarray(rhs_host, dtype=np.float64)
            if rhs.size != n ** 3 * (P + 1) ** 3:
                raise ValueError("rhs has the wrong size")
            req.rhs = rhs.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        rid = ctypes.c_int64()
        _check(lib().dg_server_submit(self.handle, ctypes.byref(req), ctypes.byref(rid)))
        return rid.value

    def poll(self, rid):
        info = dg_solve_info()
        rc = lib().dg_server_poll(self.handle, rid, ctypes.byref(info))
        if rc < 0:
            raise DGError(rc, last_error())
        return rc, info.as_dict()

    def fetch(self, rid, ndof):
        out = np.empty(ndof)
        _check(lib().dg_server_fetch(self.handle, rid,
                                     out.ctypes.data_as(ctypes.POINTER(ctypes.c_double))))
        return out

    def drain(self):
        _check(lib().dg_server_drain(self.handle))

    def stats(self):
        st = dg_server_stats()
        _check(lib().dg_server_get_stats(self.handle, ctypes.byref(st)))
        return st.as_dict()

    def destroy(self):
        if self.handle:
            lib().dg_server_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass
