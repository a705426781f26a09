"""Python binding of the C ABI in include/ibr.h (argument marshalling only).

Every numerical step runs inside ``libibr.so``; this module converts NumPy
arrays to the layouts the ABI documents and raises ``IbrError`` on any status
other than IBR_OK.  There is no fallback: if the library is missing the import
fails loudly.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libibr.so")

FP64, MIXED = 0, 1
PC_LOWER, PC_FULL = 0, 1
WALLS_NONE, WALLS_NOSLIP, WALLS_BOX = 0, 1, 2
ADVECT_CENTRED, ADVECT_SL = 0, 1
MOB_ANALYTIC, MOB_FITTED, MOB_AUTO = 0, 1, 2

STATUS = {0: "IBR_OK", 1: "IBR_EINVAL", 2: "IBR_ENOMEM", 3: "IBR_ENOCONV", 4: "IBR_EBREAKDOWN",
          5: "IBR_EFACTOR", 6: "IBR_ENUMERIC", 7: "IBR_EDEVICE", 8: "IBR_ESTATE"}


class IbrError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__("%s: %s" % (STATUS.get(status, status), msg))
        self.status = status


class Params(ctypes.Structure):
    _fields_ = [("dim", ctypes.c_int), ("n", ctypes.c_int), ("h", ctypes.c_double),
                ("rho", ctypes.c_double), ("eta", ctypes.c_double), ("dt", ctypes.c_double),
                ("precision", ctypes.c_int), ("pc", ctypes.c_int), ("n_s", ctypes.c_int),
                ("restart", ctypes.c_int), ("max_iters", ctypes.c_int), ("rtol", ctypes.c_double),
                ("mg_pre", ctypes.c_int), ("mg_post", ctypes.c_int), ("mg_coarse", ctypes.c_int),
                ("device", ctypes.c_int), ("stream", ctypes.c_void_p), ("graphs", ctypes.c_int),
                ("walls", ctypes.c_int), ("advection", ctypes.c_int), ("mobility", ctypes.c_int)]


class Info(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int), ("restarts", ctypes.c_int), ("ps_applications", ctypes.c_int),
                ("vcycles", ctypes.c_int), ("status", ctypes.c_int), ("rel_residual", ctypes.c_double),
                ("ms", ctypes.c_double), ("max_mobility_shift", ctypes.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


EXPORTS = ["ibr_default_params", "ibr_status_string", "ibr_create", "ibr_destroy", "ibr_last_error",
           "ibr_footprint_bytes", "ibr_set_bodies", "ibr_set_velocities", "ibr_set_rhs", "ibr_solve",
           "ibr_step", "ibr_get_solution", "ibr_get_markers", "ibr_apply_operator", "ibr_spread",
           "ibr_interp", "ibr_vcycle", "ibr_precondition", "ibr_mobility_block", "ibr_advect",
           "ibr_timer_enable", "ibr_timer_read", "ibr_mobility_inverse", "ibr_set_rhs_dev",
           "ibr_get_solution_dev", "ibr_reset", "ibr_set_free_bodies", "ibr_get_velocities",
           "ibr_spread_noalloc", "ibr_set_wall_velocity"]
NOALLOC_SCRATCH_BYTES = 32 << 20


def _devptr(x):
    """Device address of x: None, an int, or an object with data_ptr() (a
    float64 contiguous tensor).  The library checks that it is device memory."""
    if x is None:
        return None
    if isinstance(x, int):
        return x
    if hasattr(x, "data_ptr"):
        if str(getattr(x, "dtype", "torch.float64")) != "torch.float64":
            raise TypeError("device arrays must be float64")
        if hasattr(x, "is_contiguous") and not x.is_contiguous():
            raise ValueError("device arrays must be contiguous")
        return x.data_ptr()
    raise TypeError("expected a device tensor or address, got %r" % type(x))


def load(path=LIB_PATH):
    if not os.path.exists(path):
        raise ImportError("libibr.so not built (run __graft_entry__.build()): %s" % path)
    # torch ships its own HIP runtime under the same soname; loading torch first
    # makes the library bind to that copy, so the process has one runtime and
    # torch's device memory and streams are valid handles for the library
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    lib = ctypes.CDLL(path)
    P = ctypes.POINTER
    d = ctypes.c_double
    vp = ctypes.c_void_p
    dp = P(d)
    ip = P(ctypes.c_int)
    sig = {
        "ibr_default_params": (None, [P(Params)]),
        "ibr_status_string": (ctypes.c_char_p, [ctypes.c_int]),
        "ibr_create": (ctypes.c_int, [P(Params), P(vp)]),
        "ibr_destroy": (None, [vp]),
        "ibr_last_error": (ctypes.c_char_p, [vp]),
        "ibr_footprint_bytes": (ctypes.c_size_t, [P(Params), ctypes.c_int, ctypes.POINTER(ctypes.c_int)]),
        "ibr_set_bodies": (ctypes.c_int, [vp, ctypes.c_int, ip, dp, dp]),
        "ibr_set_velocities": (ctypes.c_int, [vp, dp, dp]),
        "ibr_set_wall_velocity": (ctypes.c_int, [vp, dp, dp]),
        "ibr_set_rhs": (ctypes.c_int, [vp, dp, dp]),
        "ibr_set_rhs_dev": (ctypes.c_int, [vp, vp, vp]),
        "ibr_solve": (ctypes.c_int, [vp, ctypes.c_int, P(Info)]),
        "ibr_step": (ctypes.c_int, [vp, P(Info)]),
        "ibr_reset": (ctypes.c_int, [vp]),
        "ibr_set_free_bodies": (ctypes.c_int, [vp, ip, dp, dp]),
        "ibr_get_velocities": (ctypes.c_int, [vp, dp, dp]),
        "ibr_get_solution": (ctypes.c_int, [vp, dp, dp, dp, dp, dp]),
        "ibr_get_solution_dev": (ctypes.c_int, [vp, vp, vp, vp, vp, vp]),
        "ibr_get_markers": (ctypes.c_int, [vp, dp, dp]),
        "ibr_apply_operator": (ctypes.c_int, [vp, dp, dp]),
        "ibr_spread": (ctypes.c_int, [vp, dp, dp]),
        "ibr_interp": (ctypes.c_int, [vp, dp, dp]),
        "ibr_vcycle": (ctypes.c_int, [vp, d, d, ctypes.c_int, dp, dp]),
        "ibr_precondition": (ctypes.c_int, [vp, dp, dp]),
        "ibr_mobility_block": (ctypes.c_int, [vp, ctypes.c_int, dp, dp]),
        "ibr_advect": (ctypes.c_int, [vp, dp, dp]),
        "ibr_mobility_inverse": (ctypes.c_int, [vp, ctypes.c_int, dp]),
        "ibr_timer_enable": (ctypes.c_int, [ctypes.c_char_p, ctypes.c_int]),
        "ibr_timer_read": (ctypes.c_int, [ctypes.c_char_p, dp, P(ctypes.c_long), dp]),
        "ibr_spread_noalloc": (ctypes.c_int, [P(Params), ctypes.c_int, vp, vp, vp, ctypes.c_char_p,
                                              ctypes.c_size_t]),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    return lib


_LIB = None


def lib():
    global _LIB
    if _LIB is None:
        _LIB = load()
    return _LIB


def _dptr(a):
    if a is None:
        return None
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def default_params(**kw) -> Params:
    p = Params()
    lib().ibr_default_params(ctypes.byref(p))
    for k, v in kw.items():
        if not hasattr(p, k):
            raise KeyError(k)
        setattr(p, k, v)
    return p


@dataclass
class Solution:
    u: np.ndarray
    p: np.ndarray
    lam: np.ndarray
    F: np.ndarray
    T: np.ndarray


class Solver:
    """One ibr_ctx: a grid size with resident buffers, bodies and solution."""

    def __init__(self, **params):
        self._lib = lib()
        self.params = default_params(**params)
        self._ctx = ctypes.c_void_p()
        st = self._lib.ibr_create(ctypes.byref(self.params), ctypes.byref(self._ctx))
        if st != 0:
            raise IbrError(st, "ibr_create failed")
        self.dim = self.params.dim
        self.n = self.params.n
        self.C = self.n ** self.dim
        self.N = 0
        self.nb = 0
        self.nq = 0

    def close(self):
        if self._ctx:
            self._lib.ibr_destroy(self._ctx)
            self._ctx = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def _check(self, st, what):
        if st != 0:
            msg = self._lib.ibr_last_error(self._ctx)
            raise IbrError(st, "%s: %s" % (what, msg.decode() if msg else ""))

    @property
    def NV(self):
        return (self.dim + 1) * self.C + self.dim * self.N + self.nq

    # ------------------------------------------------------------ problem
    def set_bodies(self, R, offsets, centres):
        R = _f64(R).reshape(-1, self.dim)
        off = np.ascontiguousarray(offsets, dtype=np.int32)
        X = _f64(centres).reshape(-1, self.dim)
        nb = len(off) - 1
        self._check(self._lib.ibr_set_bodies(self._ctx, nb, off.ctypes.data_as(ctypes.POINTER(ctypes.c_int)),
                                             _dptr(R), _dptr(X)), "ibr_set_bodies")
        self.N = int(off[-1])
        self.nb = nb
        self.nq = 0
        self._offsets = off.copy()

    def set_free_bodies(self, free=None, F=None, T=None):
        """Bodies with free[p] move under the applied force F[p] and torque
        T[p] (their velocities become unknowns); free=None makes every body
        prescribed again."""
        nr = 3 if self.dim == 3 else 1
        if free is None or not np.any(free):
            self._check(self._lib.ibr_set_free_bodies(self._ctx, None, None, None), "ibr_set_free_bodies")
            self.nq = 0
            return
        fm = np.ascontiguousarray(np.asarray(free) != 0, dtype=np.int32)
        F = _f64(F).reshape(self.nb, self.dim)
        T = _f64(T).reshape(self.nb, nr)
        self._check(self._lib.ibr_set_free_bodies(self._ctx, fm.ctypes.data_as(ctypes.POINTER(ctypes.c_int)),
                                                  _dptr(F), _dptr(T)), "ibr_set_free_bodies")
        self.nq = self.nb * (self.dim + nr)

    def velocities(self):
        """(U [nb, dim], Omega [nb, 1 or 3]): solved for free bodies, prescribed otherwise."""
        U = np.zeros((self.nb, self.dim))
        Om = np.zeros((self.nb, 3 if self.dim == 3 else 1))
        self._check(self._lib.ibr_get_velocities(self._ctx, _dptr(U), _dptr(Om)), "ibr_get_velocities")
        return U, Om

    def set_velocities(self, U, Omega):
        U = _f64(U).reshape(self.nb, self.dim)
        Om = _f64(Omega).reshape(self.nb, 3 if self.dim == 3 else 1)
        self._check(self._lib.ibr_set_velocities(self._ctx, _dptr(U), _dptr(Om)), "ibr_set_velocities")

    def set_wall_velocity(self, lo, hi=None):
        """Walls moving with velocities lo (at coordinate 0 of the last axis)
        and hi (at n h); hi defaults to lo; None puts them back at rest."""
        if lo is None:
            self._check(self._lib.ibr_set_wall_velocity(self._ctx, None, None), "ibr_set_wall_velocity")
            return
        lo = _f64(lo).reshape(self.dim)
        hi = lo if hi is None else _f64(hi).reshape(self.dim)
        self._check(self._lib.ibr_set_wall_velocity(self._ctx, _dptr(lo), _dptr(hi)), "ibr_set_wall_velocity")

    def set_problem(self, prob):
        self.set_bodies(prob.R, prob.offsets, prob.centres)
        self.set_velocities(prob.U, prob.Omega)

    def set_rhs(self, g=None, hp=None):
        g = None if g is None else _f64(g)
        hp = None if hp is None else _f64(hp)
        self._check(self._lib.ibr_set_rhs(self._ctx, _dptr(g), _dptr(hp)), "ibr_set_rhs")

    def set_rhs_dev(self, g=None, hp=None):
        """set_rhs from device arrays: float64 contiguous tensors on the
        context's GPU (anything with data_ptr()), or raw device addresses."""
        self._check(self._lib.ibr_set_rhs_dev(self._ctx, _devptr(g), _devptr(hp)), "ibr_set_rhs_dev")

    def solution_dev(self, u=None, p=None, lam=None, F=None, T=None):
        """Copy the solution into caller-owned device arrays (see set_rhs_dev)."""
        self._check(self._lib.ibr_get_solution_dev(self._ctx, _devptr(u), _devptr(p), _devptr(lam), _devptr(F),
                                                   _devptr(T)), "ibr_get_solution_dev")

    def solve(self, warm_start=False, check=True):
        info = Info()
        st = self._lib.ibr_solve(self._ctx, 1 if warm_start else 0, ctypes.byref(info))
        if check:
            self._check(st, "ibr_solve")
        return info.as_dict()

    def step(self, check=True):
        info = Info()
        st = self._lib.ibr_step(self._ctx, ctypes.byref(info))
        if check:
            self._check(st, "ibr_step")
        return info.as_dict()

    def reset(self):
        """Fluid at rest and no advection history: the next step() starts a new run."""
        self._check(self._lib.ibr_reset(self._ctx), "ibr_reset")

    def solution(self) -> Solution:
        d, n = self.dim, self.n
        u = np.zeros((d,) + (n,) * d)
        p = np.zeros((n,) * d)
        lam = np.zeros((self.N, d))
        F = np.zeros((self.nb, d))
        T = np.zeros((self.nb, 3 if d == 3 else 1))
        self._check(self._lib.ibr_get_solution(self._ctx, _dptr(u), _dptr(p), _dptr(lam), _dptr(F), _dptr(T)),
                    "ibr_get_solution")
        return Solution(u, p, lam, F, T)

    def forces(self):
        """Force F[nb][dim] and torque T[nb][3 or 1] on the bodies (no field copies)."""
        F = np.zeros((self.nb, self.dim))
        T = np.zeros((self.nb, 3 if self.dim == 3 else 1))
        self._check(self._lib.ibr_get_solution(self._ctx, None, None, None, _dptr(F), _dptr(T)),
                    "ibr_get_solution")
        return F, T

    def markers(self):
        R = np.zeros((self.N, self.dim))
        X = np.zeros((self.nb, self.dim))
        self._check(self._lib.ibr_get_markers(self._ctx, _dptr(R), _dptr(X)), "ibr_get_markers")
        return R, X

    # ------------------------------------------------------------ single operators
    def apply_operator(self, x):
        x = _f64(x).reshape(-1)
        y = np.zeros(self.NV)
        self._check(self._lib.ibr_apply_operator(self._ctx, _dptr(x), _dptr(y)), "ibr_apply_operator")
        return y

    def spread(self, lam):
        lam = _f64(lam).reshape(self.N, self.dim)
        f = np.zeros((self.dim,) + (self.n,) * self.dim)
        self._check(self._lib.ibr_spread(self._ctx, _dptr(lam), _dptr(f)), "ibr_spread")
        return f

    def interp(self, u):
        u = _f64(u)
        V = np.zeros((self.N, self.dim))
        self._check(self._lib.ibr_interp(self._ctx, _dptr(u), _dptr(V)), "ibr_interp")
        return V

    def vcycle(self, c0, c1, b):
        b = _f64(b)
        nf = b.shape[0] if b.ndim == self.dim + 1 else 1
        x = np.zeros_like(b)
        self._check(self._lib.ibr_vcycle(self._ctx, float(c0), float(c1), nf, _dptr(b), _dptr(x)), "ibr_vcycle")
        return x

    def precondition(self, r):
        r = _f64(r).reshape(-1)
        z = np.zeros(self.NV)
        self._check(self._lib.ibr_precondition(self._ctx, _dptr(r), _dptr(z)), "ibr_precondition")
        return z

    def mobility_block(self, body):
        off = self._offsets
        nrows = self.dim * (off[body + 1] - off[body])
        M = np.zeros((nrows, nrows))
        sh = ctypes.c_double()
        self._check(self._lib.ibr_mobility_block(self._ctx, body, _dptr(M), ctypes.byref(sh)), "ibr_mobility_block")
        return M, sh.value

    def mobility_inverse(self, body):
        off = self._offsets
        nrows = self.dim * (off[body + 1] - off[body])
        Mi = np.zeros((nrows, nrows))
        self._check(self._lib.ibr_mobility_inverse(self._ctx, body, _dptr(Mi)), "ibr_mobility_inverse")
        return Mi

    def advect(self, u):
        u = _f64(u)
        N = np.zeros_like(u)
        self._check(self._lib.ibr_advect(self._ctx, _dptr(u), _dptr(N)), "ibr_advect")
        return N


TIMERS = ("rb_fine", "ortho_dot", "ortho_axpy", "stokes_apply", "vcycle", "wall_rb_fine", "rb_red_prolong")


def timer_enable(kernel, stride=1):
    """Time every stride-th launch of a kernel class (0 switches the timer off)."""
    st = lib().ibr_timer_enable(kernel.encode(), int(stride))
    if st != 0:
        raise IbrError(st, "unknown timer %r" % kernel)


def timer_read(kernel):
    ms = ctypes.c_double()
    n = ctypes.c_long()
    b = ctypes.c_double()
    st = lib().ibr_timer_read(kernel.encode(), ctypes.byref(ms), ctypes.byref(n), ctypes.byref(b))
    if st != 0:
        raise IbrError(st, "ibr_timer_read(%r)" % kernel)
    return {"ms": ms.value, "launches": n.value, "bytes": b.value}


def spread_noalloc(R, lam, f, nmarkers=None, stream=None, **params):
    """f = S lam without a context or any device allocation (ibr_spread_noalloc):
    R [N, dim], lam [N, dim] and f [dim, n..] are float64 device arrays
    (tensors, or addresses with nmarkers given) on params' device;
    asynchronous on ``stream`` (a torch stream, a raw handle, or None for the
    null stream).  params: dim, n, h, walls, device."""
    p = default_params(**params)
    if stream is not None:
        p.stream = getattr(stream, "cuda_stream", stream)
    nm = nmarkers if nmarkers is not None else (0 if R is None else int(R.shape[0]))
    buf = ctypes.create_string_buffer(512)
    st = lib().ibr_spread_noalloc(ctypes.byref(p), nm, _devptr(R), _devptr(lam), _devptr(f), buf, 512)
    if st != 0:
        raise IbrError(st, "ibr_spread_noalloc: " + buf.value.decode())


def footprint_bytes(markers_per_body, **params):
    """Device bytes a context with these parameters would hold for bodies of
    markers_per_body[b] markers each."""
    counts = np.ascontiguousarray(np.asarray(markers_per_body, dtype=np.int32).ravel())
    p = default_params(**params)
    ptr = counts.ctypes.data_as(ctypes.POINTER(ctypes.c_int)) if counts.size else None
    return int(lib().ibr_footprint_bytes(ctypes.byref(p), int(counts.size), ptr))


def from_problem(prob, **kw):
    """Solver for a synthetic Problem (grid parameters taken from it)."""
    params = dict(dim=prob.dim, n=prob.n, h=prob.h, rho=prob.rho, eta=prob.eta, dt=prob.dt,
                  walls=getattr(prob, "walls", 0))
    if params["walls"]:
        params["n_s"] = 4      # between walls P_S^-1 is a weaker Stokes preconditioner (Sec. 7.1)
    params.update(kw)
    s = Solver(**params)
    s.set_bodies(prob.R, prob.offsets, prob.centres)
    s.set_velocities(prob.U, prob.Omega)
    return s
