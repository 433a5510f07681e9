"""ctypes binding of the plain CPU reference (TEST INFRASTRUCTURE).

Only the test suite, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` import this package.  It loads ``liboracle_f64.so`` (double) or
``liboracle_f80.so`` (x87 long double), built from ``slbm_oracle.c`` by
``oracle/build.py``.  See ``slbm_oracle.h`` for the method and its
citations.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))

_D = C.POINTER(C.c_double)
_I = C.POINTER(C.c_int32)
_U8 = C.POINTER(C.c_uint8)

DIRICHLET = 1
NEUMANN = 2


class _Problem(C.Structure):
    _fields_ = [
        ("nx", C.c_int32), ("ny", C.c_int32),
        ("lam", C.c_double), ("mu", C.c_double), ("rho", C.c_double),
        ("tau", C.c_double), ("force", C.c_double * 2),
        ("periodic_x", C.c_int32), ("periodic_y", C.c_int32),
        ("neumann_order", C.c_int32),
        ("mask", _U8),
        ("n_links", C.c_int32),
        ("link_site", _I), ("link_dir", _I), ("link_q", _D),
        ("link_group", _I), ("link_group2", _I),
        ("link_normal", _D), ("link_normal2", _D),
        ("n_groups", C.c_int32),
        ("group_kind", _I), ("group_value", _D), ("group_profile", _I),
        ("group_ramp_time", _D),
    ]


_libs = {}


def _lib(extended: bool):
    name = "liboracle_f80.so" if extended else "liboracle_f64.so"
    if name in _libs:
        return _libs[name]
    path = os.path.join(HERE, name)
    if not os.path.exists(path):
        from . import build as _b
        _b.build()
    L = C.CDLL(path)
    L.oracle_create.restype = C.c_void_p
    L.oracle_create.argtypes = [C.POINTER(_Problem), C.c_char_p, C.c_int]
    L.oracle_destroy.argtypes = [C.c_void_p]
    L.oracle_init_fields.argtypes = [C.c_void_p, _D, _D, _D, _D]
    L.oracle_init_fields.restype = C.c_int
    L.oracle_step.argtypes = [C.c_void_p, C.c_int64]
    L.oracle_step_count.argtypes = [C.c_void_p]
    L.oracle_step_count.restype = C.c_int64
    L.oracle_moments.argtypes = [C.c_void_p, _D, _D, _D, _D]
    L.oracle_displacement.argtypes = [C.c_void_p, _D]
    L.oracle_get_populations.argtypes = [C.c_void_p, _D]
    L.oracle_set_populations.argtypes = [C.c_void_p, _D]
    L.oracle_lattice_params.argtypes = [C.c_void_p, _D]
    L.oracle_equilibrium.argtypes = [C.c_double, _D, _D, _D]
    L.oracle_set_threads.argtypes = [C.c_int]
    L.oracle_set_threads.restype = C.c_int
    _libs[name] = L
    return L


def _ptr(a, t):
    return a.ctypes.data_as(t) if a is not None else None


class Oracle:
    """One plate advanced by the CPU reference.  ``plate`` is a
    :class:`slbm_workloads.Plate`."""

    def __init__(self, plate, extended: bool = False):
        self.L = _lib(extended)
        self.plate = plate
        p = plate
        L = p.links
        self._keep = dict(
            mask=np.ascontiguousarray(p.mask.ravel(), dtype=np.uint8),
            site=np.ascontiguousarray(L["site"], dtype=np.int32),
            dir=np.ascontiguousarray(L["dir"], dtype=np.int32),
            q=np.ascontiguousarray(L["q"], dtype=np.float64),
            g1=np.ascontiguousarray(L["group"], dtype=np.int32),
            g2=np.ascontiguousarray(L["group2"], dtype=np.int32),
            n1=np.ascontiguousarray(L["normal"], dtype=np.float64),
            n2=np.ascontiguousarray(L["normal2"], dtype=np.float64),
            gk=np.array([g.kind for g in p.groups] or [0], dtype=np.int32),
            gv=np.array([g.value for g in p.groups] or [(0.0, 0.0)], dtype=np.float64),
            gp=np.array([g.profile for g in p.groups] or [0], dtype=np.int32),
            gr=np.array([g.ramp_time for g in p.groups] or [0.0], dtype=np.float64),
        )
        k = self._keep
        prob = _Problem(
            nx=p.nx, ny=p.ny, lam=p.lam, mu=p.mu, rho=p.rho, tau=p.tau,
            force=(C.c_double * 2)(*p.force),
            periodic_x=int(p.periodic_x), periodic_y=int(p.periodic_y),
            neumann_order=int(p.neumann_order),
            mask=_ptr(k["mask"], _U8), n_links=len(L),
            link_site=_ptr(k["site"], _I), link_dir=_ptr(k["dir"], _I), link_q=_ptr(k["q"], _D),
            link_group=_ptr(k["g1"], _I), link_group2=_ptr(k["g2"], _I),
            link_normal=_ptr(k["n1"], _D), link_normal2=_ptr(k["n2"], _D),
            n_groups=len(p.groups), group_kind=_ptr(k["gk"], _I), group_value=_ptr(k["gv"], _D),
            group_profile=_ptr(k["gp"], _I), group_ramp_time=_ptr(k["gr"], _D))
        err = C.create_string_buffer(512)
        h = self.L.oracle_create(C.byref(prob), err, 512)
        if not h:
            raise ValueError("oracle: " + err.value.decode())
        self.h = h
        self.n = p.nx * p.ny

    def __del__(self):
        h = getattr(self, "h", None)
        if h:
            self.L.oracle_destroy(h)
            self.h = None

    def init_fields(self, rho=None, vel=None, sigma=None, u=None):
        arrs = [None if a is None else np.ascontiguousarray(a, dtype=np.float64).ravel()
                for a in (rho, vel, sigma, u)]
        rc = self.L.oracle_init_fields(self.h, *[_ptr(a, _D) for a in arrs])
        if rc != 0:
            raise ValueError("oracle: bad initial fields")

    def step(self, n=1):
        self.L.oracle_step(self.h, int(n))

    @property
    def step_count(self):
        return int(self.L.oracle_step_count(self.h))

    def moments(self):
        """(rho [ny,nx], j [2,ny,nx], P [3,ny,nx], sigma [3,ny,nx]) in user units."""
        ny, nx = self.plate.ny, self.plate.nx
        rho = np.empty(self.n)
        j = np.empty(2 * self.n)
        P = np.empty(3 * self.n)
        s = np.empty(3 * self.n)
        self.L.oracle_moments(self.h, _ptr(rho, _D), _ptr(j, _D), _ptr(P, _D), _ptr(s, _D))
        return rho.reshape(ny, nx), j.reshape(2, ny, nx), P.reshape(3, ny, nx), s.reshape(3, ny, nx)

    def displacement(self):
        u = np.empty(2 * self.n)
        self.L.oracle_displacement(self.h, _ptr(u, _D))
        return u.reshape(2, self.plate.ny, self.plate.nx)

    def populations(self):
        f = np.empty(9 * self.n)
        self.L.oracle_get_populations(self.h, _ptr(f, _D))
        return f.reshape(9, self.plate.ny, self.plate.nx)

    def set_populations(self, f):
        f = np.ascontiguousarray(f, dtype=np.float64).ravel()
        assert f.size == 9 * self.n
        self.L.oracle_set_populations(self.h, _ptr(f, _D))

    def lattice_params(self):
        out = np.empty(6)
        self.L.oracle_lattice_params(self.h, _ptr(out, _D))
        return dict(lam=out[0], mu=out[1], tau=out[2], dt_user=out[3], s_sigma=out[4], s_v=out[5])


def equilibrium(rho, j, P, extended=False):
    """eq:fieq in lattice units: P = (xx, yy, xy)."""
    L = _lib(extended)
    j = np.ascontiguousarray(j, dtype=np.float64)
    P = np.ascontiguousarray(P, dtype=np.float64)
    out = np.empty(9)
    L.oracle_equilibrium(float(rho), _ptr(j, _D), _ptr(P, _D), _ptr(out, _D))
    return out


def set_threads(n, extended=False):
    """OpenMP threads of later reference calls (0: the runtime default);
    returns the number in effect."""
    return _lib(extended).oracle_set_threads(int(n))
