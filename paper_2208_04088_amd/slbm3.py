"""ctypes binding of the three-dimensional step (include/slbm3.h) in
libslbm.so.  Argument marshalling only: every step runs in the library's HIP
kernels; there is no fallback (loading raises if the library is missing).
"""
from __future__ import annotations

import ctypes as C

import numpy as np

from . import slbm as S

EXPORTS = ["slbm3_create", "slbm3_init_fields", "slbm3_step", "slbm3_sync", "slbm3_moments",
           "slbm3_displacement", "slbm3_displacement_device", "slbm3_moments_device", "slbm3_time",
           "slbm3_device_bytes", "slbm3_save", "slbm3_load", "slbm3_destroy"]


class Wall(C.Structure):
    _fields_ = [("kind", C.c_int32), ("value", C.c_double * 3), ("q", C.c_double), ("profile", C.c_int32),
                ("ramp_time", C.c_double)]


class Link(C.Structure):
    _fields_ = [("site", C.c_int32), ("dir", C.c_int32), ("q", C.c_double), ("group", C.c_int32),
                ("normal", C.c_double * 3), ("group2", C.c_int32), ("normal2", C.c_double * 3)]


class BCGroup(C.Structure):
    _fields_ = [("kind", C.c_int32), ("value", C.c_double * 3), ("pressure", C.c_double), ("profile", C.c_int32),
                ("ramp_time", C.c_double)]


class Params3(C.Structure):
    _fields_ = [
        ("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32),
        ("lam", C.c_double), ("mu", C.c_double), ("rho", C.c_double), ("tau", C.c_double),
        ("body_force", C.c_double * 3),
        ("periodic_x", C.c_int32),
        ("walls", Wall * 2),
        ("neumann_order", C.c_int32),
        ("mask", C.c_void_p), ("n_links", C.c_int64), ("links", C.c_void_p),
        ("n_groups", C.c_int32), ("groups", C.c_void_p),
        ("precision", C.c_int32), ("device", C.c_int32), ("stream", C.c_void_p),
    ]


_bound = False


def lib():
    """libslbm.so with the slbm3_* signatures set."""
    global _bound
    L = S.lib()
    if _bound:
        return L
    vp, i64, dp = C.c_void_p, C.c_int64, C.c_void_p
    sig = {
        "slbm3_create": [C.POINTER(Params3), C.POINTER(vp)],
        "slbm3_init_fields": [vp, dp, dp, dp, dp],
        "slbm3_step": [vp, i64],
        "slbm3_sync": [vp],
        "slbm3_moments": [vp, dp, dp, dp, dp],
        "slbm3_displacement": [vp, dp],
        "slbm3_displacement_device": [vp, vp],
        "slbm3_moments_device": [vp, vp, vp, vp, vp, C.c_int32],
        "slbm3_time": [vp, C.POINTER(i64), C.POINTER(C.c_double)],
        "slbm3_device_bytes": [vp, C.POINTER(i64)],
        "slbm3_save": [vp, vp, C.POINTER(C.c_size_t)],
        "slbm3_load": [vp, vp, C.c_size_t],
        "slbm3_destroy": [vp],
    }
    for name, args in sig.items():
        f = getattr(L, name)
        f.argtypes = args
        f.restype = C.c_int
    _bound = True
    return L


LINK_FIELDS = ("site", "dir", "q", "group", "normal", "group2", "normal2")


def marshal(box, precision=S.FP32, device=0, stream=None):
    """(slbm3_params, keep) for a :class:`slbm_workloads.box3d.Box3`; `keep`
    holds the arrays the params point to until slbm3_create has copied them."""
    if isinstance(precision, str):
        precision = S.PRECISION[precision]
    walls = (Wall * 2)()
    for k in range(2):
        walls[k] = Wall(0, (C.c_double * 3)(0.0, 0.0, 0.0), 0.5, 0, 0.0)
    if box.x_walls is not None:
        for k, w in enumerate(box.x_walls):
            walls[k] = Wall(int(w.kind), (C.c_double * 3)(*w.value), float(w.q), int(getattr(w, "profile", 0)),
                            float(getattr(w, "ramp_time", 0.0)))
    prm = Params3(nx=box.nx, ny=box.ny, nz=box.nz, lam=box.lam, mu=box.mu, rho=box.rho, tau=box.tau,
                  body_force=(C.c_double * 3)(*box.force), periodic_x=int(box.x_walls is None),
                  walls=walls, neumann_order=int(box.neumann_order), precision=int(precision),
                  device=int(device), stream=stream)
    keep = []
    if box.mask is not None:
        mask = np.ascontiguousarray(box.mask, dtype=np.uint8)
        if mask.shape != (box.nz, box.ny, box.nx):
            raise ValueError("mask shape must be (nz, ny, nx)")
        links = np.zeros(0 if box.links is None else len(box.links), dtype=Link)
        links["group2"] = -1
        if box.links is not None:
            for f in LINK_FIELDS:
                if f in box.links.dtype.names:
                    links[f] = box.links[f]
        groups = (BCGroup * max(1, len(box.groups or [])))()
        for k, g in enumerate(box.groups or []):
            groups[k] = BCGroup(int(g.kind), (C.c_double * 3)(*g.value), float(getattr(g, "pressure", 0.0)),
                                int(getattr(g, "profile", 0)), float(getattr(g, "ramp_time", 0.0)))
        prm.mask = mask.ctypes.data
        prm.n_links = len(links)
        prm.links = links.ctypes.data if len(links) else None
        prm.n_groups = len(box.groups or [])
        prm.groups = C.cast(groups, C.c_void_p)
        keep = [mask, links, groups]
    return prm, keep


class Solver3:
    """One box resident on the GPU (slbm3_create ... slbm3_destroy)."""

    def __init__(self, box, precision="fp32", device=0, stream=None):
        L = lib()
        self.box = box
        prm, keep = marshal(box, precision, device, stream)
        h = C.c_void_p()
        S._check(L.slbm3_create(C.byref(prm), C.byref(h)))
        del keep
        self.h = h
        self.n = box.nx * box.ny * box.nz
        self.shape = (box.nz, box.ny, box.nx)

    def close(self):
        if getattr(self, "h", None):
            lib().slbm3_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def init_fields(self, rho=None, vel=None, sigma=None, u=None):
        arrs = [None if a is None else np.ascontiguousarray(a, dtype=np.float64).ravel()
                for a in (rho, vel, sigma, u)]
        for a, k in zip(arrs, (1, 3, 6, 3)):
            if a is not None and a.size != k * self.n:
                raise ValueError("field size does not match the box")
        S._check(lib().slbm3_init_fields(self.h, *[S._p(a) for a in arrs]))

    def step(self, n=1):
        S._check(lib().slbm3_step(self.h, int(n)))

    def sync(self):
        S._check(lib().slbm3_sync(self.h))

    def moments(self):
        """(rho [nz,ny,nx], j [3,...], P [6,...], sigma [6,...]) in user units."""
        rho = np.empty(self.n)
        j = np.empty(3 * self.n)
        P = np.empty(6 * self.n)
        s = np.empty(6 * self.n)
        S._check(lib().slbm3_moments(self.h, S._p(rho), S._p(j), S._p(P), S._p(s)))
        return rho.reshape(self.shape), j.reshape((3,) + self.shape), P.reshape((6,) + self.shape), \
            s.reshape((6,) + self.shape)

    def displacement(self):
        u = np.empty(3 * self.n)
        S._check(lib().slbm3_displacement(self.h, S._p(u)))
        return u.reshape((3,) + self.shape)

    def displacement_device(self, ptr):
        """Writes [3][nz][ny][nx] doubles to device pointer ``ptr`` (e.g. a torch
        tensor's data_ptr()) on the handle's stream."""
        S._check(lib().slbm3_displacement_device(self.h, C.c_void_p(int(ptr))))

    def moments_device(self, rho=0, j=0, P=0, sigma=0, dtype="fp64"):
        """The moments of :meth:`moments` into device pointers (0 skips one), as
        doubles ("fp64") or floats ("fp32"), on the handle's stream."""
        ptrs = [C.c_void_p(int(p)) if p else None for p in (rho, j, P, sigma)]
        S._check(lib().slbm3_moments_device(self.h, *ptrs, S.PRECISION[dtype]))

    def time(self):
        st, t = C.c_int64(), C.c_double()
        S._check(lib().slbm3_time(self.h, C.byref(st), C.byref(t)))
        return st.value, t.value

    def device_bytes(self):
        b = C.c_int64()
        S._check(lib().slbm3_device_bytes(self.h, C.byref(b)))
        return b.value

    def save(self):
        """The whole state as a host byte array (slbm3_save)."""
        n = C.c_size_t(0)
        S._check(lib().slbm3_save(self.h, None, C.byref(n)))
        buf = np.empty(n.value, dtype=np.uint8)
        S._check(lib().slbm3_save(self.h, buf.ctypes.data, C.byref(n)))
        return buf

    def load(self, buf):
        """Restores a state from save() on a box of the same shape, geometry
        and precision (slbm3_load)."""
        buf = np.ascontiguousarray(buf, dtype=np.uint8)
        S._check(lib().slbm3_load(self.h, buf.ctypes.data, buf.size))
