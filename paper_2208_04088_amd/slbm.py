"""ctypes binding of libslbm.so (include/slbm.h).  Argument marshalling only:
every step of the method runs in the library's HIP kernels.

The library is loaded from this package directory.  There is no fallback: if
libslbm.so is missing or fails to load, importing the binding raises.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libslbm.so")

SLBM_OK = 0
STATUS = {0: "SLBM_OK", -1: "SLBM_E_INVAL", -2: "SLBM_E_NOMEM", -3: "SLBM_E_DEVICE",
          -4: "SLBM_E_DIVERGED", -5: "SLBM_E_UNSUPPORTED", -6: "SLBM_E_BUDGET"}
FP64, FP32 = 0, 1
PRECISION = {"fp64": FP64, "f64": FP64, "fp32": FP32, "f32": FP32}

EXPORTS = [
    "slbm_create", "slbm_init_fields", "slbm_step", "slbm_sync", "slbm_moments",
    "slbm_displacement", "slbm_displacement_device", "slbm_displacement_device_noalloc", "slbm_moments_device", "slbm_time", "slbm_set_launch", "slbm_set_xcd_group", "slbm_get_launch", "slbm_autotune",
    "slbm_boundary_lists", "slbm_tile_list_layout", "slbm_save", "slbm_load", "slbm_device_bytes", "slbm_destroy", "slbm_copy", "slbm_last_error",
    "slbm_batch_create", "slbm_batch_add", "slbm_batch_step", "slbm_batch_poll", "slbm_batch_handle",
    "slbm_batch_remaining", "slbm_batch_displacement", "slbm_batch_remove", "slbm_batch_set_launch",
    "slbm_batch_set_xcd_group", "slbm_batch_get_launch", "slbm_batch_autotune", "slbm_batch_sync",
    "slbm_batch_wait",
    "slbm_batch_bytes", "slbm_batch_destroy",
]

LINK_DTYPE = np.dtype([("site", "<i4"), ("dir", "<i4"), ("q", "<f8"), ("group", "<i4"),
                       ("group2", "<i4"), ("normal", "<f8", (2,)), ("normal2", "<f8", (2,))],
                      align=True)
GROUP_DTYPE = np.dtype([("kind", "<i4"), ("profile", "<i4"), ("value", "<f8", (2,)),
                        ("ramp_time", "<f8")], align=True)


class SlbmError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{STATUS.get(code, code)}: {msg}")
        self.code = code


class Params(C.Structure):
    _fields_ = [
        ("nx", C.c_int32), ("ny", C.c_int32),
        ("lam", C.c_double), ("mu", C.c_double), ("rho", C.c_double),
        ("tau", C.c_double), ("body_force", C.c_double * 2),
        ("periodic_x", C.c_int32), ("periodic_y", C.c_int32),
        ("precision", C.c_int32), ("neumann_order", C.c_int32),
        ("mask", C.c_void_p),
        ("n_links", C.c_int32), ("links", C.c_void_p),
        ("n_groups", C.c_int32), ("groups", C.c_void_p),
        ("device", C.c_int32), ("stream", C.c_void_p),
    ]


_lib = None


def lib():
    """The loaded libslbm.so (raises if it is not built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"libslbm.so not built at {LIB_PATH}; run `python -m paper_2208_04088_amd.build`")
    L = C.CDLL(LIB_PATH)
    vp, i32, i64, dp = C.c_void_p, C.c_int32, C.c_int64, C.c_void_p
    sig = {
        "slbm_create": [C.POINTER(Params), C.POINTER(vp)],
        "slbm_init_fields": [vp, dp, dp, dp, dp],
        "slbm_step": [vp, i64],
        "slbm_sync": [vp],
        "slbm_moments": [vp, dp, dp, dp, dp],
        "slbm_displacement": [vp, dp],
        "slbm_displacement_device": [vp, vp],
        "slbm_displacement_device_noalloc": [vp, vp],
        "slbm_moments_device": [vp, vp, vp, vp, vp, i32],
        "slbm_time": [vp, C.POINTER(i64), C.POINTER(C.c_double)],
        "slbm_set_launch": [vp, i32, i32],
        "slbm_set_xcd_group": [vp, i32],
        "slbm_get_launch": [vp, C.POINTER(i32), C.POINTER(i32), C.POINTER(i32)],
        "slbm_boundary_lists": [vp, C.POINTER(i32), C.POINTER(C.c_int64), C.POINTER(i32)],
        "slbm_tile_list_layout": [i32, i32, i32, i32, i32, i32, vp, vp, vp, vp, C.c_int64,
                                  C.POINTER(C.c_int64), C.POINTER(C.c_int64), C.POINTER(i32)],
        "slbm_autotune": [vp, C.POINTER(i32), C.POINTER(i32), C.POINTER(C.c_double)],
        "slbm_save": [vp, vp, C.POINTER(C.c_size_t)],
        "slbm_load": [vp, vp, C.c_size_t],
        "slbm_device_bytes": [vp, C.POINTER(i64)],
        "slbm_destroy": [vp],
        "slbm_copy": [vp, vp, C.c_size_t, i32, vp],
        "slbm_batch_create": [i64, i32, vp, C.POINTER(vp)],
        "slbm_batch_add": [vp, C.POINTER(Params), i64, C.POINTER(i32)],
        "slbm_batch_step": [vp, i64],
        "slbm_batch_poll": [vp, C.POINTER(i32), i32, C.POINTER(i32)],
        "slbm_batch_handle": [vp, i32, C.POINTER(vp)],
        "slbm_batch_displacement": [vp, i32, vp],
        "slbm_batch_remaining": [vp, i32, C.POINTER(i64)],
        "slbm_batch_remove": [vp, i32],
        "slbm_batch_set_launch": [vp, i32, i32],
        "slbm_batch_set_xcd_group": [vp, i32],
        "slbm_batch_get_launch": [vp, C.POINTER(i32), C.POINTER(i32), C.POINTER(i32)],
        "slbm_batch_autotune": [vp, i64, C.POINTER(i32), C.POINTER(i32), C.POINTER(i32), C.POINTER(C.c_double)],
        "slbm_batch_sync": [vp],
        "slbm_batch_wait": [vp, i32],
        "slbm_batch_bytes": [vp, C.POINTER(i64), C.POINTER(i64)],
        "slbm_batch_destroy": [vp],
    }
    for name, args in sig.items():
        f = getattr(L, name)
        f.argtypes = args
        f.restype = C.c_int
    L.slbm_last_error.argtypes = []
    L.slbm_last_error.restype = C.c_char_p
    _lib = L
    return L


def _check(rc):
    if rc != SLBM_OK:
        raise SlbmError(rc, lib().slbm_last_error().decode())


def _p(a):
    return None if a is None else a.ctypes.data


def marshal(plate, precision=FP32, device=0, stream=None):
    """slbm_params for a :class:`slbm_workloads.Plate`, plus the arrays it points to."""
    if isinstance(precision, str):
        precision = PRECISION[precision]
    mask = np.ascontiguousarray(plate.mask.ravel(), dtype=np.uint8)
    links = np.zeros(len(plate.links), dtype=LINK_DTYPE)
    for f in LINK_DTYPE.names:
        links[f] = plate.links[f]
    groups = np.zeros(max(len(plate.groups), 1), dtype=GROUP_DTYPE)
    for i, g in enumerate(plate.groups):
        groups[i] = (g.kind, g.profile, g.value, g.ramp_time)
    prm = Params(nx=plate.nx, ny=plate.ny, lam=plate.lam, mu=plate.mu, rho=plate.rho, tau=plate.tau,
                 body_force=(C.c_double * 2)(*plate.force), periodic_x=int(plate.periodic_x),
                 periodic_y=int(plate.periodic_y), precision=int(precision),
                 neumann_order=int(plate.neumann_order), mask=mask.ctypes.data,
                 n_links=len(links), links=links.ctypes.data if len(links) else None,
                 n_groups=len(plate.groups), groups=groups.ctypes.data,
                 device=int(device), stream=stream)
    return prm, (mask, links, groups)


def copy(dst_ptr, src_ptr, nbytes, device=0, stream=None):
    """slbm_copy: plain device copy (the streaming reference)."""
    _check(lib().slbm_copy(C.c_void_p(int(dst_ptr)), C.c_void_p(int(src_ptr)), int(nbytes), int(device),
                           None if stream is None else C.c_void_p(int(stream))))


def tile_list_layout(nx, ny, link_sites, rows, periodic_x=False, periodic_y=False):
    """slbm_tile_list_layout (host only): (tile_start, rec_link, rec_pos,
    most) of the two-step kernel's per-tile cut-link lists."""
    sites = np.ascontiguousarray(link_sites, dtype=np.int32)
    nt, nr, most = C.c_int64(), C.c_int64(), C.c_int32()
    args = (int(nx), int(ny), int(bool(periodic_x)), int(bool(periodic_y)), int(rows), len(sites),
            sites.ctypes.data if len(sites) else None)
    _check(lib().slbm_tile_list_layout(*args, None, None, None, 0, C.byref(nt), C.byref(nr), C.byref(most)))
    start = np.empty(nt.value + 1, dtype=np.int32)
    link = np.empty(max(nr.value, 1), dtype=np.int32)
    pos = np.empty(max(nr.value, 1), dtype=np.int32)
    _check(lib().slbm_tile_list_layout(*args, start.ctypes.data, link.ctypes.data, pos.ctypes.data, nr.value,
                                       C.byref(nt), C.byref(nr), C.byref(most)))
    return start, link[:nr.value], pos[:nr.value], most.value


class Solver:
    """One plate resident on the GPU (slbm_create ... slbm_destroy)."""

    def __init__(self, plate, precision="fp32", device=0, stream=None):
        L = lib()
        self.plate = plate
        prm, keep = marshal(plate, precision, device, stream)
        h = C.c_void_p()
        _check(L.slbm_create(C.byref(prm), C.byref(h)))
        self.h = h
        self.n = plate.nx * plate.ny

    def close(self):
        if getattr(self, "h", None):
            lib().slbm_destroy(self.h)
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
        _check(lib().slbm_init_fields(self.h, *[_p(a) for a in arrs]))

    def step(self, n=1):
        _check(lib().slbm_step(self.h, int(n)))

    def sync(self):
        _check(lib().slbm_sync(self.h))

    def moments(self):
        ny, nx = self.plate.ny, self.plate.nx
        rho = np.empty(self.n)
        j = np.empty(2 * self.n)
        P = np.empty(3 * self.n)
        s = np.empty(3 * self.n)
        _check(lib().slbm_moments(self.h, _p(rho), _p(j), _p(P), _p(s)))
        return rho.reshape(ny, nx), j.reshape(2, ny, nx), P.reshape(3, ny, nx), s.reshape(3, ny, nx)

    def displacement(self):
        u = np.empty(2 * self.n)
        _check(lib().slbm_displacement(self.h, _p(u)))
        return u.reshape(2, self.plate.ny, self.plate.nx)

    def displacement_device(self, ptr):
        """Writes [2][ny][nx] doubles to device pointer ``ptr`` (e.g. a torch
        tensor's data_ptr()) on the handle's stream."""
        _check(lib().slbm_displacement_device(self.h, C.c_void_p(int(ptr))))

    def displacement_device_noalloc(self, ptr):
        """As displacement_device, with no device allocation: the density
        scratch is the library's static per-device array (plates up to
        4096 x 4096; overlapping calls on one device race)."""
        _check(lib().slbm_displacement_device_noalloc(self.h, C.c_void_p(int(ptr))))

    def moments_device(self, rho=0, j=0, P=0, sigma=0, dtype="fp64"):
        """Writes the moments of :meth:`moments` to device pointers (e.g.
        torch tensors' data_ptr(); 0 skips one) as doubles ("fp64") or
        floats ("fp32"), on the handle's stream: rho [n], j [2][n], P [3][n],
        sigma [3][n]."""
        ptrs = [C.c_void_p(int(p)) if p else None for p in (rho, j, P, sigma)]
        _check(lib().slbm_moments_device(self.h, *ptrs, PRECISION[dtype]))

    def time(self):
        st = C.c_int64()
        t = C.c_double()
        _check(lib().slbm_time(self.h, C.byref(st), C.byref(t)))
        return st.value, t.value

    def set_launch(self, seg_rows, strip=0):
        _check(lib().slbm_set_launch(self.h, int(seg_rows), int(strip)))

    def set_xcd_group(self, group):
        """0: contiguous bands of tiles per XCD; g > 0: interleaved groups of g."""
        _check(lib().slbm_set_xcd_group(self.h, int(group)))

    def launch(self):
        """(rows per tile, strip, XCD group) in use."""
        r, st, g = C.c_int32(), C.c_int32(), C.c_int32()
        _check(lib().slbm_get_launch(self.h, C.byref(r), C.byref(st), C.byref(g)))
        return r.value, st.value, g.value

    def boundary_lists(self):
        """slbm_boundary_lists: (rows per tile the per-tile cut-link lists of
        the two-step kernel were built for, 0 if none; records; most in one
        tile)."""
        r, n, m = C.c_int32(), C.c_int64(), C.c_int32()
        _check(lib().slbm_boundary_lists(self.h, C.byref(r), C.byref(n), C.byref(m)))
        return r.value, n.value, m.value

    def autotune(self):
        """Picks the fastest launch shape for this plate; returns
        (rows per tile, strip width, us per step)."""
        seg = C.c_int32()
        strip = C.c_int32()
        us = C.c_double()
        _check(lib().slbm_autotune(self.h, C.byref(seg), C.byref(strip), C.byref(us)))
        return seg.value, strip.value, us.value

    def save(self):
        n = C.c_size_t(0)
        _check(lib().slbm_save(self.h, None, C.byref(n)))
        buf = np.empty(n.value, dtype=np.uint8)
        _check(lib().slbm_save(self.h, buf.ctypes.data, C.byref(n)))
        return buf

    def load(self, buf):
        buf = np.ascontiguousarray(buf, dtype=np.uint8)
        _check(lib().slbm_load(self.h, buf.ctypes.data, buf.size))

    def device_bytes(self):
        b = C.c_int64()
        _check(lib().slbm_device_bytes(self.h, C.byref(b)))
        return b.value


class _BorrowedSolver(Solver):
    """A plate owned by a batch: the single-plate readout calls on its handle
    (the library refuses calls that would step or change it)."""

    def __init__(self, plate, handle):
        self.plate = plate
        self.h = handle
        self.n = plate.nx * plate.ny

    def _owned(self, *args, **kw):
        raise SlbmError(-1, "the plate belongs to a batch: step it with Batch.step")

    step = init_fields = load = autotune = set_launch = set_xcd_group = _owned

    def close(self):
        self.h = None        # the batch frees it


class Batch:
    """Plates advanced together (slbm_batch_*)."""

    def __init__(self, budget_bytes, device=0, stream=None):
        b = C.c_void_p()
        _check(lib().slbm_batch_create(int(budget_bytes), int(device), stream, C.byref(b)))
        self.b = b
        self.plates = {}

    def add(self, plate, nsteps, precision="fp32"):
        prm, keep = marshal(plate, precision)
        slot = C.c_int32()
        _check(lib().slbm_batch_add(self.b, C.byref(prm), int(nsteps), C.byref(slot)))
        self.plates[slot.value] = plate
        return slot.value

    def step(self, k):
        _check(lib().slbm_batch_step(self.b, int(k)))

    def poll(self):
        n = C.c_int32()
        _check(lib().slbm_batch_poll(self.b, None, 0, C.byref(n)))
        buf = (C.c_int32 * max(n.value, 1))()
        _check(lib().slbm_batch_poll(self.b, buf, n.value, C.byref(n)))
        return [buf[i] for i in range(n.value)]

    def solver(self, slot):
        h = C.c_void_p()
        _check(lib().slbm_batch_handle(self.b, int(slot), C.byref(h)))
        return _BorrowedSolver(self.plates[slot], h)

    def displacement(self, slot):
        """The plate's displacement [2, ny, nx] in cells."""
        p = self.plates[slot]
        u = np.empty((2, p.ny, p.nx))
        _check(lib().slbm_batch_displacement(self.b, int(slot), u.ctypes.data_as(C.c_void_p)))
        return u

    def remaining(self, slot):
        r = C.c_int64()
        _check(lib().slbm_batch_remaining(self.b, int(slot), C.byref(r)))
        return r.value

    def remove(self, slot):
        _check(lib().slbm_batch_remove(self.b, int(slot)))
        self.plates.pop(slot, None)

    def set_launch(self, rows, strip):
        _check(lib().slbm_batch_set_launch(self.b, int(rows), int(strip)))

    def set_xcd_group(self, group):
        """0: contiguous bands of tiles per XCD; g > 0: interleaved groups of g."""
        _check(lib().slbm_batch_set_xcd_group(self.b, int(group)))

    def launch(self):
        """(rows per tile, strip, XCD group) of the batched launch."""
        r, st, g = C.c_int32(), C.c_int32(), C.c_int32()
        _check(lib().slbm_batch_get_launch(self.b, C.byref(r), C.byref(st), C.byref(g)))
        return r.value, st.value, g.value

    def autotune(self, max_steps):
        """slbm_batch_autotune: picks the launch shape on the resident plates
        with real steps (at most max_steps); returns (rows, strip, XCD group,
        us per step)."""
        r, st, g, us = C.c_int32(), C.c_int32(), C.c_int32(), C.c_double()
        _check(lib().slbm_batch_autotune(self.b, int(max_steps), C.byref(r), C.byref(st), C.byref(g),
                                         C.byref(us)))
        return r.value, st.value, g.value, us.value

    def sync(self):
        _check(lib().slbm_batch_sync(self.b))

    def wait(self, in_flight):
        """Blocks until at most `in_flight` step calls are still queued or
        running (slbm_batch_wait)."""
        _check(lib().slbm_batch_wait(self.b, int(in_flight)))

    def bytes(self):
        u, t = C.c_int64(), C.c_int64()
        _check(lib().slbm_batch_bytes(self.b, C.byref(u), C.byref(t)))
        return u.value, t.value

    def close(self):
        if getattr(self, "b", None):
            lib().slbm_batch_destroy(self.b)
            self.b = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
