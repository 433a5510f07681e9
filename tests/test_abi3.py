"""The three-dimensional C ABI without a GPU: libslbm.so exports every
function include/slbm3.h declares, slbm3_params has the header's layout,
invalid boxes are rejected on the host, and a valid one fails loudly when no
device is present."""
import ctypes as C
import os
import re
import subprocess

import numpy as np
import pytest

from paper_2208_04088_amd import slbm as S
from paper_2208_04088_amd import slbm3 as S3
from slbm_workloads import box3d as B

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "slbm3.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(slbm3_[a-z_]+)\s*\(", text)))


def test_library_exports_every_declared_function():
    L = S3.lib()
    names = declared_functions()
    assert len(names) == 13
    missing = [n for n in names if not hasattr(L, n)]
    assert not missing, missing
    assert sorted(S3.EXPORTS) == names


def test_struct_layout_matches_header(tmp_path):
    src = tmp_path / "layout3.c"
    cname = {"lam": "lambda", "tau": "tau_bar"}
    lines = ["#include <stdio.h>", "#include <stddef.h>", '#include "slbm3.h"', "int main(void){",
             'printf("slbm3_params %zu\\n", sizeof(slbm3_params));',
             'printf("slbm3_wall %zu\\n", sizeof(slbm3_wall));',
             'printf("slbm3_wall.value %zu\\n", offsetof(slbm3_wall, value));',
             'printf("slbm3_link %zu\\n", sizeof(slbm3_link));',
             'printf("slbm3_bc_group %zu\\n", sizeof(slbm3_bc_group));']
    for f, _ in S3.Link._fields_:
        lines.append(f'printf("slbm3_link.{f} %zu\\n", offsetof(slbm3_link, {f}));')
    for f, _ in S3.BCGroup._fields_:
        lines.append(f'printf("slbm3_bc_group.{f} %zu\\n", offsetof(slbm3_bc_group, {f}));')
    for f, _ in S3.Params3._fields_:
        lines.append(f'printf("slbm3_params.{f} %zu\\n", offsetof(slbm3_params, {cname.get(f, f)}));')
    lines.append("return 0;}")
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout3"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    out = dict(l.rsplit(" ", 1) for l in subprocess.run([str(exe)], capture_output=True, text=True,
                                                         check=True).stdout.split("\n") if l)
    assert int(out["slbm3_params"]) == C.sizeof(S3.Params3)
    assert int(out["slbm3_wall"]) == C.sizeof(S3.Wall)
    assert int(out["slbm3_wall.value"]) == S3.Wall.value.offset
    for f, _ in S3.Params3._fields_:
        assert int(out[f"slbm3_params.{f}"]) == getattr(S3.Params3, f).offset, f
    # the link records are the workloads' LINK3_DTYPE, byte for byte
    assert int(out["slbm3_link"]) == C.sizeof(S3.Link) == B.LINK3_DTYPE.itemsize == 80
    for f, _ in S3.Link._fields_:
        assert int(out[f"slbm3_link.{f}"]) == getattr(S3.Link, f).offset == B.LINK3_DTYPE.fields[f][1], f
    assert int(out["slbm3_bc_group"]) == C.sizeof(S3.BCGroup)
    for f, _ in S3.BCGroup._fields_:
        assert int(out[f"slbm3_bc_group.{f}"]) == getattr(S3.BCGroup, f).offset, f


def _create(box, **over):
    prm, keep = S3.marshal(box, "fp32")
    for k, v in over.items():
        setattr(prm, k, v)
    h = C.c_void_p()
    L = S3.lib()
    rc = L.slbm3_create(C.byref(prm), C.byref(h))
    if rc == 0:
        L.slbm3_destroy(h)
    return rc, L.slbm_last_error().decode()


def _slab():
    return B.slab3(8, 4, 3, B.Wall3(B.DIRICHLET), B.Wall3(B.NEUMANN, (1e-5, 0.0, 0.0)))


@pytest.mark.parametrize("case", ["nx", "nz", "tau", "mu", "rho", "lambda", "precision", "wall_kind"])
def test_invalid_boxes_are_rejected_on_the_host(case):
    over = {"nx": dict(nx=0), "nz": dict(nz=-2), "tau": dict(tau=0.5), "mu": dict(mu=0.0),
            "rho": dict(rho=-1.0), "lambda": dict(lam=-0.06), "precision": dict(precision=5)}.get(case, {})
    box = _slab()
    if case == "wall_kind":
        box.x_walls = (B.Wall3(3), box.x_walls[1])
    rc, msg = _create(box, **over)
    assert rc == -1, (rc, msg)
    assert msg


def test_too_large_a_box_is_unsupported():
    """At most 2^29 sites: one more plane of 1024 x 1024 is refused on the
    host (a box of exactly 2^29 sites is run by the GPU tests)."""
    rc, msg = _create(B.periodic_box3(1024, 1024, 513))
    assert rc == -5, (rc, msg)


def test_valid_box_without_a_gpu_fails_loudly():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    rc, msg = _create(_slab())
    assert rc == -3, (rc, msg)


def test_device_outputs_reject_a_null_handle():
    L = S3.lib()
    assert L.slbm3_displacement_device(None, None) == -1
    assert L.slbm3_moments_device(None, None, None, None, None, 0) == -1
    n = C.c_size_t(0)
    assert L.slbm3_save(None, None, C.byref(n)) == -1
    assert L.slbm3_load(None, None, 0) == -1


def _cavity():
    groups = [B.BCGroup3(B.NEUMANN, (0.0, 0.0, 0.0), 1e-4), B.BCGroup3(B.DIRICHLET)]
    return B.sphere_box3(12, 11, 10, [B.Sphere3(5.6, 5.3, 4.8, 2.3, 0)], groups)


def _set(box, field, i, value):
    links = box.links.copy()
    links[field][i] = value
    box.links = links


@pytest.mark.parametrize("case", ["site_range", "dir", "void_start", "material_end", "q0", "q_big", "group",
                                  "normal", "twice", "missing", "group_kind", "walls", "no_mask"])
def test_invalid_cut_links_are_rejected_on_the_host(case):
    """Every check slbm3_create documents for a general geometry, one at a
    time, on a valid cavity: the call fails with SLBM_E_INVAL and a message
    before any device work."""
    box = _cavity()
    over = {}
    void = int(np.flatnonzero(box.mask.ravel() == 0)[0])
    if case == "site_range":
        _set(box, "site", 3, box.n_sites)
    elif case == "dir":
        _set(box, "dir", 0, 19)
    elif case == "void_start":
        _set(box, "site", 0, void)
    elif case == "material_end":
        # the opposite direction from the same site ends in the material,
        # whose link back is not listed (a crack with one face)
        d = int(box.links["dir"][0])
        _set(box, "dir", 0, d + 1 if d % 2 else d - 1)
    elif case == "q0":
        _set(box, "q", 2, 0.0)
    elif case == "q_big":
        _set(box, "q", 2, 1.5)
    elif case == "group":
        _set(box, "group", 1, 2)
    elif case == "normal":
        _set(box, "normal", 4, (1.0, 1e-3, 0.0))
    elif case == "twice":
        box.links = np.concatenate([box.links, box.links[:1]])
    elif case == "missing":
        box.links = box.links[1:]
    elif case == "group_kind":
        box.groups[1] = B.BCGroup3(7)
    elif case == "walls":
        over = dict(periodic_x=0)
    elif case == "no_mask":
        over = dict(mask=None)
    rc, msg = _create(box, **over)
    assert rc == -1, (case, rc, msg)
    assert msg


def _cracked():
    groups = [B.BCGroup3(B.NEUMANN), B.BCGroup3(B.NEUMANN, (1e-5, 0.0, 0.0))]
    return B.sphere_box3(12, 11, 10, [B.Sphere3(3.6, 5.3, 4.8, 2.1, 0)], groups,
                         cracks=[B.PennyCrack3(8.2, 5.1, 4.5, 2.4, 0, 1)])


def test_one_sided_crack_is_rejected_on_the_host():
    box = _cracked()
    box.links = box.links[box.links["group"] != 1]    # the crack's upper face missing
    rc, msg = _create(box)
    assert rc == -1 and "link back" in msg, (rc, msg)


def _block():
    return B.block_box3(9, 8, 7, (2, 2, 2), (6, 5, 4), list(range(6)),
                        [B.BCGroup3(B.NEUMANN)] * 3 + [B.BCGroup3(B.DIRICHLET)] * 3)


@pytest.mark.parametrize("case", ["group2_range", "normal2_unit", "normal2_skew"])
def test_invalid_edge_links_are_rejected_on_the_host(case):
    box = _block()
    edge = int(np.flatnonzero(box.links["group2"] >= 0)[0])
    if case == "group2_range":
        _set(box, "group2", edge, 6)
    elif case == "normal2_unit":
        _set(box, "normal2", edge, (0.0, 1.1, 0.0))
    else:
        n = box.links["normal"][edge]
        m = box.links["normal2"][edge]
        _set(box, "normal2", edge, tuple((m + 0.5 * n) / np.linalg.norm(m + 0.5 * n)))
    rc, msg = _create(box)
    assert rc == -1 and msg, (case, rc, msg)


@pytest.mark.parametrize("case", ["group_profile", "group_ramp", "wall_profile", "wall_ramp", "edge_profiles",
                                  "many_ramps"])
def test_invalid_time_profiles_are_rejected_on_the_host(case):
    if case in ("wall_profile", "wall_ramp"):
        box = _slab()
        w = box.x_walls[1]
        box.x_walls = (box.x_walls[0], B.Wall3(w.kind, w.value, profile=5 if case == "wall_profile" else B.RAMP,
                                               ramp_time=0.0))
        rc, msg = _create(box)
        assert rc == -1 and msg, (case, rc, msg)
        return
    box = _block() if case == "edge_profiles" else _cavity()
    if case == "group_profile":
        box.groups[0] = B.BCGroup3(B.NEUMANN, profile=3)
    elif case == "group_ramp":
        box.groups[0] = B.BCGroup3(B.NEUMANN, profile=B.RAMP, ramp_time=-1.0)
    elif case == "edge_profiles":
        # the -x face ramped, the -y face (which shares an edge with it) not
        box.groups[0] = B.BCGroup3(B.NEUMANN, profile=B.RAMP, ramp_time=3.0)
    else:
        box.groups = [B.BCGroup3(B.NEUMANN, profile=B.RAMP, ramp_time=1.0 + k) for k in range(16)]
        rc, msg = _create(box)
        assert rc == -5 and msg, (case, rc, msg)
        return
    rc, msg = _create(box)
    assert rc == -1 and msg, (case, rc, msg)


@pytest.mark.parametrize("make", [_cavity, _cracked, _block])
def test_valid_geometry_without_a_gpu_fails_loudly(make):
    """A valid cavity, or cavity and crack, passes the host checks and then
    fails for want of a device."""
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    box = make()
    assert len(box.links) > 0 and box.n_material < box.n_sites
    rc, msg = _create(box)
    assert rc == -3, (rc, msg)


def _mutate(box, rng):
    """One seeded change to a valid geometry: a field of one link record
    (site, direction, q, group, second group, a normal), a record dropped,
    repeated, added with a changed site or direction, the records shuffled,
    a record moved to a neighbouring site, or one site of the mask flipped.
    Some changes keep the geometry valid (a shuffle, a new unit normal on a
    face link), most do not."""
    L = box.links.copy()
    n, ng = box.n_sites, len(box.groups)
    kind = str(rng.choice(["site", "dir", "q", "group", "group2", "normal", "normal2", "drop", "repeat",
                           "shuffle", "mask", "move", "add_site", "add_dir"]))
    i = int(rng.integers(len(L)))
    if kind.startswith("add_"):
        L = np.concatenate([L, L[i:i + 1]])
        i, kind = len(L) - 1, kind[4:]
    if kind == "site":
        L["site"][i] = int(rng.integers(-5, n + 5))
    elif kind == "dir":
        L["dir"][i] = int(rng.integers(-1, 21))
    elif kind == "q":
        L["q"][i] = rng.choice([-0.1, 0.0, 1e-6, 0.3, 1.0, 1.0000001, 2.0])
    elif kind == "group":
        L["group"][i] = int(rng.integers(-2, ng + 2))
    elif kind == "group2":
        L["group2"][i] = int(rng.integers(-3, ng + 2))
    elif kind in ("normal", "normal2"):
        if rng.random() < 0.5:
            v = rng.normal(size=3)
            L[kind][i] = v / np.linalg.norm(v)
        else:
            L[kind][i] = L[kind][i] * (1 + rng.choice([1e-7, -1e-7, 1e-11]))
    elif kind == "drop":
        L = np.delete(L, i)
    elif kind == "repeat":
        L = np.concatenate([L, L[i:i + 1]])
    elif kind == "shuffle":
        L = L[rng.permutation(len(L))]
    elif kind == "mask":
        m = box.mask.copy()
        m.ravel()[int(rng.integers(n))] ^= 1
        box.mask = m
    else:                                               # move
        L["site"][i] = (int(L["site"][i]) + int(rng.choice([-1, 1, -box.nx, box.nx]))) % n
    box.links = L


def test_host_checks_agree_with_the_reference():
    """The library's host checks of a general geometry and the CPU
    reference's, written apart, accept and refuse the same geometries: 900
    seeded changes (one or two each) to a cavity, a cavity with a crack and a
    block with edges."""
    from oracle.slbm3d import Oracle3D
    rng = np.random.default_rng(2208)
    outcomes = {True: 0, False: 0}
    for it in range(900):
        box = (_cavity, _cracked, _block)[it % 3]()
        for _ in range(int(rng.integers(1, 3))):
            _mutate(box, rng)
        try:
            Oracle3D(box)
            ref_ok = True
        except ValueError:
            ref_ok = False
        rc, msg = _create(box)
        assert rc in (0, -3, -1), (it, rc, msg)
        assert (rc != -1) == ref_ok, (it, rc, msg)
        outcomes[ref_ok] += 1
    assert min(outcomes.values()) > 50, outcomes
