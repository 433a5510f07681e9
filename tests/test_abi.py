"""The C ABI without a GPU: the library loads, exports every function the
header declares, its structs have the layout the header states, and invalid
problems are rejected on the host before any device call."""
import ctypes as C
import os
import re
import subprocess

import numpy as np
import pytest

from paper_2208_04088_amd import slbm as S
from slbm_workloads import geometry as G

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "slbm.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(slbm_[a-z_]+)\s*\(", text)))


def test_library_exports_every_declared_function():
    L = S.lib()
    names = declared_functions()
    assert len(names) >= 12
    missing = [n for n in names if not hasattr(L, n)]
    assert not missing, missing
    assert sorted(S.EXPORTS) == names


def test_struct_layout_matches_header(tmp_path):
    src = tmp_path / "layout.c"
    fields = {
        "slbm_params": [f for f, _ in S.Params._fields_],
        "slbm_link": list(S.LINK_DTYPE.names),
        "slbm_bc_group": list(S.GROUP_DTYPE.names),
    }
    cname = {"lam": "lambda"}
    lines = ["#include <stdio.h>", "#include <stddef.h>", '#include "slbm.h"', "int main(void){"]
    for st, fl in fields.items():
        lines.append(f'printf("{st} %zu\\n", sizeof({st}));')
        for f in fl:
            lines.append(f'printf("{st}.{f} %zu\\n", offsetof({st}, {cname.get(f, f)}));')
    lines.append("return 0;}")
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    out = dict(l.rsplit(" ", 1) for l in subprocess.run([str(exe)], capture_output=True, text=True,
                                                         check=True).stdout.split("\n") if l)
    assert int(out["slbm_params"]) == C.sizeof(S.Params)
    for f, _ in S.Params._fields_:
        assert int(out[f"slbm_params.{f}"]) == getattr(S.Params, f).offset, f
    for dt, st in ((S.LINK_DTYPE, "slbm_link"), (S.GROUP_DTYPE, "slbm_bc_group")):
        assert int(out[st]) == dt.itemsize
        for f in dt.names:
            assert int(out[f"{st}.{f}"]) == dt.fields[f][1], f


def _plate():
    n = 12
    walls = G.edge_walls(n, n, left=0, right=1, bottom=1, top=1)
    walls.append(G.Circle(6.2, 5.8, 2.3, 1))
    return G.build_plate(n, n, lam=0.05, mu=0.05, tau=0.55, walls=walls,
                         groups=[G.BCGroup(G.DIRICHLET), G.BCGroup(G.NEUMANN, (1e-5, 0.0))])


def _create(plate, **over):
    prm, keep = S.marshal(plate, "fp32")
    for k, v in over.items():
        setattr(prm, k, v)
    h = C.c_void_p()
    rc = S.lib().slbm_create(C.byref(prm), C.byref(h))
    if rc == 0:
        S.lib().slbm_destroy(h)
    return rc, S.lib().slbm_last_error().decode()


def _mutated(fn):
    p = _plate()
    L = p.links.copy()
    fn(p, L)
    p.links = L
    return p


@pytest.mark.parametrize("case", [
    "q_zero", "q_big", "bad_group", "bad_group2", "normal", "dup", "void_site", "dir",
    "uncut_leaves", "one_sided", "tau", "mu", "rho", "order", "precision"])
def test_invalid_problems_are_rejected_on_the_host(case):
    over = {}
    p = _plate()
    if case == "q_zero":
        p = _mutated(lambda p, L: L["q"].__setitem__(0, 0.0))
    elif case == "q_big":
        p = _mutated(lambda p, L: L["q"].__setitem__(3, 1.5))
    elif case == "bad_group":
        p = _mutated(lambda p, L: L["group"].__setitem__(1, 7))
    elif case == "bad_group2":
        p = _mutated(lambda p, L: L["group2"].__setitem__(1, 9))
    elif case == "normal":
        p = _mutated(lambda p, L: L["normal"].__setitem__(2, (0.5, 0.5)))
    elif case == "dup":
        p.links = np.concatenate([p.links, p.links[:1]])
    elif case == "void_site":
        p = _mutated(lambda p, L: None)
        p.mask = p.mask.copy()
        p.mask.flat[int(p.links["site"][0])] = 0
    elif case == "dir":
        p = _mutated(lambda p, L: L["dir"].__setitem__(0, 9))
    elif case == "uncut_leaves":
        p.links = p.links[1:]
    elif case == "one_sided":
        # cut an interior link from one end only
        extra = np.zeros(1, dtype=p.links.dtype)
        extra[0] = (5 * 12 + 2, 1, 0.5, 1, -1, (1.0, 0.0), (0.0, 0.0))
        p.links = np.concatenate([p.links, extra])
    elif case == "tau":
        over["tau"] = 0.5
    elif case == "mu":
        over["mu"] = 0.0
    elif case == "rho":
        over["rho"] = -1.0
    elif case == "order":
        over["neumann_order"] = 2
    elif case == "precision":
        over["precision"] = 7
    rc, msg = _create(p, **over)
    assert rc == -1, (rc, msg)
    assert msg


def test_valid_problem_without_a_gpu_fails_loudly():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    rc, msg = _create(_plate())
    assert rc == -3, (rc, msg)


def test_device_moments_reject_a_null_handle():
    """slbm_moments_device checks its arguments before any device call."""
    L = S.lib()
    assert L.slbm_moments_device(None, None, None, None, None, S.FP64) == -1
    assert "handle" in L.slbm_last_error().decode()


def test_batch_displacement_rejects_a_null_batch():
    L = S.lib()
    assert L.slbm_batch_displacement(None, 0, None) == -1


def test_too_large_a_grid_is_unsupported():
    """At most 2^28 sites: one more row of 16384 is refused on the host,
    before the mask is read (a grid of exactly 2^28 sites is run by the GPU
    tests)."""
    rc, msg = _create(_plate(), nx=16384, ny=16385)
    assert rc == -5, (rc, msg)


def test_launch_configuration_calls_reject_a_null_handle():
    L = S.lib()
    assert L.slbm_set_xcd_group(None, 8) == -1
    assert L.slbm_get_launch(None, None, None, None) == -1
    assert L.slbm_batch_set_xcd_group(None, 8) == -1


def _cracked_plate():
    """A 14 x 10 plate with an edge crack entering from the left edge (links
    through the crack's mouth carry two walls)."""
    walls = G.edge_walls(14, 10, left=0, right=0, bottom=1, top=2)
    walls.append(G.HLine(4.5, -0.5, 6.5, 0))
    return G.build_plate(14, 10, lam=0.05, mu=0.05, tau=0.55, walls=walls,
                         groups=[G.BCGroup(G.NEUMANN), G.BCGroup(G.NEUMANN, (0.0, -1e-5)),
                                 G.BCGroup(G.NEUMANN, (0.0, 1e-5))])


def _mutate(p, rng):
    """One seeded change to a valid plate: a field of one link record (site,
    direction, q, group, second group, a normal), a record dropped, repeated,
    added with a changed site or direction, the records shuffled, a record
    moved to a neighbouring site, or one site of the mask flipped."""
    L = p.links.copy()
    n, ng = p.nx * p.ny, len(p.groups)
    kind = str(rng.choice(["site", "dir", "q", "group", "group2", "normal", "normal2", "drop", "repeat",
                           "shuffle", "mask", "move", "add_site", "add_dir"]))
    i = int(rng.integers(len(L)))
    if kind.startswith("add_"):
        L = np.concatenate([L, L[i:i + 1]])
        i, kind = len(L) - 1, kind[4:]
    if kind == "site":
        L["site"][i] = int(rng.integers(-5, n + 5))
    elif kind == "dir":
        L["dir"][i] = int(rng.integers(-1, 11))
    elif kind == "q":
        L["q"][i] = rng.choice([-0.1, 0.0, 1e-6, 0.3, 1.0, 1.0000001, 2.0])
    elif kind == "group":
        L["group"][i] = int(rng.integers(-2, ng + 2))
    elif kind == "group2":
        L["group2"][i] = int(rng.integers(-3, ng + 2))
    elif kind in ("normal", "normal2"):
        if rng.random() < 0.5:
            v = rng.normal(size=2)
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
        m = p.mask.copy()
        m.ravel()[int(rng.integers(n))] ^= 1
        p.mask = m
    else:                                               # move
        L["site"][i] = (int(L["site"][i]) + int(rng.choice([-1, 1, -p.nx, p.nx]))) % n
    p.links = L


def test_host_checks_agree_with_the_reference():
    """The library's host checks of a plate and the CPU reference's, written
    apart, accept and refuse the same plates: 1200 seeded changes (one or two
    each) to a plate with a hole and to a plate with an edge crack."""
    from oracle import Oracle
    rng = np.random.default_rng(2208)
    outcomes = {True: 0, False: 0}
    for it in range(1200):
        p = (_plate, _cracked_plate)[it % 2]()
        for _ in range(int(rng.integers(1, 3))):
            _mutate(p, rng)
        try:
            Oracle(p)
            ref_ok = True
        except ValueError:
            ref_ok = False
        rc, msg = _create(p)
        assert rc in (0, -3, -1), (it, rc, msg)
        assert (rc != -1) == ref_ok, (it, rc, msg)
        outcomes[ref_ok] += 1
    assert min(outcomes.values()) > 100, outcomes


def test_isolated_site_is_refused_on_the_host():
    """A material site with all 8 links cut (an island of one site) is
    refused: the kernels' per-site flag byte would read as void.  A pair of
    sites, each keeping one uncut link, is accepted."""
    def islands(sites):
        nx, ny = 9, 7
        mask = np.zeros((ny, nx), np.uint8)
        for x, y in sites:
            mask[y, x] = 1
        recs = []
        for x, y in sites:
            for k in range(1, 9):
                if mask[(y + G.CY[k]) % ny, (x + G.CX[k]) % nx]:
                    continue
                c = np.array([G.CX[k], G.CY[k]], dtype=float)
                recs.append((y * nx + x, k, 0.5, 0, -1, tuple(c / np.linalg.norm(c)), (0.0, 0.0)))
        return G.Plate(nx, ny, 0.05, 0.05, 1.0, 0.55, mask, np.array(recs, dtype=G.LINK_DTYPE),
                       [G.BCGroup(G.DIRICHLET)], periodic_x=True, periodic_y=True)
    rc, msg = _create(islands([(3, 3)]))
    assert rc == -1 and "every link is cut" in msg, (rc, msg)
    rc, msg = _create(islands([(3, 3), (4, 3)]))
    assert rc in (0, -3), (rc, msg)


def _declared(header):
    """(name, parameter types) of every function a header declares."""
    text = re.sub(r"/\*.*?\*/", "", open(os.path.join(ROOT, "include", header)).read(), flags=re.S)
    out = []
    for m in re.finditer(r"\bint\s+(slbm3?_[a-z_0-9]+)\s*\(([^)]*)\)\s*;", text):
        out.append((m.group(1), [p.strip().rsplit(" ", 1)[0] for p in m.group(2).split(",")]))
    return out


@pytest.mark.parametrize("header", ["slbm.h", "slbm3.h"])
def test_every_entry_point_refuses_a_null_handle(header):
    """Every function of the two headers that takes a handle or a batch (or,
    for the create calls, the parameter block) returns SLBM_E_INVAL with a
    message when given NULL for it, NULL for every pointer and zero for every
    number, before any device call; the destroy calls take NULL as a no-op."""
    L = C.CDLL(S.LIB_PATH)                         # no argument types: plain C calls
    L.slbm_last_error.restype = C.c_char_p
    seen = 0
    for name, types in _declared(header):
        if name in ("slbm_tile_list_layout", "slbm_copy"):
            continue                               # no handle (host layout; a plain copy)
        args = []
        for t in types:
            if "*" in t or t in ("slbm_handle", "slbm3_handle", "slbm_batch"):
                args.append(C.c_void_p(None))
            elif t in ("int64_t", "size_t"):
                args.append(C.c_int64(0))
            else:
                args.append(C.c_int32(0))
        f = getattr(L, name)
        f.restype = C.c_int
        rc = f(*args)
        if name.endswith("_destroy"):
            assert rc == 0, name
        else:
            assert rc == -1 and L.slbm_last_error(), (name, rc)
        seen += 1
    assert seen == (35 if header == "slbm.h" else 13)
