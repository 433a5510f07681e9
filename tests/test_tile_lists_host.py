"""The per-tile cut-link lists of the two-step kernel, host side
(slbm_tile_list_layout, no device): against a brute-force walk over every
tile's reach.

A tile of R rows of a 58-column strip reaches rows y0 - 3 .. y0 + R + 2 and
columns xs - 3 .. xs + 60 (wave w, lane l at y0 - 3 + w, xs - 3 + l); on a
periodic axis positions wrap, elsewhere positions off the grid hold nothing.
Every cut link whose site sits at a position of the reach is a record of that
tile, with that position.  The GPU tests check that evaluating the rules from
these lists gives the same state as site by site; this pins the lists
themselves, including the wrap of plates narrower than a strip.
"""
import collections

import numpy as np
import pytest

from slbm_workloads import configs
from slbm_workloads import geometry as G


@pytest.fixture(scope="module")
def slbm_host():
    from paper_2208_04088_amd import slbm as S
    S.lib()
    return S


def brute_force(nx, ny, px, py, R, sites):
    at = collections.defaultdict(list)
    for i, s in enumerate(sites):
        at[int(s)].append(i)
    nstrips, ntr = -(-nx // 58), -(-ny // R)
    tiles = []
    for t in range(nstrips * ntr):
        st, tr = t % nstrips, t // nstrips
        recs = []
        for w in range(R + 6):
            y = tr * R - 3 + w
            if not 0 <= y < ny:
                if not py:
                    continue
                y %= ny
            for l in range(64):
                x = st * 58 - 3 + l
                if not 0 <= x < nx:
                    if not px:
                        continue
                    x %= nx
                recs += [(i, (w << 8) | l) for i in at.get(y * nx + x, ())]
        tiles.append(sorted(recs))
    return tiles


def plates():
    yield "hole", configs.hole_plate(200, 80.0, lam=0.05, tau=0.55)
    yield "crack", configs.edge_crack_plate(180, 90, 60)
    yield "square", configs.square_clamped_pulled(70)
    mu = 0.05
    groups = [G.BCGroup(G.DIRICHLET, (0.0, 0.0)), G.BCGroup(G.NEUMANN, (1e-5, 0.0))]
    yield "periodic", G.build_plate(64, 40, lam=0.04, mu=mu, tau=0.55, periodic_x=True, periodic_y=True,
                                    walls=[G.Circle(29.0, 22.0, 7.0, 0), G.Circle(51.0, 10.0, 4.0, 1)],
                                    groups=groups)
    yield "narrow_periodic", G.build_plate(5, 9, lam=0.04, mu=mu, tau=0.55, periodic_x=True,
                                           walls=[G.HLine(-0.5, 0), G.HLine(8.5, 1)], groups=groups)
    yield "one_column", G.build_plate(1, 7, lam=0.04, mu=mu, tau=0.55, periodic_x=True,
                                      walls=[G.HLine(-0.5, 0), G.HLine(6.5, 1)], groups=groups)


@pytest.mark.parametrize("rows", [1, 3, 10])
@pytest.mark.parametrize("name,plate", list(plates()), ids=[n for n, _ in plates()])
def test_layout_matches_brute_force(slbm_host, name, plate, rows):
    sites = np.asarray(plate.links["site"], dtype=np.int32)
    px, py = bool(plate.periodic_x), bool(plate.periodic_y)
    start, link, pos, most = slbm_host.tile_list_layout(plate.nx, plate.ny, sites, rows, px, py)
    want = brute_force(plate.nx, plate.ny, px, py, rows, sites)
    assert len(start) == len(want) + 1 and start[0] == 0
    got = [sorted(zip(link[start[t]:start[t + 1]].tolist(), pos[start[t]:start[t + 1]].tolist()))
           for t in range(len(want))]
    assert got == want
    assert most == max(len(t) for t in want)
    # every link appears in at least one tile (its own strip and rows)
    assert set(link.tolist()) == set(range(len(sites)))


def test_layout_rejects_bad_input(slbm_host):
    with pytest.raises(slbm_host.SlbmError):
        slbm_host.tile_list_layout(10, 10, [0, 5], 0)
    with pytest.raises(slbm_host.SlbmError):
        slbm_host.tile_list_layout(10, 10, [0, 5], 11)
    with pytest.raises(slbm_host.SlbmError):
        slbm_host.tile_list_layout(10, 10, [0, 100], 4)
