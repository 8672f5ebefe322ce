"""Oracle pins: site numbering (eq. i_s), checkerboard colour (eq. i_c),
periodic and double-layered torus neighbours (Sec. 2, Sec. 2.2)."""
import itertools
from collections import deque

import numpy as np
import pytest


def test_site_number_and_coordinates(oracle_mod):
    ext = [4, 6, 2, 8]
    L = oracle_mod.Lattice(ext)
    assert L.V == 4 * 6 * 2 * 8
    for s in range(L.V):
        x = L.site_coords(s)
        # eq. (i_s), 0-based: s = x0 + n0 (x1 + n1 (x2 + n2 x3)), x0 fastest
        assert s == x[0] + 4 * (x[1] + 6 * (x[2] + 2 * x[3]))
        assert L.site_index(x) == s
        # eq. (i_c): colour = parity of the coordinate sum
        assert L.parity(s) == sum(x) % 2


@pytest.mark.parametrize("ext", [[4, 4], [4, 6, 2], [2, 4, 4, 6]])
def test_pbc_neighbours(oracle_mod, ext):
    L = oracle_mod.Lattice(ext)
    D = len(ext)
    for s in range(L.V):
        x = L.site_coords(s)
        for d in range(D):
            for sg in (+1, -1):
                lo, so = L.neighbor(0, s, d, sg)
                assert lo == 0
                y = list(x)
                y[d] = (y[d] + sg) % ext[d]
                assert L.site_index(y) == so
                # one step changes the colour (extents even)
                assert L.parity(so) != L.parity(s)
                assert L.neighbor(lo, so, d, -sg) == (0, s)


@pytest.mark.parametrize("ext,mask", [([4, 4], 0b11), ([4, 4, 4, 2], 0b1111), ([4, 4, 4, 2], 0b0111),
                                      ([4, 2, 4], 0b001)])
def test_dlt_neighbours(oracle_mod, ext, mask):
    L = oracle_mod.Lattice(ext, nlat=2, dlt_mask=mask)
    D = len(ext)
    for d in range(D):
        for sg in (+1, -1):
            image = set()
            for layer in (0, 1):
                for s in range(L.V):
                    lo, so = L.neighbor(layer, s, d, sg)
                    image.add((lo, so))
                    assert L.neighbor(lo, so, d, -sg) == (layer, s)
                    x = L.site_coords(s)
                    wraps = (x[d] == ext[d] - 1 and sg > 0) or (x[d] == 0 and sg < 0)
                    flips = wraps and ((mask >> d) & 1)
                    assert lo == (1 - layer if flips else layer)
                    assert L.parity(so) != L.parity(s)
            assert len(image) == 2 * L.V      # the neighbour map is a bijection


@pytest.mark.parametrize("ext,nlat,mask", [([4, 4, 2, 4], 1, 0), ([4, 4, 2, 4], 2, 0b1111), ([4, 2, 4], 2, 0b011)])
def test_each_link_in_2_dm1_plaquettes(oracle_mod, ext, nlat, mask):
    L = oracle_mod.Lattice(ext, nlat=nlat, dlt_mask=mask)
    D = len(ext)
    count = {}
    for layer in range(nlat):
        for s in range(L.V):
            for mu, nu in itertools.combinations(range(D), 2):
                a = L.neighbor(layer, s, mu, +1)
                b = L.neighbor(layer, s, nu, +1)
                for key in [(layer, s, mu), (a[0], a[1], nu), (b[0], b[1], mu), (layer, s, nu)]:
                    count[key] = count.get(key, 0) + 1
    assert len(count) == nlat * L.V * D
    assert set(count.values()) == {2 * (D - 1)}


def test_dlt_doubles_the_shortest_wrap(oracle_mod):
    # On a 2D DLT glued in both directions, the copy of a site in the other
    # layer is N steps away (one wrap); returning to the same site through
    # the boundary takes two wraps, length 2N in lattice steps, sqrt(2) N
    # along the diagonal (Sec. 2.2).
    N = 6
    L = oracle_mod.Lattice([N, N], nlat=2, dlt_mask=0b11)
    dist = {(0, 0): 0}
    q = deque([(0, 0)])
    while q:
        node = q.popleft()
        for d in range(2):
            for sg in (+1, -1):
                nb = L.neighbor(node[0], node[1], d, sg)
                if nb not in dist:
                    dist[nb] = dist[node] + 1
                    q.append(nb)
    assert len(dist) == 2 * N * N
    assert dist[(1, 0)] == N
    # walking straight N steps along direction 0 returns to layer 1, 2N returns home
    node = (0, 0)
    for k in range(2 * N):
        node = L.neighbor(node[0], node[1], 0, +1)
        if k == N - 1:
            assert node == (1, 0)
    assert node == (0, 0)


@pytest.mark.parametrize("kw", [dict(extents=[3, 4]), dict(extents=[4]), dict(extents=[4, 4], nlat=3),
                                dict(extents=[4, 4], dlt_mask=1), dict(extents=[4, 4], lat2test=True),
                                dict(extents=[0, 4])])
def test_invalid_geometry_rejected(oracle_mod, kw):
    ext = kw.pop("extents")
    with pytest.raises(ValueError):
        oracle_mod.Lattice(ext, **kw)
