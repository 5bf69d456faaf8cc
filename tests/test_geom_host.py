"""The library's device geometry, built for the host (tests/host_geom), against
brute-force enumeration and the oracle's index maps (no GPU).

site_geometry / three_hop_geometry / link_sign / tile_block / xcd_block are the
__host__ __device__ functions of qx_device.h that every kernel calls; here they
run on the CPU over whole lattices, including the 32^4 and 48^4 shapes the
benchmark uses."""
import ctypes
import itertools
import os

import numpy as np
import pytest

import oracle

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "tests", "host_geom", "libqx_geom_host.so")
SHAPES = [(2, 2, 2, 2), (4, 4, 4, 4), (4, 2, 2, 6), (2, 4, 6, 8), (6, 6, 6, 6), (8, 8, 8, 12),
          (8, 4, 2, 2), (16, 16, 16, 32), (12, 12, 12, 12), (32, 32, 32, 32)]


@pytest.fixture(scope="module")
def geo():
    if not os.path.exists(LIB):
        import __graft_entry__

        __graft_entry__.build_geom_host()
    L = ctypes.CDLL(LIB)
    P = ctypes.c_void_p
    L.qxg_maps.argtypes = [P, ctypes.c_int, P, P, P]
    L.qxg_tile_perm.argtypes = [P, ctypes.c_int, P]
    L.qxg_xcd_perm.argtypes = [ctypes.c_int, P]
    L.qxg_tile_bijection_failures.argtypes = [ctypes.c_int, ctypes.c_int]
    L.qxg_tile_bijection_failures.restype = ctypes.c_int64
    return L


def _p(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def maps(geo, dims, anti):
    V = int(np.prod(dims))
    d = np.array(dims, dtype=np.int32)
    lex = np.empty(V, np.int32)
    nbr = np.empty((V, 16), np.int32)
    sign = np.empty((V, 4), np.int32)
    geo.qxg_maps(_p(d), int(anti), _p(lex), _p(nbr), _p(sign))
    return lex, nbr, sign


def coords_of_lex(dims, lex):
    """Coordinates (x0 fastest) of lexicographic indices, vectorised."""
    c = np.empty((len(lex), 4), np.int64)
    t = lex.astype(np.int64)
    for mu in range(4):
        c[:, mu] = t % dims[mu]
        t //= dims[mu]
    return c


def eo_of_coords(dims, c):
    lex = c[:, 0] + dims[0] * (c[:, 1] + dims[1] * (c[:, 2] + dims[2] * c[:, 3]))
    par = c.sum(axis=1) % 2
    return par * (int(np.prod(dims)) // 2) + (lex >> 1)


@pytest.mark.parametrize("dims", SHAPES)
def test_device_geometry_matches_enumeration(geo, dims):
    V = int(np.prod(dims))
    hv = V // 2
    lex, nbr, sign = maps(geo, dims, False)
    # the one-hop maps equal the oracle's, which are pinned by brute force
    o_lex, o_nbr = oracle.index_maps(dims)
    assert np.array_equal(lex, o_lex)
    assert np.array_equal(nbr[:, :8], o_nbr)
    # independently: coordinates from lex, eo from coordinates, x +- mu and x +- 3 mu
    c = coords_of_lex(dims, lex)
    eo = np.arange(V)
    assert np.array_equal(eo_of_coords(dims, c), eo)
    assert np.array_equal(np.sort(lex), np.arange(V))
    assert ((c.sum(axis=1) % 2) == (eo >= hv)).all()
    for mu in range(4):
        for k, step in ((mu, 1), (4 + mu, -1), (8 + mu, 3), (12 + mu, -3)):
            y = c.copy()
            y[:, mu] = (y[:, mu] + step) % dims[mu]
            assert np.array_equal(nbr[:, k], eo_of_coords(dims, y)), (dims, k)
    # eta_mu(x) = (-1)^(x_0 + ... + x_{mu-1}), periodic: no boundary sign
    for mu in range(4):
        eta = np.where(c[:, :mu].sum(axis=1) % 2 == 1, -1, 1)
        assert np.array_equal(sign[:, mu], eta)


@pytest.mark.parametrize("dims", [(4, 4, 4, 4), (4, 2, 2, 6), (8, 8, 8, 12)])
def test_device_link_signs_antiperiodic(geo, dims):
    lex, _, sign = maps(geo, dims, True)
    c = coords_of_lex(dims, lex)
    for mu in range(4):
        eta = np.where(c[:, :mu].sum(axis=1) % 2 == 1, -1, 1)
        bc = np.where((mu == 3) & (c[:, 3] == dims[3] - 1), -1, 1)
        assert np.array_equal(sign[:, mu], eta * bc)


def test_tile_block_bijection_exhaustive(geo):
    """Orders 0-5 are bijections of the block range for every L2, L3 even up to
    48 and 1-4 blocks per (z, t) plane."""
    assert geo.qxg_tile_bijection_failures(48, 4) == 0


@pytest.mark.parametrize("dims", [(16, 16, 16, 16), (32, 32, 32, 32), (48, 48, 48, 48),
                                  (16, 16, 16, 32), (24, 24, 24, 24), (8, 8, 8, 8),
                                  (12, 12, 12, 12), (32, 32, 32, 64)])
@pytest.mark.parametrize("order", [2, 3, 4, 5])
def test_tile_block_bijection_real_shapes(geo, dims, order):
    hv = int(np.prod(dims)) // 2
    nb = hv // 64
    out = np.empty(nb, np.int32)
    assert geo.qxg_tile_perm(_p(np.array(dims, np.int32)), order, _p(out)) == nb
    assert np.array_equal(np.sort(out), np.arange(nb))
    s2 = dims[0] // 2 * dims[1]
    if order >= 4:
        cut = dims[2] if order == 4 else dims[3]
        if s2 % 64 or cut % 8:
            assert np.array_equal(out, np.arange(nb))
            return
        # slab k (positions [k nb/8, (k+1) nb/8)) covers one eighth of the cut
        # extent, every plane of it, in plane-major order
        P = s2 // 64
        plane = out // P
        z, t = plane % dims[2], plane // dims[2]
        w = cut // 8
        per = nb // 8
        for k in range(8):
            zs = z[k * per:(k + 1) * per] if order == 4 else t[k * per:(k + 1) * per]
            assert zs.min() == k * w and zs.max() == (k + 1) * w - 1
        walk = t if order == 4 else z
        assert np.all(np.diff(walk[:per]) >= 0)  # the other extent is walked in order
        return
    if s2 % 64 == 0 and dims[3] >= 4:
        # tiled: position bl's block lies in the (z, t) plane the tile walk names
        P = s2 // 64
        plane = out // P
        z, t = plane % dims[2], plane // dims[2]
        # consecutive positions move at most a tile apart in t
        assert np.abs(np.diff(t))[: 4 * P].max() <= 1
        assert np.array_equal(out % P, np.arange(nb) % P)
        assert z.min() == 0 and t.max() == dims[3] - 1
    else:
        assert np.array_equal(out, np.arange(nb))


@pytest.mark.parametrize("G", list(range(1, 70)) + [1000, 4096, 8191, 8192, 8193, 41472])
def test_xcd_block_bijection(geo, G):
    """The XCD-contiguous remapping is a bijection, and dispatch index b lands in
    the (b mod 8)-th contiguous range."""
    out = np.empty(G, np.int32)
    geo.qxg_xcd_perm(G, _p(out))
    assert np.array_equal(np.sort(out), np.arange(G))
    q, r = divmod(G, 8)
    starts = [x * (q + 1) if x < r else r * (q + 1) + (x - r) * q for x in range(8)]
    sizes = [q + 1 if x < r else q for x in range(8)]
    b = np.arange(G)
    x = b % 8
    assert (out >= np.array(starts)[x]).all() and (out < np.array(starts)[x] + np.array(sizes)[x]).all()
