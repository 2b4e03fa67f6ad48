"""Index arithmetic of the 3D transfer kernels, replayed on the CPU.

The restriction and prolongation kernels walk 64-point slice segments.  In
3D each lane decodes its (x, y) from its slice-local index with an FP32
square root, and the kernels form storage indices incrementally instead of
from the closed-form layout: the restriction takes the 15 fine neighbours of
2P relative to the index of 2P and derives whether each lies in the macro,
and its support mask, from P's position; the prolongation forms the coarse
slice bases once per segment.  These tests replay that arithmetic lane by
lane and compare it with the closed-form layout (slice bases, row starts,
support masks) and checks that every offset is a non-negative 32-bit value, for every point of small levels and for the edge slices of
the largest 3D level.
"""
import numpy as np
import pytest

OFF3 = [(0, 0, -1), (1, 0, -1), (0, 1, -1), (-1, 1, -1), (0, -1, 0), (1, -1, 0), (-1, 0, 0), (0, 0, 0),
        (1, 0, 0), (-1, 1, 0), (0, 1, 0), (0, -1, 1), (1, -1, 1), (-1, 0, 1), (0, 0, 1)]


def tet(n):
    return n * (n + 1) * (n + 2) // 6


def slice_base(N, z):
    return tet(N + 1) - tet(N + 1 - z)


def rs(S, y):
    return y * (S + 2) - (y * (y + 1)) // 2


def idx3(N, x, y, z):
    return slice_base(N, z) + rs(N - z, y) + x


def support_mask(N, x, y, z):
    return ((N - x - y - z) != 0) * 1 | (x != 0) * 2 | (y != 0) * 4 | (z != 0) * 8


def decode(S, r, ulp=0):
    """slice_point's FP32 decode; ulp = -1 / +1 moves the root by one ulp
    (the hardware root is within one ulp of the correctly rounded one)."""
    b = np.float32(2 * S + 3)
    disc = (b * b - np.float32(8) * r.astype(np.float32)).astype(np.float32)
    root = np.sqrt(disc)
    if ulp:
        root = np.nextafter(root, np.float32(np.inf if ulp > 0 else -np.inf)).astype(np.float32)
    yy = np.clip(((b - root) * np.float32(0.5)).astype(np.int64), 0, S)
    yy = np.where(rs(S, yy) > r, yy - 1, yy)
    yy = np.where((yy < S) & (rs(S, np.minimum(yy + 1, S)) <= r), yy + 1, yy)
    return r - rs(S, yy), yy


def check_decode(N, zs):
    for z in zs:
        S = N - z
        r = np.arange((S + 1) * (S + 2) // 2, dtype=np.int64)
        for u in (0, -1, 1):
            x, y = decode(S, r, u)
            assert (x >= 0).all() and (y >= 0).all() and (x + y <= S).all(), (N, z, u)
            assert np.array_equal(rs(S, y) + x, r), (N, z, u)


def check_restrict(Nc, zs):
    Nf = 2 * Nc
    for z in zs:
        S_c = Nc - z
        r = np.arange((S_c + 1) * (S_c + 2) // 2, dtype=np.int64)
        x, y = decode(S_c, r)
        x0, y0, z0, far = x == 0, y == 0, np.full(x.shape, z == 0), x + y + z == Nc
        zf, S = 2 * z, Nf - 2 * z
        yf, xf = 2 * y, 2 * x
        za = zf - 1 if zf > 0 else 0
        fb = slice_base(Nf, za)  # the anchor: first point of slice 2z - 1 (slice 0 at z = 0)
        tb = slice_base(Nf, zf) - fb
        c = tb + rs(S, yf) + xf
        ln = S + 1 - yf
        up = c + (S + 1) * (S + 2) // 2 - yf
        dn = c - tb + yf
        rel = [dn, dn + 1, dn + ln + 1, dn + ln, c - ln - 1, c - ln, c - 1, c, c + 1, c + ln - 1, c + ln,
               up - ln, up - ln + 1, up - 1, up]
        for s, (dx, dy, dz) in enumerate(OFF3):
            sd = dx + dy + dz
            inn = (dx >= 0) | ~x0
            inn &= (dy >= 0) | ~y0
            inn &= (dz >= 0) | ~z0
            inn &= (sd <= 0) | ~far
            mask = np.where(far & (sd == 0), 0, 1) | np.where(x0 & (dx == 0), 0, 2) | \
                np.where(y0 & (dy == 0), 0, 4) | np.where(z0 & (dz == 0), 0, 8)
            fx, fy, fz = xf + dx, yf + dy, np.full(x.shape, zf + dz)
            want_in = (fx >= 0) & (fy >= 0) & (fz >= 0) & (fx + fy + fz <= Nf)
            assert np.array_equal(inn, want_in), (Nc, z, s)
            if want_in.any():
                k = want_in
                assert (rel[s][k] >= 0).all() and (rel[s][k] * 8 < 2 ** 32).all()  # unsigned 32-bit offsets
                assert np.array_equal(fb + rel[s][k], idx3(Nf, fx[k], fy[k], fz[k])), (Nc, z, s)
                assert np.array_equal(mask[k], support_mask(Nf, fx[k], fy[k], fz[k])), (Nc, z, s)


def check_prolong(Nc, zs):
    Nf = 2 * Nc
    for z in zs:
        S = Nf - z
        r = np.arange((S + 1) * (S + 2) // 2, dtype=np.int64)
        x, y = decode(S, r)
        px, py, pz = x & 1, y & 1, z & 1
        sx = px
        sy = np.where((px == 1) & (py == 1), -1, py)
        sz = np.where((pz == 1) & ((px ^ py) == 1), -1, pz)
        zl, zh = z >> 1, (z + 1) >> 1
        bl = slice_base(Nc, zl)
        dh = slice_base(Nc, zh) - bl
        zu = np.where(sz < 0, zh, zl)
        zv = np.where(sz > 0, zh, zl)
        ou = np.where(sz < 0, dh, 0) + rs(Nc - zu, (y - sy) >> 1) + ((x - sx) >> 1)
        ov = np.where(sz > 0, dh, 0) + rs(Nc - zv, (y + sy) >> 1) + ((x + sx) >> 1)
        assert (ou >= 0).all() and (ov >= 0).all() and (ou * 8 < 2 ** 32).all() and (ov * 8 < 2 ** 32).all()
        iu, iv = bl + ou, bl + ov
        # the closed form of the two coarse endpoints
        ju = idx3(Nc, (x - sx) >> 1, (y - sy) >> 1, (z - sz) >> 1)
        jv = idx3(Nc, (x + sx) >> 1, (y + sy) >> 1, (z + sz) >> 1)
        assert np.array_equal(iu, ju) and np.array_equal(iv, jv), (Nc, z)
        # both endpoints are coarse points of the macro
        for xs, ys, zs_ in (((x - sx) >> 1, (y - sy) >> 1, (z - sz) >> 1), ((x + sx) >> 1, (y + sy) >> 1, (z + sz) >> 1)):
            assert (xs >= 0).all() and (ys >= 0).all() and (xs + ys + zs_ <= Nc).all()
        assert np.array_equal(slice_base(Nf, z) + r, idx3(Nf, x, y, z))


@pytest.mark.parametrize("L", range(0, 9))
def test_3d_decode_every_slice(L):
    N = 1 << L
    check_decode(N, range(N + 1))


def test_3d_decode_level_11_slices():
    N = 1 << 11
    check_decode(N, [0, 1, 2, 511, 1024, 1500, N - 2, N - 1, N])


@pytest.mark.parametrize("Lc", range(0, 8))
def test_3d_restriction_indices_every_point(Lc):
    Nc = 1 << Lc
    check_restrict(Nc, range(Nc + 1))


@pytest.mark.parametrize("Lc", range(1, 8))
def test_3d_prolongation_indices_every_point(Lc):
    Nc = 1 << Lc
    check_prolong(Nc, range(2 * Nc + 1))


def test_3d_transfer_indices_level_11_edge_slices():
    check_restrict(1 << 10, [0, 1, 2, 512, 1021, 1022, 1023, 1024])
    check_prolong(1 << 10, [0, 1, 2, 3, 1025, 2045, 2046, 2047, 2048])


def test_replay_catches_a_wrong_slice_offset():
    """The replay has teeth: an off-by-one in the offset of the slice below
    moves the slice-below neighbours."""
    Nc = 8
    Nf = 2 * Nc
    z = 2
    S = Nf - 2 * z
    r = np.arange((Nc - z + 1) * (Nc - z + 2) // 2, dtype=np.int64)
    x, y = decode(Nc - z, r)
    tb = slice_base(Nf, 2 * z) - slice_base(Nf, 2 * z - 1)
    c = tb + rs(S, 2 * y) + 2 * x
    dn_wrong = c - tb + 2 * y - 1
    assert not np.array_equal(slice_base(Nf, 2 * z - 1) + dn_wrong, idx3(Nf, 2 * x, 2 * y, 2 * z - 1))


def nbr_offsets3(N, y, z):
    """nbr_offsets3 (rows.hpp): the 15 neighbours' storage offsets relative
    to the point, used by the V-cycle tail's stencil rows and the point
    form of the restriction."""
    S = N - z
    d = S + 1 - y
    up = (S + 1) * (S + 2) // 2 - y
    dn = y - (S + 2) * (S + 3) // 2
    return [dn, dn + 1, dn + d + 1, dn + d, -d - 1, -d, -1, 0 * d, 1 + 0 * d, d - 1, d, up - d, up - d + 1, up - 1,
            up]


@pytest.mark.parametrize("L", range(0, 7))
def test_3d_neighbour_offsets_every_point(L):
    N = 1 << L
    for z in range(N + 1):
        S = N - z
        r = np.arange((S + 1) * (S + 2) // 2, dtype=np.int64)
        x, y = decode(S, r)
        i = idx3(N, x, y, z)
        off = nbr_offsets3(N, y, z)
        for o, (dx, dy, dz) in enumerate(OFF3):
            nx, ny, nz = x + dx, y + dy, z + dz
            k = (nx >= 0) & (ny >= 0) & (nz >= 0) & (nx + ny + nz <= N)
            if k.any():
                assert np.array_equal((i + off[o])[k], idx3(N, nx[k], ny[k], np.full(k.sum(), nz))), (N, z, o)
