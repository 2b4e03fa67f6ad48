"""Every load of the stencil walks stays inside its macro's storage (CPU).

The 2D and 3D walks (stencil_kernels.hip) load whole wave rows with
unconditional loads whose row and column indices are clamped into the macro
(ldrow: row clamped to [0, min(last, S)], column to the row's length), or, on
interior 2D tiles, advance row addresses incrementally with no clamp.  A
clamp that lets an index leave the triangle (a row past the apex makes the
column bound S - row negative, which as an unsigned byte offset lands
gigabytes away) faults the GPU, so this test replays that index arithmetic
on the CPU, lane by lane, for every wave tile of small levels and for the
tiles near the apex and the far face at the largest levels, and checks each
element offset against the macro's point count.

The replay follows the kernels' loops: the tile lists are the ones the mesh
set-up builds (2D: bands of H rows, 62-column tiles; 3D: pencils of 4 rows x
8 slices), the rows and slices each tile loads are those of tile2d,
tile2d_fast and pencil3d, and the clamps are ldrow's.  Small 3D levels use
runs of slice segments instead (seg3d), whose per-lane neighbour indices are
replayed at the end of this file.
"""
import numpy as np
import pytest

W62 = 62
LANES = np.arange(64)


def rs32(S, y):
    return y * (S + 2) - ((y * (y + 1)) >> 1)


def tri_points(N):
    return (N + 1) * (N + 2) // 2


def tet_count(n):
    return n * (n + 1) * (n + 2) // 6


def slice_base(N, z):
    return tet_count(N + 1) - tet_count(N + 1 - z)


def ldrow(S, r, last, xc):
    """Element offset ldrow reads: row clamped to [0, min(last, S)], column
    to the row (xc >= 0 per lane)."""
    rr = min(max(r, 0), min(last, S))
    return rs32(S, rr) + np.minimum(xc, S - rr)


def tiles2d(N, H):
    return [(x0, y0) for y0 in range(0, N + 1, H) for x0 in range(0, N + 1 - y0, W62)]


def inner2d(x0, y0, N, H):
    return x0 >= 1 and y0 >= 1 and x0 + y0 + W62 + H <= N


def loads_tile2d(x0, y0, N, H, U, with_b):
    """Element offsets of every load of one clamped 2D tile (tile2d)."""
    xc = np.maximum(x0 - 1 + LANES, 0)
    y1 = min(y0 + H, N - x0 + 1)
    out = [ldrow(N, y0 - 1, y1, xc), ldrow(N, y0, y1, xc)]
    for k in range(U):
        out.append(ldrow(N, y0 + 1 + k, y1, xc))
        if with_b:
            out.append(ldrow(N, y0 + k, y1 - 1, xc))
    for k in range(H):
        if k + U < H:
            out.append(ldrow(N, y0 + 1 + k + U, y1, xc))
            if with_b:
                out.append(ldrow(N, y0 + k + U, y1 - 1, xc))
    return out


def loads_tile2d_fast(x0, y0, N, H):
    """Element offsets of an interior 2D tile (tile2d_fast): rows y0-1 ..
    y0+H at columns x0-1 .. x0+62, addresses advanced by the row length;
    returns them with the row each belongs to."""
    col = x0 - 1 + LANES
    out = []
    p = rs32(N, y0 - 1)
    step = N + 2 - y0  # length of row y0 - 1
    for r in range(y0 - 1, y0 + H + 1):
        out.append((r, p + col))
        p += step
        step -= 1
    return out


def check_2d(N, H, U, tiles, with_b=True):
    P = tri_points(N)
    n = 0
    for x0, y0 in tiles:
        if inner2d(x0, y0, N, H):
            for r, off in loads_tile2d_fast(x0, y0, N, H):
                cols = off - rs32(N, r)
                assert r <= N and (cols >= 0).all() and (cols <= N - r).all(), (x0, y0, r)
                n += off.size
        else:
            for off in loads_tile2d(x0, y0, N, H, U, with_b):
                assert (off >= 0).all() and (off < P).all(), (N, x0, y0)
                n += off.size
    return n


def loads_pencil3d(x0, y0, z0, N, PR, PZ, with_b):
    """Element offsets of every load of one 3D pencil (pencil3d): a ring of
    five slices from z0-1 and one more slice per output slice, rows y0-1 ..
    y0+PR of each (clamped), and the b rows y0 .. y0+PR-1 of slices z0 ..
    z0+PZ-1."""
    xc = np.maximum(x0 - 1 + LANES, 0)
    out = []

    def ld(zb, zp, y):
        S = N - min(zp, N)
        return zb + ldrow(S, y, S, xc)

    def next_base(zb, zp):
        S = N - zp
        return zb if zp >= N else zb + (S + 1) * (S + 2) // 2

    lb = slice_base(N, z0 - 1) if z0 > 0 else 0
    lz = max(z0 - 1, 0)
    for i in range(5):
        for j in range(PR + 2):
            out.append(ld(lb, lz, y0 - 1 + j))
        if z0 - 1 + i >= 0:
            lb = next_base(lb, lz)
            lz = min(lz + 1, N)
    zb = slice_base(N, z0)
    if with_b:
        for j in range(PR):
            out.append(ld(zb, z0, y0 + j))
    for k in range(PZ):
        z = z0 + k
        zb1 = next_base(zb, min(z, N))
        if with_b and k + 1 < PZ:
            for j in range(PR):
                out.append(ld(zb1, z + 1, y0 + j))
        for j in range(PR + 2):
            out.append(ld(lb, lz, y0 - 1 + j))
        lb = next_base(lb, lz)
        lz = min(lz + 1, N)
        zb = zb1
    return out


def pencils(N, PR, PZ):
    return [(x0, y0, z0) for z0 in range(0, N + 1, PZ) for y0 in range(0, N + 1 - z0, PR)
            for x0 in range(0, N + 1 - y0 - z0, W62)]


def check_3d(N, PR, PZ, tiles, with_b=True):
    P = tet_count(N + 1)
    for x0, y0, z0 in tiles:
        for off in loads_pencil3d(x0, y0, z0, N, PR, PZ, with_b):
            assert (off >= 0).all() and (off < P).all(), (N, x0, y0, z0)


@pytest.mark.parametrize("L", range(0, 10))
@pytest.mark.parametrize("H,U", [(8, 8), (16, 8)])  # FP64 and FP32 tiles
def test_2d_walk_every_tile_small_levels(L, H, U):
    N = 1 << L
    assert check_2d(N, H, U, tiles2d(N, H)) > 0


@pytest.mark.parametrize("L", [14, 15])
@pytest.mark.parametrize("H,U", [(8, 8), (16, 8)])
def test_2d_walk_apex_and_hypotenuse_tiles_large_levels(L, H, U):
    N = 1 << L
    tl = [(x0, y0) for (x0, y0) in tiles2d(N, H) if y0 >= N - 256 or x0 + y0 >= N - W62 - H - 2 or x0 == 0]
    assert len(tl) > 1000
    check_2d(N, H, U, tl)


@pytest.mark.parametrize("L", range(0, 9))
def test_3d_walk_every_pencil_small_levels(L):
    """Pencils of 4 rows x 8 slices (the library uses them from N = 256 on;
    the index arithmetic is replayed at every level up to that one)."""
    N = 1 << L
    check_3d(N, 4, 8, pencils(N, 4, 8))


def test_3d_walk_apex_and_far_face_pencils_level_11():
    N = 1 << 11
    tl = [(x0, y0, z0) for z0 in range(0, N + 1, 8) for y0 in range(0, N + 1 - z0, 4)
          for x0 in range(0, N + 1 - y0 - z0, W62)
          if z0 >= N - 64 or y0 + z0 >= N - 64
          or (x0 + y0 + z0 >= N - W62 - 16 and y0 % 128 == 0 and z0 % 128 == 0)]
    assert len(tl) > 1000
    check_3d(N, 4, 8, tl)


def test_replay_catches_an_unclamped_apex_row():
    """The replay has teeth: without the clamp of the row into the triangle
    (the cause of an earlier out-of-bounds load), the apex tile of level 14
    reads past the macro."""
    N = 1 << 14
    x0, y0 = 0, N - N % 8  # the band holding the apex row
    xc = np.maximum(x0 - 1 + LANES, 0)
    y1 = min(y0 + 8, N - x0 + 1)
    r = y0 + 1 + 7  # a ring row past the apex
    rr = min(max(r, 0), y1)  # the row clamped to `last` only
    col = np.minimum(xc, N - rr)  # negative bound: N - rr = -1
    offsets = rs32(N, rr) + (col.astype(np.int64) & 0xFFFFFFFF)  # the column offset is unsigned
    assert (offsets >= tri_points(N)).any()


# ---------------------------------------------------------------- slice runs
# The 3D run kernel (seg3d, levels up to N = 128): a wave takes up to 4 x 64
# consecutive points of one slice; each lane decodes its (x, y) and forms its
# 15 neighbour indices from its own index, relative to the first point of
# slice z - 1 (slice 0 at z = 0), clamped into the three slices around z
# unless 1 <= z <= N - 2.
OFF3 = [(0, 0, -1), (1, 0, -1), (0, 1, -1), (-1, 1, -1), (0, -1, 0), (1, -1, 0), (-1, 0, 0), (0, 0, 0),
        (1, 0, 0), (-1, 1, 0), (0, 1, 0), (0, -1, 1), (1, -1, 1), (-1, 0, 1), (0, 0, 1)]


def seg_xy(S, r, ulp=0):
    """The kernel's decode, in FP32.  numpy's float32 root is correctly
    rounded; the hardware root may be one ulp off, which ulp = -1 / +1
    replays."""
    b = np.float32(2 * S + 3)
    disc = (b * b - np.float32(8) * r.astype(np.float32)).astype(np.float32)
    root = np.sqrt(disc)
    if ulp:
        root = np.nextafter(root, np.float32(np.inf if ulp > 0 else -np.inf)).astype(np.float32)
    yy = ((b - root) * np.float32(0.5)).astype(np.int64)
    yy = np.clip(yy, 0, S)
    yy = np.where(rs32(S, yy) > r, yy - 1, yy)
    up = (yy < S) & (rs32(S, np.minimum(yy + 1, S)) <= r)
    yy = np.where(up, yy + 1, yy)
    return r - rs32(S, yy), yy


def seg_indices(N, z, r):
    """Neighbour indices (relative to the anchor slice) of slice-local points r."""
    S = N - z
    Ts = (S + 1) * (S + 2) // 2
    Tb = (S + 2) * (S + 3) // 2 if z > 0 else 0
    za = max(z - 1, 0)
    hi = min(tet_count(N + 1) - slice_base(N, za) - 1, Tb + 2 * Ts)
    x, y = seg_xy(S, r)
    d = S + 1 - y
    p = Tb + r
    pu = p + Ts - y
    pd = r + y
    idx = np.stack([pd, pd + 1, pd + d + 1, pd + d, p - d - 1, p - d, p - 1, p, p + 1, p + d - 1, p + d,
                    pu - d, pu - d + 1, pu - 1, pu])
    if not (1 <= z <= N - 2):
        idx = np.clip(idx, 0, hi)
    return x, y, idx, slice_base(N, za)


def check_runs(N):
    P = tet_count(N + 1)
    for z in range(N + 1):
        S = N - z
        Ts = (S + 1) * (S + 2) // 2
        r = np.arange(Ts, dtype=np.int64)
        x, y, idx, a = seg_indices(N, z, r)
        assert (x >= 0).all() and (x + y <= S).all()
        assert np.array_equal(rs32(S, y) + x, r), (N, z)  # the decode is exact
        for u in (-1, 1):
            xu, yu = seg_xy(S, r, u)
            assert np.array_equal(xu, x) and np.array_equal(yu, y), (N, z, u)
        absidx = a + idx
        assert (absidx >= 0).all() and (absidx < P).all(), (N, z)
        assert (idx >= 0).all() and (idx.astype(np.int64) * 8 < 2 ** 32).all()  # unsigned 32-bit byte offsets
        for o, (dx, dy, dz) in enumerate(OFF3):
            nx, ny, nz = x + dx, y + dy, z + dz
            ins = (nx >= 0) & (ny >= 0) & (nz >= 0) & (nx + ny + nz <= N)
            want = slice_base(N, nz) + rs32(N - nz, ny[ins]) + nx[ins] if nz <= N else None
            if ins.any():
                assert np.array_equal(absidx[o][ins], want), (N, z, o)
    return True


@pytest.mark.parametrize("L", range(1, 9))
def test_3d_runs_every_point_small_levels(L):
    """Every point of every slice: the decode is exact, every neighbour
    inside the macro gets its storage index, every index stays inside the
    macro's storage, byte offsets fit 32 bits."""
    assert check_runs(1 << L)


def test_3d_runs_level_11_edge_slices():
    """Level 11 (N = 2048, the largest supported 3D level): the slices where
    the clamps act and a few in between, every point."""
    N = 1 << 11
    P = tet_count(N + 1)
    for z in [0, 1, 2, 3, 1024, N - 3, N - 2, N - 1, N]:
        S = N - z
        Ts = (S + 1) * (S + 2) // 2
        r = np.arange(Ts, dtype=np.int64)
        x, y, idx, a = seg_indices(N, z, r)
        assert np.array_equal(rs32(S, y) + x, r)
        for u in (-1, 1):
            xu, yu = seg_xy(S, r, u)
            assert np.array_equal(xu, x) and np.array_equal(yu, y), (z, u)
        assert ((a + idx) >= 0).all() and ((a + idx) < P).all()
        assert (idx >= 0).all() and (idx * 8 < 2 ** 32).all()
