"""CPU emulation of the D3Q19 two-step pass (k_sweep2_3d) before it runs on a
GPU: the schedule of the LDS ring and every index it forms.

A workgroup owns a column of 62 x TY nodes (64 lanes with a one-lane halo on
each side, TY + 2 rows with a one-row halo) and a chunk of ZC planes, and
marches up the chunk.  At logical plane i (z = z0 - 1 + i) phase 1 runs step
t on the column with its halo and writes the post-collision populations to
the ring, split by the z component of their velocity: c_z = 0 and c_z = -1
into slot i & 1, c_z = +1 kept in registers and written to slot i & 1 after
phase 2 (whose reads of slot i & 1 still need plane i - 2).  Phase 2 runs
step t + 1 on plane i - 1 of the column's own nodes, gathering c_z = +1 from
plane i - 2, c_z = 0 from plane i - 1 and c_z = -1 from plane i; at a wall
the populations that come from beyond it are -f*_opp of the node itself plus
the wall term.

The emulation tracks symbolic contents (which plane's, row's and lane's
population sits in every ring cell) and checks, for grids from 1 x 1 x 1 up,
with and without walls, for every tile shape and chunk length:
  * every phase-2 gather gets exactly the value a single sweep's gather would
    read from the intermediate state (pull, periodic x and y, walls or
    periodic z);
  * every global index is inside the grid and every node is stored once;
  * no ring cell is read before it is written in the right iteration.
"""
import itertools

import pytest

# Eq. 6 velocities
C = [(0, 0, 0), (1, 0, 0), (-1, 0, 0), (0, 1, 0), (0, -1, 0), (0, 0, 1), (0, 0, -1),
     (1, 1, 0), (-1, -1, 0), (1, -1, 0), (-1, 1, 0), (1, 0, 1), (-1, 0, -1), (-1, 0, 1), (1, 0, -1),
     (0, 1, 1), (0, -1, -1), (0, 1, -1), (0, -1, 1)]
OPP = [C.index((-a, -b, -c)) for a, b, c in C]
TILE_W = 62


def wrap(v, n):
    if v < 0:
        v += n
    while v >= n:
        v -= n
    return v


def single_sweep_gather(x, y, z, k, nx, ny, nz, wall):
    """What the one-sweep gather reads for population k at (x, y, z) from the
    state after step t: f*_k at the source node (x - c_k), or the wall form."""
    cx, cy, cz = C[k]
    if wall and ((cz == 1 and z == 0) or (cz == -1 and z == nz - 1)):
        return ("wall", 0 if cz == 1 else 1, OPP[k], (x, y, z))
    return ("f*", k, (wrap(x - cx, nx), wrap(y - cy, ny), wrap(z - cz, nz)))


def emulate(nx, ny, nz, wall, ty, nw, zc):
    tr = ty + 2
    tiles_x, tiles_y, tiles_z = (nx + TILE_W - 1) // TILE_W, (ny + ty - 1) // ty, (nz + zc - 1) // zc
    stored = {}
    for tz, tyi, tx in itertools.product(range(tiles_z), range(tiles_y), range(tiles_x)):
        x0, y0, z0 = tx * TILE_W, tyi * ty, tz * zc
        zend = min(z0 + zc, nz)
        ring_p = [[[None] * 64 for _ in range(tr)] for _ in range(2)]   # c_z = +1, per pop implied
        ring_0 = [[[None] * 64 for _ in range(tr)] for _ in range(2)]
        ring_m = [[[None] * 64 for _ in range(tr)] for _ in range(2)]
        for i in range(zend - z0 + 2):
            zl = z0 - 1 + i
            # phase 1
            regs = {}
            p1 = (0 <= zl < nz) if wall else True
            zg = zl if wall else wrap(zl, nz)
            for wv in range(nw):
                for r in range(wv, tr, nw):
                    yg = wrap(y0 - 1 + r, ny)
                    for lane in range(64):
                        xg = wrap(x0 - 1 + lane, nx)
                        if p1:
                            node = (xg, yg, zg)
                            assert 0 <= xg < nx and 0 <= yg < ny and 0 <= zg < nz
                            ring_0[i & 1][r][lane] = ("plane", node)
                            ring_m[i & 1][r][lane] = ("plane", node)
                            regs[(r, lane)] = ("plane", node)
            # phase 2 (plane i - 1)
            if i >= 2:
                zc2 = zl - 1
                assert z0 <= zc2 < zend
                lo, hi = wall and zc2 == 0, wall and zc2 == nz - 1
                for wv in range(nw):
                    for r in range(1 + wv, ty + 1, nw):
                        for lane in range(1, TILE_W + 1):
                            x, y = x0 + lane - 1, y0 + r - 1
                            if not (x < nx and y < ny):
                                continue
                            for k in range(19):
                                cx, cy, cz = C[k]
                                if (cz == 1 and lo) or (cz == -1 and hi):
                                    ring = ring_m if cz == 1 else ring_p
                                    cell = ring[(i - 1) & 1][r][lane]
                                    assert cell is not None
                                    got = ("wall", 0 if cz == 1 else 1, OPP[k], cell[1])
                                else:
                                    ring = ring_p if cz == 1 else (ring_m if cz == -1 else ring_0)
                                    slot = (i & 1) if cz != 0 else ((i - 1) & 1)
                                    cell = ring[slot][r - cy][lane - cx]
                                    assert cell is not None, (k, r, lane, i)
                                    got = ("f*", k, cell[1])
                                want = single_sweep_gather(x, y, zc2, k, nx, ny, nz, wall)
                                assert got == want, (nx, ny, nz, wall, ty, zc, (x, y, zc2), k, got, want)
                            key = (x, y, zc2)
                            assert key not in stored
                            stored[key] = True
            # the c_z = +1 populations of plane i after phase 2
            for (r, lane), v in regs.items():
                ring_p[i & 1][r][lane] = v
    assert len(stored) == nx * ny * nz


SHAPES = [(14, 16), (6, 8), (2, 4), (6, 4), (4, 6)]
GRIDS = [(1, 1, 1), (2, 1, 3), (3, 2, 2), (5, 4, 7), (61, 3, 4), (63, 7, 5), (64, 6, 3), (65, 13, 9), (130, 5, 4)]


@pytest.mark.parametrize("ty,nw", SHAPES)
@pytest.mark.parametrize("wall", [True, False])
def test_two_step_3d_schedule(ty, nw, wall):
    for (nx, ny, nz), zc in itertools.product(GRIDS, (1, 2, 3, 8)):
        emulate(nx, ny, nz, wall, ty, nw, zc)


def general_index3(n, nx, ny, nz, k):
    """Pull source index of population k at node n by the node geometry of the
    one-sweep kernels (periodic wrap on every axis; the wall case is handled
    before the index is used)."""
    xy = nx * ny
    z = n // xy
    y = (n - z * xy) // nx
    x = n - z * xy - y * nx
    om = [nx - 1 if x == 0 else -1, (ny - 1) * nx if y == 0 else -nx, (nz - 1) * xy if z == 0 else -xy]
    op = [-(nx - 1) if x == nx - 1 else 1, -(ny - 1) * nx if y == ny - 1 else nx,
          -(nz - 1) * xy if z == nz - 1 else xy]
    off = 0
    for a, c in enumerate(C[k]):
        off += om[a] if c == 1 else (op[a] if c == -1 else 0)
    return n + off


def three(v, n):
    return [n - 1 if v == 0 else v - 1, v, 0 if v == n - 1 else v + 1]


@pytest.mark.parametrize("wall", [True, False])
def test_two_step_3d_phase1_offsets(wall):
    """Phase 1 gathers from a wave-uniform source row offset (plane z - c_z and
    row y - c_y, periodic, as (z ny + y) nx elements) plus one of three per-lane
    column offsets (x - c_x, periodic): every index equals the node
    geometry's and lies inside the grid; at a wall the own node's index."""
    for (nx, ny, nz) in GRIDS + [(62, 1, 2), (128, 3, 3)]:
        for zg in range(nz):
            zs = three(zg, nz)
            for yg in range(ny):
                ys = three(yg, ny)
                rows = {(dy, dz): (zs[1 + dz] * ny + ys[1 + dy]) * nx for dy in (-1, 0, 1) for dz in (-1, 0, 1)}
                for xg in range(nx):
                    cols = three(xg, nx)
                    n = (zg * ny + yg) * nx + xg
                    for k in range(19):
                        cx, cy, cz = C[k]
                        if wall and ((cz == 1 and zg == 0) or (cz == -1 and zg == nz - 1)):
                            idx = rows[(0, 0)] + cols[1]
                            assert idx == n
                        else:
                            idx = rows[(-cy, -cz)] + cols[1 - cx]
                            assert idx == general_index3(n, nx, ny, nz, k)
                        assert 0 <= idx < nx * ny * nz
