"""CPU check of the source indices that the scalar-row and row-wave gathers
form (D2Q9), against the general node geometry of the one-node-per-thread
kernels, before any of them runs on a GPU.

The general form (node_geometry + gather): node n = y nx + x, neighbour
offsets om/op per axis with periodic wrap, source index n + sum of the
offsets for the components of c_k (pull: x - c_k; transposed: x + c_k).
The scalar-row forms: source row y -/+ c_y chosen from three wave-uniform
rows, source column x -/+ c_x from three per-lane columns.  Every index
must be equal and inside the grid, for every tile shape, tile, lane and row,
on grids from 1 x 1 up (narrower and lower than a tile included).
"""
import pytest

CX = [0, 1, 0, -1, 0, 1, -1, -1, 1]
CY = [0, 0, 1, 0, -1, 1, 1, -1, -1]
TILE_W = 62   # interior columns of a 64-lane tile


def wrap(v, n):
    if v < 0:
        v += n
    while v >= n:
        v -= n
    return v


def general_index(n, nx, ny, k, sign):
    """Source index of population k at node n by the node geometry: sign = -1
    for the pull gather (x - c_k), +1 for the transposed gather (x + c_k)."""
    y = n // nx
    x = n - y * nx
    om = [nx - 1 if x == 0 else -1, (ny - 1) * nx if y == 0 else -nx]
    op = [-(nx - 1) if x == nx - 1 else 1, -(ny - 1) * nx if y == ny - 1 else nx]
    off = 0
    for a, c in enumerate((CX[k], CY[k])):
        c = -c if sign > 0 else c   # x + c is the pull form of -c
        off += om[a] if c == 1 else (op[a] if c == -1 else 0)
    return n + off


def three(v, n):
    """Periodic v - 1, v, v + 1, indexed by d + 1 for the coordinate v + d."""
    return [n - 1 if v == 0 else v - 1, v, 0 if v == n - 1 else v + 1]


def row_form_index(x, y, nx, ny, k, sign):
    cols, rows = three(x, nx), three(y, ny)
    return rows[1 + sign * CY[k]] * nx + cols[1 + sign * CX[k]]


def shared_rows_first(j, tr, nw):
    """Row of slot j = wave + pass * nw of a two-sweep adjoint tile of tr rows:
    with several rows per wave the four rows shared with the neighbouring
    tiles come first."""
    if tr // nw == 1 or j < 2:
        return j
    return tr - 4 + j if j < 4 else j - 2


@pytest.mark.parametrize("tr,nw", [(8, 4), (8, 8), (12, 4), (16, 4), (16, 8), (16, 16), (12, 6), (4, 4), (8, 2)])
def test_shared_rows_first_is_a_permutation(tr, nw):
    rows = [shared_rows_first(wv + i * nw, tr, nw) for wv in range(nw) for i in range(tr // nw)]
    assert sorted(rows) == list(range(tr))
    if tr // nw > 1 and nw >= 4:
        assert sorted(shared_rows_first(wv, tr, nw) for wv in range(4)) == [0, 1, tr - 2, tr - 1]


SIZES = [(a, b) for a in (1, 2, 3, 61, 62, 63, 64, 65) for b in (1, 2, 3, 7, 14, 15, 17)] + [(130, 33)]


@pytest.mark.parametrize("th,nw", [(14, 8), (14, 4), (10, 6), (6, 4), (6, 8), (14, 16)])
def test_two_step_phase1_rows(th, nw):
    """Phase 1 of a two-step tile (64 lanes x th + 2 rows from (x0 - 1, y0 - 1),
    coordinates wrapped), pull gather."""
    tr = th + 2
    for nx, ny in SIZES:
        for ty in range((ny + th - 1) // th):
            for tx in range((nx + TILE_W - 1) // TILE_W):
                x0, y0 = tx * TILE_W, ty * th
                for lane in range(64):
                    xg = wrap(x0 - 1 + lane, nx)
                    for wv in range(nw):
                        for i in range(tr // nw):
                            yg = wrap(y0 - 1 + wv + i * nw, ny)
                            n = yg * nx + xg
                            for k in range(9):
                                got = row_form_index(xg, yg, nx, ny, k, -1)
                                assert got == general_index(n, nx, ny, k, -1)
                                assert 0 <= got < nx * ny


@pytest.mark.parametrize("th,nw", [(6, 4), (10, 4), (10, 12)])
def test_two_sweep_adjoint_rows(th, nw):
    """Both phases of the two-sweep adjoint tile (nw waves): phase 1 gathers
    the forward state (pull) and psi (transposed) on the tile and halo; phase 2
    gathers the forward state at the tile's own nodes."""
    tr = th + 2
    for nx, ny in SIZES:
        for ty in range((ny + th - 1) // th):
            for tx in range((nx + TILE_W - 1) // TILE_W):
                x0, y0 = tx * TILE_W, ty * th
                for lane in range(64):
                    xg = wrap(x0 - 1 + lane, nx)
                    own = 1 <= lane <= TILE_W and x0 + lane - 1 < nx
                    for wv in range(nw):
                        for i in range(tr // nw):
                            yg = wrap(y0 - 1 + shared_rows_first(wv + i * nw, tr, nw), ny)
                            n = yg * nx + xg
                            for k in range(9):
                                for sign in (-1, 1):
                                    got = row_form_index(xg, yg, nx, ny, k, sign)
                                    assert got == general_index(n, nx, ny, k, sign)
                                    assert 0 <= got < nx * ny
                        if own:
                            assert x0 + lane - 1 == xg
                            r = 1 + wv
                            while r <= th and y0 + r - 1 < ny:
                                y = y0 + r - 1
                                n = y * nx + xg
                                for k in range(9):
                                    got = row_form_index(xg, y, nx, ny, k, -1)
                                    assert got == general_index(n, nx, ny, k, -1)
                                    assert 0 <= got < nx * ny
                                r += nw


@pytest.mark.parametrize("nx", [64, 128, 192])
def test_adjoint_row_waves(nx):
    """One-sweep adjoint on widths that are multiples of 64: the 64 nodes of a
    wave share their row (taken from the wave's first node), both gathers."""
    for ny in (1, 2, 3, 5, 9):
        for n in range(nx * ny):
            nw = n & ~63
            y = nw // nx
            x = n - y * nx
            assert y == n // nx   # the wave's first node is in the lane's row
            for k in range(9):
                for sign in (-1, 1):
                    got = row_form_index(x, y, nx, ny, k, sign)
                    assert got == general_index(n, nx, ny, k, sign)
                    assert 0 <= got < nx * ny


OPP9 = [0, 3, 4, 1, 2, 7, 8, 5, 6]


@pytest.mark.parametrize("th,nw", [(14, 8), (14, 4), (10, 6), (6, 4), (6, 8), (14, 16)])
def test_two_step_walls_schedule(th, nw):
    """The D2Q9 two-step tile with anti-bounce-back walls at both ends of y
    (x periodic): phase 1 computes only the rows inside the walls and loads,
    for a population that would come from beyond a wall, the node's own
    opposite population; phase 2 gathers every population from the LDS cell
    of the node it comes from, or from the node's own cell for the wall form.
    Every such source must be what the one-sweep gather reads, every LDS cell
    read must have been written, and every node is stored once."""
    for nx, ny in SIZES:
        stored = set()
        tiles_x, tiles_y = (nx + TILE_W - 1) // TILE_W, (ny + th - 1) // th
        for ty in range(tiles_y):
            for tx in range(tiles_x):
                x0, y0 = tx * TILE_W, ty * th
                lds = {}
                # phase 1
                for wv in range(nw):
                    for i in range((th + 2) // nw):
                        r = wv + i * nw
                        yl = y0 - 1 + r
                        if yl < 0 or yl >= ny:
                            continue
                        for lane in range(64):
                            xg = wrap(x0 - 1 + lane, nx)
                            for k in range(9):
                                wl = (CY[k] == 1 and yl == 0) or (CY[k] == -1 and yl == ny - 1)
                                src = (xg, yl) if wl else (wrap(xg - CX[k], nx), yl - CY[k])
                                assert 0 <= src[0] < nx and 0 <= src[1] < ny
                            lds[(r, lane)] = (xg, yl)
                # phase 2
                for wv in range(nw):
                    r = 1 + wv
                    while r <= th:
                        y = y0 + r - 1
                        if y >= ny:
                            break
                        for lane in range(1, TILE_W + 1):
                            x = x0 + lane - 1
                            for k in range(9):
                                wl = (CY[k] == 1 and y == 0) or (CY[k] == -1 and y == ny - 1)
                                if wl:
                                    got = ("wall", OPP9[k], lds[(r, lane)])
                                    want = ("wall", OPP9[k], (wrap(x, nx), y))
                                else:
                                    cell = lds.get((r - CY[k], lane - CX[k]))
                                    assert cell is not None, (nx, ny, tx, ty, r, lane, k)
                                    got = ("f*", k, cell)
                                    want = ("f*", k, (wrap(wrap(x, nx) - CX[k], nx), y - CY[k]))
                                assert got == want, (nx, ny, th, nw, x, y, k, got, want)
                            if x < nx:
                                assert (x, y) not in stored
                                stored.add((x, y))
                        r += nw
        assert len(stored) == nx * ny
