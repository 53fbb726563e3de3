"""CPU model of the full-row fused kernel's schedule (k_stepR).

N time levels run as a pipeline down a chunk of rows, one barrier per row
step: level L computes row y = yb - (N-1) + it - 2(L-1) at step `it`, over
[yb - span, ye + span) with span = N - L. Level 1 pulls from the lattice;
levels above pull from LDS rings of the level below:

- c_y = -1 directions (pulled from row y + 1): 2 slots, s mod 2;
- c_y =  0 directions (row y):                2 slots, s mod 2;
- c_y = +1 directions (row y - 1):            3 slots, s mod 3;

where s is the step in which the level below wrote the row (the same step
count for every level, so the kernel's six-step unrolled loops name every
slot by a constant);

a level writes direction i of column c at LDS column (c + c_ix) mod nx,
so every pull reads the puller's own column; the c_y >= 0 pulls of the next
row are read one step ahead (for the first row, in the step before it), the
c_y = -1 pulls in the row's own step. Lanes past the lattice take its last
column. The model checks that every read finds the value it names, that no
slot is read and written in the same step (the kernel has no barrier
between them), that every output node is written once, and that the result
equals N plain periodic BGK steps (Eqs. bgkCollision, equilibrium).
"""
import numpy as np
import pytest

CX = [0, 1, 0, -1, 0, 1, -1, -1, 1]
CY = [0, 0, 1, 0, -1, 1, 1, -1, -1]
GJ = [0, 1, 0, 2, 0, 1, 2, 1, 2]  # direction-row of a direction within its group
W = np.array([4 / 9] + [1 / 9] * 4 + [1 / 36] * 4)


def collide(f, omega):
    rho = f.sum(0)
    ux = sum(CX[i] * f[i] for i in range(9)) / rho
    uy = sum(CY[i] * f[i] for i in range(9)) / rho
    out = np.empty_like(f)
    for i in range(9):
        cu = 3 * (CX[i] * ux + CY[i] * uy)
        feq = W[i] * rho * (1 + cu + 0.5 * cu * cu - 1.5 * (ux * ux + uy * uy))
        out[i] = f[i] + omega * (feq - f[i])
    return out


def plain_steps(f, omega, n):
    for _ in range(n):
        g = np.stack([np.roll(np.roll(f[i], CY[i], 0), CX[i], 1) for i in range(9)])
        f = collide(g, omega)
    return f


def slot(level, r, i, col, y0):
    """LDS location of row r, direction i, column col of ring `level` (the
    output of level + 1), in a chunk whose level 1 starts at row y0: the row
    is written in step r - y0 + 2 level."""
    s = r - y0 + 2 * level
    assert s >= 0
    if CY[i] < 0:
        return (level, s % 2, GJ[i], col)
    if CY[i] == 0:
        return (level, 2 + s % 2, GJ[i], col)
    return (level, 4 + s % 3, GJ[i], col)


def run_schedule(nx, ny, n_lvl, rows, lanes, omega=1.3, seed=0):
    rg = n_lvl - 1
    h = max(8, min(rows, ny))
    rng = np.random.default_rng(seed)
    src = 1 / 9 + 0.01 * rng.standard_normal((9, ny, nx))
    dst = np.full((9, ny, nx), np.nan)
    count = np.zeros((ny, nx), int)
    for yb in range(0, ny, h):
        ye = min(ny, yb + h)
        lds, tag, ahead = {}, {}, {}
        for it in range(ye - yb + 3 * rg):
            reads, writes = set(), []

            def read(level, lane, c, i, r):
                # pull of direction i for row r of `level`: row r - c_y of the
                # level below, at the lane's own column
                key = slot(level - 2, r - CY[i], i, c, yb - rg)
                # the kernel's slots in step it: (it + 1) mod 2, (it + 1) mod 3
                assert key[1] == [(it + 1) % 2, 2 + (it + 1) % 2, 4 + (it + 1) % 3][CY[i] + 1]
                assert tag.get(key) == (r - CY[i], (c - CX[i]) % nx, i), (level, it, lane, i, r)
                reads.add(key)
                return lds[key]

            for level in range(1, n_lvl + 1):
                span = rg - (level - 1)
                y = yb - rg + it - 2 * (level - 1)
                y_lo, y_hi = yb - span, ye + span
                for lane in range(lanes):
                    c = min(lane, nx - 1)
                    if level > 1 and y == y_lo - 1:  # the first row's read-ahead
                        ahead[(level, lane, y + 1)] = {i: read(level, lane, c, i, y + 1)
                                                       for i in range(9) if CY[i] >= 0}
                    if not y_lo <= y < y_hi:
                        continue
                    if level == 1:
                        f = np.array([src[i, (y - CY[i]) % ny, (c - CX[i]) % nx] for i in range(9)])
                    else:
                        f = np.empty(9)
                        got = ahead.pop((level, lane, y))
                        for i in range(9):
                            f[i] = read(level, lane, c, i, y) if CY[i] < 0 else got[i]
                        if y + 1 < y_hi:
                            ahead[(level, lane, y + 1)] = {i: read(level, lane, c, i, y + 1)
                                                           for i in range(9) if CY[i] >= 0}
                    g = collide(f[:, None], omega)[:, 0]
                    if level < n_lvl:
                        writes += [(slot(level - 1, y, i, (c + CX[i]) % nx, yb - rg), (y, c, i), g[i])
                                   for i in range(9)]
                        assert slot(level - 1, y, 0, 0, yb - rg)[1] == 2 + it % 2  # written in step it
                    else:
                        assert 0 <= y < ny
                        if lane < nx:
                            count[y, c] += 1
                        elif not np.isnan(dst[0, y, c]):
                            assert np.array_equal(dst[:, y, c], g)  # an idle lane: the same bits
                        dst[:, y, c] = g
            written = set()
            for key, t, v in writes:
                if key in written:
                    assert lds[key] == v and tag[key] == t  # idle lanes write the same value
                lds[key], tag[key] = v, t
                written.add(key)
            assert not written & reads, ("slot read and written in one step", it)
    assert (count == 1).all()
    return np.abs(dst - plain_steps(src, omega, n_lvl)).max()


@pytest.mark.parametrize("nx, ny, n_lvl, rows, lanes", [
    (20, 12, 6, 8, 64),    # several chunks, idle lanes
    (3, 5, 5, 8, 64),      # every column wraps
    (17, 9, 7, 8, 64),     # 7 levels
    (5, 3, 8, 8, 64),      # 8 levels on 3 rows: rows wrap more than once
    (70, 13, 4, 8, 128),   # two waves of columns
    (1, 4, 6, 8, 64),      # one column: every direction lands on it
    (4, 1, 5, 8, 64),      # one row: every pull wraps to it
])
def test_row_pipeline_schedule(nx, ny, n_lvl, rows, lanes):
    assert run_schedule(nx, ny, n_lvl, rows, lanes) < 1e-14
