"""CPU model of the strip window kernel's schedule (k_stepW).

N time levels, one wave each, run as a pipeline down a chunk of rows of a
strip of W <= 64 - 2(N - 1) columns, one barrier per iteration: level L
computes row y = yb - (N-1) + it - 2(L-1) at iteration `it`, over
[yb - span, ye + span) and the strip's columns widened by span = N - L on
each side (lane l holds global column x0 - span + l, LDS column l + L - 1).
Level 1 pulls from the lattice; levels above pull direction i from LDS
column lc - c_ix of the ring the level below wrote, by the group of its
c_y, each group a ring of rows named by the row r (offset by 12, a
multiple of 2, 3 and 4, to keep slots positive):

- c_y = -1 (read one iteration after it is written): 2 rows, (r + 12) mod 2;
- c_y =  0 (two iterations after):                   3 rows, (r + 12) mod 3;
- c_y = +1 (three iterations after):                 4 rows, (r + 12) mod 4;

so that the level computing row y reads slots (y + 13) mod 2, (y + 12)
mod 3 and (y + 11) mod 4, the kernel's expressions. The model checks that every
read finds the row, column and direction it expects, that no slot is read
and written in the same iteration (no barrier between them), that every
output node is written once, and that the result equals N plain periodic
BGK steps (Eqs. bgkCollision, equilibrium).
"""
import numpy as np
import pytest

from test_row_pipeline_schedule import CX, CY, GJ, collide, plain_steps


def write_slot(i, r):
    """group and slot of row r's direction i in the ring it is written to"""
    return [("a", (r + 12) % 2), ("b", (r + 12) % 3), ("c", (r + 12) % 4)][CY[i] + 1]


def read_slot(i, y):
    """group and slot the level computing row y reads direction i from"""
    return [("a", (y + 13) % 2), ("b", (y + 12) % 3), ("c", (y + 11) % 4)][CY[i] + 1]


def strips_of(nx, n):
    wmax = 64 - 2 * (n - 1)
    strips = (nx + wmax - 1) // wmax
    return (nx + strips - 1) // strips, strips


def run_strips(nx, ny, n_lvl, rows, omega=1.2, seed=1):
    rg = n_lvl - 1
    h = max(8, min(rows, ny))
    W, strips = strips_of(nx, n_lvl)
    rng = np.random.default_rng(seed)
    src = 1 / 9 + 0.01 * rng.standard_normal((9, ny, nx))
    dst = np.full((9, ny, nx), np.nan)
    count = np.zeros((ny, nx), int)
    for strip in range(strips):
        x0 = strip * W
        w = min(W, nx - x0)
        for yb in range(0, ny, h):
            ye = min(ny, yb + h)
            lds, tag = {}, {}
            for it in range(ye - yb + 3 * rg):
                reads, writes = set(), []
                for level in range(1, n_lvl + 1):
                    span = rg - (level - 1)
                    y = yb - rg + it - 2 * (level - 1)
                    if not yb - span <= y < ye + span:
                        continue
                    for lane in range(64):
                        if lane >= w + 2 * span:
                            continue
                        gc = (x0 - span + lane) % nx
                        lc = lane + level - 1
                        assert 0 <= lc < 64
                        if level == 1:
                            f = np.array([src[i, (y - CY[i]) % ny, (gc - CX[i]) % nx] for i in range(9)])
                        else:
                            f = np.empty(9)
                            for i in range(9):
                                key = (level - 2, read_slot(i, y), GJ[i], lc - CX[i])
                                # row y - c_y of the level below, global column gc - c_x
                                assert tag.get(key) == (y - CY[i], (gc - CX[i]) % nx, i), (strip, yb, it, level, lane, i)
                                reads.add(key)
                                f[i] = lds[key]
                        g = collide(f[:, None], omega)[:, 0]
                        if level < n_lvl:
                            writes += [((level - 1, write_slot(i, y), GJ[i], lc), (y, gc, i), g[i]) for i in range(9)]
                        else:
                            assert span == 0 and lane < w and 0 <= y < ny
                            count[y, gc] += 1
                            dst[:, y, gc] = g
                written = set()
                for key, t, v in writes:
                    assert key not in written  # each LDS cell is written by one lane per iteration
                    lds[key], tag[key] = v, t
                    written.add(key)
                assert not written & reads, ("slot read and written in one iteration", it)
    assert (count == 1).all()
    return np.abs(dst - plain_steps(src, omega, n_lvl)).max()


@pytest.mark.parametrize("nx, ny, n_lvl, rows", [
    (70, 20, 4, 8),     # two strips, several chunks
    (5, 3, 4, 64),      # one narrow strip: every column and row wraps
    (130, 9, 3, 8),     # three strips at N = 3
    (64, 12, 2, 8),     # two levels
    (1, 4, 4, 8),       # one column
])
def test_window_strip_schedule(nx, ny, n_lvl, rows):
    assert run_strips(nx, ny, n_lvl, rows) < 1e-14
