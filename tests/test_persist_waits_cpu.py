"""Host check of the reasoning behind the many-steps kernel's waits.

Before its step s a tile waits for the step counters of its neighbouring
tiles: every tile within one tile of it (x periodic; y periodic or closed by
walls), or every tile of its replica when a ragged tail is one node thick.
That is enough if each tile U that, in step s - 1, writes a node the tile
reads in step s (its own nodes and their one-node ring, for phi) or reads a
node the tile overwrites in step s (its push destinations) is in that set.
This test builds those read and write sets node by node for the push scheme
of the two-phase step (ring reads with periodic wrap or the wall mirror, push
writes with periodic wrap or halfway bounce-back) and checks the rule on
every grid and tile size in a small range, thin tails included."""
import itertools

import pytest


def _tiles(nx, ny, tx, ty):
    gx, gy = -(-nx // tx), -(-ny // ty)
    return gx, gy, {(bx, by): {(x, y) for x in range(bx * tx, min(nx, (bx + 1) * tx))
                               for y in range(by * ty, min(ny, (by + 1) * ty))}
                    for bx in range(gx) for by in range(gy)}


def _reads(nodes, nx, ny, walls):
    out = set()
    for x, y in nodes:
        for dx, dy in itertools.product((-1, 0, 1), repeat=2):
            yy = y + dy
            if walls:
                yy = min(max(yy, 0), ny - 1)  # mirror ghost: the boundary row itself
            out.add(((x + dx) % nx, yy % ny))
    return out


def _writes(nodes, nx, ny, walls):
    out = set()
    for x, y in nodes:
        for dx, dy in itertools.product((-1, 0, 1), repeat=2):
            yy = y + dy
            if walls and not 0 <= yy < ny:
                out.add((x, y))  # halfway bounce-back: back into the node itself
            else:
                out.add(((x + dx) % nx, yy % ny))
    return out


def _watched(b, gx, gy, nx, ny, tx, ty, walls):
    thin = (gx > 1 and nx - (gx - 1) * tx < 2) or (gy > 1 and ny - (gy - 1) * ty < 2)
    bx, by = b
    out = set()
    for u in itertools.product(range(gx), range(gy)):
        if u == b:
            continue
        ddx = min(abs(u[0] - bx), gx - abs(u[0] - bx))
        ddy = abs(u[1] - by) if walls else min(abs(u[1] - by), gy - abs(u[1] - by))
        if thin or (ddx <= 1 and ddy <= 1):
            out.add(u)
    return out


@pytest.mark.parametrize("walls", [False, True])
@pytest.mark.parametrize("tx,ty", [(2, 2), (2, 3), (3, 2), (4, 4), (3, 5)])
def test_neighbour_waits_cover_every_dependency(tx, ty, walls):
    for nx, ny in itertools.product(range(1, 14), range(1, 14)):
        gx, gy, tiles = _tiles(nx, ny, tx, ty)
        R = {b: _reads(n, nx, ny, walls) for b, n in tiles.items()}
        W = {b: _writes(n, nx, ny, walls) for b, n in tiles.items()}
        for b in tiles:
            need = {u for u in tiles if u != b and (W[u] & R[b] or R[u] & W[b])}
            missing = need - _watched(b, gx, gy, nx, ny, tx, ty, walls)
            assert not missing, (nx, ny, b, sorted(missing))


def test_a_one_node_tail_needs_the_wider_wait():
    """Without the thin-tail rule a one-row last tile lets tiles two apart
    depend on each other (the check above would fail)."""
    nx, ny, tx, ty, walls = 4, 13, 4, 4, False  # rows 0-3, 4-7, 8-11, 12
    gx, gy, tiles = _tiles(nx, ny, tx, ty)
    R = {b: _reads(n, nx, ny, walls) for b, n in tiles.items()}
    W = {b: _writes(n, nx, ny, walls) for b, n in tiles.items()}
    b = (0, 0)
    need = {u for u in tiles if u != b and (W[u] & R[b] or R[u] & W[b])}
    assert (0, 2) in need  # two tiles away, reached through the one-row tile (0, 3)
