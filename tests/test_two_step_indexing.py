"""CPU models of the two-step kernels' index arithmetic, checked against the one-step edge rule
and the launch sequence.  They restate, in Python, what step2_kernel / pool_tile compute for each
thread (the halo mapping of the first step, the LDS offsets of the second, the outlet lookups)
and what pool_buf counts, and check the invariants the kernels rely on: every LDS read is in
bounds and falls on a node the first step wrote, that node is the one the global rule
(edge_source) names, every lattice node is owned by exactly one tile, and the buffer pool_buf
names is the one the launch sequence leaves the state in."""
import itertools
import random

import pytest

CX = [0, 1, 0, -1, 0, 1, -1, -1, 1]
CY = [0, 0, 1, 0, -1, 1, 1, -1, -1]
MIRROR_Y = [0, 1, 4, 3, 2, 8, 7, 6, 5]


def edge_source(a, x, y, nx, ny, xper, yper):
    """The one-step kernel's source of direction a at node (x, y) (global coordinates)."""
    sx, sy, pa = x - CX[a], y - CY[a], a
    if sy < 0 or sy >= ny:
        if yper:
            sy += ny if sy < 0 else -ny
        else:
            sy, pa = y, MIRROR_Y[a]
    if sx < 0 or sx >= nx:
        if xper:
            sx += nx if sx < 0 else -nx
        else:
            sx = 0 if sx < 0 else nx - 1
    return sx, sy, pa


def tile_source(a, x, y, x0, y0, ew, nx, ny, xper, yper):
    """The two-step kernel's LDS element and plane for direction a of node (x, y)."""
    sx, sy, pa = x - CX[a], y - CY[a], a
    if (sy < 0 or sy >= ny) and not yper:
        sy, pa = y, MIRROR_Y[a]
    if (sx < 0 or sx >= nx) and not xper:
        sx = 0 if sx < 0 else nx - 1
    return (sy - y0 + 1) * ew + (sx - x0 + 1), pa


def first_step(nx, ny, xper, yper, x0, y0, tw, th, nthreads):
    """Phase 1: LDS element -> the global node it holds, and the tile's own nodes."""
    ew, en = tw + 2, (tw + 2) * (th + 2)
    written, own = {}, set()
    for it in range(-(-en // nthreads)):
        for tid in range(nthreads):
            e = tid + it * nthreads
            lx, ly = e % ew - 1, e // ew - 1
            ux, uy = x0 + lx, y0 + ly
            x, y, live = ux, uy, e < en
            if x < 0 or x >= nx:
                if xper and -1 <= x <= nx:
                    x += nx if x < 0 else -nx
                else:
                    live = False
            if y < 0 or y >= ny:
                if yper and -1 <= y <= ny:
                    y += ny if y < 0 else -ny
                else:
                    live = False
            if live:
                assert 0 <= x < nx and 0 <= y < ny
                written[e] = (x, y)
                if 0 <= lx < tw and 0 <= ly < th and ux < nx and uy < ny:
                    own.add((x, y))
    return written, own


def check_lattice(nx, ny, xper, yper, tw, th, nthreads=512, outlet=False):
    ew, en = tw + 2, (tw + 2) * (th + 2)
    ntx, nty = -(-nx // tw), -(-ny // th)
    owned = []
    for tile in range(ntx * nty):
        x0, y0 = (tile % ntx) * tw, (tile // ntx) * th
        written, own = first_step(nx, ny, xper, yper, x0, y0, tw, th, nthreads)
        owned += own
        if x0 >= 2 and x0 + tw + 2 <= nx and y0 >= 2 and y0 + th + 2 <= ny:
            # the kernels' interior fast path: no wrap, every first-step node pulls by plain
            # shifts (pull_interior), every second-step node too (pull_tile_shifts)
            assert len(written) == en
            assert all(0 < x < nx - 1 and 0 < y < ny - 1 for x, y in written.values())
        for j in range(tw * th):
            x, y = x0 + j % tw, y0 + j // tw
            if not (x < nx and y < ny):
                continue
            for a in range(9):
                idx, pa = tile_source(a, x, y, x0, y0, ew, nx, ny, xper, yper)
                assert 0 <= idx < en and idx in written, (nx, ny, x, y, a)
                assert (written[idx], pa) == (edge_source(a, x, y, nx, ny, xper, yper)[:2],
                                              edge_source(a, x, y, nx, ny, xper, yper)[2])
            if outlet and x == nx - 1:
                # the convective rule's neighbour: direction a of node (nx - 2, y)
                assert (x, y) in own
                for a in (3, 6, 7):
                    idx, pa = tile_source(a, nx - 2, y, x0, y0, ew, nx, ny, xper, yper)
                    sx, sy, spa = edge_source(a, nx - 2, y, nx, ny, xper, yper)
                    assert idx in written and written[idx] == (sx, sy) and pa == spa
    assert sorted(owned) == sorted((x, y) for x in range(nx) for y in range(ny))


SIZES = [(1, 1), (2, 3), (5, 7), (64, 8), (128, 8), (130, 9), (200, 17), (257, 31), (129, 1),
         (1, 20), (90, 60), (400, 40)]


@pytest.mark.parametrize("tw,th", [(128, 8), (64, 8), (128, 16)])
def test_second_step_reads_what_the_first_wrote(tw, th):
    for (nx, ny), xper, yper in itertools.product(SIZES, (0, 1), (0, 1)):
        check_lattice(nx, ny, xper, yper, tw, th)


@pytest.mark.parametrize("tw,th", [(128, 8), (64, 8), (128, 16)])
def test_convective_outlet_lookups(tw, th):
    for (nx, ny), yper in itertools.product([(2, 3), (5, 7), (129, 9), (150, 40), (257, 31)], (0, 1)):
        check_lattice(nx, ny, 0, yper, tw, th, outlet=True)


def pool_buf(done, spl, spk=2):
    """The pool's buffer after `done` steps (pool.hip): launches of spk steps counted per graph
    replay, what remains of a replay last."""
    launches = (done // spl) * (-(-spl // spk)) + -(-(done % spl) // spk)
    return launches & 1


@pytest.mark.parametrize("spk", [2, 3])
def test_pool_buffer_follows_the_launch_sequence(spk):
    """Replays of spl steps in launches of spk from the replay's start (what remains last), a
    request with fewer steps left than the launch taking those, and early stops that lower the
    target to a replay boundary + 1."""
    rng = random.Random(1)
    for spl in list(range(1, 12)) + [63, 64]:
        for _ in range(100):
            target = rng.randint(1, 5 * spl + 7)
            stop_at = rng.randint(1, max(1, target // spl)) * spl if rng.random() < 0.5 else None
            buf, done, tgt = 0, 0, target
            while done < tgt:
                for j in range(0, spl, spk):
                    if done >= tgt:
                        break
                    n = min(spk, spl - j)
                    k = min(n, tgt - done)
                    assert pool_buf(done, spl, spk) == buf
                    buf ^= 1
                    done += k
                    assert pool_buf(done, spl, spk) == buf
                if stop_at is not None and done == stop_at and tgt > done + 1:
                    tgt = done + 1


def tile_source_h(a, x, y, x0, y0, ew, nx, ny, xper, yper, h):
    """tile_source<H> of lattice.hpp: the LDS element and plane of direction a of node (x, y)
    (unwrapped coordinates) in a tile that starts h nodes before (x0, y0)."""
    sx, sy, pa = x - CX[a], y - CY[a], a
    if (sy < 0 or sy >= ny) and not yper:
        sy, pa = y, MIRROR_Y[a]
    if (sx < 0 or sx >= nx) and not xper:
        sx = 0 if sx < 0 else nx - 1
    return (sy - y0 + h) * ew + (sx - x0 + h), pa


def locate(ux, uy, h, nx, ny, xper, yper):
    """step3_kernel's locate: the lattice node at unwrapped (ux, uy), or None."""
    x, y = ux, uy
    if x < 0 or x >= nx:
        if xper and -h <= x < nx + h:
            x += nx if x < 0 else -nx
        else:
            return None
    if y < 0 or y >= ny:
        if yper and -h <= y < ny + h:
            y += ny if y < 0 else -ny
        else:
            return None
    return x, y


def check_lattice3(nx, ny, xper, yper, tw=64, th=14):
    """step3_kernel's three phases on every tile: phase 2 reads, at every pull, a slot phase 1 wrote
    with the node edge_source names (and writes its result back over its own node's slot), phase 3
    reads slots phase 2 wrote with the nodes edge_source names, the interior fast path holds only
    on tiles whose phase-1 nodes are all strictly inside, and every node is stored by one tile."""
    ew, en = tw + 4, (tw + 4) * (th + 4)
    mw, mn = tw + 2, (tw + 2) * (th + 2)
    ntx, nty = -(-nx // tw), -(-ny // th)
    owned = []
    for tile in range(ntx * nty):
        x0, y0 = (tile % ntx) * tw, (tile // ntx) * th
        inner = x0 >= 3 and x0 + tw + 3 <= nx and y0 >= 3 and y0 + th + 3 <= ny
        w1 = {}
        for e in range(en):
            ux, uy = x0 + e % ew - 2, y0 + e // ew - 2
            node = (ux, uy) if inner else locate(ux, uy, 2, nx, ny, xper, yper)
            if node is not None:
                assert 0 <= node[0] < nx and 0 <= node[1] < ny
                if inner:
                    assert 0 < ux < nx - 1 and 0 < uy < ny - 1
                w1[e] = node
        w2 = {}
        for j in range(mn):
            ux, uy = x0 + j % mw - 1, y0 + j // mw - 1
            node = (ux, uy) if inner else locate(ux, uy, 1, nx, ny, xper, yper)
            if node is None:
                continue
            x, y = node
            for a in range(9):
                idx, pa = tile_source_h(a, ux, uy, x0, y0, ew, nx, ny, xper, yper, 2)
                sx, sy, spa = edge_source(a, x, y, nx, ny, xper, yper)
                assert 0 <= idx < en and w1.get(idx) == (sx, sy) and pa == spa, (nx, ny, ux, uy, a)
            slot = (j // mw + 1) * ew + j % mw + 1
            assert slot == (uy - y0 + 2) * ew + (ux - x0 + 2) and w1[slot] == (x, y)
            w2[slot] = (x, y)
        for j in range(tw * th):
            x, y = x0 + j % tw, y0 + j // tw
            if not (x < nx and y < ny):
                continue
            owned.append((x, y))
            for a in range(9):
                idx, pa = tile_source_h(a, x, y, x0, y0, ew, nx, ny, xper, yper, 2)
                sx, sy, spa = edge_source(a, x, y, nx, ny, xper, yper)
                assert idx in w2 and w2[idx] == (sx, sy) and pa == spa, (nx, ny, x, y, a)
    assert sorted(owned) == sorted((x, y) for x in range(nx) for y in range(ny))


@pytest.mark.parametrize("tw,th", [(64, 14), (128, 6)])
@pytest.mark.parametrize("xper,yper", [(0, 0), (0, 1), (1, 0), (1, 1)])
def test_three_step_phases_read_what_the_previous_wrote(xper, yper, tw, th):
    for nx, ny in [(3, 3), (4, 5), (5, 7), (64, 14), (128, 6), (130, 9), (257, 13), (200, 17),
                   (131, 1 + 12), (390, 30), (135, 45)]:
        check_lattice3(nx, ny, xper, yper, tw, th)


def test_three_step_reduction_sets_are_distinct_and_folded_before_cleared():
    """The reduction sets of kernels.hip (kMaxSteps = 3, kAccSets = 16) over random mixes of 1-, 2-
    and 3-step launches: within a launch the folded, written and cleared sets are distinct; every
    step is folded by the next launch, after its own launch and before its set is cleared again;
    every set a launch writes was cleared after its previous use was folded."""
    max_steps, sets = 3, 16
    rng = random.Random(3)
    for _ in range(200):
        t = 0
        cleared_at = {}       # set -> launch index of its last clear
        written = {}          # step -> launch index
        folded = {}           # step -> first launch that folded it
        for li in range(60):
            n = rng.choice((1, 2, 3))
            fold = [t - 1 - d for d in range(max_steps) if t - 1 - d >= 0]
            write = list(range(t, t + n))
            clear = list(range(t + n, t + n + max_steps))
            ids = [s % sets for s in fold + write + clear]
            assert len(set(ids)) == len(ids)
            for s in fold:
                folded.setdefault(s, li)
                # not cleared since the step was written
                assert cleared_at.get(s % sets, -1) < written[s]
            for s in write:
                # cleared by an earlier launch (or never used: zero at create)
                if s >= sets:
                    assert cleared_at.get(s % sets, -1) > written.get(s - sets, -1) >= 0 or s - sets not in written
                written[s] = li
            for s in clear:
                cleared_at[s % sets] = li
            t += n
        for s, li in written.items():
            if s < t - max_steps:
                assert folded[s] == li + 1
