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


def pool_buf(done, spl):
    """The pool's buffer after `done` steps (pool.hip): launches counted per graph replay."""
    launches = (done // spl) * ((spl + 1) // 2) + ((done % spl) + 1) // 2
    return launches & 1


def test_pool_buffer_follows_the_launch_sequence():
    """Replays of spl steps in pairs from the replay's start (an odd one last), a request with one
    step left taking it alone, and early stops that lower the target to a replay boundary + 1."""
    rng = random.Random(1)
    for spl in list(range(1, 12)) + [63, 64]:
        for _ in range(100):
            target = rng.randint(1, 5 * spl + 7)
            stop_at = rng.randint(1, max(1, target // spl)) * spl if rng.random() < 0.5 else None
            buf, done, tgt = 0, 0, target
            while done < tgt:
                for j in range(0, spl, 2):
                    if done >= tgt:
                        break
                    n = 2 if spl - j >= 2 else 1
                    k = 1 if tgt - done < n else n
                    assert pool_buf(done, spl) == buf
                    buf ^= 1
                    done += k
                    assert pool_buf(done, spl) == buf
                if stop_at is not None and done == stop_at and tgt > done + 1:
                    tgt = done + 1


def strip_segments(nx, ny, tw, slots, min_rows):
    """The launcher's segments per strip (kernels.hip strip_segments)."""
    nstrips = -(-nx // tw)
    nseg = max(1, (slots + nstrips // 2) // nstrips)
    cap = ny // max(min_rows, 1)
    if nseg > cap:
        nseg = cap if cap > 0 else 1
    return nseg


def check_strip_lattice(nx, ny, xper, yper, tw, R, nseg, outlet=False):
    """Model of step2s_kernel: every workgroup (strip, segment), every iteration, every thread.
    Checks that each ring read of the second step names the node and plane the one-step rule
    names, that it was written in this or the previous iteration and not overwritten since (a
    slot written by the next iteration's first phase is never one this iteration's second phase
    reads), that the inner fast paths only take interior nodes, and that every lattice node is
    owned once in each step."""
    nr = 2 * R + 2
    ew = tw + 2
    nstrips = -(-nx // tw)
    own1, own2 = [], []
    for w in range(nstrips * nseg):
        strip, seg = w % nstrips, w // nstrips
        x0 = strip * tw
        y0, y1 = ny * seg // nseg, ny * (seg + 1) // nseg
        niter = (y1 - y0 + 1) // R + 1
        xin = x0 >= 2 and x0 + tw + 2 <= nx
        threads = []                      # (lx, r, strip thread)
        for tid in range(tw * R):
            threads.append((tid % tw, tid // tw, True))
        for l in range(2 * R):
            threads.append((-1 if l < R else tw, l if l < R else l - R, False))
        ring = {}                         # slot -> (ly, x, y) written by the first phase
        age = {}                          # slot -> iteration that wrote it
        outl = {}
        for it in range(niter):
            a1 = y0 - 1 + it * R
            base = (it * R) % nr
            written_now = set()
            for lx, r, st in threads:
                ux = x0 + lx
                x1, live = ux, True
                if x1 < 0 or x1 >= nx:
                    if xper and -1 <= x1 <= nx:
                        x1 += nx if x1 < 0 else -nx
                    else:
                        live = False
                uy = a1 + r
                y, live = uy, live and uy <= y1
                if y < 0 or y >= ny:
                    if yper and -1 <= y <= ny:
                        y += ny if y < 0 else -ny
                    else:
                        live = False
                if not live:
                    continue
                assert 0 <= x1 < nx and 0 <= y < ny
                if xin and a1 >= 1 and a1 + R <= ny - 1:
                    assert 0 < x1 < nx - 1 and 0 < y < ny - 1      # pull_interior
                slot = base + r
                slot -= nr if slot >= nr else 0
                assert slot == (uy - y0 + 1) % nr
                ring[(slot, lx + 1)] = (x1, y)
                age[(slot, lx + 1)] = it
                written_now.add(slot)
                col_own = st and ux < nx
                if col_own and y0 <= uy < y1:
                    own1.append((x1, y))
                if outlet and x1 == nx - 1 and col_own:
                    outl[slot] = (x1, y)
            # second phase (strip threads)
            read_slots = set()
            for lx, r, st in threads:
                if not st:
                    continue
                x2, y = x0 + lx, a1 - 1 + r
                if not (y0 <= y < y1 and x2 < nx):
                    continue
                own2.append((x2, y))
                sc = base + r - 1
                sc += nr if sc < 0 else 0
                sc -= nr if sc >= nr else 0
                sm = nr - 1 if sc == 0 else sc - 1
                sp = 0 if sc == nr - 1 else sc + 1
                assert sc == (y - y0 + 1) % nr
                shifts = (xper or 0 < x2 < nx - 1) and (yper or 0 < y < ny - 1)
                for a in range(9):
                    if shifts:
                        sx, sy, pa = x2 - CX[a], y - CY[a], a
                    else:
                        sx, sy, pa = x2 - CX[a], y - CY[a], a
                        if (sy < 0 or sy >= ny) and not yper:
                            sy, pa = y, MIRROR_Y[a]
                        if (sx < 0 or sx >= nx) and not xper:
                            sx = 0 if sx < 0 else nx - 1
                    ss = sc if sy == y else (sm if sy < y else sp)
                    col = sx - x0 + 1
                    assert 0 <= col < ew and 0 <= ss < nr
                    key = (ss, col)
                    assert key in ring, (nx, ny, x2, y, a)
                    assert age[key] in (it, it - 1)
                    gx, gy, gpa = edge_source(a, x2, y, nx, ny, xper, yper)
                    assert ring[key] == (gx, gy) and pa == gpa, (nx, ny, x2, y, a)
                    read_slots.add(ss)
                if outlet and x2 == nx - 1:
                    assert outl[sc] == (x2, y)
                    for d in (3, 6, 7):
                        sy, pa = y - CY[d], d
                        if (sy < 0 or sy >= ny) and not yper:
                            sy, pa = y, MIRROR_Y[d]
                        ss = sc if sy == y else (sm if sy < y else sp)
                        gx, gy, gpa = edge_source(d, nx - 2, y, nx, ny, 0, yper)
                        assert ring[(ss, nx - 1 - x0 + 1)] == (gx, gy) and pa == gpa
            # the next iteration's first phase must not write a slot read here
            nxt = {(((it + 1) * R + r) % nr) for r in range(R)}
            assert not (nxt & read_slots)
    everything = sorted((x, y) for x in range(nx) for y in range(ny))
    assert sorted(own1) == everything
    assert sorted(own2) == everything


STRIP_SIZES = [(3, 3), (5, 4), (64, 8), (130, 17), (257, 31), (129, 3), (3, 40), (200, 45)]


@pytest.mark.parametrize("tw,R", [(128, 4), (64, 4), (64, 8)])
def test_strip_sweep_reads_what_the_first_step_wrote(tw, R):
    for (nx, ny), xper, yper in itertools.product(STRIP_SIZES, (0, 1), (0, 1)):
        for slots in (7, 768):
            nseg = strip_segments(nx, ny, tw, slots, 2 * R)
            check_strip_lattice(nx, ny, xper, yper, tw, R, nseg)
        # segments of every height down to one row
        for nseg in sorted({1, 2, min(ny, 5)}):
            check_strip_lattice(nx, ny, xper, yper, tw, R, nseg)


@pytest.mark.parametrize("tw,R", [(128, 4), (64, 4)])
def test_strip_sweep_convective_outlet_lookups(tw, R):
    for (nx, ny), yper in itertools.product([(3, 3), (5, 7), (129, 9), (150, 40), (257, 31)], (0, 1)):
        for nseg in (1, 3):
            check_strip_lattice(nx, ny, 0, yper, tw, R, min(nseg, ny), outlet=True)


def test_strip_segments_fill_the_chip():
    # 8192 x 2048 FP32: 64 strips of 128, 768 slots -> 12 segments of ~171 rows, one round
    assert strip_segments(8192, 2048, 128, 768, 8) == 12
    # the paper's 6048 x 2016 case: 48 strips -> 16 segments
    assert strip_segments(6048, 2016, 128, 768, 8) == 16
    # small lattices: segments of at least min_rows rows
    assert strip_segments(100, 20, 128, 768, 8) == 2
    assert strip_segments(100, 5, 128, 768, 8) == 1
