"""GPU tests of the serving pool: a request's result is the same alone and in a mix (bitwise),
equal to the single-simulation path and to the oracle, and admission respects the budget."""
import numpy as np
import pytest

from paper_1812_05401_amd import inputs as I
from tests.helpers import force_scale, oracle_sim, rel_err

pytestmark = pytest.mark.gpu


def small_requests(seed=7, n=6, storage="f64"):
    r = np.random.default_rng(seed)
    out = []
    for k in range(n):
        N = int(r.integers(70, 260))
        M = int(r.integers(40, 200))
        coll = "mrt" if k % 2 == 0 else "srt"
        bc = I.CHANNEL if k % 3 != 2 else I.ALL_PERIODIC
        u_in = (0.04, 0.0) if bc == I.CHANNEL else (0.0, 0.0)
        u0 = u_in if bc == I.CHANNEL else (0.03, 0.01)    # a periodic box starts with a drift
        bodies = I.random_bodies(N, M, seed + k, int(r.integers(1, 4)), rmin=3, rmax=min(N, M) / 5)
        out.append(I.Case(f"pool{k}", N, M, collision=coll, storage=storage,
                          tau=float(r.uniform(0.55, 0.9)), bc=bc, u_in=u_in, bodies=bodies,
                          u0=u0, steps=int(r.integers(150, 700))))
    return out


def run(pool_cls, cases, budget, slots=64, spl=32, max_nodes=0):
    pool = pool_cls(budget, max_slots=slots, steps_per_launch=spl)
    if max_nodes:
        pool.set_admission(max_nodes)
    ids = [pool.submit(c, c.steps, keep_fields=True) for c in cases]
    res, max_running = {}, 0
    while len(res) < len(ids):
        running, queued, _ = pool.advance()
        max_running = max(max_running, running)
        for k, rid in enumerate(ids):
            if k in res:
                continue
            st, _ = pool.status(rid)
            if st >= 2:
                res[k] = pool.result(rid, fields=True)
    pool.close()
    return res, max_running


@pytest.mark.parametrize("storage", ["f64", "f32"])
def test_alone_and_in_the_mix_are_bitwise_equal(gpu, storage):
    """FP64 requests (two steps per launch) and binary32 ones (three steps per launch)."""
    B = gpu
    cases = small_requests(storage=storage)
    alone = {k: run(B.Pool, [c], 1 << 30)[0][0] for k, c in enumerate(cases)}
    # a budget that holds about three of them: admission binds, requests queue and overlap
    budget = int(3 * max(B.vplbm_pool_bytes_needed(c) for c in cases))
    mix, max_running = run(B.Pool, cases, budget)
    assert 1 < max_running < len(cases)
    for k in range(len(cases)):
        (oa, fa), (om, fm) = alone[k], mix[k]
        assert oa["status"] == om["status"] == 0
        assert oa["step"] == om["step"] == cases[k].steps - 1
        assert oa["mass"] == om["mass"]
        assert np.array_equal(oa["fx"], om["fx"]) and np.array_equal(oa["fy"], om["fy"])
        for a, b in zip(fa, fm):
            assert np.array_equal(a, b)


def test_admission_cap_bounds_the_resident_nodes(gpu):
    """With a cap on resident nodes the pool runs fewer simulations at once (at least one, even
    one larger than the cap) and every result is still the one it gives alone."""
    B = gpu
    cases = small_requests(seed=5, n=6)
    sizes = sorted(c.nx * c.ny for c in cases)
    cap = sizes[0] + sizes[1]                       # at most two of the smallest fit together
    alone = {k: run(B.Pool, [c], 1 << 30)[0][0] for k, c in enumerate(cases)}
    capped, max_running = run(B.Pool, cases, 1 << 30, max_nodes=cap)
    assert 1 <= max_running <= 2
    for k in range(len(cases)):
        (oa, fa), (oc, fc) = alone[k], capped[k]
        assert oc["status"] == 0 and oa["mass"] == oc["mass"]
        for a, b in zip(fa, fc):
            assert np.array_equal(a, b)
    tiny = run(B.Pool, cases[:2], 1 << 30, max_nodes=1)[1]   # below every request: one at a time
    assert tiny == 1


def test_pool_matches_single_simulation_and_oracle(gpu):
    B = gpu
    cases = small_requests(seed=11, n=3)
    res, _ = run(B.Pool, cases, 1 << 30)
    for k, c in enumerate(cases):
        obs, (rho, ux, uy) = res[k]
        s = B.Simulation(c, stream=None)
        s.step(c.steps)
        so, srho, sux, suy = s.observables(fields=True)
        s.close()
        assert rel_err(rho, srho) <= 1e-13 and rel_err(np.stack([ux, uy]), np.stack([sux, suy])) <= 1e-12
        o = oracle_sim(c)
        o.step(c.steps)
        oo = o.obs()
        orho, oux, ouy = o.fields()
        assert rel_err(rho, orho) <= 1e-12
        assert rel_err(np.stack([ux, uy]), np.stack([oux, ouy])) <= 1e-12
        assert abs(obs["mass"] - oo["mass"]) <= 1e-12 * oo["mass"]
        sc = force_scale(oo)
        assert np.max(np.abs(obs["fx"] - oo["fx"])) <= 1e-12 * sc
        assert np.max(np.abs(obs["fy"] - oo["fy"])) <= 1e-12 * sc


def test_budget_and_argument_errors(gpu):
    B = gpu
    c = small_requests(n=1)[0]
    need = B.vplbm_pool_bytes_needed(c)
    pool = B.Pool(need - 1, max_slots=4, steps_per_launch=8)
    with pytest.raises(B.VplbmError) as e:
        pool.submit(c)
    assert e.value.code == B.EBUDGET
    moving = I.Case("m", 64, 64, bodies=[I.body("disk", 30, 30, r=5, ay=2, freq=0.01)])
    with pytest.raises(B.VplbmError) as e:
        pool.submit(moving)
    assert e.value.code == B.EINVAL
    pool.close()
    # one slot: requests run strictly one after another, first come first served
    cases = small_requests(seed=3, n=3, storage="f32")
    res, max_running = run(B.Pool, cases, 1 << 30, slots=1)
    assert max_running == 1 and len(res) == 3
    for k in range(3):
        assert res[k][0]["status"] == 0


def _drain(pool, ids, fields):
    from paper_1812_05401_amd import binding as B
    out = {}
    while len(out) < len(ids):
        pool.advance()
        for rid in ids:
            if rid in out:
                continue
            st, done = pool.status(rid)
            if st >= B.DONE:
                out[rid] = (st, done, pool.result(rid, fields=fields.get(rid, False)))
    return out


def test_cancel_queued_and_running_requests(gpu):
    """A request cancelled while queued never runs; one cancelled while running stops at the next
    advance with the steps it has done; the others finish as they would alone."""
    B = gpu
    cases = small_requests(seed=9, n=4)
    for c in cases:
        c.steps = 4000                                    # long enough to be running at the cancel
    alone = {k: run(B.Pool, [cases[k]], 1 << 30)[0][0] for k in (1, 3)}
    pool = B.Pool(1 << 30, max_slots=2, steps_per_launch=32)
    ids = [pool.submit(c, c.steps, keep_fields=True) for c in cases]
    pool.advance()                                        # admits the first two
    assert pool.status(ids[0])[0] == B.RUNNING and pool.status(ids[2])[0] == B.QUEUED
    pool.cancel(ids[0])
    pool.cancel(ids[2])
    assert pool.status(ids[2])[0] == B.CANCELLED
    res = _drain(pool, ids, {ids[0]: True, ids[1]: True, ids[3]: True})
    with pytest.raises(B.VplbmError) as e:
        pool.cancel(ids[1])
    assert e.value.code in (B.EINVAL, B.ESTATE)           # released, or finished
    pool.close()
    st, done, (obs, fields) = res[ids[0]]
    assert st == B.CANCELLED and 0 < done < cases[0].steps and obs["step"] == done - 1
    assert np.all(np.isfinite(fields[0])) and obs["mass"] == 0.0
    st, done, obs = res[ids[2]]
    assert st == B.CANCELLED and done == 0
    for k in (1, 3):
        st, done, (obs, fields) = res[ids[k]]
        oa, fa = alone[k]
        assert st == B.DONE and done == cases[k].steps and obs["mass"] == oa["mass"]
        for a, b in zip(fields, fa):
            assert np.array_equal(a, b)


def test_an_unstable_request_fails_without_affecting_the_others(gpu):
    """Host-forced instability: an initial velocity of 50 lattice units makes the density go
    non-positive within a few steps; that request is FAILED and released, the others finish as
    they would alone."""
    import copy
    B = gpu
    cases = small_requests(seed=13, n=3)
    bad = copy.copy(cases[1])
    bad.name, bad.u0 = "unstable", (50.0, 0.0)
    alone = {k: run(B.Pool, [cases[k]], 1 << 30)[0][0] for k in (0, 2)}
    pool = B.Pool(1 << 30, max_slots=4, steps_per_launch=32)
    ids = [pool.submit(c, c.steps, keep_fields=True) for c in (cases[0], bad, cases[2])]
    res = _drain(pool, ids, {ids[0]: True, ids[2]: True})
    pool.close()
    st, done, obs = res[ids[1]]
    assert st == B.FAILED and obs["status"] == 1 and done < bad.steps
    for k, rid in ((0, ids[0]), (2, ids[2])):
        st, done, (obs, fields) = res[rid]
        oa, fa = alone[k]
        assert st == B.DONE and obs["mass"] == oa["mass"]
        for a, b in zip(fields, fa):
            assert np.array_equal(a, b)


def test_create_and_destroy_release_device_memory(gpu):
    import torch
    B = gpu
    c = small_requests(seed=2, n=1)[0]
    for _ in range(3):                                     # let allocator caches settle
        B.Simulation(c, stream=None).close()
    torch.cuda.synchronize()
    free0 = torch.cuda.mem_get_info()[0]
    for _ in range(100):
        s = B.Simulation(c, stream=None)
        s.step(2)
        s.residual()
        s.close()
        p = B.Pool(1 << 28, max_slots=2, steps_per_launch=4)
        p.submit(c, 8)
        p.advance()
        p.close()
    torch.cuda.synchronize()
    assert abs(torch.cuda.mem_get_info()[0] - free0) < (64 << 20)


def test_host_log(gpu, capfd, monkeypatch):
    """VPLBM_LOG=1 logs creation, admission, graph capture and retirement on stderr."""
    B = gpu
    monkeypatch.setenv("VPLBM_LOG", "1")
    c = small_requests(seed=4, n=1)[0]
    B.Simulation(c, stream=None).close()
    run(B.Pool, [c], 1 << 30)
    err = capfd.readouterr().err
    for word in ("[vplbm] create", "[vplbm] destroy", "admit request", "capture the step graph",
                 "retire request"):
        assert word in err, word
    monkeypatch.setenv("VPLBM_LOG", "0")
    B.Simulation(c, stream=None).close()
    assert "[vplbm]" not in capfd.readouterr().err


@pytest.mark.parametrize("storage", ["f16sr", "bf16sr"])
def test_stochastic_rounding_is_the_same_in_the_pool(gpu, storage):
    """The random bits depend on the node and on the steps the simulation has run, so a pool run
    equals the single-simulation run bit for bit."""
    B = gpu
    c = small_requests(seed=21, n=1, storage=storage)[0]
    (obs, (rho, ux, uy)) = run(B.Pool, [c], 1 << 30)[0][0]
    s = B.Simulation(c, stream=None)
    s.step(c.steps)
    _, srho, sux, suy = s.observables(fields=True)
    s.close()
    assert np.array_equal(rho, srho) and np.array_equal(ux, sux) and np.array_equal(uy, suy)


@pytest.mark.parametrize("spl", [1, 7, 64])
def test_launch_shapes_match_the_single_simulation_bitwise(gpu, spl):
    """The pool takes pairs of steps per launch (triples for binary32), what remains of a replay
    last, and fewer steps for a request with fewer left.  Over step counts of every remainder and
    mixed storage formats, the fields are bitwise those of the single-simulation path."""
    B = gpu
    cases = small_requests(seed=13, n=7)
    for c, st, n in zip(cases, ("f32", "f16s", "f64", "f32d", "bf16sr", "f32", "f32"),
                        (151, 200, 97, 64, 33, 100, 65)):
        c.storage = st
        c.steps = n
    res, _ = run(B.Pool, cases, 1 << 30, spl=spl)
    for k, c in enumerate(cases):
        obs, fields = res[k]
        assert obs["status"] == 0 and obs["step"] == c.steps - 1
        s = B.Simulation(c, stream=None)
        s.step(c.steps)
        so, *sfields = s.observables(fields=True)
        s.close()
        for a, b in zip(fields, sfields):
            assert np.array_equal(a, b), f"{c.name}/{c.storage}, {c.steps} steps, {spl} per launch"
        assert abs(obs["mass"] - so["mass"]) <= 1e-13 * so["mass"]


def convective_requests(seed, storages, steps):
    """small_requests on channels with the convective outlet (Section 3.3's outlet)."""
    cases = small_requests(seed=seed, n=len(storages))
    for c, st, n in zip(cases, storages, steps):
        c.bc = I.CHANNEL_CONVECTIVE
        c.u_in = (0.04, 0.0)
        c.u0 = (0.04, 0.0)
        c.storage = st
        c.steps = n
    return cases


@pytest.mark.parametrize("spl", [1, 7, 64])
def test_convective_outlet_matches_the_single_simulation_bitwise(gpu, spl):
    """Requests with a convective outlet in the pool: binary32 takes three steps per launch on its
    14-row tiles, the outlet's records passed from phase to phase in LDS; the other formats take
    pairs of steps; the records in memory follow the population buffers.  Over step counts of
    every residue modulo 2 and 3 and the storage formats, alone and in a mix with outlet-free
    requests, the fields are bitwise those of the single-simulation path."""
    B = gpu
    conv = convective_requests(17, ("f32", "f64", "f16s", "f32d", "bf16sr", "f16sr", "f32", "f32"),
                               (151, 200, 97, 64, 33, 101, 200, 96))
    plain = small_requests(seed=19, n=3, storage="f32")
    res, _ = run(B.Pool, conv + plain, 1 << 30, spl=spl)
    alone = {k: run(B.Pool, [c], 1 << 30, spl=spl)[0][0] for k, c in enumerate(conv[:2])}
    for k, c in enumerate(conv + plain):
        obs, fields = res[k]
        assert obs["status"] == 0 and obs["step"] == c.steps - 1
        s = B.Simulation(c, stream=None)
        s.step(c.steps)
        so, *sfields = s.observables(fields=True)
        s.close()
        for a, b in zip(fields, sfields):
            assert np.array_equal(a, b), f"{c.name}/{c.storage}, {c.steps} steps, {spl} per launch"
        assert abs(obs["mass"] - so["mass"]) <= 1e-13 * so["mass"]
        if k in alone:
            for a, b in zip(alone[k][1], fields):
                assert np.array_equal(a, b)


def test_convective_outlet_in_the_pool_matches_the_oracle(gpu):
    """FP64 requests with the convective outlet against the oracle (its outlet reading) to 1e-12."""
    B = gpu
    cases = convective_requests(23, ("f64", "f64"), (300, 257))
    res, _ = run(B.Pool, cases, 1 << 30, spl=16)
    for k, c in enumerate(cases):
        obs, (rho, ux, uy) = res[k]
        o = oracle_sim(c)
        o.step(c.steps)
        oo = o.obs()
        orho, oux, ouy = o.fields()
        assert rel_err(rho, orho) <= 1e-12
        assert rel_err(np.stack([ux, uy]), np.stack([oux, ouy])) <= 1e-12
        assert abs(obs["mass"] - oo["mass"]) <= 1e-12 * oo["mass"]
        sc = force_scale(oo)
        assert np.max(np.abs(obs["fx"] - oo["fx"])) <= 1e-12 * sc
        assert np.max(np.abs(obs["fy"] - oo["fy"])) <= 1e-12 * sc


def test_tile_table_growth_mid_run(gpu):
    """A request runs alone (1184 tiles), then three more join (4736 tiles: the device tile table
    outgrows its first 4096 entries and the graph is captured again); a 128² request joins
    last.  Every request's fields are bitwise those of the single-simulation path, binary32
    (three steps per launch) and FP64 (two) alike."""
    B = gpu
    cases = []
    for k, st in enumerate(("f32", "f32", "f64", "f32")):
        c = I.Case(f"big{k}", 1024, 1024, collision="mrt" if k % 2 == 0 else "srt", storage=st,
                   tau=0.6 + 0.05 * k, bc=I.CHANNEL, u_in=(0.04, 0.0), u0=(0.04, 0.0),
                   bodies=[I.body("disk", 300 + 40 * k, 511.5, r=40), I.body("rect", 600, 300, hx=20, hy=30)],
                   steps=97 + 10 * k)
        cases.append(c)
    small = small_requests(seed=29, n=1, storage="f32")[0]
    small.steps = 131
    pool = B.Pool(4 << 30, max_slots=8, steps_per_launch=16)
    ids = [pool.submit(cases[0], cases[0].steps, keep_fields=True)]
    pool.advance()
    pool.advance()                                       # the first request runs alone
    ids += [pool.submit(c, c.steps, keep_fields=True) for c in cases[1:]]
    pool.advance()
    ids.append(pool.submit(small, small.steps, keep_fields=True))
    res = {}
    while len(res) < len(ids):
        pool.advance()
        for k, rid in enumerate(ids):
            if k not in res and pool.status(rid)[0] >= 2:
                res[k] = pool.result(rid, fields=True)
    pool.close()
    for k, c in enumerate(cases + [small]):
        obs, fields = res[k]
        assert obs["status"] == 0 and obs["step"] == c.steps - 1
        s = B.Simulation(c, stream=None)
        s.step(c.steps)
        so, *sfields = s.observables(fields=True)
        s.close()
        for a, b in zip(fields, sfields):
            assert np.array_equal(a, b), f"{c.name}/{c.storage}"
        assert abs(obs["mass"] - so["mass"]) <= 1e-13 * so["mass"]


def test_many_tiny_lattices(gpu):
    """300 lattices from 3 x 3 to 40 x 40 in one pool (ragged tiles, periodic edges narrower
    than the three-step kernel's two-node halo, every storage format, both collisions, 300
    slots): each is bitwise the single-simulation run of as many steps."""
    B = gpu
    r = np.random.default_rng(31)
    storages = ("f32", "f64", "f16s", "bf16s", "f32d", "f16sr", "bf16sr")
    cases = []
    for k in range(300):
        nx, ny = int(r.integers(3, 41)), int(r.integers(3, 41))
        periodic = k % 2 == 0
        bc = I.ALL_PERIODIC if periodic else I.CHANNEL
        u = (0.02, 0.01) if periodic else (0.03, 0.0)
        bodies = []
        if min(nx, ny) >= 12 and k % 3 == 0:
            bodies = [I.body("disk", nx / 2, ny / 2, r=min(nx, ny) / 5, omega=0.002)]
        cases.append(I.Case(f"tiny{k}", nx, ny, collision="mrt" if k % 4 < 2 else "srt",
                            storage=storages[k % len(storages)], tau=0.6 + 0.3 * r.random(), bc=bc,
                            u_in=(0.03, 0.0) if not periodic else (0.0, 0.0), u0=u, bodies=bodies,
                            steps=int(r.integers(1, 60))))
    res, max_running = run(B.Pool, cases, 1 << 30, slots=300, spl=7)
    assert max_running == 300
    for k, c in enumerate(cases):
        obs, fields = res[k]
        assert obs["status"] == 0 and obs["step"] == c.steps - 1
        s = B.Simulation(c, stream=None)
        s.step(c.steps)
        so, *sfields = s.observables(fields=True)
        s.close()
        for a, b in zip(fields, sfields):
            assert np.array_equal(a, b), f"{c.name} {c.nx}x{c.ny} {c.storage}, {c.steps} steps"
        assert abs(obs["mass"] - so["mass"]) <= 1e-12 * abs(so["mass"])
