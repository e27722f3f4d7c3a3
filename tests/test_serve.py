"""The serving driver (serve.py): the Poisson-stream replay through the pool and one request at a
time, and the fixed-batch measurement, on a handful of small requests."""
import math

import pytest

from paper_1812_05401_amd import inputs as I
from paper_1812_05401_amd import serve


def test_fixed_batch_rejects_bad_arguments_before_any_gpu_work():
    with pytest.raises(ValueError, match="outlet"):
        serve.fixed_batch(1, 128, 300, outlet="open")
    with pytest.raises(ValueError, match="replay"):
        serve.fixed_batch(1, 128, 64, steps_per_launch=64)


@pytest.mark.gpu
def test_stream_through_the_pool_and_one_at_a_time(gpu):
    """Six small requests arriving within a few milliseconds: both replays finish every request,
    count the same lattice updates and report no failures; the pool's most resident at once is
    at least one and at most the number of requests."""
    reqs = I.serving_requests(n=6, nmin=128, nmax=192, steps_range=(300, 300), rate_per_s=2000.0)
    pool, results = serve.run_pool(reqs, 1 << 30, steps_per_launch=64)
    fifo = serve.run_fifo(reqs)
    for s in (pool, fifo):
        assert s["requests"] == 6 and s["failed"] == 0
        assert s["lattice_updates"] == sum(r.case.nodes * 300 for r in reqs)
        assert 0 < s["p50_s"] <= s["p99_s"] <= s["max_s"] and math.isfinite(s["aggregate_mlups"])
    assert 1 <= pool["max_running"] <= 6
    assert sorted(results) == sorted(r.rid for r in reqs)
    assert all(res["status"] == 0 and res["step"] == 299 for res in results.values())


@pytest.mark.gpu
def test_fixed_batch_with_the_convective_outlet(gpu):
    pool_g, single_g, streams_g, nfail = serve.fixed_batch(2, 128, 200, steps_per_launch=64,
                                                           outlet="convective")
    assert nfail == 0 and pool_g > 0 and single_g > 0 and streams_g > 0
