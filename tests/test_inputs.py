"""CPU checks of the seeded input generators (no method arithmetic): the serving stream keeps the
constraints its recipe states, and the column-blockage measure it uses matches closed forms."""
import math

import numpy as np

from paper_1812_05401_amd import inputs as I


def test_column_blockage_closed_forms():
    n = 200
    # one disk: the widest chord is the diameter
    assert abs(I.column_blockage([I.body("disk", 100.0, 80.0, r=30.0)], n) - 60.0 / n) < 1e-12
    # one rectangle: its full height wherever it spans
    assert abs(I.column_blockage([I.body("rect", 50.0, 80.0, hx=10.0, hy=25.0)], n) - 50.0 / n) < 1e-12
    # two bodies in the same columns add (overlap counted twice); apart they do not
    stacked = [I.body("disk", 100.0, 50.0, r=20.0), I.body("rect", 100.0, 150.0, hx=5.0, hy=10.0)]
    assert abs(I.column_blockage(stacked, n) - (40.0 + 20.0) / n) < 1e-12
    apart = [I.body("disk", 40.0, 50.0, r=20.0), I.body("disk", 160.0, 150.0, r=10.0)]
    assert abs(I.column_blockage(apart, n) - 40.0 / n) < 1e-12
    assert I.column_blockage([], n) == 0.0


def test_serving_stream_keeps_its_recipe():
    reqs = I.serving_requests(n=256)
    assert len(reqs) == 256
    arrivals = np.array([r.arrival for r in reqs])
    assert arrivals[0] == 0.0 and np.all(np.diff(arrivals) >= 0)
    for r in reqs:
        c = r.case
        N = c.nx
        assert c.ny == N and 128 <= N <= 1024 and N % 32 == 0
        assert c.storage == "f32" and c.collision == I.MRT and c.bc == I.CHANNEL
        assert 1 <= len(c.bodies) <= 8 and 1000 <= c.steps <= 20000
        assert c.tau >= 0.56
        area = 0.0
        for b in c.bodies:
            rad = b["r"] if b["kind"] == "disk" else b["hx"]
            assert 8.0 <= rad <= min(64.0, N / 8.0) + 1e-12
            assert b["cx"] - rad >= 4.0 - 1e-9 and N / 8.0 - 1e-9 <= b["cx"] <= 5.0 * N / 8.0 + 1e-9
            assert b["cy"] - rad >= 6.0 - 1e-9 and b["cy"] + rad <= N - 7.0 + 1e-9
            area += math.pi * rad * rad if b["kind"] == "disk" else 4.0 * rad * rad
        assert area <= 0.2 * N * N
        assert I.column_blockage(c.bodies, N) <= 0.4
        re = 0.05 * c.diameter / ((c.tau - 0.5) / 3.0)
        assert 50.0 - 1e-6 <= re <= 500.0 + 1e-6


def test_serving_stream_is_reproducible():
    a = I.serving_requests(n=16)
    b = I.serving_requests(n=16)
    for x, y in zip(a, b):
        assert x.arrival == y.arrival and x.case.steps == y.case.steps and x.case.bodies == y.case.bodies
