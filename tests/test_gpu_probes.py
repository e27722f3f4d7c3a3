"""The measurement probes (libvplbm_probes.so) on the GPU: each pattern the bench reports runs and
gives a launch time that orders as the patterns' work does, the copy and FMA rates are below the
chip's datasheet figures, and bad arguments are refused before any device work."""
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def probes(gpu):
    from paper_1812_05401_amd import probes as P
    P.load()
    return P


def test_patterns_run_on_every_tile(probes):
    nx, ny = 1024, 336          # a whole number of every probe tile (128 x 2/8/16/6, 64 x 8/14)
    for spl, tile in [(1, (128, 2)), (2, (128, 8)), (2, (64, 8)), (2, (128, 16)), (3, (64, 14)),
                      (3, (128, 8)), (3, (128, 6)), (3, (64, 8))]:
        us = probes.pattern_us(nx, ny, spl, tile, launches=8)
        assert 0.5 < us < 5000.0, (spl, tile, us)


def test_pattern_times_scale_with_the_lattice(probes):
    """At 8192 x 2048 a launch moves 1.2 GB: no pattern beats 8 TB/s, and the one-step pattern
    is not slower than the three-step one (which does three updates' arithmetic in a launch)."""
    nodes = 8192 * 2048
    t1 = probes.pattern_us(8192, 2048, 1, (128, 2), launches=16)
    t3 = probes.pattern_us(8192, 2044, 3, (64, 14), launches=16)
    for t, n in ((t1, nodes), (t3, 8192 * 2044)):
        assert 73 * n / (t * 1e-6) / 1e9 < 8000.0
    assert t1 < t3 * 1.05


def test_copy_and_fma_rates(probes):
    gbs = probes.copy_gbs(256 << 20, reps=5)
    assert 500.0 < gbs < 16000.0            # read + write bytes over the datasheet's 8 TB/s each way
    fma = probes.fma_rate(reps=5)
    assert 5e12 < fma < 39.4e12              # at most the 39.3 T lane-instructions/s issue rate


def test_bad_arguments(probes):
    with pytest.raises(probes.ProbeError):
        probes.pattern_us(1000, 2048, 2, (128, 8))
    with pytest.raises(probes.ProbeError):
        probes.pattern_us(8192, 2048, 4, (128, 8))
    with pytest.raises(probes.ProbeError):
        probes.copy_gbs(1000)
