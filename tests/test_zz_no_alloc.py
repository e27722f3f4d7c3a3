"""The allocation-free momentum exchange (vplbm_momentum_exchange_noalloc) through the C ABI:
its device output equals the allocating entry point's (vplbm_momentum_exchange) to the FP64 bar,
on two calls in a row, the second on a smaller lattice, both through the static scratch it shares
on the GPU.  It must pass alone in a fresh process and after the other tests."""
import zlib

import numpy as np
import pytest

from paper_1812_05401_amd import inputs as I
from tests.helpers import gpu_sim
from tests.test_gpu_parity import CASES, build_case

pytestmark = pytest.mark.gpu

TOL64 = 1e-12


def _noalloc(g):
    import torch
    from paper_1812_05401_amd import binding as B
    out = torch.full((2 * B.MAX_BODIES,), float("nan"), dtype=torch.float64, device="cuda")
    torch.cuda.synchronize()
    B.vplbm_momentum_exchange_noalloc(g.h, out.data_ptr())
    torch.cuda.synchronize()
    o = out.cpu().numpy()
    return o[0::2][:g.nbodies], o[1::2][:g.nbodies]


def _scale(g):
    """The link terms' summed magnitude bound: (fluid-solid links) x 2 max f."""
    solid = g.mask() != 0
    links = sum(int(np.sum(~solid & np.roll(solid, (-ey, -ex), axis=(0, 1))))
                for ex in (-1, 0, 1) for ey in (-1, 0, 1) if ex or ey)
    return max(links, 1) * 2.0 * float(np.max(np.abs(g.populations())))


def test_noalloc_matches_the_allocating_call_twice_second_smaller(gpu):
    big, small = CASES[0], CASES[13]          # 131 x 67 periodic, then 150 x 40 convective channel
    sims = []
    for spec, steps in ((big, 120), (small, 60)):
        seed = zlib.crc32(spec[0].encode()) % 10000
        case, ids = build_case(*spec, seed=seed)
        g = gpu_sim(case, device_mask=ids is None)
        g.init_fields(*I.random_fields(case.nx, case.ny, seed, u_mean=case.u_in))
        g.step(steps)
        sims.append((spec[0], g))
    assert sims[1][1].nx * sims[1][1].ny < sims[0][1].nx * sims[0][1].ny
    for name, g in sims:
        fx, fy = _noalloc(g)
        rx, ry = g.momentum_exchange()
        sc = _scale(g)
        err = max(np.max(np.abs(fx - rx)), np.max(np.abs(fy - ry))) / sc
        print(f"{name}: noalloc {fx} {fy} vs {rx} {ry}: rel {err:.2e}", flush=True)
        assert np.all(np.isfinite(fx)) and np.all(np.isfinite(fy))
        assert err <= TOL64
        # the same state again: the fixed summation order gives the same bits
        fx2, fy2 = _noalloc(g)
        assert np.array_equal(fx, fx2) and np.array_equal(fy, fy2)


def test_noalloc_rejects_host_memory_and_oversized_lattices(gpu):
    from paper_1812_05401_amd import binding as B
    g = gpu_sim(I.Case("tiny", 8, 8, bc=I.ALL_PERIODIC))
    host = np.zeros(2 * B.MAX_BODIES)
    with pytest.raises(B.VplbmError) as e:
        B.vplbm_momentum_exchange_noalloc(g.h, host.ctypes.data)
    assert e.value.code == B.EINVAL
    import torch
    out = torch.zeros(2 * B.MAX_BODIES, dtype=torch.float64, device="cuda")
    big = gpu_sim(I.Case("over", 8192, 2049, storage="f16s", bc=I.ALL_PERIODIC))
    with pytest.raises(B.VplbmError) as e:
        B.vplbm_momentum_exchange_noalloc(big.h, out.data_ptr())
    assert e.value.code == B.EINVAL and "16777216" in str(e.value)
