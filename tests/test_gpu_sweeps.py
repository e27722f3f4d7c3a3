"""The paper's shear-flow claims (Section 3.1, Fig. 3) reproduced on the GPU through the serving
pool: the error vanishes at SRT tau = 1/2 + sqrt(6)/4 and at MRT Lambda = 3/8 for any tau, and
does not elsewhere."""
import math

import pytest

from paper_1812_05401_amd import sweeps as S

pytestmark = pytest.mark.gpu


def test_shear_optimum_through_the_pool(gpu):
    pts = [S.shear_case("srt", 0.5 + math.sqrt(6) / 4), S.shear_case("srt", 0.8),
           S.shear_case("mrt", 1.5, 0.375), S.shear_case("mrt", 10.0, 0.375),
           S.shear_case("mrt", 1.5, 3 / 16)]
    res = {r["label"]: (r["l2_error"], r["status"]) for r in S.run(pts)}
    errs = [res[p.label][0] for p in pts]
    assert all(res[p.label][1] == 0 for p in pts)
    assert errs[0] < 1e-6 and errs[2] < 1e-6 and errs[3] < 1e-6
    assert errs[1] > 1e-3 and errs[4] > 1e-3
