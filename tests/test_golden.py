"""The oracle's constants against the values printed in the paper (tests/golden/paper_printed.json)
and the printed parameter sets against one another."""
from fractions import Fraction as Fr
import json
import math
import os

import numpy as np

import oracle as O

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_printed.json")))


def test_weights_and_matrix_as_printed():
    _, w = O.lattice()
    assert np.allclose(w, [float(Fr(x)) for x in GOLD["eq5_weights"]], rtol=0, atol=1e-17)
    assert np.array_equal(O.moment_matrix(), np.array(GOLD["eq13_moment_matrix"], dtype=float))


def test_rate_pattern_as_printed():
    s = O.mrt_rates(0.8, 3 / 16)
    pat = GOLD["eq14_rate_pattern"]
    for i, p in enumerate(pat):
        if p == "0":
            assert s[i] == 0
        elif p == "s_n":
            assert s[i] == 1 / 0.8
        else:
            assert s[i] == s[4] and s[4] != s[1]


def test_printed_optimum_pair_is_consistent():
    """Section 3.1: SRT means s_n = s_q = 1/tau, so Lambda = (tau - 1/2)^2; the printed optimum
    tau = 1/2 + sqrt(6)/4 and Lambda = 3/8 are the same point."""
    tau = 0.5 + math.sqrt(6) / 4
    assert abs((tau - 0.5) ** 2 - float(Fr(GOLD["sec3_1_optimum_mrt_lambda"]))) < 1e-15


def test_cylinder_parameters_are_consistent():
    """Section 3.3: 30 D x 10 D with D = 201 nodes is the printed 6048 x 2016 lattice to within a
    node per diameter, and nu = U D / Re matches tau = 0.56 through Eq. 6."""
    c = GOLD["sec3_3_cylinder"]
    assert abs(c["nx"] / c["D"] - c["length_D"]) < 0.1 and abs(c["ny"] / c["D"] - c["height_D"]) < 0.05
    nu = c["U"] * c["D"] / c["Re"]
    assert abs((0.5 + 3 * nu) - c["tau"]) < 0.005
