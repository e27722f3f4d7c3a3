"""CPU model of the DPP wave sum (lattice.hpp, wave_sum with DPP = true).  The lane patterns are
read from the source (the dpp_double control words and the lanes whose row sums are added),
decoded as the GCN DPP controls they name (quad_perm, row_half_mirror, row_mirror), and applied
to symbolic lane values: after the four exchanges every lane of a row of 16 must hold each of its
row's lanes exactly once, and the final sum must hold each of the 64 lanes exactly once.  A wrong
control word (a lane pattern that repeats or skips a lane) fails here; the GPU tests check the
sums themselves against the oracle."""
import collections
import os
import re

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LATTICE = os.path.join(ROOT, "paper_1812_05401_amd", "csrc", "lattice.hpp")


def wave_sum_source():
    src = open(LATTICE).read()
    start = src.index("__device__ __forceinline__ double wave_sum(double v)")
    body = src[start:src.index("\n}\n", start)]
    dpp_branch = body[body.index("if constexpr (DPP)"):body.index("} else {")]
    return dpp_branch


def decode(ctrl):
    """Source lane within a row of 16 for destination lane l, for the DPP controls used."""
    if ctrl <= 0xFF:                                     # quad_perm: 2 bits per lane of a quad
        sel = [(ctrl >> (2 * k)) & 3 for k in range(4)]
        return lambda l: (l & ~3) | sel[l & 3]
    if ctrl == 0x141:                                    # row_half_mirror
        return lambda l: (l & 8) | (7 - (l & 7))
    if ctrl == 0x140:                                    # row_mirror
        return lambda l: 15 - l
    raise AssertionError(f"unmodelled DPP control {ctrl:#x}")


def test_dpp_wave_sum_counts_every_lane_once():
    src = wave_sum_source()
    ctrls = [int(c, 16) for c in re.findall(r"dpp_double<(0x[0-9A-Fa-f]+)>", src)]
    assert len(ctrls) == 4, src
    lanes = [int(l) for l in re.findall(r"lane_double\(v, (\d+)\)", src)]
    assert sorted(lanes) == [0, 16, 32, 48], src

    v = [collections.Counter({l: 1}) for l in range(64)]   # lane -> multiset of contributing lanes
    for ctrl in ctrls:
        src_lane = decode(ctrl)
        v = [v[l] + v[(l & ~15) | src_lane(l & 15)] for l in range(64)]
    for l in range(64):
        row = l & ~15
        assert v[l] == collections.Counter(range(row, row + 16)), (l, v[l])
    total = collections.Counter()
    for l in lanes:
        total += v[l]
    assert total == collections.Counter(range(64))


def test_quad_perm_decoding():
    """The two quad_perm words are the xor-1 and xor-2 exchanges their comments name."""
    f1, f2 = decode(0xB1), decode(0x4E)
    assert [f1(l) for l in range(8)] == [1, 0, 3, 2, 5, 4, 7, 6]
    assert [f2(l) for l in range(8)] == [2, 3, 0, 1, 6, 7, 4, 5]
