"""The C ABI without a GPU: the library loads, exports every symbol include/vplbm.h declares, and
rejects bad arguments on the host before any device work."""
import ctypes as C
import os
import re

import pytest

from paper_1812_05401_amd import binding as B

HEADER = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include", "vplbm.h")


def declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(vplbm_[a-z_0-9]+)\s*\(", text)))


def test_header_declares_the_five_calls():
    names = declared()
    for n in ("vplbm_create", "vplbm_set_mask", "vplbm_step", "vplbm_observables", "vplbm_destroy"):
        assert n in names


def test_library_exports_every_declared_symbol():
    lib = B.load()
    for n in declared():
        assert hasattr(lib, n), n


def test_binding_covers_the_header():
    assert sorted(n for n, _, _ in B.SIGNATURES) == declared()


def test_bytes_per_update():
    assert B.vplbm_bytes_per_update("f64") == 145
    assert B.vplbm_bytes_per_update("f32") == 73
    assert B.vplbm_bytes_per_update("f32d") == 73
    assert B.vplbm_bytes_per_update("f16s") == 37
    assert B.vplbm_bytes_per_update("bf16s") == 37
    assert B.vplbm_bytes_per_update("f16sr") == 37
    assert B.vplbm_bytes_per_update("bf16sr") == 37
    with pytest.raises(B.VplbmError):
        B.vplbm_bytes_per_update(7)


BAD = [
    (dict(nx=2, ny=10), "sides"),
    (dict(nx=10, ny=2), "sides"),
    (dict(nx=10, ny=10, tau=0.5), "tau"),
    (dict(nx=10, ny=10, tau=float("nan")), "tau"),
    (dict(nx=10, ny=10, eta=0.0), "eta"),
    (dict(nx=10, ny=10, collision="mrt", lam=0.0), "Lambda"),
    (dict(nx=10, ny=10, storage=9), "storage"),
    (dict(nx=10, ny=10, collision=5), "collision"),
    (dict(nx=10, ny=10, rho0=-1.0), "rho0"),
    (dict(nx=10, ny=10, bc=("periodic", "outflow", "periodic", "periodic")), "x edges"),
    (dict(nx=10, ny=10, bc=("outflow", "velocity", "periodic", "periodic")), "x edges"),
    (dict(nx=10, ny=10, bc=("periodic", "periodic", "freeslip", "periodic")), "y edges"),
    (dict(nx=10, ny=10, bc=("velocity", "outflow", "freeslip", "freeslip"), u_in=(1.5, 0)), "inlet"),
    (dict(nx=10, ny=10, ring=1), "ring"),
    (dict(nx=10, ny=10, bc=("velocity", "convective", "freeslip", "freeslip")), "convection speed"),
    (dict(nx=100000, ny=100000), "too large"),
    (dict(nx=10, ny=10, u0=(float("nan"), 0.0)), "initial velocity"),
]


@pytest.mark.parametrize("kw,word", BAD)
def test_create_rejects_bad_configs(kw, word):
    with pytest.raises(B.VplbmError) as e:
        B.vplbm_create(B.make_config(**kw))
    assert e.value.code == B.EINVAL
    assert word in str(e.value)


def test_create_rejects_wrong_abi_version():
    cfg = B.make_config(10, 10)
    cfg.abi_version = 99
    with pytest.raises(B.VplbmError) as e:
        B.vplbm_create(cfg)
    assert e.value.code == B.EINVAL and "abi_version" in str(e.value)


def test_null_and_foreign_handles_are_rejected():
    lib = B.load()
    assert lib.vplbm_destroy(None) == B.OK
    bogus = C.c_void_p(0xDEADBEEF)
    obs = B.Obs()
    n = C.c_int64()
    s = C.c_void_p()
    assert lib.vplbm_step(bogus, 1) == B.EINVAL
    assert lib.vplbm_step(None, 1) == B.EINVAL
    assert lib.vplbm_observables(bogus, C.byref(obs), None, None, None) == B.EINVAL
    assert lib.vplbm_set_mask(bogus, None, None, 0) == B.EINVAL
    assert lib.vplbm_destroy(bogus) == B.EINVAL
    assert lib.vplbm_steps_done(bogus, C.byref(n)) == B.EINVAL
    k = C.c_int32()
    assert lib.vplbm_steps_per_launch(bogus, C.byref(k)) == B.EINVAL
    assert lib.vplbm_stream(bogus, C.byref(s)) == B.EINVAL
    assert lib.vplbm_get_populations(bogus, None) == B.EINVAL
    assert lib.vplbm_force_series(bogus, 0, 1, None) == B.EINVAL
    r = C.c_double()
    assert lib.vplbm_residual(bogus, C.byref(r)) == B.EINVAL
    assert lib.vplbm_momentum_exchange(bogus, None, None) == B.EINVAL
    assert "invalid handle" in B.last_error()
    assert lib.vplbm_pool_set_stop(bogus, 0, 1e-6, 10) == B.EINVAL
    assert lib.vplbm_pool_residual(bogus, 0, C.byref(r)) == B.EINVAL
    assert lib.vplbm_pool_set_admission(bogus, 1000) == B.EINVAL
    assert lib.vplbm_pool_cancel(bogus, 0) == B.EINVAL
    assert lib.vplbm_pool_advance(None, None, None, None) == B.EINVAL
    assert "invalid pool" in B.last_error()


def test_plain_16_bit_names_select_stochastic_rounding():
    """"f16" and "bf16" are the stochastically rounded formats (the mass-keeping defaults)."""
    assert B.STORAGE["f16"] == B.F16SR and B.STORAGE["bf16"] == B.BF16SR
    assert B.make_config(8, 8, storage="bf16").storage == B.BF16SR


def test_probe_library_exports_its_header():
    """libvplbm_probes.so (the measurement probes bench.py times) exports every call
    include/vplbm_probes.h declares and rejects bad arguments before any device work."""
    from paper_1812_05401_amd import probes as P
    text = open(os.path.join(os.path.dirname(HEADER), "vplbm_probes.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = sorted(set(re.findall(r"\b(vplbm_probe_[a-z_0-9]+)\s*\(", text)))
    assert len(names) == 4
    lib = P.load()
    for n in names:
        assert hasattr(lib, n), n
    out = C.c_double()
    assert lib.vplbm_probe_pattern(8192, 2048, 2, 100, 8, 10, C.byref(out)) == -1
    assert "no probe" in P.load().vplbm_probe_last_error().decode()
    assert lib.vplbm_probe_pattern(1000, 2048, 2, 128, 8, 10, C.byref(out)) == -1
    assert lib.vplbm_probe_pattern(8192, 2048, 1, 128, 2, 0, C.byref(out)) == -1
    assert lib.vplbm_probe_copy(1000, 5, C.byref(out)) == -1
    assert lib.vplbm_probe_fma(0, C.byref(out)) == -1
    assert lib.vplbm_probe_fma(5, None) == -1
