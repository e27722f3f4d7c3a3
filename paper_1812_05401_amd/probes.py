"""ctypes binding of the measurement probes (include/vplbm_probes.h, libvplbm_probes.so).

The probes advance no simulation: they time the step kernels' memory access patterns with a
trivial per-node update, a 16-byte copy and FP32 FMA chains, the ceilings bench.py reports the
step kernels against.  Argument marshalling only.
"""
import ctypes as C
import os

from . import build as _build

_lib = None


class ProbeError(RuntimeError):
    pass


def load():
    global _lib
    if _lib is None:
        if not os.path.exists(_build.PROBE_LIB):
            raise ProbeError(f"{_build.PROBE_LIB} is not built: run python -m paper_1812_05401_amd.build")
        L = C.CDLL(_build.PROBE_LIB)
        L.vplbm_probe_pattern.restype = C.c_int
        L.vplbm_probe_pattern.argtypes = [C.c_int32] * 6 + [C.POINTER(C.c_double)]
        L.vplbm_probe_copy.restype = C.c_int
        L.vplbm_probe_copy.argtypes = [C.c_uint64, C.c_int32, C.POINTER(C.c_double)]
        L.vplbm_probe_fma.restype = C.c_int
        L.vplbm_probe_fma.argtypes = [C.c_int32, C.POINTER(C.c_double)]
        L.vplbm_probe_last_error.restype = C.c_char_p
        L.vplbm_probe_last_error.argtypes = []
        _lib = L
    return _lib


def _check(rc):
    if rc != 0:
        raise ProbeError(f"probe failed ({rc}): {load().vplbm_probe_last_error().decode()}")


def pattern_us(nx, ny, steps_per_launch, tile=(128, 8), launches=64):
    """Mean launch time (us) of the access-pattern probe with `steps_per_launch` updates per launch."""
    out = C.c_double()
    _check(load().vplbm_probe_pattern(nx, ny, steps_per_launch, tile[0], tile[1], launches, C.byref(out)))
    return out.value


def copy_gbs(nbytes, reps=20):
    """Copy bandwidth (read + write bytes per second / 1e9) of a 16-byte-per-thread copy."""
    out = C.c_double()
    _check(load().vplbm_probe_copy(nbytes, reps, C.byref(out)))
    return out.value


def fma_rate(reps=20):
    """Lane FMAs per second of independent FP32 FMA chains (one VALU instruction per lane per FMA)."""
    out = C.c_double()
    _check(load().vplbm_probe_fma(reps, C.byref(out)))
    return out.value
