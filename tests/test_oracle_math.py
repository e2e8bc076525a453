"""Pins of the oracle's elementary functions (explicit operation sequences,
independent of the platform's math library) against the C library and exact
special values: every result lies within a few units in the last place of
the correctly rounded value."""
import ctypes
import math

import numpy as np
import pytest

import oracle


def _fn(name):
    f = getattr(oracle.lib(), name)
    f.argtypes = [ctypes.c_double]
    f.restype = ctypes.c_double
    return f


def ulp_err(got, ref):
    got = np.asarray(got, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    u = np.spacing(np.abs(ref))
    return np.abs(got - ref) / u


def sweep(lo, hi, n=20000, seed=0, log=False):
    rng = np.random.default_rng(seed)
    if log:
        return np.exp(rng.uniform(math.log(lo), math.log(hi), n))
    return rng.uniform(lo, hi, n)


@pytest.mark.parametrize("name,ref,xs,maxulp", [
    ("or_exp", math.exp, sweep(-745, 709, 20000), 2.0),
    ("or_exp", math.exp, sweep(-2, 2, 20000, 1), 2.0),
    ("or_expm1", math.expm1, sweep(-50, 5, 20000), 3.0),
    ("or_expm1", math.expm1, -sweep(1e-300, 1.5, 20000, 2, log=True), 3.0),
    ("or_log", math.log, sweep(1e-300, 1e300, 20000, 3, log=True), 3.0),
    ("or_log", math.log, sweep(0.5, 2.0, 20000, 4), 3.0),
    ("or_log1p", math.log1p, sweep(-0.999999, 10, 20000, 5), 4.0),
    ("or_log1p", math.log1p, -sweep(1e-300, 0.5, 20000, 6, log=True), 4.0),
    ("or_atanh", math.atanh, sweep(-0.999999, 0.999999, 20000, 7), 5.0),
])
def test_elementary_function_accuracy(name, ref, xs, maxulp):
    f = _fn(name)
    got = np.array([f(float(x)) for x in xs])
    want = np.array([ref(float(x)) for x in xs])
    assert ulp_err(got, want).max() <= maxulp


def test_sincos_accuracy():
    lib = oracle.lib()
    lib.or_sincos.argtypes = [ctypes.c_double, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double)]
    xs = np.concatenate([sweep(0, 2 * math.pi, 20000, 8), sweep(-20, 20, 5000, 9),
                         [0.0, math.pi / 4, math.pi / 2, math.pi, 1.5 * math.pi]])
    s, c = ctypes.c_double(), ctypes.c_double()
    es, ec = [], []
    for x in xs:
        lib.or_sincos(float(x), ctypes.byref(s), ctypes.byref(c))
        # absolute error relative to 1 ulp of 1 (the values are O(1))
        es.append(abs(s.value - math.sin(x)) / 2.0 ** -53)
        ec.append(abs(c.value - math.cos(x)) / 2.0 ** -53)
    assert max(es) <= 4 and max(ec) <= 4


def test_special_values():
    assert _fn("or_exp")(0.0) == 1.0 and _fn("or_exp")(-1000.0) == 0.0
    assert math.isinf(_fn("or_exp")(1000.0))
    assert _fn("or_expm1")(0.0) == 0.0 and _fn("or_expm1")(1e-300) == 1e-300
    assert _fn("or_log")(1.0) == 0.0 and _fn("or_log1p")(0.0) == 0.0
    assert _fn("or_log1p")(1e-300) == 1e-300 and math.isinf(_fn("or_log1p")(-1.0))
    assert _fn("or_atanh")(0.0) == 0.0
    assert _fn("or_log")(math.e) == pytest.approx(1.0, rel=2e-16)
