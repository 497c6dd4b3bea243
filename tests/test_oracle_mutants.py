"""Plant plausible mistakes in copies of the oracle and show the pins catch them.

Each mutant is a textual edit of oracle/sos_oracle.c (a sign, a dropped term,
a swapped state or index), compiled to a throw-away library in a temp dir. The
real oracle is never modified. A mutant passes this test only if at least one
pin in tests/pins.py rejects it.
"""
import ctypes
import os
import subprocess

import numpy as np
import pytest

from tests import pins

SRC = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "oracle",
                   "sos_oracle.c")
_dp = ctypes.POINTER(ctypes.c_double)

FORWARD_MUTANTS = {
    "feedback_sign_a1": ("z1 = b1 * u - a1 * y + z2;", "z1 = b1 * u + a1 * y + z2;"),
    "feedback_operand_a2": ("z2 = b2 * u - a2 * y;", "z2 = b2 * u - a2 * u;"),
    "dropped_b2": ("z2 = b2 * u - a2 * y;", "z2 = - a2 * y;"),
    "swapped_state_in_output": ("const double y = b0 * u + z1;", "const double y = b0 * u + z2;"),
    "unnormalized_a1": ("c[3] = row[4] / a0;", "c[3] = row[4];"),
    "zf_wrong_component": ("    state[0] = z1;", "    state[0] = z2;"),
    "zi_components_swapped": (
        "double st[2] = {zi ? zi[2 * k] : 0.0, zi ? zi[2 * k + 1] : 0.0};\n        tdf2_section(c, y, y, n, st);",
        "double st[2] = {zi ? zi[2 * k + 1] : 0.0, zi ? zi[2 * k] : 0.0};\n        tdf2_section(c, y, y, n, st);"),
    "b1_index_shift": ("z1 = b1 * u - a1 * y + z2;", "z1 = b2 * u - a1 * y + z2;"),
}

VJP_MUTANTS = {
    "vjp_gb1_wrong_adjoint": ("gb1 += g1 * u[t];", "gb1 += g2 * u[t];"),
    "vjp_state_shift": ("const double g2p = g1;", "const double g2p = g2;"),
    "vjp_a0_sign": ("gs[3] = -(gb0 * b0", "gs[3] = (gb0 * b0"),
    "vjp_ga1_operand": ("ga1 -= g1 * v[t];", "ga1 -= g1 * u[t];"),
    "vjp_total_adjoint_sign": ("const double gyt = gx[t] - a1 * g1 - a2 * g2;",
                               "const double gyt = gx[t] + a1 * g1 - a2 * g2;"),
}


def _build_mutant(tmp_path, name, old, new):
    src = open(SRC).read()
    assert src.count(old) >= 1, ("mutation anchor not found", name)
    mut = src.replace(old, new, 1)
    c = tmp_path / (name + ".c")
    so = tmp_path / (name + ".so")
    c.write_text(mut)
    subprocess.check_call(["gcc", "-O2", "-fPIC", "-shared", "-o", str(so), str(c), "-lpthread"])
    lib = ctypes.CDLL(str(so))
    lib.oracle_sosfilt.argtypes = [_dp, ctypes.c_int, _dp, ctypes.c_int64, _dp, _dp, _dp]
    lib.oracle_sosfilt_vjp.argtypes = [_dp, ctypes.c_int, _dp, ctypes.c_int64, _dp, _dp, _dp,
                                       _dp, _dp, _dp]

    def p(a):
        return None if a is None else a.ctypes.data_as(_dp)

    def sosfilt(sos, x, zi=None):
        sos = np.ascontiguousarray(sos, dtype=np.float64).reshape(-1, 6)
        x = np.ascontiguousarray(x, dtype=np.float64).reshape(-1)
        K = sos.shape[0]
        z = None if zi is None else np.ascontiguousarray(zi, dtype=np.float64).reshape(K, 2)
        y = np.empty_like(x)
        zf = np.empty((K, 2))
        lib.oracle_sosfilt(p(sos), K, p(x), x.size, p(z), p(y), p(zf))
        return y, zf

    def vjp(sos, x, zi, gy, gzf=None):
        sos = np.ascontiguousarray(sos, dtype=np.float64).reshape(-1, 6)
        x = np.ascontiguousarray(x, dtype=np.float64).reshape(-1)
        K = sos.shape[0]
        z = None if zi is None else np.ascontiguousarray(zi, dtype=np.float64).reshape(K, 2)
        gy = np.ascontiguousarray(gy, dtype=np.float64)
        g2 = None if gzf is None else np.ascontiguousarray(gzf, dtype=np.float64).reshape(K, 2)
        gx = np.empty_like(x)
        gzi = np.empty((K, 2))
        gs = np.empty((K, 6))
        lib.oracle_sosfilt_vjp(p(sos), K, p(x), x.size, p(z), p(gy), p(g2), p(gx), p(gzi), p(gs))
        return gx, gzi, gs

    return sosfilt, vjp


def _rejected(fn):
    try:
        with np.errstate(all="ignore"):
            fn()
    except (AssertionError, FloatingPointError, ValueError, ZeroDivisionError):
        return True
    return False


@pytest.mark.parametrize("name", sorted(FORWARD_MUTANTS))
def test_forward_mutant_is_caught(tmp_path, name):
    old, new = FORWARD_MUTANTS[name]
    sosfilt, _ = _build_mutant(tmp_path, name, old, new)
    caught = [c.__name__ for c in pins.ALL_FORWARD if _rejected(lambda: c(sosfilt))]
    assert caught, "no pin rejected mutant %s" % name


@pytest.mark.parametrize("name", sorted(VJP_MUTANTS))
def test_vjp_mutant_is_caught(tmp_path, name):
    old, new = VJP_MUTANTS[name]
    sosfilt, vjp = _build_mutant(tmp_path, name, old, new)
    assert _rejected(lambda: pins.check_vjp_finite_differences(sosfilt, vjp)), name
