"""The kernel's algorithm, modelled in float64 numpy (tests/dccr_model.py),
reproduces the oracle: this checks the readings of the paper's omitted
steps (IC terms, level recursion, sign of the state correction, state at
sample n-1) before and independently of the HIP code."""
import numpy as np
import pytest

import oracle
from tests import dccr_model as M
from tests.pins import biquad_from_poles


def _rows(K, seed, r_hi=0.99):
    g = np.random.default_rng(seed)
    return np.stack([biquad_from_poles(g.uniform(0.5, r_hi), g.uniform(0, np.pi),
                                       b=tuple(g.normal(size=3))) for _ in range(K)])


@pytest.mark.parametrize("N,L", [(2, 4), (4, 4), (8, 4), (16, 8), (32, 2), (8, 16)])
@pytest.mark.parametrize("K", [1, 3])
def test_model_matches_oracle(N, L, K):
    rows = _rows(K, 100 + N + L + K)
    g = np.random.default_rng(N * L + K)
    zi = g.normal(size=(K, 2))
    for n in (1, 2, 3, N * L - 1, N * L, N * L + 1, 5 * N * L + 3):
        x = g.normal(size=n)
        y, zf = M.filter_model(rows, x, zi, N=N, L=L, window=3, seed=n)
        yr, zfr = oracle.sosfilt(rows, x, zi)
        assert np.max(np.abs(y - yr)) < 1e-10 * max(1, np.max(np.abs(yr))), (N, L, K, n)
        assert np.max(np.abs(zf - zfr)) < 1e-10 * max(1, np.max(np.abs(zfr))), (N, L, K, n)


@pytest.mark.parametrize("N,L", [(2, 4), (4, 4), (8, 4), (16, 8), (32, 2), (8, 16)])
@pytest.mark.parametrize("K", [1, 3])
def test_ph_model_matches_oracle(N, L, K):
    """The PH solver (particular solution from rest, then the homogeneous
    correction from the scanned TDF-II carries) reproduces the oracle."""
    rows = _rows(K, 200 + N + L + K)
    g = np.random.default_rng(N * L + K + 7)
    zi = g.normal(size=(K, 2))
    for n in (1, 2, 3, N * L - 1, N * L, N * L + 1, 5 * N * L + 3):
        x = g.normal(size=n)
        y, zf = M.filter_model(rows, x, zi, N=N, L=L, window=3, seed=n, solver="ph")
        yr, zfr = oracle.sosfilt(rows, x, zi)
        assert np.max(np.abs(y - yr)) < 1e-10 * max(1, np.max(np.abs(yr))), (N, L, K, n)
        assert np.max(np.abs(zf - zfr)) < 1e-10 * max(1, np.max(np.abs(zfr))), (N, L, K, n)


def test_ph_correction_is_eq11_in_state_coordinates():
    """Eq. (11) corrects the particular solution with u_{2,m} y[-2] + u_{1,m}
    y[-1] (DF-I output history, u from powers of Phi); the kernel uses
    g[m] s1 + g[m-1] s2 on the TDF-II state. With the input history folded
    into the particular solution the two agree: for zero lane input, the
    correction alone must equal the free response from (y[-2], y[-1])."""
    b0, b1, b2, a1, a2 = 1.0, 0.0, 0.0, -1.2, 0.6
    Phi = np.array([[0.0, 1.0], [-a2, -a1]])
    ym2, ym1 = 0.7, -0.3
    N = 12
    # TDF-II state of a pure recursive section whose last outputs are (y[-2], y[-1])
    s = np.array([[-(a1 * ym1 + a2 * ym2), -a2 * ym1]])
    corr = M.homogeneous_correct(np.zeros((1, N)), s, (b0, b1, b2, a1, a2))[0]
    u2 = np.array([-np.linalg.matrix_power(Phi, m + 1)[1, 0] for m in range(N)])
    u1 = np.array([-np.linalg.matrix_power(Phi, m + 1)[1, 1] for m in range(N)])
    assert np.allclose(corr, -(u2 * ym2 + u1 * ym1), atol=1e-14)


def test_model_random_completion_orders():
    rows = _rows(4, 7)
    x = np.random.default_rng(8).normal(size=40 * 32 + 5)
    yr, zfr = oracle.sosfilt(rows, x)
    for seed in range(6):
        for window in (1, 2, 5, 64):
            y, zf = M.filter_model(rows, x, None, N=8, L=4, window=window, seed=seed)
            assert np.max(np.abs(y - yr)) < 1e-10 * np.max(np.abs(yr))
            assert np.max(np.abs(zf - zfr)) < 1e-10 * np.max(np.abs(zfr))


def test_level_recursion_closed_form():
    """e_i = -2 r^(2^i) cos(2^i th), f_i = r^(2^(i+1)) for a complex pole pair."""
    r, th = 0.93, 1.234
    a1, a2 = -2 * r * np.cos(th), r * r
    e, f = M.level_coefs(a1, a2, 6)
    for i in range(7):
        assert abs(e[i] - (-2 * r ** (2 ** i) * np.cos(2 ** i * th))) < 1e-13
        assert abs(f[i] - r ** (2 ** (i + 1))) < 1e-13


def test_reduced_recurrence_holds():
    """y[n] + e_i y[n-2^i] + f_i y[n-2^(i+1)] = (prod_j<i A_j(-z^(2^j)) B(z) x)[n]."""
    row = _rows(1, 3)[0]
    b0, b1, b2, a1, a2 = M.normalized(row)
    x = np.random.default_rng(4).normal(size=400)
    y, _ = oracle.sosfilt(row.reshape(1, 6), x)
    e, f = M.level_coefs(a1, a2, 5)
    poly = np.array([b0, b1, b2])
    for i in range(1, 6):
        s = 1 << (i - 1)
        Aneg = np.zeros(2 * s + 1)
        Aneg[0], Aneg[s], Aneg[2 * s] = 1.0, -e[i - 1], f[i - 1]
        poly = np.convolve(poly, Aneg)
        rhs = np.convolve(x, poly)[:400]
        S = 1 << i
        lhs = y.copy()
        lhs[S:] += e[i] * y[:-S]
        lhs[2 * S:] += f[i] * y[:-2 * S]
        assert np.max(np.abs(lhs - rhs)) < 1e-11


def test_printed_sign_of_state_correction_is_wrong():
    """Eq. (24) as printed (minus C^(l+1)) disagrees with the scan of Eq. (13);
    the corrected sign, (-C)^(l+1) = Phi^(N(l+1)), agrees."""
    row = _rows(1, 9)[0]
    b0, b1, b2, a1, a2 = M.normalized(row)
    N, L = 8, 4
    Phi = np.array([[0.0, 1.0], [-a2, -a1]])       # acts on DF-I pairs [y[-2], y[-1]]
    C = -np.linalg.matrix_power(Phi, N)
    g = np.random.default_rng(10)
    we = g.normal(size=(L, 2))
    ym1 = g.normal(size=2)
    ye = np.zeros((L, 2))
    prev = ym1
    for l in range(L):                               # Eq. (13)
        ye[l] = we[l] - C @ prev
        prev = ye[l]
    ye0 = np.zeros((L, 2))
    prev = np.zeros(2)
    for l in range(L):
        ye0[l] = we[l] - C @ prev
        prev = ye0[l]
    printed = np.stack([ye0[l] - np.linalg.matrix_power(C, l + 1) @ ym1 for l in range(L)])
    corrected = np.stack([ye0[l] + np.linalg.matrix_power(-C, l + 1) @ ym1 for l in range(L)])
    assert np.max(np.abs(corrected - ye)) < 1e-12
    assert np.max(np.abs(printed - ye)) > 1e-3


def test_vjp_model_matches_oracle():
    """The backward kernel's formulation (reversed-time 1/A, 3-tap FIR, lambda
    correlations) reproduces the oracle's reverse sweep."""
    g = np.random.default_rng(50)
    for K, n in ((1, 40), (3, 57), (4, 2), (2, 1)):
        rows = _rows(K, 60 + K)
        rows[0] *= 1.3                         # a0 != 1
        x = g.normal(size=n)
        zi = g.normal(size=(K, 2))
        gy = g.normal(size=n)
        gzf = g.normal(size=(K, 2))
        gx, gzi, gs = M.vjp_model(rows, x, zi, gy, gzf)
        rx, rzi, rs = oracle.sosfilt_vjp(rows, x, zi, gy, gzf)
        assert np.max(np.abs(gx - rx)) < 1e-10 * max(1, np.max(np.abs(rx)))
        assert np.max(np.abs(gzi - rzi)) < 1e-10 * max(1, np.max(np.abs(rzi)))
        assert np.max(np.abs(gs - rs)) < 1e-10 * max(1, np.max(np.abs(rs)))
