"""Independent pins for the FP64 oracle.

Each check takes the oracle's entry points (``sosfilt(sos, x, zi) -> (y, zf)``
and ``vjp(sos, x, zi, gy, gzf) -> (gx, gzi, gsos)``) and compares them with
something the paper or plain mathematics fixes, never with a retyped copy of
the oracle's own TDF-II loop:

* closed-form impulse responses of one biquad (complex, real and repeated
  poles) and of a cascade (convolution of per-section closed forms);
* the steady-state response to a sinusoid, |H(e^{jw})| cos(wn + arg H);
* Butterworth design facts (unit DC gain, -3 dB at the cutoff, zero at Nyquist);
* superposition in x and in zi, and chaining of chunks through zf -> zi;
* Eq. (1) of the paper evaluated as a direct-form-I loop on tiny inputs, with
  the initial state given as past samples (maps onto TDF-II zi);
* the multi-block system of Sec. II-B, Eqs. (2)-(3), assembled densely in the
  stride-N permuted order and solved with numpy.linalg.solve, group by group;
* scipy.signal.sosfilt in float64;
* central finite differences of the forward program for every gradient.

A check raises AssertionError on failure. tests/test_oracle_mutants.py
re-runs these checks against deliberately broken copies of the oracle to show
that plausible mistakes do not pass.
"""
from __future__ import annotations

import numpy as np


# ----------------------------------------------------------------- helpers

def biquad_from_poles(r, th, b=(1.0, 0.3, -0.2)):
    """Section with complex pole pair r e^{+-j th}: a = [1, -2 r cos th, r^2]."""
    return np.array([b[0], b[1], b[2], 1.0, -2.0 * r * np.cos(th), r * r])


def closed_form_impulse(row, n):
    """Impulse response of one section from the closed form of 1/A(z).

    Complex poles r e^{+-j th}: g[m] = r^m sin((m+1) th) / sin th.
    Real distinct poles p1, p2: g[m] = (p1^{m+1} - p2^{m+1}) / (p1 - p2).
    Repeated pole p: g[m] = (m+1) p^m.
    Then h[m] = (b0 g[m] + b1 g[m-1] + b2 g[m-2]) / a0."""
    b0, b1, b2, a0, a1, a2 = [float(v) for v in row]
    a1 /= a0
    a2 /= a0
    m = np.arange(n, dtype=np.float64)
    disc = a1 * a1 - 4.0 * a2
    if disc < -1e-14:
        r = np.sqrt(a2)
        th = np.arccos(-a1 / (2.0 * r))
        g = r ** m * np.sin((m + 1) * th) / np.sin(th)
    elif disc > 1e-14:
        p1 = (-a1 + np.sqrt(disc)) / 2.0
        p2 = (-a1 - np.sqrt(disc)) / 2.0
        g = (p1 ** (m + 1) - p2 ** (m + 1)) / (p1 - p2)
    else:
        p = -a1 / 2.0
        g = (m + 1) * p ** m
    h = b0 * g
    h[1:] += b1 * g[:-1]
    h[2:] += b2 * g[:-2]
    return h / a0


def freq_response(sos, w):
    """H(e^{jw}) of the cascade as a product of per-section rational functions."""
    z = np.exp(-1j * w)
    H = 1.0 + 0j
    for b0, b1, b2, a0, a1, a2 in np.asarray(sos, dtype=np.float64):
        H *= (b0 + b1 * z + b2 * z * z) / (a0 + a1 * z + a2 * z * z)
    return H


def rel_err(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    den = max(np.linalg.norm(b), 1e-300)
    return float(np.linalg.norm(a - b) / den)


# ------------------------------------------------------------------ checks

def check_impulse_closed_forms(sosfilt):
    cases = [
        biquad_from_poles(0.9, 0.7),
        biquad_from_poles(0.99, 2.5, b=(0.5, -1.0, 0.25)),
        biquad_from_poles(0.5, 0.05, b=(2.0, 0.0, 0.0)),
        np.array([1.0, 0.4, 0.1, 1.0, -(0.8 + -0.3), 0.8 * -0.3]),     # real poles 0.8, -0.3
        np.array([0.7, -0.2, 0.05, 1.0, -2 * 0.6, 0.36]),              # repeated pole 0.6
        np.array([2.0, 0.8, 0.6, 2.0, -1.2, 0.5]),                     # a0 != 1
        np.array([0.0, 1.0, 0.5, 1.0, -0.5, 0.25]),                    # b0 == 0
    ]
    n = 300
    x = np.zeros(n)
    x[0] = 1.0
    for row in cases:
        y, _ = sosfilt(row.reshape(1, 6), x)
        h = closed_form_impulse(row, n)
        err = np.max(np.abs(y - h)) / np.max(np.abs(h))
        assert err < 1e-12, ("impulse closed form", row, err)


def check_cascade_impulse(sosfilt):
    g = np.random.default_rng(11)
    for K in (2, 3, 5):
        rows = np.stack([biquad_from_poles(g.uniform(0.3, 0.95), g.uniform(0.1, 3.0),
                                           b=tuple(g.normal(size=3))) for _ in range(K)])
        n = 256
        h = np.zeros(n)
        h[0] = 1.0
        for row in rows:              # convolution of the per-section closed forms
            h = np.convolve(h, closed_form_impulse(row, n))[:n]
        x = np.zeros(n)
        x[0] = 1.0
        y, _ = sosfilt(rows, x)
        assert np.max(np.abs(y - h)) < 1e-12 * max(1.0, np.max(np.abs(h))), ("cascade impulse", K)


def check_steady_state_sinusoid(sosfilt):
    g = np.random.default_rng(12)
    rows = np.stack([biquad_from_poles(g.uniform(0.3, 0.9), g.uniform(0.1, 3.0),
                                       b=tuple(g.normal(size=3))) for _ in range(3)])
    n = 2000
    t = np.arange(n)
    for w in (0.05, 0.7, 2.9):
        y, _ = sosfilt(rows, np.cos(w * t))
        H = freq_response(rows, w)
        ref = np.abs(H) * np.cos(w * t + np.angle(H))
        tail = slice(n - 500, n)      # transient has decayed below 1e-13 by then
        assert np.max(np.abs(y[tail] - ref[tail])) < 1e-10, ("steady state", w)


def check_butterworth_facts(sosfilt):
    from scipy.signal import butter

    sos = butter(2, 0.2, output="sos")
    # bilinear closed form of the 2nd-order Butterworth at 0.2*Nyquist
    W = np.tan(0.1 * np.pi)
    d = 1.0 + np.sqrt(2.0) * W + W * W
    b = np.array([W * W, 2 * W * W, W * W]) / d
    a = np.array([1.0, 2.0 * (W * W - 1.0) / d, (1.0 - np.sqrt(2.0) * W + W * W) / d])
    assert np.allclose(sos[0, :3], b, atol=1e-15) and np.allclose(sos[0, 3:], a, atol=1e-15)
    n = 4000
    t = np.arange(n)
    for K in (1, 2, 4, 8):
        s = butter(2 * K, 0.2, output="sos")
        tail = slice(n - 200, n)
        y, _ = sosfilt(s, np.ones(n))                    # DC gain 1
        assert np.max(np.abs(y[tail] - 1.0)) < 1e-9, ("DC", K)
        y, _ = sosfilt(s, (-1.0) ** t)                   # zero at Nyquist
        assert np.max(np.abs(y[tail])) < 1e-9, ("Nyquist", K)
        y, _ = sosfilt(s, np.cos(0.2 * np.pi * t))       # -3 dB at the cutoff
        amp = np.sqrt(2.0 * np.mean(y[tail] ** 2))       # 200 samples = 20 whole periods
        assert abs(amp - 1.0 / np.sqrt(2.0)) < 1e-9, ("cutoff", K, amp)


def check_superposition(sosfilt):
    g = np.random.default_rng(13)
    K = 4
    rows = np.stack([biquad_from_poles(g.uniform(0.5, 0.99), g.uniform(0, np.pi),
                                       b=tuple(g.normal(size=3))) for _ in range(K)])
    x1 = g.normal(size=500)
    x2 = g.normal(size=500)
    zi = g.normal(size=(K, 2))
    ya, zfa = sosfilt(rows, x1, zi)
    yb, zfb = sosfilt(rows, x1, None)
    yc, zfc = sosfilt(rows, np.zeros(500), zi)
    assert np.max(np.abs(ya - (yb + yc))) < 1e-12 * np.max(np.abs(ya)), "superposition x/zi"
    assert np.max(np.abs(zfa - (zfb + zfc))) < 1e-12 * np.max(np.abs(zfa)), "superposition zf"
    y1, _ = sosfilt(rows, x1)
    y2, _ = sosfilt(rows, x2)
    y3, _ = sosfilt(rows, 2.5 * x1 - 0.75 * x2)
    assert np.max(np.abs(y3 - (2.5 * y1 - 0.75 * y2))) < 1e-12 * np.max(np.abs(y3)), "linearity"


def check_chunk_chaining(sosfilt):
    g = np.random.default_rng(14)
    K = 3
    rows = np.stack([biquad_from_poles(g.uniform(0.5, 0.99), g.uniform(0, np.pi),
                                       b=tuple(g.normal(size=3))) for _ in range(K)])
    x = g.normal(size=3000)
    zi = g.normal(size=(K, 2))
    yw, zfw = sosfilt(rows, x, zi)
    cuts = np.sort(g.choice(np.arange(1, 3000), size=7, replace=False))
    parts = []
    z = zi
    for a, b in zip(np.r_[0, cuts], np.r_[cuts, 3000]):
        yp, z = sosfilt(rows, x[a:b], z)
        parts.append(yp)
    yc = np.concatenate(parts)
    assert np.max(np.abs(yc - yw)) <= 1e-13 * np.max(np.abs(yw)), "chunk chaining y"
    assert np.max(np.abs(z - zfw)) <= 1e-13 * np.max(np.abs(zfw)), "chunk chaining zf"
    y0, zf0 = sosfilt(rows, x[:0], zi)                    # empty input: zf = zi
    assert y0.size == 0 and np.array_equal(zf0, zi), "empty input"


def check_direct_form_one(sosfilt):
    """Eq. (1) as a literal DF-I loop, initial conditions given as past samples."""
    g = np.random.default_rng(15)
    for trial in range(4):
        b0, b1, b2 = g.normal(size=3)
        r, th = g.uniform(0.3, 0.98), g.uniform(0, np.pi)
        a1, a2 = -2 * r * np.cos(th), r * r
        row = np.array([[b0, b1, b2, 1.0, a1, a2]])
        n = 40
        xs = g.normal(size=n + 2)             # xs[0], xs[1] are x[-2], x[-1]
        ys = np.zeros(n + 2)
        ys[0], ys[1] = g.normal(size=2)       # y[-2], y[-1]
        for t in range(2, n + 2):
            ys[t] = b0 * xs[t] + b1 * xs[t - 1] + b2 * xs[t - 2] - a1 * ys[t - 1] - a2 * ys[t - 2]
        # the same past expressed as a TDF-II state before sample 0
        s1 = b1 * xs[1] + b2 * xs[0] - a1 * ys[1] - a2 * ys[0]
        s2 = b2 * xs[1] - a2 * ys[1]
        y, zf = sosfilt(row, xs[2:], np.array([[s1, s2]]))
        assert np.max(np.abs(y - ys[2:])) < 1e-12 * max(1, np.max(np.abs(ys))), "DF-I"
        zf_ref = [b1 * xs[-1] + b2 * xs[-2] - a1 * ys[-1] - a2 * ys[-2], b2 * xs[-1] - a2 * ys[-1]]
        assert np.max(np.abs(zf[0] - zf_ref)) < 1e-12 * max(1, np.max(np.abs(ys))), "DF-I zf"


def multiblock_matrices(N, L, a1, a2, b1, b2):
    """Dense A, B (NL x NL) and A_-, B_- (NL x 2) of Eqs. (2)-(3), in the stride-N
    permuted order: row m*L + l holds sample l*N + m of the group."""
    I = np.eye(L)
    R = np.eye(L, k=-1)                 # lower shift: (R v)_l = v_{l-1}
    def blocks(c1, c2):
        M = np.zeros((N * L, N * L))
        def put(i, j, blk):
            M[i * L:(i + 1) * L, j * L:(j + 1) * L] += blk
        for m in range(N):
            put(m, m, I)
            if m >= 1:
                put(m, m - 1, c1 * I)
            if m >= 2:
                put(m, m - 2, c2 * I)
        # corner coupling: the first two blocks reach the previous lane's end
        put(0, N - 1, c1 * R)
        put(0, N - 2, c2 * R)
        put(1, N - 1, c2 * R)
        return M
    A = blocks(a1, a2)
    Bm = blocks(b1, b2)
    # initial-state couplings, columns ordered as [v[-2], v[-1]]
    Am = np.zeros((N * L, 2))
    Bmm = np.zeros((N * L, 2))
    Am[0, :] = [a2, a1]             # sample 0: a2 y[-2] + a1 y[-1]
    Am[L, :] = [0.0, a2]            # sample 1: a2 y[-1]
    Bmm[0, :] = [b2, b1]
    Bmm[L, :] = [0.0, b2]
    return A, Bm, Am, Bmm


def check_multiblock_dense(sosfilt):
    """Solve A y = B x + B_- x_-1 - A_- y_-1 group by group and compare with the
    oracle over the whole signal (b0 = 1 as in Eq. (1))."""
    g = np.random.default_rng(16)
    for (N, L) in ((8, 4), (4, 8), (3, 5), (16, 4)):
        r, th = g.uniform(0.4, 0.97), g.uniform(0, np.pi)
        a1, a2 = -2 * r * np.cos(th), r * r
        b1, b2 = g.normal(size=2)
        A, Bm, Am, Bmm = multiblock_matrices(N, L, a1, a2, b1, b2)
        C = N * L
        G = 3
        x = g.normal(size=G * C)
        perm = np.array([l * N + m for m in range(N) for l in range(L)])   # row -> sample
        ym1 = np.zeros(2)
        xm1 = np.zeros(2)
        out = np.zeros(G * C)
        for grp in range(G):
            xg = x[grp * C:(grp + 1) * C]
            rhs = Bm @ xg[perm] + Bmm @ xm1 - Am @ ym1
            yperm = np.linalg.solve(A, rhs)
            yg = np.empty(C)
            yg[perm] = yperm
            out[grp * C:(grp + 1) * C] = yg
            ym1 = yg[-2:].copy()
            xm1 = xg[-2:].copy()
        y, _ = sosfilt(np.array([[1.0, b1, b2, 1.0, a1, a2]]), x)
        assert np.max(np.abs(y - out)) < 1e-11 * max(1.0, np.max(np.abs(out))), ("multiblock", N, L)


def check_scipy(sosfilt):
    from scipy.signal import sosfilt as sp_sosfilt

    g = np.random.default_rng(17)
    for K in (1, 4, 8):
        rows = np.stack([biquad_from_poles(g.uniform(0.5, 0.995), g.uniform(0, np.pi),
                                           b=tuple(g.normal(size=3))) for _ in range(K)])
        x = g.normal(size=4000)
        zi = g.normal(size=(K, 2))
        y, zf = sosfilt(rows, x, zi)
        ys, zfs = sp_sosfilt(rows, x, zi=zi)
        assert rel_err(y, ys) < 1e-12 and rel_err(zf, zfs) < 1e-12, ("scipy", K)


def _fd(f, p, h):
    return (f(p + h) - f(p - h)) / (2 * h)


def check_vjp_finite_differences(sosfilt, vjp):
    g = np.random.default_rng(18)
    K = 3
    rows = np.stack([biquad_from_poles(g.uniform(0.4, 0.9), g.uniform(0.2, 2.8),
                                       b=tuple(g.normal(size=3))) for _ in range(K)])
    rows[1, :] *= 1.7                      # a0 != 1 on one section
    n = 60
    x = g.normal(size=n)
    zi = g.normal(size=(K, 2))
    gy = g.normal(size=n)
    gzf = g.normal(size=(K, 2))

    def loss(s, xx, z):
        y, zf = sosfilt(s, xx, z)
        return float(np.dot(gy, y) + np.sum(gzf * zf))

    gx, gzi, gsos = vjp(rows, x, zi, gy, gzf)
    h = 1e-6
    for i in range(n):
        e = np.zeros(n)
        e[i] = 1.0
        fd = _fd(lambda d: loss(rows, x + d * e, zi), 0.0, h)
        assert abs(fd - gx[i]) < 1e-6 * max(1.0, abs(fd)), ("gx", i, fd, gx[i])
    for k in range(K):
        for j in range(2):
            e = np.zeros((K, 2))
            e[k, j] = 1.0
            fd = _fd(lambda d: loss(rows, x, zi + d * e), 0.0, h)
            assert abs(fd - gzi[k, j]) < 1e-6 * max(1.0, abs(fd)), ("gzi", k, j)
        for j in range(6):
            e = np.zeros((K, 6))
            e[k, j] = 1.0
            hh = h * max(1.0, abs(rows[k, j]))
            fd = _fd(lambda d: loss(rows + d * e, x, zi), 0.0, hh)
            assert abs(fd - gsos[k, j]) < 1e-5 * max(1.0, abs(fd)), ("gsos", k, j, fd, gsos[k, j])


ALL_FORWARD = [
    check_impulse_closed_forms,
    check_cascade_impulse,
    check_steady_state_sinusoid,
    check_butterworth_facts,
    check_superposition,
    check_chunk_chaining,
    check_direct_form_one,
    check_multiblock_dense,
    check_scipy,
]
