"""Float64 numpy model of the GPU algorithm, used to check its algebra.

This is a test double for the kernel's *algorithm*, not a second oracle and not
the HIP code: it follows the same steps (lane = N consecutive samples, L lanes
per group, one divide-and-conquer level then one-sided cyclic reduction per
parity, cross-lane scan of the zero-state terminal states, decoupled lookback
between groups under a randomised completion order, back substitution with
the initial-condition terms) so that the readings of the paper's omitted steps
can be checked against the oracle on the CPU.

Readings modelled here (Zhai & Paris Part II):
* Eq. (23) generalised to a b0 != 1 feed-forward: the level-1 right-hand side is
  r1 = B(z) A(-z) x, whose taps are
  [b0, b1 - a1 b0, b2 - a1 b1 + a2 b0, a2 b1 - a1 b2, a2 b2].
* Level recursion (Part I Eq. (41), absent from this paper):
  e_{i+1} = 2 f_i - e_i^2, f_{i+1} = f_i^2, starting from e_1 = 2 a2 - a1^2,
  f_1 = a2^2, i.e. A_{i+1}(w^2) = A_i(w) A_i(-w).
* The lane's incoming state is the TDF-II pair (s1, s2); it enters the lane's
  recurrence only on its first two samples. At reduction level i the single
  row per parity whose references fall before the lane start (position
  2^i - 1 for the odd chain, 2^i - 2 for the even chain) receives the
  initial-condition term g[n] s1 + g[n-1] s2, g being the impulse response of
  1/A(z); every other row is the plain two-term back substitution. No division
  by e_i anywhere.
* Eqs. (24)-(25) with the sign corrected: the state after m lanes/groups is
  T^m s_in + (zero-state terminal state), T = [[-a1, 1], [-a2, 0]] acting on
  TDF-II states.
"""
from __future__ import annotations

import numpy as np


def normalized(row):
    b0, b1, b2, a0, a1, a2 = [float(v) for v in row]
    return b0 / a0, b1 / a0, b2 / a0, a1 / a0, a2 / a0


def level_coefs(a1, a2, levels):
    e = [a1, 2 * a2 - a1 * a1]
    f = [a2, a2 * a2]
    while len(e) <= levels:
        e.append(2 * f[-1] - e[-1] ** 2)
        f.append(f[-1] ** 2)
    return e, f


def impulse_1_over_A(a1, a2, n):
    g = np.zeros(n)
    g[0] = 1.0
    if n > 1:
        g[1] = -a1
    for m in range(2, n):
        g[m] = -a1 * g[m - 1] - a2 * g[m - 2]
    return g


def Tmat(a1, a2):
    return np.array([[-a1, 1.0], [-a2, 0.0]])


def lane_zero_state(u, c):
    """Fold + two-chain reduction on every lane at zero incoming state.
    u: L x N section input. Returns r (reduced right-hand sides, in place layout)
    and the lanes' zero-state terminal TDF-II states t (L x 2)."""
    b0, b1, b2, a1, a2 = c
    L, N = u.shape
    LOG = N.bit_length() - 1
    taps = [b0, b1 - a1 * b0, b2 - a1 * b1 + a2 * b0, a2 * b1 - a1 * b2, a2 * b2]
    r = np.zeros_like(u)
    for n in range(N):
        for k in range(5):
            if n - k >= 0:
                r[:, n] += taps[k] * u[:, n - k]
    e, f = level_coefs(a1, a2, LOG)
    for i in range(1, LOG):
        s = 1 << i
        for n in range(N - 1, -1, -1):
            if (n + 1) % (2 * s) == 0 or (n + 2) % (2 * s) == 0:
                v = r[:, n].copy()
                if n - s >= 0:
                    v -= e[i] * r[:, n - s]
                if n - 2 * s >= 0:
                    v += f[i] * r[:, n - 2 * s]
                r[:, n] = v
    y1, y2 = r[:, N - 1], r[:, N - 2]
    t = np.stack([b1 * u[:, N - 1] + b2 * u[:, N - 2] - a1 * y1 - a2 * y2,
                  b2 * u[:, N - 1] - a2 * y1], axis=1)
    return r, t


def lane_scan(t, TN):
    """Inclusive Kogge-Stone scan P[l] = t[l] + TN P[l-1] with the uniform
    matrices TN^(2^k), as the wave does it with cross-lane moves."""
    L = t.shape[0]
    P = t.copy()
    M = TN.copy()
    d = 1
    while d < L:
        Q = np.zeros_like(P)
        Q[d:] = P[:-d]
        P = P + Q @ M.T
        M = M @ M
        d *= 2
    return P


def back_substitute(r, s_lane, c):
    b0, b1, b2, a1, a2 = c
    L, N = r.shape
    LOG = N.bit_length() - 1
    e, f = level_coefs(a1, a2, LOG)
    g = np.r_[impulse_1_over_A(a1, a2, N), 0.0]      # g[-1] reads the trailing 0
    s1, s2 = s_lane[:, 0], s_lane[:, 1]
    y = np.zeros_like(r)
    y[:, N - 1] = r[:, N - 1] + g[N - 1] * s1 + g[N - 2] * s2
    y[:, N - 2] = r[:, N - 2] + g[N - 2] * s1 + g[N - 3] * s2
    for i in range(LOG - 1, 0, -1):
        s = 1 << i
        for n0 in (s - 1, s - 2):
            y[:, n0] = r[:, n0] + g[n0] * s1 + g[n0 - 1] * s2
            for n in range(n0 + 2 * s, N, 2 * s):
                y[:, n] = r[:, n] - e[i] * y[:, n - s] - f[i] * y[:, n - 2 * s]
    return y


def lane_particular(u, c):
    """PH (Sec. II-C): every lane's samples through the section from rest,
    the feed-forward B(z) and then the recursion 1/A(z) of Eq. (9) with zero
    history. Returns the particular solution w (L x N) and the lanes'
    zero-state terminal TDF-II states t (L x 2)."""
    b0, b1, b2, a1, a2 = c
    L, N = u.shape
    v = b0 * u
    v[:, 1:] += b1 * u[:, :-1]
    v[:, 2:] += b2 * u[:, :-2]
    w = np.zeros_like(u)
    for n in range(N):
        w[:, n] = v[:, n]
        if n >= 1:
            w[:, n] -= a1 * w[:, n - 1]
        if n >= 2:
            w[:, n] -= a2 * w[:, n - 2]
    t = np.stack([b1 * u[:, N - 1] + b2 * u[:, N - 2] - a1 * w[:, N - 1] - a2 * w[:, N - 2],
                  b2 * u[:, N - 1] - a2 * w[:, N - 1]], axis=1)
    return w, t


def homogeneous_correct(w, s_lane, c):
    """PH: add the free response of each lane's incoming TDF-II state (s1, s2)
    to every sample, y[m] = w[m] + g[m] s1 + g[m-1] s2 (the role of Eq. (11))."""
    a1, a2 = c[3], c[4]
    N = w.shape[1]
    g = np.r_[impulse_1_over_A(a1, a2, N), 0.0]      # g[-1] reads the trailing 0
    m = np.arange(N)
    return w + s_lane[:, 0:1] * g[m] + s_lane[:, 1:2] * g[m - 1]


def filter_model(sos, x, zi=None, N=8, L=4, window=3, seed=0, solver="dccr"):
    """Whole cascade over a signal of any length with the kernel's algorithm.
    Groups resolve their incoming states by decoupled lookback under a random
    interleaving of group progress. solver: "dccr" (fold, two-chain reduction,
    back substitution) or "ph" (particular solution, homogeneous correction);
    the scan and the lookback are the same. Returns (y, zf)."""
    zero_state, correct = ((lane_particular, homogeneous_correct) if solver == "ph"
                           else (lane_zero_state, back_substitute))
    sos = np.asarray(sos, dtype=np.float64).reshape(-1, 6)
    K = sos.shape[0]
    x = np.asarray(x, dtype=np.float64)
    n = x.size
    C = N * L
    G = max(1, -(-n // C))
    coefs = [normalized(row) for row in sos]
    zi = np.zeros((K, 2)) if zi is None else np.asarray(zi, dtype=np.float64).reshape(K, 2)
    if n == 0:
        return x.copy(), zi.copy()
    xp = np.zeros(G * C)
    xp[:n] = x
    data = [xp[g * C:(g + 1) * C].reshape(L, N).copy() for g in range(G)]
    agg = {}
    inc = {}
    zf = np.zeros((K, 2))
    rs = np.random.default_rng(seed)
    # per-group program counter: (section, phase); phases 0 local, 1 lookback
    pc = [[0, 0] for _ in range(G)]
    local = [None] * G
    last = (n - 1) // C
    pos_last = (n - 1) - last * C
    while any(p[0] < K for p in pc):
        live = [g for g in range(G) if pc[g][0] < K]
        g = int(rs.choice(live))
        s, ph = pc[g]
        c = coefs[s]
        TN = np.linalg.matrix_power(Tmat(c[3], c[4]), N)
        TC = np.linalg.matrix_power(TN, L)
        if ph == 0:
            u = data[g]
            r, t = zero_state(u, c)
            P = lane_scan(t, TN)
            local[g] = (u, r, P)
            if g == 0:
                inc[(0, s)] = TC @ zi[s] + P[-1]
            else:
                agg[(g, s)] = P[-1]
            pc[g][1] = 1
            continue
        # lookback: inspect a window of predecessors, compose if resolvable
        u, r, P = local[g]
        if g == 0:
            s_in = zi[s]
        else:
            acc = np.zeros(2)
            Macc = np.eye(2)
            base = g - 1
            s_in = None
            while True:
                idx = [base - j for j in range(window) if base - j >= 0]
                found = None
                ok = True
                vals = []
                for j, h in enumerate(idx):
                    if (h, s) in inc:
                        vals.append(inc[(h, s)])
                        found = j
                        break
                    if (h, s) in agg:
                        vals.append(agg[(h, s)])
                    else:
                        ok = False
                        break
                if not ok:
                    break                              # not resolvable yet: yield
                part = sum(np.linalg.matrix_power(TC, j) @ v for j, v in enumerate(vals))
                acc = acc + Macc @ part
                if found is not None:
                    s_in = acc
                    break
                Macc = Macc @ np.linalg.matrix_power(TC, len(vals))
                base -= len(vals)
            if s_in is None:
                continue
            inc[(g, s)] = TC @ s_in + P[-1]
        # incoming state of every lane, then the corrected section output
        Pexc = np.vstack([np.zeros(2), P[:-1]])
        pw = [np.linalg.matrix_power(TN, l) for l in range(L)]
        s_lane = np.stack([pw[l] @ s_in + Pexc[l] for l in range(L)])
        y = correct(r, s_lane, c)
        if g == last:
            # state after sample n-1 of this section (not at the padded group end)
            l1, p1 = divmod(pos_last, N)
            if p1 >= 1:
                xi1, xi2, yo1, yo2 = u[l1, p1], u[l1, p1 - 1], y[l1, p1], y[l1, p1 - 1]
                b0, b1, b2, a1, a2 = c
                zf[s] = [b1 * xi1 + b2 * xi2 - a1 * yo1 - a2 * yo2, b2 * xi1 - a2 * yo1]
            else:
                b0, b1, b2, a1, a2 = c
                ss = s_lane[l1]
                xv, yv = u[l1, 0], y[l1, 0]
                zf[s] = [b1 * xv - a1 * yv + ss[1], b2 * xv - a2 * yv]
        data[g] = y
        pc[g] = [s + 1, 0]
    y = np.concatenate([d.reshape(-1) for d in data])[:n]
    return y, zf


def vjp_model(sos, x, zi, gy, gzf):
    """The adjoint as the backward kernel computes it: per section, from the
    last to the first, in reversed time r = n-1-t:
      lam'[r] = g'[r] - a1 lam'[r-1] - a2 lam'[r-2],  (lam'[-1], lam'[-2]) = gzf[k]
      g_prev'[r] = b0 lam'[r] + b1 lam'[r-1] + b2 lam'[r-2]
      gb_i = sum_r lam'[r-i] u'[r],  ga_i = -sum_r lam'[r-i] v'[r]   (i = 0, 1, 2)
      gzi = (lam'[n-1], lam'[n-2])
    u, v = the section's forward input and output. Gradients w.r.t. raw rows
    follow from the normalised ones through the division by a0."""
    sos = np.asarray(sos, dtype=np.float64).reshape(-1, 6)
    K = sos.shape[0]
    x = np.asarray(x, dtype=np.float64)
    n = x.size
    zi = np.zeros((K, 2)) if zi is None else np.asarray(zi, dtype=np.float64)
    gzf = np.zeros((K, 2)) if gzf is None else np.asarray(gzf, dtype=np.float64)
    acts = [x.copy()]
    for k in range(K):
        b0, b1, b2, a1, a2 = normalized(sos[k])
        z1, z2 = zi[k]
        out = np.empty(n)
        for t in range(n):
            y = b0 * acts[-1][t] + z1
            z1 = b1 * acts[-1][t] - a1 * y + z2
            z2 = b2 * acts[-1][t] - a2 * y
            out[t] = y
        acts.append(out)
    g = np.asarray(gy, dtype=np.float64)[::-1].copy()
    gzi = np.zeros((K, 2))
    gsos = np.zeros((K, 6))
    for k in range(K - 1, -1, -1):
        b0, b1, b2, a1, a2 = normalized(sos[k])
        up, vp = acts[k][::-1], acts[k + 1][::-1]
        lam = np.zeros(n + 2)              # lam[j + 2] holds lam'[j]; lam'[-1], lam'[-2] first
        lam[1], lam[0] = gzf[k][0], gzf[k][1]
        for r in range(n):
            lam[r + 2] = g[r] - a1 * lam[r + 1] - a2 * lam[r]
        L0, L1, L2 = lam[2:], lam[1:-1], lam[:-2]
        gb = np.array([L0 @ up, L1 @ up, L2 @ up])
        ga = np.array([-(L1 @ vp), -(L2 @ vp)])
        gzi[k] = [L0[n - 1], L0[n - 2] if n >= 2 else gzf[k][0]]
        a0 = sos[k, 3]
        gsos[k, :3] = gb / a0
        gsos[k, 4:] = ga / a0
        gsos[k, 3] = -(gb @ np.array([b0, b1, b2]) + ga @ np.array([a1, a2])) / a0
        g = b0 * L0 + b1 * L1 + b2 * L2
    return g[::-1].copy(), gzi, gsos
