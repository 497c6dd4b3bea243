"""Numpy model of the whole-cascade block-Toeplitz algorithm (test double).

Not an oracle and not the HIP code: it follows the steps of the matrix-core
path so that its algebra and its FP32 behaviour can be checked on the CPU
against the oracle. Sec. II-B's split (a non-recursive block-Toeplitz product,
then a recursion coupled only through carried state) is taken over the whole
cascade, the K sections' TDF-II states stacked into one state s:
  * per column of M consecutive samples, y = T x + O s and
    s' = A s + Gam x, with T the lower-triangular Toeplitz matrix of the
    cascade's impulse response, O = [c Phi^i], Gam = [Phi^(M-1-k) gamma],
    A = Phi^M;
  * columns form tiles, tiles form groups, groups form chunks; the columns'
    and tiles' end states from rest are composed by inclusive Kogge-Stone
    scans with powers of A and of A^TC; a chunk's aggregate is its end state
    from rest, and its incoming state comes from a decoupled lookback over
    the chunks before it (the aggregates of its nearest predecessors up to
    one whose inclusive state is known, each reaching this chunk through
    H^d, H the chunk map);
  * the state may be rescaled by a diagonal D of powers of two, which
    changes no result in exact arithmetic.
Every matrix is formed in FP64 and rounded once to `dtype`, as the tables.
"""
from __future__ import annotations

import numpy as np

S = 16


def cascade_ss(sos):
    """One-sample state map Phi, input vector gamma, output row c and
    feedthrough d of the cascade on stacked TDF-II states (FP64)."""
    sos = np.asarray(sos, np.float64)
    K = sos.shape[0]

    def step(s, x):
        s = s.copy()
        v = x
        for k in range(K):
            b0, b1, b2, a0, a1, a2 = sos[k] / sos[k, 3]
            y = b0 * v + s[2 * k]
            z1 = b1 * v - a1 * y + s[2 * k + 1]
            z2 = b2 * v - a2 * y
            s[2 * k], s[2 * k + 1] = z1, z2
            v = y
        return s, v

    phi = np.zeros((S, S))
    c = np.zeros(S)
    for i in range(2 * K):
        e = np.zeros(S)
        e[i] = 1.0
        phi[:, i], c[i] = step(e, 0.0)
    g, d = step(np.zeros(S), 1.0)
    return phi, g, c, d


def balance(phi, g, c, M):
    """Power-of-two scale per state entry equalising its Gam-row and O-column
    energy over one column."""
    P = np.eye(S)
    gr = np.zeros(S)
    oc = np.zeros(S)
    for _ in range(M):
        gr += (P @ g) ** 2
        oc += (c @ P) ** 2
        P = phi @ P
    D = np.ones(S)
    m = (gr > 0) & (oc > 0)
    D[m] = 2.0 ** np.rint(0.25 * np.log2(gr[m] / oc[m]))
    return D


def _mpow(X, e):
    R = np.eye(S)
    B = X.copy()
    while e:
        if e & 1:
            R = R @ B
        B = B @ B
        e >>= 1
    return R


def _scan(U, levels):
    """Inclusive Kogge-Stone over the columns of U with levels[j] = X^(2^j)."""
    P = U.copy()
    d = 1
    for Xd in levels:
        sh = np.zeros_like(P)
        sh[:, d:] = P[:, :-d]
        P = P + (Xd @ sh).astype(P.dtype)
        d *= 2
    return P


def run(sos, x, zi=None, dtype=np.float64, M=64, TC=16, NT=16, NG=8, balanced=True, rng=None):
    """Filter x (1-D) with the cascade; returns (y, zf) in float64. rng:
    random lookback lengths (where each walk finds an inclusive state)."""
    phi, g, c, d = cascade_ss(sos)
    K = np.asarray(sos).shape[0]
    D = balance(phi, g, c, M) if balanced else np.ones(S)
    Di = 1.0 / D
    phs = Di[:, None] * phi * D[None, :]
    gs = Di * g
    cs = c * D
    P = [np.eye(S)]
    for _ in range(M):
        P.append(phs @ P[-1])
    h = np.array([d] + [cs @ P[i - 1] @ gs for i in range(1, M)])
    T = np.zeros((M, M))
    for i in range(M):
        T[i, :i + 1] = h[i::-1]
    Gam = np.stack([P[M - 1 - k] @ gs for k in range(M)], 1)
    O = np.stack([cs @ P[i] for i in range(M)], 0)
    A = P[M]
    B = _mpow(A, TC)
    G = _mpow(B, NT)
    H = _mpow(G, NG)
    nlev = lambda X, cols: [_mpow(X, 1 << j) for j in range(int(np.log2(cols)))]
    f = lambda X: np.asarray(X, dtype)
    T, Gam, O, G1 = f(T), f(Gam), f(O), f(G)
    Alev, Blev = [f(X) for X in nlev(A, TC)], [f(X) for X in nlev(B, NT)]
    Acol = [f(_mpow(A, j)) for j in range(TC)]
    Btile = [f(_mpow(B, j)) for j in range(NT)]
    Hpow = [f(_mpow(H, j)) for j in range(64)]
    x = np.asarray(x, np.float64)
    n = x.size
    CG = M * TC * NT
    groups = -(-n // CG)
    chunks = -(-groups // NG)
    xp = np.zeros(chunks * NG * CG)
    xp[:n] = x
    X = f(xp).reshape(chunks, NG, NT, TC, M)
    y = np.zeros(chunks * NG * CG)
    s0 = np.zeros(S, dtype)
    if zi is not None:
        s0[:2 * K] = (np.asarray(zi, np.float64).reshape(-1) * Di[:2 * K]).astype(dtype)
    agg, inc = [None] * chunks, [None] * chunks
    zf_state = None
    for t in range(chunks):
        # sweep 1: the chunk's end state from rest
        GPs = []
        s = np.zeros(S, dtype)
        for j in range(NG):
            tot = np.stack([_scan(Gam @ X[t, j, k].T, Alev)[:, -1] for k in range(NT)], 1)
            GP = _scan(tot, Blev)
            GPs.append(GP)
            s = GP[:, -1] + G1 @ s
        agg[t] = s
        # lookback: the aggregates of the J nearest predecessors, then the
        # inclusive state of the next one, each through H^distance (J < 63;
        # random when rng is given: the walk ends wherever an inclusive state
        # is found)
        if t == 0:
            sin = s0
        else:
            J = 0 if rng is None else int(rng.integers(0, min(t, 63)))
            acc = Hpow[J] @ inc[t - 1 - J]
            for p in range(J):
                acc = acc + Hpow[p] @ agg[t - 1 - p]
            sin = acc
        inc[t] = agg[t] + Hpow[1] @ sin
        # sweep 2: outputs
        s = sin
        for j in range(NG):
            GP = GPs[j]
            for k in range(NT):
                st = (GP[:, k - 1] if k else np.zeros(S, dtype)) + Btile[k] @ s
                Xt = X[t, j, k].T
                Pc = _scan(Gam @ Xt, Alev)
                Sin = np.stack([(Pc[:, cidx - 1] if cidx else np.zeros(S, dtype)) + Acol[cidx] @ st
                                for cidx in range(TC)], 1)
                Yt = T @ Xt + O @ Sin
                base = ((t * NG + j) * NT + k) * TC * M
                y[base:base + TC * M] = Yt.T.reshape(-1)
                # final state of a signal ending inside this tile
                last = n - 1 - base
                if 0 <= last < TC * M:
                    cs_, rr = last // M, last % M + 1
                    sv = Sin[:, cs_].astype(np.float64)
                    xc = xp[base + cs_ * M: base + cs_ * M + rr]
                    for xi in xc:
                        sv = phs @ sv + gs * xi
                    zf_state = sv
            s = GP[:, -1] + G1 @ s
    return y[:n], (zf_state * D)[:2 * K].reshape(K, 2)
