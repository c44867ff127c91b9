"""Dense assembly of the normal-equation matrix for tiny configurations.

A second, independent construction of the operator from the definitions:
explicit matrices for the wavelet transform (Kronecker products of 1-D
periodic analysis matrices), the bilinear projection (Kronecker product of two
1-D interpolation matrices), the Fried stencil, low-order aggregation, the
2x2 noise blocks and the tip/tilt projector.  Only the filter taps, the pupil
mask and the prior values are taken from the oracle (each has its own pins).
"""
import math

import numpy as np
import scipy.sparse as sp

import oracle as O


def analysis_matrix(M, h):
    g = np.array([(-1.0) ** n * h[len(h) - 1 - n] for n in range(len(h))])
    A = np.zeros((M, M))
    for k in range(M // 2):
        for n in range(len(h)):
            A[k, (2 * k + n) % M] += h[n]
            A[M // 2 + k, (2 * k + n) % M] += g[n]
    return A


def wavelet_matrix(N, levels, h):
    W = np.eye(N * N)
    for lev in range(levels):
        M = N >> lev
        A1 = analysis_matrix(M, h)
        step = np.kron(A1, np.eye(M)) @ np.kron(np.eye(M), A1)
        E = np.eye(N * N)
        sel = np.array([x * N + y for x in range(M) for y in range(M)])
        E[np.ix_(sel, sel)] = step
        W = E @ W
    return W


def interp_matrix(n_sub, D, scale, shift, N, d):
    B = np.zeros((n_sub + 1, N))
    for i in range(n_sub + 1):
        X = scale * (i - n_sub / 2.0) * (D / n_sub) + shift
        u = X / d + N / 2.0
        i0 = min(max(int(math.floor(u)), 0), N - 2)
        t = u - i0
        B[i, i0] += 1.0 - t
        B[i, i0 + 1] += t
    return B


def fried_matrix(mask):
    n = mask.shape[0]
    act = [(i, j) for i in range(n) for j in range(n) if mask[i, j]]
    S = len(act)
    G = np.zeros((2 * S, (n + 1) ** 2))

    def node(i, j):
        return i * (n + 1) + j

    for q, (i, j) in enumerate(act):
        G[q, node(i + 1, j)] += 0.5
        G[q, node(i, j)] -= 0.5
        G[q, node(i + 1, j + 1)] += 0.5
        G[q, node(i, j + 1)] -= 0.5
        G[S + q, node(i, j + 1)] += 0.5
        G[S + q, node(i, j)] -= 0.5
        G[S + q, node(i + 1, j + 1)] += 0.5
        G[S + q, node(i + 1, j)] -= 0.5
    return G, act


def aggregation_matrix(mask, act, k):
    n = mask.shape[0]
    b = n // k
    cells = []
    for ci in range(k):
        for cj in range(k):
            members = [q for q, (i, j) in enumerate(act) if i // b == ci and j // b == cj]
            if members:
                cells.append(members)
    S = len(act)
    Q = np.zeros((2 * len(cells), 2 * S))
    for c, members in enumerate(cells):
        for q in members:
            Q[c, q] = 1.0 / len(members)
            Q[len(cells) + c, S + q] = 1.0 / len(members)
    return Q


def block_matrix(blocks):
    S = blocks.shape[0]
    C = np.zeros((2 * S, 2 * S))
    for q in range(S):
        a, b, c = blocks[q]
        C[q, q], C[q, S + q], C[S + q, q], C[S + q, S + q] = a, b, b, c
    return C


def tt_projector(S):
    one = np.zeros((2 * S, 2))
    one[:S, 0] = 1.0 / math.sqrt(S)
    one[S:, 1] = 1.0 / math.sqrt(S)
    return np.eye(2 * S) - one @ one.T


def assemble(cfg, sigmas, cinv_blocks=None, precond_only=False):
    """Returns (A, list of per-sensor (A~_m, N_m)) with A the full matrix."""
    sysm = O.System(cfg, sigmas, cinv_blocks)
    h = O.db3_lowpass()
    Wl = [wavelet_matrix(L["n"], cfg["levels"], h) if cfg["levels"] else np.eye(L["n"] ** 2)
          for L in cfg["layers"]]
    W = sp.block_diag(Wl).toarray()
    parts = []
    A = np.zeros((sysm.n, sysm.n))
    for m, w in enumerate(cfg["wfs"]):
        sen = sysm.sensors[m]
        mask = sen["mask"]
        if w.get("kind", "sh") == "phase":
            n = mask.shape[0]
            on = np.zeros((n + 1, n + 1), bool)
            for i in range(n):
                for j in range(n):
                    if mask[i, j]:
                        on[i:i + 2, j:j + 2] = True
            idx = np.flatnonzero(on.ravel())
            G = np.zeros((len(idx), (n + 1) ** 2))
            G[np.arange(len(idx)), idx] = 1.0
        else:
            G, act = fried_matrix(mask)
            if w["tt_aggregate"]:
                G = aggregation_matrix(mask, act, w["tt_aggregate"]) @ G
        cols = []
        for L in cfg["layers"]:
            s = 1.0 - L["altitude"] / w["H"] if w["lgs"] else 1.0
            Bx = interp_matrix(w["n_sub"], cfg["diameter"], s, w["theta"][0] * L["altitude"],
                               L["n"], L["spacing"])
            By = interp_matrix(w["n_sub"], cfg["diameter"], s, w["theta"][1] * L["altitude"],
                               L["n"], L["spacing"])
            cols.append(np.kron(Bx, By))
        P = np.hstack(cols)
        At = G @ P @ W.T
        Cinv = block_matrix(sen["blocks"]) if not sen["phase"] else np.diag(sen["blocks"][:, 0])
        if precond_only:
            Nm = Cinv
            if not w["in_precond"]:
                continue
        elif w["remove_tt"]:
            T = tt_projector(sen["S"])
            Nm = T @ Cinv @ T
        else:
            Nm = Cinv
        parts.append((At, Nm))
        A += At.T @ Nm @ At
    A += cfg["alpha"] * np.diag(sysm.D)
    return A, parts, sysm
