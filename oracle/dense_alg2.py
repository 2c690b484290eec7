"""Literal dense transcription of the paper's tensorized environmental selection
(Alg. 2: OP1 offspring cooperation, OP2 update indexing with N x N index
matrices, OP3 elite selection over the columns). TEST INFRASTRUCTURE ONLY.

Memory is O(N^2): meant for tiny N only, as the brute-force definition against
which the C oracle's reverse-neighbour pull is pinned. Written in numpy from
the algorithm's steps, independently of the C code (own aggregation too).

Readings taken where the printed algorithm is ambiguous:
  R14  population 2's OP1 blend uses its own switch S2 (the print repeats S1).
  R15  H(.) of a boolean is its indicator.
  R17  OP3 draws candidates from the post-OP1 offspring (the ones OP2 judged).
  R18  OP3 returns the selected candidate row, not the parent array's row.
  R19  "argmin(CV)" keeps every index attaining the minimum CV.
  NaN  aggregation or CV values are read as +inf (they never win).
  Eq. (10)'s masked blend H(C) A + (1 - H(C)) B stands for a conditional
       branch, so it is applied as a select: a NaN in the operand that is not
       chosen does not leak through 0 * NaN.
"""
from __future__ import annotations

import numpy as np


def agg_rows(kind: int, theta: float, F: np.ndarray, W: np.ndarray, z: np.ndarray) -> np.ndarray:
    """Aggregation of rows F (n x m) at weights W (n x m): PBI of Eq. (7) with a
    unit direction (R13) for kind 0, Tchebycheff for kind 1."""
    F = np.atleast_2d(F)
    W = np.atleast_2d(W)
    if kind == 1:
        return np.max(W * np.abs(F - z), axis=1)
    wn = W / np.linalg.norm(W, axis=1, keepdims=True)
    diff = F - z
    d1 = np.abs(np.sum(diff * wn, axis=1))
    d2 = np.linalg.norm(diff - d1[:, None] * wn, axis=1)
    return d1 + theta * d2


def _inf(a):
    a = np.array(a, dtype=np.float64, copy=True)
    a[np.isnan(a)] = np.inf
    return a


def dense_select(F, CV, Fo, CVo, W, z, B, kind=0, theta=5.0):
    """Winners of Alg. 2 for both populations.

    F[p] (N x m), CV[p] (N): parents; Fo[p], CVo[p]: offspring of population p;
    W (N x m); z (m); B[p] (N x t_p). Returns (sw, win) with sw[p][i] = 1 when
    population p's new offspring i came from the other population, and
    win[p][j] = index i of the winning new offspring or -1 (parent kept)."""
    N = W.shape[0]
    I_sub = np.arange(N)

    # ---- OP1, vmapped over subproblems i (Eq. (11)) ----
    g1 = _inf(agg_rows(kind, theta, Fo[0], W, z))
    g2 = _inf(agg_rows(kind, theta, Fo[1], W, z))
    cv1 = _inf(CVo[0])
    cv2 = _inf(CVo[1])
    S1 = ((g1 > g2) & (cv1 == cv2)) | (cv2 < cv1)
    S2 = g2 > g1
    H1 = S1[:, None]
    H2 = S2[:, None]
    newF = [np.where(H1, Fo[1], Fo[0]), np.where(H2, Fo[0], Fo[1])]
    newCV = [np.where(S1, cv2, cv1), np.where(S2, cv1, cv2)]
    sw = [S1.astype(np.uint8), S2.astype(np.uint8)]

    # ---- OP2, vmapped over offspring i: rows of I_p (Eq. (12)) ----
    I = [np.empty((N, N), dtype=np.int64), np.empty((N, N), dtype=np.int64)]
    for i in range(N):
        for p in range(2):
            b = B[p][i]
            g_old = _inf(agg_rows(kind, theta, F[p][b], W[b], z))
            g_new = _inf(agg_rows(kind, theta, np.repeat(newF[p][i:i + 1], len(b), 0), W[b], z))
            if p == 0:
                cv_old = _inf(CV[0][b])
                cv_new = newCV[0][i]
                S = ((g_old > g_new) & (cv_old == cv_new)) | (cv_new < cv_old)
            else:
                S = g_old > g_new
            M = np.zeros(N)
            M[b] = S.astype(np.float64)
            I[p][i] = (M * (-1) + (1 - M) * I_sub).astype(np.int64)

    # ---- OP3, vmapped over parents j: columns of I_p (Eq. (13)) ----
    win = [np.full(N, -1, dtype=np.int32), np.full(N, -1, dtype=np.int32)]
    for p in range(2):
        for j in range(N):
            col = I[p][:, j]
            hit = col == -1
            Fc = np.where(hit[:, None], newF[p], F[p][j][None, :])
            gc = _inf(agg_rows(kind, theta, Fc, np.repeat(W[j:j + 1], N, 0), z))
            if p == 0:
                cvc = np.where(hit, newCV[0], _inf(CV[0][j]))
                cand = np.nonzero(cvc == cvc.min())[0]      # R19: the set of minimisers
                j1 = cand[int(np.argmin(gc[cand]))]         # first occurrence on ties
            else:
                j1 = int(np.argmin(gc))
            win[p][j] = int(j1) if hit[j1] else -1
    return np.stack(sw), np.stack(win)
