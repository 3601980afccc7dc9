"""Subspace angles for the GPU tests (test helper, numpy only).

sin of the largest principal angle between span(X) and span(Y) for
matrices with orthonormal rows (sketches, k x m) or columns (row bases):
    sin theta = || (I - P_Y) X^T ||_2,   P_Y the orthogonal projector on span(Y).
"""
import numpy as np


def sin_angle_rows(X, Y):
    """Largest principal angle (sine) between the row spaces of X and Y
    (rows orthonormal, or nearly so: X is orthonormalised first)."""
    X = np.asarray(X, np.float64)
    Y = np.asarray(Y, np.float64)
    qx, _ = np.linalg.qr(X.T)
    qy, _ = np.linalg.qr(Y.T)
    return float(np.linalg.norm(qx - qy @ (qy.T @ qx), 2))


def resolvable(lam, rel_gap=1e-3):
    """Leading-block sizes j whose spectral gap (lambda_j - lambda_{j+1}) is at
    least rel_gap * lambda_1: the top-j invariant subspace is then stable
    under a perturbation of G far below that gap (Davis-Kahan)."""
    lam = np.asarray(lam, np.float64)
    gaps = (lam[:-1] - lam[1:]) / lam[0]
    return [j + 1 for j in range(len(gaps)) if gaps[j] >= rel_gap]


def sketch_angles(S_gpu, S_orc, lam, rel_gap=1e-3):
    """(angle of all k rows, {j: angle of the leading j rows} for the
    resolvable j)."""
    k = S_orc.shape[0]
    out = {j: sin_angle_rows(S_gpu[:j], S_orc[:j]) for j in resolvable(lam[:k + 1], rel_gap) if j <= k}
    return sin_angle_rows(S_gpu, S_orc), out


def row_basis_angle(R_gpu, V_orc):
    """sin of the largest angle of span(R_gpu) (n x r) against span(V_orc)
    (n x k, orthonormal columns): how far the GPU's row factor leaves the
    oracle's row space of S A."""
    q, _ = np.linalg.qr(np.asarray(R_gpu, np.float64))
    return float(np.linalg.norm(q - V_orc @ (V_orc.T @ q), 2))
