"""Comparison helpers shared by the tests (no PCA arithmetic here)."""
from __future__ import annotations

import numpy as np


def angle(a, b) -> float:
    """Sign-aligned angle between two vectors, 2*asin(|a^ - s b^|/2) with
    s = sign(a^ . b^).  Resolves angles down to ~1e-16 (acos cannot)."""
    a = np.asarray(a, dtype=np.float64).ravel()
    b = np.asarray(b, dtype=np.float64).ravel()
    na, nb = np.linalg.norm(a), np.linalg.norm(b)
    if na == 0.0 or nb == 0.0:
        return 0.0 if na == nb else np.pi / 2
    a = a / na
    b = b / nb
    s = 1.0 if float(a @ b) >= 0.0 else -1.0
    d = np.linalg.norm(a - s * b)
    return float(2.0 * np.arcsin(min(1.0, d / 2.0)))


def col_angles(A, B) -> np.ndarray:
    A = np.asarray(A)
    B = np.asarray(B)
    return np.array([angle(A[:, i], B[:, i]) for i in range(A.shape[1])])


def orth_err(Q) -> float:
    """max |Q^T Q - I| in float64."""
    Q = np.asarray(Q, dtype=np.float64)
    return float(np.abs(Q.T @ Q - np.eye(Q.shape[1])).max())


def gapped(sig, rel=0.02) -> np.ndarray:
    """Mask of components whose relative gap to both neighbours is >= rel
    (1 - s_(k+1)/s_k >= rel and 1 - s_k/s_(k-1) >= rel)."""
    s = np.asarray(sig, dtype=np.float64)
    ok = np.ones(len(s), dtype=bool)
    for k in range(len(s)):
        if k > 0 and s[k] > (1 - rel) * s[k - 1]:
            ok[k] = False
        if k + 1 < len(s) and s[k + 1] > (1 - rel) * s[k]:
            ok[k] = False
    return ok
