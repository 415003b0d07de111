"""Explicit basis-matrix least squares for tiny images -- TEST INFRASTRUCTURE.

Builds the design matrix Phi column by column straight from the model of
Eq. 12 (delta basis of Eq. 3-4 shifted circularly with ``numpy.roll``,
polynomial weights of Eq. 6 at the source pixel, polynomial background of
Eq. 2), then forms Phi^T Phi and Phi^T S and solves with ``numpy.linalg``.
It shares nothing with the C oracle beyond the written conventions:
x = axis 0, centred coordinates c = (2x - (N-1)) / (N-1), offsets inclusive
[-w, w], unknown order k (i then j), a, b, then background (p then q).
"""
from __future__ import annotations

import numpy as np


def _coords(n):
    return (2.0 * np.arange(n) - (n - 1)) / (n - 1)


def _terms(deg):
    return [(i, j) for i in range(deg + 1) for j in range(deg + 1 - i)]


def design_matrix(r, w0, w1, dk, db, const_phot=0):
    r = np.asarray(r, dtype=np.float64)
    n0, n1 = r.shape
    c0 = _coords(n0)[:, None]
    c1 = _coords(n1)[None, :]
    cols = []
    for k, (i, j) in enumerate(_terms(dk)):
        rk = c0 ** i * c1 ** j * r
        for a in range(-w0, w0 + 1):
            for b in range(-w1, w1 + 1):
                if const_phot and k > 0 and a == 0 and b == 0:
                    continue
                col = np.roll(rk, (a, b), axis=(0, 1))   # out[x] = rk[x - (a, b)]
                if a or b:
                    col = col - rk
                cols.append(col.ravel())
    for p, q in _terms(db):
        cols.append((c0 ** p * c1 ** q * np.ones_like(r)).ravel())
    return np.stack(cols, axis=1)


def normal_equations(r, s, w0, w1, dk, db, const_phot=0):
    phi = design_matrix(r, w0, w1, dk, db, const_phot)
    return phi.T @ phi, phi.T @ np.asarray(s, dtype=np.float64).ravel()


def lstsq(r, s, w0, w1, dk, db, const_phot=0):
    phi = design_matrix(r, w0, w1, dk, db, const_phot)
    coef, *_ = np.linalg.lstsq(phi, np.asarray(s, dtype=np.float64).ravel(), rcond=None)
    return coef


def difference(r, s, coef, w0, w1, dk, db, const_phot=0):
    phi = design_matrix(r, w0, w1, dk, db, const_phot)
    return np.asarray(s, dtype=np.float64) - (phi @ coef).reshape(np.shape(s))
