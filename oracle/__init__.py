"""FP64 CPU oracle for SFFT image subtraction -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the benchmark's CPU-baseline
leg may import this package. The GPU library never links, loads or calls it,
and the two share no code.

``sfft_oracle.c`` holds the plain FP64 reference (pixel-space lag sums, App. B
assembly, Jacobi-scaled Cholesky, direct circular convolve-and-subtract);
``brute`` holds an explicit basis-matrix least-squares solver for tiny
images. Every function here is pinned by tests against the paper's
definitions, closed forms and library routines (see ``tests/test_oracle*``).
No function of the oracle is "parity unpinned".
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "sfft_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lock = threading.Lock()
_lib = None

OK, EINVAL, ENOMEM, ENOTSPD = 0, -1, -2, -3


def build(force: bool = False) -> str:
    """Compile the C oracle (gcc, FP64, OpenMP) into ``liboracle.so``."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + f".tmp{os.getpid()}"
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c99",
                               "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def lib():
    global _lib
    with _lock:
        if _lib is None:
            L = ctypes.CDLL(build())
            dp = ctypes.POINTER(ctypes.c_double)
            lp = ctypes.POINTER(ctypes.c_long)
            i = ctypes.c_int
            L.orc_num_unknowns.restype = ctypes.c_long
            L.orc_num_unknowns.argtypes = [i, i, i, i, i]
            L.orc_coord.restype = ctypes.c_double
            L.orc_coord.argtypes = [ctypes.c_long, ctypes.c_long]
            L.orc_omega.argtypes = [dp, i, i, i, i, i, dp]
            L.orc_theta.argtypes = [dp, dp, i, i, i, i, i, dp]
            L.orc_lambda.argtypes = [dp, i, i, i, i, i, i, dp]
            L.orc_background_blocks.argtypes = [dp, i, i, i, dp, dp]
            L.orc_assemble.argtypes = [dp, dp, dp, dp, dp, i, i, i, i, i, dp, dp]
            L.orc_build.argtypes = [dp, dp, i, i, i, i, i, i, i, dp, dp]
            L.orc_g_entry.restype = ctypes.c_double
            L.orc_g_entry.argtypes = [dp, i, i, i, i, i, i, i, ctypes.c_long, ctypes.c_long]
            L.orc_phi_dot.restype = ctypes.c_double
            L.orc_phi_dot.argtypes = [dp, dp, i, i, i, i, i, i, i, ctypes.c_long]
            L.orc_solve.argtypes = [dp, dp, ctypes.c_long, dp]
            L.orc_stamps.argtypes = [dp, i, i, i, i, dp]
            L.orc_subtract.argtypes = [dp, dp, i, i, i, i, i, i, i, dp, dp]
            L.orc_subtract_pixels.argtypes = [dp, dp, i, i, i, i, i, i, i, dp, lp, ctypes.c_long, dp]
            L.orc_kernel_sum_field.argtypes = [dp, i, i, i, i, i, i, dp]
            L.orc_num_threads.restype = i
            _lib = L
    return _lib


def _d(a):
    a = np.ascontiguousarray(a, dtype=np.float64)
    return a, a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def nterms(deg: int) -> int:
    return (deg + 1) * (deg + 2) // 2 if deg >= 0 else 0


def terms(deg: int):
    """Monomial exponents (i, j), i ascending then j ascending, i + j <= deg."""
    return [(i, j) for i in range(deg + 1) for j in range(deg + 1 - i)]


def num_unknowns(w0, w1, dk, db, const_phot=0) -> int:
    return int(lib().orc_num_unknowns(w0, w1, dk, db, const_phot))


def kernel_unknowns(w0, w1, dk, const_phot=0):
    """List of (k, a, b) for the kernel unknowns in solver order."""
    out = []
    for k in range(nterms(dk)):
        for a in range(-w0, w0 + 1):
            for b in range(-w1, w1 + 1):
                if const_phot and k > 0 and a == 0 and b == 0:
                    continue
                out.append((k, a, b))
    return out


def coords(n0, n1):
    c0 = np.array([lib().orc_coord(x, n0) for x in range(n0)])
    c1 = np.array([lib().orc_coord(x, n1) for x in range(n1)])
    return c0, c1


def omega(r, dk, w0, w1):
    r, rp = _d(r)
    P = nterms(dk)
    out = np.zeros((P * (P + 1) // 2, 4 * w0 + 1, 4 * w1 + 1))
    _, op = _d(out)
    rc = lib().orc_omega(rp, r.shape[0], r.shape[1], dk, w0, w1, op)
    assert rc == OK
    return out


def theta(r, s, dk, w0, w1):
    r, rp = _d(r)
    s, sp = _d(s)
    out = np.zeros((nterms(dk), 2 * w0 + 1, 2 * w1 + 1))
    _, op = _d(out)
    assert lib().orc_theta(rp, sp, r.shape[0], r.shape[1], dk, w0, w1, op) == OK
    return out


def lam(r, dk, db, w0, w1):
    r, rp = _d(r)
    out = np.zeros((nterms(dk), nterms(db), 2 * w0 + 1, 2 * w1 + 1))
    _, op = _d(out)
    assert lib().orc_lambda(rp, r.shape[0], r.shape[1], dk, db, w0, w1, op) == OK
    return out


def background_blocks(s, db):
    s, sp = _d(s)
    Q = nterms(db)
    cm = np.zeros((Q, Q))
    ev = np.zeros(Q)
    _, cp_ = _d(cm)
    _, ep = _d(ev)
    assert lib().orc_background_blocks(sp, s.shape[0], s.shape[1], db, cp_, ep) == OK
    return cm, ev


def assemble(om, th, la, cm, ev, w0, w1, dk, db, const_phot=0):
    n = num_unknowns(w0, w1, dk, db, const_phot)
    G = np.zeros((n, n))
    h = np.zeros(n)
    args = [_d(x)[1] for x in (om, th, la, cm, ev)]
    # keep contiguous copies alive
    keep = [_d(x)[0] for x in (om, th, la, cm, ev)]
    args = [k.ctypes.data_as(ctypes.POINTER(ctypes.c_double)) for k in keep]
    _, gp = _d(G)
    _, hp = _d(h)
    assert lib().orc_assemble(*args, w0, w1, dk, db, const_phot, gp, hp) == OK
    return G, h


def build_system(r, s, w0, w1, dk, db, const_phot=0):
    """Normal matrix G and right-hand side h (pixel units) of the fit pair."""
    r, rp = _d(r)
    s, sp = _d(s)
    n = num_unknowns(w0, w1, dk, db, const_phot)
    G = np.zeros((n, n))
    h = np.zeros(n)
    _, gp = _d(G)
    _, hp = _d(h)
    rc = lib().orc_build(rp, sp, r.shape[0], r.shape[1], w0, w1, dk, db, const_phot, gp, hp)
    if rc != OK:
        raise ValueError(f"oracle build failed: {rc}")
    return G, h


def g_entry(r, w0, w1, dk, db, const_phot, u, v):
    r, rp = _d(r)
    return float(lib().orc_g_entry(rp, r.shape[0], r.shape[1], w0, w1, dk, db, const_phot, u, v))


def phi_dot(r, img, w0, w1, dk, db, const_phot, u):
    """Component u of Phi^T img (h_u for img = S; the gradient for img = D)."""
    r, rp = _d(r)
    img, ip = _d(img)
    return float(lib().orc_phi_dot(rp, ip, r.shape[0], r.shape[1], w0, w1, dk, db, const_phot, u))


def solve(G, h):
    """Jacobi-scaled FP64 Cholesky solve. Raises ``np.linalg.LinAlgError``
    when G is not positive definite."""
    G, gp = _d(G)
    h, hp = _d(h)
    c = np.zeros(h.shape[0])
    _, cp_ = _d(c)
    rc = lib().orc_solve(gp, hp, h.shape[0], cp_)
    if rc == ENOTSPD:
        raise np.linalg.LinAlgError("normal matrix is not positive definite")
    assert rc == OK
    return c


def stamps(coef, w0, w1, dk, const_phot=0):
    coef, cp_ = _d(coef)
    out = np.zeros((nterms(dk), 2 * w0 + 1, 2 * w1 + 1))
    _, op = _d(out)
    lib().orc_stamps(cp_, w0, w1, dk, const_phot, op)
    return out


def subtract(r, s, coef, w0, w1, dk, db, const_phot=0):
    r, rp = _d(r)
    s, sp = _d(s)
    coef, cp_ = _d(coef)
    d = np.zeros(r.shape)
    _, dp = _d(d)
    lib().orc_subtract(rp, sp, r.shape[0], r.shape[1], w0, w1, dk, db, const_phot, cp_, dp)
    return d


def subtract_pixels(r, s, coef, w0, w1, dk, db, const_phot, pixels):
    r, rp = _d(r)
    s, sp = _d(s)
    coef, cp_ = _d(coef)
    pix = np.ascontiguousarray(np.asarray(pixels, dtype=np.int64).reshape(-1, 2))
    out = np.zeros(pix.shape[0])
    _, op = _d(out)
    lib().orc_subtract_pixels(rp, sp, r.shape[0], r.shape[1], w0, w1, dk, db, const_phot, cp_,
                              pix.ctypes.data_as(ctypes.POINTER(ctypes.c_long)), pix.shape[0], op)
    return out


def kernel_sum_field(coef, n0, n1, w0, w1, dk, const_phot=0):
    coef, cp_ = _d(coef)
    out = np.zeros((n0, n1))
    _, op = _d(out)
    lib().orc_kernel_sum_field(cp_, n0, n1, w0, w1, dk, const_phot, op)
    return out


def fit(r_fit, s_fit, w0, w1, dk, db, const_phot=0):
    """Least-squares coefficients of the fit pair (build + solve)."""
    G, h = build_system(r_fit, s_fit, w0, w1, dk, db, const_phot)
    return solve(G, h)


def num_threads() -> int:
    return int(lib().orc_num_threads())
