"""CPU oracle for the stabilized DQMC Green's functions (test infrastructure).

Only the tests, the smoke check and the benchmark's CPU-baseline leg may use
this package.  It wraps the plain C oracle in sdq_oracle.c (built into
liboracle_sdq.so by `build()`), which shares no code with the GPU library.
All arrays are numpy float64, row-major.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liboracle_sdq.so")

SCHEME_LOH = 0
SCHEME_PLAIN = 1


def build() -> str:
    """Compile the oracle with gcc (plain -O2, OpenMP-free, no BLAS)."""
    src = os.path.join(HERE, "sdq_oracle.c")
    tmp = LIB_PATH + ".tmp"
    subprocess.check_call(["gcc", "-O2", "-std=c99", "-fPIC", "-shared", "-Wall",
                           "-o", tmp, src, "-lm"])
    os.replace(tmp, LIB_PATH)
    return LIB_PATH


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            build()
        L = ctypes.CDLL(LIB_PATH)
        d = ctypes.POINTER(ctypes.c_double)
        i = ctypes.POINTER(ctypes.c_int)
        c_int, c_double = ctypes.c_int, ctypes.c_double
        L.or_greens.argtypes = [c_int, c_int, c_int, d, d, c_double, c_int, d, d, d]
        L.or_greens_tdisp.argtypes = [c_int, c_int, c_int, d, d, d, c_double, c_int, c_int, d]
        L.or_greens_slice.argtypes = [c_int, c_int, c_int, d, d, c_double, c_int, d, d, d]
        L.or_logdet_grad.argtypes = [c_int, c_int, c_int, d, d, c_double, i, c_int, d]
        L.or_greens_naive.argtypes = [c_int, c_int, c_int, d, d, c_double, d]
        L.or_chain.argtypes = [c_int, c_int, c_int, d, d, d, c_double, c_int, c_int, c_int, d, d, d]
        L.or_greens_sym.argtypes = [c_int, c_int, c_int, d, d, c_double, d, d, d]
        L.or_greens_tdisp_sym.argtypes = [c_int, c_int, c_int, d, d, d, c_double, c_int, d]
        L.or_greens_stab.argtypes = [c_int, c_int, c_int, d, d, c_double, c_int, c_int, d, d, d]
        L.or_greens_tdisp_stab.argtypes = [c_int, c_int, c_int, d, d, d, c_double, c_int, c_int, c_int, d]
        L.or_svd.argtypes = [c_int, d, d, d, d]
        L.or_greens_dense.argtypes = [c_int, c_int, c_int, d, d, d, d]
        L.or_greens_tdisp_dense.argtypes = [c_int, c_int, c_int, d, c_int, d]
        L.or_cpqr.argtypes = [c_int, d, d, i]
        L.or_udt.argtypes = [c_int, d, d, d, d]
        L.or_udt_complex.argtypes = [c_int, d, d, d, d]
        L.or_greens_complex.argtypes = [c_int, c_int, c_int, d, d, d, d]
        L.or_expk_planewave.argtypes = [c_int, c_double, c_double, c_double, d]
        _lib = L
    return _lib


def _p(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _pi(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int))


def _c(a):
    return np.ascontiguousarray(a, dtype=np.float64)


class OracleError(RuntimeError):
    pass


def _chk(st):
    if st != 0:
        raise OracleError(f"oracle status {st}")


def greens(expk, field, alpha, k, scheme=SCHEME_LOH):
    """Equal-time G = (1 + B_M..B_1)^{-1}, log|det(1 + B_M..B_1)| and its sign."""
    expk, field = _c(expk), _c(field)
    m, n = field.shape
    G = np.zeros((n, n))
    ld, sg = np.zeros(1), np.zeros(1)
    _chk(lib().or_greens(n, m, k, _p(expk), _p(field), float(alpha), scheme, _p(G), _p(ld), _p(sg)))
    return G, float(ld[0]), float(sg[0])


def greens_tdisp(expk, expk_inv, field, alpha, k, l, scheme=SCHEME_LOH):
    """G(tau_l, 0) = B_l..B_1 G, 0 <= l <= M."""
    expk, expk_inv, field = _c(expk), _c(expk_inv), _c(field)
    m, n = field.shape
    G = np.zeros((n, n))
    _chk(lib().or_greens_tdisp(n, m, k, _p(expk), _p(expk_inv), _p(field), float(alpha),
                               int(l), scheme, _p(G)))
    return G


def greens_sym(expk_half, field, alpha, k):
    """G, log|det(1+B_M..B_1)| and sign for the symmetric Trotter slices
    B_l = H diag(exp(alpha f_l)) H with H = expk_half = exp(-dtau K / 2)."""
    expk_half, field = _c(expk_half), _c(field)
    m, n = field.shape
    G = np.zeros((n, n))
    ld, sg = np.zeros(1), np.zeros(1)
    _chk(lib().or_greens_sym(n, m, k, _p(expk_half), _p(field), float(alpha), _p(G), _p(ld), _p(sg)))
    return G, float(ld[0]), float(sg[0])


def greens_tdisp_sym(expk_half, expk_half_inv, field, alpha, k, l):
    """G(tau_l, 0) = B_l..B_1 G for the symmetric Trotter slices."""
    expk_half, expk_half_inv, field = _c(expk_half), _c(expk_half_inv), _c(field)
    m, n = field.shape
    G = np.zeros((n, n))
    _chk(lib().or_greens_tdisp_sym(n, m, k, _p(expk_half), _p(expk_half_inv), _p(field),
                                   float(alpha), int(l), _p(G)))
    return G


def greens_slice(expk, field, alpha, k, l):
    """G_l = (1 + B_{l-1}..B_1 B_M..B_l)^{-1}, 1 <= l <= M, plus logdet/sign."""
    expk, field = _c(expk), _c(field)
    m, n = field.shape
    G = np.zeros((n, n))
    ld, sg = np.zeros(1), np.zeros(1)
    _chk(lib().or_greens_slice(n, m, k, _p(expk), _p(field), float(alpha), int(l),
                               _p(G), _p(ld), _p(sg)))
    return G, float(ld[0]), float(sg[0])


def logdet_grad(expk, field, alpha, k, l_list):
    """Rows of d log|det(1+B_M..B_1)| / d f_{l,i} for l in l_list (1-based)."""
    expk, field = _c(expk), _c(field)
    m, n = field.shape
    ls = np.ascontiguousarray(l_list, dtype=np.int32)
    out = np.zeros((len(ls), n))
    _chk(lib().or_logdet_grad(n, m, k, _p(expk), _p(field), float(alpha), _pi(ls), len(ls), _p(out)))
    return out


def greens_naive(expk, field, alpha):
    expk, field = _c(expk), _c(field)
    m, n = field.shape
    G = np.zeros((n, n))
    _chk(lib().or_greens_naive(n, m, 1, _p(expk), _p(field), float(alpha), _p(G)))
    return G


def chain(expk, expk_inv, field, alpha, k, kind, a, b):
    """UDT of B_b..B_a (kind 0), B_a^{-1}..B_b^{-1} (1) or B_a^T..B_b^T (2)."""
    expk, field = _c(expk), _c(field)
    expk_inv = _c(expk_inv) if expk_inv is not None else np.eye(expk.shape[0])
    m, n = field.shape
    U, T, D = np.zeros((n, n)), np.zeros((n, n)), np.zeros(n)
    _chk(lib().or_chain(n, m, k, _p(expk), _p(expk_inv), _p(field), float(alpha), kind, a, b,
                        _p(U), _p(D), _p(T)))
    return U, D, T


STAB_QR, STAB_SVD = 0, 1


def greens_stab(expk, field, alpha, k, stab, scheme=SCHEME_LOH):
    """greens() with the stabilizer chosen: STAB_QR or STAB_SVD (Jacobi)."""
    expk, field = _c(expk), _c(field)
    m, n = field.shape
    G = np.zeros((n, n))
    ld, sg = np.zeros(1), np.zeros(1)
    _chk(lib().or_greens_stab(n, m, k, _p(expk), _p(field), float(alpha), scheme, stab, _p(G), _p(ld),
                              _p(sg)))
    return G, float(ld[0]), float(sg[0])


def greens_tdisp_stab(expk, expk_inv, field, alpha, k, l, stab, scheme=SCHEME_LOH):
    """greens_tdisp() with the stabilizer chosen."""
    expk, expk_inv, field = _c(expk), _c(expk_inv), _c(field)
    m, n = field.shape
    G = np.zeros((n, n))
    _chk(lib().or_greens_tdisp_stab(n, m, k, _p(expk), _p(expk_inv), _p(field), float(alpha),
                                    int(l), scheme, stab, _p(G)))
    return G


def greens_dense(slices, k):
    """Equal-time G, log|det| and sign for dense slices [m][n][n] (B_l = slices[l-1])."""
    sl = _c(slices)
    m, n = sl.shape[0], sl.shape[1]
    G = np.zeros((n, n))
    ld, sg = np.zeros(1), np.zeros(1)
    _chk(lib().or_greens_dense(n, m, k, _p(sl), _p(G), _p(ld), _p(sg)))
    return G, float(ld[0]), float(sg[0])


def greens_tdisp_dense(slices, k, l):
    """G(tau_l, 0) for dense slices [m][n][n]."""
    sl = _c(slices)
    m, n = sl.shape[0], sl.shape[1]
    G = np.zeros((n, n))
    _chk(lib().or_greens_tdisp_dense(n, m, k, _p(sl), int(l), _p(G)))
    return G


def svd(W):
    """One-sided Jacobi SVD: W = U diag(s) V^T (s descending); returns U, s, V, sweeps."""
    W = _c(W)
    n = W.shape[0]
    U, V, sv = np.zeros((n, n)), np.zeros((n, n)), np.zeros(n)
    sweeps = lib().or_svd(n, _p(W), _p(U), _p(sv), _p(V))
    return U, sv, V, sweeps


def cpqr(A):
    """Pivoted QR: returns Q, R, jpvt with A[:, jpvt] = Q @ R."""
    R = _c(A).copy()
    n = R.shape[0]
    Q = np.zeros((n, n))
    jp = np.zeros(n, dtype=np.int32)
    _chk(lib().or_cpqr(n, _p(R), _p(Q), _pi(jp)))
    return Q, R, jp


def udt(W):
    W = _c(W)
    n = W.shape[0]
    U, T, D = np.zeros((n, n)), np.zeros((n, n)), np.zeros(n)
    _chk(lib().or_udt(n, _p(W), _p(U), _p(D), _p(T)))
    return U, D, T


def udt_complex(W):
    """Complex UDT W P = Q R: U = Q, D = |diag R|, T = D^-1 R P^T (complex128)."""
    W = np.ascontiguousarray(W, dtype=np.complex128)
    n = W.shape[0]
    U, T, D = np.zeros((n, n), np.complex128), np.zeros((n, n), np.complex128), np.zeros(n)
    _chk(lib().or_udt_complex(n, _p(W.view(np.float64)), _p(U.view(np.float64)), _p(D),
                              _p(T.view(np.float64))))
    return U, D, T


def greens_complex(slices, k):
    """Complex dense slices [m, n, n] (complex128): G (complex), log|det(1+B)|
    and the phase det(1+B)/|det(1+B)| (complex)."""
    sl = np.ascontiguousarray(slices, dtype=np.complex128)
    m, n, _ = sl.shape
    G = np.zeros((n, n), np.complex128)
    ld, ph = np.zeros(1), np.zeros(2)
    _chk(lib().or_greens_complex(n, m, int(k), _p(sl.view(np.float64)), _p(G.view(np.float64)),
                                 _p(ld), _p(ph)))
    return G, float(ld[0]), complex(ph[0], ph[1])


def expk_planewave(L, t, dtau, s=1.0):
    """exp(-s dtau K) of the periodic square lattice from plane waves."""
    out = np.zeros((L * L, L * L))
    _chk(lib().or_expk_planewave(L, float(t), float(dtau), float(s), _p(out)))
    return out
