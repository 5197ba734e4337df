"""Arbitrary-precision brute force for tiny lattices (test pin for the oracle).

The paper benchmarks every stabilization scheme against an arbitrary-precision
computation of the plain definitions (Sec. 4.1, Sec. 5.2, Sec. 6.2).  This
module does the same with mpmath: it multiplies the slice matrices with no
stabilization at all, at `dps` decimal digits, and then applies the plain
definitions
    G         = (1 + B_M ... B_1)^{-1}
    G(tau_l,0) = B_l ... B_1 G
    G_l       = (1 + B_{l-1} ... B_1 B_M ... B_l)^{-1}
    logdet    = log|det(1 + B_M ... B_1)|.
The float64 inputs (expk, field) are taken as exact.  It shares no code with
the oracle or with the GPU library.
"""
from __future__ import annotations

import mpmath
import numpy as np


class Brute:
    def __init__(self, expk, field, alpha, dps=320, perturb=None):
        """perturb = (l, i, h): field[l-1][i] += h, with h taken exactly at
        `dps` digits (used for finite differences well below float64 eps)."""
        self.ctx = mpmath.MPContext()
        self.ctx.dps = dps
        mp = self.ctx
        self.n = expk.shape[0]
        self.m = field.shape[0]
        self.E = [[mp.mpf(float(x)) for x in row] for row in expk]
        al = mp.mpf(float(alpha))
        f = [[mp.mpf(float(x)) for x in row] for row in field]
        if perturb is not None:
            l, i, h = perturb
            f[l - 1][i] += mp.mpf(h)
        self.v = [[mp.exp(al * x) for x in row] for row in f]
        self._prefix = None

    def slice_apply(self, q, W):
        """B_q W with B_q = E diag(v_q), q 1-based."""
        n, E, v = self.n, self.E, self.v[q - 1]
        S = [[v[i] * W[i][j] for j in range(n)] for i in range(n)]
        out = []
        for i in range(n):
            Ei = E[i]
            row = []
            for j in range(n):
                acc = self.ctx.mpf(0)
                for p in range(n):
                    acc += Ei[p] * S[p][j]
                row.append(acc)
            out.append(row)
        return out

    def eye(self):
        mp = self.ctx
        return [[mp.mpf(1) if i == j else mp.mpf(0) for j in range(self.n)] for i in range(self.n)]

    def prefixes(self):
        """[B_0..B_1 = I, B_1, B_2 B_1, ..., B_M..B_1]"""
        if self._prefix is None:
            P = [self.eye()]
            W = P[0]
            for q in range(1, self.m + 1):
                W = self.slice_apply(q, W)
                P.append(W)
            self._prefix = P
        return self._prefix

    def _mat(self, A):
        return self.ctx.matrix(A)

    def greens(self):
        mp = self.ctx
        B = self._mat(self.prefixes()[self.m])
        A = B + mp.eye(self.n)
        G = mp.inverse(A)
        d = mp.det(A)
        return G, mp.log(abs(d)), (1 if d > 0 else -1)

    def tdisp(self, l, G=None):
        if G is None:
            G = self.greens()[0]
        return self._mat(self.prefixes()[l]) * G

    def greens_slice(self, l):
        """G_l = (1 + X Y)^{-1}, X = B_{l-1}..B_1, Y = B_M..B_l."""
        mp = self.ctx
        X = self._mat(self.prefixes()[l - 1])
        Y = self.eye()
        for q in range(l, self.m + 1):
            Y = self.slice_apply(q, Y)
        return mp.inverse(mp.eye(self.n) + X * self._mat(Y))

    def logdet(self):
        return self.greens()[1]

    @staticmethod
    def to_np(A):
        return np.array([[float(A[i, j]) for j in range(A.cols)] for i in range(A.rows)])


class BruteDense:
    """The plain definitions for dense slices (real or complex), multiplied
    out at `dps` digits with no stabilization: G = (1 + B_M ... B_1)^{-1},
    log|det(1 + B_M ... B_1)| and det / |det| (a complex phase)."""

    def __init__(self, slices, dps=200):
        self.ctx = mpmath.MPContext()
        self.ctx.dps = dps
        mp = self.ctx
        sl = np.asarray(slices)
        self.m, self.n, _ = sl.shape
        self.B = [mp.matrix([[mp.mpc(complex(x)) for x in row] for row in s]) for s in sl]

    def greens(self):
        mp = self.ctx
        P = mp.eye(self.n)
        for q in range(self.m):
            P = self.B[q] * P
        A = P + mp.eye(self.n)
        d = mp.det(A)
        G = mp.inverse(A)
        return G, mp.log(abs(d)), complex(d / abs(d))

    @staticmethod
    def to_np(A):
        return np.array([[complex(A[i, j]) for j in range(A.cols)] for i in range(A.rows)])
