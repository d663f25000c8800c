"""Exact complex-rational linear algebra for brute-force pins on tiny systems.

Independent of numpy/LAPACK and of both solvers: Gauss-Jordan elimination over
Q(i) with Python Fractions, so the result of a tiny instance of Eq. 2 is exact.
"""
from __future__ import annotations

from fractions import Fraction


class QC:
    """Complex number with exact rational real and imaginary parts."""
    __slots__ = ("re", "im")

    def __init__(self, re=0, im=0):
        self.re = Fraction(re)
        self.im = Fraction(im)

    @staticmethod
    def from_complex(z: complex) -> "QC":
        return QC(Fraction(z.real), Fraction(z.imag))

    def __add__(self, o):
        return QC(self.re + o.re, self.im + o.im)

    def __sub__(self, o):
        return QC(self.re - o.re, self.im - o.im)

    def __mul__(self, o):
        return QC(self.re * o.re - self.im * o.im, self.re * o.im + self.im * o.re)

    def __neg__(self):
        return QC(-self.re, -self.im)

    def conj(self):
        return QC(self.re, -self.im)

    def inv(self):
        d = self.re * self.re + self.im * self.im
        if d == 0:
            raise ZeroDivisionError("singular")
        return QC(self.re / d, -self.im / d)

    def is_zero(self):
        return self.re == 0 and self.im == 0

    def __complex__(self):
        return complex(float(self.re), float(self.im))


def qmat(M):
    return [[QC.from_complex(complex(v)) for v in row] for row in M]


def qinv(M):
    """Exact inverse by Gauss-Jordan with a nonzero pivot search."""
    n = len(M)
    A = [row[:] + [QC(1 if i == j else 0) for j in range(n)] for i, row in enumerate(M)]
    for k in range(n):
        p = next((r for r in range(k, n) if not A[r][k].is_zero()), None)
        if p is None:
            raise ZeroDivisionError("singular matrix")
        A[k], A[p] = A[p], A[k]
        d = A[k][k].inv()
        A[k] = [v * d for v in A[k]]
        for r in range(n):
            if r != k and not A[r][k].is_zero():
                f = A[r][k]
                A[r] = [a - f * c for a, c in zip(A[r], A[k])]
    return [row[n:] for row in A]


def qmul(A, B):
    n, m, k = len(A), len(B[0]), len(B)
    return [[sum((A[i][t] * B[t][j] for t in range(k)), QC()) for j in range(m)] for i in range(n)]


def qH(A):
    return [[A[j][i].conj() for j in range(len(A))] for i in range(len(A[0]))]


def to_complex(A):
    import numpy as np
    return np.array([[complex(v) for v in row] for row in A], dtype=np.complex128)
