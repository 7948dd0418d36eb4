"""A small lazy algebra of linear operators for the oracle.

Magnus exponents (Section 2) are linear combinations of A(t) = -i H(t) at
quadrature nodes, plus (for M4 and M6) commutators of such combinations.  This
module keeps them as expression trees so that the same exponent can be
evaluated as a dense matrix (for eigendecomposition) or applied to a vector
without ever forming products of sparse matrices (for Taylor series at large
dimension).  Nothing here reorders or fuses the arithmetic beyond what the
definitions state: a commutator [X, Y] v is X(Y v) - Y(X v).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp


class Op:
    def matvec(self, v):
        raise NotImplementedError

    def dense(self) -> np.ndarray:
        raise NotImplementedError

    def norm_bound(self) -> float:
        """An upper bound on the spectral norm."""
        raise NotImplementedError

    # algebra
    def __add__(self, other):
        return Lin([(1.0, self), (1.0, other)])

    def __sub__(self, other):
        return Lin([(1.0, self), (-1.0, other)])

    def __rmul__(self, c):
        return Lin([(c, self)])

    def __neg__(self):
        return Lin([(-1.0, self)])


class Mat(Op):
    """A stored matrix (numpy array or scipy sparse)."""

    def __init__(self, M):
        self.M = M
        self._nb = None

    def matvec(self, v):
        return self.M @ v

    def dense(self):
        return self.M.toarray() if sp.issparse(self.M) else np.asarray(self.M)

    def norm_bound(self):
        # ||M||_2 <= sqrt(||M||_1 ||M||_inf)
        if self._nb is None:
            A = abs(self.M)
            if sp.issparse(A):
                r = float(np.max(np.asarray(A.sum(axis=1)))) if A.shape[0] else 0.0
                c = float(np.max(np.asarray(A.sum(axis=0)))) if A.shape[0] else 0.0
            else:
                r = float(np.max(A.sum(axis=1))) if A.size else 0.0
                c = float(np.max(A.sum(axis=0))) if A.size else 0.0
            self._nb = float(np.sqrt(r * c))
        return self._nb


class Lin(Op):
    """sum_k c_k X_k with scalar (complex) coefficients."""

    def __init__(self, terms):
        flat = []
        for c, X in terms:
            if isinstance(X, Lin):
                flat.extend((c * c2, X2) for c2, X2 in X.terms)
            else:
                flat.append((c, X))
        # merge coefficients of the same stored object
        merged: dict[int, list] = {}
        order = []
        for c, X in flat:
            k = id(X)
            if k in merged:
                merged[k][0] += c
            else:
                merged[k] = [c, X]
                order.append(k)
        self.terms = [(merged[k][0], merged[k][1]) for k in order]

    def matvec(self, v):
        out = np.zeros_like(v, dtype=np.complex128)
        for c, X in self.terms:
            if c != 0:
                out += c * X.matvec(v)
        return out

    def dense(self):
        out = None
        for c, X in self.terms:
            D = c * X.dense()
            out = D if out is None else out + D
        return out

    def norm_bound(self):
        return float(sum(abs(c) * X.norm_bound() for c, X in self.terms))


class Comm(Op):
    """[X, Y] = X Y - Y X."""

    def __init__(self, X: Op, Y: Op):
        self.X, self.Y = X, Y

    def matvec(self, v):
        return self.X.matvec(self.Y.matvec(v)) - self.Y.matvec(self.X.matvec(v))

    def dense(self):
        X, Y = self.X.dense(), self.Y.dense()
        return X @ Y - Y @ X

    def norm_bound(self):
        return 2.0 * self.X.norm_bound() * self.Y.norm_bound()
