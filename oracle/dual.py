"""Forward-mode dual numbers over NumPy arrays (test infrastructure).

A ``Dual`` carries a value array ``v`` of shape S and a tangent array ``d`` of
shape (n, *S): one directional derivative per tangent slot.  The oracle's
per-pair code is written once against the small function set in ``ops`` and
runs either on plain floats/arrays (value) or on Duals (value + exact
derivative of the piecewise-smooth cost, with discrete decisions -- floor
cells, hit tests, folds -- taken on the value and treated as constant).
"""
from __future__ import annotations

import numpy as np


class Dual:
    __slots__ = ("v", "d")
    __array_ufunc__ = None  # numpy operands defer to Dual's reflected operators

    def __init__(self, v, d):
        self.v = np.asarray(v, dtype=np.float64)
        self.d = np.asarray(d, dtype=np.float64)

    @property
    def n(self) -> int:
        return self.d.shape[0]

    @staticmethod
    def variable(value: float, slot: int, n: int) -> "Dual":
        d = np.zeros((n,))
        d[slot] = 1.0
        return Dual(np.float64(value), d)

    # --- helpers -----------------------------------------------------------
    def _lift(self, other):
        if isinstance(other, Dual):
            return other
        o = np.asarray(other, dtype=np.float64)
        return Dual(o, np.zeros((self.n,) + o.shape))

    @staticmethod
    def _bd(d, v_shape):
        # broadcast a tangent (n, *S) against a value shape
        return d.reshape(d.shape[:1] + (1,) * (len(v_shape) - (d.ndim - 1)) + d.shape[1:])

    def _pair(self, other):
        o = self._lift(other)
        shape = np.broadcast(self.v, o.v).shape
        return o, shape

    # --- arithmetic ----------------------------------------------------------
    def __add__(self, other):
        o, sh = self._pair(other)
        return Dual(self.v + o.v, self._bd(self.d, sh) + self._bd(o.d, sh))

    __radd__ = __add__

    def __sub__(self, other):
        o, sh = self._pair(other)
        return Dual(self.v - o.v, self._bd(self.d, sh) - self._bd(o.d, sh))

    def __rsub__(self, other):
        return self._lift(other) - self

    def __mul__(self, other):
        o, sh = self._pair(other)
        return Dual(self.v * o.v, self._bd(self.d, sh) * o.v + self.v * self._bd(o.d, sh))

    __rmul__ = __mul__

    def __truediv__(self, other):
        o, sh = self._pair(other)
        inv = 1.0 / o.v
        return Dual(self.v * inv, (self._bd(self.d, sh) - self.v * inv * self._bd(o.d, sh)) * inv)

    def __rtruediv__(self, other):
        return self._lift(other) / self

    def __neg__(self):
        return Dual(-self.v, -self.d)

    def __getitem__(self, idx):
        if not isinstance(idx, tuple):
            idx = (idx,)
        return Dual(self.v[idx], self.d[(slice(None),) + idx])

    def __repr__(self):
        return f"Dual(v={self.v!r}, d.shape={self.d.shape})"


def value(x):
    return x.v if isinstance(x, Dual) else np.asarray(x, dtype=np.float64)


def tangent(x, n):
    if isinstance(x, Dual):
        return x.d
    x = np.asarray(x, dtype=np.float64)
    return np.zeros((n,) + x.shape)


class ops:
    """Elementary functions dispatching on Dual vs. plain arrays."""

    @staticmethod
    def sqrt(x):
        if isinstance(x, Dual):
            s = np.sqrt(x.v)
            return Dual(s, x.d * (0.5 / s))
        return np.sqrt(x)

    @staticmethod
    def sin(x):
        if isinstance(x, Dual):
            return Dual(np.sin(x.v), x.d * np.cos(x.v))
        return np.sin(x)

    @staticmethod
    def cos(x):
        if isinstance(x, Dual):
            return Dual(np.cos(x.v), -x.d * np.sin(x.v))
        return np.cos(x)

    @staticmethod
    def arcsin(x):
        if isinstance(x, Dual):
            return Dual(np.arcsin(x.v), x.d / np.sqrt(1.0 - x.v * x.v))
        return np.arcsin(x)

    @staticmethod
    def arctan2(y, x):
        if isinstance(y, Dual) or isinstance(x, Dual):
            n = y.n if isinstance(y, Dual) else x.n
            yv, xv = value(y), value(x)
            r2 = xv * xv + yv * yv
            v = np.arctan2(yv, xv)
            dy, dx = tangent(y, n), tangent(x, n)
            return Dual(v, (xv * dy - yv * dx) / r2)
        return np.arctan2(y, x)

    @staticmethod
    def where(mask, a, b):
        """Select elementwise by a boolean mask computed on values."""
        if isinstance(a, Dual) or isinstance(b, Dual):
            n = a.n if isinstance(a, Dual) else b.n
            av, bv = value(a), value(b)
            sh = np.broadcast(mask, av, bv).shape
            ad = np.broadcast_to(Dual._bd(tangent(a, n), sh), (n,) + sh)
            bd = np.broadcast_to(Dual._bd(tangent(b, n), sh), (n,) + sh)
            return Dual(np.where(mask, av, bv), np.where(mask, ad, bd))
        return np.where(mask, a, b)

    @staticmethod
    def sum(x, mask=None):
        if isinstance(x, Dual):
            if mask is None:
                return Dual(x.v.sum(), x.d.reshape(x.n, -1).sum(axis=1))
            return Dual(x.v[mask].sum(), x.d[:, mask].sum(axis=1))
        x = np.asarray(x)
        return x.sum() if mask is None else x[mask].sum()
