"""Exhaustive dense-dictionary matching pursuit in numpy -- TEST INFRASTRUCTURE ONLY.

A second, independent implementation of the grid search of the residue-based
ACT (Sec. III-A; the projection P = D X^T of Sec. IV-A), for tiny grids only.
It materialises the whole dictionary D (K x N) with numpy broadcasting,
normalises its rows, and runs matching pursuit with the grid parameters (no
continuous refinement).  It shares no code with act_oracle.c; tests use it to
pin the C oracle's axis values, flat index order, tie-break and residual loop.
"""
from __future__ import annotations

import numpy as np


def axis(lo: float, hi: float, count: int, half_open: bool) -> np.ndarray:
    if count == 1:
        return np.array([lo], dtype=np.float64)
    if half_open:
        return lo + np.arange(count) * ((hi - lo) / count)
    v = lo + np.arange(count) * ((hi - lo) / (count - 1))
    v[-1] = hi
    return v


def dictionary(fs: float, n: int, tc, fc, c, logdt) -> np.ndarray:
    """Rows = unit-norm real Gaussian chirplets, index order (tc, fc, c, logdt)."""
    TC, FC, C, LD = np.meshgrid(tc, fc, c, logdt, indexing="ij")
    TC, FC, C, LD = (x.reshape(-1, 1) for x in (TC, FC, C, LD))
    t = (np.arange(n) / fs)[None, :]
    tau = t - TC
    D = np.exp(-0.5 * (tau / np.exp(LD)) ** 2) * np.cos(2 * np.pi * (C * tau ** 2 + FC * tau))
    return D / np.linalg.norm(D, axis=1, keepdims=True)


def mp(D: np.ndarray, s: np.ndarray, order: int):
    """Plain MP over the rows of D: returns indices, coefficients, energies, residual."""
    r = np.array(s, dtype=np.float64)
    idx, coef, energy = [], [], [float(r @ r)]
    for _ in range(order):
        p = D @ r
        i = int(np.argmax(np.abs(p)))  # first maximum = lowest flat index
        ck = float(D[i] @ r)
        r = r - ck * D[i]
        idx.append(i)
        coef.append(ck)
        energy.append(float(r @ r))
    return np.array(idx), np.array(coef), np.array(energy), r
