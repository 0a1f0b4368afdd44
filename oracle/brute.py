"""Exhaustive dense-dictionary matching pursuit in numpy -- TEST INFRASTRUCTURE ONLY.

A second, independent implementation of the grid search of the residue-based
ACT (Sec. III-A; the projection P = D X^T of Sec. IV-A), for tiny grids only.
It materialises the whole dictionary D (K x N) with numpy broadcasting,
normalises its rows, and runs matching pursuit with the grid parameters (no
continuous refinement).  It shares no code with act_oracle.c; tests use it to
pin the C oracle's axis values, flat index order, tie-break and residual loop.
"""
from __future__ import annotations

import itertools

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


# --------------------------------------------------------------------------
# LEM-inspired hierarchical search (Sec. VII), written independently of the C
# oracle: numpy arrays for the candidate sets, one dense matrix of unit atoms
# per stage, and a stable sort for the top-k.  No continuous refinement: the
# stage winner is the order's atom.
# --------------------------------------------------------------------------

def unit_atoms(fs: float, n: int, theta: np.ndarray) -> np.ndarray:
    """Rows = unit-norm real chirplets at the parameter rows of theta [m, 4]
    (t_c, f_c, c, ln dt); a row whose raw norm is below 1e-300 is zero."""
    th = np.atleast_2d(theta)
    tau = (np.arange(n) / fs)[None, :] - th[:, 0:1]
    D = np.exp(-0.5 * (tau / np.exp(th[:, 3:4])) ** 2) * np.cos(2 * np.pi * (th[:, 2:3] * tau ** 2 + th[:, 1:2] * tau))
    nrm = np.linalg.norm(D, axis=1, keepdims=True)
    return np.where(nrm >= 1e-300, D / np.where(nrm >= 1e-300, nrm, 1.0), 0.0)


def lem_snap(x: np.ndarray, lo: np.ndarray, hi: np.ndarray, step: np.ndarray) -> np.ndarray:
    """Nearest point of the lattice lo + j*step (round half up), pulled back
    inside [lo, hi]; a one-value axis (hi == lo) maps to lo."""
    v = lo + np.floor((x - lo) / step + 0.5) * step
    v = np.where(v > hi, lo + np.floor((hi - lo) / step) * step, v)
    v = np.maximum(v, lo)
    return np.where(hi > lo, v, lo)


def lem_top(cands: np.ndarray, scores: np.ndarray, k: int) -> np.ndarray:
    """The k best distinct parameter rows by |score|; equal scores keep the
    earlier row (a stable sort on -|score|)."""
    kept = []
    for j in np.argsort(-np.abs(scores), kind="stable"):
        if any(np.array_equal(cands[j], q) for q in kept):
            continue
        kept.append(cands[j])
        if len(kept) == k:
            break
    return np.array(kept)


def lem_mp(fs: float, n: int, lo, hi, steps, radius, topk: int, lhs: np.ndarray, s: np.ndarray):
    """Hierarchical matching pursuit of one signal: for every order, the
    Latin-hypercube rows lhs[k] ([samples, 4] in [0,1)) map onto the hull
    [lo, hi] and snap to the level-0 steps; the top-k distinct atoms by
    |<g, r>| seed, at each level l >= 1, the families q + i*steps[l]
    (|i_d| <= radius[d], members outside the hull dropped), pooled and cut to
    the top-k again; the best one is subtracted with c = <g, r>.
    Returns theta [order, 4], coef [order], energy [order+1], residual."""
    lo, hi = np.asarray(lo, float), np.asarray(hi, float)
    steps = np.asarray(steps, float)
    offs = np.array(list(itertools.product(*[range(-int(rd), int(rd) + 1) for rd in radius])), dtype=float)
    r = np.array(s, dtype=np.float64)
    thetas, coefs, energy = [], [], [float(r @ r)]
    for u in lhs:
        cand = lem_snap(lo + u * (hi - lo), lo, hi, steps[0])
        kept = lem_top(cand, unit_atoms(fs, n, cand) @ r, topk)
        for lv in range(1, len(steps)):
            fam = (kept[:, None, :] + offs[None, :, :] * steps[lv]).reshape(-1, 4)
            fam = fam[np.all((fam >= lo) & (fam <= hi), axis=1)]
            kept = lem_top(fam, unit_atoms(fs, n, fam) @ r, topk)
        g = unit_atoms(fs, n, kept[0])[0]
        ck = float(g @ r)
        r = r - ck * g
        thetas.append(kept[0])
        coefs.append(ck)
        energy.append(float(r @ r))
    return np.array(thetas), np.array(coefs), np.array(energy), r
