"""FP64 CPU oracle of the residue-based ACT -- TEST INFRASTRUCTURE ONLY.

Only the test suite, ``__graft_entry__.smoke()`` and the benchmark's
``cpu_baseline`` leg may import this package.  The product path (the HIP
library and its Python binding) never imports, links or runs anything here,
and nothing here imports the product path: the two share only the seeded
workload generator, which holds none of the method's arithmetic.

Two independent implementations live here:
  * ``act_oracle.c`` (ctypes, built with gcc, FP64, no -ffast-math), the
    step-by-step oracle: atoms, norms, correlations, arg-max, refinement,
    matching pursuit, reconstruction;
  * ``brute.py`` (numpy), an exhaustive dense-dictionary matching pursuit
    for tiny grids, used to pin the C oracle's selection loop.

Parity status per function (the pins are in tests/test_oracle_pins.py):
  atoms / norms        pinned: closed-form Gaussian integral, scipy chirp, FFT
  correlate / argmax   pinned: FFT special case, numpy brute force; the
                       top-2 gap against a full numpy sort of |p|
  correlate_many       equal bit for bit to correlate row by row
  objective / gradient pinned: central finite differences, scipy L-BFGS-B optimum
  refine               pinned: off-grid recovery, scipy optimum, monotone J;
                       its coordinate scales against the Gaussian-moment
                       closed forms of the unit atom's metric (real and complex)
  decompose            pinned: MP identities, one-iteration recovery, brute force
  reconstruct          pinned: a_P + r_P = s
  LEM search           pinned: exhaustive search when the families cover the
                       grid (numpy brute force), an independent numpy
                       implementation of every stage with non-covering
                       families, MP identities
  complex atoms        pinned: FFT magnitude special case, central differences,
                       one-order recovery at any phase, projection identities
  prior ACT (contrast) pinned: continuous-time norm of Eq. (1)'s prefactor,
                       numpy brute force of the un-normalised dictionary,
                       central differences of its objective, the closed form
                       of the repeated update, normalised residue above 1
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from typing import Optional, Tuple

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "act_oracle.c")
_LIB = os.path.join(_HERE, "liboracle_act.so")

FLAG_NONFINITE = 1
FLAG_REFINE_REJECTED = 2
FLAG_LINESEARCH = 4


def build(force: bool = True) -> str:
    """Compile the C oracle with gcc (FP64, no contraction, no fast-math)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-ffp-contract=off", "-fno-fast-math",
                               "-std=c11", "-fPIC", "-shared", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


class _Axis(ctypes.Structure):
    _fields_ = [("lo", ctypes.c_double), ("hi", ctypes.c_double),
                ("count", ctypes.c_int32), ("half_open", ctypes.c_int32)]


class _Grid(ctypes.Structure):
    _fields_ = [("fs", ctypes.c_double), ("n", ctypes.c_int32), ("pad", ctypes.c_int32),
                ("ax", _Axis * 4)]


_lib = None


class _Lem(ctypes.Structure):
    _fields_ = [("samples", ctypes.c_int32), ("levels", ctypes.c_int32), ("topk", ctypes.c_int32),
                ("pad", ctypes.c_int32), ("radius", ctypes.c_int32 * 4), ("step", (ctypes.c_double * 4) * 8)]


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build(force=True)
        lib = ctypes.CDLL(_LIB)
        P = ctypes.POINTER
        d, i32, i64 = ctypes.c_double, ctypes.c_int32, ctypes.c_int64
        pd, pi32, pi64 = P(d), P(i32), P(i64)
        pg = P(_Grid)
        lib.oracle_num_threads.restype = ctypes.c_int
        lib.oracle_arange_count.argtypes = [d, d, d]
        lib.oracle_arange_count.restype = i64
        lib.oracle_axis_value.argtypes = [P(_Axis), i32]
        lib.oracle_axis_value.restype = d
        lib.oracle_grid_size.argtypes = [pg]
        lib.oracle_grid_size.restype = i64
        lib.oracle_grid_theta.argtypes = [pg, i64, pd]
        lib.oracle_atom_raw.argtypes = [d, i32, pd, pd]
        lib.oracle_atom_unit.argtypes = [d, i32, pd, pd]
        lib.oracle_atom_unit.restype = d
        lib.oracle_correlate.argtypes = [pg, pd, i64, i64, pd]
        lib.oracle_correlate_many.argtypes = [pg, i32, pd, i64, i64, pd]
        lib.oracle_correlate_complex_many.argtypes = [pg, i32, pd, i64, i64, pd]
        lib.oracle_norms.argtypes = [pg, i64, i64, pd]
        lib.oracle_argmax.argtypes = [pd, i64, pd]
        lib.oracle_argmax.restype = i64
        lib.oracle_objective.argtypes = [d, i32, pd, pd, pd, pd]
        lib.oracle_objective.restype = d
        lib.oracle_refine.argtypes = [d, i32, pd, pd, pd, pd, pd, i32, pd, pd]
        lib.oracle_refine.restype = ctypes.c_int
        lib.oracle_refine_box.argtypes = [pg, pd, pd, pd]
        lib.oracle_refine_scales.argtypes = [d, i32, pd, pd, pd, pd, pd]
        lib.oracle_refine_scales_complex.argtypes = [d, i32, pd, pd, pd, pd, pd]
        lib.oracle_refine_many.argtypes = [pg, i32, pd, pd, i32, pd, pd, pi32]
        lib.oracle_decompose.argtypes = [pg, i32, pd, i32, i32, pd, pd, pd, pd, pi64, pd, pd, pi32]
        lib.oracle_reconstruct.argtypes = [d, i32, i32, pd, pd, pd]
        lib.oracle_atom_prior.argtypes = [d, i32, pd, pd]
        lib.oracle_correlate_prior.argtypes = [pg, pd, i64, i64, pd]
        lib.oracle_objective_prior.argtypes = [d, i32, pd, pd, pd]
        lib.oracle_objective_prior.restype = d
        lib.oracle_refine_prior.argtypes = [d, i32, pd, pd, pd, pd, pd, i32, pd, pd]
        lib.oracle_refine_prior.restype = ctypes.c_int
        lib.oracle_decompose_prior.argtypes = [pg, i32, pd, i32, i32, pd, pd, pd, pd, pi64, pd, pi32]
        lib.oracle_lem_decompose.argtypes = [pg, P(_Lem), i32, pd, pd, i32, i32, pd, pd, pd, pd, pd, pi32]
        lib.oracle_correlate_complex.argtypes = [pg, pd, i64, i64, pd]
        lib.oracle_objective_complex.argtypes = [d, i32, pd, pd, pd]
        lib.oracle_objective_complex.restype = d
        lib.oracle_refine_complex.argtypes = [d, i32, pd, pd, pd, pd, pd, i32, pd, pd]
        lib.oracle_refine_complex.restype = ctypes.c_int
        lib.oracle_decompose_complex.argtypes = [pg, i32, pd, i32, i32, pd, pd, pd, pd, pd, pi64, pd, pd, pi32]
        lib.oracle_atom_complex.argtypes = [d, i32, pd, pd, pd]
        lib.oracle_fit_complex.argtypes = [d, i32, pd, pd, pd]
        _lib = lib
    return _lib


def _p(a: np.ndarray, ct=ctypes.c_double):
    return a.ctypes.data_as(ctypes.POINTER(ct))


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float64)


def make_grid(grid) -> _Grid:
    """ctypes grid from a workloads.Grid (fs, n, four axes)."""
    g = _Grid()
    g.fs = float(grid.fs)
    g.n = int(grid.n)
    for k, a in enumerate(grid.axes):
        g.ax[k].lo, g.ax[k].hi = float(a.lo), float(a.hi)
        g.ax[k].count, g.ax[k].half_open = int(a.count), int(bool(a.half_open))
    return g


def num_threads() -> int:
    return int(_load().oracle_num_threads())


def arange_count(start: float, stop: float, step: float) -> int:
    return int(_load().oracle_arange_count(start, stop, step))


def axis_values(axis) -> np.ndarray:
    lib = _load()
    a = _Axis(float(axis.lo), float(axis.hi), int(axis.count), int(bool(axis.half_open)))
    return np.array([lib.oracle_axis_value(ctypes.byref(a), j) for j in range(axis.count)])


def grid_size(grid) -> int:
    g = make_grid(grid)
    return int(_load().oracle_grid_size(ctypes.byref(g)))


def grid_theta(grid, i: int) -> np.ndarray:
    g = make_grid(grid)
    out = np.zeros(4)
    _load().oracle_grid_theta(ctypes.byref(g), int(i), _p(out))
    return out


def atom_raw(fs: float, n: int, theta) -> np.ndarray:
    out = np.zeros(n)
    _load().oracle_atom_raw(float(fs), int(n), _p(_f64(theta)), _p(out))
    return out


def atom_unit(fs: float, n: int, theta) -> Tuple[np.ndarray, float]:
    out = np.zeros(n)
    nrm = _load().oracle_atom_unit(float(fs), int(n), _p(_f64(theta)), _p(out))
    return out, float(nrm)


def correlate(grid, r, begin: int = 0, count: Optional[int] = None) -> np.ndarray:
    g = make_grid(grid)
    if count is None:
        count = grid_size(grid) - begin
    r = _f64(r)
    assert r.shape == (grid.n,)
    out = np.zeros(count)
    _load().oracle_correlate(ctypes.byref(g), _p(r), int(begin), int(count), _p(out))
    return out


def correlate_many(grid, R, begin: int = 0, count: Optional[int] = None,
                   complex_atoms: bool = False) -> np.ndarray:
    """Scores of the atoms [begin, begin+count) against every row of R
    ([m, N]); row t equals correlate(grid, R[t]) (or correlate_complex) bit
    for bit.  Each atom is synthesised once for all rows."""
    g = make_grid(grid)
    if count is None:
        count = grid_size(grid) - begin
    R = _f64(np.atleast_2d(R))
    assert R.shape[1] == grid.n
    out = np.zeros((R.shape[0], count))
    fn = _load().oracle_correlate_complex_many if complex_atoms else _load().oracle_correlate_many
    fn(ctypes.byref(g), R.shape[0], _p(R), int(begin), int(count), _p(out))
    return out


def argmax_many(grid, R, complex_atoms: bool = False):
    """Exhaustive arg-max (Sec. III-A) of every row of R over the whole
    dictionary: (indices, relative top-2 gaps, |p| of the winners)."""
    P = correlate_many(grid, R, complex_atoms=complex_atoms)
    idx, gap, top = [], [], []
    for row in P:
        i, gp = argmax(row)
        idx.append(i)
        gap.append(gp)
        top.append(abs(row[i]))
    return np.array(idx, dtype=np.int64), np.array(gap), np.array(top)


def norms(grid, begin: int = 0, count: Optional[int] = None) -> np.ndarray:
    g = make_grid(grid)
    if count is None:
        count = grid_size(grid) - begin
    out = np.zeros(count)
    _load().oracle_norms(ctypes.byref(g), int(begin), int(count), _p(out))
    return out


def argmax(p) -> Tuple[int, float]:
    p = _f64(p)
    gap = ctypes.c_double(0.0)
    i = _load().oracle_argmax(_p(p), p.size, ctypes.byref(gap))
    return int(i), float(gap.value)


def objective(fs: float, theta, r, want_dr: bool = False):
    """(J, dJ/dtheta[4], dJ/dr or None) of J = <r,g>^2/<g,g>."""
    r = _f64(r)
    grad = np.zeros(4)
    dr = np.zeros(r.size) if want_dr else None
    J = _load().oracle_objective(float(fs), r.size, _p(_f64(theta)), _p(r), _p(grad),
                                 _p(dr) if dr is not None else None)
    return float(J), grad, dr


def refine_box(grid):
    g = make_grid(grid)
    step, lo, hi = np.zeros(4), np.zeros(4), np.zeros(4)
    _load().oracle_refine_box(ctypes.byref(g), _p(step), _p(lo), _p(hi))
    return step, lo, hi


def refine_scales(grid, theta0, complex_atoms: bool = False) -> np.ndarray:
    step, lo, hi = refine_box(grid)
    h = np.zeros(4)
    fn = _load().oracle_refine_scales_complex if complex_atoms else _load().oracle_refine_scales
    fn(float(grid.fs), int(grid.n), _p(_f64(theta0)), _p(step), _p(lo), _p(hi), _p(h))
    return h


def refine(grid, r, theta0, steps: int = 30):
    """Refined theta, J(theta), flags for one residual and start point."""
    step, lo, hi = refine_box(grid)
    th = np.zeros(4)
    J = ctypes.c_double(0.0)
    fl = _load().oracle_refine(float(grid.fs), int(grid.n), _p(_f64(r)), _p(_f64(theta0)),
                               _p(step), _p(lo), _p(hi), int(steps), _p(th), ctypes.byref(J))
    return th, float(J.value), int(fl)


def refine_many(grid, r, theta0, steps: int = 30):
    r = _f64(r)
    theta0 = _f64(theta0)
    m = r.shape[0]
    g = make_grid(grid)
    th = np.zeros((m, 4))
    J = np.zeros(m)
    fl = np.zeros(m, dtype=np.int32)
    _load().oracle_refine_many(ctypes.byref(g), m, _p(r), _p(theta0), int(steps), _p(th), _p(J),
                               _p(fl, ctypes.c_int32))
    return th, J, fl


def decompose(grid, signals, order: int, refine_steps: int = 30):
    """Residue-based MP of each row of ``signals`` ([B, N] or [N])."""
    s = _f64(np.atleast_2d(signals))
    B, n = s.shape
    assert n == grid.n
    g = make_grid(grid)
    out = dict(
        resid=np.zeros((B, n)), approx=np.zeros((B, n)), theta=np.zeros((B, order, 4)),
        coef=np.zeros((B, order)), index=np.zeros((B, order), dtype=np.int64),
        energy=np.zeros((B, order + 1)), gap=np.zeros((B, order)),
        flags=np.zeros(B, dtype=np.int32))
    _load().oracle_decompose(ctypes.byref(g), B, _p(s), int(order), int(refine_steps),
                             _p(out["resid"]), _p(out["approx"]), _p(out["theta"]),
                             _p(out["coef"]), _p(out["index"], ctypes.c_int64),
                             _p(out["energy"]), _p(out["gap"]), _p(out["flags"], ctypes.c_int32))
    return out


def reconstruct(fs: float, n: int, theta, coef) -> np.ndarray:
    theta = _f64(theta).reshape(-1, 4)
    coef = _f64(coef).reshape(-1)
    out = np.zeros(n)
    _load().oracle_reconstruct(float(fs), int(n), theta.shape[0], _p(theta), _p(coef), _p(out))
    return out


# ---------------------------------------------------------------------------
# The prior ACT (Sec. III-A, Table "Comparison of algorithmic properties"):
# un-normalised atoms with Eq. (1)'s prefactor; search, refinement and
# coefficient against the original signal.
# ---------------------------------------------------------------------------

def atom_prior(fs: float, n: int, theta) -> np.ndarray:
    out = np.zeros(n)
    _load().oracle_atom_prior(float(fs), int(n), _p(_f64(theta)), _p(out))
    return out


def correlate_prior(grid, s, begin: int = 0, count: Optional[int] = None) -> np.ndarray:
    s = _f64(s)
    K = grid_size(grid)
    count = K - begin if count is None else count
    out = np.zeros(count)
    g = make_grid(grid)
    _load().oracle_correlate_prior(ctypes.byref(g), _p(s), int(begin), int(count), _p(out))
    return out


def objective_prior(fs: float, theta, s):
    """(J, dJ/dtheta) of J = <s, g(theta)>^2 with the un-normalised atom."""
    s = _f64(s)
    grad = np.zeros(4)
    J = _load().oracle_objective_prior(float(fs), s.size, _p(_f64(theta)), _p(s), _p(grad))
    return float(J), grad


def refine_prior(grid, s, theta0, steps: int = 30):
    step, lo, hi = refine_box(grid)
    th = np.zeros(4)
    J = ctypes.c_double(0.0)
    fl = _load().oracle_refine_prior(float(grid.fs), int(grid.n), _p(_f64(s)), _p(_f64(theta0)),
                                     _p(step), _p(lo), _p(hi), int(steps), _p(th), ctypes.byref(J))
    return th, float(J.value), int(fl)


def decompose_prior(grid, signals, order: int, refine_steps: int = 30):
    """The prior ACT over `order` orders for each row of ``signals``."""
    s = _f64(np.atleast_2d(signals))
    B, n = s.shape
    assert n == grid.n
    g = make_grid(grid)
    out = dict(resid=np.zeros((B, n)), approx=np.zeros((B, n)), theta=np.zeros((B, order, 4)),
               coef=np.zeros((B, order)), index=np.zeros((B, order), dtype=np.int64),
               energy=np.zeros((B, order + 1)), flags=np.zeros(B, dtype=np.int32))
    _load().oracle_decompose_prior(ctypes.byref(g), B, _p(s), int(order), int(refine_steps),
                                   _p(out["resid"]), _p(out["approx"]), _p(out["theta"]), _p(out["coef"]),
                                   _p(out["index"], ctypes.c_int64), _p(out["energy"]),
                                   _p(out["flags"], ctypes.c_int32))
    return out


# ---------------------------------------------------------------------------
# LEM-inspired hierarchical coarse-to-fine search (Sec. VII)
# ---------------------------------------------------------------------------

def make_lem(cfg) -> _Lem:
    """cfg: samples, levels, topk, radius[4], steps[levels+1][4] (axes t_c s,
    f_c Hz, c Hz/s, ln dt)."""
    L = _Lem()
    L.samples, L.levels, L.topk = int(cfg.samples), int(cfg.levels), int(cfg.topk)
    for d in range(4):
        L.radius[d] = int(cfg.radius[d])
    for lv, row in enumerate(cfg.steps):
        for d in range(4):
            L.step[lv][d] = float(row[d])
    return L


def lem_decompose(grid, signals, lhs, cfg, order: int, refine_steps: int = 30):
    """Hierarchical search + refinement per order; lhs [B][order][samples][4]."""
    s = _f64(np.atleast_2d(signals))
    B, n = s.shape
    lhs = _f64(lhs)
    assert lhs.shape == (B, order, cfg.samples, 4)
    g = make_grid(grid)
    L = make_lem(cfg)
    out = dict(resid=np.zeros((B, n)), approx=np.zeros((B, n)), theta=np.zeros((B, order, 4)),
               coef=np.zeros((B, order)), energy=np.zeros((B, order + 1)), flags=np.zeros(B, dtype=np.int32))
    _load().oracle_lem_decompose(ctypes.byref(g), ctypes.byref(L), B, _p(s), _p(lhs), int(order),
                                 int(refine_steps), _p(out["resid"]), _p(out["approx"]), _p(out["theta"]),
                                 _p(out["coef"]), _p(out["energy"]), _p(out["flags"], ctypes.c_int32))
    return out


# ---------------------------------------------------------------------------
# Complex (analytic) atoms: Eq. (1) literally, |<g_hat, r>| selection,
# amplitude-and-phase least-squares update of the real residual.
# ---------------------------------------------------------------------------

def correlate_complex(grid, r, begin: int = 0, count: Optional[int] = None) -> np.ndarray:
    r = _f64(r)
    K = grid_size(grid)
    count = K - begin if count is None else count
    out = np.zeros(count)
    g = make_grid(grid)
    _load().oracle_correlate_complex(ctypes.byref(g), _p(r), int(begin), int(count), _p(out))
    return out


def objective_complex(fs: float, theta, r):
    r = _f64(r)
    grad = np.zeros(4)
    J = _load().oracle_objective_complex(float(fs), r.size, _p(_f64(theta)), _p(r), _p(grad))
    return float(J), grad


def refine_complex(grid, r, theta0, steps: int = 30):
    step, lo, hi = refine_box(grid)
    th = np.zeros(4)
    J = ctypes.c_double(0.0)
    fl = _load().oracle_refine_complex(float(grid.fs), int(grid.n), _p(_f64(r)), _p(_f64(theta0)),
                                       _p(step), _p(lo), _p(hi), int(steps), _p(th), ctypes.byref(J))
    return th, float(J.value), int(fl)


def atom_complex(fs: float, n: int, theta) -> Tuple[np.ndarray, np.ndarray]:
    """(E cos phi, E sin phi) of the raw complex atom at theta."""
    u, v = np.zeros(n), np.zeros(n)
    _load().oracle_atom_complex(float(fs), int(n), _p(_f64(theta)), _p(u), _p(v))
    return u, v


def fit_complex(fs: float, theta, r) -> np.ndarray:
    """Least-squares amplitudes (alpha, beta) of r on the atom's two parts."""
    r = _f64(r)
    ab = np.zeros(2)
    _load().oracle_fit_complex(float(fs), r.size, _p(_f64(theta)), _p(r), _p(ab))
    return ab


def decompose_complex(grid, signals, order: int, refine_steps: int = 30):
    s = _f64(np.atleast_2d(signals))
    B, n = s.shape
    assert n == grid.n
    g = make_grid(grid)
    out = dict(resid=np.zeros((B, n)), approx=np.zeros((B, n)), theta=np.zeros((B, order, 4)),
               coef_re=np.zeros((B, order)), coef_im=np.zeros((B, order)),
               index=np.zeros((B, order), dtype=np.int64), energy=np.zeros((B, order + 1)),
               gap=np.zeros((B, order)), flags=np.zeros(B, dtype=np.int32))
    _load().oracle_decompose_complex(ctypes.byref(g), B, _p(s), int(order), int(refine_steps),
                                     _p(out["resid"]), _p(out["approx"]), _p(out["theta"]), _p(out["coef_re"]),
                                     _p(out["coef_im"]), _p(out["index"], ctypes.c_int64), _p(out["energy"]),
                                     _p(out["gap"]), _p(out["flags"], ctypes.c_int32))
    return out
