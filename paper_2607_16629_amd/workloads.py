"""Seeded synthetic workloads for the residue-based ACT matching-pursuit search.

This module is the only thing the HIP path and the oracle share.  It draws
random numbers and writes plain arrays; it contains none of the method's
arithmetic (no correlation, no selection, no refinement, no projection).
The one formula it evaluates is the *signal model* of the workloads: each
test signal is a sum of unit-norm real Gaussian chirplets (the real part of
the Gaussian chirplet of Eq. (1), Sec. II-A) with random off-grid
parameters, plus white or pink noise scaled exactly to a target SNR.

Grids follow the paper's statement of the dictionary as a sampled 4-D
parameter space (Sec. III-A, Table "Parameter ranges"):
  * time centre  t_c in seconds, half-open from 0 over the signal,
    t_c[j] = j * (N / n_tc) / fs;
  * frequency centre f_c in Hz, chirp rate c in Hz/s (the coefficient of
    (t - t_c)^2 in Eq. (1)) and log-duration ln(dt / 1 s), each sampled
    with both end points included.
An axis is the tuple (lo, hi, count, half_open); its j-th value is
lo + j * ((hi - lo) / d) with d = count for a half-open axis and d = count-1
otherwise (the last value of a closed axis is hi exactly).

Seeds: numpy SeedSequence([2607, 16629, cfg]) with one spawned stream per
channel, so that channel b of a workload never depends on the batch size.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import List, Optional, Tuple

import numpy as np

FS_HZ = 256.0
FC_RANGE = (1.0, 64.0)
C_RANGE = (-20.0, 20.0)
LOGDT_RANGE = (math.log(0.05), 0.0)


@dataclass(frozen=True)
class Axis:
    lo: float
    hi: float
    count: int
    half_open: bool

    def values(self) -> np.ndarray:
        d = self.count if self.half_open else self.count - 1
        if self.count == 1:
            return np.array([self.lo])
        step = (self.hi - self.lo) / d
        v = np.array([self.lo + j * step for j in range(self.count)])
        if not self.half_open:
            v[-1] = self.hi
        return v

    def spacing(self) -> float:
        if self.count <= 1:
            return 1.0
        d = self.count if self.half_open else self.count - 1
        return (self.hi - self.lo) / d

    @staticmethod
    def arange(start: float, stop: float, step: float) -> "Axis":
        """Half-open (start, stop, step) axis, numpy.arange counting rule."""
        count = int(math.ceil((stop - start) / step))
        return Axis(start, start + count * step, count, True)


@dataclass(frozen=True)
class Grid:
    """Sampling rate, signal length and the four parameter axes
    (t_c [s], f_c [Hz], c [Hz/s], ln dt [ln s]) of one dictionary."""
    fs: float
    n: int
    tc: Axis
    fc: Axis
    c: Axis
    logdt: Axis

    @property
    def axes(self) -> Tuple[Axis, Axis, Axis, Axis]:
        return (self.tc, self.fc, self.c, self.logdt)

    @property
    def shape(self) -> Tuple[int, int, int, int]:
        return tuple(a.count for a in self.axes)

    @property
    def size(self) -> int:
        k = 1
        for a in self.axes:
            k *= a.count
        return k

    def unflatten(self, i: int) -> Tuple[int, int, int, int]:
        n_tc, n_fc, n_c, n_ld = self.shape
        i_ld = i % n_ld
        i //= n_ld
        i_c = i % n_c
        i //= n_c
        i_fc = i % n_fc
        i_tc = i // n_fc
        return i_tc, i_fc, i_c, i_ld

    def theta(self, i: int) -> np.ndarray:
        vals = [a.values() for a in self.axes]
        return np.array([v[j] for v, j in zip(vals, self.unflatten(i))])


def eeg_grid(n: int, n_tc: int, n_fc: int, n_c: int, n_ld: int,
             fs: float = FS_HZ) -> Grid:
    """The EEG-like grid family used by every workload: t_c half-open over
    the signal, f_c 1..64 Hz, c -20..20 Hz/s, dt 0.05..1 s (log-spaced)."""
    return Grid(fs, n,
                Axis(0.0, n / fs, n_tc, True),
                Axis(FC_RANGE[0], FC_RANGE[1], n_fc, False),
                Axis(C_RANGE[0], C_RANGE[1], n_c, False),
                Axis(LOGDT_RANGE[0], LOGDT_RANGE[1], n_ld, False))


def paper_table_grids():
    """(start, stop, step) ranges printed in the paper's parameter table
    (Sec. III-B, Table "Parameter ranges"), as half-open axes.  The time
    centre there is in samples; it is converted with the sampling rate
    only when a signal is attached, so counts are unit-free."""
    return {
        "EEG": (Axis.arange(0, 256, 16), Axis.arange(0.5, 15, 0.5),
                Axis.arange(-10, 10, 0.5), Axis.arange(-4, 1, 0.5)),
        "EMG": (Axis.arange(0, 200, 32), Axis.arange(20, 450, 10),
                Axis.arange(-10, 10, 0.75), Axis.arange(-4, 0, 0.3)),
        "Radar": (Axis.arange(0, 256, 16), Axis.arange(10, 8533, 100),
                  Axis.arange(-10, 10, 0.75), Axis.arange(-4, 0, 0.3)),
    }


# ----------------------------------------------------------------------------
# signal model
# ----------------------------------------------------------------------------

def _component(fs: float, n: int, theta: np.ndarray) -> np.ndarray:
    """Unit-norm real Gaussian chirplet used to *build* test signals."""
    tc, fc, c, ld = theta
    t = np.arange(n) / fs - tc
    w = np.exp(-0.5 * (t / math.exp(ld)) ** 2) * np.cos(2 * math.pi * (c * t * t + fc * t))
    nrm = math.sqrt(float(np.dot(w, w)))
    return w / nrm if nrm > 0 else w


def _hull_draw(rng: np.random.Generator, grid: Grid) -> np.ndarray:
    lo = [a.values()[0] for a in grid.axes]
    hi = [a.values()[-1] for a in grid.axes]
    return np.array([rng.uniform(l, h) for l, h in zip(lo, hi)])


def _noise(rng: np.random.Generator, n: int, pink: bool) -> np.ndarray:
    w = rng.standard_normal(n)
    if not pink:
        return w
    spec = np.fft.rfft(w)
    k = np.arange(spec.size, dtype=np.float64)
    scale = np.zeros_like(k)
    scale[1:] = k[1:] ** -0.5
    return np.fft.irfft(spec * scale, n)


def make_signal(rng: np.random.Generator, grid: Grid, n_comp: int, snr_db: float,
                pink: bool = False, amp=(0.5, 2.0)):
    """sum_j a_j * sign_j * unit_chirplet(theta_j) + noise at exactly snr_db.
    Returns (signal, thetas[n_comp,4], signed amplitudes[n_comp])."""
    clean = np.zeros(grid.n)
    thetas = np.zeros((n_comp, 4))
    amps = np.zeros(n_comp)
    for j in range(n_comp):
        th = _hull_draw(rng, grid)
        a = rng.uniform(*amp) * (1.0 if rng.uniform() < 0.5 else -1.0)
        clean += a * _component(grid.fs, grid.n, th)
        thetas[j] = th
        amps[j] = a
    noise = _noise(rng, grid.n, pink)
    pc = float(np.dot(clean, clean))
    pn = float(np.dot(noise, noise))
    if pc > 0 and pn > 0 and np.isfinite(snr_db):
        noise *= math.sqrt(pc / (pn * 10.0 ** (snr_db / 10.0)))
    elif not np.isfinite(snr_db):
        noise[:] = 0.0
    return clean + noise, thetas, amps


@dataclass
class Workload:
    name: str
    grid: Grid                       # shared grid (ragged: grid of the longest signal)
    signals: np.ndarray              # [B, N] f64 (ragged: packed, see offsets)
    order: int
    refine_steps: int
    thetas: List[np.ndarray] = field(default_factory=list)
    amps: List[np.ndarray] = field(default_factory=list)
    lengths: Optional[np.ndarray] = None   # ragged only
    offsets: Optional[np.ndarray] = None   # ragged only
    grids: Optional[List[Grid]] = None     # ragged only
    theta0: Optional[np.ndarray] = None    # refinement pairs only

    @property
    def batch(self) -> int:
        return len(self.lengths) if self.lengths is not None else self.signals.shape[0]


def _streams(cfg: int, count: int):
    ss = np.random.SeedSequence([2607, 16629, cfg])
    return [np.random.default_rng(s) for s in ss.spawn(count)]


def plain_1x512(seed_cfg: int = 1) -> Workload:
    """Plain ACT, 1 channel, N=512 at 256 Hz; 32 x 16 x 16 x 8 = 65,536 atoms;
    3 off-grid chirplets, amplitudes U(0.5, 2), white noise at 10 dB; order 5."""
    g = eeg_grid(512, 32, 16, 16, 8)
    rng = _streams(seed_cfg, 1)[0]
    s, th, a = make_signal(rng, g, 3, 10.0)
    return Workload("plain-1x512", g, s[None, :], 5, 30, [th], [a])


def fp32_1x2048(seed_cfg: int = 2, grid: Optional[Grid] = None) -> Workload:
    """Single channel at EEG-like scale: N=2048 (8 s at 256 Hz), grid
    64 x 64 x 32 x 16 = 2,097,152 atoms; 8 chirplets plus pink noise at 5 dB;
    order 10."""
    g = grid or eeg_grid(2048, 64, 64, 32, 16)
    rng = _streams(seed_cfg, 1)[0]
    s, th, a = make_signal(rng, g, 8, 5.0, pink=True)
    return Workload("fp32-1x2048", g, s[None, :], 10, 30, [th], [a])


def batched_64x2048(seed_cfg: int = 3, channels: int = 64,
                    grid: Optional[Grid] = None, order: int = 20) -> Workload:
    """Multi-channel batch: 64 channels x N=2048 on the 2,097,152-atom grid;
    4-12 chirplets per channel, white noise at SNR U(0, 20) dB; order 20."""
    g = grid or eeg_grid(2048, 64, 64, 32, 16)
    rngs = _streams(seed_cfg, channels)
    sig = np.zeros((channels, g.n))
    ths, amps = [], []
    for b, rng in enumerate(rngs):
        k = int(rng.integers(4, 13))
        snr = rng.uniform(0.0, 20.0)
        sig[b], th, a = make_signal(rng, g, k, snr)
        ths.append(th)
        amps.append(a)
    return Workload("bf16-64x2048", g, sig, order, 30, ths, amps)


def refine_pairs(seed_cfg: int = 4, pairs: int = 4096,
                 grid: Optional[Grid] = None) -> Workload:
    """Refinement pairs: each residual is one off-grid chirplet (amplitude
    U(0.5, 2)) plus white noise at 10 dB; the start point is the nearest
    grid point of the 2,097,152-atom grid (within one step on every axis)."""
    g = grid or eeg_grid(2048, 64, 64, 32, 16)
    rngs = _streams(seed_cfg, pairs)
    sig = np.zeros((pairs, g.n))
    theta0 = np.zeros((pairs, 4))
    ths = []
    vals = [a.values() for a in g.axes]
    for p, rng in enumerate(rngs):
        sig[p], th, _ = make_signal(rng, g, 1, 10.0)
        ths.append(th)
        theta0[p] = [v[int(np.argmin(np.abs(v - x)))] for v, x in zip(vals, th[0])]
    w = Workload("refine-4096", g, sig, 1, 30, ths, [])
    w.theta0 = theta0
    return w


def ragged_grid(n: int, tc_div: int, n_fc: int, n_c: int, n_ld: int, fs: float = FS_HZ) -> Grid:
    """Grid of one signal of a ragged batch: floor(n/tc_div) time centres one
    every tc_div samples (the half-open axis (0, n_tc tc_div/fs, n_tc)), and
    the EEG-like f_c / c / dt axes."""
    n_tc = n // tc_div
    g = eeg_grid(n, max(1, n_tc), n_fc, n_c, n_ld, fs)
    if n_tc == 0:  # shorter than one time-centre step: no dictionary (flagged
        # empty by the library); one t_c = 0 keeps the signal model defined
        return Grid(fs, n, Axis(0.0, 0.0, 1, True), g.fc, g.c, g.logdt)
    return Grid(fs, n, Axis(0.0, n_tc * tc_div / fs, n_tc, True), g.fc, g.c, g.logdt)


def ragged_batch(seed_cfg: int = 5, count: int = 1000, n_min: int = 256,
                 n_max: int = 16384, order: int = 15,
                 fc_c_ld: Tuple[int, int, int] = (64, 32, 16), tc_div: int = 32) -> Workload:
    """Uneven batch: lengths log-uniform in [n_min, n_max]; each signal has
    its own grid with n_tc = floor(N/32) time centres every 32 samples and
    64 x 32 x 16 (f_c, c, dt) points; 2-16 chirplets, SNR U(-5, 20) dB;
    order 15."""
    rngs = _streams(seed_cfg, count)
    lens, grids, parts, ths, amps = [], [], [], [], []
    for rng in rngs:
        n = int(round(math.exp(rng.uniform(math.log(n_min), math.log(n_max)))))
        g = ragged_grid(n, tc_div, *fc_c_ld)
        k = int(rng.integers(2, 17))
        s, th, a = make_signal(rng, g, k, rng.uniform(-5.0, 20.0))
        lens.append(n)
        grids.append(g)
        parts.append(s)
        ths.append(th)
        amps.append(a)
    lens = np.array(lens, dtype=np.int32)
    offs = np.zeros(count, dtype=np.int64)
    offs[1:] = np.cumsum(lens[:-1])
    w = Workload("ragged-1000", grids[int(np.argmax(lens))], np.concatenate(parts),
                 order, 30, ths, amps)
    w.lengths, w.offsets, w.grids = lens, offs, grids
    return w


def paper_eeg_grid() -> Grid:
    """The paper's EEG parameter grid (Sec. III-B, Table "Parameter ranges":
    t_c 0..256 step 16 samples, f_c 0.5..15 step 0.5 Hz, c -10..10 step 0.5,
    logDt -4..1 step 0.5; 185,600 atoms) on 1 s windows at 256 Hz, t_c in
    seconds."""
    _, fc, c, ld = paper_table_grids()["EEG"]
    return Grid(FS_HZ, 256, Axis(0.0, 1.0, 16, True), fc, c, ld)


def eeg_sweep(seed_cfg: int = 6, windows: int = 50, order: int = 200) -> Workload:
    """Synthetic stand-in for the paper's convergence and old-vs-new study
    (Sec. III-B/III-C: 50 consecutive 1 s EEG windows, orders up to 200):
    per window 3-8 chirplets over the grid hull plus pink noise at
    SNR U(5, 20) dB."""
    g = paper_eeg_grid()
    sig = np.zeros((windows, g.n))
    ths, amps = [], []
    for b, rng in enumerate(_streams(seed_cfg, windows)):
        s, th, a = make_signal(rng, g, int(rng.integers(3, 9)), rng.uniform(5.0, 20.0), pink=True)
        sig[b] = s
        ths.append(th)
        amps.append(a)
    return Workload("eeg-sweep", g, sig, order, 30, ths, amps)



@dataclass
class LemConfig:
    """Hierarchical search settings: LHS samples, refinement levels, top-k,
    neighbourhood radius per axis (in steps) and the step per level and axis
    (axes t_c [s], f_c [Hz], c [Hz/s], ln dt)."""
    samples: int
    levels: int
    topk: int
    radius: Tuple[int, int, int, int]
    steps: Tuple[Tuple[float, float, float, float], ...]


def paper_lem_config(fs: float = FS_HZ, samples: int = 512) -> LemConfig:
    """The paper's LEM settings (Sec. VII-A): 2 refinement levels, top-4,
    step schedule (t_c, f_c, logDt, c) = (64, 2.0, 2.0, 5.0), (32, 1.0, 1.0,
    2.5), (16, 0.5, 0.5, 0.5) with t_c in samples, radius 2 steps for t_c, f_c
    and c and 1 for logDt; the LHS sample count is not given (512 here)."""
    sched = [(64, 2.0, 2.0, 5.0), (32, 1.0, 1.0, 2.5), (16, 0.5, 0.5, 0.5)]
    steps = tuple((tc / fs, f, c, ld) for tc, f, ld, c in sched)
    return LemConfig(samples, 2, 4, (2, 2, 2, 1), steps)


def lem_lhs(seed_cfg: int, batch: int, order: int, samples: int) -> np.ndarray:
    """Latin-hypercube uniforms [batch][order][samples][4]: per axis a random
    permutation of the strata plus a uniform jitter inside each stratum."""
    out = np.zeros((batch, order, samples, 4))
    for b, rng in enumerate(_streams(seed_cfg, batch)):
        for k in range(order):
            for d in range(4):
                out[b, k, :, d] = (rng.permutation(samples) + rng.uniform(size=samples)) / samples
    return out


def lem_eeg(seed_cfg: int = 7, windows: int = 19, order: int = 10) -> Workload:
    """Synthetic stand-in for the paper's LEM study (Sec. VII-A: 2 s EEG
    epochs of 512 samples, the EEG parameter ranges of its table, order 10,
    19 measured epochs): 3-8 chirplets over the grid hull plus pink noise at
    SNR U(5, 20) dB per window."""
    _, fc, c, ld = paper_table_grids()["EEG"]
    g = Grid(FS_HZ, 512, Axis(0.0, 1.0, 16, True), fc, c, ld)
    sig = np.zeros((windows, g.n))
    for b, rng in enumerate(_streams(seed_cfg, windows)):
        sig[b], _, _ = make_signal(rng, g, int(rng.integers(3, 9)), rng.uniform(5.0, 20.0), pink=True)
    return Workload("lem-eeg", g, sig, order, 30)
