"""Python binding of libact (the C ABI in include/act.h).

Argument marshalling only: every step of the method runs in the HIP library.
PyTorch provides device memory and the current stream.  There is no CPU
fallback: if libact.so is missing or no GPU is present, the calls raise.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional

import torch

from .workloads import Grid

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libact.so")

ACT_OK, ACT_ERR_INVALID, ACT_ERR_NOMEM, ACT_ERR_HIP, ACT_ERR_UNSUPPORTED = range(5)
ACT_DICT_SYNTH, ACT_DICT_TABLE, ACT_DICT_LAG = 0, 1, 2
ACT_PREC_F64, ACT_PREC_F32, ACT_PREC_BF16, ACT_PREC_F16 = 0, 1, 2, 3
FLAG_NONFINITE, FLAG_REFINE_REJECTED, FLAG_CAND_OVERFLOW, FLAG_RAGGED_EMPTY, FLAG_BAD_LENGTH = 1, 2, 8, 16, 32
Q_ATOMS, Q_TABLE_BYTES, Q_N_PAD, Q_CAND_CAP, Q_WORKSPACE_BYTES, Q_LAG_RESIDENT = range(6)
LEM_SCRATCH_BYTES = 16 << 20  # ACT_LEM_SCRATCH_BYTES: act_lem_decompose_noalloc's device array

_DICTS = {"synth": ACT_DICT_SYNTH, "table": ACT_DICT_TABLE, "lag": ACT_DICT_LAG}
_PRECS = {"f64": ACT_PREC_F64, "f32": ACT_PREC_F32, "bf16": ACT_PREC_BF16, "f16": ACT_PREC_F16}


class ActError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{msg} (status {status})")
        self.status = status


class _Axis(ctypes.Structure):
    _fields_ = [("lo", ctypes.c_double), ("hi", ctypes.c_double),
                ("count", ctypes.c_int32), ("half_open", ctypes.c_int32)]


class _Grid(ctypes.Structure):
    _fields_ = [("fs_hz", ctypes.c_double), ("n_samples", ctypes.c_int32),
                ("reserved", ctypes.c_int32), ("tc_s", _Axis), ("fc_hz", _Axis),
                ("c_hz_per_s", _Axis), ("logdt_ln_s", _Axis)]


class _PlanDesc(ctypes.Structure):
    _fields_ = [("grid", _Grid), ("dict", ctypes.c_int32), ("prec", ctypes.c_int32),
                ("max_batch", ctypes.c_int32), ("cand_cap", ctypes.c_int32),
                ("refine_steps", ctypes.c_int32), ("ragged", ctypes.c_int32),
                ("ragged_tc_div", ctypes.c_int32), ("support_cut", ctypes.c_int32),
                ("prior_act", ctypes.c_int32), ("complex_atoms", ctypes.c_int32)]


EXPORTS = ("act_plan", "act_plan_destroy", "act_plan_query", "act_search_flops", "act_search_executed",
           "act_decompose", "act_lem_decompose", "act_probe_read", "act_probe_mfma", "act_refine_f32",
           "act_lem_decompose_noalloc",
           "act_refine", "act_value_and_grad", "act_reconstruct", "act_correlate", "act_tune",
           "act_set_launch_shape", "act_timing_enable", "act_timing_read", "act_status_string", "act_last_error")
PHASES = ("search", "rerun", "rescore", "select_refine_update")

_lib = None


class _LaunchShape(ctypes.Structure):
    _fields_ = [("grid_per_cu", ctypes.c_int32), ("chan_per_fc", ctypes.c_int32),
                ("from_cache", ctypes.c_int32), ("form", ctypes.c_int32), ("ms", ctypes.c_double)]


class _LemDesc(ctypes.Structure):
    _fields_ = [("samples", ctypes.c_int32), ("levels", ctypes.c_int32), ("topk", ctypes.c_int32),
                ("reserved", ctypes.c_int32), ("radius", ctypes.c_int32 * 4),
                ("step", (ctypes.c_double * 4) * 8)]


def make_lem_desc(cfg) -> _LemDesc:
    """cfg: samples, levels, topk, radius[4], steps[levels+1][4]."""
    d = _LemDesc()
    d.samples, d.levels, d.topk = int(cfg.samples), int(cfg.levels), int(cfg.topk)
    for a in range(4):
        d.radius[a] = int(cfg.radius[a])
    for lv, row in enumerate(cfg.steps):
        for a in range(4):
            d.step[lv][a] = float(row[a])
    return d


def load() -> ctypes.CDLL:
    """Loads libact.so; raises if it was not built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with paper_2607_16629_amd.build.build()")
    lib = ctypes.CDLL(LIB_PATH)
    vp, i32, i64, d = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double
    lib.act_plan.argtypes = [ctypes.POINTER(_PlanDesc), vp, ctypes.POINTER(vp)]
    lib.act_lem_decompose.argtypes = [vp, ctypes.POINTER(_LemDesc), i32, vp, vp, vp, i32, vp, vp, vp, vp, vp]
    lib.act_lem_decompose.restype = ctypes.c_int
    lib.act_lem_decompose_noalloc.argtypes = [vp, ctypes.POINTER(_LemDesc), i32, vp, vp, vp, i32, vp, vp, vp, vp, vp]
    lib.act_lem_decompose_noalloc.restype = ctypes.c_int
    lib.act_plan.restype = ctypes.c_int
    lib.act_plan_destroy.argtypes = [vp]
    lib.act_plan_destroy.restype = None
    lib.act_plan_query.argtypes = [vp, i32]
    lib.act_plan_query.restype = i64
    lib.act_search_flops.argtypes = [vp, i32, ctypes.POINTER(ctypes.c_double)]
    lib.act_search_flops.restype = i32
    lib.act_search_executed.argtypes = [vp, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(i64)]
    lib.act_search_executed.restype = i32
    lib.act_probe_read.argtypes = [vp, i64, i32, vp, vp]
    lib.act_probe_read.restype = i32
    lib.act_probe_mfma.argtypes = [i32, i32, i32, vp, ctypes.POINTER(ctypes.c_double), vp]
    lib.act_probe_mfma.restype = i32
    lib.act_decompose.argtypes = [vp, i32, vp, vp, vp, vp, i32, vp, vp, vp, vp, vp, vp, vp]
    lib.act_decompose.restype = ctypes.c_int
    lib.act_refine.argtypes = [vp, i32, vp, vp, i32, vp, vp, vp, vp]
    lib.act_refine.restype = ctypes.c_int
    lib.act_refine_f32.argtypes = [vp, i32, vp, vp, i32, vp, vp, vp, vp]
    lib.act_refine_f32.restype = ctypes.c_int
    lib.act_value_and_grad.argtypes = [vp, i32, i32, vp, vp, vp, vp, vp, vp]
    lib.act_value_and_grad.restype = ctypes.c_int
    lib.act_reconstruct.argtypes = [vp, i32, i32, vp, vp, vp, vp, vp, vp]
    lib.act_reconstruct.restype = ctypes.c_int
    lib.act_correlate.argtypes = [vp, i32, vp, i64, i64, vp, vp]
    lib.act_correlate.restype = ctypes.c_int
    lib.act_tune.argtypes = [vp, i32, vp, vp, vp, i32, ctypes.c_char_p, ctypes.POINTER(_LaunchShape), vp]
    lib.act_tune.restype = ctypes.c_int
    lib.act_set_launch_shape.argtypes = [vp, i32, ctypes.POINTER(_LaunchShape)]
    lib.act_set_launch_shape.restype = ctypes.c_int
    lib.act_timing_enable.argtypes = [vp, i32]
    lib.act_timing_enable.restype = ctypes.c_int
    lib.act_timing_read.argtypes = [vp, ctypes.POINTER(d), ctypes.POINTER(i64)]
    lib.act_timing_read.restype = ctypes.c_int
    lib.act_status_string.argtypes = [ctypes.c_int]
    lib.act_status_string.restype = ctypes.c_char_p
    lib.act_last_error.argtypes = []
    lib.act_last_error.restype = ctypes.c_char_p
    _lib = lib
    return lib


def _check(status: int):
    if status != ACT_OK:
        lib = load()
        raise ActError(status, f"{lib.act_status_string(status).decode()}: {lib.act_last_error().decode()}")


def _ptr(t: Optional[torch.Tensor]):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _device_tensor(x, dtype) -> torch.Tensor:
    t = torch.as_tensor(x, dtype=dtype)
    if not t.is_cuda:
        t = t.cuda()
    return t.contiguous()


def make_desc(grid: Grid, dict_: str = "table", prec: str = "f32", max_batch: int = 1,
              cand_cap: int = 0, refine_steps: int = 30, ragged: bool = False,
              ragged_tc_div: int = 32, support_cut: bool = False, prior_act: bool = False,
              complex_atoms: bool = False) -> _PlanDesc:
    g = _Grid()
    g.fs_hz = float(grid.fs)
    g.n_samples = int(grid.n)
    for name, a in zip(("tc_s", "fc_hz", "c_hz_per_s", "logdt_ln_s"), grid.axes):
        setattr(g, name, _Axis(float(a.lo), float(a.hi), int(a.count), int(bool(a.half_open))))
    desc = _PlanDesc()
    desc.grid = g
    desc.dict = _DICTS[dict_]
    desc.prec = _PRECS[prec]
    desc.max_batch = int(max_batch)
    desc.cand_cap = int(cand_cap)
    desc.refine_steps = int(refine_steps)
    desc.ragged = int(bool(ragged))
    desc.ragged_tc_div = int(ragged_tc_div)
    desc.support_cut = int(bool(support_cut))
    desc.prior_act = int(bool(prior_act))
    desc.complex_atoms = int(bool(complex_atoms))
    return desc


def probe_read(buf: torch.Tensor, blocks_per_cu: int, sink: torch.Tensor):
    """One streaming read of `buf` (a CUDA tensor) on the current stream."""
    assert buf.is_cuda and buf.is_contiguous() and sink.is_cuda and sink.dtype == torch.float32
    _check(load().act_probe_read(_ptr(buf), buf.numel() * buf.element_size(), int(blocks_per_cu), _ptr(sink),
                                 _stream()))


def probe_mfma(prec: str, iters: int, blocks_per_cu: int, sink: torch.Tensor) -> float:
    """One MFMA-loop launch on the current stream; returns its flops."""
    assert sink.is_cuda and sink.dtype == torch.float32
    f = ctypes.c_double(0.0)
    _check(load().act_probe_mfma(_PRECS[prec], int(iters), int(blocks_per_cu), _ptr(sink), ctypes.byref(f),
                                 _stream()))
    return f.value


class Plan:
    """Owns an act_plan_t.  See include/act.h for every call's contract."""

    def __init__(self, grid: Grid, dict_: str = "table", prec: str = "f32", max_batch: int = 1,
                 cand_cap: int = 0, refine_steps: int = 30, ragged: bool = False,
                 ragged_tc_div: int = 32, support_cut: bool = False, prior_act: bool = False,
                 complex_atoms: bool = False):
        lib = load()
        if not torch.cuda.is_available():
            raise RuntimeError("libact needs a ROCm GPU; none is visible")
        self.grid = grid
        self.dict = dict_
        self.prec = prec
        self.max_batch = max_batch
        self.refine_steps = refine_steps
        self.ragged = ragged
        self.support_cut = support_cut
        self.prior_act = prior_act
        self.complex_atoms = complex_atoms
        self._desc = make_desc(grid, dict_, prec, max_batch, cand_cap, refine_steps, ragged,
                               ragged_tc_div, support_cut, prior_act, complex_atoms)
        h = ctypes.c_void_p()
        _check(lib.act_plan(ctypes.byref(self._desc), _stream(), ctypes.byref(h)))
        self._h = h

    def close(self):
        if getattr(self, "_h", None):
            load().act_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def query(self, key: int) -> int:
        return int(load().act_plan_query(self._h, key))

    def search_flops(self, batch: int) -> float:
        """Matrix-core flops of one pass-0 search of `batch` channels (lag-table plans)."""
        out = ctypes.c_double(0.0)
        _check(load().act_search_flops(self._h, int(batch), ctypes.byref(out)))
        return out.value

    def search_executed(self):
        """(flops, launches) the pass-0 searches executed since the last read,
        counted on the device (lag-table and FP16 synthesis plans); resets."""
        f = ctypes.c_double(0.0)
        n = ctypes.c_int64(0)
        _check(load().act_search_executed(self._h, ctypes.byref(f), ctypes.byref(n)))
        return f.value, int(n.value)

    @property
    def atoms(self) -> int:
        return self.query(Q_ATOMS)

    @property
    def n_pad(self) -> int:
        return self.query(Q_N_PAD)

    @property
    def table_bytes(self) -> int:
        return self.query(Q_TABLE_BYTES)

    def act_timing_enable(self, enable: bool = True):
        _check(load().act_timing_enable(self._h, int(bool(enable))))

    def act_timing_read(self) -> dict:
        """{phase: (total ms, launches)} since the last read (synchronises)."""
        ms = (ctypes.c_double * 4)()
        n = (ctypes.c_int64 * 4)()
        _check(load().act_timing_read(self._h, ms, n))
        return {PHASES[i]: (float(ms[i]), int(n[i])) for i in range(4)}

    def alloc_outputs(self, batch: int, order: int, approx: bool = True):
        dev = torch.device("cuda")
        n = self.grid.n
        return dict(
            approx=torch.empty(batch, n, dtype=torch.float64, device=dev) if approx else None,
            theta=torch.empty(batch, order, 4, dtype=torch.float64, device=dev),
            # complex atoms: an amplitude pair per order
            coef=torch.empty((batch, order, 2) if self.complex_atoms else (batch, order), dtype=torch.float64,
                             device=dev),
            index=torch.empty(batch, order, dtype=torch.int64, device=dev),
            energy=torch.empty(batch, order + 1, dtype=torch.float64, device=dev),
            gap=torch.empty(batch, order, dtype=torch.float64, device=dev),
            flags=torch.empty(batch, dtype=torch.int32, device=dev))

    def act_decompose(self, resid: torch.Tensor, order: int, out: dict):
        """In-place on `resid` ([B, N] f64 CUDA): signals in, residuals out."""
        assert resid.is_cuda and resid.dtype == torch.float64 and resid.is_contiguous()
        B = resid.shape[0]
        _check(load().act_decompose(
            self._h, B, None, None, _ptr(resid), _ptr(out["approx"]), int(order),
            _ptr(out["theta"]), _ptr(out["coef"]), _ptr(out["index"]), _ptr(out["energy"]),
            _ptr(out["gap"]), _ptr(out["flags"]), _stream()))
        return out

    def decompose(self, signals, order: int, approx: bool = True) -> dict:
        resid = _device_tensor(signals, torch.float64).reshape(-1, self.grid.n).clone()
        out = self.alloc_outputs(resid.shape[0], order, approx)
        self.act_decompose(resid, order, out)
        out["resid"] = resid
        return out

    def act_decompose_ragged(self, resid: torch.Tensor, lengths: torch.Tensor,
                             offsets: torch.Tensor, order: int, out: dict):
        """Ragged batch: resid is the packed f64 CUDA signals (in place),
        lengths int32 and offsets int64 CUDA tensors."""
        assert resid.is_cuda and resid.dtype == torch.float64 and resid.is_contiguous()
        assert lengths.dtype == torch.int32 and offsets.dtype == torch.int64
        B = lengths.shape[0]
        _check(load().act_decompose(
            self._h, B, _ptr(lengths), _ptr(offsets), _ptr(resid), _ptr(out["approx"]), int(order),
            _ptr(out["theta"]), _ptr(out["coef"]), _ptr(out["index"]), _ptr(out["energy"]),
            _ptr(out["gap"]), _ptr(out["flags"]), _stream()))
        return out

    def act_lem_decompose(self, resid: torch.Tensor, lhs: torch.Tensor, cfg, order: int, out: dict):
        """Hierarchical (LEM-inspired) decomposition in place on `resid` ([B, N]
        f64 CUDA); lhs [B, order, samples, 4] f64 CUDA uniforms."""
        assert resid.is_cuda and resid.dtype == torch.float64 and resid.is_contiguous()
        assert lhs.is_cuda and lhs.dtype == torch.float64 and lhs.is_contiguous()
        B = resid.shape[0]
        assert tuple(lhs.shape) == (B, order, cfg.samples, 4)
        desc = make_lem_desc(cfg)
        _check(load().act_lem_decompose(
            self._h, ctypes.byref(desc), B, _ptr(lhs), _ptr(resid), _ptr(out["approx"]), int(order),
            _ptr(out["theta"]), _ptr(out["coef"]), _ptr(out["energy"]), _ptr(out["flags"]), _stream()))
        return out

    def act_lem_decompose_noalloc(self, resid: torch.Tensor, lhs: torch.Tensor, cfg, order: int, out: dict):
        """act_lem_decompose with its workspace in the library's fixed device
        array (no device allocation inside the call)."""
        assert resid.is_cuda and resid.dtype == torch.float64 and resid.is_contiguous()
        assert lhs.is_cuda and lhs.dtype == torch.float64 and lhs.is_contiguous()
        B = resid.shape[0]
        assert tuple(lhs.shape) == (B, order, cfg.samples, 4)
        desc = make_lem_desc(cfg)
        _check(load().act_lem_decompose_noalloc(
            self._h, ctypes.byref(desc), B, _ptr(lhs), _ptr(resid), _ptr(out["approx"]), int(order),
            _ptr(out["theta"]), _ptr(out["coef"]), _ptr(out["energy"]), _ptr(out["flags"]), _stream()))
        return out

    def lem_decompose(self, signals, lhs, cfg, order: int) -> dict:
        resid = _device_tensor(signals, torch.float64).reshape(-1, self.grid.n).clone()
        lhs = _device_tensor(lhs, torch.float64).contiguous()
        out = self.alloc_outputs(resid.shape[0], order)
        self.act_lem_decompose(resid, lhs, cfg, order, out)
        out["resid"] = resid
        return out

    def decompose_ragged(self, packed, lengths, offsets, order: int) -> dict:
        resid = _device_tensor(packed, torch.float64).reshape(-1).clone()
        lengths = _device_tensor(lengths, torch.int32)
        offsets = _device_tensor(offsets, torch.int64)
        B = lengths.shape[0]
        out = self.alloc_outputs(B, order, approx=False)
        out["approx"] = torch.empty_like(resid)
        self.act_decompose_ragged(resid, lengths, offsets, order, out)
        out["resid"] = resid
        return out

    def act_reconstruct_ragged(self, theta, coef, lengths, offsets, total: int) -> torch.Tensor:
        theta = _device_tensor(theta, torch.float64)
        coef = _device_tensor(coef, torch.float64)
        lengths = _device_tensor(lengths, torch.int32)
        offsets = _device_tensor(offsets, torch.int64)
        B, order = coef.shape
        out = torch.zeros(total, dtype=torch.float64, device=coef.device)
        _check(load().act_reconstruct(self._h, B, order, _ptr(theta), _ptr(coef), _ptr(lengths),
                                      _ptr(offsets), _ptr(out), _stream()))
        return out

    def act_refine(self, resid, theta0, steps: int):
        """Refinement of every row: act_refine for an FP64 residual (numpy
        arrays are taken as FP64), act_refine_f32 for an FP32 CUDA tensor."""
        f32 = isinstance(resid, torch.Tensor) and resid.dtype == torch.float32
        resid = _device_tensor(resid, torch.float32 if f32 else torch.float64).reshape(-1, self.grid.n)
        theta0 = _device_tensor(theta0, torch.float64).reshape(-1, 4)
        m = resid.shape[0]
        theta = torch.empty(m, 4, dtype=torch.float64, device=resid.device)
        value = torch.empty(m, dtype=torch.float64, device=resid.device)
        flags = torch.empty(m, dtype=torch.int32, device=resid.device)
        fn = load().act_refine_f32 if f32 else load().act_refine
        _check(fn(self._h, m, _ptr(resid), _ptr(theta0), int(steps), _ptr(theta), _ptr(value), _ptr(flags),
                  _stream()))
        return theta, value, flags

    def act_value_and_grad(self, resid: torch.Tensor, theta: torch.Tensor, want_dr: bool = True):
        """J, dJ/dtheta, dJ/dr for each row; resid is f64 or f32 [m, N]."""
        assert resid.is_cuda and resid.is_contiguous() and resid.dtype in (torch.float64, torch.float32)
        theta = _device_tensor(theta, torch.float64).reshape(-1, 4)
        m = resid.shape[0]
        dtype = ACT_PREC_F64 if resid.dtype == torch.float64 else ACT_PREC_F32
        value = torch.empty(m, dtype=torch.float64, device=resid.device)
        dtheta = torch.empty(m, 4, dtype=torch.float64, device=resid.device)
        dr = torch.empty_like(resid) if want_dr else None
        _check(load().act_value_and_grad(self._h, m, dtype, _ptr(resid), _ptr(theta), _ptr(value),
                                         _ptr(dtheta), _ptr(dr), _stream()))
        return value, dtheta, dr

    def act_reconstruct(self, theta, coef) -> torch.Tensor:
        theta = _device_tensor(theta, torch.float64)
        coef = _device_tensor(coef, torch.float64)
        B, order = coef.shape[:2]
        assert coef.dim() == (3 if self.complex_atoms else 2)
        out = torch.empty(B, self.grid.n, dtype=torch.float64, device=coef.device)
        _check(load().act_reconstruct(self._h, B, order, _ptr(theta), _ptr(coef), None, None,
                                      _ptr(out), _stream()))
        return out

    def act_tune(self, resid, reps: int = 3, cache: Optional[str] = None, lengths=None, offsets=None) -> dict:
        """Times the search's launch shapes on `resid` (plain: [B, N] f64; ragged:
        the packed signals with lengths/offsets) and keeps the fastest for this
        batch size; `cache` is an optional text file of earlier choices."""
        if self.ragged:
            resid = _device_tensor(resid, torch.float64).reshape(-1)
            lengths = _device_tensor(lengths, torch.int32)
            offsets = _device_tensor(offsets, torch.int64)
            B, lp, op = lengths.shape[0], _ptr(lengths), _ptr(offsets)
        else:
            resid = _device_tensor(resid, torch.float64).reshape(-1, self.grid.n)
            B, lp, op = resid.shape[0], None, None
        shape = _LaunchShape()
        _check(load().act_tune(self._h, B, lp, op, _ptr(resid), int(reps),
                               cache.encode() if cache else None, ctypes.byref(shape), _stream()))
        return {"grid_per_cu": shape.grid_per_cu, "chan_per_fc": shape.chan_per_fc, "form": shape.form,
                "from_cache": bool(shape.from_cache), "ms": shape.ms}

    def act_set_launch_shape(self, batch: int, grid_per_cu: int = 1, chan_per_fc: int = 0, form: int = 0):
        """Applies a search launch shape to later calls with `batch` channels."""
        shape = _LaunchShape(grid_per_cu=grid_per_cu, chan_per_fc=chan_per_fc, form=form)
        _check(load().act_set_launch_shape(self._h, int(batch), ctypes.byref(shape)))

    def act_correlate(self, resid, begin: int, count: int) -> torch.Tensor:
        resid = _device_tensor(resid, torch.float64).reshape(-1, self.grid.n)
        B = resid.shape[0]
        out = torch.empty(B, count, dtype=torch.float64, device=resid.device)
        _check(load().act_correlate(self._h, B, _ptr(resid), int(begin), int(count), _ptr(out),
                                    _stream()))
        return out


def act_plan(grid: Grid, **kw) -> Plan:
    return Plan(grid, **kw)


class ChirpletObjective(torch.autograd.Function):
    """J(theta; r) = <r, g(theta)>^2 / <g, g> per row, with the hand-written
    forward and adjoint kernels (act_value_and_grad) as forward and backward."""

    @staticmethod
    def forward(ctx, resid: torch.Tensor, theta: torch.Tensor, plan: Plan):
        value, dtheta, dr = plan.act_value_and_grad(resid.contiguous(), theta.detach(),
                                                    want_dr=resid.requires_grad)
        ctx.save_for_backward(dtheta, dr if dr is not None else torch.empty(0, device=resid.device))
        ctx.has_dr = dr is not None
        return value.to(theta.dtype)

    @staticmethod
    def backward(ctx, grad_out: torch.Tensor):
        dtheta, dr = ctx.saved_tensors
        g = grad_out.to(torch.float64)
        d_theta = (g[:, None] * dtheta).to(grad_out.dtype)
        d_resid = (g[:, None].to(dr.dtype) * dr) if ctx.has_dr else None
        return d_resid, d_theta, None


def chirplet_objective(resid: torch.Tensor, theta: torch.Tensor, plan: Plan) -> torch.Tensor:
    return ChirpletObjective.apply(resid, theta, plan)
