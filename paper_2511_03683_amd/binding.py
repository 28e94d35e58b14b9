"""ctypes binding of libephbte.so (include/ephbte.h).

Argument marshalling only: every function below checks tensor placement and
shapes, converts them to device pointers and the caller's current HIP stream,
and calls the C entry point of the same name.  There is no fallback: if the
HIP library is missing or a tensor is not on the plan's GPU, an exception is
raised.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libephbte.so")

OK, INVALID_ARGUMENT, UNSUPPORTED_DTYPE, OUT_OF_MEMORY = 0, 1, 2, 3
HIP_ERROR, NOT_CONVERGED, NONFINITE, PLAN_MISMATCH = 4, 5, 6, 7
F32, F64 = 1, 2

_P = ctypes.c_void_p


class EphbteError(RuntimeError):
    def __init__(self, status: int, where: str, detail: str):
        self.status = status
        super().__init__(f"{where}: {status_string(status)} ({status}): {detail}")


class Problem(ctypes.Structure):
    _fields_ = [("n_states", ctypes.c_int32), ("state_k", _P), ("state_band", _P), ("eps", _P),
                ("kgrid", ctypes.c_int32 * 3), ("qgrid", ctypes.c_int32 * 3),
                ("n_modes", ctypes.c_int32), ("hw", _P), ("n_channels", ctypes.c_int64),
                ("ch_i", _P), ("ch_j", _P), ("ch_nu", _P), ("g2", _P),
                ("sigma", ctypes.c_double), ("n_q_norm", ctypes.c_double),
                ("dtype", ctypes.c_int32), ("device", ctypes.c_int32)]


class BuildOpts(ctypes.Structure):
    _fields_ = [("energy_nsigma", ctypes.c_double), ("g2_min", ctypes.c_double),
                ("elastic_modes", ctypes.c_uint32), ("statistics", ctypes.c_int32),
                ("reserved", ctypes.c_int32 * 2)]


class Tuning(ctypes.Structure):
    _fields_ = [("chunk_entries", ctypes.c_int32), ("block_threads", ctypes.c_int32),
                ("xcd_map", ctypes.c_int32), ("batch_partners", ctypes.c_int32),
                ("tile_entries", ctypes.c_int32), ("layout", ctypes.c_int32),
                ("fp64_exp", ctypes.c_int32), ("table_order", ctypes.c_int32),
                ("pair_window", ctypes.c_int32), ("pair_threads", ctypes.c_int32),
                ("pair_order", ctypes.c_int32), ("pair_rows", ctypes.c_int32)]


_LIB = None

SYMBOLS = {
    "ephbte_build_channels": ([ctypes.POINTER(Problem), ctypes.POINTER(BuildOpts),
                               ctypes.POINTER(_P)], ctypes.c_int32),
    "ephbte_layout_host": ([ctypes.POINTER(Problem), ctypes.POINTER(BuildOpts), _P, _P, _P, _P],
                           ctypes.c_int32),
    "ephbte_collision_integral": ([_P, ctypes.c_int32, _P, ctypes.c_int64, _P, ctypes.c_int32,
                                   _P, ctypes.c_int64, _P], ctypes.c_int32),
    "ephbte_collision_integral_noalloc": ([_P, _P, _P, _P, _P], ctypes.c_int32),
    "ephbte_collision_vjp": ([_P, ctypes.c_int32, _P, ctypes.c_int64, _P, ctypes.c_int32, _P,
                              ctypes.c_int64, _P, ctypes.c_int64, _P, ctypes.c_int32, _P],
                             ctypes.c_int32),
    "ephbte_rt_step": ([_P, ctypes.c_int32, _P, ctypes.c_int64, _P, ctypes.c_double,
                        ctypes.c_int32, ctypes.c_int32, _P], ctypes.c_int32),
    "ephbte_rt_adjoint": ([_P, _P, _P, ctypes.c_double, ctypes.c_int32, ctypes.c_int32, _P, _P,
                           _P, ctypes.c_int32, _P], ctypes.c_int32),
    "ephbte_iterate_transport": ([_P, _P, _P, ctypes.c_double, _P, ctypes.c_double,
                                  ctypes.c_int32, _P, _P, _P, _P, _P], ctypes.c_int32),
    "ephbte_update_g2": ([_P, _P, _P], ctypes.c_int32),
    "ephbte_set_tuning": ([_P, ctypes.POINTER(Tuning)], ctypes.c_int32),
    "ephbte_autotune": ([_P, ctypes.c_int32, ctypes.POINTER(Tuning), ctypes.c_char_p], ctypes.c_int32),
    "ephbte_plan_info": ([_P, _P], ctypes.c_int32),
    "ephbte_kernel_timing": ([_P, ctypes.c_int32, ctypes.POINTER(ctypes.c_double),
                              ctypes.POINTER(ctypes.c_int64)], ctypes.c_int32),
    "ephbte_set_field": ([_P, _P], ctypes.c_int32),
    "ephbte_phonon_rate": ([_P, _P, _P, _P, _P], ctypes.c_int32),
    "ephbte_rt_step_coupled": ([_P, _P, _P, ctypes.c_double, ctypes.c_int32, _P], ctypes.c_int32),
    "ephbte_phonon_rate_vjp": ([_P, _P, _P, _P, _P, _P, _P, ctypes.c_int32, _P], ctypes.c_int32),
    "ephbte_collision_vjp_nph": ([_P, _P, _P, _P, _P, _P], ctypes.c_int32),
    "ephbte_rt_adjoint_coupled": ([_P, _P, _P, ctypes.c_double, ctypes.c_int32, ctypes.c_int32, _P, _P, _P,
                                   _P, _P, ctypes.c_int32, _P], ctypes.c_int32),
    "ephbte_plan_bytes": ([_P], ctypes.c_int64),
    "ephbte_destroy": ([_P], None),
    "ephbte_status_string": ([ctypes.c_int32], ctypes.c_char_p),
    "ephbte_last_error": ([], ctypes.c_char_p),
}


def load_library(path: Optional[str] = None):
    """Load libephbte.so (built by build_lib.py); raises if it is missing."""
    global _LIB
    if _LIB is not None:
        return _LIB
    path = path or LIB_PATH
    # torch ships its own HIP runtime with the same soname as /opt/rocm's;
    # importing it first makes this library bind to that one runtime instead
    # of bringing a second copy into the process.
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    if not os.path.exists(path):
        raise ImportError(f"{path} is missing: build the HIP library first "
                          "(python -m paper_2511_03683_amd.build_lib)")
    lib = ctypes.CDLL(path)
    for name, (args, res) in SYMBOLS.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = res
    _LIB = lib
    return lib


def status_string(status: int) -> str:
    return load_library().ephbte_status_string(int(status)).decode()


def last_error() -> str:
    return load_library().ephbte_last_error().decode()


def _check(status: int, where: str, allow=()):
    if status != OK and status not in allow:
        raise EphbteError(status, where, last_error())
    return status


# ---------------------------------------------------------------- helpers
def _np(a, dtype):
    return np.ascontiguousarray(a, dtype=dtype)


def _problem(system, dtype: int, device: int):
    """ctypes Problem plus the numpy arrays it points into (kept alive)."""
    keep = dict(state_k=_np(system.state_k, np.int32), state_band=_np(system.state_band, np.int8),
                eps=_np(system.eps, np.float64),
                hw=_np(system.hw, np.float64), ch_i=_np(system.ch_i, np.int32),
                ch_j=_np(system.ch_j, np.int32), ch_nu=_np(system.ch_nu, np.int8),
                g2=_np(system.g2, np.float64))
    pr = Problem()
    pr.n_states = int(keep["eps"].size)
    pr.state_k = keep["state_k"].ctypes.data
    pr.state_band = keep["state_band"].ctypes.data
    pr.eps = keep["eps"].ctypes.data
    pr.kgrid[:] = [int(x) for x in system.kgrid]
    pr.qgrid[:] = [int(x) for x in system.qgrid]
    pr.n_modes = int(system.n_modes)
    pr.hw = keep["hw"].ctypes.data
    pr.n_channels = int(keep["g2"].size)
    pr.ch_i = keep["ch_i"].ctypes.data
    pr.ch_j = keep["ch_j"].ctypes.data
    pr.ch_nu = keep["ch_nu"].ctypes.data
    pr.g2 = keep["g2"].ctypes.data
    pr.sigma = float(system.sigma)
    pr.n_q_norm = float(system.n_q_norm)
    pr.dtype = int(dtype)
    pr.device = int(device)
    return pr, keep


def _dtype_code(dtype) -> int:
    if dtype in (F32, "f32", "float32", np.float32):
        return F32
    if dtype in (F64, "f64", "float64", np.float64):
        return F64
    try:
        import torch
        if dtype == torch.float32:
            return F32
        if dtype == torch.float64:
            return F64
    except ImportError:
        pass
    raise ValueError(f"unsupported dtype {dtype!r}")


class Plan:
    """Owns an ephbte_plan handle (device channel layout)."""

    def __init__(self, handle, system, dtype: int, device: int):
        self.handle = ctypes.c_void_p(handle)
        self.n_states = int(system.n_states)
        self.n_channels = int(system.n_channels)
        self.n_modes = int(system.n_modes)
        self.n_q = int(np.prod(system.qgrid))
        self.dtype = dtype
        self.device = device
        self.statistics = "fermi"

    @property
    def torch_dtype(self):
        import torch
        return torch.float64 if self.dtype == F64 else torch.float32

    def close(self):
        if self.handle is not None and self.handle.value:
            load_library().ephbte_destroy(self.handle)
        self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _stream(device):
    import torch
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


def _dev_tensor(plan: Plan, t, name, shape_last=None, dtype=None):
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a CUDA (HIP) tensor")
    if t.device.index != plan.device:
        raise ValueError(f"{name} is on {t.device}, the plan is on cuda:{plan.device}")
    want = dtype or plan.torch_dtype
    if t.dtype != want:
        raise TypeError(f"{name} must be {want}, got {t.dtype}")
    if shape_last is not None and t.shape[-1] != shape_last:
        raise ValueError(f"{name} must have last dimension {shape_last}, got {tuple(t.shape)}")
    if t.stride(-1) != 1:
        raise ValueError(f"{name} must have unit stride in its last dimension")
    return t


def _batch(plan, t, name):
    """(B, ld) of a [S] or [B, S] tensor with unit inner stride."""
    _dev_tensor(plan, t, name, shape_last=plan.n_states)
    if t.dim() == 1:
        return 1, plan.n_states
    if t.dim() == 2:
        return int(t.shape[0]), int(t.stride(0)) if t.shape[0] > 1 else plan.n_states
    raise ValueError(f"{name} must be [S] or [B, S]")


# ---------------------------------------------------------------- entry points
STATISTICS = {"fermi": 0, "bose": 1}


def _opts(energy_nsigma: float, g2_min: float, elastic_modes: int = 0, statistics: str = "fermi"):
    """BuildOpts pointer, or None (defaults) when every option is 0."""
    if statistics not in STATISTICS:
        raise ValueError("statistics must be 'fermi' or 'bose'")
    if not energy_nsigma and not g2_min and not elastic_modes and statistics == "fermi":
        return None
    o = BuildOpts()
    o.energy_nsigma = float(energy_nsigma)
    o.g2_min = float(g2_min)
    o.elastic_modes = int(elastic_modes)
    o.statistics = STATISTICS[statistics]
    return ctypes.byref(o)


def build_channels(system, dtype="f64", device: Optional[int] = None,
                   energy_nsigma: float = 0.0, g2_min: float = 0.0, elastic_modes: int = 0,
                   statistics: str = "fermi") -> Plan:
    """Build the device channel layout of a problem (see ephbte_build_channels).
    energy_nsigma > 0 and g2_min > 0 select channels; elastic_modes is the bit
    mask of elastic (hw = 0, N = 0) mechanisms; statistics "bose" makes the
    states phonon modes with occupations n (blocking factors 1 + n: phonon-phonon
    scattering; ephbte_build_opts)."""
    lib = load_library()
    code = _dtype_code(dtype)
    if device is None:
        import torch
        device = torch.cuda.current_device()
    pr, keep = _problem(system, code, device)
    h = ctypes.c_void_p()
    _check(lib.ephbte_build_channels(ctypes.byref(pr), _opts(energy_nsigma, g2_min, elastic_modes, statistics),
                                     ctypes.byref(h)), "build_channels")
    del keep
    plan = Plan(h.value, system, code, device)
    plan.statistics = statistics
    return plan


def layout_host(system, energy_nsigma: float = 0.0, g2_min: float = 0.0, elastic_modes: int = 0):
    """Host-only layout view: (row_ptr, partner, mode, channel) numpy arrays
    over the channels the selection keeps."""
    lib = load_library()
    pr, keep = _problem(system, F64, -1)
    S, E = int(system.n_states), 2 * int(system.n_channels)
    row_ptr = np.zeros(S + 1, np.int64)
    partner = np.zeros(E, np.int32)
    mode = np.zeros(E, np.int8)
    chan = np.zeros(E, np.int32)
    _check(lib.ephbte_layout_host(ctypes.byref(pr), _opts(energy_nsigma, g2_min, elastic_modes),
                                  row_ptr.ctypes.data, partner.ctypes.data, mode.ctypes.data,
                                  chan.ctypes.data), "layout_host")
    del keep
    n = int(row_ptr[S])
    return row_ptr, partner[:n], mode[:n], chan[:n]


def _nph_arg(plan: Plan, nph, B: int, f):
    """1 when nph holds one table per vector ([B, Nq, n_modes]), 0 when one
    [Nq, n_modes] table serves the whole batch."""
    _dev_tensor(plan, nph, "nph")
    if not nph.is_contiguous():
        raise ValueError("nph must be contiguous")
    tab = plan.n_q * plan.n_modes
    if nph.dim() == 3 and f.dim() == 2:
        if nph.shape[0] != B or nph.numel() != B * tab:
            raise ValueError("a per-vector nph must be [B, Nq, n_modes]")
        return 1
    if nph.numel() != tab:
        raise ValueError("nph must be a [Nq, n_modes] tensor (or [B, Nq, n_modes] with f [B, S])")
    return 0


def collision_integral(plan: Plan, f, nph, out=None):
    """I[f] for f [S] or [B, S]; nph [Nq, n_modes], or [B, Nq, n_modes] for a
    bath per vector (device tensors)."""
    import torch
    B, ldf = _batch(plan, f, "f")
    per_batch = _nph_arg(plan, nph, B, f)
    if out is None:
        out = torch.empty((B, plan.n_states) if f.dim() == 2 else (plan.n_states,),
                          dtype=plan.torch_dtype, device=f.device)
    Bo, ldi = _batch(plan, out, "out")
    if Bo != B:
        raise ValueError("out batch differs from f batch")
    _check(load_library().ephbte_collision_integral(plan.handle, B, f.data_ptr(), ldf,
                                                    nph.data_ptr(), per_batch, out.data_ptr(),
                                                    ldi, _stream(f.device)), "collision_integral")
    return out


def collision_integral_noalloc(plan: Plan, f, nph, out):
    """I[f] for one vector f [S] into out [S] through the allocation-free entry
    point (its workspaces sit in the library's static device scratch)."""
    B, _ = _batch(plan, f, "f")
    Bo, _ = _batch(plan, out, "out")
    if B != 1 or Bo != 1 or f.dim() != 1 or out.dim() != 1:
        raise ValueError("the allocation-free pass takes one vector f [S] and out [S]")
    if _nph_arg(plan, nph, 1, f) != 0:
        raise ValueError("the allocation-free pass takes one shared bath nph [Nq, n_modes]")
    _check(load_library().ephbte_collision_integral_noalloc(
        plan.handle, f.data_ptr(), nph.data_ptr(), out.data_ptr(), _stream(f.device)),
        "collision_integral_noalloc")
    return out


def collision_vjp(plan: Plan, f, nph, gI, want_f=True, gg2=None, accumulate=False):
    """(dL/df, dL/d|g|^2) given gI = dL/dI.  gg2 (FP64 [n_channels]) is
    allocated when None and want_g2 is implied by passing gg2=True."""
    import torch
    B, ldf = _batch(plan, f, "f")
    Bg, ldg = _batch(plan, gI, "gI")
    if Bg != B:
        raise ValueError("gI batch differs from f batch")
    per_batch = _nph_arg(plan, nph, B, f)
    gf = None
    if want_f:
        gf = torch.empty_like(f, memory_format=torch.contiguous_format)
    if gg2 is True:
        gg2 = torch.zeros(plan.n_channels, dtype=torch.float64, device=f.device)
    if gg2 is not None:
        _dev_tensor(plan, gg2, "gg2", dtype=torch.float64)
        if gg2.numel() != plan.n_channels or not gg2.is_contiguous():
            raise ValueError("gg2 must be a contiguous FP64 [n_channels] tensor")
    ldgf = plan.n_states
    _check(load_library().ephbte_collision_vjp(
        plan.handle, B, f.data_ptr(), ldf, nph.data_ptr(), per_batch, gI.data_ptr(), ldg,
        gf.data_ptr() if gf is not None else None, ldgf,
        gg2.data_ptr() if gg2 is not None else None, 1 if accumulate else 0,
        _stream(f.device)), "collision_vjp")
    return gf, gg2


def rt_step(plan: Plan, f, nph, dt_fs: float, n_steps: int, use_graph: bool = False):
    """Advance f ([S] or [B, S], in place) by n_steps RK4 steps."""
    B, ldf = _batch(plan, f, "f")
    _dev_tensor(plan, nph, "nph")
    _check(load_library().ephbte_rt_step(plan.handle, B, f.data_ptr(), ldf, nph.data_ptr(),
                                         float(dt_fs), int(n_steps), 1 if use_graph else 0,
                                         _stream(f.device)), "rt_step")
    return f


def rt_adjoint(plan: Plan, f0, nph, dt_fs: float, n_steps: int, checkpoint_every: int, gfT,
               want_f=True, gg2=None, accumulate=False):
    """(dL/df0, dL/d|g|^2) through n_steps RK4 steps from f0 given dL/df(T)."""
    import torch
    _dev_tensor(plan, f0, "f0", shape_last=plan.n_states)
    _dev_tensor(plan, gfT, "gfT", shape_last=plan.n_states)
    if f0.dim() != 1 or gfT.dim() != 1:
        raise ValueError("rt_adjoint takes one vector (B = 1)")
    gf0 = torch.empty_like(f0) if want_f else None
    if gg2 is True:
        gg2 = torch.zeros(plan.n_channels, dtype=torch.float64, device=f0.device)
    if gg2 is not None:
        _dev_tensor(plan, gg2, "gg2", dtype=torch.float64)
    _check(load_library().ephbte_rt_adjoint(
        plan.handle, f0.data_ptr(), nph.data_ptr(), float(dt_fs), int(n_steps),
        int(checkpoint_every), gfT.data_ptr(), gf0.data_ptr() if gf0 is not None else None,
        gg2.data_ptr() if gg2 is not None else None, 1 if accumulate else 0,
        _stream(f0.device)), "rt_adjoint")
    return gf0, gg2


def iterate_transport(plan: Plan, f0, vel, T_K: float, nph, tol: float = 1e-8,
                      max_iter: int = 100, want_x: bool = False, raise_on_nonconv=False):
    """Mobility (cm^2/Vs, 3x3) of the linearised BTE; see ephbte_iterate_transport."""
    import torch
    _dev_tensor(plan, f0, "f0", shape_last=plan.n_states)
    _dev_tensor(plan, vel, "vel", shape_last=3)
    if vel.shape[0] != plan.n_states or not vel.is_contiguous():
        raise ValueError("vel must be a contiguous [S, 3] tensor")
    x = torch.empty((plan.n_states, 3), dtype=plan.torch_dtype, device=f0.device) if want_x else None
    mob = np.zeros(9)
    iters = ctypes.c_int32(0)
    resid = ctypes.c_double(0.0)
    st = load_library().ephbte_iterate_transport(
        plan.handle, f0.data_ptr(), vel.data_ptr(), float(T_K), nph.data_ptr(), float(tol),
        int(max_iter), x.data_ptr() if x is not None else None, mob.ctypes.data,
        ctypes.byref(iters), ctypes.byref(resid), _stream(f0.device))
    _check(st, "iterate_transport", allow=() if raise_on_nonconv else (NOT_CONVERGED,))
    stagnated = st == NOT_CONVERGED and "stagnated" in last_error()
    return dict(mu=mob.reshape(3, 3), iters=int(iters.value), resid=float(resid.value),
                converged=(st == OK), stagnated=stagnated, x=x)


def update_g2(plan: Plan, g2):
    """Replace every channel's |g|^2 (FP64 device tensor in caller order)."""
    import torch
    _dev_tensor(plan, g2, "g2", dtype=torch.float64)
    if g2.numel() != plan.n_channels or not g2.is_contiguous():
        raise ValueError("g2 must be a contiguous FP64 [n_channels] tensor")
    _check(load_library().ephbte_update_g2(plan.handle, g2.data_ptr(), _stream(g2.device)),
           "update_g2")


def set_tuning(plan: Plan, chunk_entries=0, block_threads=0, xcd_map=0, batch_partners=0,
               tile_entries=0, layout=0, fp64_exp=0, table_order=0, pair_window=0, pair_threads=0,
               pair_order=0, pair_rows=0):
    """Knobs left at 0 keep the plan's value; tile_entries=-1 restores its default;
    layout 1 = duplicated rows, 2 = single copy over entries, 3 = single copy
    over pair records (B = 1 forward pass); fp64_exp 1 = table, 2 = polynomial;
    table_order 1 = the modes of one q adjacent, 2 = one block per mode;
    pair_window / pair_threads: LDS window (states) and workgroup size of the
    pair-record passes; pair_order 1 = the records of their LDS tiles sorted by
    q (in groups of pair_rows table rows, a power of 2), 2 = by destination."""
    t = Tuning()
    t.chunk_entries, t.block_threads, t.xcd_map = int(chunk_entries), int(block_threads), int(xcd_map)
    t.batch_partners, t.tile_entries, t.layout = int(batch_partners), int(tile_entries), int(layout)
    t.fp64_exp, t.table_order = int(fp64_exp), int(table_order)
    t.pair_window, t.pair_threads = int(pair_window), int(pair_threads)
    t.pair_order, t.pair_rows = int(pair_order), int(pair_rows)
    _check(load_library().ephbte_set_tuning(plan.handle, ctypes.byref(t)), "set_tuning")


def autotune(plan: Plan, batch: int = 1, cache_path: Optional[str] = None) -> dict:
    """Time and apply the fastest tuning (see ephbte_autotune); with cache_path
    a tuning stored for this plan's key is applied without timing."""
    t = Tuning()
    path = None if cache_path is None else os.fsencode(cache_path)
    _check(load_library().ephbte_autotune(plan.handle, int(batch), ctypes.byref(t), path), "autotune")
    return dict(chunk_entries=t.chunk_entries, block_threads=t.block_threads, xcd_map=t.xcd_map,
                batch_partners=t.batch_partners, tile_entries=t.tile_entries)


def phonon_rate(plan: Plan, f, nph, out=None):
    """dN/dt [Nq, n_modes] of the phonons from the channel list for f [S]."""
    import torch
    B, _ = _batch(plan, f, "f")
    if f.dim() != 1:
        raise ValueError("phonon_rate takes one occupation vector f [S]")
    _dev_tensor(plan, nph, "nph")
    if nph.numel() != plan.n_q * plan.n_modes or not nph.is_contiguous():
        raise ValueError("nph must be a contiguous [Nq, n_modes] tensor")
    if out is None:
        out = torch.empty((plan.n_q, plan.n_modes), dtype=plan.torch_dtype, device=f.device)
    _dev_tensor(plan, out, "out")
    if out.numel() != plan.n_q * plan.n_modes or not out.is_contiguous():
        raise ValueError("out must be a contiguous [Nq, n_modes] tensor")
    _check(load_library().ephbte_phonon_rate(plan.handle, f.data_ptr(), nph.data_ptr(),
                                             out.data_ptr(), _stream(f.device)), "phonon_rate")
    return out


def rt_step_coupled(plan: Plan, f, nph, dt_fs: float, n_steps: int):
    """Advance f [S] and nph [Nq, n_modes] (in place) together by n_steps
    coupled RK4 steps (see ephbte_rt_step_coupled)."""
    B, _ = _batch(plan, f, "f")
    if f.dim() != 1 or not f.is_contiguous():
        raise ValueError("rt_step_coupled takes one contiguous occupation vector f [S]")
    _dev_tensor(plan, nph, "nph")
    if nph.numel() != plan.n_q * plan.n_modes or not nph.is_contiguous():
        raise ValueError("nph must be a contiguous [Nq, n_modes] tensor")
    _check(load_library().ephbte_rt_step_coupled(plan.handle, f.data_ptr(), nph.data_ptr(), float(dt_fs),
                                                 int(n_steps), _stream(f.device)), "rt_step_coupled")
    return f, nph


def _bins(plan: Plan, t, name):
    _dev_tensor(plan, t, name)
    if t.numel() != plan.n_q * plan.n_modes or not t.is_contiguous():
        raise ValueError(f"{name} must be a contiguous [Nq, n_modes] tensor")


def _vec1(plan: Plan, t, name):
    B, _ = _batch(plan, t, name)
    if t.dim() != 1 or not t.is_contiguous():
        raise ValueError(f"{name} must be one contiguous vector [S]")


def collision_vjp_nph(plan: Plan, f, nph, gI, out=None):
    """dL/dN [Nq, n_modes] of L = gI . I[f, N] (see ephbte_collision_vjp_nph)."""
    import torch
    _vec1(plan, f, "f")
    _vec1(plan, gI, "gI")
    _bins(plan, nph, "nph")
    if out is None:
        out = torch.empty((plan.n_q, plan.n_modes), dtype=plan.torch_dtype, device=f.device)
    _bins(plan, out, "out")
    _check(load_library().ephbte_collision_vjp_nph(plan.handle, f.data_ptr(), nph.data_ptr(), gI.data_ptr(),
                                                   out.data_ptr(), _stream(f.device)), "collision_vjp_nph")
    return out


def phonon_rate_vjp(plan: Plan, f, nph, gR, want_f=True, want_nph=True, gg2=None, accumulate=False):
    """(dL/df, dL/dN, dL/d|g|^2) of L = gR . dN/dt (see ephbte_phonon_rate_vjp);
    gg2=True allocates the FP64 [n_channels] gradient."""
    import torch
    _vec1(plan, f, "f")
    _bins(plan, nph, "nph")
    _bins(plan, gR, "gR")
    gf = torch.empty_like(f) if want_f else None
    gN = torch.empty_like(nph) if want_nph else None
    if gg2 is True:
        gg2 = torch.zeros(plan.n_channels, dtype=torch.float64, device=f.device)
    if gg2 is not None:
        _dev_tensor(plan, gg2, "gg2", dtype=torch.float64)
        if gg2.numel() != plan.n_channels or not gg2.is_contiguous():
            raise ValueError("gg2 must be a contiguous FP64 [n_channels] tensor")
    _check(load_library().ephbte_phonon_rate_vjp(
        plan.handle, f.data_ptr(), nph.data_ptr(), gR.data_ptr(),
        gf.data_ptr() if gf is not None else None, gN.data_ptr() if gN is not None else None,
        gg2.data_ptr() if gg2 is not None else None, 1 if accumulate else 0, _stream(f.device)),
        "phonon_rate_vjp")
    return gf, gN, gg2


def rt_adjoint_coupled(plan: Plan, f0, nph0, dt_fs: float, n_steps: int, checkpoint_every: int,
                       gfT=None, gNT=None, want_f=True, want_nph=True, gg2=None, accumulate=False):
    """(dL/df0, dL/dnph0, dL/d|g|^2) through n_steps coupled RK4 steps for a loss
    with gradients gfT [S] and gNT [Nq, n_modes] at the end (see
    ephbte_rt_adjoint_coupled)."""
    import torch
    _vec1(plan, f0, "f0")
    _bins(plan, nph0, "nph0")
    if gfT is not None:
        _vec1(plan, gfT, "gfT")
    if gNT is not None:
        _bins(plan, gNT, "gNT")
    gf = torch.empty_like(f0) if want_f else None
    gN = torch.empty_like(nph0) if want_nph else None
    if gg2 is True:
        gg2 = torch.zeros(plan.n_channels, dtype=torch.float64, device=f0.device)
    if gg2 is not None:
        _dev_tensor(plan, gg2, "gg2", dtype=torch.float64)
        if gg2.numel() != plan.n_channels or not gg2.is_contiguous():
            raise ValueError("gg2 must be a contiguous FP64 [n_channels] tensor")
    _check(load_library().ephbte_rt_adjoint_coupled(
        plan.handle, f0.data_ptr(), nph0.data_ptr(), float(dt_fs), int(n_steps), int(checkpoint_every),
        gfT.data_ptr() if gfT is not None else None, gNT.data_ptr() if gNT is not None else None,
        gf.data_ptr() if gf is not None else None, gN.data_ptr() if gN is not None else None,
        gg2.data_ptr() if gg2 is not None else None, 1 if accumulate else 0, _stream(f0.device)),
        "rt_adjoint_coupled")
    return gf, gN, gg2


def set_field(plan: Plan, rates) -> None:
    """Field term of rt_step / rt_adjoint: rates[a] = F_a / (hbar dk_a) in 1/fs
    (see ephbte_set_field); (0, 0, 0) switches it off."""
    r = np.ascontiguousarray(rates, dtype=np.float64)
    if r.shape != (3,):
        raise ValueError("rates must hold 3 values")
    _check(load_library().ephbte_set_field(plan.handle, r.ctypes.data), "set_field")


def kernel_timing(plan: Plan, start: bool):
    """Launch timing of the forward pass's main kernel (see
    ephbte_kernel_timing): start=True clears and starts it; start=False stops
    it and returns (mean_ms, launches) of the eager launches since the start."""
    mean = ctypes.c_double(0.0)
    n = ctypes.c_int64(0)
    _check(load_library().ephbte_kernel_timing(plan.handle, 1 if start else 0, ctypes.byref(mean),
                                               ctypes.byref(n)), "kernel_timing")
    return None if start else (float(mean.value), int(n.value))


def plan_info(plan: Plan) -> dict:
    out = np.zeros(12, np.int64)
    _check(load_library().ephbte_plan_info(plan.handle, out.ctypes.data), "plan_info")
    keys = ["n_states", "n_channels", "entries", "chunks", "dtype", "device", "bytes",
            "chunk_entries", "block_threads", "channels_kept", "layout", "pair_records"]
    return {k: int(v) for k, v in zip(keys, out)}


def plan_bytes(plan: Plan) -> int:
    return int(load_library().ephbte_plan_bytes(plan.handle))


def destroy(plan: Plan) -> None:
    plan.close()
