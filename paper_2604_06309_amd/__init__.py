"""Python binding of libdmfe, the MI355X-native DMFE solver (DYNAMITE, arXiv 2604.06309).

Argument marshalling only: every array operation runs in the HIP kernels of
``libdmfe.so``; PyTorch is used for device memory and streams.  The functions
``dmfe_*`` mirror the C-ABI of ``include/dmfe.h`` one to one; ``Solver`` is a
small convenience wrapper around a handle.

Importing this module does not need a GPU; creating a solver does.  If the
library has not been built, every call raises ``RuntimeError`` (there is no
fallback path).
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libdmfe.so")

MAX_TERMS = 8
MAX_P = 16

OK, DONE = 0, 1
ERR_INVALID, ERR_NOMEM, ERR_CAPACITY, ERR_STEP_UNDERFLOW = -1, -2, -3, -4
ERR_NONFINITE, ERR_DEVICE, ERR_UNSUPPORTED, ERR_BUFFER = -5, -6, -7, -8
UNIFORM, ADAPTIVE = 0, 1
FP64, FP32_COMP = 0, 1
# theta-interpolation schemes (DMFE_INTERP_*)
INTERP_INDEX_LAGRANGE, INTERP_THETA_LAGRANGE, INTERP_INDEX_FH, INTERP_THETA_FH = 0, 1, 2, 3
SCHEME_DP5, SCHEME_SSPRK104 = 0, 1
F_T_GRID, F_THETA, F_THETA_C, F_NU, F_C, F_R, F_DC, F_DR, F_ENERGY, F_MU = range(10)
K_HIST_INTEGRAL, K_STAGE_PREP, K_RK, K_SPARSIFY = range(4)
K_COUNT = 4


class dmfe_params(ctypes.Structure):
    _fields_ = [("n_terms", ctypes.c_int32), ("p", ctypes.c_int32 * MAX_TERMS),
                ("a2", ctypes.c_double * MAX_TERMS), ("T", ctypes.c_double), ("beta0", ctypes.c_double),
                ("t_max", ctypes.c_double), ("mode", ctypes.c_int32), ("precision", ctypes.c_int32),
                ("h", ctypes.c_double), ("N", ctypes.c_int64), ("L", ctypes.c_int32), ("M_cap", ctypes.c_int32),
                ("eps", ctypes.c_double), ("dt0", ctypes.c_double), ("dt_min", ctypes.c_double),
                ("s", ctypes.c_int32), ("auto_passes", ctypes.c_int32), ("grid_alpha", ctypes.c_double),
                ("grid_delta", ctypes.c_double), ("scheme_policy", ctypes.c_int32), ("theta_interp", ctypes.c_int32),
                ("fh_d", ctypes.c_int32), ("log_r", ctypes.c_int32)]


class dmfe_resources(ctypes.Structure):
    _fields_ = [("device", ctypes.c_int32), ("reserved0", ctypes.c_int32), ("stream", ctypes.c_void_p),
                ("workspace", ctypes.c_void_p), ("workspace_bytes", ctypes.c_size_t)]


class dmfe_step_info(ctypes.Structure):
    _fields_ = [("accepted", ctypes.c_int64), ("rejected", ctypes.c_int64), ("reverts", ctypes.c_int64),
                ("sparsify_calls", ctypes.c_int64), ("removed", ctypes.c_int64), ("rhs_evals", ctypes.c_int64),
                ("M", ctypes.c_int64), ("scheme", ctypes.c_int32), ("nb_valid", ctypes.c_int32),
                ("t", ctypes.c_double), ("dt", ctypes.c_double), ("eps_rk", ctypes.c_double)]

    def as_dict(self) -> dict:
        return {k: getattr(self, k) for k, _ in self._fields_ if k != "reserved0"}


class dmfe_control(ctypes.Structure):
    _fields_ = [("eps", ctypes.c_double), ("dt", ctypes.c_double), ("dt_min", ctypes.c_double),
                ("rho", ctypes.c_double), ("M", ctypes.c_int64), ("scheme", ctypes.c_int32),
                ("policy", ctypes.c_int32)]


class dmfe_pool_params(ctypes.Structure):
    _fields_ = [("max_instances", ctypes.c_int32), ("reserved0", ctypes.c_int32), ("max_bytes", ctypes.c_size_t)]


class dmfe_pool_stats(ctypes.Structure):
    _fields_ = [("running", ctypes.c_int32), ("queued", ctypes.c_int32), ("finished_unreleased", ctypes.c_int32),
                ("reserved0", ctypes.c_int32), ("ticks", ctypes.c_int64), ("bytes_free", ctypes.c_size_t),
                ("bytes_total", ctypes.c_size_t)]


class dmfe_pool_times(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int32), ("done", ctypes.c_int32), ("queue_s", ctypes.c_double),
                ("service_s", ctypes.c_double), ("total_s", ctypes.c_double)]


_lib = None

# exported symbol -> (restype, argtypes)
_vp, _i32, _i64, _d, _sz = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double, ctypes.c_size_t
SIGNATURES = {
    "dmfe_footprint": (_i32, [ctypes.POINTER(dmfe_params), ctypes.POINTER(_sz)]),
    "dmfe_create": (_i32, [ctypes.POINTER(dmfe_params), ctypes.POINTER(dmfe_resources), ctypes.POINTER(_vp)]),
    "dmfe_step": (_i32, [_vp, _d, _i64, ctypes.POINTER(dmfe_step_info)]),
    "dmfe_sparsify": (_i32, [_vp, _i32, ctypes.POINTER(_i64)]),
    "dmfe_read": (_i32, [_vp, _i32, _i64, _i64, _vp, _sz, _i32, ctypes.POINTER(_sz)]),
    "dmfe_get_info": (_i32, [_vp, ctypes.POINTER(dmfe_step_info)]),
    "dmfe_set_history": (_i32, [_vp, _i64, _i64, _vp, _vp, _vp, _vp, _vp, _i32, _d, _i32]),
    "dmfe_rhs": (_i32, [_vp, _d, _vp, _vp, _i64, _vp, _vp, _vp, _vp]),
    "dmfe_rhs_noalloc": (_i32, [_vp, _d, _vp, _vp, _i64, _vp, _vp, _vp, _vp]),
    "dmfe_destroy": (None, [_vp]),
    "dmfe_status_string": (ctypes.c_char_p, [_i32]),
    "dmfe_last_error": (ctypes.c_char_p, []),
    "dmfe_param_record": (_i32, [_vp, ctypes.c_char_p, ctypes.c_size_t, ctypes.POINTER(ctypes.c_size_t)]),
    "dmfe_snapshot_save": (_i32, [_vp, ctypes.c_char_p, _i32, _i32]),
    "dmfe_grid": (_i32, [ctypes.POINTER(dmfe_params), _vp, _vp, _vp, _vp]),
    "dmfe_control_update": (_i32, [ctypes.POINTER(dmfe_control), _d, ctypes.POINTER(_i32), ctypes.POINTER(_i32)]),
    "dmfe_sparsify_select": (_i32, [_vp, _i64, _i64, _d, _vp, ctypes.POINTER(_i64)]),
    "dmfe_timing": (_i32, [_vp, _i32]),
    "dmfe_timing_select": (_i32, [_vp, ctypes.c_uint32]),
    "dmfe_checkpoint_save": (_i32, [_vp, ctypes.c_char_p, _i32]),
    "dmfe_checkpoint_wait": (_i32, [_vp]),
    "dmfe_checkpoint_load": (_i32, [ctypes.c_char_p, ctypes.POINTER(dmfe_resources), ctypes.POINTER(_vp)]),
    "dmfe_pool_create": (_i32, [ctypes.POINTER(dmfe_pool_params), ctypes.POINTER(dmfe_resources),
                                ctypes.POINTER(_vp)]),
    "dmfe_pool_submit": (_i32, [_vp, ctypes.POINTER(dmfe_params), ctypes.POINTER(ctypes.c_uint64)]),
    "dmfe_pool_run": (_i32, [_vp, _i64, ctypes.POINTER(dmfe_pool_stats)]),
    "dmfe_pool_poll": (_i32, [_vp, ctypes.POINTER(ctypes.c_uint64), _i32, ctypes.POINTER(_i32)]),
    "dmfe_pool_result": (_i32, [_vp, ctypes.c_uint64, ctypes.POINTER(dmfe_step_info),
                                ctypes.POINTER(dmfe_pool_times)]),
    "dmfe_pool_read": (_i32, [_vp, ctypes.c_uint64, _i32, _i64, _i64, _vp, _sz, _i32, ctypes.POINTER(_sz)]),
    "dmfe_pool_release": (_i32, [_vp, ctypes.c_uint64]),
    "dmfe_pool_set_history": (_i32, [_vp, ctypes.c_uint64, _i64, _i64, _vp, _vp, _vp, _vp, _vp, _i32, _d, _i32]),
    "dmfe_pool_destroy": (None, [_vp]),
    "dmfe_timing_read": (_i32, [_vp, _i32, ctypes.POINTER(_i64), ctypes.POINTER(_d), ctypes.POINTER(_i64)]),
}


def lib() -> ctypes.CDLL:
    """The loaded libdmfe.so (raises RuntimeError if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"libdmfe.so not built ({LIB_PATH}); run python -m paper_2604_06309_amd.build")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


class DmfeError(RuntimeError):
    def __init__(self, status: int, where: str):
        msg = lib().dmfe_status_string(status).decode()
        extra = lib().dmfe_last_error().decode()
        super().__init__(f"{where}: {msg} ({status})" + (f": {extra}" if extra and status == ERR_DEVICE else ""))
        self.status = status


def _check(st: int, where: str, allow=(OK, DONE)) -> int:
    if st not in allow:
        raise DmfeError(st, where)
    return st


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


# ----------------------------------------------------------------------------- parameters
def make_params(terms: dict, T: float, *, beta0: float = 0.0, t_max: float = 1e4, mode: int = ADAPTIVE,
                precision: int = FP64, h: float = 0.05, N: int = 1000, L: int = 512, M_cap: int = 0,
                eps: float = 1e-8, dt0: float = 1e-4, dt_min: float = 1e-12, s: int = 10, auto_passes: int = 1,
                scheme_policy: int = 0, grid_alpha: float = 0.0, grid_delta: float = 0.0,
                theta_interp: int = INTERP_INDEX_LAGRANGE, fh_d: int = 3, log_r: bool = False) -> dmfe_params:
    """terms maps p -> a_p^2 (f(q) = sum_p a_p^2 q^p / 2, Sec. 2.1).  theta_interp,
    fh_d and log_r choose the theta-stencil (Sec. 3.3) and the log-R option."""
    p = dmfe_params()
    p.n_terms = len(terms)
    for k, (pp, a2) in enumerate(sorted(terms.items())):
        p.p[k] = int(pp)
        p.a2[k] = float(a2)
    p.T, p.beta0, p.t_max = float(T), float(beta0), float(t_max)
    p.mode, p.precision, p.h, p.N = int(mode), int(precision), float(h), int(N)
    p.L, p.M_cap, p.eps, p.dt0, p.dt_min = int(L), int(M_cap), float(eps), float(dt0), float(dt_min)
    p.s, p.auto_passes, p.scheme_policy = int(s), int(auto_passes), int(scheme_policy)
    p.grid_alpha, p.grid_delta = float(grid_alpha), float(grid_delta)
    p.theta_interp, p.fh_d, p.log_r = int(theta_interp), int(fh_d), int(bool(log_r))
    return p


# ----------------------------------------------------------------------------- C-ABI mirrors
def dmfe_footprint(params: dmfe_params) -> int:
    b = ctypes.c_size_t()
    _check(lib().dmfe_footprint(ctypes.byref(params), ctypes.byref(b)), "dmfe_footprint")
    return b.value


def dmfe_create(params: dmfe_params, device: int = 0, stream: int = 0, workspace: int = 0,
                workspace_bytes: int = 0) -> int:
    r = dmfe_resources()
    r.device, r.stream, r.workspace, r.workspace_bytes = device, stream or None, workspace or None, workspace_bytes
    h = ctypes.c_void_p()
    _check(lib().dmfe_create(ctypes.byref(params), ctypes.byref(r), ctypes.byref(h)), "dmfe_create", (OK,))
    return h.value


def dmfe_step(h: int, t_target: float, max_steps: int) -> tuple[int, dmfe_step_info]:
    info = dmfe_step_info()
    st = lib().dmfe_step(h, t_target, max_steps, ctypes.byref(info))
    return st, info


def dmfe_sparsify(h: int, passes: int = 1) -> int:
    r = ctypes.c_int64()
    _check(lib().dmfe_sparsify(h, passes, ctypes.byref(r)), "dmfe_sparsify")
    return r.value


def dmfe_read(h: int, field: int, first: int, count: int, dst=None, dst_on_device: bool = False) -> int:
    """Copy into dst (numpy array or device pointer int); returns bytes needed."""
    need = ctypes.c_size_t()
    if dst is None:
        _check(lib().dmfe_read(h, field, first, count, None, 0, 0, ctypes.byref(need)), "dmfe_read")
        return need.value
    if isinstance(dst, np.ndarray):
        ptr, nbytes, on_dev = _ptr(dst), dst.nbytes, 0
    else:
        ptr, nbytes, on_dev = int(dst.data_ptr()), dst.numel() * dst.element_size(), 1
    _check(lib().dmfe_read(h, field, first, count, ptr, nbytes, on_dev, ctypes.byref(need)), "dmfe_read")
    return need.value


def dmfe_get_info(h: int) -> dmfe_step_info:
    info = dmfe_step_info()
    _check(lib().dmfe_get_info(h, ctypes.byref(info)), "dmfe_get_info")
    return info


def _history_args(t_hist, C, R, dC, dR, nb):
    M = int(len(t_hist))
    nb = M if nb is None else int(nb)
    if isinstance(C, np.ndarray):
        arrs = [np.ascontiguousarray(a, dtype=np.float64) for a in (t_hist, C, R, dC, dR)]
        ptrs, on_dev = [_ptr(a) for a in arrs], 0
    else:
        arrs = [a.contiguous().double() for a in (t_hist, C, R, dC, dR)]
        ptrs, on_dev = [a.data_ptr() for a in arrs], 1
    return M, nb, arrs, ptrs, on_dev


def dmfe_set_history(h: int, t_hist, C, R, dC, dR, nb: Optional[int] = None, dt: float = 0.0,
                     scheme: int = -1) -> None:
    """Host numpy arrays ([M], [M, L] x4) or CUDA tensors of the same shapes."""
    M, nb, arrs, ptrs, on_dev = _history_args(t_hist, C, R, dC, dR, nb)
    _check(lib().dmfe_set_history(h, M, nb, *ptrs, on_dev, dt, scheme), "dmfe_set_history")


def dmfe_pool_set_history(pool: int, rid: int, t_hist, C, R, dC, dR, nb: Optional[int] = None, dt: float = 0.0,
                          scheme: int = -1) -> None:
    """dmfe_set_history on an admitted pooled solve between two steps."""
    M, nb, arrs, ptrs, on_dev = _history_args(t_hist, C, R, dC, dR, nb)
    _check(lib().dmfe_pool_set_history(pool, rid, M, nb, *ptrs, on_dev, dt, scheme), "dmfe_pool_set_history")


def dmfe_rhs(h: int, t: float, yC, yR, nb: int):
    """yC, yR: CUDA float64 tensors [L].  Returns (dC/dt, dR/dt) tensors, mu, diag[2]."""
    import torch
    outC = torch.empty_like(yC)
    outR = torch.empty_like(yR)
    mu = ctypes.c_double()
    diag = np.zeros(2)
    _check(lib().dmfe_rhs(h, t, yC.data_ptr(), yR.data_ptr(), nb, outC.data_ptr(), outR.data_ptr(),
                          ctypes.byref(mu), _ptr(diag)), "dmfe_rhs")
    return outC, outR, mu.value, diag


def dmfe_rhs_noalloc(h: int, t: float, yC, yR, nb: int, outC, outR):
    """As dmfe_rhs, writing into the caller's CUDA float64 tensors outC, outR [L];
    the library allocates nothing (its transient buffers are a static device array).
    Returns mu, diag[2]."""
    mu = ctypes.c_double()
    diag = np.zeros(2)
    _check(lib().dmfe_rhs_noalloc(h, t, yC.data_ptr(), yR.data_ptr(), nb, outC.data_ptr(), outR.data_ptr(),
                                  ctypes.byref(mu), _ptr(diag)), "dmfe_rhs_noalloc")
    return mu.value, diag


def dmfe_timing(h: int, enable: bool) -> None:
    _check(lib().dmfe_timing(h, int(enable)), "dmfe_timing")


def dmfe_timing_select(h: int, kernels) -> None:
    """Time only the given kernel ids (K_*) while timing is on."""
    mask = 0
    for k in kernels:
        mask |= 1 << int(k)
    _check(lib().dmfe_timing_select(h, mask), "dmfe_timing_select")


def dmfe_timing_read(h: int, kernel: int) -> tuple[int, float, int]:
    n, ms, sl = ctypes.c_int64(), ctypes.c_double(), ctypes.c_int64()
    _check(lib().dmfe_timing_read(h, kernel, ctypes.byref(n), ctypes.byref(ms), ctypes.byref(sl)),
           "dmfe_timing_read")
    return n.value, ms.value, sl.value


def dmfe_destroy(h: int) -> None:
    if h:
        lib().dmfe_destroy(h)


def dmfe_checkpoint_save(h: int, path: str, async_write: bool = False) -> None:
    _check(lib().dmfe_checkpoint_save(h, os.fsencode(path), int(async_write)), "dmfe_checkpoint_save")


def dmfe_checkpoint_wait(h: int) -> None:
    _check(lib().dmfe_checkpoint_wait(h), "dmfe_checkpoint_wait")


def dmfe_checkpoint_load(path: str, device: int = 0, stream: int = 0, workspace: int = 0,
                         workspace_bytes: int = 0) -> int:
    r = dmfe_resources()
    r.device, r.stream, r.workspace, r.workspace_bytes = device, stream or None, workspace or None, workspace_bytes
    h = ctypes.c_void_p()
    _check(lib().dmfe_checkpoint_load(os.fsencode(path), ctypes.byref(r), ctypes.byref(h)), "dmfe_checkpoint_load")
    return h.value


def dmfe_status_string(status: int) -> str:
    return lib().dmfe_status_string(status).decode()


def load_snapshot(path: str) -> dict:
    """Read a file written by dmfe_snapshot_save: theta, t, E, mu (float64), C and R
    ([M_kept, L_kept] float32), the strides, L, M and the parameter record text."""
    raw = open(path, "rb").read()
    if raw[:8] != b"DMFESNP1":
        raise ValueError(f"{path}: not a DMFE snapshot")
    version, header = np.frombuffer(raw, np.uint32, 2, 8)
    if version != 1:
        raise ValueError(f"{path}: snapshot version {version}")
    L, M, ts, ss, Lk, Mk = (int(v) for v in np.frombuffer(raw, np.int64, 6, 16))
    rb = int(np.frombuffer(raw, np.uint64, 1, 64)[0])
    off = int(header)
    record = raw[off:off + rb].rstrip(b"\0").decode()
    off += rb
    out = {"L": L, "M": M, "theta_stride": ts, "slice_stride": ss, "record": record}
    for name, n in (("theta", Lk), ("t", Mk), ("E", Mk), ("mu", Mk)):
        out[name] = np.frombuffer(raw, np.float64, n, off).copy()
        off += 8 * n
    for name in ("C", "R"):
        out[name] = np.frombuffer(raw, np.float32, Mk * Lk, off).reshape(Mk, Lk).copy()
        off += 4 * Mk * Lk
    if off != len(raw):
        raise ValueError(f"{path}: {len(raw) - off} bytes past the snapshot")
    return out


def dmfe_param_record(h: int) -> str:
    """The solve's human-readable parameter record (key = value lines)."""
    need = ctypes.c_size_t()
    st = lib().dmfe_param_record(h, None, 0, ctypes.byref(need))
    _check(st, "dmfe_param_record", (OK, ERR_BUFFER))
    buf = ctypes.create_string_buffer(need.value)
    _check(lib().dmfe_param_record(h, buf, need.value, ctypes.byref(need)), "dmfe_param_record")
    return buf.value.decode()


def dmfe_last_error() -> str:
    return lib().dmfe_last_error().decode()


def dmfe_grid(params: dmfe_params):
    L = params.L
    th, thc, nu = np.zeros(L), np.zeros(L), np.zeros(L)
    g = ctypes.c_double()
    _check(lib().dmfe_grid(ctypes.byref(params), _ptr(th), _ptr(thc), _ptr(nu), ctypes.byref(g)), "dmfe_grid")
    return th, thc, nu, g.value


def dmfe_control_update(ctl: dmfe_control, eps_rk: float):
    acc = ctypes.c_int32()
    nrev = ctypes.c_int32()
    st = lib().dmfe_control_update(ctypes.byref(ctl), eps_rk, ctypes.byref(acc), ctypes.byref(nrev))
    return st, bool(acc.value), nrev.value


def dmfe_sparsify_select(eps_n: np.ndarray, last: int, thr: float):
    e = np.ascontiguousarray(eps_n, dtype=np.float64)
    drop = np.zeros(e.size, dtype=np.uint8)
    rem = ctypes.c_int64()
    _check(lib().dmfe_sparsify_select(_ptr(e), e.size, last, thr, _ptr(drop), ctypes.byref(rem)),
           "dmfe_sparsify_select")
    return rem.value, drop.astype(bool)


# ----------------------------------------------------------------------------- serving pool
def dmfe_pool_create(max_instances: int, device: int, stream: int, arena_ptr: int, arena_bytes: int,
                     max_bytes: int = 0) -> int:
    pp = dmfe_pool_params()
    pp.max_instances, pp.max_bytes = max_instances, max_bytes
    r = dmfe_resources()
    r.device, r.stream, r.workspace, r.workspace_bytes = device, stream or None, arena_ptr, arena_bytes
    h = ctypes.c_void_p()
    _check(lib().dmfe_pool_create(ctypes.byref(pp), ctypes.byref(r), ctypes.byref(h)), "dmfe_pool_create", (OK,))
    return h.value


def dmfe_pool_submit(pool: int, params: dmfe_params) -> int:
    rid = ctypes.c_uint64()
    _check(lib().dmfe_pool_submit(pool, ctypes.byref(params), ctypes.byref(rid)), "dmfe_pool_submit", (OK,))
    return rid.value


def dmfe_pool_run(pool: int, max_ticks: int) -> dmfe_pool_stats:
    st = dmfe_pool_stats()
    _check(lib().dmfe_pool_run(pool, max_ticks, ctypes.byref(st)), "dmfe_pool_run", (OK,))
    return st


def dmfe_pool_poll(pool: int, cap: int = 4096) -> list[int]:
    ids = (ctypes.c_uint64 * cap)()
    n = ctypes.c_int32()
    _check(lib().dmfe_pool_poll(pool, ids, cap, ctypes.byref(n)), "dmfe_pool_poll", (OK,))
    return [ids[k] for k in range(n.value)]


def dmfe_pool_result(pool: int, rid: int) -> tuple[dmfe_step_info, dmfe_pool_times]:
    info, tm = dmfe_step_info(), dmfe_pool_times()
    _check(lib().dmfe_pool_result(pool, rid, ctypes.byref(info), ctypes.byref(tm)), "dmfe_pool_result", (OK,))
    return info, tm


def dmfe_pool_read(pool: int, rid: int, field: int, first: int, count: int, dst: Optional[np.ndarray] = None) -> int:
    need = ctypes.c_size_t()
    if dst is None:
        _check(lib().dmfe_pool_read(pool, rid, field, first, count, None, 0, 0, ctypes.byref(need)), "dmfe_pool_read")
        return need.value
    _check(lib().dmfe_pool_read(pool, rid, field, first, count, _ptr(dst), dst.nbytes, 0, ctypes.byref(need)),
           "dmfe_pool_read")
    return need.value


def dmfe_pool_release(pool: int, rid: int) -> None:
    _check(lib().dmfe_pool_release(pool, rid), "dmfe_pool_release", (OK,))


def dmfe_pool_destroy(pool: int) -> None:
    if pool:
        lib().dmfe_pool_destroy(pool)


class Pool:
    """A serving pool over a caller-owned arena (a torch uint8 tensor on the device)."""

    def __init__(self, arena_bytes: int, max_instances: int = 256, stream=None):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("Pool needs a GPU (HIP device)")
        dev = torch.cuda.current_device()
        self.stream = stream if stream is not None else torch.cuda.current_stream(dev)
        self.arena = torch.empty(arena_bytes, dtype=torch.uint8, device=f"cuda:{dev}")
        self.p = dmfe_pool_create(max_instances, dev, self.stream.cuda_stream, self.arena.data_ptr(), arena_bytes)

    def submit(self, params: dmfe_params) -> int:
        return dmfe_pool_submit(self.p, params)

    def run(self, max_ticks: int = 1 << 40) -> dmfe_pool_stats:
        return dmfe_pool_run(self.p, max_ticks)

    def poll(self) -> list[int]:
        return dmfe_pool_poll(self.p)

    def result(self, rid: int):
        return dmfe_pool_result(self.p, rid)

    def read(self, rid: int, field: int, first: int = 0, count: Optional[int] = None, L: Optional[int] = None):
        if count is None:
            count = int(self.result(rid)[0].M) - first
        need = dmfe_pool_read(self.p, rid, field, first, count)
        out = np.empty(need // 8)
        dmfe_pool_read(self.p, rid, field, first, count, out)
        if L is not None and field in (F_C, F_R, F_DC, F_DR):
            out = out.reshape(count, L)
        return out

    def release(self, rid: int) -> None:
        dmfe_pool_release(self.p, rid)

    def set_history(self, rid: int, t_hist, C, R, dC, dR, nb=None, dt: float = 0.0, scheme: int = -1) -> None:
        dmfe_pool_set_history(self.p, rid, t_hist, C, R, dC, dR, nb, dt, scheme)

    def close(self):
        if getattr(self, "p", None):
            dmfe_pool_destroy(self.p)
            self.p = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ----------------------------------------------------------------------------- convenience wrapper
class Solver:
    """One solver handle on the current CUDA device and stream."""

    def __init__(self, params: dmfe_params, device: Optional[int] = None, stream=None, use_workspace: bool = False):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("Solver needs a GPU (HIP device)")
        lib()
        self.params = params
        dev = torch.cuda.current_device() if device is None else device
        self.stream = stream if stream is not None else torch.cuda.current_stream(dev)
        self._ws = None
        ws, wsb = 0, 0
        if use_workspace:
            nbytes = dmfe_footprint(params)
            self._ws = torch.empty(nbytes, dtype=torch.uint8, device=f"cuda:{dev}")
            ws, wsb = self._ws.data_ptr(), nbytes
        self.h = dmfe_create(params, dev, self.stream.cuda_stream, ws, wsb)

    @classmethod
    def load(cls, path: str, params: dmfe_params, device: Optional[int] = None, stream=None) -> "Solver":
        """Restore a solver from a checkpoint file written by checkpoint(); `params`
        must be the saved solve's parameters (they size the handle's view)."""
        import torch
        self = cls.__new__(cls)
        lib()
        self.params = params
        dev = torch.cuda.current_device() if device is None else device
        self.stream = stream if stream is not None else torch.cuda.current_stream(dev)
        self._ws = None
        self.h = dmfe_checkpoint_load(path, dev, self.stream.cuda_stream)
        return self

    def checkpoint(self, path: str, async_write: bool = False) -> None:
        dmfe_checkpoint_save(self.h, path, async_write)

    def checkpoint_wait(self) -> None:
        dmfe_checkpoint_wait(self.h)

    def close(self):
        if getattr(self, "h", None):
            dmfe_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def step(self, t_target: float = float("inf"), max_steps: int = 1 << 62) -> tuple[int, dmfe_step_info]:
        st, info = dmfe_step(self.h, t_target, max_steps)
        _check(st, "dmfe_step")
        return st, info

    def sparsify(self, passes: int = 1) -> int:
        return dmfe_sparsify(self.h, passes)

    def info(self) -> dmfe_step_info:
        return dmfe_get_info(self.h)

    def param_record(self) -> str:
        """Human-readable record of the solve: library build, device, parameters, grid, state."""
        return dmfe_param_record(self.h)

    def snapshot(self, path: str, theta_stride: int = 4, slice_stride: int = 1) -> None:
        """Compressed snapshot for post-processing (every theta_stride-th node, every
        slice_stride-th slice, FP32 C and R); read it back with load_snapshot()."""
        _check(lib().dmfe_snapshot_save(self.h, os.fsencode(path), int(theta_stride), int(slice_stride)),
               "dmfe_snapshot_save")

    def read(self, field: int, first: int = 0, count: Optional[int] = None) -> np.ndarray:
        """Host copy of a field.  Adaptive: C/R/DC/DR -> [count, L]; uniform C/R -> packed rows."""
        if count is None:
            info = self.info()
            count = self.params.L if field in (F_THETA, F_THETA_C, F_NU) else int(info.M) - first
        need = dmfe_read(self.h, field, first, count)
        out = np.empty(need // 8, dtype=np.float64)
        dmfe_read(self.h, field, first, count, out)
        if self.params.mode == ADAPTIVE and field in (F_C, F_R, F_DC, F_DR):
            out = out.reshape(count, self.params.L)
        return out

    def set_history(self, t_hist, C, R, dC, dR, nb=None, dt: float = 0.0, scheme: int = -1) -> None:
        dmfe_set_history(self.h, t_hist, C, R, dC, dR, nb, dt, scheme)

    def rhs(self, t: float, yC, yR, nb: int):
        return dmfe_rhs(self.h, t, yC, yR, nb)

    def timing(self, enable: bool, kernels=None) -> None:
        """Per-launch HIP events on (of the given kernel ids only, default all) or off."""
        if enable:
            dmfe_timing_select(self.h, range(K_COUNT) if kernels is None else kernels)
        dmfe_timing(self.h, enable)

    def timing_read(self, kernel: int) -> tuple[int, float, int]:
        return dmfe_timing_read(self.h, kernel)
