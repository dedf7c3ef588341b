"""Python binding of the gfx950 band-limited PDE-LDDMM library (ctypes).

Argument marshalling only: every step of the method runs in the HIP library
(liblddmm_bl.so, C ABI in include/lddmm_bl.h).  PyTorch provides device
memory and the stream; tensors must live on a ROCm device, be contiguous and
have the context's element type (float64 for FP64, float32 otherwise).
Loading fails loudly when the library has not been built.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass
from typing import Optional, Sequence, Tuple

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liblddmm_bl.so")

IMAGE_TRANSPORT = 1
STATE_EQUATION = 2
DEFORMATION_STATE = 3
FP64, FP32, BF16_DFT = 0, 1, 2
SL_RK2, EULER_RK4 = 0, 1

FIELD_VELOCITY, FIELD_DEP_BACKWARD, FIELD_DEP_FORWARD, FIELD_DIV_V = 0, 1, 2, 3
FIELD_STATE, FIELD_M1, FIELD_ADJOINT0, FIELD_INC_STATE, FIELD_INC_ADJOINT = 4, 5, 6, 7, 8
FIELD_INVERSE_STATE, FIELD_JACOBIAN_STATE, FIELD_IMAGE, FIELD_ADJOINT_GRID = 9, 10, 11, 12

STATUS = {
    0: "OK", -1: "E_ARG", -2: "E_OOM", -3: "E_HIP", -4: "E_NONFINITE", -5: "E_STATE",
    1: "W_MAXITER", 2: "W_LINESEARCH", 3: "W_NEGCURV",
}

EXPORTS = [
    "lddmm_bl_create", "lddmm_bl_destroy", "lddmm_bl_last_error", "lddmm_bl_set_images",
    "lddmm_bl_state_solve", "lddmm_bl_adjoint_solve", "lddmm_bl_hess_matvec", "lddmm_bl_gn_solve",
    "lddmm_bl_jacobian", "lddmm_bl_project", "lddmm_bl_project_noalloc", "lddmm_bl_include", "lddmm_bl_get_field", "lddmm_bl_dot",
    "lddmm_bl_profile_enable", "lddmm_bl_profile_read", "lddmm_bl_gn_solve_batched",
    "lddmm_bl_tune_candidates", "lddmm_bl_tune_get", "lddmm_bl_tune_set", "lddmm_bl_tune_table",
    "lddmm_nn_create", "lddmm_nn_create_out", "lddmm_nn_info", "lddmm_nn_forward", "lddmm_nn_backward", "lddmm_nn_zero_grad",
    "lddmm_nn_step", "lddmm_nn_get", "lddmm_nn_set", "lddmm_nn_save", "lddmm_nn_load", "lddmm_nn_destroy",
    "lddmm_nn_pool_pair",
    "lddmm_nn_velocity", "lddmm_nn_loss",
]


class Params(ctypes.Structure):
    _fields_ = [
        ("dim", ctypes.c_int32), ("n", ctypes.c_int32 * 3), ("k", ctypes.c_int32 * 3),
        ("nt", ctypes.c_int32), ("variant", ctypes.c_int32), ("alpha", ctypes.c_double),
        ("s", ctypes.c_int32), ("sigma2", ctypes.c_double), ("precision", ctypes.c_int32),
        ("integrator", ctypes.c_int32), ("nonstationary", ctypes.c_int32),
    ]


class GNOpts(ctypes.Structure):
    _fields_ = [
        ("max_gn", ctypes.c_int32), ("max_pcg", ctypes.c_int32), ("grad_rtol", ctypes.c_double),
        ("grad_ref_inf", ctypes.c_double), ("fixed_iters", ctypes.c_int32), ("energy_target", ctypes.c_double),
        ("ml_inner", ctypes.c_int32),
    ]


LOG_MAX = 64


class GNReport(ctypes.Structure):
    _fields_ = [
        ("gn_iters", ctypes.c_int32), ("pcg_iters_total", ctypes.c_int32), ("backtracks", ctypes.c_int32),
        ("hess_matvecs", ctypes.c_int32), ("E0", ctypes.c_double), ("E", ctypes.c_double),
        ("mse_rel", ctypes.c_double), ("grad_inf_rel", ctypes.c_double), ("det_min", ctypes.c_double),
        ("det_max", ctypes.c_double), ("seconds", ctypes.c_double), ("log_count", ctypes.c_int32),
        ("log_pcg", ctypes.c_int32 * LOG_MAX), ("log_negcurv", ctypes.c_int32 * LOG_MAX),
        ("log_backtracks", ctypes.c_int32 * LOG_MAX),
    ]

    def as_dict(self):
        """Report fields; the per-iteration decision log as a list of (pcg, negcurv, backtracks)."""
        d = {name: getattr(self, name) for name, _ in self._fields_ if not name.startswith("log_")}
        n = self.log_count
        d["decisions"] = [(self.log_pcg[i], self.log_negcurv[i], self.log_backtracks[i]) for i in range(n)]
        return d


_lib = None


def load_library(path: str = LIB_PATH) -> ctypes.CDLL:
    """Load liblddmm_bl.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"HIP library not built: {path} is missing (run python -m paper_2006_06823_amd.build)")
    lib = ctypes.CDLL(path)
    vp, i32, i64, dp = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.POINTER(ctypes.c_double)
    sig = {
        "lddmm_bl_create": [ctypes.POINTER(Params), vp, ctypes.POINTER(vp)],
        "lddmm_bl_destroy": [vp],
        "lddmm_bl_set_images": [vp, vp, vp],
        "lddmm_bl_state_solve": [vp, vp, vp, dp],
        "lddmm_bl_adjoint_solve": [vp, vp, dp],
        "lddmm_bl_hess_matvec": [vp, vp, vp],
        "lddmm_bl_gn_solve": [vp, ctypes.POINTER(GNOpts), vp, vp, i32, ctypes.POINTER(GNReport)],
        "lddmm_bl_jacobian": [vp, vp, dp],
        "lddmm_bl_project": [vp, vp, vp, i32],
        "lddmm_bl_project_noalloc": [vp, vp, vp, i32],
        "lddmm_bl_include": [vp, vp, vp, i32],
        "lddmm_bl_get_field": [vp, i32, i32, vp, ctypes.POINTER(i64)],
        "lddmm_bl_dot": [vp, vp, vp, i64, dp],
        "lddmm_bl_gn_solve_batched": [ctypes.POINTER(Params), i32, ctypes.POINTER(vp), ctypes.POINTER(vp),
                                      ctypes.POINTER(vp), ctypes.POINTER(GNOpts), vp, ctypes.POINTER(GNReport)],
    }
    ip = ctypes.POINTER(i32)
    sig.update({
        "lddmm_nn_create": [i32, ip, i32, i32, ctypes.c_uint64, vp, ctypes.POINTER(vp)],
        "lddmm_nn_create_out": [i32, ip, i32, i32, i32, ctypes.c_uint64, vp, ctypes.POINTER(vp)],
        "lddmm_nn_info": [vp, ip, ip, ctypes.POINTER(i64)],
        "lddmm_nn_forward": [vp, vp, i32, vp],
        "lddmm_nn_backward": [vp, vp, i32],
        "lddmm_nn_zero_grad": [vp],
        "lddmm_nn_step": [vp, ctypes.c_double],
        "lddmm_nn_get": [vp, i32, vp],
        "lddmm_nn_set": [vp, vp],
        "lddmm_nn_save": [vp, ctypes.c_char_p],
        "lddmm_nn_load": [vp, ctypes.c_char_p],
        "lddmm_nn_destroy": [vp],
        "lddmm_nn_pool_pair": [vp, vp, vp, ip, vp],
        "lddmm_nn_velocity": [vp, vp, i32, ip, vp],
        "lddmm_nn_loss": [vp, vp, vp, i32, ip, ctypes.c_double, i32, vp, dp],
    })
    for name, args in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = ctypes.c_int
    lib.lddmm_bl_profile_enable.argtypes = [i32]
    lib.lddmm_bl_profile_enable.restype = ctypes.c_int
    lib.lddmm_bl_profile_read.argtypes = [ctypes.c_char_p, i64]
    lib.lddmm_bl_profile_read.restype = i64
    lib.lddmm_bl_tune_candidates.argtypes = [ctypes.c_char_p]
    lib.lddmm_bl_tune_candidates.restype = i32
    lib.lddmm_bl_tune_get.argtypes = [ctypes.c_char_p]
    lib.lddmm_bl_tune_get.restype = i32
    lib.lddmm_bl_tune_set.argtypes = [ctypes.c_char_p, i32]
    lib.lddmm_bl_tune_set.restype = ctypes.c_int
    lib.lddmm_bl_tune_table.argtypes = [ctypes.c_char_p, i64]
    lib.lddmm_bl_tune_table.restype = i64
    lib.lddmm_bl_last_error.argtypes = [vp]
    lib.lddmm_bl_last_error.restype = ctypes.c_char_p
    _lib = lib
    return lib


class LddmmError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


def _ptr(t: Optional[torch.Tensor]):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


@dataclass
class Problem:
    """Problem description; n and k are per-axis grid and band sizes (d = len(n))."""
    n: Sequence[int]
    k: Sequence[int]
    nt: int = 10
    variant: int = IMAGE_TRANSPORT
    alpha: float = 0.0025
    s: int = 2
    sigma2: float = 1.0
    precision: int = FP32
    integrator: int = 0     # SL_RK2; EULER_RK4: the explicit RK comparator (deformation state only)
    nonstationary: bool = False  # a velocity per time node: v~ of shape (nt + 1, d, *k)


def make_params(prob: "Problem") -> Params:
    p = Params()
    d = len(prob.n)
    p.dim = d
    for j in range(3):
        p.n[j] = int(prob.n[j]) if j < d else 1
        p.k[j] = int(prob.k[j]) if j < d else 1
    p.nt, p.variant, p.alpha, p.s, p.sigma2, p.precision = (
        prob.nt, prob.variant, prob.alpha, prob.s, prob.sigma2, prob.precision)
    p.integrator = prob.integrator
    p.nonstationary = 1 if prob.nonstationary else 0
    return p


def gn_solve_batched(problems, I0s, I1s, vs, max_gn=10, max_pcg=5, grad_rtol=1e-3, grad_ref_inf=0.0,
                     fixed_iters=False, device=None):
    """Batched Gauss-Newton-Krylov over subjects of uneven sizes (velocities updated in place).

    Returns (status, [report dict per subject]).  All tensors float32 on one ROCm device.
    """
    lib = load_library()
    B = len(problems)
    dev = torch.device(device) if device is not None else torch.device("cuda", torch.cuda.current_device())
    for t in list(I0s) + list(I1s) + list(vs):
        if t.dtype != torch.float32 or t.device.type != "cuda" or not t.is_contiguous():
            raise TypeError("batched tensors must be contiguous float32 ROCm tensors")
    params = (Params * B)(*[make_params(p) for p in problems])
    arr = lambda ts: (ctypes.c_void_p * B)(*[t.data_ptr() for t in ts])
    opts = GNOpts(max_gn, max_pcg, grad_rtol, grad_ref_inf, 1 if fixed_iters else 0, 0.0, 0)
    reps = (GNReport * B)()
    stream = torch.cuda.Stream(device=dev)
    stream.wait_stream(torch.cuda.current_stream(dev))
    st = lib.lddmm_bl_gn_solve_batched(params, B, arr(I0s), arr(I1s), arr(vs), ctypes.byref(opts),
                                       ctypes.c_void_p(stream.cuda_stream), reps)
    if st < 0:
        raise LddmmError(st, lib.lddmm_bl_last_error(None).decode())
    torch.cuda.current_stream(dev).wait_stream(stream)
    return st, [reps[i].as_dict() for i in range(B)]


class Context:
    """One registration problem on the current ROCm device and stream."""

    def __init__(self, prob: Problem, device: Optional[torch.device] = None, stream=None):
        self.lib = load_library()
        self.prob = prob
        self.dim = len(prob.n)
        self.nt = int(prob.nt)
        self.nonstationary = bool(prob.nonstationary)
        self.n = tuple(int(x) for x in prob.n)
        self.k = tuple(int(x) for x in prob.k)
        self.dtype = torch.float64 if prob.precision == FP64 else torch.float32
        self.device = torch.device(device) if device is not None else torch.device("cuda", torch.cuda.current_device())
        # a dedicated non-default stream: the library captures its Hessian matvec into a HIP graph on it
        self.stream = stream if stream is not None else torch.cuda.Stream(device=self.device)
        p = make_params(prob)
        h = ctypes.c_void_p()
        with torch.cuda.device(self.device):
            st = self.lib.lddmm_bl_create(ctypes.byref(p), ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(h))
        if st != 0:
            raise LddmmError(st, "lddmm_bl_create: " + self.lib.lddmm_bl_last_error(None).decode())
        self.h = h

    # -- helpers -----------------------------------------------------------
    def close(self):
        if getattr(self, "h", None):
            self.lib.lddmm_bl_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _order(self):
        """Make the library's stream wait for work queued on the caller's current stream."""
        cur = torch.cuda.current_stream(self.device)
        if cur != self.stream:
            self.stream.wait_stream(cur)

    def _after(self):
        """Make the caller's current stream wait for work the library only enqueued (no host wait)."""
        cur = torch.cuda.current_stream(self.device)
        if cur != self.stream:
            cur.wait_stream(self.stream)

    def _check(self, st, allow_warn=False):
        if st < 0 or (st > 0 and not allow_warn):
            raise LddmmError(st, self.lib.lddmm_bl_last_error(self.h).decode())
        return st

    def _grid_shape(self, ncomp=None):
        return self.n if ncomp is None else (ncomp,) + self.n

    def _bl_shape(self, ncomp=None):
        return self.k if ncomp is None else (ncomp,) + self.k

    def _vshape(self):
        """Shape of velocity-like arrays (velocity, gradient, Hessian directions): (dim, *k), or
        (nt + 1, dim, *k) for a non-stationary problem."""
        return ((self.nt + 1,) if self.nonstationary else ()) + self._bl_shape(self.dim)

    def _arg(self, t: torch.Tensor, shape, name):
        if not isinstance(t, torch.Tensor) or t.device.type != "cuda":
            raise TypeError(f"{name} must be a ROCm device tensor")
        if t.dtype != self.dtype:
            raise TypeError(f"{name} must be {self.dtype}")
        if tuple(t.shape) != tuple(shape):
            raise ValueError(f"{name} has shape {tuple(t.shape)}, expected {tuple(shape)}")
        if not t.is_contiguous():
            raise ValueError(f"{name} must be contiguous")
        return t

    def empty_grid(self, ncomp=None):
        return torch.empty(self._grid_shape(ncomp), dtype=self.dtype, device=self.device)

    def empty_bl(self, ncomp=None):
        return torch.empty(self._bl_shape(ncomp), dtype=self.dtype, device=self.device)

    # -- C ABI calls -----------------------------------------------------------
    def set_images(self, I0: torch.Tensor, I1: torch.Tensor):
        self._arg(I0, self.n, "I0")
        self._arg(I1, self.n, "I1")
        self._order()
        self._check(self.lib.lddmm_bl_set_images(self.h, _ptr(I0), _ptr(I1)))

    def state_solve(self, v: torch.Tensor, want_m1: bool = False) -> Tuple[Tuple[float, float, float], Optional[torch.Tensor]]:
        self._arg(v, self._vshape(), "v")
        m1 = self.empty_grid() if want_m1 else None
        E = (ctypes.c_double * 3)()
        self._order()
        self._check(self.lib.lddmm_bl_state_solve(self.h, _ptr(v), _ptr(m1), E))
        return (E[0], E[1], E[2]), m1

    def adjoint_solve(self) -> Tuple[torch.Tensor, float]:
        g = torch.empty(self._vshape(), dtype=self.dtype, device=self.device)
        ginf = ctypes.c_double()
        self._order()
        self._check(self.lib.lddmm_bl_adjoint_solve(self.h, _ptr(g), ctypes.byref(ginf)))
        return g, ginf.value

    def hess_matvec(self, dv: torch.Tensor, out: Optional[torch.Tensor] = None) -> torch.Tensor:
        """H dv into out, enqueued on the context's stream; the current stream waits for it (no host wait)."""
        self._arg(dv, self._vshape(), "dv")
        out = torch.empty(self._vshape(), dtype=self.dtype, device=self.device) if out is None else \
            self._arg(out, self._vshape(), "out")
        self._order()
        self._check(self.lib.lddmm_bl_hess_matvec(self.h, _ptr(dv), _ptr(out)))
        self._after()
        return out

    def gn_solve(self, v: torch.Tensor, max_gn=10, max_pcg=5, grad_rtol=1e-3, grad_ref_inf=0.0,
                 fixed_iters=False, Z: Optional[torch.Tensor] = None, energy_target=0.0, ml_inner=0):
        """Gauss-Newton-Krylov in place on v; returns (status, report dict).

        energy_target > 0 also stops the run once the objective is at or below it; ml_inner > 0 selects the
        two-level spectral preconditioner with that many inner coarse PCG iterations."""
        self._arg(v, self._vshape(), "v")
        o = GNOpts(max_gn, max_pcg, grad_rtol, grad_ref_inf, 1 if fixed_iters else 0, float(energy_target),
                   int(ml_inner))
        rep = GNReport()
        r = 0
        if Z is not None:
            r = Z.shape[0]
            self._arg(Z, (r, self.dim) + self.k, "Z")
        self._order()
        st = self.lib.lddmm_bl_gn_solve(self.h, ctypes.byref(o), _ptr(v), _ptr(Z), r, ctypes.byref(rep))
        self._check(st, allow_warn=True)
        return st, rep.as_dict()

    def jacobian(self, want_map: bool = False):
        det = torch.empty(self.n, dtype=torch.float64, device=self.device) if want_map else None
        mm = (ctypes.c_double * 2)()
        self._order()
        self._check(self.lib.lddmm_bl_jacobian(self.h, _ptr(det), mm))
        return (mm[0], mm[1]), det

    def project(self, grid: torch.Tensor, ncomp: int = 1) -> torch.Tensor:
        self._arg(grid, self._grid_shape(ncomp if ncomp > 1 else None), "grid")
        out = self.empty_bl(ncomp if ncomp > 1 else None)
        self._order()
        self._check(self.lib.lddmm_bl_project(self.h, _ptr(grid), _ptr(out), ncomp))
        return out

    def project_noalloc(self, grid: torch.Tensor, out: torch.Tensor, ncomp: int = 1) -> torch.Tensor:
        """pi into a caller-given output, with the library's static workspace (no device allocation
        in the call); enqueued on the context's stream."""
        self._arg(grid, self._grid_shape(ncomp if ncomp > 1 else None), "grid")
        self._arg(out, self._bl_shape(ncomp if ncomp > 1 else None), "out")
        self._order()
        self._check(self.lib.lddmm_bl_project_noalloc(self.h, _ptr(grid), _ptr(out), ncomp))
        self._after()
        return out

    def include(self, bl: torch.Tensor, ncomp: int = 1) -> torch.Tensor:
        self._arg(bl, self._bl_shape(ncomp if ncomp > 1 else None), "bl")
        out = self.empty_grid(ncomp if ncomp > 1 else None)
        self._order()
        self._check(self.lib.lddmm_bl_include(self.h, _ptr(bl), _ptr(out), ncomp))
        return out

    def get_field(self, which: int, index: int = 0) -> torch.Tensor:
        cnt = ctypes.c_int64()
        self._check(self.lib.lddmm_bl_get_field(self.h, which, index, None, ctypes.byref(cnt)))
        out = torch.empty(cnt.value, dtype=self.dtype, device=self.device)
        self._check(self.lib.lddmm_bl_get_field(self.h, which, index, _ptr(out), ctypes.byref(cnt)))
        return out

    def dot(self, a: torch.Tensor, b: torch.Tensor) -> float:
        if a.numel() != b.numel() or a.dtype != self.dtype or b.dtype != self.dtype:
            raise ValueError("dot: size or dtype mismatch")
        r = ctypes.c_double()
        self._order()
        self._check(self.lib.lddmm_bl_dot(self.h, _ptr(a), _ptr(b), a.numel(), ctypes.byref(r)))
        return r.value


def profile_enable(on: bool = True) -> None:
    """Start (clearing old records) or stop per-kernel event timing in the library."""
    load_library().lddmm_bl_profile_enable(1 if on else 0)


def profile_read():
    """Collect per-kernel timings: {name: dict(count, ms, bytes, flops)}."""
    lib = load_library()
    need = lib.lddmm_bl_profile_read(None, 0)
    buf = ctypes.create_string_buffer(int(need))
    lib.lddmm_bl_profile_read(buf, need)
    out = {}
    for line in buf.value.decode().splitlines():
        name, count, ms, nbytes, flops = line.split("\t")
        out[name] = dict(count=int(count), ms=float(ms), bytes=float(nbytes), flops=float(flops))
    return out


def tune_candidates(family: str = "brick") -> int:
    """Number of kernel variants the autotuner chooses from for a key family."""
    return int(load_library().lddmm_bl_tune_candidates(family.encode()))


def tune_get(key: str) -> int:
    """Cached autotuner choice of a key such as 'brick:128x128x128:gs2' (-1: none)."""
    return int(load_library().lddmm_bl_tune_get(key.encode()))


def tune_set(key: str, choice: int) -> None:
    """Fix (or with -1 forget) the autotuner choice of a key."""
    st = load_library().lddmm_bl_tune_set(key.encode(), int(choice))
    if st != 0:
        raise LddmmError(st, f"lddmm_bl_tune_set({key!r}, {choice}) rejected")


def tune_table() -> dict:
    """The autotuner cache: {key: choice}."""
    lib = load_library()
    need = lib.lddmm_bl_tune_table(None, 0)
    if need < 0:
        raise LddmmError(-1, "lddmm_bl_tune_table failed")
    buf = ctypes.create_string_buffer(int(need))
    lib.lddmm_bl_tune_table(buf, need)
    out = {}
    for line in buf.value.decode().splitlines():
        k, v = line.rsplit("=", 1)
        out[k] = int(v)
    return out


def brick_tune_keys(n) -> list:
    """The brick autotuner keys of a grid shape (3D, or 2D held as n0 = 1)."""
    n = tuple(int(x) for x in n)
    if len(n) == 2:
        n = (1,) + n
    return [f"brick:{n[0]}x{n[1]}x{n[2]}:gs{w}" for w in (1, 2, 3)]


class WarmStartNet:
    """The warm-start network (lddmm_nn_* in the C ABI) on one ROCm device.

    levels 3^3 convolutions (stride 2 but the last, or with out_size > 0 stride 2 while the grid
    is larger than out_size and 1 afterwards; ReLU) with the given channels on a
    [B][2][in_size]^3 float input, then a 1^3 head to 3 (1 + rank_r) channels: grid samples of
    the three velocity components (and of rank_r preconditioner directions) on a coarse
    out_size^3 grid.  All tensors are contiguous float32 on the device; the library works on
    its own stream, ordered after the caller's.
    """

    def __init__(self, channels=(16, 32, 64, 128), in_size=64, seed=0, device=None, rank_r=0, out_size=0):
        self.lib = load_library()
        self.device = torch.device(device) if device is not None else torch.device("cuda", torch.cuda.current_device())
        self.stream = torch.cuda.Stream(device=self.device)
        self.channels = tuple(int(c) for c in channels)
        self.in_size = int(in_size)
        self.rank_r = int(rank_r)
        self.req_out = int(out_size)
        ch = (ctypes.c_int32 * len(channels))(*self.channels)
        h = ctypes.c_void_p()
        with torch.cuda.device(self.device):
            st = self.lib.lddmm_nn_create_out(len(channels), ch, self.in_size, self.req_out, self.rank_r, seed,
                                              ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(h))
        if st != 0:
            raise LddmmError(st, "lddmm_nn_create_out: " + self.lib.lddmm_bl_last_error(None).decode())
        self.h = h
        osz, oc, npar = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int64()
        self._check(self.lib.lddmm_nn_info(self.h, ctypes.byref(osz), ctypes.byref(oc), ctypes.byref(npar)), "info")
        self.out_size, self.nparam = osz.value, npar.value

    def close(self):
        if getattr(self, "h", None):
            self.lib.lddmm_nn_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, st, what):
        if st != 0:
            raise LddmmError(st, f"lddmm_nn_{what}: " + self.lib.lddmm_bl_last_error(None).decode())

    def _order(self):
        cur = torch.cuda.current_stream(self.device)
        if cur != self.stream:
            self.stream.wait_stream(cur)

    def _dev(self, t, shape, name):
        if not isinstance(t, torch.Tensor) or t.device.type != "cuda" or t.dtype != torch.float32:
            raise TypeError(f"{name} must be a float32 ROCm tensor")
        if shape is not None and tuple(t.shape) != tuple(shape):
            raise ValueError(f"{name} has shape {tuple(t.shape)}, expected {tuple(shape)}")
        if not t.is_contiguous():
            raise ValueError(f"{name} must be contiguous")
        return t

    def out_shape(self, B):
        return (B, 3 * (1 + self.rank_r)) + (self.out_size,) * 3

    def pool_pair(self, I0, I1, slot):
        """Box-average an image pair into one input slot [2][in_size]^3 (a view of the batch tensor)."""
        self._dev(I0, None, "I0")
        self._dev(I1, tuple(I0.shape), "I1")
        self._dev(slot, (2,) + (self.in_size,) * 3, "slot")
        n = (ctypes.c_int32 * 3)(*I0.shape)
        self._order()
        self._check(self.lib.lddmm_nn_pool_pair(self.h, _ptr(I0), _ptr(I1), n, _ptr(slot)), "pool_pair")

    def forward(self, x):
        B = x.shape[0]
        self._dev(x, (B, 2) + (self.in_size,) * 3, "x")
        out = torch.empty(self.out_shape(B), dtype=torch.float32, device=self.device)
        self._order()
        self._check(self.lib.lddmm_nn_forward(self.h, _ptr(x), B, _ptr(out)), "forward")
        return out

    def backward(self, dout):
        self._dev(dout, None, "dout")
        self._order()
        self._check(self.lib.lddmm_nn_backward(self.h, _ptr(dout), dout.shape[0]), "backward")

    def zero_grad(self):
        self._check(self.lib.lddmm_nn_zero_grad(self.h), "zero_grad")

    def step(self, lr):
        self._check(self.lib.lddmm_nn_step(self.h, float(lr)), "step")

    def velocity(self, out, K):
        """Band-limited coefficients of the outputs: [B][3][K] (rank_r = 0) or [B][1 + r][3][K]."""
        B = out.shape[0]
        self._dev(out, self.out_shape(B), "out")
        v = torch.empty((B, 1 + self.rank_r, 3) + tuple(K), dtype=torch.float32, device=self.device)
        k = (ctypes.c_int32 * 3)(*K)
        self._order()
        self._check(self.lib.lddmm_nn_velocity(self.h, _ptr(out), B, k, _ptr(v)), "velocity")
        return v[:, 0] if self.rank_r == 0 else v

    def save(self, path):
        """Write the architecture and master parameters (lddmm_nn_save)."""
        self._check(self.lib.lddmm_nn_save(self.h, os.fsencode(path)), "save")

    def load(self, path):
        """Read parameters written by save into this network (same architecture)."""
        self._check(self.lib.lddmm_nn_load(self.h, os.fsencode(path)), "load")

    def loss(self, out, v_target, alpha=0.0025, s=2, want_grad=True):
        B = out.shape[0]
        self._dev(out, self.out_shape(B), "out")
        self._dev(v_target, None, "v_target")
        if v_target.dim() != 5 or v_target.shape[:2] != (B, 3):
            raise ValueError("v_target must be [B][3][K0][K1][K2]")
        dout = torch.empty_like(out) if want_grad else None
        k = (ctypes.c_int32 * 3)(*v_target.shape[2:])
        r = ctypes.c_double()
        self._order()
        self._check(self.lib.lddmm_nn_loss(self.h, _ptr(out), _ptr(v_target), B, k, alpha, s, _ptr(dout),
                                           ctypes.byref(r)), "loss")
        return r.value, dout

    def get(self, which=0):
        import numpy as np
        buf = np.empty(self.nparam, dtype=np.float32)
        self._check(self.lib.lddmm_nn_get(self.h, which, buf.ctypes.data_as(ctypes.c_void_p)), "get")
        return buf

    def set(self, params):
        import numpy as np
        buf = np.ascontiguousarray(params, dtype=np.float32)
        if buf.size != self.nparam:
            raise ValueError(f"expected {self.nparam} parameters, got {buf.size}")
        self._check(self.lib.lddmm_nn_set(self.h, buf.ctypes.data_as(ctypes.c_void_p)), "set")
