"""Python binding of libfresco (ctypes over the C ABI in include/fresco.h).

Argument marshalling only: every step of an evaluation runs in the HIP
library.  Device buffers are torch tensors on a HIP device (torch is used for
memory and streams); if the compiled library is missing, importing this module
raises -- there is no fallback.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# FRESCO_LIB: an alternative build of the library to load (the host-sanitizer
# run of the argument checks uses one); by default libfresco.so beside this file
LIB_PATH = os.environ.get("FRESCO_LIB") or os.path.join(_HERE, "libfresco.so")

F32, F64 = 0, 1
WEIGHT_ABS, WEIGHT_RELATIVE = 0, 1
OK, EINVAL, ENOMEM, EHIP, ENOTSUP, ENONFINITE, ELINESEARCH = 0, -1, -2, -3, -4, -5, -6
STAGES = ["bin", "spread", "fold", "fft_rows_fwd", "fft_cols_fwd", "modes", "fft_cols_inv",
          "fft_rows_inv", "interp"]
# stages made of exactly one kernel launch
SINGLE_KERNEL_STAGES = ["spread", "fold", "fft_rows_fwd", "fft_cols_fwd", "modes",
                        "fft_cols_inv", "fft_rows_inv", "interp"]


class FrescoError(RuntimeError):
    def __init__(self, code: int, where: str):
        self.code = code
        msg = _lib.fresco_error_string(code).decode() if _lib is not None else str(code)
        hip = _lib.fresco_last_hip_error() if _lib is not None else 0
        super().__init__(f"{where}: {msg} (status {code}, last hipError {hip})")


class Problem(ctypes.Structure):
    _fields_ = [
        ("dim", ctypes.c_int32),
        ("dtype", ctypes.c_int32),
        ("n", ctypes.c_int64),
        ("box", ctypes.c_double * 3),
        ("kmax", ctypes.c_int32 * 3),
        ("k_cut", ctypes.c_double),
        ("s0", ctypes.POINTER(ctypes.c_double)),
        ("w", ctypes.POINTER(ctypes.c_double)),
        ("weight_mode", ctypes.c_int32),
        ("tol", ctypes.c_double),
        ("upsampfac", ctypes.c_double),
    ]


class PlanInfo(ctypes.Structure):
    _fields_ = [
        ("dim", ctypes.c_int32),
        ("dtype", ctypes.c_int32),
        ("n", ctypes.c_int64),
        ("nf", ctypes.c_int32 * 3),
        ("kmax", ctypes.c_int32 * 3),
        ("width", ctypes.c_int32),
        ("beta", ctypes.c_double),
        ("tile", ctypes.c_int32 * 3),
        ("nbins", ctypes.c_int64),
        ("n_constrained", ctypes.c_int64),
        ("device_bytes", ctypes.c_int64),
        ("col_split", ctypes.c_int32),
        ("bin_ranges", ctypes.c_int32),
        ("bin_levels", ctypes.c_int32),
        ("slack", ctypes.c_int32),
    ]


class PairProblem(ctypes.Structure):
    _fields_ = [
        ("dim", ctypes.c_int32),
        ("dtype", ctypes.c_int32),
        ("n", ctypes.c_int64),
        ("box", ctypes.c_double * 3),
        ("sigma", ctypes.c_double),
        ("eps", ctypes.c_double),
        ("alpha", ctypes.c_double),
    ]


class LbfgsOpts(ctypes.Structure):
    _fields_ = [
        ("m", ctypes.c_int32),
        ("max_backtracks", ctypes.c_int32),
        ("max_step", ctypes.c_double),
        ("c1", ctypes.c_double),
        ("shrink", ctypes.c_double),
        ("gtol", ctypes.c_double),
    ]


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built; run python -m paper_2305_15693_amd.build")
    lib = ctypes.CDLL(LIB_PATH)
    vp = ctypes.c_void_p
    i = ctypes.c_int
    lib.fresco_create.argtypes = [ctypes.POINTER(vp), ctypes.POINTER(Problem), vp]
    lib.fresco_create.restype = i
    lib.fresco_destroy.argtypes = [vp]
    lib.fresco_destroy.restype = i
    lib.fresco_plan_info_get.argtypes = [vp, ctypes.POINTER(PlanInfo)]
    lib.fresco_plan_info_get.restype = i
    lib.fresco_structure_factor.argtypes = [vp, vp, vp]
    lib.fresco_structure_factor.restype = i
    lib.fresco_structure_factor_backward.argtypes = [vp, vp, vp, vp, ctypes.c_int32]
    lib.fresco_structure_factor_backward.restype = i
    lib.fresco_loss_grad.argtypes = [vp, vp, ctypes.POINTER(ctypes.c_double), vp]
    lib.fresco_loss_grad.restype = i
    lib.fresco_loss_grad_async.argtypes = [vp, vp, vp, vp]
    lib.fresco_loss_grad_async.restype = i
    lib.fresco_step.argtypes = [vp, vp, ctypes.POINTER(LbfgsOpts), ctypes.c_int32,
                                ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int32)]
    lib.fresco_step.restype = i
    lib.fresco_reset_history.argtypes = [vp]
    lib.fresco_reset_history.restype = i
    dpp = ctypes.POINTER(ctypes.c_double)
    lib.fresco_set_target.argtypes = [vp, dpp, dpp, ctypes.c_double, ctypes.c_int32]
    lib.fresco_set_target.restype = i
    lib.fresco_step_sequence.argtypes = [vp, vp, ctypes.c_int32, ctypes.POINTER(dpp),
                                         ctypes.POINTER(dpp),
                                         ctypes.c_double, ctypes.c_int32,
                                         ctypes.POINTER(LbfgsOpts), ctypes.c_int32, dpp,
                                         ctypes.POINTER(ctypes.c_int32), vp]
    lib.fresco_step_sequence.restype = i
    lib.fresco_pair_replace_overlaps.argtypes = [vp, vp, ctypes.c_double, vp, ctypes.c_int64,
                                                 ctypes.POINTER(ctypes.c_int64)]
    lib.fresco_pair_replace_overlaps.restype = i
    lib.fresco_overlap_cycles.argtypes = [vp, vp, vp, ctypes.POINTER(LbfgsOpts), ctypes.c_int32,
                                          ctypes.c_int32, ctypes.c_double, vp, ctypes.c_int64,
                                          dpp, ctypes.POINTER(ctypes.c_int32),
                                          ctypes.POINTER(ctypes.c_int64)]
    lib.fresco_overlap_cycles.restype = i
    lib.fresco_q_create.argtypes = [ctypes.POINTER(vp), ctypes.c_int32, ctypes.c_int32,
                                    ctypes.c_int64, ctypes.c_int64, vp]
    lib.fresco_q_create.restype = i
    lib.fresco_q_destroy.argtypes = [vp]
    lib.fresco_q_destroy.restype = i
    lib.fresco_q_set.argtypes = [vp, ctypes.c_int64, dpp, dpp, dpp]
    lib.fresco_q_set.restype = i
    lib.fresco_q_structure_factor.argtypes = [vp, vp, vp, vp, vp]
    lib.fresco_q_structure_factor.restype = i
    lib.fresco_q_loss_grad.argtypes = [vp, vp, vp, ctypes.POINTER(ctypes.c_double), vp]
    lib.fresco_q_loss_grad.restype = i
    lib.fresco_q_loss_grad_strengths.argtypes = [vp, vp, vp, ctypes.POINTER(ctypes.c_double), vp]
    lib.fresco_q_loss_grad_strengths.restype = i
    lib.fresco_ewald_transmission.argtypes = [vp, vp, vp, ctypes.c_int32, dpp, ctypes.c_int32,
                                              dpp, ctypes.c_int32, dpp]
    lib.fresco_ewald_transmission.restype = i
    lib.fresco_q_last_hip_error.argtypes = [vp]
    lib.fresco_q_last_hip_error.restype = i
    lib.fresco_set_pair_correlation_target.argtypes = [vp, dpp, dpp]
    lib.fresco_set_pair_correlation_target.restype = i
    lib.fresco_pair_correlation_loss_grad.argtypes = [vp, vp, ctypes.POINTER(ctypes.c_double),
                                                      vp, vp]
    lib.fresco_pair_correlation_loss_grad.restype = i
    lib.fresco_set_strengths.argtypes = [vp, vp]
    lib.fresco_set_strengths.restype = i
    lib.fresco_loss_grad_strengths.argtypes = [vp, vp, ctypes.POINTER(ctypes.c_double), vp, vp]
    lib.fresco_loss_grad_strengths.restype = i
    lib.fresco_set_timing.argtypes = [vp, ctypes.c_uint32]
    lib.fresco_set_timing.restype = i
    lib.fresco_set_timing_reps.argtypes = [vp, ctypes.c_int32]
    lib.fresco_set_timing_reps.restype = i
    lib.fresco_read_timing.argtypes = [vp, ctypes.POINTER(ctypes.c_double),
                                       ctypes.POINTER(ctypes.c_int64), i]
    lib.fresco_read_timing.restype = i
    lib.fresco_pair_create.argtypes = [ctypes.POINTER(vp), ctypes.POINTER(PairProblem), vp]
    lib.fresco_pair_create.restype = i
    lib.fresco_pair_destroy.argtypes = [vp]
    lib.fresco_pair_destroy.restype = i
    lib.fresco_pair_energy_grad.argtypes = [vp, vp, ctypes.POINTER(ctypes.c_double), vp]
    lib.fresco_pair_energy_grad.restype = i
    lib.fresco_pair_energy_grad_async.argtypes = [vp, vp, vp, vp]
    lib.fresco_pair_energy_grad_async.restype = i
    lib.fresco_pair_energy_grad_noalloc.argtypes = [ctypes.POINTER(PairProblem), vp, vp, vp, vp]
    lib.fresco_pair_energy_grad_noalloc.restype = i
    lib.fresco_attach_pair.argtypes = [vp, vp, ctypes.c_double]
    lib.fresco_attach_pair.restype = i
    lib.fresco_batch_create.argtypes = [ctypes.POINTER(vp), ctypes.c_int32,
                                        ctypes.POINTER(Problem), vp]
    lib.fresco_batch_create.restype = i
    lib.fresco_batch_destroy.argtypes = [vp]
    lib.fresco_batch_destroy.restype = i
    lib.fresco_batch_offsets.argtypes = [vp, ctypes.POINTER(ctypes.c_int64)]
    lib.fresco_batch_offsets.restype = i
    lib.fresco_batch_loss_grad.argtypes = [vp, vp, ctypes.POINTER(ctypes.c_double), vp]
    lib.fresco_batch_loss_grad.restype = i
    lib.fresco_batch_loss_grad_async.argtypes = [vp, vp, vp, vp]
    lib.fresco_batch_loss_grad_async.restype = i
    lib.fresco_batch_step.argtypes = [vp, vp, ctypes.POINTER(LbfgsOpts), ctypes.c_int32,
                                      ctypes.POINTER(ctypes.c_double),
                                      ctypes.POINTER(ctypes.c_int32)]
    lib.fresco_batch_step.restype = i
    lib.fresco_batch_reset_history.argtypes = [vp]
    lib.fresco_batch_reset_history.restype = i
    lib.fresco_batch_autotune.argtypes = [vp, vp, vp, ctypes.c_int32,
                                          ctypes.POINTER(ctypes.c_int32)]
    lib.fresco_batch_autotune.restype = i
    lib.fresco_batch_last_hip_error.argtypes = []
    lib.fresco_batch_last_hip_error.restype = i
    lib.fresco_error_string.argtypes = [i]
    lib.fresco_error_string.restype = ctypes.c_char_p
    lib.fresco_last_hip_error.argtypes = []
    lib.fresco_last_hip_error.restype = i
    return lib


_lib = _load()


def lib():
    return _lib


def _check(code: int, where: str):
    if code != OK:
        raise FrescoError(code, where)


def _torch():
    import torch
    return torch


class Context:
    """One problem (box, mode cube, targets, weights, accuracy) bound to a stream.

    w_cube / s0_cube: host arrays on the mode cube (2M_0+1, ..., 2M_{d-1}+1), C order
    (see include/fresco.h).  When w_cube is None the weight is 1 on 0 < |n| <= k_cut.
    """

    def __init__(self, dim: int, n: int, box, kmax, *, w_cube=None, s0_cube=None,
                 k_cut: float = 0.0, relative: bool = False, tol: float = 1e-6,
                 dtype: str = "f32", stream=None, device=None):
        torch = _torch()
        self.dim = int(dim)
        self.n = int(n)
        self.dtype = dtype
        self.torch_dtype = torch.float32 if dtype == "f32" else torch.float64
        self.device = torch.device(device) if device is not None else torch.device("cuda", torch.cuda.current_device())
        box = np.broadcast_to(np.asarray(box, dtype=np.float64), (self.dim,))
        kmax = np.broadcast_to(np.asarray(kmax, dtype=np.int64), (self.dim,))
        self.box = tuple(float(x) for x in box)
        self.kmax = tuple(int(x) for x in kmax)
        self.cube_shape = tuple(2 * m + 1 for m in self.kmax)
        p = Problem()
        p.dim = self.dim
        p.dtype = F32 if dtype == "f32" else F64
        p.n = self.n
        for a in range(3):
            p.box[a] = self.box[a] if a < self.dim else 1.0
            p.kmax[a] = self.kmax[a] if a < self.dim else 0
        p.k_cut = float(k_cut)
        self._w = self._s0 = None
        if w_cube is not None:
            self._w = np.ascontiguousarray(np.asarray(w_cube, dtype=np.float64).reshape(self.cube_shape))
            p.w = self._w.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        if s0_cube is not None:
            self._s0 = np.ascontiguousarray(np.asarray(s0_cube, dtype=np.float64).reshape(self.cube_shape))
            p.s0 = self._s0.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        p.weight_mode = WEIGHT_RELATIVE if relative else WEIGHT_ABS
        p.tol = float(tol)
        p.upsampfac = 2.0
        if stream is None:
            stream = torch.cuda.current_stream(self.device)
        self.stream = stream
        h = ctypes.c_void_p()
        with torch.cuda.device(self.device):
            _check(_lib.fresco_create(ctypes.byref(h), ctypes.byref(p), ctypes.c_void_p(stream.cuda_stream)),
                   "fresco_create")
        self._h = h
        self._loss = ctypes.c_double(0.0)
        self._calls = 0          # calls that took positions (each may replace the held state)
        self._sf_token = None

    # ------------------------------------------------------------------
    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            _lib.fresco_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def handle(self):
        return self._h

    def plan_info(self) -> dict:
        info = PlanInfo()
        _check(_lib.fresco_plan_info_get(self._h, ctypes.byref(info)), "fresco_plan_info_get")
        d = self.dim
        return dict(dim=info.dim, dtype=info.dtype, n=info.n, nf=list(info.nf)[:d],
                    kmax=list(info.kmax)[:d], width=info.width, beta=info.beta,
                    tile=list(info.tile)[:d], nbins=info.nbins,
                    n_constrained=info.n_constrained, device_bytes=info.device_bytes,
                    col_split=info.col_split, bin_ranges=info.bin_ranges,
                    bin_levels=info.bin_levels, slack=info.slack)

    def default_max_step(self) -> float:
        """0.1 of the mean interparticle spacing L / N^(1/d) (smallest side)."""
        return 0.1 * min(self.box) / self.n ** (1.0 / self.dim)

    def step(self, pos, n_iter: int, *, m: int = 8, max_step: float = None, c1: float = 1e-4,
             shrink: float = 0.5, max_backtracks: int = 20, gtol: float = 0.0):
        """n_iter L-BFGS iterations on pos (updated in place).  Returns (loss, evaluations)."""
        o = LbfgsOpts()
        o.m = m
        o.max_backtracks = max_backtracks
        o.max_step = self.default_max_step() if max_step is None else float(max_step)
        o.c1 = c1
        o.shrink = shrink
        o.gtol = gtol
        loss = ctypes.c_double(0.0)
        nev = ctypes.c_int32(0)
        _check(_lib.fresco_step(self._h, self._pos(pos), ctypes.byref(o), int(n_iter),
                                ctypes.byref(loss), ctypes.byref(nev)), "fresco_step")
        return float(loss.value), int(nev.value)

    def attach_pair(self, pair, weight: float = 1.0):
        """Add weight * E of a PairContext to every loss evaluation (None detaches)."""
        _check(_lib.fresco_attach_pair(self._h, pair.handle if pair is not None else None,
                                       float(weight)), "fresco_attach_pair")
        self._pair = pair  # keep it alive while attached

    def reset_history(self):
        _check(_lib.fresco_reset_history(self._h), "fresco_reset_history")

    def _cube(self, a):
        if a is None:
            return None, None
        arr = np.ascontiguousarray(np.asarray(a, dtype=np.float64).reshape(self.cube_shape))
        return arr, arr.ctypes.data_as(ctypes.POINTER(ctypes.c_double))

    def _opts(self, m=8, max_step=None, c1=1e-4, shrink=0.5, max_backtracks=20, gtol=0.0):
        o = LbfgsOpts()
        o.m = m
        o.max_backtracks = max_backtracks
        o.max_step = self.default_max_step() if max_step is None else float(max_step)
        o.c1 = c1
        o.shrink = shrink
        o.gtol = gtol
        return o

    def set_target(self, s0_cube=None, w_cube=None, k_cut: float = 0.0, relative: bool = False):
        """New target and weights for the same geometry (fresco_set_target)."""
        s0, s0p = self._cube(s0_cube)
        w, wp = self._cube(w_cube)
        _check(_lib.fresco_set_target(self._h, s0p, wp, float(k_cut),
                                      WEIGHT_RELATIVE if relative else WEIGHT_ABS),
               "fresco_set_target")

    def step_sequence(self, pos, n_iter: int, *, s0_cubes=None, w_cubes=None, k_cut: float = 0.0,
                      relative: bool = False, frames: bool = True, **opts):
        """Warm-started minimisations over a sequence of targets (fresco_step_sequence):
        per-frame lists of S0 and weight cubes (either may be None: S0 = 0, or weight 1
        on 0 < |n| <= k_cut).  Returns (losses, evaluations, frames [T][n][d] or None)."""
        torch = _torch()
        T = len(s0_cubes) if s0_cubes is not None else len(w_cubes)

        def table(cubes):
            if cubes is None:
                return [], None
            keep = [self._cube(c) for c in cubes]
            return keep, (ctypes.POINTER(ctypes.c_double) * max(T, 1))(*[k[1] for k in keep])

        ks, s0a = table(s0_cubes)
        kw, wa = table(w_cubes)
        losses = (ctypes.c_double * max(T, 1))()
        nev = (ctypes.c_int32 * max(T, 1))()
        fr = (torch.empty((T, self.n, self.dim), dtype=self.torch_dtype, device=self.device)
              if frames else None)
        o = self._opts(**opts)
        _check(_lib.fresco_step_sequence(self._h, self._pos(pos), T, s0a, wa, float(k_cut),
                                         WEIGHT_RELATIVE if relative else WEIGHT_ABS,
                                         ctypes.byref(o), int(n_iter), losses, nev,
                                         ctypes.c_void_p(fr.data_ptr()) if fr is not None else None),
               "fresco_step_sequence")
        del ks, kw
        return list(losses)[:T], list(nev)[:T], fr

    def overlap_cycles(self, pair, pos, n_iter: int, max_cycles: int, threshold: float, fresh,
                       **opts):
        """Minimisation / overlap-removal cycles (fresco_overlap_cycles).  fresh: [m][d]
        replacement positions.  Returns (loss, cycles, replaced)."""
        o = self._opts(**opts)
        loss = ctypes.c_double(0.0)
        cyc = ctypes.c_int32(0)
        rep = ctypes.c_int64(0)
        _check(_lib.fresco_overlap_cycles(self._h, pair.handle, self._pos(pos), ctypes.byref(o),
                                          int(n_iter), int(max_cycles), float(threshold),
                                          ctypes.c_void_p(fresh.data_ptr()), int(fresh.shape[0]),
                                          ctypes.byref(loss), ctypes.byref(cyc), ctypes.byref(rep)),
               "fresco_overlap_cycles")
        return float(loss.value), int(cyc.value), int(rep.value)

    def grid_shape(self):
        """Shape of arrays on the fine grid, C order (axis 0 fastest): (nf_{d-1}, ..., nf_0)."""
        return tuple(reversed(self.plan_info()["nf"]))

    def set_pair_correlation_target(self, g0=None, wg=None):
        """Target g0 and weights W_g of the pair-correlation loss on the fine grid
        (arrays of grid_shape(); wg None disables the term)."""
        shape = self.grid_shape()
        a = None if g0 is None else np.ascontiguousarray(np.asarray(g0, np.float64).reshape(shape))
        b = None if wg is None else np.ascontiguousarray(np.asarray(wg, np.float64).reshape(shape))
        dp = ctypes.POINTER(ctypes.c_double)
        _check(_lib.fresco_set_pair_correlation_target(
            self._h, None if a is None else a.ctypes.data_as(dp),
            None if b is None else b.ctypes.data_as(dp)), "fresco_set_pair_correlation_target")

    def pair_correlation_loss_grad(self, pos, grad=None, want_g: bool = False):
        """(L_g, dL_g/dr [n][d], g on the fine grid or None)."""
        torch = _torch()
        if grad is None:
            grad = torch.empty((self.n, self.dim), dtype=self.torch_dtype, device=self.device)
        g = (torch.empty(self.grid_shape(), dtype=self.torch_dtype, device=self.device)
             if want_g else None)
        _check(_lib.fresco_pair_correlation_loss_grad(
            self._h, self._pos(pos), ctypes.byref(self._loss), ctypes.c_void_p(grad.data_ptr()),
            ctypes.c_void_p(g.data_ptr()) if g is not None else None),
            "fresco_pair_correlation_loss_grad")
        return float(self._loss.value), grad, g

    def set_strengths(self, c):
        """Point strengths for every later evaluation (a [n] tensor of the context's
        dtype on its device; the context keeps a copy), or None for unit strengths."""
        if c is None:
            _check(_lib.fresco_set_strengths(self._h, None), "fresco_set_strengths")
            return
        if c.device != self.device or c.dtype != self.torch_dtype or c.numel() != self.n \
                or not c.is_contiguous():
            raise ValueError(f"strengths must be a contiguous [{self.n}] {self.torch_dtype} "
                             f"tensor on {self.device}")
        _check(_lib.fresco_set_strengths(self._h, ctypes.c_void_p(c.data_ptr())),
               "fresco_set_strengths")

    def loss_grad_strengths(self, pos, grad=None, grad_c=None):
        """(loss, dL/dr [n][d], dL/dc [n]) with the strengths set on the context."""
        torch = _torch()
        if grad is None:
            grad = torch.empty((self.n, self.dim), dtype=self.torch_dtype, device=self.device)
        if grad_c is None:
            grad_c = torch.empty((self.n,), dtype=self.torch_dtype, device=self.device)
        _check(_lib.fresco_loss_grad_strengths(self._h, self._pos(pos), ctypes.byref(self._loss),
                                               ctypes.c_void_p(grad.data_ptr()),
                                               ctypes.c_void_p(grad_c.data_ptr())),
               "fresco_loss_grad_strengths")
        return float(self._loss.value), grad, grad_c

    def set_timing(self, stages, reps: int = 1):
        """Bracket the named stages (see STAGES) with HIP events; [] turns it off.
        reps: launches of the spread and interp kernels per bracket (timing only)."""
        mask = 0
        for s in stages:
            mask |= 1 << STAGES.index(s)
        _check(_lib.fresco_set_timing(self._h, mask), "fresco_set_timing")
        _check(_lib.fresco_set_timing_reps(self._h, int(reps)), "fresco_set_timing_reps")

    def read_timing(self, reset: bool = True) -> dict:
        """{stage: (total ms, timed evaluations)} since the last reset."""
        ms = (ctypes.c_double * len(STAGES))()
        cnt = (ctypes.c_int64 * len(STAGES))()
        _check(_lib.fresco_read_timing(self._h, ms, cnt, 1 if reset else 0), "fresco_read_timing")
        return {STAGES[s]: (ms[s], cnt[s]) for s in range(len(STAGES)) if cnt[s]}

    def _pos(self, pos):
        if pos.device != self.device or pos.dtype != self.torch_dtype:
            raise ValueError(f"positions must be {self.torch_dtype} on {self.device}")
        if tuple(pos.shape) != (self.n, self.dim) or not pos.is_contiguous():
            raise ValueError(f"positions must be a contiguous [{self.n}][{self.dim}] tensor")
        self._calls += 1
        return ctypes.c_void_p(pos.data_ptr())

    def structure_factor(self, pos, out=None):
        torch = _torch()
        if out is None:
            out = torch.empty(self.cube_shape, dtype=self.torch_dtype, device=self.device)
        _check(_lib.fresco_structure_factor(self._h, self._pos(pos), ctypes.c_void_p(out.data_ptr())),
               "fresco_structure_factor")
        self._sf_token = (self._calls, pos.data_ptr())
        return out

    def sf_token(self):
        """Identifies the latest structure_factor call while no other call has run."""
        return self._sf_token

    def structure_factor_backward(self, pos, gS, grad=None, token=None):
        """grad = sum_n gS(n) dS(n)/dr (backward of structure_factor; see
        fresco_structure_factor_backward).  gS: mode cube of dF/dS.  token: the
        sf_token() taken right after the forward call; when no other call has run
        on this context since, the forward's state is reused, else recomputed."""
        torch = _torch()
        if (gS.device != self.device or gS.dtype != self.torch_dtype
                or tuple(gS.shape) != self.cube_shape or not gS.is_contiguous()):
            raise ValueError(f"gS must be a contiguous {self.cube_shape} {self.torch_dtype} tensor "
                             f"on {self.device}")
        if grad is None:
            grad = torch.empty((self.n, self.dim), dtype=self.torch_dtype, device=self.device)
        reuse = token is not None and token == self._sf_token and token[0] == self._calls \
            and token[1] == pos.data_ptr()
        _check(_lib.fresco_structure_factor_backward(self._h, self._pos(pos),
                                                     ctypes.c_void_p(gS.data_ptr()),
                                                     ctypes.c_void_p(grad.data_ptr()),
                                                     1 if reuse else 0),
               "fresco_structure_factor_backward")
        return grad

    def loss_grad(self, pos, grad=None):
        torch = _torch()
        if grad is None:
            grad = torch.empty((self.n, self.dim), dtype=self.torch_dtype, device=self.device)
        _check(_lib.fresco_loss_grad(self._h, self._pos(pos), ctypes.byref(self._loss),
                                     ctypes.c_void_p(grad.data_ptr())), "fresco_loss_grad")
        return float(self._loss.value), grad

    def loss_grad_async(self, pos, loss_dev, grad):
        _check(_lib.fresco_loss_grad_async(self._h, self._pos(pos), ctypes.c_void_p(loss_dev.data_ptr()),
                                           ctypes.c_void_p(grad.data_ptr())), "fresco_loss_grad_async")
        return loss_dev, grad


def pair_energy_grad_noalloc(pos, energy_dev, grad, box, *, sigma: float = 0.5, eps: float = 1.0,
                             alpha: float = 2.0, stream=None):
    """Pair energy (into the device double energy_dev) and gradient (into grad) at
    pos without a pair context and without any allocation (the library's fixed
    scratch; include/fresco.h, fresco_pair_energy_grad_noalloc).  pos and grad are
    [n][d] tensors of one dtype on the current device; enqueued on stream
    (default: the current stream)."""
    torch = _torch()
    n, dim = int(pos.shape[0]), int(pos.shape[1])
    if pos.dtype not in (torch.float32, torch.float64) or grad.dtype != pos.dtype:
        raise ValueError("pos and grad must both be float32 or both float64")
    if tuple(grad.shape) != (n, dim) or not pos.is_contiguous() or not grad.is_contiguous():
        raise ValueError("pos and grad must be contiguous [n][d] tensors")
    if energy_dev.dtype != torch.float64 or energy_dev.numel() < 1:
        raise ValueError("energy_dev must hold a float64")
    box = np.broadcast_to(np.asarray(box, dtype=np.float64), (dim,))
    p = PairProblem()
    p.dim = dim
    p.dtype = F32 if pos.dtype == torch.float32 else F64
    p.n = n
    for a in range(3):
        p.box[a] = float(box[a]) if a < dim else 1.0
    p.sigma, p.eps, p.alpha = float(sigma), float(eps), float(alpha)
    if stream is None:
        stream = torch.cuda.current_stream(pos.device)
    _check(_lib.fresco_pair_energy_grad_noalloc(ctypes.byref(p), ctypes.c_void_p(pos.data_ptr()),
                                                ctypes.c_void_p(energy_dev.data_ptr()),
                                                ctypes.c_void_p(grad.data_ptr()),
                                                ctypes.c_void_p(stream.cuda_stream)),
           "fresco_pair_energy_grad_noalloc")
    return energy_dev, grad


class QContext:
    """Structure factor, NUwNU loss and Ewald transmission at arbitrary wave vectors
    with free boundary conditions (include/fresco.h, fresco_q_*)."""

    def __init__(self, dim: int, n: int, max_q: int, *, dtype: str = "f32", stream=None,
                 device=None):
        torch = _torch()
        self.dim, self.n, self.max_q, self.dtype = int(dim), int(n), int(max_q), dtype
        self.torch_dtype = torch.float32 if dtype == "f32" else torch.float64
        self.device = torch.device(device) if device is not None else torch.device("cuda", torch.cuda.current_device())
        if stream is None:
            stream = torch.cuda.current_stream(self.device)
        self.stream = stream
        self.K = 0
        h = ctypes.c_void_p()
        with torch.cuda.device(self.device):
            _check(_lib.fresco_q_create(ctypes.byref(h), self.dim, F32 if dtype == "f32" else F64,
                                        self.n, self.max_q, ctypes.c_void_p(stream.cuda_stream)),
                   "fresco_q_create")
        self._h = h

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            _lib.fresco_q_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _pos(self, pos):
        if pos.device != self.device or pos.dtype != self.torch_dtype:
            raise ValueError(f"positions must be {self.torch_dtype} on {self.device}")
        if tuple(pos.shape) != (self.n, self.dim) or not pos.is_contiguous():
            raise ValueError(f"positions must be a contiguous [{self.n}][{self.dim}] tensor")
        return ctypes.c_void_p(pos.data_ptr())

    def _c(self, c):
        if c is None:
            return None
        if c.device != self.device or c.dtype != self.torch_dtype or c.numel() != self.n:
            raise ValueError("strengths must be [n] of the context's dtype on its device")
        return ctypes.c_void_p(c.data_ptr())

    def set(self, q, W=None, S0=None):
        dp = ctypes.POINTER(ctypes.c_double)
        q = np.ascontiguousarray(np.asarray(q, np.float64).reshape(-1, self.dim))
        K = len(q)
        Wa = None if W is None else np.ascontiguousarray(np.asarray(W, np.float64).ravel())
        Sa = None if S0 is None else np.ascontiguousarray(np.asarray(S0, np.float64).ravel())
        _check(_lib.fresco_q_set(self._h, K, q.ctypes.data_as(dp),
                                 None if Wa is None else Wa.ctypes.data_as(dp),
                                 None if Sa is None else Sa.ctypes.data_as(dp)), "fresco_q_set")
        self.K = K

    def structure_factor(self, pos, c=None, want_rho: bool = False):
        torch = _torch()
        S = torch.empty(self.K, dtype=torch.float64, device=self.device)
        rho = torch.empty((self.K, 2), dtype=torch.float64, device=self.device) if want_rho else None
        _check(_lib.fresco_q_structure_factor(self._h, self._pos(pos), self._c(c),
                                              ctypes.c_void_p(S.data_ptr()),
                                              ctypes.c_void_p(rho.data_ptr()) if want_rho else None),
               "fresco_q_structure_factor")
        return (S, rho) if want_rho else S

    def loss_grad(self, pos, c=None, grad=None):
        torch = _torch()
        if grad is None:
            grad = torch.empty((self.n, self.dim), dtype=self.torch_dtype, device=self.device)
        loss = ctypes.c_double(0.0)
        _check(_lib.fresco_q_loss_grad(self._h, self._pos(pos), self._c(c), ctypes.byref(loss),
                                       ctypes.c_void_p(grad.data_ptr())), "fresco_q_loss_grad")
        return float(loss.value), grad

    def loss_grad_strengths(self, pos, c, grad_c=None):
        """(loss, dL/dc [n]) for the weights c of the points (fresco_q_loss_grad_strengths)."""
        torch = _torch()
        if grad_c is None:
            grad_c = torch.empty(self.n, dtype=self.torch_dtype, device=self.device)
        loss = ctypes.c_double(0.0)
        _check(_lib.fresco_q_loss_grad_strengths(self._h, self._pos(pos), self._c(c),
                                                 ctypes.byref(loss),
                                                 ctypes.c_void_p(grad_c.data_ptr())),
               "fresco_q_loss_grad_strengths")
        return float(loss.value), grad_c

    def ewald_transmission(self, pos, k, dirs, ns: int, c=None):
        """T[n_k][n_dir] of the Ewald construction (fresco_ewald_transmission)."""
        dp = ctypes.POINTER(ctypes.c_double)
        k = np.ascontiguousarray(np.asarray(k, np.float64).ravel())
        dirs = np.ascontiguousarray(np.asarray(dirs, np.float64).reshape(-1, self.dim))
        T = np.zeros((len(k), len(dirs)))
        _check(_lib.fresco_ewald_transmission(self._h, self._pos(pos), self._c(c), len(k),
                                              k.ctypes.data_as(dp), len(dirs),
                                              dirs.ctypes.data_as(dp), int(ns), T.ctypes.data_as(dp)),
               "fresco_ewald_transmission")
        self.K = 0
        return T


class PairContext:
    """Soft-core repulsion U = (eps/alpha)(1 - r/sigma)^alpha, r < sigma, on a cell
    list (include/fresco.h, fresco_pair_*)."""

    def __init__(self, dim: int, n: int, box, *, sigma: float = 0.5, eps: float = 1.0,
                 alpha: float = 2.0, dtype: str = "f32", stream=None, device=None):
        torch = _torch()
        self.dim = int(dim)
        self.n = int(n)
        self.dtype = dtype
        self.torch_dtype = torch.float32 if dtype == "f32" else torch.float64
        self.device = torch.device(device) if device is not None else torch.device("cuda", torch.cuda.current_device())
        box = np.broadcast_to(np.asarray(box, dtype=np.float64), (self.dim,))
        p = PairProblem()
        p.dim = self.dim
        p.dtype = F32 if dtype == "f32" else F64
        p.n = self.n
        for a in range(3):
            p.box[a] = float(box[a]) if a < self.dim else 1.0
        p.sigma, p.eps, p.alpha = float(sigma), float(eps), float(alpha)
        if stream is None:
            stream = torch.cuda.current_stream(self.device)
        self.stream = stream
        h = ctypes.c_void_p()
        with torch.cuda.device(self.device):
            _check(_lib.fresco_pair_create(ctypes.byref(h), ctypes.byref(p),
                                           ctypes.c_void_p(stream.cuda_stream)), "fresco_pair_create")
        self._h = h
        self._e = ctypes.c_double(0.0)

    @property
    def handle(self):
        return self._h

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            _lib.fresco_pair_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _pos(self, pos):
        if pos.device != self.device or pos.dtype != self.torch_dtype:
            raise ValueError(f"positions must be {self.torch_dtype} on {self.device}")
        if tuple(pos.shape) != (self.n, self.dim) or not pos.is_contiguous():
            raise ValueError(f"positions must be a contiguous [{self.n}][{self.dim}] tensor")
        return ctypes.c_void_p(pos.data_ptr())

    def replace_overlaps(self, pos, threshold: float, fresh) -> int:
        """Replace every point that lies closer than threshold to a point of lower index
        by the next row of fresh, in index order (fresco_pair_replace_overlaps); returns
        the number replaced."""
        n = ctypes.c_int64(0)
        st = _lib.fresco_pair_replace_overlaps(self._h, self._pos(pos), float(threshold),
                                               ctypes.c_void_p(fresh.data_ptr()),
                                               int(fresh.shape[0]), ctypes.byref(n))
        if st == EINVAL and n.value > fresh.shape[0]:
            raise FrescoError(st, f"fresco_pair_replace_overlaps ({n.value} overlaps, "
                                  f"{fresh.shape[0]} fresh rows)")
        _check(st, "fresco_pair_replace_overlaps")
        return int(n.value)

    def energy_grad(self, pos, grad=None):
        torch = _torch()
        if grad is None:
            grad = torch.empty((self.n, self.dim), dtype=self.torch_dtype, device=self.device)
        _check(_lib.fresco_pair_energy_grad(self._h, self._pos(pos), ctypes.byref(self._e),
                                            ctypes.c_void_p(grad.data_ptr())), "fresco_pair_energy_grad")
        return float(self._e.value), grad

    def energy_grad_async(self, pos, energy_dev, grad):
        _check(_lib.fresco_pair_energy_grad_async(self._h, self._pos(pos),
                                                  ctypes.c_void_p(energy_dev.data_ptr()),
                                                  ctypes.c_void_p(grad.data_ptr())),
               "fresco_pair_energy_grad_async")
        return energy_dev, grad


class BatchContext:
    """A ragged batch of independent problems (include/fresco.h, fresco_batch_*).

    items: list of dicts with keys n, box, and optionally w_cube, s0_cube, k_cut,
    relative; all share dim, kmax, tol and dtype.  Positions and gradients are the
    [n_b][dim] rows of every configuration concatenated in order.
    """

    def __init__(self, dim: int, kmax, items, *, tol: float = 1e-6, dtype: str = "f32",
                 stream=None, device=None):
        torch = _torch()
        self.dim = int(dim)
        self.dtype = dtype
        self.torch_dtype = torch.float32 if dtype == "f32" else torch.float64
        self.device = torch.device(device) if device is not None else torch.device("cuda", torch.cuda.current_device())
        kmax = np.broadcast_to(np.asarray(kmax, dtype=np.int64), (self.dim,))
        self.kmax = tuple(int(x) for x in kmax)
        self.cube_shape = tuple(2 * m + 1 for m in self.kmax)
        self.nb = len(items)
        probs = (Problem * self.nb)()
        self._keep = []
        for b, it in enumerate(items):
            p = probs[b]
            p.dim = self.dim
            p.dtype = F32 if dtype == "f32" else F64
            p.n = int(it["n"])
            box = np.broadcast_to(np.asarray(it["box"], dtype=np.float64), (self.dim,))
            for a in range(3):
                p.box[a] = float(box[a]) if a < self.dim else 1.0
                p.kmax[a] = self.kmax[a] if a < self.dim else 0
            p.k_cut = float(it.get("k_cut", 0.0))
            if it.get("w_cube") is not None:
                w = np.ascontiguousarray(np.asarray(it["w_cube"], dtype=np.float64).reshape(self.cube_shape))
                self._keep.append(w)
                p.w = w.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
            if it.get("s0_cube") is not None:
                s0 = np.ascontiguousarray(np.asarray(it["s0_cube"], dtype=np.float64).reshape(self.cube_shape))
                self._keep.append(s0)
                p.s0 = s0.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
            p.weight_mode = WEIGHT_RELATIVE if it.get("relative", False) else WEIGHT_ABS
            p.tol = float(tol)
            p.upsampfac = 2.0
        if stream is None:
            stream = torch.cuda.current_stream(self.device)
        self.stream = stream
        h = ctypes.c_void_p()
        with torch.cuda.device(self.device):
            _check(_lib.fresco_batch_create(ctypes.byref(h), self.nb, probs,
                                            ctypes.c_void_p(stream.cuda_stream)), "fresco_batch_create")
        self._h = h
        self._keep = None
        off = (ctypes.c_int64 * (self.nb + 1))()
        _check(_lib.fresco_batch_offsets(self._h, off), "fresco_batch_offsets")
        self.offsets = np.array(list(off), dtype=np.int64)
        self.rows = int(self.offsets[-1])

    @property
    def handle(self):
        return self._h

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            _lib.fresco_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _pos(self, pos):
        if pos.device != self.device or pos.dtype != self.torch_dtype:
            raise ValueError(f"positions must be {self.torch_dtype} on {self.device}")
        if tuple(pos.shape) != (self.rows, self.dim) or not pos.is_contiguous():
            raise ValueError(f"positions must be a contiguous [{self.rows}][{self.dim}] tensor")
        return ctypes.c_void_p(pos.data_ptr())

    def loss_grad(self, pos, grad=None):
        """(per-configuration losses as a numpy array, concatenated gradient)."""
        torch = _torch()
        if grad is None:
            grad = torch.empty((self.rows, self.dim), dtype=self.torch_dtype, device=self.device)
        losses = np.zeros(self.nb)
        _check(_lib.fresco_batch_loss_grad(self._h, self._pos(pos),
                                           losses.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                           ctypes.c_void_p(grad.data_ptr())), "fresco_batch_loss_grad")
        return losses, grad

    def loss_grad_async(self, pos, losses_dev, grad):
        _check(_lib.fresco_batch_loss_grad_async(
            self._h, self._pos(pos),
            ctypes.c_void_p(losses_dev.data_ptr()) if losses_dev is not None else None,
            ctypes.c_void_p(grad.data_ptr())), "fresco_batch_loss_grad_async")
        return losses_dev, grad

    def step(self, pos, n_iter: int, *, m: int = 8, max_step: float, c1: float = 1e-4,
             shrink: float = 0.5, max_backtracks: int = 20, gtol: float = 0.0):
        """n_iter L-BFGS iterations on the batch (pos updated in place).
        Returns (total loss, evaluations)."""
        o = LbfgsOpts()
        o.m = m
        o.max_backtracks = max_backtracks
        o.max_step = float(max_step)
        o.c1 = c1
        o.shrink = shrink
        o.gtol = gtol
        loss = ctypes.c_double(0.0)
        nev = ctypes.c_int32(0)
        _check(_lib.fresco_batch_step(self._h, self._pos(pos), ctypes.byref(o), int(n_iter),
                                      ctypes.byref(loss), ctypes.byref(nev)), "fresco_batch_step")
        return float(loss.value), int(nev.value)

    def reset_history(self):
        _check(_lib.fresco_batch_reset_history(self._h), "fresco_batch_reset_history")

    def autotune(self, pos, reps: int = 5) -> int:
        """Pick the fastest workgroup size for this batch; returns it."""
        torch = _torch()
        grad = torch.empty((self.rows, self.dim), dtype=self.torch_dtype, device=self.device)
        t = ctypes.c_int32(0)
        _check(_lib.fresco_batch_autotune(self._h, self._pos(pos), ctypes.c_void_p(grad.data_ptr()),
                                          int(reps), ctypes.byref(t)), "fresco_batch_autotune")
        return int(t.value)
