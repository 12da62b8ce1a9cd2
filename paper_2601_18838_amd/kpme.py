"""Thin Python binding of the C ABI in include/kpme.h (argument marshalling only).

Every step of the reciprocal path runs in libkpme.so's gfx950 kernels; this
module only checks tensor dtypes/devices, passes raw pointers and the current
HIP stream, and turns status codes into exceptions.  There is no fallback: if
libkpme.so is missing or the device is not a gfx950, calls raise.
"""
import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libkpme.so")

FP64, FP32, BF16X3, FP16X3 = 0, 1, 2, 3
STAGES = ("spread", "grid_sum", "skp_stage1", "skp_stage2", "skp_finalize", "gather", "energy")
PRECISIONS = {"fp64": FP64, "fp32": FP32, "bf16x3": BF16X3, "fp16x3": FP16X3}
STATUS = {0: "KPME_SUCCESS", 1: "KPME_ERROR_INVALID_VALUE", 2: "KPME_ERROR_NOT_SUPPORTED",
          3: "KPME_ERROR_OUT_OF_MEMORY", 4: "KPME_ERROR_DEVICE", 5: "KPME_ERROR_NUMERICAL"}


class KpmeError(RuntimeError):
    def __init__(self, status, message):
        super().__init__(f"{STATUS.get(status, status)}: {message}")
        self.status = status


class PlanInfo(ctypes.Structure):
    _fields_ = [("grid", ctypes.c_int * 3), ("spline_order", ctypes.c_int),
                ("precision", ctypes.c_int), ("rank", ctypes.c_int), ("r0", ctypes.c_int),
                ("total_terms", ctypes.c_int), ("max_particles", ctypes.c_int64),
                ("beta", ctypes.c_double), ("theta_norm", ctypes.c_double),
                ("trunc_err", ctypes.c_double), ("zero_mode", ctypes.c_double),
                ("workspace_bytes", ctypes.c_size_t), ("skp_method", ctypes.c_int),
                ("quad_N", ctypes.c_int), ("quad_h", ctypes.c_double),
                ("sym_err", ctypes.c_double), ("interpolation", ctypes.c_int),
                ("mode_cutoff", ctypes.c_int), ("skp_form", ctypes.c_int)]


class PlanOptions(ctypes.Structure):
    _fields_ = [("skp_method", ctypes.c_int), ("quad_h", ctypes.c_double),
                ("interpolation", ctypes.c_int), ("mode_cutoff", ctypes.c_int),
                ("skp_form", ctypes.c_int)]


METHODS = {"nested_svd": 0, "sinc": 1}
INTERPOLATIONS = {"bspline": 0, "lagrange": 1}
FORMS = {"circulant": 0, "rect": 1}


def _options(method, quad_h, interpolation="bspline", mode_cutoff=0, form="circulant"):
    return PlanOptions(METHODS[method], float(quad_h), INTERPOLATIONS[interpolation],
                       int(mode_cutoff), FORMS[form])


_lib = None
_P = ctypes.c_void_p
_I64 = ctypes.c_int64
_D = ctypes.c_double
_INT = ctypes.c_int
_DP = ctypes.POINTER(ctypes.c_double)
_IP = ctypes.POINTER(ctypes.c_int)

_SIGNATURES = {
    "kpme_plan_create": [ctypes.POINTER(_P), _DP, _IP, _INT, _D, _INT, _D, _INT, _I64, _INT],
    "kpme_plan_create_ex": [ctypes.POINTER(_P), _DP, _IP, _INT, _D, _INT, _D, _INT, _I64, _INT,
                            ctypes.POINTER(PlanOptions)],
    "kpme_plan_destroy": [_P],
    "kpme_plan_info": [_P, ctypes.POINTER(PlanInfo)],
    "kpme_spread": [_P, _I64, _P, _P, _P, _P],
    "kpme_skp_apply": [_P, _P, _P, _P],
    "kpme_gather": [_P, _I64, _P, _P, _P, _P, _P, _P],
    "kpme_energy": [_P, _I64, _P, _P, _P, _P],
    "kpme_energy_noalloc": [_P, _I64, _P, _P, _P, _P],
    "kpme_evaluate": [_P, _I64, _P, _P, _P, _P, _P, _P],
    "kpme_evaluate_backward": [_P, _I64, _P, _P, _P, _P, _P, _P, _P],
    "kpme_factors_compute": [_DP, _IP, _INT, _D, _INT, _D, _INT, _IP, _DP, _DP, _DP, _DP,
                             _IP, _DP],
    "kpme_factors_compute_ex": [_DP, _IP, _INT, _D, _INT, _D, ctypes.POINTER(PlanOptions), _INT,
                                _IP, _DP, _DP, _DP, _DP, _IP, _DP],
    "kpme_batch_create": [ctypes.POINTER(_P), _INT, _DP, _IP, _IP, _DP, _IP, _INT,
                          ctypes.POINTER(_I64), _INT],
    "kpme_batch_destroy": [_P],
    "kpme_batch_info": [_P, _IP, _IP],
    "kpme_plan_profile": [_P, _INT],
    "kpme_plan_autotune": [_P, _P],
    "kpme_plan_profile_read": [_P, _DP, ctypes.POINTER(_I64)],
    "kpme_batch_evaluate": [_P, ctypes.POINTER(_I64), _P, _P, _P, _P, _P, _P],
}


def lib():
    """Load libkpme.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: run `python -m paper_2601_18838_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        for name, args in _SIGNATURES.items():
            fn = getattr(L, name)
            fn.argtypes = args
            fn.restype = ctypes.c_int
        L.kpme_status_string.argtypes = [ctypes.c_int]
        L.kpme_status_string.restype = ctypes.c_char_p
        L.kpme_last_error.argtypes = []
        L.kpme_last_error.restype = ctypes.c_char_p
        L.kpme_device_count.argtypes = []
        L.kpme_device_count.restype = ctypes.c_int
        L.kpme_plan_stage2_parts.argtypes = [_P]
        L.kpme_plan_stage2_parts.restype = ctypes.c_int
        L.kpme_plan_stage1_split.argtypes = [_P]
        L.kpme_plan_stage1_split.restype = ctypes.c_int
        L.kpme_plan_stage2_streams.argtypes = [_P]
        L.kpme_plan_stage2_streams.restype = ctypes.c_int
        _lib = L
    return _lib


def _check(status):
    if status != 0:
        raise KpmeError(status, lib().kpme_last_error().decode())


def _dbl3(x):
    return (ctypes.c_double * 3)(*[float(v) for v in x])


def _int3(x):
    return (ctypes.c_int * 3)(*[int(v) for v in x])


def device_count():
    return lib().kpme_device_count()


def factors_compute(box, grid, order, beta, rank=0, tol=1e-6, max_terms=4096,
                    method="nested_svd", quad_h=0.0, interpolation="bspline", mode_cutoff=0):
    """Host FP64 factor construction (no device needed): dict of numpy arrays."""
    L = lib()
    K = [int(k) for k in grid]
    n = ctypes.c_int(0)
    om = np.zeros(max_terms)
    v = [np.zeros(max_terms * K[j]) for j in range(3)]
    grp = np.zeros(max_terms, np.int32)
    info = np.zeros(6)
    opts = _options(method, quad_h, interpolation, mode_cutoff)
    dp = lambda a: a.ctypes.data_as(_DP)
    _check(L.kpme_factors_compute_ex(_dbl3(box), _int3(K), int(order), float(beta), int(rank),
                                     float(tol), ctypes.byref(opts), max_terms, ctypes.byref(n),
                                     dp(om), dp(v[0]), dp(v[1]), dp(v[2]),
                                     grp.ctypes.data_as(_IP), dp(info)))
    R = n.value
    return {"omega": om[:R].copy(), "group": grp[:R].copy(),
            "vec": [v[j][:R * K[j]].reshape(R, K[j]).copy() for j in range(3)],
            "theta_norm": info[0], "trunc_err": info[1], "zero_mode": info[2],
            "quad_N": int(info[3]), "quad_h": info[4], "sym_err": info[5]}


def _stream():
    import torch
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


class Plan:
    """A device plan: factors and workspace for one box/grid/order/beta/rank."""

    def __init__(self, box, grid, order, beta, rank=0, tol=1e-6, precision="fp32",
                 max_particles=1, device=0, method="nested_svd", quad_h=0.0,
                 interpolation="bspline", mode_cutoff=0, form="circulant"):
        import torch
        self.precision = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
        self.dtype = torch.float64 if self.precision == FP64 else torch.float32
        self.box = tuple(float(b) for b in box)
        self.grid = tuple(int(k) for k in grid)
        self.order = int(order)
        self.beta = float(beta)
        self.device = torch.device("cuda", device)
        self._h = _P()
        opts = _options(method, quad_h, interpolation, mode_cutoff, form)
        _check(lib().kpme_plan_create_ex(ctypes.byref(self._h), _dbl3(box), _int3(grid),
                                         self.order, self.beta, int(rank), float(tol),
                                         self.precision, int(max_particles), int(device),
                                         ctypes.byref(opts)))
        info = PlanInfo()
        _check(lib().kpme_plan_info(self._h, ctypes.byref(info)))
        self.info = {f: getattr(info, f) for f, _ in PlanInfo._fields_}
        self.info["grid"] = tuple(info.grid)

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            try:
                lib().kpme_plan_destroy(h)
            except Exception:
                pass
            self._h = None

    # -- marshalling ------------------------------------------------------
    def _t(self, x, shape=None):
        import torch
        if x is None:
            return None
        if not (isinstance(x, torch.Tensor) and x.device == self.device and x.dtype == self.dtype
                and x.is_contiguous()):
            raise TypeError(f"expected a contiguous {self.dtype} tensor on {self.device}")
        if shape is not None and tuple(x.shape) != tuple(shape):
            raise ValueError(f"expected shape {shape}, got {tuple(x.shape)}")
        return x

    @staticmethod
    def _p(x):
        return None if x is None else ctypes.c_void_p(x.data_ptr())

    def new_grid(self):
        import torch
        return torch.empty(self.grid, dtype=self.dtype, device=self.device)

    # -- the C entry points ---------------------------------------------
    def spread(self, pos, q, out=None):
        n = q.shape[0]
        self._t(pos, (n, 3)); self._t(q, (n,))
        out = self.new_grid() if out is None else self._t(out, self.grid)
        _check(lib().kpme_spread(self._h, n, self._p(pos), self._p(q), self._p(out), _stream()))
        return out

    def skp_apply(self, grid_in, out=None):
        self._t(grid_in, self.grid)
        out = self.new_grid() if out is None else self._t(out, self.grid)
        _check(lib().kpme_skp_apply(self._h, self._p(grid_in), self._p(out), _stream()))
        return out

    def gather(self, pos, q, phi_grid, potentials=True, forces=True):
        import torch
        n = pos.shape[0]
        self._t(pos, (n, 3)); self._t(phi_grid, self.grid)
        if q is not None:
            self._t(q, (n,))
        pot = torch.empty(n, dtype=self.dtype, device=self.device) if potentials else None
        frc = torch.empty((n, 3), dtype=self.dtype, device=self.device) if forces else None
        _check(lib().kpme_gather(self._h, n, self._p(pos), self._p(q), self._p(phi_grid),
                                 self._p(pot), self._p(frc), _stream()))
        return pot, frc

    def energy(self, q, pot):
        import torch
        n = q.shape[0]
        self._t(q, (n,)); self._t(pot, (n,))
        e4 = torch.empty(4, dtype=torch.float64, device=self.device)
        _check(lib().kpme_energy(self._h, n, self._p(q), self._p(pot), self._p(e4), _stream()))
        return e4

    def energy_noalloc(self, q, pot, out):
        """kpme_energy_noalloc: the energy reduction into the caller's
        4-double device tensor `out`, with the library's fixed scratch array
        (no allocation by the library or by this call)."""
        n = q.shape[0]
        self._t(q, (n,)); self._t(pot, (n,))
        _check(lib().kpme_energy_noalloc(self._h, n, self._p(q), self._p(pot), self._p(out),
                                         _stream()))
        return out

    def evaluate(self, pos, q, potentials=True, forces=True, energy=True, out=None):
        """Whole path; returns (energy4 [4] float64 tensor, pot, force)."""
        import torch
        n = q.shape[0]
        self._t(pos, (n, 3)); self._t(q, (n,))
        if out is not None:
            e4, pot, frc = out
        else:
            e4 = torch.empty(4, dtype=torch.float64, device=self.device) if energy else None
            pot = torch.empty(n, dtype=self.dtype, device=self.device) if potentials else None
            frc = torch.empty((n, 3), dtype=self.dtype, device=self.device) if forces else None
        _check(lib().kpme_evaluate(self._h, n, self._p(pos), self._p(q), self._p(pot),
                                   self._p(frc), self._p(e4), _stream()))
        return e4, pot, frc

    def autotune(self):
        """Run the library's autotuner (stage-2 streams and split, stage-1 split)
        on the current stream; returns the stage-2 split."""
        _check(lib().kpme_plan_autotune(self._h, _stream()))
        return self.stage2_parts()

    def stage2_parts(self):
        return lib().kpme_plan_stage2_parts(self._h)

    def stage1_split(self):
        return lib().kpme_plan_stage1_split(self._h)

    def stage2_streams(self):
        return lib().kpme_plan_stage2_streams(self._h)

    def profile(self, enable=True):
        """Switch the library's per-stage hipEvent timers on or off."""
        _check(lib().kpme_plan_profile(self._h, 1 if enable else 0))

    def profile_read(self):
        """{stage: (total_ms, launches)} since the last read (waits for the events)."""
        ms = (ctypes.c_double * len(STAGES))()
        cnt = (ctypes.c_int64 * len(STAGES))()
        _check(lib().kpme_plan_profile_read(self._h, ms, cnt))
        return {name: (ms[i], cnt[i]) for i, name in enumerate(STAGES)}

    def evaluate_backward(self, pos, q, g_energy=None, g_pot=None, want_pos=True, want_q=True):
        """Gradients of g_energy * energy4[3] + g_pot . pot (see include/kpme.h).

        g_energy: None, a Python number, or a one-element float64 device tensor."""
        import torch
        n = q.shape[0]
        self._t(pos, (n, 3)); self._t(q, (n,))
        if g_pot is not None:
            self._t(g_pot, (n,))
        if g_energy is not None and not isinstance(g_energy, torch.Tensor):
            g_energy = torch.tensor([float(g_energy)], dtype=torch.float64, device=self.device)
        if g_energy is not None:
            g_energy = g_energy.reshape(1).to(device=self.device, dtype=torch.float64).contiguous()
        gp = torch.empty((n, 3), dtype=self.dtype, device=self.device) if want_pos else None
        gq = torch.empty(n, dtype=self.dtype, device=self.device) if want_q else None
        _check(lib().kpme_evaluate_backward(self._h, n, self._p(pos), self._p(q),
                                            self._p(g_energy), self._p(g_pot), self._p(gp),
                                            self._p(gq), _stream()))
        return gp, gq


class BatchPlan:
    """Independent systems evaluated by one replayed HIP graph (kpme_batch_*):
    batched launches (one per stage and kernel instance over all systems)
    where every system's kernels have that form, else per-system branches."""

    def __init__(self, boxes, grids, orders, betas, ranks, precision="fp16x3",
                 max_particles=None, device=0):
        import torch
        count = len(grids)
        self.count = count
        self.precision = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
        self.dtype = torch.float64 if self.precision == FP64 else torch.float32
        self.device = torch.device("cuda", device)
        box = (ctypes.c_double * (3 * count))(*[float(x) for b in boxes for x in b])
        grd = (ctypes.c_int * (3 * count))(*[int(x) for g in grids for x in g])
        order = (ctypes.c_int * count)(*[int(x) for x in orders])
        beta = (ctypes.c_double * count)(*[float(x) for x in betas])
        rank = (ctypes.c_int * count)(*[int(x) for x in ranks])
        nmax = (ctypes.c_int64 * count)(*[int(x) for x in max_particles])
        self._h = _P()
        _check(lib().kpme_batch_create(ctypes.byref(self._h), count, box, grd, order, beta,
                                       rank, self.precision, nmax, int(device)))

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            try:
                lib().kpme_batch_destroy(h)
            except Exception:
                pass
            self._h = None

    def evaluate(self, n, pos, q, pot=None, force=None, energy=None):
        """n: per-system counts; pos (sum n, 3) and q (sum n) concatenated in order.
        Returns (energy4 [count, 4], pot, force).  Outputs not passed in are
        the BatchPlan's own buffers, allocated once per total count and reused
        by later calls (so repeated calls replay one recorded graph); the next
        call overwrites them."""
        import torch
        total = int(sum(n))
        for t, shape in ((pos, (total, 3)), (q, (total,))):
            if not (isinstance(t, torch.Tensor) and t.device == self.device
                    and t.dtype == self.dtype and t.is_contiguous() and tuple(t.shape) == shape):
                raise TypeError(f"expected a contiguous {self.dtype} tensor of shape {shape}")
        own = getattr(self, "_own", None)
        if own is None or own[1].shape[0] != total:
            own = (torch.empty((self.count, 4), dtype=torch.float64, device=self.device),
                   torch.empty(total, dtype=self.dtype, device=self.device),
                   torch.empty((total, 3), dtype=self.dtype, device=self.device))
            self._own = own
        energy = own[0] if energy is None else energy
        pot = own[1] if pot is None else pot
        force = own[2] if force is None else force
        nn = (ctypes.c_int64 * self.count)(*[int(x) for x in n])
        p = lambda t: ctypes.c_void_p(t.data_ptr())
        _check(lib().kpme_batch_evaluate(self._h, nn, p(pos), p(q), p(pot), p(force),
                                         p(energy), _stream()))
        return energy, pot, force

    def info(self):
        """(form, launches) of the current recording: form 1 = one launch per
        stage and kernel instance for all systems, 0 = per-system graph
        branches, -1 = nothing recorded; launches = kernels per replay."""
        form, launches = ctypes.c_int(), ctypes.c_int()
        _check(lib().kpme_batch_info(self._h, ctypes.byref(form), ctypes.byref(launches)))
        return form.value, launches.value


def _autograd_function():
    import torch

    class KPMEFunction(torch.autograd.Function):
        """(pos, q) -> (E, pot): E = E_rec + E_self + E_neutral (float64, 0-d),
        pot the reciprocal potentials; backward runs the library's adjoint."""

        @staticmethod
        def forward(ctx, pos, q, plan):
            e4, pot, _ = plan.evaluate(pos.contiguous(), q.contiguous(), forces=False)
            ctx.plan = plan
            ctx.save_for_backward(pos, q)
            return e4[3], pot

        @staticmethod
        def backward(ctx, g_e, g_pot):
            pos, q = ctx.saved_tensors
            plan = ctx.plan
            gp, gq = plan.evaluate_backward(
                pos.contiguous(), q.contiguous(),
                g_energy=None if g_e is None else g_e.detach(),
                g_pot=None if g_pot is None else g_pot.detach().to(plan.dtype).contiguous(),
                want_pos=ctx.needs_input_grad[0], want_q=ctx.needs_input_grad[1])
            return gp, gq, None

    return KPMEFunction


_KPME_FN = None


def kpme_energy_and_potentials(pos, q, plan):
    """Differentiable reciprocal evaluation: returns (E, pot); see KPMEFunction."""
    global _KPME_FN
    if _KPME_FN is None:
        _KPME_FN = _autograd_function()
    return _KPME_FN.apply(pos, q, plan)
