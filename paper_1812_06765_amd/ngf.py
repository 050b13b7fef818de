"""Python binding of the C ABI in ``include/ngfreg.h`` (argument marshalling only).

Every computation runs in the HIP library ``libngfreg.so`` built from
``csrc/``; this module only checks tensor shapes, dtypes and devices, passes
raw device pointers and the current HIP stream, and turns status codes into
exceptions.  There is no fallback: if the library is missing or no GPU is
visible, the calls raise.

Method names follow the C ABI without the ``ngf_`` prefix.
"""

from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libngfreg.so")

OK, E_ARG, E_SHAPE, E_STATE, E_LEVEL, E_OOM, E_HIP, E_NONFINITE = 0, -1, -2, -3, -4, -5, -6, -7
INFO_OK, INFO_CONVERGED, INFO_MAX_ITER, INFO_LINESEARCH_FAIL, INFO_NONFINITE = 0, 1, 2, 3, 4
MAX_LEVELS = 12
STATUS_NAMES = {0: "OK", -1: "E_ARG", -2: "E_SHAPE", -3: "E_STATE", -4: "E_LEVEL",
                -5: "E_OOM", -6: "E_HIP", -7: "E_NONFINITE"}


class Grid(ctypes.Structure):
    _fields_ = [("m", ctypes.c_int32 * 3), ("h", ctypes.c_double * 3)]


class Params(ctypes.Structure):
    _fields_ = [("alpha", ctypes.c_double), ("tau", ctypes.c_double), ("rho", ctypes.c_double),
                ("levels", ctypes.c_int32), ("ratio", ctypes.c_int32),
                ("max_iter", ctypes.c_int32), ("lbfgs_mem", ctypes.c_int32),
                ("tol_J", ctypes.c_double), ("early_stop", ctypes.c_int32),
                ("reserved", ctypes.c_int32)]


class Report(ctypes.Structure):
    _fields_ = [("levels", ctypes.c_int32), ("iters", ctypes.c_int32 * MAX_LEVELS),
                ("evals", ctypes.c_int32 * MAX_LEVELS), ("info", ctypes.c_int32 * MAX_LEVELS),
                ("J", ctypes.c_double * MAX_LEVELS), ("ms", ctypes.c_double * MAX_LEVELS)]


class IterRecord(ctypes.Structure):
    _fields_ = [("level", ctypes.c_int32), ("iter", ctypes.c_int32), ("evals", ctypes.c_int32),
                ("reserved", ctypes.c_int32), ("J", ctypes.c_double), ("D", ctypes.c_double),
                ("S", ctypes.c_double), ("gmax", ctypes.c_double), ("t", ctypes.c_double),
                ("us", ctypes.c_double)]


ITER_FIELDS = ("level", "iter", "evals", "J", "D", "S", "gmax", "t", "us")


def write_jsonl(records, path):
    """Write iteration records (dicts as Context.iteration_log returns them)
    as JSON lines, one record per line."""
    import json
    with open(path, "w") as f:
        for r in records:
            f.write(json.dumps({k: r[k] for k in ITER_FIELDS}) + "\n")


class NgfError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


_lib = None
_P = ctypes.c_void_p


def load():
    """Load libngfreg.so (after torch, so that it binds to torch's HIP runtime)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is not built; run python -m paper_1812_06765_amd.build")
    lib = ctypes.CDLL(LIB_PATH)
    i32, f64 = ctypes.c_int32, ctypes.c_double
    sig = {
        "ngf_version": ([], ctypes.c_char_p),
        "ngf_create": ([ctypes.POINTER(Params), _P, ctypes.POINTER(_P)], i32),
        "ngf_destroy": ([_P], None),
        "ngf_last_error": ([_P], ctypes.c_char_p),
        "ngf_set_params": ([_P, ctypes.POINTER(Params)], i32),
        "ngf_build_pyramid": ([_P, _P, _P, ctypes.POINTER(Grid), i32], i32),
        "ngf_level_info": ([_P, i32, ctypes.POINTER(Grid), ctypes.POINTER(Grid)], i32),
        "ngf_level_images": ([_P, i32, _P, _P], i32),
        "ngf_index_map": ([_P, i32, i32, _P, _P, _P], i32),
        "ngf_identity": ([_P, i32, _P], i32),
        "ngf_eval_J_grad": ([_P, i32, _P, ctypes.POINTER(f64), _P, ctypes.POINTER(f64)], i32),
        "ngf_eval_J_device": ([_P, ctypes.POINTER(_P)], i32),
        "ngf_eval_J_grad_f64": ([_P, i32, _P, ctypes.POINTER(f64), _P, ctypes.POINTER(f64)],
                                i32),
        "ngf_lbfgs_reset": ([_P, i32, _P], i32),
        "ngf_lbfgs_step": ([_P, ctypes.POINTER(f64), ctypes.POINTER(i32)], i32),
        "ngf_lbfgs_get": ([_P, _P, _P, ctypes.POINTER(f64)], i32),
        "ngf_lbfgs_state_size": ([_P, ctypes.POINTER(ctypes.c_size_t)], i32),
        "ngf_lbfgs_save": ([_P, _P, ctypes.c_size_t], i32),
        "ngf_lbfgs_load": ([_P, _P, ctypes.c_size_t], i32),
        "ngf_set_iteration_log": ([_P, i32], i32),
        "ngf_iteration_log": ([_P, ctypes.POINTER(IterRecord), i32, ctypes.POINTER(i32)], i32),
        "ngf_prolongate": ([_P, i32, _P, _P], i32),
        "ngf_register": ([_P, _P, _P, ctypes.POINTER(Grid), _P, i32, ctypes.POINTER(Report)], i32),
        "ngf_register_levels": ([_P, _P, ctypes.POINTER(Report)], i32),
        "ngf_eval_pair": ([_P, ctypes.POINTER(Grid), ctypes.POINTER(ctypes.c_int32 * 3), _P, _P,
                           _P, _P, ctypes.POINTER(f64), _P, _P, _P], i32),
        "ngf_set_profiling": ([_P, i32, i32], i32),
        "ngf_set_kernel": ([_P, i32], i32),
        "ngf_set_driver": ([_P, i32], i32),
        "ngf_set_faults": ([_P, i32], i32),
        "ngf_eval_pair_static": ([_P, ctypes.POINTER(Grid), ctypes.POINTER(ctypes.c_int32 * 3),
                                  _P, _P, _P, _P, ctypes.POINTER(f64), _P, _P, _P], i32),
        "ngf_eval_J_grad_T": ([_P, i32, _P, _P, ctypes.POINTER(ctypes.c_double), _P, _P, _P],
                              i32),
        "ngf_set_node_grid": ([_P, ctypes.POINTER(i32)], i32),
        "ngf_apply_P": ([_P, i32, _P, _P], i32),
        "ngf_apply_PT": ([_P, i32, _P, _P, i32], i32),
        "ngf_get_kernel": ([_P, i32, ctypes.POINTER(i32)], i32),
        "ngf_kernel_time": ([_P, i32, ctypes.POINTER(i32), ctypes.POINTER(f64),
                             ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int64)],
                            i32),
        "ngf_batch_create": ([ctypes.POINTER(Params), i32, ctypes.POINTER(_P)], i32),
        "ngf_batch_destroy": ([_P], None),
        "ngf_batch_last_error": ([_P], ctypes.c_char_p),
        "ngf_batch_set_kernel": ([_P, i32], i32),
        "ngf_batch_set_mode": ([_P, i32], i32),
        "ngf_batch_register": ([_P, i32, ctypes.POINTER(_P), ctypes.POINTER(_P),
                                ctypes.POINTER(Grid), ctypes.POINTER(_P), _P,
                                ctypes.POINTER(Report)], i32),
        "ngf_batch_build": ([_P, i32, ctypes.POINTER(_P), ctypes.POINTER(_P),
                             ctypes.POINTER(Grid), _P], i32),
        "ngf_batch_eval": ([_P, i32, ctypes.POINTER(_P), ctypes.POINTER(f64),
                            ctypes.POINTER(_P), _P], i32),
    }
    for name, (args, res) in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = res
    _lib = lib
    return lib


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _grid(m, h) -> Grid:
    g = Grid()
    for d in range(3):
        g.m[d] = int(m[d])
        g.h[d] = float(h[d])
    return g


@dataclass
class LevelInfo:
    m: tuple
    h: tuple
    my: tuple
    hy: tuple


class Context:
    """An ngf_ctx bound to the current torch HIP stream of ``device``."""

    def __init__(self, alpha=0.1, tau=1.0, rho=1.0, levels=1, ratio=2, max_iter=50,
                 lbfgs_mem=5, tol_J=1e-6, early_stop=False, device="cuda"):
        self.lib = load()
        if not torch.cuda.is_available():
            raise RuntimeError("no HIP device visible: the ngf library has no CPU path")
        self.device = torch.device(device)
        self.stream = torch.cuda.current_stream(self.device)
        self.p = Params(float(alpha), float(tau), float(rho), int(levels), int(ratio),
                        int(max_iter), int(lbfgs_mem), float(tol_J), int(bool(early_stop)), 0)
        h = _P()
        st = self.lib.ngf_create(ctypes.byref(self.p), ctypes.c_void_p(self.stream.cuda_stream),
                                 ctypes.byref(h))
        if st != OK:
            raise NgfError(st, "ngf_create failed")
        self.h = h
        self.levels = int(levels)

    def close(self):
        if getattr(self, "h", None):
            self.lib.ngf_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def _chk(self, st):
        if st != OK:
            msg = self.lib.ngf_last_error(self.h).decode()
            raise NgfError(st, msg)

    def _f32(self, t, shape=None, name="tensor"):
        if not (isinstance(t, torch.Tensor) and t.dtype == torch.float32 and t.is_cuda
                and t.is_contiguous()):
            raise TypeError(f"{name} must be a contiguous float32 tensor on the GPU")
        if shape is not None and tuple(t.shape) != tuple(shape):
            raise ValueError(f"{name} has shape {tuple(t.shape)}, expected {tuple(shape)}")
        return t

    # -- parameters -------------------------------------------------------
    def set_params(self, **kw):
        for k, v in kw.items():
            setattr(self.p, k, type(getattr(self.p, k))(v))
        self._chk(self.lib.ngf_set_params(self.h, ctypes.byref(self.p)))

    # -- pyramid -----------------------------------------------------------
    def build_pyramid(self, R, T, h=(1.0, 1.0, 1.0)):
        host = not R.is_cuda
        if host:
            R = R.detach().to(torch.float32).contiguous()
            T = T.detach().to(torch.float32).contiguous()
        else:
            self._f32(R, name="R")
            self._f32(T, R.shape, name="T")
        if tuple(R.shape) != tuple(T.shape) or R.dim() != 3:
            raise ValueError("R and T must be 3D arrays of one shape")
        g = _grid(R.shape, h)
        self._chk(self.lib.ngf_build_pyramid(self.h, _ptr(R), _ptr(T), ctypes.byref(g),
                                             int(host)))

    def level_info(self, level) -> LevelInfo:
        gi, gd = Grid(), Grid()
        self._chk(self.lib.ngf_level_info(self.h, int(level), ctypes.byref(gi), ctypes.byref(gd)))
        return LevelInfo(tuple(gi.m), tuple(gi.h), tuple(gd.m), tuple(gd.h))

    def level_images(self, level):
        li = self.level_info(level)
        R = torch.empty(li.m, dtype=torch.float32, device=self.device)
        T = torch.empty(li.m, dtype=torch.float32, device=self.device)
        self._chk(self.lib.ngf_level_images(self.h, int(level), _ptr(R), _ptr(T)))
        return R, T

    def index_map(self, level, axis):
        m = self.level_info(level).m[axis]
        j0 = torch.empty(m, dtype=torch.int32, device=self.device)
        w0 = torch.empty(m, dtype=torch.float32, device=self.device)
        w1 = torch.empty(m, dtype=torch.float32, device=self.device)
        self._chk(self.lib.ngf_index_map(self.h, int(level), int(axis), _ptr(j0), _ptr(w0),
                                         _ptr(w1)))
        return j0, w0, w1

    def identity(self, level):
        li = self.level_info(level)
        y = torch.empty((3,) + li.my, dtype=torch.float32, device=self.device)
        self._chk(self.lib.ngf_identity(self.h, int(level), _ptr(y)))
        return y

    # -- evaluation --------------------------------------------------------
    def eval_J_grad(self, level, y, want_grad=True, out=None):
        """Returns (J, grad or None, (D, S)); J and (D, S) are Python floats."""
        li = self.level_info(level)
        self._f32(y, (3,) + li.my, "y")
        g = None
        if want_grad:
            g = out if out is not None else torch.empty_like(y)
            self._f32(g, y.shape, "grad")
        J = ctypes.c_double()
        DS = (ctypes.c_double * 2)()
        self._chk(self.lib.ngf_eval_J_grad(self.h, int(level), _ptr(y), ctypes.byref(J), _ptr(g),
                                           DS))
        return J.value, g, (DS[0], DS[1])

    def eval_J_grad_f64(self, level, y, want_grad=True):
        """The float64 evaluation: y a contiguous float64 GPU tensor shaped like
        the level's deformation.  Returns (J, grad or None, (D, S))."""
        li = self.level_info(level)
        if not (isinstance(y, torch.Tensor) and y.dtype == torch.float64 and y.is_cuda
                and y.is_contiguous() and tuple(y.shape) == (3,) + li.my):
            raise TypeError(f"y must be a contiguous float64 GPU tensor of shape {(3,) + li.my}")
        g = torch.empty_like(y) if want_grad else None
        J = ctypes.c_double()
        DS = (ctypes.c_double * 2)()
        self._chk(self.lib.ngf_eval_J_grad_f64(self.h, int(level), _ptr(y), ctypes.byref(J),
                                               _ptr(g), DS))
        return J.value, g, (DS[0], DS[1])

    def eval_J_grad_async(self, level, y, grad):
        """Enqueue an evaluation without synchronising (J stays on the device)."""
        self._chk(self.lib.ngf_eval_J_grad(self.h, int(level), _ptr(y), None, _ptr(grad), None))

    # -- L-BFGS ------------------------------------------------------------
    def lbfgs_reset(self, level, y0):
        self._f32(y0, (3,) + self.level_info(level).my, "y0")
        self._chk(self.lib.ngf_lbfgs_reset(self.h, int(level), _ptr(y0)))

    def lbfgs_step(self):
        J = ctypes.c_double()
        info = ctypes.c_int32()
        self._chk(self.lib.ngf_lbfgs_step(self.h, ctypes.byref(J), ctypes.byref(info)))
        return J.value, info.value

    def lbfgs_get(self, level):
        my = self.level_info(level).my
        y = torch.empty((3,) + my, dtype=torch.float32, device=self.device)
        g = torch.empty_like(y)
        J = ctypes.c_double()
        self._chk(self.lib.ngf_lbfgs_get(self.h, _ptr(y), _ptr(g), ctypes.byref(J)))
        return y, g, J.value

    def lbfgs_save(self) -> bytes:
        """The L-BFGS state left by lbfgs_reset / lbfgs_step (level, iterate,
        gradient, stored pairs, device state block) as bytes."""
        n = ctypes.c_size_t()
        self._chk(self.lib.ngf_lbfgs_state_size(self.h, ctypes.byref(n)))
        buf = ctypes.create_string_buffer(n.value)
        self._chk(self.lib.ngf_lbfgs_save(self.h, buf, n))
        return buf.raw

    def lbfgs_load(self, state: bytes):
        """Resume from lbfgs_save's bytes (same pyramid shapes and memory);
        lbfgs_step then continues as it would have after the save."""
        buf = ctypes.create_string_buffer(bytes(state), len(state))
        self._chk(self.lib.ngf_lbfgs_load(self.h, buf, len(state)))

    def set_iteration_log(self, enable=True):
        """Record every accepted L-BFGS step (and each level's start point);
        clears the log."""
        self._chk(self.lib.ngf_set_iteration_log(self.h, int(bool(enable))))

    def iteration_log(self, path=None):
        """The records since the log was cleared, as dicts with the keys
        level, iter, evals, J, D, S, gmax, t, us; also written to ``path`` as
        JSON lines when given."""
        n = ctypes.c_int32()
        self._chk(self.lib.ngf_iteration_log(self.h, None, 0, ctypes.byref(n)))
        arr = (IterRecord * max(n.value, 1))()
        self._chk(self.lib.ngf_iteration_log(self.h, arr, n.value, ctypes.byref(n)))
        recs = [{k: getattr(arr[i], k) for k in ITER_FIELDS} for i in range(n.value)]
        if path is not None:
            write_jsonl(recs, path)
        return recs

    def prolongate(self, coarse_level, yc):
        fine = self.level_info(coarse_level - 1).my
        yf = torch.empty((3,) + fine, dtype=torch.float32, device=self.device)
        self._chk(self.lib.ngf_prolongate(self.h, int(coarse_level), _ptr(yc), _ptr(yf)))
        return yf

    # -- registration --------------------------------------------------------
    @staticmethod
    def _report(rep: Report):
        return [dict(level=lev, iters=rep.iters[lev], evals=rep.evals[lev], J=rep.J[lev],
                     info=rep.info[lev], ms=rep.ms[lev]) for lev in range(rep.levels)]

    def register(self, R, T, h=(1.0, 1.0, 1.0)):
        """Full registration from R, T (device tensors, or CPU tensors for the
        host-pointer path).  Returns (y at level 0, per-level report)."""
        host = not R.is_cuda
        if host:
            R = R.detach().to(torch.float32).contiguous()
            T = T.detach().to(torch.float32).contiguous()
        else:
            self._f32(R, name="R")
            self._f32(T, R.shape, name="T")
        g = _grid(R.shape, h)
        ng = getattr(self, "node_grid", None)
        my = tuple((ng[d] if ng and ng[d] else int(R.shape[d]) // self.p.ratio + 1)
                   for d in range(3))
        y = torch.empty((3,) + my, dtype=torch.float32,
                        device="cpu" if host else self.device)
        if host:
            y = y.pin_memory()
        rep = Report()
        self._chk(self.lib.ngf_register(self.h, _ptr(R), _ptr(T), ctypes.byref(g), _ptr(y),
                                        int(host), ctypes.byref(rep)))
        return y, self._report(rep)

    def register_levels(self, out=None):
        my = self.level_info(0).my
        y = out if out is not None else torch.empty((3,) + my, dtype=torch.float32,
                                                    device=self.device)
        rep = Report()
        self._chk(self.lib.ngf_register_levels(self.h, _ptr(y), ctypes.byref(rep)))
        return y, self._report(rep)

    # -- differentiation form -------------------------------------------------
    def eval_pair(self, R, T, y, h=(1.0, 1.0, 1.0), grad_y=True, grad_T=True, gscale=None,
                  J_dev=None, sync=True, static=False):
        """J and gradients with respect to y and T on an explicit pair.

        Returns (J or None, grad_y or None, grad_T or None).  ``gscale`` is an
        optional device float64 scalar multiplying both gradients; ``J_dev``
        an optional device float64 scalar receiving J; with ``sync=False`` J
        is not brought to the host.  ``static=True`` calls the variant that
        allocates nothing (scratch in a static device array of the library).
        """
        self._f32(R, name="R")
        self._f32(T, R.shape, name="T")
        my = tuple(int(R.shape[d]) // self.p.ratio + 1 for d in range(3))
        self._f32(y, (3,) + my, "y")
        g = _grid(R.shape, h)
        myc = (ctypes.c_int32 * 3)(*my)
        gy = torch.empty_like(y) if grad_y else None
        gT = torch.empty_like(T) if grad_T else None
        for t, name in ((gscale, "gscale"), (J_dev, "J_dev")):
            if t is not None and not (t.dtype == torch.float64 and t.is_cuda and t.numel() == 1):
                raise TypeError(f"{name} must be a one-element float64 tensor on the GPU")
        J = ctypes.c_double()
        fn = self.lib.ngf_eval_pair_static if static else self.lib.ngf_eval_pair
        self._chk(fn(self.h, ctypes.byref(g), ctypes.byref(myc), _ptr(R), _ptr(T), _ptr(y),
                     _ptr(gscale), ctypes.byref(J) if sync else None, _ptr(J_dev), _ptr(gy),
                     _ptr(gT)))
        return (J.value if sync else None), gy, gT

    # -- standalone grid conversion -----------------------------------------
    PT_SCHEMES = {"gather": 0, "atomic": 1, "redblack": 2}

    def eval_J_grad_T(self, level, y, grad_y=True, grad_T=True, gscale=None, J_dev=None,
                      sync=True):
        """The differentiation form on pyramid level ``level`` (no allocation
        in the library).  Returns (J or None, grad_y or None, grad_T or None)."""
        li = self.level_info(level)
        self._f32(y, (3,) + li.my, "y")
        gy = torch.empty_like(y) if grad_y else None
        gT = torch.empty(li.m, dtype=torch.float32, device=self.device) if grad_T else None
        J = ctypes.c_double()
        self._chk(self.lib.ngf_eval_J_grad_T(self.h, int(level), _ptr(y), _ptr(gscale),
                                             ctypes.byref(J) if sync else None, _ptr(J_dev),
                                             _ptr(gy), _ptr(gT)))
        return (J.value if sync else None), gy, gT

    def apply_P(self, level, y):
        li = self.level_info(level)
        self._f32(y, (3,) + li.my, "y")
        yh = torch.empty((3,) + li.m, dtype=torch.float32, device=self.device)
        self._chk(self.lib.ngf_apply_P(self.h, int(level), _ptr(y), _ptr(yh)))
        return yh

    def apply_PT(self, level, z, scheme="gather"):
        li = self.level_info(level)
        self._f32(z, (3,) + li.m, "z")
        out = torch.empty((3,) + li.my, dtype=torch.float32, device=self.device)
        self._chk(self.lib.ngf_apply_PT(self.h, int(level), _ptr(z), _ptr(out),
                                        int(self.PT_SCHEMES.get(scheme, scheme))))
        return out

    # -- kernel choice --------------------------------------------------------
    VARIANTS = {"by_size": -2, "auto": -1, "tile3d": 0, "march64x8": 1, "march64x20": 2, "march64x32": 3,
                "march32x8": 4, "march32x20": 5, "march32x32": 6, "tile3d_small": 7, "tile3d_tiny": 8,
                "march64x16": 9, "march32x16": 10, "march32fit": 11, "march64fit": 12,
                "march32sq": 13, "general": 14}

    def set_kernel(self, variant):
        """Image-pass variant: 'auto' (autotune), 'by_size' (size rule), a name
        of VARIANTS, or its number."""
        v = self.VARIANTS.get(variant, variant)
        self._chk(self.lib.ngf_set_kernel(self.h, int(v)))

    def set_driver(self, mode):
        """Line search of register(): 'device' (default) or 'host'."""
        self._chk(self.lib.ngf_set_driver(self.h, {"device": 0, "host": 1}[mode]))

    def set_node_grid(self, my0=None):
        """Level-0 deformation-grid node counts per axis (None or 0 entries:
        m/ratio + 1), with 2 to 16 image cells per node cell.  Takes effect at
        the next build_pyramid / register."""
        if my0 is None:
            self._chk(self.lib.ngf_set_node_grid(self.h, None))
        else:
            arr = (ctypes.c_int32 * 3)(*[int(v) for v in my0])
            self._chk(self.lib.ngf_set_node_grid(self.h, arr))
        self.node_grid = None if my0 is None else tuple(int(v) for v in my0)

    FAULT_REJECT_STEPS = 1
    FAULT_ALLOC = 2

    def set_faults(self, flags):
        """Failure injection for tests of the error paths: a bit set of
        FAULT_REJECT_STEPS (every line-search trial fails) and FAULT_ALLOC
        (every device allocation fails); 0 clears."""
        self._chk(self.lib.ngf_set_faults(self.h, int(flags)))

    def get_kernel(self, level):
        v = ctypes.c_int32()
        self._chk(self.lib.ngf_get_kernel(self.h, int(level), ctypes.byref(v)))
        return v.value

    # -- profiling -----------------------------------------------------------
    def set_profiling(self, enable=True, level=-1):
        """HIP-event timing of the image-pass launches on ``level`` (-1: all)."""
        self._chk(self.lib.ngf_set_profiling(self.h, int(bool(enable)), int(level)))

    def kernel_time(self, level=-1):
        """(launches, total ms, voxels, nodes) of the recorded image-pass
        launches on ``level`` (-1: all); clears the record."""
        n = ctypes.c_int32()
        ms = ctypes.c_double()
        vox = ctypes.c_int64()
        nod = ctypes.c_int64()
        self._chk(self.lib.ngf_kernel_time(self.h, int(level), ctypes.byref(n), ctypes.byref(ms),
                                           ctypes.byref(vox), ctypes.byref(nod)))
        return n.value, ms.value, vox.value, nod.value


def version() -> str:
    return load().ngf_version().decode()


class Batch:
    """An ngf_batch: independent registrations of many image pairs of any
    shapes on one device, either level by level with one batched launch
    sequence per L-BFGS round over all pairs (graph mode), or on ``workers``
    host threads with a context each (threads mode).  Each pair's result
    equals the single-pair ``Context.register`` result for the same
    image-pass variants."""

    def __init__(self, alpha=0.1, tau=1.0, rho=1.0, levels=1, ratio=2, max_iter=50,
                 lbfgs_mem=5, tol_J=1e-6, early_stop=False, workers=4, mode="graph",
                 device="cuda"):
        self.lib = load()
        if not torch.cuda.is_available():
            raise RuntimeError("no HIP device visible: the ngf library has no CPU path")
        self.device = torch.device(device)
        self.p = Params(float(alpha), float(tau), float(rho), int(levels), int(ratio),
                        int(max_iter), int(lbfgs_mem), float(tol_J), int(bool(early_stop)), 0)
        h = _P()
        with torch.cuda.device(self.device):
            st = self.lib.ngf_batch_create(ctypes.byref(self.p), int(workers), ctypes.byref(h))
        if st != OK:
            raise NgfError(st, "ngf_batch_create failed")
        self.h = h
        self.built = []
        self.set_mode(mode)

    def close(self):
        if getattr(self, "h", None):
            self.lib.ngf_batch_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _chk(self, st):
        if st != OK:
            raise NgfError(st, self.lib.ngf_batch_last_error(self.h).decode())

    def set_kernel(self, variant):
        v = Context.VARIANTS.get(variant, variant)
        self._chk(self.lib.ngf_batch_set_kernel(self.h, int(v)))

    def set_mode(self, mode):
        """'graph' (default: batched launches per round, captured as a
        hipGraph) or 'threads' (worker threads, one context each)."""
        self._chk(self.lib.ngf_batch_set_mode(self.h, {"graph": 0, "threads": 1}[mode]))
        self.mode = mode

    def register(self, Rs, Ts, hs=None, out=None):
        """Register pairs (Rs[i], Ts[i]) (contiguous float32 device tensors)
        with spacings hs[i] (default 1).  Returns (list of y, list of
        per-level reports)."""
        n = len(Rs)
        if len(Ts) != n:
            raise ValueError("as many templates as references are needed")
        hs = hs if hs is not None else [(1.0, 1.0, 1.0)] * n
        grids = (Grid * max(n, 1))()
        ys = []
        for i in range(n):
            for name, t in (("R", Rs[i]), ("T", Ts[i])):
                if not (isinstance(t, torch.Tensor) and t.dtype == torch.float32 and t.is_cuda
                        and t.is_contiguous() and t.dim() == 3):
                    raise TypeError(f"{name}[{i}] must be a contiguous 3D float32 GPU tensor")
            if tuple(Rs[i].shape) != tuple(Ts[i].shape):
                raise ValueError(f"pair {i}: R and T differ in shape")
            grids[i] = _grid(Rs[i].shape, hs[i])
            my = tuple(int(v) // self.p.ratio + 1 for v in Rs[i].shape)
            y = out[i] if out is not None else torch.empty((3,) + my, dtype=torch.float32,
                                                           device=self.device)
            ys.append(y)
        arr = lambda ts: (_P * max(n, 1))(*[t.data_ptr() for t in ts])
        reps = (Report * max(n, 1))()
        stream = torch.cuda.current_stream(self.device).cuda_stream
        self._chk(self.lib.ngf_batch_register(self.h, n, arr(Rs), arr(Ts), grids, arr(ys),
                                              ctypes.c_void_p(stream), reps))
        # graph mode leaves the pairs built in its pair contexts
        self.built = [tuple(int(v) for v in R.shape) for R in Rs] if self.mode == "graph" else []
        return ys, [Context._report(reps[i]) for i in range(n)]

    def build(self, Rs, Ts, hs=None):
        """Pyramids of the pairs (Rs[i], Ts[i]) for ``eval``."""
        n = len(Rs)
        if len(Ts) != n:
            raise ValueError("as many templates as references are needed")
        hs = hs if hs is not None else [(1.0, 1.0, 1.0)] * n
        grids = (Grid * max(n, 1))()
        for i in range(n):
            for name, t in (("R", Rs[i]), ("T", Ts[i])):
                if not (isinstance(t, torch.Tensor) and t.dtype == torch.float32 and t.is_cuda
                        and t.is_contiguous() and t.dim() == 3):
                    raise TypeError(f"{name}[{i}] must be a contiguous 3D float32 GPU tensor")
            if tuple(Rs[i].shape) != tuple(Ts[i].shape):
                raise ValueError(f"pair {i}: R and T differ in shape")
            grids[i] = _grid(Rs[i].shape, hs[i])
        arr = lambda ts: (_P * max(n, 1))(*[t.data_ptr() for t in ts])
        stream = torch.cuda.current_stream(self.device).cuda_stream
        self._chk(self.lib.ngf_batch_build(self.h, n, arr(Rs), arr(Ts), grids,
                                           ctypes.c_void_p(stream)))
        self.built = [tuple(int(v) for v in R.shape) for R in Rs]

    def node_shape(self, i, level=0):
        """Node counts of pair i's deformation grid on ``level``."""
        return tuple((int(v) // self.p.ratio >> level) + 1 for v in self.built[i])

    def eval(self, level, ys, want_grad=True):
        """J and grad J of every built pair at ys[i] (contiguous float32
        device tensors of node_shape(i, level)), in batched launches.
        Returns (list of J, list of gradients or None)."""
        n = len(self.built)
        if len(ys) != n:
            raise ValueError(f"{n} pairs are built, {len(ys)} deformations given")
        for i, y in enumerate(ys):
            if not (isinstance(y, torch.Tensor) and y.dtype == torch.float32 and y.is_cuda
                    and y.is_contiguous()):
                raise TypeError(f"y[{i}] must be a contiguous float32 GPU tensor")
            if tuple(y.shape) != (3,) + self.node_shape(i, level):
                raise ValueError(f"y[{i}] has shape {tuple(y.shape)}")
        gs = [torch.empty_like(y) for y in ys] if want_grad else None
        arr = lambda ts: (_P * max(n, 1))(*[t.data_ptr() for t in ts])
        J = (ctypes.c_double * max(n, 1))()
        stream = torch.cuda.current_stream(self.device).cuda_stream
        self._chk(self.lib.ngf_batch_eval(self.h, int(level), arr(ys), J,
                                          arr(gs) if gs is not None else None,
                                          ctypes.c_void_p(stream)))
        return [J[i] for i in range(n)], gs
