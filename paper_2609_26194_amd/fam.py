"""Thin Python binding of the FAM C ABI (include/fam.h).

Argument marshalling only: every step of the scheme runs in the HIP kernels of
libfam.so.  PyTorch provides device memory (float64 CUDA/HIP tensors) and the
stream: each context owns a dedicated torch stream (default priority) that is
ordered after the caller's current stream on entry and before it on exit, so
the library can capture its steps into HIP graphs.

The module-level functions carry the C names (fam_init, fam_step, ...); the
class ``Fam`` wraps one context.
"""
import ctypes
import os
from dataclasses import dataclass

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libfam.so")

FAM_OK, FAM_ERR_ARG, FAM_ERR_DEVICE, FAM_ERR_NOMEM, FAM_ERR_NONPHYSICAL, FAM_ERR_STATE, FAM_ERR_SIZE = \
    0, -1, -2, -3, -4, -5, -6
SYSTEMS = {"advection": 0, "burgers": 1, "euler": 2}
BCS = {"periodic": 0, "transmissive": 1}
OES = {"off": 0, "type1": 1, "type2": 2}


class FamError(RuntimeError):
    def __init__(self, status, what):
        self.status = status
        super().__init__(f"{what}: {_status_str(status)} ({status})")


class NonPhysicalError(FamError):
    pass


class _CConfig(ctypes.Structure):
    _fields_ = [
        ("dim", ctypes.c_int), ("nx", ctypes.c_int), ("ny", ctypes.c_int),
        ("x0", ctypes.c_double), ("x1", ctypes.c_double), ("y0", ctypes.c_double), ("y1", ctypes.c_double),
        ("k", ctypes.c_int), ("system", ctypes.c_int), ("gamma", ctypes.c_double),
        ("ax", ctypes.c_double), ("ay", ctypes.c_double),
        ("bc_x", ctypes.c_int), ("bc_y", ctypes.c_int), ("oe", ctypes.c_int),
        ("oe_gamma_k", ctypes.c_double), ("cfl", ctypes.c_double), ("k6_jump_from_table", ctypes.c_int),
        ("pp", ctypes.c_int), ("dt_rule", ctypes.c_int), ("dmr", ctypes.c_int),
        ("char_vars", ctypes.c_int),
    ]


@dataclass
class FamConfig:
    """Python mirror of fam_config (string enums)."""
    dim: int
    nx: int
    ny: int = 1
    x0: float = 0.0
    x1: float = 1.0
    y0: float = 0.0
    y1: float = 1.0
    k: int = 5
    system: str = "euler"
    gamma: float = 1.4
    a: tuple = (1.0, 0.0)
    bc_x: str = "periodic"
    bc_y: str = "periodic"
    oe: str = "type2"
    oe_gamma_k: float = 0.0
    cfl: float = 0.2
    k6_jump_from_table: bool = False
    pp: bool = False
    dt_rule: int = 0
    dmr: bool = False
    char_vars: bool = False

    def to_c(self):
        return _CConfig(self.dim, self.nx, self.ny if self.dim == 2 else 1, self.x0, self.x1, self.y0, self.y1,
                        self.k, SYSTEMS[self.system], self.gamma, float(self.a[0]), float(self.a[1]),
                        BCS[self.bc_x], BCS[self.bc_y], OES[self.oe], self.oe_gamma_k, self.cfl,
                        int(self.k6_jump_from_table), int(self.pp), int(self.dt_rule), int(self.dmr),
                        int(self.char_vars))

    @property
    def ncomp(self):
        return self.dim + 2 if self.system == "euler" else 1

    def state_shape(self):
        if self.dim == 1:
            return (self.ncomp, 2, self.nx)
        return (self.ncomp, 3, self.ny, self.nx)


_lib = None


def load_library():
    """Load libfam.so; raises if it is missing (there is no fallback path)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with paper_2609_26194_amd/build.py")
    lib = ctypes.CDLL(LIB_PATH)
    P, D, I, VP = ctypes.POINTER(ctypes.c_double), ctypes.c_double, ctypes.c_int, ctypes.c_void_p
    sig = {
        "fam_init": (I, [ctypes.POINTER(_CConfig), VP, ctypes.POINTER(VP)]),
        "fam_init_batched": (I, [ctypes.POINTER(_CConfig), I, VP, ctypes.POINTER(VP)]),
        "fam_state_len": (ctypes.c_size_t, [VP]),
        "fam_instance_offset": (ctypes.c_size_t, [VP, I]),
        "fam_num_instances": (I, [VP]),
        "fam_step": (I, [VP, VP, D, VP]),
        "fam_run": (I, [VP, VP, D, I, D, ctypes.POINTER(I), P]),
        "fam_set_time": (I, [VP, D]),
        "fam_step_static": (I, [ctypes.POINTER(_CConfig), VP, VP, D, D, VP, VP]),
        "fam_dt": (I, [VP, VP, D, VP]),
        "fam_stage": (I, [VP, I, VP, VP, VP, VP]),
        "fam_oe": (I, [VP, VP, VP, VP]),
        "fam_check": (I, [VP]),
        "fam_adjoint": (I, [VP, VP, I, D, I, VP, VP, P]),
        "fam_autotune": (I, [VP, VP, I, ctypes.POINTER(I)]),
        "fam_set_tiling": (I, [VP, I, I]),
        "fam_dbg_recon": (I, [VP, VP, VP]),
        "fam_dbg_oe_factors": (I, [VP, VP, VP, VP]),
        "fam_destroy": (None, [VP]),
        "fam_status_str": (ctypes.c_char_p, [I]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def _status_str(s):
    try:
        return load_library().fam_status_str(s).decode()
    except Exception:  # pragma: no cover
        return "status"


def _check(status, what):
    if status == FAM_OK:
        return
    if status == FAM_ERR_NONPHYSICAL:
        raise NonPhysicalError(status, what)
    raise FamError(status, what)


def _ptr(t):
    if t is None:
        return None
    if not (t.is_cuda and t.dtype == torch.float64 and t.is_contiguous()):
        raise ValueError("state tensors must be contiguous float64 tensors on the GPU")
    return ctypes.c_void_p(t.data_ptr())


# ---------------------------------------------------------------------------
# C-named functions
# ---------------------------------------------------------------------------
def fam_init(cfg, stream_handle):
    lib = load_library()
    h = ctypes.c_void_p()
    _check(lib.fam_init(ctypes.byref(cfg.to_c()), ctypes.c_void_p(stream_handle), ctypes.byref(h)), "fam_init")
    return h


def fam_init_batched(cfgs, stream_handle):
    lib = load_library()
    arr = (_CConfig * len(cfgs))(*[c.to_c() for c in cfgs])
    h = ctypes.c_void_p()
    _check(lib.fam_init_batched(arr, len(cfgs), ctypes.c_void_p(stream_handle), ctypes.byref(h)),
           "fam_init_batched")
    return h


def fam_step(h, U, dt_fixed=0.0, dt_used=None):
    _check(load_library().fam_step(h, _ptr(U), float(dt_fixed), _ptr(dt_used)), "fam_step")


def fam_run(h, U, t_final=0.0, max_steps=0, dt_fixed=0.0):
    n, t = ctypes.c_int(0), ctypes.c_double(0.0)
    _check(load_library().fam_run(h, _ptr(U), float(t_final), int(max_steps), float(dt_fixed),
                                  ctypes.byref(n), ctypes.byref(t)), "fam_run")
    return n.value, t.value


def fam_step_static(cfg, stream_handle, U, t=0.0, dt_fixed=0.0, dt_used=None, flag=None):
    """One step on U without a context or any allocation (fam.h); flag: int32 GPU tensor or None."""
    if flag is not None and not (flag.is_cuda and flag.dtype == torch.int32):
        raise ValueError("flag: an int32 GPU tensor")
    fp = None if flag is None else ctypes.c_void_p(flag.data_ptr())
    _check(load_library().fam_step_static(ctypes.byref(cfg.to_c()), ctypes.c_void_p(stream_handle), _ptr(U),
                                          float(t), float(dt_fixed), _ptr(dt_used), fp), "fam_step_static")


def fam_set_time(h, t):
    _check(load_library().fam_set_time(h, float(t)), "fam_set_time")


def fam_dt(h, U, dt_fixed, dt_dev):
    _check(load_library().fam_dt(h, _ptr(U), float(dt_fixed), _ptr(dt_dev)), "fam_dt")


def fam_stage(h, s, U0, Us, Uout, dt_dev):
    _check(load_library().fam_stage(h, int(s), _ptr(U0), _ptr(Us), _ptr(Uout), _ptr(dt_dev)), "fam_stage")


def fam_oe(h, Un, Uout, dt_dev):
    _check(load_library().fam_oe(h, _ptr(Un), _ptr(Uout), _ptr(dt_dev)), "fam_oe")


def fam_set_tiling(h, stage_H, oe_H):
    _check(load_library().fam_set_tiling(h, int(stage_H), int(oe_H)), "fam_set_tiling")


def fam_dbg_recon(h, U, vals):
    _check(load_library().fam_dbg_recon(h, _ptr(U), _ptr(vals)), "fam_dbg_recon")


def fam_dbg_oe_factors(h, Un, dt_dev, delta):
    _check(load_library().fam_dbg_oe_factors(h, _ptr(Un), _ptr(dt_dev), _ptr(delta)), "fam_dbg_oe_factors")


def fam_check(h):
    _check(load_library().fam_check(h), "fam_check")


def fam_adjoint(h, U0, nsteps, dt, checkpoint_every, dJdUT, dJdU0):
    J = ctypes.c_double(0.0)
    _check(load_library().fam_adjoint(h, _ptr(U0), int(nsteps), float(dt), int(checkpoint_every),
                                      _ptr(dJdUT), _ptr(dJdU0), ctypes.byref(J)), "fam_adjoint")
    return J.value


def fam_autotune(h, U, reps=5):
    choice = (ctypes.c_int * 2)()
    _check(load_library().fam_autotune(h, _ptr(U), int(reps), choice), "fam_autotune")
    return int(choice[0]), int(choice[1])


def fam_state_len(h):
    return int(load_library().fam_state_len(h))


def fam_instance_offset(h, i):
    return int(load_library().fam_instance_offset(h, int(i)))


def fam_destroy(h):
    load_library().fam_destroy(h)


# ---------------------------------------------------------------------------
# context wrapper
# ---------------------------------------------------------------------------
class Fam:
    """One FAM context (single instance, or a batch of 2D instances)."""

    def __init__(self, cfg, batch=None, device="cuda"):
        if not torch.cuda.is_available():
            raise RuntimeError("the FAM library needs a HIP device")
        self.device = torch.device(device)
        self.stream = torch.cuda.Stream(device=self.device)
        self.cfgs = list(batch) if batch is not None else [cfg]
        self.cfg = self.cfgs[0]
        if batch is not None:
            self.h = fam_init_batched(self.cfgs, self.stream.cuda_stream)
        else:
            self.h = fam_init(cfg, self.stream.cuda_stream)
        self.len = fam_state_len(self.h)

    def close(self):
        if getattr(self, "h", None) is not None:
            torch.cuda.current_stream(self.device).synchronize()
            fam_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _enter(self):
        self.stream.wait_stream(torch.cuda.current_stream(self.device))

    def _leave(self):
        torch.cuda.current_stream(self.device).wait_stream(self.stream)

    def _call(self, fn, *args):
        self._enter()
        try:
            return fn(self.h, *args)
        finally:
            self._leave()

    def offsets(self):
        return [fam_instance_offset(self.h, i) for i in range(len(self.cfgs))]

    def _state(self, *Ts):
        for T in Ts:
            if T.numel() != self.len:
                raise ValueError(f"state has {T.numel()} values, the context expects {self.len}")
            _ptr(T)

    def _dt(self, d):
        if d is not None and (d.numel() < len(self.cfgs) or d.dtype != torch.float64 or not d.is_cuda):
            raise ValueError("time-step buffer: float64 GPU tensor with one value per instance")

    def step(self, U, dt_fixed=0.0, dt_used=None):
        self._state(U)
        self._dt(dt_used)
        return self._call(fam_step, U, dt_fixed, dt_used)

    def run(self, U, t_final=0.0, max_steps=0, dt_fixed=0.0):
        self._state(U)
        return self._call(fam_run, U, t_final, max_steps, dt_fixed)

    def set_time(self, t=0.0):
        """Set the context clock (the time the next step starts from)."""
        return self._call(fam_set_time, t)

    def dt(self, U, dt_fixed=0.0):
        self._state(U)
        out = torch.empty(len(self.cfgs), dtype=torch.float64, device=self.device)
        self._call(fam_dt, U, dt_fixed, out)
        return out

    def stage(self, s, U0, Us, Uout, dt_dev):
        self._state(U0, Us, Uout)
        self._dt(dt_dev)
        return self._call(fam_stage, s, U0, Us, Uout, dt_dev)

    def oe(self, Un, Uout, dt_dev):
        self._state(Un, Uout)
        self._dt(dt_dev)
        return self._call(fam_oe, Un, Uout, dt_dev)

    def check(self):
        return self._call(fam_check)

    def set_tiling(self, stage_H, oe_H):
        """Launch shapes of a single 2D instance (stage_H = 0: the limiter's segment list)."""
        return self._call(fam_set_tiling, stage_H, oe_H)

    def _cells_shape(self):
        c = self.cfgs[0]
        return (c.ny, c.nx) if c.dim == 2 else (c.nx,)

    def dbg_recon(self, U):
        """Point values of the stage reconstruction at every cell's flux points (test export):
        [ncomp, 32, ny, nx] in 2D, [ncomp, 6, nx] in 1D (point order as in fam.h)."""
        self._state(U)
        c = self.cfgs[0]
        npts = 32 if c.dim == 2 else 6
        vals = torch.empty((c.ncomp, npts) + self._cells_shape(), dtype=torch.float64, device=self.device)
        self._call(fam_dbg_recon, U, vals)
        return vals

    def dbg_oe_factors(self, Un, dt_dev):
        """OE damping factor delta of every cell for Un and the time step in dt_dev (test export)."""
        self._state(Un)
        self._dt(dt_dev)
        delta = torch.empty(self._cells_shape(), dtype=torch.float64, device=self.device)
        self._call(fam_dbg_oe_factors, Un, dt_dev, delta)
        return delta

    def autotune(self, U, reps=5):
        """Pick the fastest launch shapes for this context on state U (read only)."""
        self._state(U)
        return self._call(fam_autotune, U, reps)

    def adjoint(self, U0, nsteps, dt, checkpoint_every, dJdUT=None):
        self._state(U0)
        if dJdUT is not None:
            self._state(dJdUT)
        dJdU0 = torch.empty_like(U0)
        J = self._call(fam_adjoint, U0, nsteps, dt, checkpoint_every, dJdUT, dJdU0)
        return J, dJdU0
