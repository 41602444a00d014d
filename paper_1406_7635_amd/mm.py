"""Python binding of libmm (include/mm.h): argument marshalling only.

Every computation happens in the HIP library; this module converts torch
tensors and Python values into the C ABI's pointers and structs.  Importing it
does not touch the GPU; creating a Context needs the built libmm.so (it raises
if the library is missing -- there is no fallback path).
"""
import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.environ.get("MM_LIBRARY") or os.path.join(_HERE, "libmm.so")
NREG = 256
NPAIR = NREG * (NREG + 1) // 2
PREC = {"fp32": 0, "bf16": 1, "fp16": 2}  # mm_precision

c_int32, c_int64, c_double, c_void_p = ctypes.c_int32, ctypes.c_int64, ctypes.c_double, ctypes.c_void_p

STATUS = {0: "MM_OK", -1: "MM_EINVAL", -2: "MM_ENOMEM", -3: "MM_EDEVICE", -4: "MM_EUNSUPPORTED",
          -5: "MM_ENONFINITE", -6: "MM_ESTEP", -7: "MM_ENOTCONVERGED", -8: "MM_ESTATE", -9: "MM_ESCRATCH"}


class Grid(ctypes.Structure):
    _fields_ = [("nx", c_int32), ("ny", c_int32), ("nz", c_int32),
                ("dx", c_double), ("dy", c_double), ("dz", c_double), ("pbc", c_int32 * 3)]


class Params(ctypes.Structure):
    _fields_ = [("msat", c_double * NREG), ("aex", c_double * NREG), ("alpha", c_double * NREG),
                ("ku1", c_double * NREG), ("ku2", c_double * NREG),
                ("anis_u", (c_double * 3) * NREG), ("bext", (c_double * 3) * NREG),
                ("exch_scale", c_double * NPAIR), ("gamma_ll", c_double)]


class SolverOpts(ctypes.Structure):
    _fields_ = [("max_err", c_double), ("headroom", c_double), ("dt_min", c_double),
                ("dt_max", c_double), ("precess", c_int32), ("reserved", c_int32)]


class RunStats(ctypes.Structure):
    _fields_ = [("steps", c_int64), ("rejects", c_int64), ("evals", c_int64),
                ("t", c_double), ("dt", c_double), ("err", c_double)]


class Info(ctypes.Structure):
    _fields_ = [("px", c_int32), ("py", c_int32), ("pz", c_int32), ("kx", c_int32),
                ("ncomp", c_int32), ("reserved", c_int32), ("ncell", c_int64),
                ("khat_elems", c_int64), ("device_bytes", c_int64)]


EXPORTS = {
    "mm_create": (c_int32, [ctypes.POINTER(c_void_p), ctypes.POINTER(Grid), ctypes.POINTER(Params), c_void_p, c_void_p]),
    "mm_demag_kernel_init": (c_int32, [c_void_p]),
    "mm_set_params": (c_int32, [c_void_p, ctypes.POINTER(Params)]),
    "mm_set_demag": (c_int32, [c_void_p, c_int32]),
    "mm_set_temperature": (c_int32, [c_void_p, c_void_p, ctypes.c_uint64]),
    "mm_thermal_field": (c_int32, [c_void_p, c_double, ctypes.c_uint64, c_void_p]),
    "mm_set_cubic_anisotropy": (c_int32, [c_void_p, c_void_p, c_void_p, c_void_p]),
    "mm_set_dmi": (c_int32, [c_void_p, c_void_p]),
    "mm_set_run_graphs": (c_int32, [c_void_p, c_int32]),
    "mm_set_excitation": (c_int32, [c_void_p, c_int32, c_void_p, c_double, c_double, c_double, c_double]),
    "mm_beff": (c_int32, [c_void_p, c_void_p, c_void_p, c_void_p]),
    "mm_beff_noalloc": (c_int32, [c_void_p, c_void_p, c_void_p, c_void_p]),
    "mm_llg_torque": (c_int32, [c_void_p, c_void_p, c_void_p, c_void_p, c_int32]),
    "mm_torque": (c_int32, [c_void_p, c_void_p, c_void_p, c_int32]),
    "mm_rk4_step": (c_int32, [c_void_p, c_void_p, c_double, c_int32]),
    "mm_rk45_step": (c_int32, [c_void_p, c_void_p, ctypes.POINTER(c_double), ctypes.POINTER(c_double),
                               ctypes.POINTER(SolverOpts), ctypes.POINTER(c_int32), ctypes.POINTER(c_double)]),
    "mm_rk23_step": (c_int32, [c_void_p, c_void_p, ctypes.POINTER(c_double), ctypes.POINTER(c_double),
                               ctypes.POINTER(SolverOpts), ctypes.POINTER(c_int32), ctypes.POINTER(c_double)]),
    "mm_run": (c_int32, [c_void_p, c_void_p, c_int32, c_double, c_int64, ctypes.POINTER(c_double),
                         ctypes.POINTER(c_double), ctypes.POINTER(SolverOpts), ctypes.POINTER(RunStats)]),
    "mm_relax": (c_int32, [c_void_p, c_void_p, ctypes.POINTER(SolverOpts), c_double, c_int64,
                           ctypes.POINTER(c_double), ctypes.POINTER(c_double), ctypes.POINTER(c_int64)]),
    "mm_energy": (c_int32, [c_void_p, c_void_p, ctypes.POINTER(c_double)]),
    "mm_max_torque": (c_int32, [c_void_p, c_void_p, c_int32, ctypes.POINTER(c_double)]),
    "mm_solver_reset": (c_int32, [c_void_p]),
    "mm_get_info": (c_int32, [c_void_p, ctypes.POINTER(Info)]),
    "mm_state_size": (c_int32, [c_void_p, ctypes.POINTER(c_int64)]),
    "mm_state_save": (c_int32, [c_void_p, c_void_p, c_int64]),
    "mm_state_load": (c_int32, [c_void_p, c_void_p, c_int64, c_void_p]),
    "mm_demag_tensor_dump": (c_int32, [c_void_p, c_void_p]),
    "mm_demag_kernel_dump": (c_int32, [c_void_p, c_void_p]),
    "mm_exchange_dump": (c_int32, [c_void_p, c_void_p]),
    "mm_set_conv_precision": (c_int32, [c_void_p, c_int32]),
    "mm_timing_enable": (c_int32, [c_void_p, c_int32, c_int32]),
    "mm_timing_read": (c_int32, [c_void_p, c_int32, ctypes.POINTER(c_int64), ctypes.POINTER(c_double)]),
    "mm_batch_create": (c_int32, [ctypes.POINTER(c_void_p), c_int32, ctypes.POINTER(Grid), ctypes.POINTER(Params),
                                  c_void_p, c_void_p]),
    "mm_batch_demag_kernel_init": (c_int32, [c_void_p]),
    "mm_batch_member": (c_int32, [c_void_p, c_int32, ctypes.POINTER(c_int64), ctypes.POINTER(c_int64)]),
    "mm_batch_beff": (c_int32, [c_void_p, c_void_p, c_void_p]),
    "mm_batch_start": (c_int32, [c_void_p, c_int32, c_double, c_double, c_double, ctypes.POINTER(SolverOpts)]),
    "mm_batch_run": (c_int32, [c_void_p, c_void_p, c_int64, ctypes.POINTER(c_int64), ctypes.POINTER(c_int32)]),
    "mm_batch_stats": (c_int32, [c_void_p, c_int32, ctypes.POINTER(RunStats), ctypes.POINTER(c_int32)]),
    "mm_batch_stats_all": (c_int32, [c_void_p, ctypes.POINTER(RunStats), ctypes.POINTER(c_int32)]),
    "mm_batch_set_graph": (c_int32, [c_void_p, c_int32]),
    "mm_batch_set_grid": (c_int32, [c_void_p, c_int32, c_int32]),
    "mm_batch_get_grid": (c_int32, [c_void_p, c_int32, ctypes.POINTER(c_int32)]),
    "mm_batch_set_tile": (c_int32, [c_void_p, c_int32, c_int32]),
    "mm_batch_get_tile": (c_int32, [c_void_p, c_int32, ctypes.POINTER(c_int32)]),
    "mm_batch_autotune": (c_int32, [c_void_p, c_void_p]),
    "mm_batch_destroy": (None, [c_void_p]),
    "mm_sno_create": (c_int32, [ctypes.POINTER(c_void_p), c_int32, c_int32, c_void_p, c_int64, c_double,
                                c_void_p]),
    "mm_sno_set_weights": (c_int32, [c_void_p, c_void_p, c_int64]),
    "mm_sno_eval": (c_int32, [c_void_p, c_void_p, c_void_p]),
    "mm_sno_destroy": (None, [c_void_p]),
    "mm_set_surrogate": (c_int32, [c_void_p, c_void_p, c_double]),
    "mm_surrogate_stats": (c_int32, [c_void_p, ctypes.POINTER(c_int64), ctypes.POINTER(c_int64),
                                     ctypes.POINTER(c_double)]),
    "mm_sno_train_create": (c_int32, [ctypes.POINTER(c_void_p), c_int32, c_int32, c_int32, c_void_p, c_int64,
                                      c_void_p]),
    "mm_sno_train_grad": (c_int32, [c_void_p, c_void_p, c_void_p, c_void_p, ctypes.POINTER(c_double)]),
    "mm_sno_train_step": (c_int32, [c_void_p, c_void_p, c_void_p, c_double, ctypes.POINTER(c_double)]),
    "mm_sno_train_get_weights": (c_int32, [c_void_p, c_void_p]),
    "mm_sno_train_destroy": (None, [c_void_p]),
    "mm_destroy": (None, [c_void_p]),
    "mm_strerror": (ctypes.c_char_p, [c_int32]),
}

_lib = None


def load():
    """Load libmm.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("libmm.so is not built (python -m paper_1406_7635_amd.build)")
        lib = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in EXPORTS.items():
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _lib = lib
    return _lib


class MMError(RuntimeError):
    def __init__(self, status, where):
        self.status = status
        msg = load().mm_strerror(status).decode()
        super().__init__("%s: %s (%s)" % (where, STATUS.get(status, status), msg))


def _check(status, where):
    if status != 0:
        raise MMError(status, where)


def params_struct(p):
    """Fill the C struct from a dict of region tables (see synth.empty_params)."""
    s = Params()
    for key in ("msat", "aex", "alpha", "ku1", "ku2"):
        np.ctypeslib.as_array(getattr(s, key))[:] = np.asarray(p[key], dtype=np.float64)
    np.ctypeslib.as_array(s.anis_u)[:] = np.asarray(p["anis_u"], dtype=np.float64).reshape(NREG, 3)
    np.ctypeslib.as_array(s.bext)[:] = np.asarray(p["bext"], dtype=np.float64).reshape(NREG, 3)
    np.ctypeslib.as_array(s.exch_scale)[:] = np.asarray(p["exch_scale"], dtype=np.float64)
    s.gamma_ll = float(p.get("gamma_ll", 0.0) or 0.0)
    return s


def solver_opts(max_err=1e-5, headroom=0.8, dt_min=0.0, dt_max=0.0, precess=True):
    return SolverOpts(max_err, headroom, dt_min, dt_max, 1 if precess else 0, 0)


def _ptr(t):
    return c_void_p(t.data_ptr()) if t is not None else c_void_p(0)


class Context:
    """One simulation grid on the current CUDA (HIP) device.

    grid (nx, ny, nz), cell (dx, dy, dz) in m, region uint8 [nz, ny, nx]
    (numpy or tensor), params dict of region tables; pbc (Px, Py, Pz): images
    per side along each axis (0: open boundary)."""

    def __init__(self, grid, cell, region, params, demag=True, stream=None, pbc=(0, 0, 0)):
        import torch

        self._torch = torch
        lib = load()
        self.grid = tuple(int(v) for v in grid)
        self.cell = tuple(float(v) for v in cell)
        nx, ny, nz = self.grid
        self.shape = (3, nz, ny, nx)
        self.device = torch.device("cuda", torch.cuda.current_device())
        reg = torch.as_tensor(np.ascontiguousarray(region, dtype=np.uint8)
                              if not isinstance(region, torch.Tensor) else region)
        if tuple(reg.shape) != (nz, ny, nx):
            raise ValueError("region must have shape (nz, ny, nx) = %s" % ((nz, ny, nx),))
        self._region = reg.to(self.device, torch.uint8).contiguous()
        self._stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        self.pbc = tuple(int(v) for v in pbc)
        g = Grid(nx, ny, nz, *self.cell, (c_int32 * 3)(*self.pbc))
        self._params = params_struct(params)
        handle = c_void_p()
        _check(lib.mm_create(ctypes.byref(handle), ctypes.byref(g), ctypes.byref(self._params),
                             _ptr(self._region), c_void_p(self._stream.cuda_stream)), "mm_create")
        self._h = handle
        if "kc" in params:
            self.set_cubic_anisotropy(params["kc"], params["anis_c1"], params["anis_c2"])
        if "dind" in params:
            self.set_dmi(params["dind"])
        self.demag = bool(demag)
        if self.demag:
            _check(lib.mm_demag_kernel_init(self._h), "mm_demag_kernel_init")
        else:
            _check(lib.mm_set_demag(self._h, 0), "mm_set_demag")

    # -- helpers -----------------------------------------------------------
    def _vec(self, m, name="m"):
        t = self._torch
        if not isinstance(m, t.Tensor) or m.dtype != t.float32 or m.device != self.device \
                or tuple(m.shape) != self.shape or not m.is_contiguous():
            raise ValueError("%s must be a contiguous float32 %s tensor on %s" % (name, self.shape, self.device))
        return m

    def new_field(self):
        return self._torch.empty(self.shape, dtype=self._torch.float32, device=self.device)

    def close(self):
        if getattr(self, "_h", None):
            load().mm_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- API -----------------------------------------------------------------
    def set_params(self, params):
        """New region tables; a params dict with cubic keys ("kc", "anis_c1",
        "anis_c2") or the DMI key "dind" also sets those terms."""
        self._params = params_struct(params)
        _check(load().mm_set_params(self._h, ctypes.byref(self._params)), "mm_set_params")
        if "kc" in params:
            self.set_cubic_anisotropy(params["kc"], params["anis_c1"], params["anis_c2"])
        if "dind" in params:
            self.set_dmi(params["dind"])

    def set_demag(self, enable):
        if enable and not self.demag:
            _check(load().mm_demag_kernel_init(self._h), "mm_demag_kernel_init")
        self.demag = bool(enable)
        _check(load().mm_set_demag(self._h, 1 if enable else 0), "mm_set_demag")

    def beff(self, m, want_demag=False):
        m = self._vec(m)
        b = self.new_field()
        bd = self.new_field() if want_demag else None
        _check(load().mm_beff(self._h, _ptr(m), _ptr(b), _ptr(bd)), "mm_beff")
        return (b, bd) if want_demag else b

    def beff_noalloc(self, m, b, bd=None):
        """mm_beff_noalloc into caller tensors b (and bd); the spectrum is the
        library's static per-GPU array, so the call allocates nothing."""
        bd = self._vec(bd, "bd") if bd is not None else None
        _check(load().mm_beff_noalloc(self._h, _ptr(self._vec(m)), _ptr(self._vec(b, "b")), _ptr(bd)),
               "mm_beff_noalloc")
        return b

    def llg_torque(self, m, beff, precess=True):
        tau = self.new_field()
        _check(load().mm_llg_torque(self._h, _ptr(self._vec(m)), _ptr(self._vec(beff, "beff")), _ptr(tau),
                                    1 if precess else 0), "mm_llg_torque")
        return tau

    def torque(self, m, precess=True):
        tau = self.new_field()
        _check(load().mm_torque(self._h, _ptr(self._vec(m)), _ptr(tau), 1 if precess else 0), "mm_torque")
        return tau

    def rk4_step(self, m, dt, precess=True):
        _check(load().mm_rk4_step(self._h, _ptr(self._vec(m)), float(dt), 1 if precess else 0), "mm_rk4_step")

    def rk45_step(self, m, t, dt, opts=None):
        return self._embedded(load().mm_rk45_step, "mm_rk45_step", m, t, dt, opts)

    def rk23_step(self, m, t, dt, opts=None):
        return self._embedded(load().mm_rk23_step, "mm_rk23_step", m, t, dt, opts)

    def _embedded(self, fn, name, m, t, dt, opts):
        t_, dt_, acc, err = c_double(t), c_double(dt), c_int32(0), c_double(0.0)
        o = opts if opts is not None else solver_opts()
        _check(fn(self._h, _ptr(self._vec(m)), ctypes.byref(t_), ctypes.byref(dt_), ctypes.byref(o),
                  ctypes.byref(acc), ctypes.byref(err)), name)
        return bool(acc.value), t_.value, dt_.value, err.value

    def run(self, m, t_end, t=0.0, dt=1e-14, solver=45, max_attempts=10 ** 9, opts=None):
        """Device-controlled adaptive run; returns (t, dt, stats dict)."""
        t_, dt_ = c_double(t), c_double(dt)
        st = RunStats()
        o = opts if opts is not None else solver_opts()
        _check(load().mm_run(self._h, _ptr(self._vec(m)), int(solver), float(t_end), int(max_attempts),
                             ctypes.byref(t_), ctypes.byref(dt_), ctypes.byref(o), ctypes.byref(st)), "mm_run")
        return t_.value, dt_.value, {k: getattr(st, k) for k, _ in RunStats._fields_}

    def set_temperature(self, temp, seed=0):
        """Temperature in K: a scalar (every region) or 256 values per region;
        seed of the thermal generator (resets its step counter)."""
        t = np.broadcast_to(np.asarray(temp, dtype=np.float64), (256,)).copy()
        self._temp = t
        _check(load().mm_set_temperature(self._h, t.ctypes.data_as(c_void_p), int(seed) & ((1 << 64) - 1)),
               "mm_set_temperature")

    def set_cubic_anisotropy(self, kc, c1, c2):
        """Cubic anisotropy per region: kc [256, 3] (Kc1, Kc2, Kc3) in J/m^3, axes
        c1, c2 [256, 3]; kc None removes it."""
        if kc is None:
            _check(load().mm_set_cubic_anisotropy(self._h, None, None, None), "mm_set_cubic_anisotropy")
            return
        arrs = [np.ascontiguousarray(np.broadcast_to(np.asarray(v, dtype=np.float64), (256, 3))) for v in (kc, c1, c2)]
        self._cub = arrs
        _check(load().mm_set_cubic_anisotropy(self._h, *(x.ctypes.data_as(c_void_p) for x in arrs)),
               "mm_set_cubic_anisotropy")

    def set_excitation(self, slot, g, a=0.0, b=1.0, omega=0.0, phi=0.0):
        """Excitation term `slot`: (a + b sin(omega t + phi)) * g, g a float32
        [3, nz, ny, nx] tensor on the device (kept alive here); g None clears."""
        if not hasattr(self, "_exc"):
            self._exc = {}
        if g is None:
            self._exc.pop(slot, None)
            _check(load().mm_set_excitation(self._h, int(slot), None, 0.0, 0.0, 0.0, 0.0), "mm_set_excitation")
            return
        self._exc[slot] = self._vec(g, "g")
        _check(load().mm_set_excitation(self._h, int(slot), _ptr(self._exc[slot]), float(a), float(b), float(omega),
                                        float(phi)), "mm_set_excitation")

    def set_run_graphs(self, enable):
        """Replay a captured attempt in run() (on by default)."""
        _check(load().mm_set_run_graphs(self._h, 1 if enable else 0), "mm_set_run_graphs")

    def set_dmi(self, dind):
        """Induced DMI constant D per region (J/m^2, scalar or 256 values);
        None removes it."""
        if dind is None:
            _check(load().mm_set_dmi(self._h, None), "mm_set_dmi")
            return
        self._dind = np.ascontiguousarray(np.broadcast_to(np.asarray(dind, dtype=np.float64), (256,)))
        _check(load().mm_set_dmi(self._h, self._dind.ctypes.data_as(c_void_p)), "mm_set_dmi")

    def thermal_field(self, dt, step):
        """The thermal field [3, nz, ny, nx] (T) of generator step `step` at time step dt."""
        out = self.new_field()
        _check(load().mm_thermal_field(self._h, float(dt), int(step), _ptr(out)), "mm_thermal_field")
        return out

    def relax(self, m, max_err=1e-5, min_max_err=1e-9, max_steps=100000):
        e, tq, n = c_double(), c_double(), c_int64()
        o = solver_opts(max_err=max_err, precess=False)
        st = load().mm_relax(self._h, _ptr(self._vec(m)), ctypes.byref(o), float(min_max_err), int(max_steps),
                             ctypes.byref(e), ctypes.byref(tq), ctypes.byref(n))
        if st not in (0, -7):
            _check(st, "mm_relax")
        return {"energy": e.value, "max_torque": tq.value, "steps": n.value, "converged": st == 0}

    def energy(self, m):
        out = (c_double * 5)()
        _check(load().mm_energy(self._h, _ptr(self._vec(m)), out), "mm_energy")
        return dict(zip(("demag", "exch", "anis", "zeeman", "total"), list(out)))

    def max_torque(self, m, precess=True):
        v = c_double()
        _check(load().mm_max_torque(self._h, _ptr(self._vec(m)), 1 if precess else 0, ctypes.byref(v)),
               "mm_max_torque")
        return v.value

    def reset_solver(self):
        _check(load().mm_solver_reset(self._h), "mm_solver_reset")

    def info(self):
        inf = Info()
        _check(load().mm_get_info(self._h, ctypes.byref(inf)), "mm_get_info")
        return {k: getattr(inf, k) for k, _ in Info._fields_}

    def state_save(self):
        """Solver state (bytes) that continues a run bit for bit with the same
        m and the (t, dt) mm_run returned (mm_state_save)."""
        n = c_int64()
        _check(load().mm_state_size(self._h, ctypes.byref(n)), "mm_state_size")
        buf = ctypes.create_string_buffer(n.value)
        _check(load().mm_state_save(self._h, buf, n.value), "mm_state_save")
        return buf.raw

    def state_load(self, state, m):
        """Restore a saved solver state; m holds the saved magnetisation."""
        buf = ctypes.create_string_buffer(bytes(state), len(state))
        _check(load().mm_state_load(self._h, buf, len(state), _ptr(self._vec(m))), "mm_state_load")

    def tensor_dump(self):
        """FP64 real-space tensor octant [6, nz, ny, nx] as the GPU computes it."""
        nx, ny, nz = self.grid
        out = self._torch.empty((6, nz, ny, nx), dtype=self._torch.float64, device=self.device)
        _check(load().mm_demag_tensor_dump(self._h, _ptr(out)), "mm_demag_tensor_dump")
        return out

    def kernel_dump(self):
        out = self._torch.empty(self.info()["khat_elems"], dtype=self._torch.float32, device=self.device)
        _check(load().mm_demag_kernel_dump(self._h, _ptr(out)), "mm_demag_kernel_dump")
        return out

    def exchange_dump(self):
        nx, ny, nz = self.grid
        out = self._torch.empty((6, nz, ny, nx), dtype=self._torch.float32, device=self.device)
        _check(load().mm_exchange_dump(self._h, _ptr(out)), "mm_exchange_dump")
        return out

    def set_conv_precision(self, prec):
        """DFT arithmetic of the y convolution: 'fp32', or 'bf16' / 'fp16' split
        precision on the matrix cores (2D grids with padded y length 2048)."""
        _check(load().mm_set_conv_precision(self._h, PREC[prec] if isinstance(prec, str) else int(prec)),
               "mm_set_conv_precision")

    def set_surrogate(self, surrogate, tol=1e-4):
        """Inner Dormand-Prince stages of run() take B_demag from `surrogate`
        (an mm.Surrogate, or None to detach), checked against the exact field
        at every attempt's last stage; a miss falls back to the exact path."""
        self._surrogate = surrogate
        _check(load().mm_set_surrogate(self._h, surrogate._h if surrogate is not None else c_void_p(0),
                                       float(tol)), "mm_set_surrogate")

    def surrogate_stats(self):
        n, f, e = c_int64(), c_int64(), c_double()
        _check(load().mm_surrogate_stats(self._h, ctypes.byref(n), ctypes.byref(f), ctypes.byref(e)),
               "mm_surrogate_stats")
        return {"surrogate_steps": n.value, "fallbacks": f.value, "last_err": e.value}

    def timing_enable(self, which, enable=True):
        _check(load().mm_timing_enable(self._h, int(which), 1 if enable else 0), "mm_timing_enable")

    def timing_read(self, which):
        n, ms = c_int64(), c_double()
        _check(load().mm_timing_read(self._h, int(which), ctypes.byref(n), ctypes.byref(ms)), "mm_timing_read")
        return n.value, ms.value


BATCH_PASSES = ("x", "conv2d", "y", "z4", "z8", "z16", "yz4", "yz8", "finalize")  # mm_batch_set_grid pass ids
BATCH_TILES = ("wide", "narrow")  # mm_batch_set_tile shapes


class Batch:
    """An ensemble of independent grids advanced together (mm_batch_*).

    members: list of dicts with "grid" (nx, ny, nz), "cell" (dx, dy, dz),
    "region" uint8 [nz, ny, nx] and "params" (dict of region tables).  State
    and field tensors are the members' [3, nz, ny, nx] arrays back to back
    (member i at floats [3 off_i, 3 off_i + 3 ncell_i))."""

    def __init__(self, members, stream=None):
        import torch

        self._torch = torch
        lib = load()
        n = len(members)
        self.n = n
        self.device = torch.device("cuda", torch.cuda.current_device())
        grids = (Grid * n)()
        params = (Params * n)()
        regs = []
        self.grids = []
        for i, mb in enumerate(members):
            nx, ny, nz = (int(v) for v in mb["grid"])
            grids[i] = Grid(nx, ny, nz, *(float(v) for v in mb["cell"]), (c_int32 * 3)(0, 0, 0))
            params[i] = params_struct(mb["params"])
            r = np.ascontiguousarray(mb["region"], dtype=np.uint8)
            if r.shape != (nz, ny, nx):
                raise ValueError("member %d: region must have shape %s" % (i, (nz, ny, nx)))
            regs.append(r.reshape(-1))
            self.grids.append((nx, ny, nz))
        self._region = torch.from_numpy(np.concatenate(regs)).to(self.device)
        self._stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        handle = c_void_p()
        _check(lib.mm_batch_create(ctypes.byref(handle), n, grids, params, _ptr(self._region),
                                   c_void_p(self._stream.cuda_stream)), "mm_batch_create")
        self._h = handle
        self.offsets, self.ncells = [], []
        for i in range(n):
            off, nc = c_int64(), c_int64()
            _check(lib.mm_batch_member(self._h, i, ctypes.byref(off), ctypes.byref(nc)), "mm_batch_member")
            self.offsets.append(off.value)
            self.ncells.append(nc.value)
        self.ncell = sum(self.ncells)
        _check(lib.mm_batch_demag_kernel_init(self._h), "mm_batch_demag_kernel_init")

    def close(self):
        if getattr(self, "_h", None):
            load().mm_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _vec(self, m, name="m"):
        t = self._torch
        if not isinstance(m, t.Tensor) or m.dtype != t.float32 or m.device != self.device \
                or m.numel() != 3 * self.ncell or not m.is_contiguous():
            raise ValueError("%s must be a contiguous float32 tensor of %d elements on %s"
                             % (name, 3 * self.ncell, self.device))
        return m

    def new_field(self):
        return self._torch.empty(3 * self.ncell, dtype=self._torch.float32, device=self.device)

    def member(self, t, i):
        """View of member i's [3, nz, ny, nx] block of an ensemble array."""
        nx, ny, nz = self.grids[i]
        o = 3 * self.offsets[i]
        return t[o:o + 3 * self.ncells[i]].view(3, nz, ny, nx)

    def pack(self, arrays):
        """Ensemble array from the members' [3, nz, ny, nx] arrays (numpy or tensors)."""
        out = self.new_field()
        for i, a in enumerate(arrays):
            self.member(out, i).copy_(self._torch.as_tensor(np.asarray(a, dtype=np.float32)))
        return out

    def beff(self, m):
        b = self.new_field()
        _check(load().mm_batch_beff(self._h, _ptr(self._vec(m)), _ptr(b)), "mm_batch_beff")
        return b

    def start(self, solver=45, t0=0.0, dt0=1e-14, t_end=float("inf"), opts=None):
        o = opts if opts is not None else solver_opts()
        _check(load().mm_batch_start(self._h, int(solver), float(t0), float(dt0), float(t_end), ctypes.byref(o)),
               "mm_batch_start")

    def run(self, m, max_attempts):
        """Attempt steps of every running member; returns (attempts, members still running)."""
        na, act = c_int64(), c_int32()
        _check(load().mm_batch_run(self._h, _ptr(self._vec(m)), int(max_attempts), ctypes.byref(na),
                                   ctypes.byref(act)), "mm_batch_run")
        return na.value, act.value

    def stats(self, i):
        st, status = RunStats(), c_int32()
        _check(load().mm_batch_stats(self._h, int(i), ctypes.byref(st), ctypes.byref(status)), "mm_batch_stats")
        d = {k: getattr(st, k) for k, _ in RunStats._fields_}
        d["status"] = status.value
        return d

    def stats_all(self):
        """Per-member counters as arrays (steps, rejects, evals, t, dt, err, status)."""
        st, status = (RunStats * self.n)(), (c_int32 * self.n)()
        _check(load().mm_batch_stats_all(self._h, st, status), "mm_batch_stats_all")
        out = {k: np.array([getattr(s, k) for s in st]) for k, _ in RunStats._fields_}
        out["status"] = np.array(list(status))
        return out

    def set_graph(self, enable):
        _check(load().mm_batch_set_graph(self._h, 1 if enable else 0), "mm_batch_set_graph")

    def set_grid(self, pass_, grid):
        p = BATCH_PASSES.index(pass_) if isinstance(pass_, str) else int(pass_)
        _check(load().mm_batch_set_grid(self._h, p, int(grid)), "mm_batch_set_grid")

    def get_grid(self, pass_):
        p = BATCH_PASSES.index(pass_) if isinstance(pass_, str) else int(pass_)
        g = c_int32()
        _check(load().mm_batch_get_grid(self._h, p, ctypes.byref(g)), "mm_batch_get_grid")
        return g.value

    def set_tile(self, pass_, tile):
        """Tile shape of the x passes ("x") or the 2D y convolution
        ("conv2d"): "wide" or "narrow"."""
        p = BATCH_PASSES.index(pass_) if isinstance(pass_, str) else int(pass_)
        t = BATCH_TILES.index(tile) if isinstance(tile, str) else int(tile)
        _check(load().mm_batch_set_tile(self._h, p, t), "mm_batch_set_tile")

    def get_tile(self, pass_):
        p = BATCH_PASSES.index(pass_) if isinstance(pass_, str) else int(pass_)
        t = c_int32()
        _check(load().mm_batch_get_tile(self._h, p, ctypes.byref(t)), "mm_batch_get_tile")
        return BATCH_TILES[t.value]

    def autotune(self, m):
        """Tuned persistent grids per pass (0: a pass no member uses); the
        tuned tile shapes are read with get_tile."""
        _check(load().mm_batch_autotune(self._h, _ptr(self._vec(m))), "mm_batch_autotune")
        return {name: self.get_grid(i) for i, name in enumerate(BATCH_PASSES)}


SNO_NWEIGHTS = 2101603  # MM_SNO_NWEIGHTS


class Surrogate:
    """The spectral neural operator (mm_sno_*): predicted B_demag of m on an
    nx x ny x 1 grid, B = out_scale * network(m).  weights: the flat FP32
    array (numpy), rounded to BF16 by the library."""

    def __init__(self, nx, ny, weights, out_scale, stream=None):
        import torch

        self._torch = torch
        self.grid = (int(nx), int(ny), 1)
        self.device = torch.device("cuda", torch.cuda.current_device())
        self._stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        w = np.ascontiguousarray(weights, dtype=np.float32)
        h = c_void_p()
        _check(load().mm_sno_create(ctypes.byref(h), int(nx), int(ny), w.ctypes.data_as(c_void_p), w.size,
                                    float(out_scale), c_void_p(self._stream.cuda_stream)), "mm_sno_create")
        self._h = h

    def set_weights(self, weights):
        w = np.ascontiguousarray(weights, dtype=np.float32)
        _check(load().mm_sno_set_weights(self._h, w.ctypes.data_as(c_void_p), w.size), "mm_sno_set_weights")

    def __call__(self, m, out=None):
        nx, ny, _ = self.grid
        t = self._torch
        if not isinstance(m, t.Tensor) or m.dtype != t.float32 or m.numel() != 3 * nx * ny \
                or not m.is_contiguous() or m.device != self.device:
            raise ValueError("m must be a contiguous float32 tensor of 3 x %d x %d on %s" % (ny, nx, self.device))
        b = out if out is not None else t.empty((3, 1, ny, nx), dtype=t.float32, device=self.device)
        _check(load().mm_sno_eval(self._h, _ptr(m), _ptr(b)), "mm_sno_eval")
        return b

    def close(self):
        if getattr(self, "_h", None):
            load().mm_sno_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class SurrogateTrainer:
    """Training of the surrogate on the GPU (mm_sno_train_*): FP32 master
    weights, Adam, batches of `batch` samples on an nx x ny grid.  m and
    target: float32 tensors [batch, 3, ny, nx] (or [batch, 3, 1, ny, nx]) on
    the device, target in the network's output units (B_demag / out_scale)."""

    def __init__(self, nx, ny, batch, weights, stream=None):
        import torch

        self._torch = torch
        self.grid = (int(nx), int(ny))
        self.batch = int(batch)
        self.device = torch.device("cuda", torch.cuda.current_device())
        self._stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        w = np.ascontiguousarray(weights, dtype=np.float32)
        h = c_void_p()
        _check(load().mm_sno_train_create(ctypes.byref(h), int(nx), int(ny), int(batch), w.ctypes.data_as(c_void_p),
                                          w.size, c_void_p(self._stream.cuda_stream)), "mm_sno_train_create")
        self._h = h

    def _batch(self, x, name):
        t = self._torch
        nx, ny = self.grid
        if not isinstance(x, t.Tensor) or x.dtype != t.float32 or x.device != self.device \
                or x.numel() != self.batch * 3 * nx * ny or not x.is_contiguous():
            raise ValueError("%s must be a contiguous float32 tensor of %d x 3 x %d x %d on %s"
                             % (name, self.batch, ny, nx, self.device))
        return x

    def grad(self, m, target):
        """(loss, gradient tensor of MM_SNO_NWEIGHTS floats) without an update."""
        g = self._torch.empty(SNO_NWEIGHTS, dtype=self._torch.float32, device=self.device)
        loss = c_double()
        _check(load().mm_sno_train_grad(self._h, _ptr(self._batch(m, "m")), _ptr(self._batch(target, "target")),
                                        _ptr(g), ctypes.byref(loss)), "mm_sno_train_grad")
        return loss.value, g

    def step(self, m, target, lr, want_loss=True):
        """One Adam step; returns the batch loss before the update (or None)."""
        loss = c_double()
        _check(load().mm_sno_train_step(self._h, _ptr(self._batch(m, "m")), _ptr(self._batch(target, "target")),
                                        float(lr), ctypes.byref(loss) if want_loss else None), "mm_sno_train_step")
        return loss.value if want_loss else None

    def weights(self):
        out = np.empty(SNO_NWEIGHTS, dtype=np.float32)
        _check(load().mm_sno_train_get_weights(self._h, out.ctypes.data_as(c_void_p)), "mm_sno_train_get_weights")
        return out

    def close(self):
        if getattr(self, "_h", None):
            load().mm_sno_train_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
