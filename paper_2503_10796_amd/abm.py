"""ctypes binding of libabm (the C ABI in include/abm.h).

Argument marshalling only: every step of the method runs in the HIP kernels
of ``libabm.so``.  PyTorch provides device memory (the workspace) and the
stream.  Importing this module fails loudly when the library is not built.
"""
import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libabm.so")

POS, DIAM, VOL, GROWTH, UID, STATIC, NZ, NBR_COUNT, CONTACT_COUNT, FORCE, DISP, BOX, AGE = range(13)
_FIELD_TYPES = {POS: (np.float64, 3), DIAM: (np.float64, 1), VOL: (np.float64, 1), GROWTH: (np.float64, 1),
                UID: (np.uint64, 1), STATIC: (np.uint8, 1), NZ: (np.int32, 1), NBR_COUNT: (np.int32, 1),
                CONTACT_COUNT: (np.int32, 1), FORCE: (np.float64, 3), DISP: (np.float64, 3), BOX: (np.int64, 1),
                AGE: (np.int32, 1)}
DIAG = 1
RECORD = 2

OK, ERR_ARG, ERR_CAPACITY, ERR_NONFINITE, ERR_HIP = 0, -1, -2, -3, -4


class AbmError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"libabm error {code}: {msg}")
        self.code = code


class Params(ctypes.Structure):
    _fields_ = [
        ("dt", ctypes.c_double), ("k", ctypes.c_double), ("gamma", ctypes.c_double),
        ("adherence", ctypes.c_double), ("mass", ctypes.c_double), ("max_disp", ctypes.c_double),
        ("box_len", ctypes.c_double), ("div_vol", ctypes.c_double), ("shift_frac", ctypes.c_double),
        ("detect_static", ctypes.c_int32), ("resort_every", ctypes.c_int32),
        ("seed", ctypes.c_uint64), ("sim_id", ctypes.c_uint32), ("flags", ctypes.c_uint32),
        ("brownian_rate", ctypes.c_double), ("death_prob", ctypes.c_double), ("division_prob", ctypes.c_double),
        ("min_age", ctypes.c_int32), ("reserved", ctypes.c_int32),
    ]


def params(dt=0.01, k=2.0, gamma=1.0, adherence=1.8, mass=0.1, max_disp=3.0, box_len=15.0, div_vol=0.0,
           shift_frac=0.125, detect_static=False, resort_every=0, seed=0, sim_id=0, diag=False, record=False,
           brownian_rate=0.0, death_prob=0.0, division_prob=1.0, min_age=0):
    flags = (DIAG if diag else 0) | (RECORD if record else 0)
    return Params(dt, k, gamma, adherence, mass, max_disp, box_len, div_vol, shift_frac, int(bool(detect_static)),
                  int(resort_every), int(seed), int(sim_id), flags, float(brownian_rate), float(death_prob),
                  float(division_prob), int(min_age), 0)


_lib = None
_vp = ctypes.c_void_p
_i64p = ctypes.POINTER(ctypes.c_int64)


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built: run `python -m paper_2503_10796_amd.build` "
                               "(the HIP library is the only compute path)")
        L = ctypes.CDLL(LIB_PATH)
        L.abm_last_error.restype = ctypes.c_char_p
        L.abm_batch_workspace_bytes.restype = ctypes.c_size_t
        L.abm_batch_workspace_bytes.argtypes = [ctypes.c_int, _i64p, _i64p]
        L.abm_batch_create.argtypes = [ctypes.c_int, ctypes.POINTER(Params), _i64p, _vp, _vp, _vp, _vp, _vp,
                                       ctypes.c_int, _i64p, _i64p, _vp, ctypes.c_size_t, _vp, ctypes.POINTER(_vp)]
        L.abm_batch_restore.argtypes = [_vp, _vp, _vp, _vp, _vp, ctypes.c_int64, ctypes.c_int]
        L.abm_batch_schedule.argtypes = [_vp] + [ctypes.POINTER(ctypes.c_int)] * 4
        L.abm_batch_step.argtypes = [_vp, ctypes.c_int]
        L.abm_batch_num_agents.argtypes = [_vp, _i64p]
        L.abm_batch_fp64_agents.argtypes = [_vp, _i64p]
        L.abm_batch_query.argtypes = [_vp, ctypes.c_int, ctypes.c_int, _vp, ctypes.c_int, ctypes.c_int64, _i64p]
        L.abm_batch_grid.argtypes = [_vp, ctypes.c_int, _vp, _vp, _vp]
        L.abm_batch_stats.argtypes = [_vp, ctypes.c_double, _vp, _vp, _vp, _vp]
        L.abm_batch_hist.argtypes = [_vp, ctypes.c_double, _vp, ctypes.c_int]
        L.abm_batch_tune.argtypes = [_vp, ctypes.c_int, ctypes.POINTER(ctypes.c_int)]
        L.abm_batch_set_sweep_grid.argtypes = [_vp, ctypes.c_int]
        L.abm_batch_destroy.argtypes = [_vp]
        L.abm_batch_set_timing.argtypes = [_vp, ctypes.c_int]
        L.abm_batch_sweep_time.argtypes = [_vp, ctypes.POINTER(ctypes.c_double), _i64p]
        L.abm_pop_workspace_bytes.restype = ctypes.c_size_t
        L.abm_pop_workspace_bytes.argtypes = [ctypes.POINTER(Params), ctypes.c_int64, ctypes.c_int64]
        L.abm_pop_create.argtypes = [ctypes.POINTER(Params), ctypes.c_int64, _vp, _vp, _vp, _vp, _vp, ctypes.c_int,
                                     _vp, ctypes.c_size_t, ctypes.c_int64, ctypes.c_int64, _vp, ctypes.POINTER(_vp)]
        L.abm_pop_step.argtypes = [_vp, ctypes.c_int]
        L.abm_pop_num_agents.argtypes = [_vp, _i64p]
        L.abm_pop_query.argtypes = [_vp, ctypes.c_int, _vp, ctypes.c_int, ctypes.c_int64, _i64p]
        L.abm_pop_stats.argtypes = [_vp, ctypes.c_double, _vp, _vp, _vp, _vp]
        L.abm_pop_destroy.argtypes = [_vp]
        _ip = ctypes.POINTER(ctypes.c_int)
        _fp = ctypes.POINTER(ctypes.c_float)
        L.abm_mlp_workspace_bytes.restype = ctypes.c_size_t
        L.abm_mlp_workspace_bytes.argtypes = [_ip, ctypes.c_int, ctypes.c_int]
        L.abm_mlp_create.argtypes = [_ip, ctypes.c_int, ctypes.c_int, ctypes.c_uint64, _vp, ctypes.c_size_t, _vp,
                                     ctypes.POINTER(_vp)]
        L.abm_mlp_train_step.argtypes = [_vp, _vp, _vp, ctypes.c_int, ctypes.c_float, _fp]
        L.abm_mlp_grads.argtypes = [_vp, _vp, _vp, ctypes.c_int, _vp, _fp]
        L.abm_mlp_infer.argtypes = [_vp, _vp, _vp, ctypes.c_int]
        L.abm_mlp_infer_noalloc.argtypes = [_vp, _vp, _vp, ctypes.c_int]
        L.abm_mlp_get_params.argtypes = [_vp, _vp, ctypes.c_size_t]
        L.abm_mlp_set_params.argtypes = [_vp, _vp, ctypes.c_size_t]
        L.abm_mlp_num_params.restype = ctypes.c_size_t
        L.abm_mlp_num_params.argtypes = [_vp]
        L.abm_mlp_destroy.argtypes = [_vp]
        L.abm_sir_workspace_bytes.restype = ctypes.c_size_t
        L.abm_sir_workspace_bytes.argtypes = [ctypes.POINTER(SirParams), ctypes.c_int64, ctypes.c_int]
        L.abm_sir_create.argtypes = [ctypes.POINTER(SirParams), ctypes.c_int64, _vp, _vp, ctypes.c_int, _vp,
                                     ctypes.c_size_t, _vp, _vp]
        L.abm_sir_step.argtypes = [_vp, ctypes.c_int, _vp]
        L.abm_sir_query.argtypes = [_vp, ctypes.c_int, _vp, ctypes.c_int, ctypes.c_int64]
        L.abm_sir_counts.argtypes = [_vp, _i64p, _i64p]
        L.abm_sir_grid.argtypes = [_vp, _i64p, ctypes.POINTER(ctypes.c_double)]
        L.abm_sir_set_timing.argtypes = [_vp, ctypes.c_int]
        L.abm_sir_kernel_time.argtypes = [_vp, ctypes.POINTER(ctypes.c_double), _i64p]
        L.abm_sir_destroy.argtypes = [_vp]
        L.abm_soma_workspace_bytes.restype = ctypes.c_size_t
        L.abm_soma_workspace_bytes.argtypes = [ctypes.POINTER(SomaParams), ctypes.c_int64]
        L.abm_soma_create.argtypes = [ctypes.POINTER(SomaParams), ctypes.c_int64, _vp, _vp, _vp, _vp,
                                      ctypes.c_size_t, _vp, _vp]
        L.abm_soma_step.argtypes = [_vp, ctypes.c_int]
        L.abm_soma_query.argtypes = [_vp, ctypes.c_int, _vp, ctypes.c_int, ctypes.c_int64]
        L.abm_soma_set_timing.argtypes = [_vp, ctypes.c_int]
        L.abm_soma_kernel_time.argtypes = [_vp, ctypes.POINTER(ctypes.c_double), _i64p]
        L.abm_soma_destroy.argtypes = [_vp]
        _lib = L
    return _lib


def check(rc):
    if rc != 0:
        raise AbmError(rc, lib().abm_last_error().decode())


def _torch():
    import torch
    return torch


def _stream_handle(stream):
    torch = _torch()
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _arg(a, dtype, on_device, keep):
    """Host numpy array or device tensor -> pointer (kept alive in `keep`)."""
    if a is None:
        return None
    if on_device:
        keep.append(a)
        return ctypes.c_void_p(a.data_ptr())
    arr = np.ascontiguousarray(a, dtype=dtype)
    keep.append(arr)
    return arr.ctypes.data_as(ctypes.c_void_p)


# SIR epidemiology (abm_sir_*): states, boundaries, query fields
SUSCEPTIBLE, INFECTED, RECOVERED = 0, 1, 2
TOROIDAL, CLOSED = 0, 1
SIR_POS, SIR_STATE, SIR_UID = 0, 1, 2


class SirParams(ctypes.Structure):
    _fields_ = [
        ("space", ctypes.c_double), ("radius", ctypes.c_double), ("infection_prob", ctypes.c_double),
        ("recovery_prob", ctypes.c_double), ("speed", ctypes.c_double), ("boundary", ctypes.c_int32),
        ("sim_id", ctypes.c_uint32), ("seed", ctypes.c_uint64),
    ]


def sir_params(space, radius, infection_prob, recovery_prob, speed, boundary=TOROIDAL, seed=0, sim_id=0):
    return SirParams(float(space), float(radius), float(infection_prob), float(recovery_prob), float(speed),
                     int(boundary), int(sim_id), int(seed))


class Sir:
    """One SIR population (the abm_sir_* entry points); pos: host n x 3
    float64 in [0, space], state: host uint8 (0, 1, 2)."""

    def __init__(self, p, pos, state, hist_cap=1024, stream=None):
        torch = _torch()
        L = lib()
        self._params = p
        pos = np.ascontiguousarray(pos, dtype=np.float64).reshape(-1, 3)
        state = np.ascontiguousarray(state, dtype=np.uint8)
        self.n = int(pos.shape[0])
        nbytes = L.abm_sir_workspace_bytes(ctypes.byref(p), self.n, int(hist_cap))
        if nbytes == 0:
            raise AbmError(ERR_ARG, "invalid SIR parameters or sizes")
        self.workspace = torch.empty(nbytes + 256, dtype=torch.uint8, device="cuda")
        self._stream = _stream_handle(stream)
        h = ctypes.c_void_p()
        check(L.abm_sir_create(ctypes.byref(p), self.n, pos.ctypes.data_as(ctypes.c_void_p),
                               state.ctypes.data_as(ctypes.c_void_p), int(hist_cap),
                               ctypes.c_void_p(self.workspace.data_ptr()), nbytes + 256, self._stream,
                               ctypes.byref(h)))
        self.h = h

    def step(self, n_iter=1, counts=False):
        """Advance n_iter iterations; with counts=True returns the (n_iter, 3)
        numbers of susceptible, infected and recovered persons after each."""
        out = np.zeros((max(int(n_iter), 1), 3), dtype=np.int64) if counts else None
        check(lib().abm_sir_step(self.h, int(n_iter), out.ctypes.data_as(ctypes.c_void_p) if counts else None))
        return out[: int(n_iter)] if counts else None

    def query(self, field):
        dt, width = {SIR_POS: (np.float64, 3), SIR_STATE: (np.uint8, 1), SIR_UID: (np.uint32, 1)}[field]
        out = np.zeros((max(self.n, 1), width) if width > 1 else max(self.n, 1), dtype=dt)
        check(lib().abm_sir_query(self.h, int(field), out.ctypes.data_as(ctypes.c_void_p), 0, max(self.n, 1)))
        return out[: self.n]

    def counts(self):
        it = ctypes.c_int64(0)
        c = np.zeros(3, dtype=np.int64)
        check(lib().abm_sir_counts(self.h, ctypes.byref(it), c.ctypes.data_as(_i64p)))
        return it.value, c

    def grid(self):
        dims = ctypes.c_int64(0)
        lb = ctypes.c_double(0.0)
        check(lib().abm_sir_grid(self.h, ctypes.byref(dims), ctypes.byref(lb)))
        return dims.value, lb.value

    def set_timing(self, on):
        check(lib().abm_sir_set_timing(self.h, int(bool(on))))

    def kernel_time(self):
        ms = ctypes.c_double(0.0)
        k = ctypes.c_int64(0)
        check(lib().abm_sir_kernel_time(self.h, ctypes.byref(ms), ctypes.byref(k)))
        return ms.value, k.value

    def __del__(self):
        h = getattr(self, "h", None)
        if h is not None and _lib is not None:
            _lib.abm_sir_destroy(h)
            self.h = None

    def close(self):
        self.__del__()


# Diffusion with secreting, chemotactic cells (abm_soma_*): query fields
SOMA_POS, SOMA_TYPE, SOMA_CONC = 0, 1, 2


class SomaParams(ctypes.Structure):
    _fields_ = [
        ("lo", ctypes.c_double), ("space", ctypes.c_double), ("resolution", ctypes.c_int32),
        ("n_substances", ctypes.c_int32), ("diffusion", ctypes.c_double), ("decay", ctypes.c_double),
        ("dt", ctypes.c_double), ("secretion", ctypes.c_double), ("gradient_weight", ctypes.c_double),
    ]


def soma_params(lo=0.0, space=100.0, resolution=20, n_substances=2, diffusion=1.0, decay=0.01, dt=1.0,
                secretion=1.0, gradient_weight=0.75):
    return SomaParams(float(lo), float(space), int(resolution), int(n_substances), float(diffusion), float(decay),
                      float(dt), float(secretion), float(gradient_weight))


class Soma:
    """Concentration grids and chemotactic cells (the abm_soma_* entry
    points); pos: host n x 3 float64 inside the space, cell_type: host int32,
    conc: host n_substances x R x R x R float64 ([s, z, y, x]) or None."""

    def __init__(self, p, pos, cell_type, conc=None, stream=None):
        torch = _torch()
        L = lib()
        self._params = p
        pos = np.ascontiguousarray(pos, dtype=np.float64).reshape(-1, 3)
        cell_type = np.ascontiguousarray(cell_type, dtype=np.int32)
        self.n = int(pos.shape[0])
        self.R, self.nsub = int(p.resolution), int(p.n_substances)
        nbytes = L.abm_soma_workspace_bytes(ctypes.byref(p), self.n)
        if nbytes == 0:
            raise AbmError(ERR_ARG, "invalid diffusion parameters or sizes")
        self.workspace = torch.empty(nbytes + 256, dtype=torch.uint8, device="cuda")
        self._stream = _stream_handle(stream)
        c = None if conc is None else np.ascontiguousarray(conc, dtype=np.float64)
        h = ctypes.c_void_p()
        check(L.abm_soma_create(ctypes.byref(p), self.n, pos.ctypes.data_as(ctypes.c_void_p),
                                cell_type.ctypes.data_as(ctypes.c_void_p),
                                None if c is None else c.ctypes.data_as(ctypes.c_void_p),
                                ctypes.c_void_p(self.workspace.data_ptr()), nbytes + 256, self._stream,
                                ctypes.byref(h)))
        self.h = h

    def step(self, n_iter=1):
        check(lib().abm_soma_step(self.h, int(n_iter)))

    def query(self, field):
        if field == SOMA_CONC:
            out = np.zeros((self.nsub, self.R, self.R, self.R), dtype=np.float64)
            cap = out.size
        elif field == SOMA_POS:
            out = np.zeros((max(self.n, 1), 3), dtype=np.float64)
            cap = max(self.n, 1)
        else:
            out = np.zeros(max(self.n, 1), dtype=np.int32)
            cap = max(self.n, 1)
        check(lib().abm_soma_query(self.h, int(field), out.ctypes.data_as(ctypes.c_void_p), 0, cap))
        return out if field == SOMA_CONC else out[: self.n]

    def set_timing(self, on):
        check(lib().abm_soma_set_timing(self.h, int(bool(on))))

    def kernel_time(self):
        ms = ctypes.c_double(0.0)
        k = ctypes.c_int64(0)
        check(lib().abm_soma_kernel_time(self.h, ctypes.byref(ms), ctypes.byref(k)))
        return ms.value, k.value

    def __del__(self):
        h = getattr(self, "h", None)
        if h is not None and _lib is not None:
            _lib.abm_soma_destroy(h)
            self.h = None

    def close(self):
        self.__del__()


class Batch:
    """Independent simulations advanced together (one graph launch per iteration).

    pos, diam, vol, growth, uid: concatenated over simulations (simulation-major),
    numpy arrays (host) or CUDA tensors (device, float64/uint64)."""

    def __init__(self, plist, n0, pos, diam, vol=None, growth=None, uid=None, capacity=None,
                 box_capacity=None, stream=None):
        torch = _torch()
        L = lib()
        self.n_sims = len(plist)
        n0 = np.asarray(n0, dtype=np.int64)
        cap = np.asarray(capacity if capacity is not None else n0, dtype=np.int64).reshape(-1)
        if cap.size == 1 and self.n_sims > 1:
            cap = np.full(self.n_sims, cap[0], dtype=np.int64)
        bcap = (np.asarray(box_capacity, dtype=np.int64).reshape(-1) if box_capacity is not None
                else 2 * cap + 65536)
        if bcap.size == 1 and self.n_sims > 1:
            bcap = np.full(self.n_sims, bcap[0], dtype=np.int64)
        self._n0, self._cap, self._bcap = n0, cap, bcap
        self._params = (Params * self.n_sims)(*plist)
        nbytes = L.abm_batch_workspace_bytes(self.n_sims, cap.ctypes.data_as(_i64p), bcap.ctypes.data_as(_i64p))
        if nbytes == 0:
            raise AbmError(ERR_ARG, "invalid capacities")
        self.workspace = torch.empty(nbytes + 256, dtype=torch.uint8, device="cuda")
        on_dev = hasattr(pos, "data_ptr")
        keep = []
        h = ctypes.c_void_p()
        self._stream = _stream_handle(stream)
        rc = L.abm_batch_create(self.n_sims, self._params, n0.ctypes.data_as(_i64p),
                                _arg(pos, np.float64, on_dev, keep), _arg(diam, np.float64, on_dev, keep),
                                _arg(vol, np.float64, on_dev, keep), _arg(growth, np.float64, on_dev, keep),
                                _arg(uid, np.uint64, on_dev, keep), int(on_dev), cap.ctypes.data_as(_i64p),
                                bcap.ctypes.data_as(_i64p), ctypes.c_void_p(self.workspace.data_ptr()),
                                nbytes + 256, self._stream, ctypes.byref(h))
        check(rc)
        self.h = h

    def __del__(self):
        h = getattr(self, "h", None)
        if h is not None and _lib is not None:
            _lib.abm_batch_destroy(h)
            self.h = None

    def close(self):
        self.__del__()

    def step(self, n_iter=1):
        check(lib().abm_batch_step(self.h, int(n_iter)))

    def num_agents(self):
        out = np.zeros(self.n_sims, dtype=np.int64)
        check(lib().abm_batch_num_agents(self.h, out.ctypes.data_as(_i64p)))
        return out

    def fp64_agents(self):
        """Agents decided on the FP64 path in the last iteration (whole batch)."""
        out = np.zeros(1, dtype=np.int64)
        check(lib().abm_batch_fp64_agents(self.h, out.ctypes.data_as(_i64p)))
        return int(out[0])

    def query(self, field, sim=0):
        dt, width = _FIELD_TYPES[field]
        n = int(self.num_agents()[sim])
        out = np.zeros((max(n, 1), width) if width > 1 else max(n, 1), dtype=dt)
        got = ctypes.c_int64(0)
        check(lib().abm_batch_query(self.h, int(sim), int(field), out.ctypes.data_as(ctypes.c_void_p), 0,
                                    max(n, 1), ctypes.byref(got)))
        return out[: got.value]

    def query_device(self, field, dst, sim=0):
        got = ctypes.c_int64(0)
        dt, width = _FIELD_TYPES[field]
        check(lib().abm_batch_query(self.h, int(sim), int(field), ctypes.c_void_p(dst.data_ptr()), 1,
                                    dst.numel() // width, ctypes.byref(got)))
        return got.value

    def grid(self, sim=0):
        lo = np.zeros(3)
        L = ctypes.c_double(0)
        dims = np.zeros(3, dtype=np.int64)
        check(lib().abm_batch_grid(self.h, int(sim), lo.ctypes.data_as(ctypes.c_void_p), ctypes.byref(L),
                                   dims.ctypes.data_as(ctypes.c_void_p)))
        return lo, L.value, dims

    def stats(self, hist_rmax=400.0):
        c = np.zeros((self.n_sims, 3)); rg = np.zeros(self.n_sims); rm = np.zeros(self.n_sims)
        h = np.zeros((self.n_sims, 32), dtype=np.float32)
        check(lib().abm_batch_stats(self.h, float(hist_rmax), c.ctypes.data_as(ctypes.c_void_p),
                                    rg.ctypes.data_as(ctypes.c_void_p), rm.ctypes.data_as(ctypes.c_void_p),
                                    h.ctypes.data_as(ctypes.c_void_p)))
        return c, rg, rm, h

    def hist_device(self, out, hist_rmax=400.0):
        check(lib().abm_batch_hist(self.h, float(hist_rmax), ctypes.c_void_p(out.data_ptr()), 1))

    def restore(self, is_static=None, nz=None, next_uid=None, iteration=0, age=None):
        keep = []
        check(lib().abm_batch_restore(self.h, _arg(is_static, np.uint8, False, keep), _arg(nz, np.int32, False, keep),
                                      _arg(age, np.int32, False, keep), _arg(next_uid, np.uint64, False, keep),
                                      int(iteration), 0))

    def tune(self, n_trial_iters=3):
        b = ctypes.c_int(0)
        check(lib().abm_batch_tune(self.h, int(n_trial_iters), ctypes.byref(b)))
        return b.value

    def schedule(self):
        """The launch schedule in use: dict of sweep_grid, dense_grid,
        dense_waves, resort_every."""
        v = [ctypes.c_int(0) for _ in range(4)]
        check(lib().abm_batch_schedule(self.h, *[ctypes.byref(x) for x in v]))
        return dict(zip(("sweep_grid", "dense_grid", "dense_waves", "resort_every"), (x.value for x in v)))

    def set_sweep_grid(self, workgroups):
        check(lib().abm_batch_set_sweep_grid(self.h, int(workgroups)))

    def set_timing(self, on=True):
        check(lib().abm_batch_set_timing(self.h, int(bool(on))))

    def sweep_time(self):
        """(summed sweep milliseconds, number of sweeps) since the last call."""
        ms = ctypes.c_double(0.0)
        n = ctypes.c_int64(0)
        check(lib().abm_batch_sweep_time(self.h, ctypes.byref(ms), ctypes.byref(n)))
        return ms.value, n.value


class Population(Batch):
    """One simulation (the abm_pop_* entry points)."""

    def __init__(self, p, pos, diam, vol=None, growth=None, uid=None, capacity=None, box_capacity=None,
                 stream=None):
        torch = _torch()
        L = lib()
        self.n_sims = 1
        n = int(pos.shape[0])
        cap = int(capacity if capacity is not None else n)
        bcap = int(box_capacity if box_capacity is not None else 2 * cap + 65536)
        self._params = (Params * 1)(p)
        nbytes = L.abm_pop_workspace_bytes(self._params, cap, bcap)
        if nbytes == 0:
            raise AbmError(ERR_ARG, "invalid capacities")
        self.workspace = torch.empty(nbytes + 256, dtype=torch.uint8, device="cuda")
        on_dev = hasattr(pos, "data_ptr")
        keep = []
        h = ctypes.c_void_p()
        self._stream = _stream_handle(stream)
        check(L.abm_pop_create(self._params, n, _arg(pos, np.float64, on_dev, keep), _arg(diam, np.float64, on_dev, keep),
                               _arg(vol, np.float64, on_dev, keep), _arg(growth, np.float64, on_dev, keep),
                               _arg(uid, np.uint64, on_dev, keep), int(on_dev),
                               ctypes.c_void_p(self.workspace.data_ptr()), nbytes + 256, cap, bcap, self._stream,
                               ctypes.byref(h)))
        self.h = h

    def step(self, n_iter=1):
        check(lib().abm_pop_step(self.h, int(n_iter)))

    def query(self, field, sim=0):
        dt, width = _FIELD_TYPES[field]
        n = int(self.num_agents()[0])
        out = np.zeros((max(n, 1), width) if width > 1 else max(n, 1), dtype=dt)
        got = ctypes.c_int64(0)
        check(lib().abm_pop_query(self.h, int(field), out.ctypes.data_as(ctypes.c_void_p), 0, max(n, 1),
                                  ctypes.byref(got)))
        return out[: got.value]


class Mlp:
    """Surrogate MLP on the GPU (BF16 matrix-core GEMMs, FP32 master weights).

    Inputs and outputs are CUDA float32 tensors; parameters use the layout of
    the C ABI (per layer W [out, in] row-major, then b)."""

    def __init__(self, dims=(35, 256, 256, 256, 32), max_batch=4096, seed=0, stream=None):
        torch = _torch()
        L = lib()
        self.dims = tuple(int(d) for d in dims)
        self.max_batch = int(max_batch)
        d = (ctypes.c_int * len(self.dims))(*self.dims)
        nbytes = L.abm_mlp_workspace_bytes(d, len(self.dims), self.max_batch)
        if nbytes == 0:
            raise AbmError(ERR_ARG, "invalid MLP dims or batch")
        self.workspace = torch.empty(nbytes + 256, dtype=torch.uint8, device="cuda")
        self._stream = _stream_handle(stream)
        h = ctypes.c_void_p()
        check(L.abm_mlp_create(d, len(self.dims), self.max_batch, int(seed), ctypes.c_void_p(self.workspace.data_ptr()),
                               nbytes + 256, self._stream, ctypes.byref(h)))
        self.h = h
        self.n_params = int(L.abm_mlp_num_params(h))

    def __del__(self):
        h = getattr(self, "h", None)
        if h is not None and _lib is not None:
            _lib.abm_mlp_destroy(h)
            self.h = None

    @staticmethod
    def _dev(t):
        torch = _torch()
        t = t if hasattr(t, "data_ptr") else torch.as_tensor(np.asarray(t, dtype=np.float32))
        return t.to(device="cuda", dtype=torch.float32).contiguous()

    def train_step(self, x, y, lr=1e-3, want_loss=True):
        x, y = self._dev(x), self._dev(y)
        loss = ctypes.c_float()
        check(lib().abm_mlp_train_step(self.h, ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(y.data_ptr()),
                                       x.shape[0], float(lr), ctypes.byref(loss) if want_loss else None))
        return float(loss.value) if want_loss else None

    def grads(self, x, y):
        torch = _torch()
        x, y = self._dev(x), self._dev(y)
        g = torch.empty(self.n_params, dtype=torch.float32, device="cuda")
        loss = ctypes.c_float()
        check(lib().abm_mlp_grads(self.h, ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(y.data_ptr()), x.shape[0],
                                  ctypes.c_void_p(g.data_ptr()), ctypes.byref(loss)))
        return float(loss.value), g

    def infer(self, x, out=None):
        torch = _torch()
        x = self._dev(x)
        y = out if out is not None else torch.empty((x.shape[0], self.dims[-1]), dtype=torch.float32, device="cuda")
        check(lib().abm_mlp_infer(self.h, ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(y.data_ptr()), x.shape[0]))
        return y

    def infer_noalloc(self, x, out):
        """The forward pass through abm_mlp_infer_noalloc: x and out are
        device FP32 tensors the caller allocated (batch x dims[0], batch x
        dims[-1]); the library allocates nothing."""
        check(lib().abm_mlp_infer_noalloc(self.h, ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(out.data_ptr()),
                                          x.shape[0]))
        return out

    def get_params(self):
        torch = _torch()
        p = torch.empty(self.n_params, dtype=torch.float32, device="cuda")
        check(lib().abm_mlp_get_params(self.h, ctypes.c_void_p(p.data_ptr()), self.n_params))
        return p

    def set_params(self, theta):
        p = self._dev(theta)
        check(lib().abm_mlp_set_params(self.h, ctypes.c_void_p(p.data_ptr()), p.numel()))
        _torch().cuda.current_stream().synchronize()
