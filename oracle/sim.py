"""ctypes front end of the C oracle (``liboracle.so``).

Test infrastructure only (see the package docstring).  ``OracleSim`` owns
numpy arrays for one population and advances it with ``orc_step``; the
module-level helpers expose the oracle's definitions (pair force, Morton
code, Philox4x32-10, division direction, diameter from volume, statistics).
"""
import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None

_dp = ctypes.POINTER(ctypes.c_double)
_u8p = ctypes.POINTER(ctypes.c_uint8)
_i32p = ctypes.POINTER(ctypes.c_int32)
_i64p = ctypes.POINTER(ctypes.c_int64)
_u64p = ctypes.POINTER(ctypes.c_uint64)


class OrcParams(ctypes.Structure):
    _fields_ = [
        ("dt", ctypes.c_double), ("k", ctypes.c_double), ("gamma", ctypes.c_double),
        ("adherence", ctypes.c_double), ("mass", ctypes.c_double), ("max_disp", ctypes.c_double),
        ("box_len", ctypes.c_double), ("div_vol", ctypes.c_double), ("shift_frac", ctypes.c_double),
        ("detect_static", ctypes.c_int32), ("brute_force", ctypes.c_int32),
        ("seed", ctypes.c_uint64), ("sim_id", ctypes.c_uint32), ("pad", ctypes.c_uint32),
        ("brownian_rate", ctypes.c_double), ("death_prob", ctypes.c_double), ("division_prob", ctypes.c_double),
        ("min_age", ctypes.c_int32), ("pad2", ctypes.c_int32),
    ]


class OrcState(ctypes.Structure):
    _fields_ = [
        ("n", ctypes.c_int64), ("cap", ctypes.c_int64), ("next_uid", ctypes.c_int64), ("iter", ctypes.c_int64),
        ("x", _dp), ("y", _dp), ("z", _dp), ("diam", _dp), ("vol", _dp), ("growth", _dp),
        ("uid", _u64p), ("is_static", _u8p), ("nz", _i32p),
        ("nbr", _i32p), ("contacts", _i32p),
        ("fx", _dp), ("fy", _dp), ("fz", _dp), ("dx", _dp), ("dy", _dp), ("dz", _dp),
        ("box", _i64p), ("sum_abs_fn", _dp), ("sum_dfn", _dp), ("sum_fn_d", _dp),
        ("moved", _u8p), ("grew", _u8p), ("divided", _u8p), ("is_new", _u8p),
        ("grid_lo", ctypes.c_double * 3), ("grid_hi", ctypes.c_double * 3), ("grid_L", ctypes.c_double),
        ("grid_dims", ctypes.c_int64 * 3),
        ("age", _i32p), ("n_removed", ctypes.c_int64),
    ]


def lib():
    """Load the oracle library, building it first if it is missing."""
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            from oracle import build as _build
            _build.build()
        L = ctypes.CDLL(_LIB_PATH)
        L.orc_step.argtypes = [ctypes.POINTER(OrcState), ctypes.POINTER(OrcParams)]
        L.orc_step.restype = ctypes.c_int
        L.orc_forces_subset.argtypes = [ctypes.POINTER(OrcState), ctypes.POINTER(OrcParams), ctypes.c_int64,
                                        _i64p, _dp, _i32p, _dp, _dp]
        L.orc_forces_subset.restype = ctypes.c_int
        L.orc_neighbour_uids.argtypes = [ctypes.POINTER(OrcState), ctypes.POINTER(OrcParams), ctypes.c_int64,
                                         ctypes.c_int, _u64p, ctypes.c_int64]
        L.orc_neighbour_uids.restype = ctypes.c_int64
        L.orc_grid_info.argtypes = [ctypes.POINTER(OrcState), ctypes.POINTER(OrcParams), _dp, _dp, _i64p, _i64p]
        L.orc_grid_info.restype = ctypes.c_int
        L.orc_morton3.argtypes = [ctypes.c_uint32] * 3
        L.orc_morton3.restype = ctypes.c_uint64
        L.orc_morton2.argtypes = [ctypes.c_uint32] * 2
        L.orc_morton2.restype = ctypes.c_uint64
        L.orc_philox4x32_10.argtypes = [ctypes.POINTER(ctypes.c_uint32)] * 3
        L.orc_philox4x32_10.restype = None
        L.orc_direction.argtypes = [ctypes.c_uint64, ctypes.c_uint32, ctypes.c_uint64, ctypes.c_uint64, _dp]
        L.orc_direction.restype = None
        L.orc_diameter_from_volume.argtypes = [ctypes.c_double]
        L.orc_diameter_from_volume.restype = ctypes.c_double
        L.orc_pair_force.argtypes = [ctypes.c_double] * 5
        L.orc_pair_force.restype = ctypes.c_double
        L.orc_displacement.argtypes = [_dp, ctypes.c_double, ctypes.c_double, ctypes.c_double, ctypes.c_double, _dp]
        L.orc_displacement.restype = None
        L.orc_stats.argtypes = [ctypes.c_int64, _dp, _dp, _dp, ctypes.c_double, _dp, _dp, _dp,
                                ctypes.POINTER(ctypes.c_float), _i64p]
        L.orc_stats.restype = None
        L.orc_draw.argtypes = [ctypes.c_uint64, ctypes.c_uint32, ctypes.c_uint32, ctypes.c_uint64, ctypes.c_uint64,
                               ctypes.POINTER(ctypes.c_uint32)]
        L.orc_draw.restype = None
        L.orc_brownian.argtypes = [ctypes.c_uint64, ctypes.c_uint32, ctypes.c_uint64, ctypes.c_uint64, ctypes.c_double,
                                   _dp]
        L.orc_brownian.restype = None
        L.orc_dies.argtypes = [ctypes.POINTER(OrcParams), ctypes.c_uint64, ctypes.c_uint64, ctypes.c_int32]
        L.orc_dies.restype = ctypes.c_int
        L.orc_divides.argtypes = [ctypes.POINTER(OrcParams), ctypes.c_uint64, ctypes.c_uint64]
        L.orc_divides.restype = ctypes.c_int
        _lib = L
    return _lib


def _ptr(a, ctype):
    return a.ctypes.data_as(ctypes.POINTER(ctype))


def make_params(dt=0.01, k=2.0, gamma=1.0, adherence=1.8, mass=0.1, max_disp=3.0, box_len=15.0,
                div_vol=0.0, shift_frac=0.125, detect_static=False, brute_force=False, seed=0, sim_id=0,
                brownian_rate=0.0, death_prob=0.0, division_prob=1.0, min_age=0):
    return OrcParams(dt, k, gamma, adherence, mass, max_disp, box_len, div_vol, shift_frac,
                     int(bool(detect_static)), int(bool(brute_force)), int(seed), int(sim_id), 0,
                     float(brownian_rate), float(death_prob), float(division_prob), int(min_age), 0)


class OracleSim:
    """One population advanced by the oracle; arrays are numpy, sized ``cap``."""

    def __init__(self, pos, diam, params, vol=None, growth=None, uid=None, cap=None, next_uid=None,
                 is_static=None, nz=None, iteration=0, age=None):
        pos = np.asarray(pos, dtype=np.float64)
        n = pos.shape[0]
        cap = n if cap is None else int(cap)
        self.cap = cap
        self.params = params
        z = lambda dt: np.zeros(cap, dtype=dt)
        self.x, self.y, self.z = z(np.float64), z(np.float64), z(np.float64)
        self.diam, self.vol, self.growth = z(np.float64), z(np.float64), z(np.float64)
        self.uid = z(np.uint64)
        self.is_static = z(np.uint8)
        self.nz = z(np.int32)
        self.nbr, self.contacts = z(np.int32), z(np.int32)
        self.fx, self.fy, self.fz = z(np.float64), z(np.float64), z(np.float64)
        self.dx, self.dy, self.dz = z(np.float64), z(np.float64), z(np.float64)
        self.box = z(np.int64)
        self.sum_abs_fn, self.sum_dfn, self.sum_fn_d = z(np.float64), z(np.float64), z(np.float64)
        self.moved, self.grew, self.divided, self.is_new = z(np.uint8), z(np.uint8), z(np.uint8), z(np.uint8)
        self.age = z(np.int32)
        if age is not None:
            self.age[:n] = np.asarray(age, dtype=np.int32)
        self.x[:n], self.y[:n], self.z[:n] = pos[:, 0], pos[:, 1], pos[:, 2]
        self.diam[:n] = np.asarray(diam, dtype=np.float64)
        if vol is None:
            vol = np.pi * self.diam[:n] ** 3 / 6.0
        self.vol[:n] = vol
        if growth is not None:
            self.growth[:n] = growth
        self.uid[:n] = np.arange(n, dtype=np.uint64) if uid is None else np.asarray(uid, dtype=np.uint64)
        if is_static is not None:
            self.is_static[:n] = is_static
        if nz is not None:
            self.nz[:n] = nz
        self.state = OrcState()
        s = self.state
        s.n, s.cap = n, cap
        s.next_uid = int(self.uid[:n].max()) + 1 if (next_uid is None and n > 0) else int(next_uid or 0)
        s.iter = int(iteration)
        for name, ct in (("x", ctypes.c_double), ("y", ctypes.c_double), ("z", ctypes.c_double),
                         ("diam", ctypes.c_double), ("vol", ctypes.c_double), ("growth", ctypes.c_double),
                         ("uid", ctypes.c_uint64), ("is_static", ctypes.c_uint8), ("nz", ctypes.c_int32),
                         ("nbr", ctypes.c_int32), ("contacts", ctypes.c_int32),
                         ("fx", ctypes.c_double), ("fy", ctypes.c_double), ("fz", ctypes.c_double),
                         ("dx", ctypes.c_double), ("dy", ctypes.c_double), ("dz", ctypes.c_double),
                         ("box", ctypes.c_int64), ("sum_abs_fn", ctypes.c_double), ("sum_dfn", ctypes.c_double),
                         ("sum_fn_d", ctypes.c_double), ("moved", ctypes.c_uint8), ("grew", ctypes.c_uint8), ("divided", ctypes.c_uint8),
                         ("is_new", ctypes.c_uint8), ("age", ctypes.c_int32)):
            setattr(s, name, _ptr(getattr(self, name), ct))

    @property
    def n(self):
        return int(self.state.n)

    @property
    def iteration(self):
        return int(self.state.iter)

    @property
    def n_removed(self):
        return int(self.state.n_removed)

    def step(self, n_iter=1):
        for _ in range(n_iter):
            rc = lib().orc_step(ctypes.byref(self.state), ctypes.byref(self.params))
            if rc != 0:
                raise RuntimeError(f"orc_step failed with {rc}")

    def pos(self):
        n = self.n
        return np.stack([self.x[:n], self.y[:n], self.z[:n]], axis=1)

    def force(self):
        n = self.n
        return np.stack([self.fx[:n], self.fy[:n], self.fz[:n]], axis=1)

    def disp(self):
        n = self.n
        return np.stack([self.dx[:n], self.dy[:n], self.dz[:n]], axis=1)

    def grid(self):
        lo = np.zeros(3)
        L = ctypes.c_double(0)
        dims = np.zeros(3, dtype=np.int64)
        box = np.zeros(max(self.n, 1), dtype=np.int64)
        lib().orc_grid_info(ctypes.byref(self.state), ctypes.byref(self.params), _ptr(lo, ctypes.c_double),
                            ctypes.byref(L), _ptr(dims, ctypes.c_int64), _ptr(box, ctypes.c_int64))
        return lo, L.value, dims, box[: self.n]

    def neighbour_uids(self, i, brute=False):
        out = np.zeros(4096, dtype=np.uint64)
        cnt = lib().orc_neighbour_uids(ctypes.byref(self.state), ctypes.byref(self.params), int(i), int(brute),
                                       _ptr(out, ctypes.c_uint64), out.size)
        if cnt < 0:
            raise RuntimeError("orc_neighbour_uids failed")
        return out[:cnt].copy()

    def forces_subset(self, sel):
        sel = np.ascontiguousarray(sel, dtype=np.int64)
        m = sel.size
        f = np.zeros((m, 3)); d = np.zeros((m, 3)); tol = np.zeros((m, 3))
        cnt = np.zeros((m, 3), dtype=np.int32)
        rc = lib().orc_forces_subset(ctypes.byref(self.state), ctypes.byref(self.params), m,
                                     _ptr(sel, ctypes.c_int64), _ptr(f, ctypes.c_double), _ptr(cnt, ctypes.c_int32),
                                     _ptr(d, ctypes.c_double), _ptr(tol, ctypes.c_double))
        if rc != 0:
            raise RuntimeError("orc_forces_subset failed")
        return f, cnt, d, tol


def pair_force(r1, r2, delta, k=2.0, gamma=1.0):
    return lib().orc_pair_force(r1, r2, delta, k, gamma)


def displacement(f, adherence=1.8, dt=0.01, mass=0.1, max_disp=3.0):
    f = np.ascontiguousarray(f, dtype=np.float64)
    d = np.zeros(3)
    lib().orc_displacement(_ptr(f, ctypes.c_double), adherence, dt, mass, max_disp, _ptr(d, ctypes.c_double))
    return d


def morton3(bx, by, bz):
    return int(lib().orc_morton3(bx, by, bz))


def morton2(bx, by):
    return int(lib().orc_morton2(bx, by))


def philox4x32_10(ctr, key):
    c = (ctypes.c_uint32 * 4)(*ctr)
    k = (ctypes.c_uint32 * 2)(*key)
    o = (ctypes.c_uint32 * 4)()
    lib().orc_philox4x32_10(c, k, o)
    return [int(v) for v in o]


def direction(seed, sim_id, uid, iteration):
    u = np.zeros(3)
    lib().orc_direction(seed, sim_id, uid, iteration, _ptr(u, ctypes.c_double))
    return u


def draw(seed, tag, sim_id, uid, iteration):
    o = (ctypes.c_uint32 * 4)()
    lib().orc_draw(seed, tag, sim_id, uid, iteration, o)
    return [int(v) for v in o]


def brownian(seed, sim_id, uid, iteration, rate):
    d = np.zeros(3)
    lib().orc_brownian(seed, sim_id, uid, iteration, rate, _ptr(d, ctypes.c_double))
    return d


def dies(params, uid, iteration, age):
    return bool(lib().orc_dies(ctypes.byref(params), uid, iteration, age))


def divides(params, uid, iteration):
    return bool(lib().orc_divides(ctypes.byref(params), uid, iteration))


TAG_BROWNIAN, TAG_DEATH, TAG_DIVISION = 0x42524F57, 0x44454154, 0x44495650


def diameter_from_volume(v):
    return lib().orc_diameter_from_volume(v)


def stats(pos, hist_rmax=400.0):
    pos = np.ascontiguousarray(pos, dtype=np.float64)
    x = np.ascontiguousarray(pos[:, 0]); y = np.ascontiguousarray(pos[:, 1]); z = np.ascontiguousarray(pos[:, 2])
    c = np.zeros(3); rg = ctypes.c_double(0); rm = ctypes.c_double(0)
    h = np.zeros(32, dtype=np.float32); cnt = np.zeros(32, dtype=np.int64)
    lib().orc_stats(pos.shape[0], _ptr(x, ctypes.c_double), _ptr(y, ctypes.c_double), _ptr(z, ctypes.c_double),
                    hist_rmax, _ptr(c, ctypes.c_double), ctypes.byref(rg), ctypes.byref(rm),
                    _ptr(h, ctypes.c_float), _ptr(cnt, ctypes.c_int64))
    return c, rg.value, rm.value, h, cnt
