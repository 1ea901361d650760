"""ctypes front end of the SIR epidemiology oracle (``sir_oracle.c`` in
``liboracle.so``): infection (Algorithm 3), recovery (Algorithm 4) and random
movement with a toroidal or closed boundary (Algorithm 5, Sec 4.4.11).

Test infrastructure only: the test suite, the smoke check and the CPU
baseline leg of the benchmark use it, never the product path.
"""
import ctypes

import numpy as np

from oracle import sim as _sim

SUSCEPTIBLE, INFECTED, RECOVERED = 0, 1, 2
TOROIDAL, CLOSED = 0, 1
TAG_INFECTION, TAG_RECOVERY, TAG_MOVE = 0x494E4645, 0x5245434F, 0x4D4F5645

_dp = ctypes.POINTER(ctypes.c_double)
_u8p = ctypes.POINTER(ctypes.c_uint8)
_i64p = ctypes.POINTER(ctypes.c_int64)
_u64p = ctypes.POINTER(ctypes.c_uint64)


class SirParams(ctypes.Structure):
    _fields_ = [
        ("space", ctypes.c_double), ("radius", ctypes.c_double), ("infection_prob", ctypes.c_double),
        ("recovery_prob", ctypes.c_double), ("speed", ctypes.c_double), ("boundary", ctypes.c_int32),
        ("sim_id", ctypes.c_uint32), ("seed", ctypes.c_uint64),
    ]


_ready = False


def lib():
    global _ready
    L = _sim.lib()
    if not _ready:
        L.orc_sir_step.argtypes = [ctypes.c_int64, _dp, _dp, _dp, _u8p, _u64p, ctypes.c_int64,
                                   ctypes.POINTER(SirParams), _i64p]
        L.orc_sir_step.restype = ctypes.c_int
        L.orc_sir_step_vector.argtypes = [ctypes.c_uint64, ctypes.c_uint32, ctypes.c_uint64, ctypes.c_uint64,
                                          ctypes.c_double, _dp]
        L.orc_sir_step_vector.restype = None
        L.orc_sir_bound.argtypes = [ctypes.c_double, ctypes.c_double, ctypes.c_int]
        L.orc_sir_bound.restype = ctypes.c_double
        L.orc_sir_dist2.argtypes = [ctypes.c_double] * 7 + [ctypes.c_int]
        L.orc_sir_dist2.restype = ctypes.c_double
        L.orc_sir_tries_infection.argtypes = [ctypes.POINTER(SirParams), ctypes.c_uint64, ctypes.c_uint64]
        L.orc_sir_tries_infection.restype = ctypes.c_int
        L.orc_sir_recovers.argtypes = [ctypes.POINTER(SirParams), ctypes.c_uint64, ctypes.c_uint64]
        L.orc_sir_recovers.restype = ctypes.c_int
        _ready = True
    return L


def make_params(space, radius, infection_prob, recovery_prob, speed, boundary=TOROIDAL, seed=0, sim_id=0):
    return SirParams(float(space), float(radius), float(infection_prob), float(recovery_prob), float(speed),
                     int(boundary), int(sim_id), int(seed))


class OracleSIR:
    """One SIR population (persons at FP64 positions with a state each)."""

    def __init__(self, pos, state, params, uid=None, iteration=0):
        pos = np.asarray(pos, dtype=np.float64)
        self.n = pos.shape[0]
        self.x = np.ascontiguousarray(pos[:, 0]) if self.n else np.zeros(0)
        self.y = np.ascontiguousarray(pos[:, 1]) if self.n else np.zeros(0)
        self.z = np.ascontiguousarray(pos[:, 2]) if self.n else np.zeros(0)
        self.state = np.ascontiguousarray(state, dtype=np.uint8).copy()
        self.uid = (np.arange(self.n, dtype=np.uint64) if uid is None
                    else np.ascontiguousarray(uid, dtype=np.uint64).copy())
        self.params = params
        self.iteration = int(iteration)

    def step(self, n_iter=1):
        """Advance n_iter iterations; returns the (n_iter, 3) counts of
        susceptible, infected and recovered persons after each."""
        L = lib()
        out = np.zeros((n_iter, 3), dtype=np.int64)
        c = np.zeros(3, dtype=np.int64)
        for k in range(n_iter):
            rc = L.orc_sir_step(self.n, _sim._ptr(self.x, ctypes.c_double), _sim._ptr(self.y, ctypes.c_double),
                                _sim._ptr(self.z, ctypes.c_double), _sim._ptr(self.state, ctypes.c_uint8),
                                _sim._ptr(self.uid, ctypes.c_uint64), self.iteration, ctypes.byref(self.params),
                                _sim._ptr(c, ctypes.c_int64))
            if rc != 0:
                raise MemoryError("orc_sir_step")
            out[k] = c
            self.iteration += 1
        return out

    def pos(self):
        return np.stack([self.x, self.y, self.z], axis=1)

    def counts(self):
        return np.bincount(self.state, minlength=3)[:3].astype(np.int64)


def step_vector(seed, sim_id, uid, iteration, speed):
    d = np.zeros(3)
    lib().orc_sir_step_vector(seed, sim_id, uid, iteration, speed, _sim._ptr(d, ctypes.c_double))
    return d


def bound(v, space, boundary):
    return lib().orc_sir_bound(float(v), float(space), int(boundary))


def dist2(a, b, space, boundary):
    return lib().orc_sir_dist2(*[float(t) for t in a], *[float(t) for t in b], float(space), int(boundary))


def tries_infection(params, uid, iteration):
    return bool(lib().orc_sir_tries_infection(ctypes.byref(params), uid, iteration))


def recovers(params, uid, iteration):
    return bool(lib().orc_sir_recovers(ctypes.byref(params), uid, iteration))
