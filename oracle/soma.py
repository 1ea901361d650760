"""ctypes front end of the diffusion and soma clustering oracle
(``soma_oracle.c`` in ``liboracle.so``): Eq 4.3, secretion (Algorithm 6)
and chemotaxis (Algorithm 7).

Test infrastructure only: the test suite, the smoke check and the CPU
baseline leg of the benchmark use it, never the product path.
"""
import ctypes

import numpy as np

from oracle import sim as _sim

_dp = ctypes.POINTER(ctypes.c_double)
_i32p = ctypes.POINTER(ctypes.c_int32)


class SomaParams(ctypes.Structure):
    _fields_ = [
        ("lo", ctypes.c_double), ("space", ctypes.c_double), ("resolution", ctypes.c_int32),
        ("n_substances", ctypes.c_int32), ("diffusion", ctypes.c_double), ("decay", ctypes.c_double),
        ("dt", ctypes.c_double), ("secretion", ctypes.c_double), ("gradient_weight", ctypes.c_double),
    ]


_ready = False


def lib():
    global _ready
    L = _sim.lib()
    if not _ready:
        P = ctypes.POINTER(SomaParams)
        L.orc_diffusion_step.argtypes = [_dp, _dp, P]
        L.orc_diffusion_step.restype = None
        L.orc_soma_voxel.argtypes = [ctypes.c_double] * 3 + [P]
        L.orc_soma_voxel.restype = ctypes.c_int64
        L.orc_soma_gradient.argtypes = [_dp, ctypes.c_double, ctypes.c_double, ctypes.c_double, P, _dp]
        L.orc_soma_gradient.restype = None
        L.orc_soma_step.argtypes = [ctypes.c_int64, _dp, _dp, _dp, _i32p, _dp, P]
        L.orc_soma_step.restype = ctypes.c_int
        _ready = True
    return L


def make_params(lo=0.0, space=100.0, resolution=20, n_substances=2, diffusion=1.0, decay=0.01, dt=1.0,
                secretion=1.0, gradient_weight=0.75):
    return SomaParams(float(lo), float(space), int(resolution), int(n_substances), float(diffusion), float(decay),
                      float(dt), float(secretion), float(gradient_weight))


def diffusion_step(u, params):
    """One step of Eq 4.3 on one substance grid u (R x R x R, indexed [z, y, x])."""
    u = np.ascontiguousarray(u, dtype=np.float64)
    out = np.empty_like(u)
    lib().orc_diffusion_step(u.ctypes.data_as(_dp), out.ctypes.data_as(_dp), ctypes.byref(params))
    return out


def gradient(u, pos, params):
    u = np.ascontiguousarray(u, dtype=np.float64)
    g = np.zeros(3)
    lib().orc_soma_gradient(u.ctypes.data_as(_dp), float(pos[0]), float(pos[1]), float(pos[2]),
                            ctypes.byref(params), g.ctypes.data_as(_dp))
    return g


def voxel(pos, params):
    return int(lib().orc_soma_voxel(float(pos[0]), float(pos[1]), float(pos[2]), ctypes.byref(params)))


class OracleSoma:
    """Cells of n_substances types and their substance grids."""

    def __init__(self, pos, cell_type, params, conc=None):
        pos = np.asarray(pos, dtype=np.float64).reshape(-1, 3)
        self.n = pos.shape[0]
        self.x = np.ascontiguousarray(pos[:, 0])
        self.y = np.ascontiguousarray(pos[:, 1])
        self.z = np.ascontiguousarray(pos[:, 2])
        self.type = np.ascontiguousarray(cell_type, dtype=np.int32).copy()
        R = params.resolution
        shape = (params.n_substances, R, R, R)
        self.u = (np.zeros(shape) if conc is None else np.ascontiguousarray(conc, dtype=np.float64).reshape(shape)
                  ).copy()
        self.params = params

    def step(self, n_iter=1):
        L = lib()
        for _ in range(n_iter):
            rc = L.orc_soma_step(self.n, self.x.ctypes.data_as(_dp), self.y.ctypes.data_as(_dp),
                                 self.z.ctypes.data_as(_dp), self.type.ctypes.data_as(_i32p),
                                 self.u.ctypes.data_as(_dp), ctypes.byref(self.params))
            if rc != 0:
                raise MemoryError("orc_soma_step")

    def pos(self):
        return np.stack([self.x, self.y, self.z], axis=1)
