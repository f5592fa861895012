"""ctypes wrapper over the plain-C FP64 MD oracle (``md_oracle.c``).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

The model follows Appendix A of the paper (shifted LJ fluid, frozen walls,
velocity Verlet, Berendsen on one velocity component, periodic in x and z)
with the body force of Eq. momentumEq (Sec. 2.1) and the time-averaged mass
flow rate of Sec. 2.1 / 2.4 as output.
"""
import ctypes
import os
from dataclasses import dataclass, fields

import numpy as np

from . import build as _build
from . import stats as _stats

_HERE = os.path.dirname(os.path.abspath(__file__))


class OraParams(ctypes.Structure):
    _fields_ = [
        ("rho", ctypes.c_double), ("T0", ctypes.c_double), ("rc", ctypes.c_double),
        ("eps_wf", ctypes.c_double), ("sigma_wf", ctypes.c_double), ("rho_wall", ctypes.c_double),
        ("wall_layers", ctypes.c_int), ("thermo_axis", ctypes.c_int),
        ("dt", ctypes.c_double), ("tau_T", ctypes.c_double),
        ("Lx_nom", ctypes.c_double), ("Lz_nom", ctypes.c_double),
        ("bin_dy", ctypes.c_double), ("n_equil", ctypes.c_int64), ("n_blocks", ctypes.c_int),
        ("n_fluid", ctypes.c_int64), ("delta", ctypes.c_double), ("cell_w", ctypes.c_double),
        ("periodic_y", ctypes.c_int), ("g_sin", ctypes.c_double),
    ]


@dataclass
class Params:
    """MD parameters in reduced LJ units (defaults = the stated readings)."""
    rho: float = 0.8
    T0: float = 1.0
    rc: float = 2.5
    eps_wf: float = 1.0
    sigma_wf: float = 1.0
    rho_wall: float = 1.0
    wall_layers: int = 4
    thermo_axis: int = 1
    dt: float = 0.005
    tau_T: float = 0.1
    Lx_nom: float = 12.0
    Lz_nom: float = 12.0
    bin_dy: float = 0.25
    n_equil: int = 0
    n_blocks: int = 0
    n_fluid: int = 0
    delta: float = 1.0
    cell_w: float = 0.0
    periodic_y: int = 0      # 1: bulk box periodic in y with period h (no walls)
    g_sin: float = 0.0       # extra body force g_sin sin(2 pi y / h) along x

    def to_c(self) -> OraParams:
        return OraParams(**{f.name: getattr(self, f.name) for f in fields(self)})


_lib = None


def lib():
    global _lib
    if _lib is None:
        path = _build.build(force=False)
        L = ctypes.CDLL(path)
        P = ctypes.POINTER
        d, i64, i32, u64, vp = ctypes.c_double, ctypes.c_int64, ctypes.c_int, ctypes.c_uint64, ctypes.c_void_p
        L.ora_create.argtypes = [P(OraParams), d, d, u64]
        L.ora_create.restype = vp
        L.ora_free.argtypes = [vp]
        L.ora_info.argtypes = [vp, P(i64), P(i64), P(d), P(i32)]
        L.ora_get_state.argtypes = [vp, P(d), P(d)]
        L.ora_set_state.argtypes = [vp, P(d), P(d)]
        L.ora_get_wall.argtypes = [vp, P(d)]
        L.ora_get_forces.argtypes = [vp, P(d), P(d)]
        L.ora_forces_brute.argtypes = [vp, P(d)]
        L.ora_forces_brute.restype = d
        L.ora_forces_cells.argtypes = [vp, P(d)]
        L.ora_forces_cells.restype = d
        L.ora_cells.argtypes = [vp, P(i32), P(i32), P(i32)]
        L.ora_run.argtypes = [vp, i64, i32, P(d)]
        L.ora_result.argtypes = [vp, P(d), P(i32)]
        L.ora_nsamples.argtypes = [vp]
        L.ora_nsamples.restype = i64
        L.ora_series.argtypes = [vp, P(d)]
        L.ora_profile.argtypes = [vp, P(d), P(d), P(i32)]
        L.ora_philox4x32_10.argtypes = [P(ctypes.c_uint32), P(ctypes.c_uint32), P(ctypes.c_uint32)]
        L.ora_lj_energy.argtypes = [d, d, d]
        L.ora_lj_energy.restype = d
        L.ora_lj_force.argtypes = [d, d, d]
        L.ora_lj_force.restype = d
        L.ora_num_threads.restype = i32
        _lib = L
    return _lib


def _ptr(a, ct=ctypes.c_double):
    return a.ctypes.data_as(ctypes.POINTER(ct))


def philox4x32_10(ctr, key):
    c = np.asarray(ctr, dtype=np.uint32)
    k = np.asarray(key, dtype=np.uint32)
    out = np.zeros(4, dtype=np.uint32)
    lib().ora_philox4x32_10(_ptr(c, ctypes.c_uint32), _ptr(k, ctypes.c_uint32), _ptr(out, ctypes.c_uint32))
    return out


def lj_energy(r, eps=1.0, sig=1.0):
    return lib().ora_lj_energy(r, eps, sig)


def lj_force(r, eps=1.0, sig=1.0):
    """Magnitude of the radial LJ force at distance r (positive = repulsive)."""
    return lib().ora_lj_force(r, eps, sig)


def num_threads():
    return lib().ora_num_threads()


class System:
    """One NEMD channel system held by the C oracle."""

    def __init__(self, h: float, g: float, seed: int, params: Params = None):
        self.params = params or Params()
        self._cp = self.params.to_c()
        self.h, self.g, self.seed = float(h), float(g), int(seed)
        self._h = lib().ora_create(ctypes.byref(self._cp), self.h, self.g, ctypes.c_uint64(self.seed))
        if not self._h:
            raise ValueError("oracle rejected the system parameters")
        nf, nw = ctypes.c_int64(), ctypes.c_int64()
        box = np.zeros(3)
        nc = np.zeros(3, dtype=np.int32)
        lib().ora_info(self._h, ctypes.byref(nf), ctypes.byref(nw), _ptr(box), _ptr(nc, ctypes.c_int))
        self.n_fluid, self.n_wall = nf.value, nw.value
        self.Lx, self.Lz = float(box[0]), float(box[2])
        self.ncell = tuple(int(c) for c in nc)

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            lib().ora_free(h)
            self._h = None

    # state -------------------------------------------------------------
    def get_state(self):
        x = np.zeros((self.n_fluid, 3))
        v = np.zeros((self.n_fluid, 3))
        lib().ora_get_state(self._h, _ptr(x), _ptr(v))
        return x, v

    def set_state(self, x, v):
        x = np.ascontiguousarray(x, dtype=np.float64)
        v = np.ascontiguousarray(v, dtype=np.float64)
        assert x.shape == (self.n_fluid, 3) and v.shape == (self.n_fluid, 3)
        lib().ora_set_state(self._h, _ptr(x), _ptr(v))

    def wall(self):
        xw = np.zeros((self.n_wall, 3))
        if self.n_wall:
            lib().ora_get_wall(self._h, _ptr(xw))
        return xw

    # forces ------------------------------------------------------------
    def forces_brute(self):
        f = np.zeros((self.n_fluid, 3))
        pe = lib().ora_forces_brute(self._h, _ptr(f))
        return f, pe

    def forces_cells(self):
        f = np.zeros((self.n_fluid, 3))
        pe = lib().ora_forces_cells(self._h, _ptr(f))
        return f, pe

    def neighbors(self, rl):
        """Per fluid atom, the sorted fluid ids and (N_f + wall id) within rl."""
        L = lib()
        L.ora_neighbors.argtypes = [ctypes.c_void_p, ctypes.c_double, ctypes.POINTER(ctypes.c_int),
                                    ctypes.POINTER(ctypes.c_int), ctypes.c_int64]
        L.ora_neighbors.restype = ctypes.c_int64
        counts = np.zeros(self.n_fluid, dtype=np.int32)
        tot = L.ora_neighbors(self._h, rl, _ptr(counts, ctypes.c_int), ctypes.POINTER(ctypes.c_int)(), 0)
        idx = np.zeros(max(tot, 1), dtype=np.int32)
        L.ora_neighbors(self._h, rl, _ptr(counts, ctypes.c_int), _ptr(idx, ctypes.c_int), tot)
        starts = np.concatenate([[0], np.cumsum(counts)])
        return [idx[starts[i]:starts[i + 1]] for i in range(self.n_fluid)]

    def cells(self):
        nx, ny, nz = self.ncell
        cell_of = np.zeros(self.n_fluid, dtype=np.int32)
        counts = np.zeros(nx * ny * nz, dtype=np.int32)
        order = np.zeros(self.n_fluid, dtype=np.int32)
        lib().ora_cells(self._h, _ptr(cell_of, ctypes.c_int), _ptr(counts, ctypes.c_int),
                        _ptr(order, ctypes.c_int))
        return cell_of, counts, order

    # dynamics ----------------------------------------------------------
    def run(self, steps: int, thermostat: bool = True, energy: bool = False):
        trace = np.zeros(steps) if energy else None
        lib().ora_run(self._h, int(steps), 1 if thermostat else 0,
                      _ptr(trace) if energy else ctypes.POINTER(ctypes.c_double)())
        return trace

    def series(self):
        n = lib().ora_nsamples(self._h)
        out = np.zeros(n)
        if n:
            lib().ora_series(self._h, _ptr(out))
        return out

    def flow_diag(self):
        """Sums over the sampled steps (see ora_flow_diag in md_oracle.c)."""
        L = lib()
        L.ora_flow_diag.argtypes = [ctypes.c_void_p, ctypes.POINTER(ctypes.c_double)]
        out = np.zeros(13)
        L.ora_flow_diag(self._h, _ptr(out))
        keys = ("disp", "wraps", "p_start", "p_now", "kick1", "kick2", "fwall_x", "fpair_x", "fwall_y_lo",
                "fwall_y_hi", "virial", "virial_yy", "samples")
        return dict(zip(keys, out.tolist()))

    def force_diag(self):
        """Wall forces on the fluid, total pair force and virial at the
        current positions."""
        L = lib()
        L.ora_force_diag.argtypes = [ctypes.c_void_p, ctypes.POINTER(ctypes.c_double)]
        out = np.zeros(11)
        L.ora_force_diag(self._h, _ptr(out))
        return {"wall_lo": out[0:3].copy(), "wall_hi": out[3:6].copy(), "total": out[6:9].copy(),
                "virial": out[9], "virial_yy": out[10]}

    def wall_force_series(self):
        L = lib()
        L.ora_wall_force_series.argtypes = [ctypes.c_void_p, ctypes.POINTER(ctypes.c_double)]
        n = lib().ora_nsamples(self._h)
        out = np.zeros(n)
        if n:
            L.ora_wall_force_series(self._h, _ptr(out))
        return out

    def pressure_series(self):
        """Per sampled step: the normal pressure on the walls,
        (F_lo,y - F_hi,y) / (2 Lx Lz), the mean of the two walls' normal
        forces per unit area (the cross-section average of P_yy, by the yy
        momentum balance; Alg. 1's pressure output of an MD run)."""
        L = lib()
        L.ora_pressure_series.argtypes = [ctypes.c_void_p, ctypes.POINTER(ctypes.c_double)]
        n = lib().ora_nsamples(self._h)
        out = np.zeros(n)
        if n:
            L.ora_pressure_series(self._h, _ptr(out))
        return out

    def displacements(self):
        L = lib()
        L.ora_displacements.argtypes = [ctypes.c_void_p, ctypes.POINTER(ctypes.c_double)]
        out = np.zeros(self.n_fluid)
        L.ora_displacements(self._h, _ptr(out))
        return out

    def profile(self):
        nb = ctypes.c_int()
        lib().ora_profile(self._h, ctypes.POINTER(ctypes.c_double)(), ctypes.POINTER(ctypes.c_double)(),
                          ctypes.byref(nb))
        mvx = np.zeros(nb.value)
        cnt = np.zeros(nb.value)
        lib().ora_profile(self._h, _ptr(mvx), _ptr(cnt), ctypes.byref(nb))
        return mvx, cnt

    def result(self):
        """Mean flux and its standard error over the sampled steps (Sec. 2.3:
        from the raw time-instantaneous data).  n_blocks = 0: Geyer's initial
        monotone sequence estimator over the per-step series, with the
        non-convergence test on its two halves; n_blocks >= 2: the block rule
        of the C oracle."""
        out = np.zeros(8)
        st = ctypes.c_int()
        lib().ora_result(self._h, _ptr(out), ctypes.byref(st))
        status = st.value
        if self.params.n_blocks == 0:
            ser = self.series()
            if len(ser) >= 2:
                mean, se = _stats.geyer(ser)
                m1, m2 = _stats.halves(ser)
                out[0], out[1], out[2] = mean, se, mean / self.h
                # non-convergence (reading of the critical-shear remark,
                # Sec. 3.2): the two halves differ by more than 8 SE, or the
                # spanwise temperature runs away
                if status == 0 and (abs(m2 - m1) > 8.0 * se or out[5] > 1.5 * self.params.T0):
                    status = -5
        res = {"flux": out[0], "flux_se": out[1], "jflux": out[2], "T": out[3:6].copy(),
               "pe": out[6], "lambda": out[7], "status": status, "n_fluid": self.n_fluid}
        # the run's pressure and its standard error (Geyer, over the per-step
        # wall pressure)
        pser = self.pressure_series()
        if len(pser) >= 2:
            res["p"], res["p_se"] = _stats.geyer(pser)
        else:
            res["p"], res["p_se"] = (float(pser[0]) if len(pser) else 0.0), 0.0
        return res


def md_flux(h, g, seed, n_sample, params: Params = None):
    """Oracle counterpart of the library's md_flux: equilibrate ``params.n_equil``
    steps, then sample ``n_sample`` steps; returns the result dictionary."""
    p = params or Params()
    s = System(h, g, seed, p)
    s.run(p.n_equil + n_sample)
    return s.result()


def block_stats(series, n_blocks=20):
    """(mean, SE, first-half mean, second-half mean) of ``n_blocks`` contiguous
    block means; the remainder is dropped from the front."""
    s = np.ascontiguousarray(series, dtype=np.float64)
    out = np.zeros(4)
    L = lib()
    L.ora_block_stats.argtypes = [ctypes.POINTER(ctypes.c_double), ctypes.c_int64, ctypes.c_int,
                                  ctypes.POINTER(ctypes.c_double)]
    L.ora_block_stats.restype = ctypes.c_int64
    B = L.ora_block_stats(_ptr(s), len(s), n_blocks, _ptr(out))
    return out[0], out[1], out[2], out[3], B
