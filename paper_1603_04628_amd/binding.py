"""ctypes binding of libhmd (include/hmd.h): argument marshalling only.

Every computation runs in the HIP library.  If ``libhmd.so`` has not been
built, importing this module raises -- there is no CPU fallback.
"""
import ctypes
import os
from dataclasses import dataclass, fields
from typing import List, Sequence

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIBPATH = os.path.join(HERE, "libhmd.so")

HMD_OK, HMD_EINVAL, HMD_EDEVICE, HMD_ENOMEM, HMD_EUNSTABLE, HMD_ENOTCONV, HMD_ENOTSPD, HMD_ENOSYS = \
    0, -1, -2, -3, -4, -5, -6, -7
STATUS_NAMES = {0: "HMD_OK", -1: "HMD_EINVAL", -2: "HMD_EDEVICE", -3: "HMD_ENOMEM", -4: "HMD_EUNSTABLE",
                -5: "HMD_ENOTCONV", -6: "HMD_ENOTSPD", -7: "HMD_ENOSYS"}

if not os.path.exists(LIBPATH):
    raise ImportError(f"{LIBPATH} is not built: run __graft_entry__.build() (hipcc, gfx950)")

_c = ctypes


def _share_torch_hip_runtime():
    """Load PyTorch's bundled HIP runtime first, when there is one.  It has
    the same soname as ROCm's, so libhmd.so then binds to it and a process
    that also uses torch holds one runtime: device pointers and streams pass
    between the two, and torch's synchronisation covers the library's work."""
    try:
        import importlib.util
        spec = importlib.util.find_spec("torch")
    except (ImportError, ValueError):
        return
    if spec is None or not spec.submodule_search_locations:
        return
    path = os.path.join(list(spec.submodule_search_locations)[0], "lib", "libamdhip64.so")
    if os.path.exists(path):
        _c.CDLL(path, mode=_c.RTLD_GLOBAL)


_share_torch_hip_runtime()
_lib = _c.CDLL(LIBPATH)
P = _c.POINTER
d, i32, i64, u64, u32, u8, vp = _c.c_double, _c.c_int, _c.c_int64, _c.c_uint64, _c.c_uint32, _c.c_uint8, _c.c_void_p


class MdParams(_c.Structure):
    _fields_ = [("rho", d), ("T0", d), ("rc", d), ("eps_wf", d), ("sigma_wf", d), ("rho_wall", d),
                ("wall_layers", i32), ("thermo_axis", i32), ("dt", d), ("tau_T", d), ("Lx_nom", d),
                ("Lz_nom", d), ("bin_dy", d), ("n_equil", i64), ("n_blocks", i32), ("n_fluid", i64),
                ("delta", d), ("force_path", i32), ("skin", d), ("cell_w", d), ("tile_alpha", d),
                ("graph_chunk", i32), ("pressure", i32)]


class MdJob(_c.Structure):
    _fields_ = [("h", d), ("g", d), ("seed", u64), ("n_sample", i64), ("rho", d)]


class MdResult(_c.Structure):
    _fields_ = [("flux", d), ("flux_se", d), ("jflux", d), ("T", d * 3), ("pe", d), ("n_fluid", i64),
                ("status", i32), ("p", d), ("p_se", d)]


def _sig(name, res, *args):
    fn = getattr(_lib, name)
    fn.restype = res
    fn.argtypes = list(args)
    return fn


_sig("hmd_md_params_default", None, P(MdParams))
_sig("hmd_create", i32, P(MdParams), i32, vp, P(vp))
_sig("hmd_destroy", None, vp)
_sig("hmd_last_error", _c.c_char_p, vp)
_sig("hmd_set_params", i32, vp, P(MdParams))
_sig("md_flux", i32, vp, d, d, u64, i64, P(d), P(d))
_sig("md_flux_batch", i32, vp, P(MdJob), i32, P(MdResult))
_sig("md_flux_batch_dev", i32, vp, P(MdJob), i32, vp, vp, vp, vp)
_sig("md_batch_create", i32, vp, P(MdJob), i32, P(vp))
_sig("md_batch_run", i32, vp, i64, i32)
_sig("md_batch_results", i32, vp, P(MdResult))
_sig("md_batch_atoms", i64, vp)
_sig("md_batch_set_timing", i32, vp, i32)
_sig("md_batch_kernel_ms", i32, vp, _c.c_char_p, P(d), P(i64))
_sig("md_batch_pair_count", i32, vp, P(i64), P(i64))
_sig("md_batch_list_builds", i32, vp, P(i64))
_sig("md_batch_get_state", i32, vp, i32, P(d), P(d), P(i64))
_sig("md_batch_forces", i32, vp, i32, P(_c.c_float), P(d))
_sig("md_batch_free", None, vp)
_sig("md_batch_set_state", i32, vp, i32, P(d), P(d))
_sig("md_batch_series", i32, vp, i32, P(d), P(i64))
_sig("md_batch_pressure_series", i32, vp, i32, P(d), P(i64))
_sig("md_series_stats", i32, vp, P(d), i32, i64, i64, i32, P(d))
_sig("md_series_stats_dev", i32, vp, vp, i32, i64, i64, i32, vp, vp)
_sig("md_series_stats_noalloc", i32, vp, vp, i32, i64, i64, i32, vp, vp)
_sig("md_sys_create", i32, vp, d, d, u64, P(vp))
_sig("md_sys_info", i32, vp, P(i64), P(i64), P(d), P(i32))
_sig("md_set_state", i32, vp, P(d), P(d))
_sig("md_get_state", i32, vp, P(d), P(d), P(i64))
_sig("md_compute_forces", i32, vp, P(_c.c_float), P(d))
_sig("md_cell_lists", i32, vp, P(u32), P(u32), P(u32))
_sig("md_run", i32, vp, i64, i32, P(d))
_sig("md_sys_profile", i32, vp, P(d), P(d))
_sig("md_sys_free", None, vp)
_sig("md_neighbor_lists", i32, vp, P(u32), P(u32), i64, P(i64))
_sig("md_sys_config", i32, vp, P(i32), P(d), P(i32), P(i32))
_sig("md_batch_config", i32, vp, P(i32), P(d), P(i32), P(i32))
_sig("md_autotune", i32, vp, P(MdJob), i32, i32, P(d), P(i32))
_sig("md_batch_tuning", i32, vp, P(d))


TUNE_COLUMNS = ("path", "skin", "tpb", "tile_alpha", "cell_w", "chunk", "ms_per_step")


def md_autotune(ctx, jobs, probe_steps=200):
    """Time the candidate configurations on these jobs (coordinate descent
    over path, skin, tile size, cell width, graph chunk); the fastest is
    kept for later batches of the same workload.  Returns one row per
    candidate with the columns of TUNE_COLUMNS."""
    arr = _jobs(jobs)
    table = np.zeros(7 * 64)
    n = i32()
    ctx.check(_lib.md_autotune(ctx.handle, arr, len(jobs), int(probe_steps), _ptr(table), _c.byref(n)))
    return table[:7 * n.value].reshape(-1, 7)


def _config(fn, h):
    path, skin, tpb, cap = i32(), d(), i32(), i32()
    fn(h, _c.byref(path), _c.byref(skin), _c.byref(tpb), _c.byref(cap))
    return {"path": path.value, "skin": skin.value, "tpb": tpb.value, "list_cap": cap.value}


def lib():
    return _lib


def _ptr(a, ct=d):
    return a.ctypes.data_as(P(ct))


class HmdError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{STATUS_NAMES.get(code, code)}: {msg}")
        self.code = code


@dataclass
class Params:
    """hmd_md_params with the library's defaults."""
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
    force_path: int = -1
    skin: float = 0.3
    cell_w: float = 0.0
    tile_alpha: float = 0.0
    graph_chunk: int = 0
    pressure: int = 0

    def to_c(self):
        return MdParams(**{f.name: getattr(self, f.name) for f in fields(self)})


class Context:
    """hmd_ctx on one HIP device (own stream unless `stream` is given)."""

    def __init__(self, params: Params = None, device: int = 0, stream: int = None):
        self.params = params or Params()
        self._h = vp()
        cp = self.params.to_c()
        rc = _lib.hmd_create(_c.byref(cp), device, vp(stream) if stream else None, _c.byref(self._h))
        if rc != HMD_OK:
            raise HmdError(rc, "hmd_create failed (no HIP device?)")

    @property
    def handle(self):
        return self._h

    def set_params(self, params: Params):
        self.params = params
        cp = params.to_c()
        self.check(_lib.hmd_set_params(self._h, _c.byref(cp)))

    def error(self) -> str:
        return (_lib.hmd_last_error(self._h) or b"").decode()

    def check(self, rc):
        if rc != HMD_OK:
            raise HmdError(rc, self.error())
        return rc

    def close(self):
        if self._h:
            _lib.hmd_destroy(self._h)
            self._h = vp()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _jobs(jobs) -> ctypes.Array:
    """(h, g, seed, n_sample[, rho]) tuples; rho <= 0 or absent: the
    context's density."""
    arr = (MdJob * len(jobs))()
    for k, j in enumerate(jobs):
        arr[k] = MdJob(float(j[0]), float(j[1]), int(j[2]), int(j[3]), float(j[4]) if len(j) > 4 else 0.0)
    return arr


def _result_dict(r: MdResult):
    return {"flux": r.flux, "flux_se": r.flux_se, "jflux": r.jflux, "T": np.array(list(r.T)), "pe": r.pe,
            "n_fluid": r.n_fluid, "status": r.status, "p": r.p, "p_se": r.p_se}


def md_flux(ctx: Context, h, g, seed, steps):
    """The micro-solve: returns (status, flux, se)."""
    f, se = d(), d()
    rc = _lib.md_flux(ctx.handle, float(h), float(g), int(seed), int(steps), _c.byref(f), _c.byref(se))
    if rc not in (HMD_OK, HMD_EUNSTABLE, HMD_ENOTCONV):
        raise HmdError(rc, ctx.error())
    return rc, f.value, se.value


def md_flux_batch(ctx: Context, jobs: Sequence) -> List[dict]:
    """jobs: sequence of (h, g, seed, n_sample)."""
    arr = _jobs(jobs)
    out = (MdResult * len(jobs))()
    ctx.check(_lib.md_flux_batch(ctx.handle, arr, len(jobs), out))
    return [_result_dict(r) for r in out]


def _torch_stream():
    import torch
    return vp(torch.cuda.current_stream().cuda_stream)


def _dev_f64(t, cols=None):
    """A contiguous float64 CUDA tensor (device pointers for the *_dev calls)."""
    import torch
    if not (isinstance(t, torch.Tensor) and t.is_cuda):
        raise HmdError(HMD_EINVAL, "expected a CUDA tensor")
    t = t.to(torch.float64).contiguous()
    return t if cols is None else t.reshape(-1, cols)


def md_flux_batch_dev(ctx: Context, jobs: Sequence):
    """md_flux_batch with results in device tensors (flux, se, status) on the
    current torch stream."""
    import torch
    arr = _jobs(jobs)
    n = len(jobs)
    f = torch.empty(n, dtype=torch.float64, device="cuda")
    se = torch.empty_like(f)
    st = torch.empty(n, dtype=torch.int32, device="cuda")
    ctx.check(_lib.md_flux_batch_dev(ctx.handle, arr, n, vp(f.data_ptr()), vp(se.data_ptr()), vp(st.data_ptr()),
                                     _torch_stream()))
    return f, se, st


def series_stats(ctx: Context, x, n_blocks: int = 0):
    """Mean, standard error and half means of each row of x (S x n, or one
    series of n): an (S, 4) array (a 4-vector for one series)."""
    a = np.ascontiguousarray(x, dtype=np.float64)
    one = a.ndim == 1
    a = a.reshape(1, -1) if one else a
    S, n = a.shape
    out = np.zeros((S, 4))
    ctx.check(_lib.md_series_stats(ctx.handle, _ptr(a), S, n, n, int(n_blocks), _ptr(out)))
    return out[0] if one else out


def series_stats_dev(ctx: Context, x, n_blocks: int = 0):
    """series_stats on a CUDA tensor (S x n): a (S, 4) float64 device tensor on
    the current torch stream."""
    import torch
    t = _dev_f64(x)
    t = t.reshape(1, -1) if t.dim() == 1 else t
    S, n = t.shape
    out = torch.empty((S, 4), dtype=torch.float64, device=t.device)
    ctx.check(_lib.md_series_stats_dev(ctx.handle, vp(t.data_ptr()), S, n, n, int(n_blocks), vp(out.data_ptr()),
                                       _torch_stream()))
    return out


def series_stats_noalloc(ctx: Context, x, out, n_blocks: int = 0):
    """md_series_stats_noalloc on CUDA tensors: x (S x n, float64, contiguous)
    and a preallocated out (S x 4, float64); the call itself allocates
    nothing on the device."""
    import torch
    if not (isinstance(x, torch.Tensor) and x.is_cuda and x.dtype == torch.float64 and x.is_contiguous()):
        raise HmdError(HMD_EINVAL, "x must be a contiguous float64 CUDA tensor")
    if not (isinstance(out, torch.Tensor) and out.is_cuda and out.dtype == torch.float64 and out.is_contiguous()):
        raise HmdError(HMD_EINVAL, "out must be a contiguous float64 CUDA tensor")
    S, n = (1, x.shape[0]) if x.dim() == 1 else x.shape
    if out.numel() < 4 * S:
        raise HmdError(HMD_EINVAL, "out needs 4 doubles per series")
    ctx.check(_lib.md_series_stats_noalloc(ctx.handle, vp(x.data_ptr()), S, n, n, int(n_blocks),
                                           vp(out.data_ptr()), _torch_stream()))
    return out


class Batch:
    """Staged batch (md_batch_*): create, run, results, per-kernel timing."""

    def __init__(self, ctx: Context, jobs: Sequence):
        self.ctx = ctx
        self.n = len(jobs)
        self._h = vp()
        ctx.check(_lib.md_batch_create(ctx.handle, _jobs(jobs), self.n, _c.byref(self._h)))

    @property
    def atoms(self) -> int:
        return _lib.md_batch_atoms(self._h)

    def run(self, steps: int, graph_chunk: int = 100):
        self.ctx.check(_lib.md_batch_run(self._h, int(steps), int(graph_chunk)))

    def results(self) -> List[dict]:
        out = (MdResult * self.n)()
        self.ctx.check(_lib.md_batch_results(self._h, out))
        return [_result_dict(r) for r in out]

    def set_timing(self, on: bool):
        self.ctx.check(_lib.md_batch_set_timing(self._h, 1 if on else 0))

    def kernel_ms(self, name: str):
        ms, n = d(), i64()
        self.ctx.check(_lib.md_batch_kernel_ms(self._h, name.encode(), _c.byref(ms), _c.byref(n)))
        return ms.value, n.value

    def pair_count(self):
        ff, wf = i64(), i64()
        self.ctx.check(_lib.md_batch_pair_count(self._h, _c.byref(ff), _c.byref(wf)))
        return ff.value, wf.value

    def n_fluid(self, sim: int) -> int:
        n = i64()
        self.ctx.check(_lib.md_batch_get_state(self._h, int(sim), None, None, _c.byref(n)))
        return n.value

    def get_state(self, sim: int):
        n = self.n_fluid(sim)
        x, v = np.zeros((n, 3)), np.zeros((n, 3))
        self.ctx.check(_lib.md_batch_get_state(self._h, int(sim), _ptr(x), _ptr(v), None))
        return x, v

    def set_state(self, sim: int, x, v):
        n = self.n_fluid(sim)
        x = np.ascontiguousarray(x, dtype=np.float64)
        v = np.ascontiguousarray(v, dtype=np.float64)
        if x.shape != (n, 3) or v.shape != (n, 3):
            raise HmdError(HMD_EINVAL, f"state of system {sim} needs ({n}, 3) arrays")
        self.ctx.check(_lib.md_batch_set_state(self._h, int(sim), _ptr(x), _ptr(v)))

    def series(self, sim: int):
        """The sampled flux series q'(t) of one system."""
        n = i64()
        self.ctx.check(_lib.md_batch_series(self._h, int(sim), None, _c.byref(n)))
        q = np.zeros(n.value)
        self.ctx.check(_lib.md_batch_series(self._h, int(sim), _ptr(q), _c.byref(n)))
        return q

    def pressure_series(self, sim: int):
        """The sampled wall-pressure series p(t) of one system (pressure on)."""
        n = i64()
        self.ctx.check(_lib.md_batch_pressure_series(self._h, int(sim), None, _c.byref(n)))
        p = np.zeros(n.value)
        self.ctx.check(_lib.md_batch_pressure_series(self._h, int(sim), _ptr(p), _c.byref(n)))
        return p

    def forces(self, sim: int):
        f = np.zeros((self.n_fluid(sim), 3), dtype=np.float32)
        pe = d()
        self.ctx.check(_lib.md_batch_forces(self._h, int(sim), _ptr(f, _c.c_float), _c.byref(pe)))
        return f, pe.value

    def list_builds(self) -> int:
        n = i64()
        self.ctx.check(_lib.md_batch_list_builds(self._h, _c.byref(n)))
        return n.value

    def config(self):
        return _config(_lib.md_batch_config, self._h)

    def tuning(self):
        out = np.zeros(8)
        self.ctx.check(_lib.md_batch_tuning(self._h, _ptr(out)))
        return {"path": int(out[0]), "skin": out[1], "tpb": int(out[2]), "tile_alpha": out[3], "cell_width": out[4],
                "graph_chunk": int(out[5]), "tiles": int(out[6]), "list_cap": int(out[7])}

    def close(self):
        if self._h:
            _lib.md_batch_free(self._h)
            self._h = vp()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class System:
    """md_sys_*: one channel system with state access (atom id order)."""

    def __init__(self, ctx: Context, h, g, seed):
        self.ctx = ctx
        self._h = vp()
        ctx.check(_lib.md_sys_create(ctx.handle, float(h), float(g), int(seed), _c.byref(self._h)))
        nf, nw = i64(), i64()
        box = np.zeros(3)
        nc = np.zeros(3, dtype=np.int32)
        ctx.check(_lib.md_sys_info(self._h, _c.byref(nf), _c.byref(nw), _ptr(box), _ptr(nc, i32)))
        self.n_fluid, self.n_wall = nf.value, nw.value
        self.Lx, self.h, self.Lz = box
        self.ncell = tuple(int(c) for c in nc)

    def get_state(self):
        x = np.zeros((self.n_fluid, 3))
        v = np.zeros((self.n_fluid, 3))
        self.ctx.check(_lib.md_get_state(self._h, _ptr(x), _ptr(v), None))
        return x, v

    def set_state(self, x, v):
        x = np.ascontiguousarray(x, dtype=np.float64)
        v = np.ascontiguousarray(v, dtype=np.float64)
        assert x.shape == (self.n_fluid, 3) and v.shape == (self.n_fluid, 3)
        self.ctx.check(_lib.md_set_state(self._h, _ptr(x), _ptr(v)))

    def forces(self):
        f = np.zeros((self.n_fluid, 3), dtype=np.float32)
        pe = d()
        self.ctx.check(_lib.md_compute_forces(self._h, _ptr(f, _c.c_float), _c.byref(pe)))
        return f, pe.value

    def cells(self):
        nx, ny, nz = self.ncell
        cell_of = np.zeros(self.n_fluid, dtype=np.uint32)
        counts = np.zeros(nx * ny * nz, dtype=np.uint32)
        order = np.zeros(self.n_fluid, dtype=np.uint32)
        self.ctx.check(_lib.md_cell_lists(self._h, _ptr(cell_of, u32), _ptr(counts, u32), _ptr(order, u32)))
        return cell_of, counts, order

    def run(self, steps: int, thermostat: bool = True, energy: bool = False):
        trace = np.zeros(int(steps)) if energy else None
        self.ctx.check(_lib.md_run(self._h, int(steps), 1 if thermostat else 0,
                                   _ptr(trace) if energy else None))
        return trace

    def config(self):
        return _config(_lib.md_sys_config, self._h)

    def neighbors(self):
        """Pair path: per atom id, sorted neighbour ids (N_f + w for wall w)."""
        counts = np.zeros(self.n_fluid, dtype=np.uint32)
        tot = i64()
        self.ctx.check(_lib.md_neighbor_lists(self._h, _ptr(counts, u32), None, 0, _c.byref(tot)))
        idx = np.zeros(max(tot.value, 1), dtype=np.uint32)
        self.ctx.check(_lib.md_neighbor_lists(self._h, _ptr(counts, u32), _ptr(idx, u32), tot.value, _c.byref(tot)))
        starts = np.concatenate([[0], np.cumsum(counts.astype(np.int64))])
        return [idx[starts[i]:starts[i + 1]] for i in range(self.n_fluid)]

    def profile(self):
        nb = int(np.ceil(self.h / self.ctx.params.bin_dy))
        mvx, cnt = np.zeros(nb), np.zeros(nb)
        self.ctx.check(_lib.md_sys_profile(self._h, _ptr(mvx), _ptr(cnt)))
        return mvx, cnt

    def close(self):
        if self._h:
            _lib.md_sys_free(self._h)
            self._h = vp()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ---------------------------------------------------------------- GP surrogate
class GpHyper(_c.Structure):
    _fields_ = [("sigma_f", d), ("ell", d), ("sigma_n", d), ("scale_mode", i32), ("range", d * 4),
                ("out_scale", i32), ("noise_mode", i32), ("kernel", i32), ("period", d)]


_sig("hmd_gp_hyper_default", None, P(GpHyper))
_sig("hmd_measure_peaks", i32, vp, P(d))
_sig("gp_fit", i32, vp, P(d), P(d), P(d), i32, i32, P(GpHyper), P(vp))
_sig("gp_append", i32, vp, P(d), d, d)
_sig("gp_predict", i32, vp, P(d), i32, P(d), P(d))
_sig("gp_predict_dev", i32, vp, vp, i32, vp, vp, vp)
_sig("gp_log_marginal", i32, vp, P(d))
_sig("gp_optimize", i32, vp, i32, P(d))
_sig("gp_hyper_get", i32, vp, P(GpHyper))
_sig("gp_size", i32, vp)
_sig("gp_inputs", i32, vp, P(d), P(i32), P(i32))
_sig("gp_outputs", i32, vp, P(d), P(d))
_sig("gp_scales", i32, vp, P(d), P(d), P(d))
_sig("gp_free", None, vp)


def gp_hyper(sigma_f=1.0, ell=1.0, sigma_n=-1.0, scale_mode=0, ranges=(16.0, 0.049), out_scale=1, noise_mode=0,
             kernel=0, period=1.0):
    h = GpHyper()
    _lib.hmd_gp_hyper_default(_c.byref(h))
    h.sigma_f, h.ell, h.sigma_n, h.scale_mode, h.out_scale = sigma_f, ell, sigma_n, scale_mode, out_scale
    h.noise_mode, h.kernel, h.period = noise_mode, kernel, period
    for k, r in enumerate(ranges):
        h.range[k] = r
    return h


class GP:
    """gp_*: FP64 Gaussian process on the device."""

    def __init__(self, ctx: Context, X, y, y_se=None, hyper: GpHyper = None):
        self.ctx = ctx
        X = np.asarray(X, dtype=np.float64)
        X = np.ascontiguousarray(X.reshape(len(y), X.shape[-1] if X.ndim == 2 else -1))
        y = np.ascontiguousarray(y, dtype=np.float64)
        self.d = X.shape[1]
        se = None if y_se is None else np.ascontiguousarray(y_se, dtype=np.float64)
        self._h = vp()
        hp = hyper or gp_hyper()
        ctx.check(_lib.gp_fit(ctx.handle, _ptr(X), _ptr(y), _ptr(se) if se is not None else None, len(y), self.d,
                              _c.byref(hp), _c.byref(self._h)))

    @property
    def handle(self):
        return self._h

    def __len__(self):
        return _lib.gp_size(self._h)

    def append(self, x, y, se=0.0):
        x = np.ascontiguousarray(x, dtype=np.float64)
        self.ctx.check(_lib.gp_append(self._h, _ptr(x), float(y), float(se)))

    def predict(self, Xs):
        Xs = np.ascontiguousarray(np.asarray(Xs, dtype=np.float64).reshape(-1, self.d))
        m = len(Xs)
        mean, var = np.zeros(m), np.zeros(m)
        self.ctx.check(_lib.gp_predict(self._h, _ptr(Xs), m, _ptr(mean), _ptr(var)))
        return mean, var

    def predict_dev(self, Xs):
        """Queries and results as CUDA tensors, on the current torch stream."""
        import torch
        Xs = _dev_f64(Xs, self.d)
        m = Xs.shape[0]
        mean = torch.empty(m, dtype=torch.float64, device=Xs.device)
        var = torch.empty_like(mean)
        self.ctx.check(_lib.gp_predict_dev(self._h, vp(Xs.data_ptr()), m, vp(mean.data_ptr()),
                                           vp(var.data_ptr()), _torch_stream()))
        return mean, var

    def log_marginal(self):
        v = d()
        self.ctx.check(_lib.gp_log_marginal(self._h, _c.byref(v)))
        return v.value

    def data(self):
        """The database: inputs (n x d), outputs and their standard errors."""
        n = len(self)
        X, y, se = np.zeros((n, self.d)), np.zeros(n), np.zeros(n)
        self.ctx.check(_lib.gp_inputs(self._h, _ptr(X), None, None))
        self.ctx.check(_lib.gp_outputs(self._h, _ptr(y), _ptr(se)))
        return X, y, se

    def scales(self):
        sc = np.zeros(self.d)
        sq, sn = d(), d()
        self.ctx.check(_lib.gp_scales(self._h, _ptr(sc), _c.byref(sq), _c.byref(sn)))
        return sc, sq.value, sn.value

    def optimize(self, which=("sigma_f", "ell")):
        """Maximise the evidence (Eq. evidenceEq) over the named
        hyperparameters; returns the maximum."""
        bits = {"sigma_f": 1, "ell": 2, "sigma_n": 4}
        mask = sum(bits[k] for k in which)
        v = d()
        self.ctx.check(_lib.gp_optimize(self._h, mask, _c.byref(v)))
        return v.value

    def hyper(self):
        h = GpHyper()
        self.ctx.check(_lib.gp_hyper_get(self._h, _c.byref(h)))
        return {"sigma_f": h.sigma_f, "ell": h.ell, "sigma_n": h.sigma_n, "noise_mode": h.noise_mode,
                "kernel": h.kernel, "period": h.period}

    def close(self):
        if self._h:
            _lib.gp_free(self._h)
            self._h = vp()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ---------------------------------------------------------------- MLP ensemble
class EnsCfg(_c.Structure):
    _fields_ = [("members", i32), ("hidden", i32), ("iters", i32), ("lr", d), ("seed", u64), ("bootstrap", i32)]


_sig("hmd_ens_cfg_default", None, P(EnsCfg))
_sig("ens_fit", i32, vp, P(d), P(d), i32, P(EnsCfg), P(vp))
_sig("ens_predict", i32, vp, P(d), i32, P(d), P(d))
_sig("ens_predict_dev", i32, vp, vp, i32, vp, vp, vp)
_sig("ens_loss", i32, vp, P(d))
_sig("ens_grad_init", i32, vp, P(d), P(d), i32, P(EnsCfg), i32, P(d), P(d), P(i32))
_sig("ens_members", i32, vp)
_sig("ens_free", None, vp)


def measure_peaks(ctx: Context):
    """hmd_measure_peaks: achievable FP32 FMA TFLOP/s, reciprocals per
    second (x 1e12), a reciprocal's time in FMAs and device-copy GB/s."""
    out = np.zeros(4)
    ctx.check(_lib.hmd_measure_peaks(ctx.handle, _ptr(out)))
    return {"fp32_fma_tflops": float(out[0]), "fp32_rcp_tops": float(out[1]),
            "rcp_cost_in_fma": float(out[2]), "copy_gbs": float(out[3])}


def ens_cfg(members=5, hidden=64, iters=5000, lr=1e-3, seed=0, bootstrap=0):
    return EnsCfg(members, hidden, iters, lr, seed, bootstrap)


class Ensemble:
    """ens_*: MLP deep ensemble trained and evaluated on the device."""

    def __init__(self, ctx: Context, X, y, cfg: EnsCfg = None):
        self.ctx = ctx
        X = np.ascontiguousarray(X, dtype=np.float64).reshape(-1, 2)
        y = np.ascontiguousarray(y, dtype=np.float64)
        self.cfg = cfg or ens_cfg()
        self._h = vp()
        ctx.check(_lib.ens_fit(ctx.handle, _ptr(X), _ptr(y), len(y), _c.byref(self.cfg), _c.byref(self._h)))

    @property
    def handle(self):
        return self._h

    def predict(self, Xs):
        Xs = np.ascontiguousarray(Xs, dtype=np.float64).reshape(-1, 2)
        m = len(Xs)
        mean, std = np.zeros(m), np.zeros(m)
        self.ctx.check(_lib.ens_predict(self._h, _ptr(Xs), m, _ptr(mean), _ptr(std)))
        return mean, std

    def predict_dev(self, Xs):
        """Queries and results as CUDA tensors, on the current torch stream."""
        import torch
        Xs = _dev_f64(Xs, 2)
        m = Xs.shape[0]
        mean = torch.empty(m, dtype=torch.float64, device=Xs.device)
        std = torch.empty_like(mean)
        self.ctx.check(_lib.ens_predict_dev(self._h, vp(Xs.data_ptr()), m, vp(mean.data_ptr()),
                                            vp(std.data_ptr()), _torch_stream()))
        return mean, std

    def losses(self):
        out = np.zeros(self.cfg.members)
        self.ctx.check(_lib.ens_loss(self._h, _ptr(out)))
        return out

    def close(self):
        if self._h:
            _lib.ens_free(self._h)
            self._h = vp()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def ens_grad_init(ctx: Context, X, y, cfg: EnsCfg, member: int):
    """(initial parameters, FP32 gradient of the MSE at them) for one member."""
    X = np.ascontiguousarray(X, dtype=np.float64).reshape(-1, 2)
    y = np.ascontiguousarray(y, dtype=np.float64)
    P_ = cfg.hidden * cfg.hidden + 5 * cfg.hidden + 1
    th, g = np.zeros(P_), np.zeros(P_)
    n = i32()
    ctx.check(_lib.ens_grad_init(ctx.handle, _ptr(X), _ptr(y), len(y), _c.byref(cfg), member, _ptr(th), _ptr(g),
                                 _c.byref(n)))
    return th, g
