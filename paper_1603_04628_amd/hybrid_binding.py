"""ctypes binding of the hybrid macro march (hybrid_* in include/hmd.h)."""
import ctypes as _c

import numpy as np

from .binding import Context, HmdError, _lib, _ptr, _sig, d, i32, i64, u64, u8, vp

P = _c.POINTER


class HybridCfg(_c.Structure):
    _fields_ = [("n_sections", i32), ("h0", d), ("amp", d), ("L", d), ("dt_macro", d), ("rho_ref", d),
                ("p_out", d), ("dp_mean", d), ("dp_amp", d), ("period", d), ("c2", d), ("tau_rel", d),
                ("tau_abs", d), ("surrogate", i32), ("audit_every", i32), ("md_sample", i64),
                ("refit_every", i32), ("seed", u64), ("mirror", i32), ("audit_batch", i32),
                ("warm_start", i32), ("pseudo_nu", d), ("pseudo_slip", d), ("pseudo_tol", d),
                ("n_min_warm", i64), ("n_min_cold", i64), ("geometry", i32), ("f_amp", d), ("f_period", d),
                ("eos", i32)]


class HybridStats(_c.Structure):
    _fields_ = [("steps", i64), ("md_calls", i64), ("audited", i64), ("audit_pass", i64), ("queries", i64),
                ("md_failed", i64), ("wall_s", d), ("md_wall_s", d), ("md_atom_steps", d),
                ("surrogate_wall_s", d), ("audit_wall_s", d), ("audit_atom_steps", d),
                ("md_equil_atom_steps", d), ("warm_starts", i64), ("md_atom_steps_cold", d),
                ("audit_pass_cal", i64), ("p_appends", i64)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


MICRO_FN = _c.CFUNCTYPE(i32, vp, i32, P(d), P(d), P(d), P(d))
MICRO_P_FN = _c.CFUNCTYPE(i32, vp, i32, P(d), P(d), P(d), P(d), P(d), P(d), P(d))

_sig("hmd_hybrid_cfg_default", None, P(HybridCfg))
_sig("hybrid_create", i32, vp, P(HybridCfg), vp, vp, P(vp))
_sig("hybrid_set_micro", i32, vp, MICRO_FN, vp)
_sig("hybrid_set_micro_p", i32, vp, MICRO_P_FN, vp)
_sig("hybrid_set_pressure_gp", i32, vp, vp)
_sig("hybrid_get_pressure", i32, vp, P(d), P(d))
_sig("hybrid_set_forcing", i32, vp, P(d), i64)
_sig("hybrid_set_rho", i32, vp, P(d))
_sig("hybrid_step", i32, vp, P(HybridStats))
_sig("hybrid_get", i32, vp, P(d), P(d), P(d), P(d), P(u8))
_sig("hybrid_flush_audits", i32, vp, P(HybridStats))
_sig("hybrid_last_plan", i32, vp, P(i32), P(i64), P(i64))
_sig("hybrid_free", None, vp)


def hybrid_cfg(**kw):
    c = HybridCfg()
    _lib.hmd_hybrid_cfg_default(_c.byref(c))
    for k, v in kw.items():
        setattr(c, k, v)
    return c


class Hybrid:
    """hybrid_*: macro march with the device GP or ensemble as surrogate.

    `micro`, when given, is a Python callable (h, g) -> (q, se) used instead
    of batched MD (kept alive by this object); with cfg.eos = 1 it is
    (h, rho, g) -> (q, se, p, p_se), and `pgp` is the pressure GP."""

    def __init__(self, ctx: Context, cfg: HybridCfg, gp=None, ens=None, micro=None, pgp=None):
        self.ctx = ctx
        self.cfg = cfg
        self.n = cfg.n_sections
        self._h = vp()
        ctx.check(_lib.hybrid_create(ctx.handle, _c.byref(cfg), gp.handle if gp is not None else None,
                                     ens.handle if ens is not None else None, _c.byref(self._h)))
        self._keep = (gp, ens, pgp)
        self._cb = None
        if pgp is not None:
            ctx.check(_lib.hybrid_set_pressure_gp(self._h, pgp.handle))
        if micro is not None and cfg.eos == 1:
            def cbp(user, n, h, rho, g, q, se, p, pse):
                try:
                    hh, rr, gg = (np.ctypeslib.as_array(a, (n,)).copy() for a in (h, rho, g))
                    qq, ss, pp, ps = micro(hh, rr, gg)
                    for dst, src in ((q, qq), (se, ss), (p, pp), (pse, ps)):
                        np.ctypeslib.as_array(dst, (n,))[:] = src
                    return 0
                except Exception:
                    return 1
            self._cb = MICRO_P_FN(cbp)
            ctx.check(_lib.hybrid_set_micro_p(self._h, self._cb, None))
        elif micro is not None:
            def cb(user, n, h, g, q, se):
                try:
                    hh = np.ctypeslib.as_array(h, (n,)).copy()
                    gg = np.ctypeslib.as_array(g, (n,)).copy()
                    qq, ss = micro(hh, gg)
                    np.ctypeslib.as_array(q, (n,))[:] = qq
                    np.ctypeslib.as_array(se, (n,))[:] = ss
                    return 0
                except Exception:
                    return 1
            self._cb = MICRO_FN(cb)
            ctx.check(_lib.hybrid_set_micro(self._h, self._cb, None))

    def set_rho(self, rho):
        rho = np.ascontiguousarray(rho, dtype=np.float64)
        self.ctx.check(_lib.hybrid_set_rho(self._h, _ptr(rho)))

    def step(self):
        st = HybridStats()
        self.ctx.check(_lib.hybrid_step(self._h, _c.byref(st)))
        return st.as_dict()

    def flush_audits(self):
        st = HybridStats()
        self.ctx.check(_lib.hybrid_flush_audits(self._h, _c.byref(st)))
        return st.as_dict()

    def get(self):
        rho, q, qs, g = (np.zeros(self.n) for _ in range(4))
        fm = np.zeros(self.n, dtype=np.uint8)
        self.ctx.check(_lib.hybrid_get(self._h, _ptr(rho), _ptr(q), _ptr(qs), _ptr(g), _ptr(fm, u8)))
        return {"rho": rho, "q": q, "q_std": qs, "g": g, "from_md": fm.astype(bool)}

    def set_forcing(self, f):
        """Per-macro-step F_ext / m on the periodic channel (empty: the
        sinusoid of the configuration)."""
        f = np.ascontiguousarray(f, dtype=np.float64)
        self.ctx.check(_lib.hybrid_set_forcing(self._h, _ptr(f) if len(f) else None, len(f)))

    def pressure(self):
        """Section pressures of the last step and their GP standard deviations."""
        p, ps = np.zeros(self.n), np.zeros(self.n)
        self.ctx.check(_lib.hybrid_get_pressure(self._h, _ptr(p), _ptr(ps)))
        return p, ps

    def last_plan(self):
        """The last step's fallback plan: prior run per section (-1 lattice,
        -2 no fallback), start-up steps per section, and the batch's."""
        prior = np.zeros(self.n, dtype=np.int32)
        ne = np.zeros(self.n, dtype=np.int64)
        be = i64()
        self.ctx.check(_lib.hybrid_last_plan(self._h, _ptr(prior, i32), _ptr(ne, i64), _c.byref(be)))
        return {"prior": prior, "n_equil": ne, "batch_equil": be.value}

    def close(self):
        if self._h:
            _lib.hybrid_free(self._h)
            self._h = vp()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


__all__ = ["Hybrid", "HybridCfg", "HybridStats", "hybrid_cfg", "HmdError"]
