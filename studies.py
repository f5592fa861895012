"""The studies of Sec. 3 on the paper's periodic benchmark channel, measured
against this library's own MD (no full-channel MD data is available):

  T1-T6  the uncertainty threshold (Sec. 3.1-3.2), from an empty flux database;
  D1-D5  the initial database (Sec. 3.3, Table preDatabases);
  S1-S4  N = 5, 10, 20, 40 subdomains, each starting from the database the
         previous case ended with (Sec. 3.4);
  F1-F2  a variable-frequency and a variable-amplitude external force,
         starting from Case 1's database (Sec. 3.4).

The reference is the all-MD march: every subdomain runs MD at every macro step,
with the same protocol and the same pressure surrogate.  Its subdomain-mean
flux series, smoothed by the App. B periodic-kernel GP over time, is the
reference of Eq. error; its MD atom-steps stand for the full MD's in
Eq. speedup.  Every case prints a progress line to stderr; the result is one
JSON object on stdout (and, with --markdown, a summary table).

    python studies.py [--cases T,D,S,F] [--markdown FILE]
"""
import argparse
import json
import sys
import time

import numpy as np

import workloads

# the paper's channel (Eqs. subsEq, heightEq) in reduced units: h_1 = 10,
# a = 2 (amp = a / h_1), L = 200, five subdomains
CH = dict(h0=10.0, amp=0.2, L=200.0, geometry=1)
N0 = 5
RHO0 = (0.782, 0.776, 0.751, 0.748, 0.771)   # the paper's initial subdomain densities (1331 ... 1312 kg/m^3)
F_A = 0.02                                    # amplitude of Eq. extForcing1 (F_ext / m)
PERIOD = 100                                  # forcing period in macro steps at N = 5
STEPS = 200                                   # two periods
MD = (2000, 8000)                             # MD protocol of every run: equilibration + sampling steps
PRE = (2000, 4000)                            # pressure pre-simulations at rest
PRE_RHOS = tuple(np.round(np.linspace(0.60, 0.95, 15), 4))
DB_RHOS = tuple(np.linspace(0.658, 0.870, 4))  # the paper's 1120-1480 kg/m^3, four densities
DB_G = tuple(np.linspace(0.0, F_A, 4))         # |F| from zero to the external amplitude, four forces
THRESH = (0.1, 0.2, 0.3, 0.5, 0.7, 0.9)        # sigma_t / sigma_f of Cases T1-T6
G_SPAN = 2.5 * F_A


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def heights(n):
    """Eqs. subsEq and heightEq."""
    s = np.arange(n) * CH["L"] / n
    a = CH["amp"] * CH["h0"]
    return a * (np.cos(2.0 * np.pi * s / CH["L"]) - 1.0) + CH["h0"]


def initial_rho(n):
    """The paper's five initial densities, linearly interpolated around the
    ring for finer subdivisions (section k of n sits at s = k L / n)."""
    s0 = np.arange(N0 + 1) / N0
    r0 = np.append(RHO0, RHO0[0])
    return np.interp(np.arange(n) / n, s0, r0)


def forcing_table(kind, steps, period, amp):
    """F_ext / m per macro step.  'sine': Eq. extForcing1; 'chirp' (Case F1):
    the period grows linearly from a tenth of `period` to `period` over the
    run, the phase being the integral of 2 pi / T; 'ramp' (Case F2): the
    amplitude grows linearly from amp to 1.25 amp at a fixed period."""
    k = np.arange(steps, dtype=np.float64)
    if kind == "sine":
        return amp * np.sin(2.0 * np.pi * k / period)
    if kind == "chirp":
        T = period / 10.0 + (period - period / 10.0) * k / steps
        phase = 2.0 * np.pi * np.concatenate([[0.0], np.cumsum(1.0 / T[:-1])])
        return amp * np.sin(phase)
    if kind == "ramp":
        return amp * (1.0 + 0.25 * k / steps) * np.sin(2.0 * np.pi * k / period)
    raise ValueError(kind)


def eq_error(q, Q):
    """Eq. error at the last step: sum |q_i - Q_i| / sum |Q_i|, in percent."""
    q, Q = np.asarray(q, dtype=np.float64), np.asarray(Q, dtype=np.float64)
    return float(100.0 * np.abs(q - Q).sum() / np.abs(Q).sum())


def eq_error_series(q, Q):
    """Eq. error at every step t (cumulative sums)."""
    q, Q = np.asarray(q, dtype=np.float64), np.asarray(Q, dtype=np.float64)
    return 100.0 * np.cumsum(np.abs(q - Q)) / np.cumsum(np.abs(Q))


class Study:
    def __init__(self, args):
        import torch  # device memory / stream plumbing only
        assert torch.cuda.is_available(), "no GPU"
        import paper_1603_04628_amd as hmd
        from paper_1603_04628_amd import binding as B
        from paper_1603_04628_amd import hybrid_binding as HB
        self.hmd, self.B, self.HB = hmd, B, HB
        self.box = workloads.batch_box()
        self.ctx = hmd.Context(hmd.Params(n_equil=MD[0], **self.box))
        self.out = {"setup": {"channel": dict(CH, n_sections=N0, rho0=list(RHO0)), "f_amp": F_A,
                              "period_steps_at_n5": PERIOD, "steps_at_n5": STEPS,
                              "md_protocol": f"{MD[0]} + {MD[1]} steps", "box": self.box}}
        self.seed = 7000

    # -- databases ----------------------------------------------------------
    def presimulate(self):
        """Pressure database: every distinct N = 5 height over a density
        sweep at rest, one batch (Sec. 2.4 pre-simulations)."""
        hmd = self.hmd
        hu = np.unique(np.round(heights(N0), 9))
        jobs = [(h, 0.0, 300000 + k, PRE[1], r) for k, (h, r) in enumerate((h, r) for h in hu for r in PRE_RHOS)]
        pctx = hmd.Context(hmd.Params(n_equil=PRE[0], pressure=1, **self.box))
        t0 = time.perf_counter()
        res = hmd.md_flux_batch(pctx, jobs)
        ok = [k for k, r in enumerate(res) if r["status"] == 0]
        self.Xp = np.array([[jobs[k][0], jobs[k][4]] for k in ok])
        self.pp = np.array([res[k]["p"] for k in ok])
        self.pse = np.array([res[k]["p_se"] for k in ok])
        g = self.B.GP(self.ctx, self.Xp, self.pp, self.pse, self.B.gp_hyper(ranges=(4.0, 0.35)))
        lml = g.optimize(("sigma_f", "ell"))
        hv = g.hyper()
        g.close()
        self.hp_p = self.B.gp_hyper(ranges=(4.0, 0.35), sigma_f=hv["sigma_f"], ell=hv["ell"])
        self.out["pressure_db"] = {"runs": len(ok), "of": len(jobs), "heights": len(hu),
                                   "densities": [float(r) for r in PRE_RHOS], "protocol": f"{PRE[0]} + {PRE[1]} at rest",
                                   "wall_s": time.perf_counter() - t0, "sigma_f": hv["sigma_f"], "ell": hv["ell"],
                                   "lml": lml, "p_range": [float(self.pp.min()), float(self.pp.max())]}
        log(f"pressure database: {len(ok)}/{len(jobs)} runs, p {self.pp.min():.3f} .. {self.pp.max():.3f}")

    def flux_database(self):
        """Table preDatabases: per channel height h_1 (inlet), h_2, h_3
        (throat), four densities x four forces (D5 holds all three heights)."""
        hmd = self.hmd
        h5 = heights(N0)
        self.h123 = (float(h5[0]), float(h5[1]), float(h5[2]))
        jobs, tags = [], []
        for t, h in enumerate(self.h123):
            for r in DB_RHOS:
                for gv in DB_G:
                    jobs.append((h, float(gv), 400000 + len(jobs), MD[1], float(r)))
                    tags.append(t)
        t0 = time.perf_counter()
        res = hmd.md_flux_batch(self.ctx, jobs)
        wall = time.perf_counter() - t0
        ok = [k for k, r in enumerate(res) if r["status"] == 0]
        self.db = {t: (np.array([[jobs[k][0], jobs[k][4], jobs[k][1]] for k in ok if tags[k] == t]),
                       np.array([res[k]["flux"] for k in ok if tags[k] == t]),
                       np.array([res[k]["flux_se"] for k in ok if tags[k] == t])) for t in range(3)}
        self.db_rate = float(sum(res[k]["n_fluid"] for k in ok)) * sum(MD) / wall
        X5, y5, s5 = self.db_union((0, 1, 2))
        # hyperparameters as the paper sets them: sigma_n from the runs' own
        # SEs, sigma_f and ell maximising the evidence over the largest
        # initial database (Sec. 2.3)
        sigma_n = float(s5.mean())
        hp = self.B.gp_hyper(ranges=(4.0, 0.212, G_SPAN), scale_mode=1, out_scale=0, sigma_n=sigma_n,
                             sigma_f=float(np.sqrt(np.mean(y5 ** 2))))
        g = self.B.GP(self.ctx, X5, y5, s5, hp)
        lml = g.optimize(("sigma_f", "ell"))
        hv = g.hyper()
        g.close()
        self.sigma_f = hv["sigma_f"]
        self.hp_q = self.B.gp_hyper(ranges=(4.0, 0.212, G_SPAN), scale_mode=1, out_scale=0, sigma_n=sigma_n,
                                    sigma_f=hv["sigma_f"], ell=hv["ell"])
        self.out["flux_db"] = {"runs": len(ok), "of": len(jobs), "per_height": [len(self.db[t][1]) for t in range(3)],
                               "heights": list(self.h123), "densities": [float(r) for r in DB_RHOS],
                               "forces": [float(v) for v in DB_G], "wall_s": wall,
                               "md_atom_steps_per_s": self.db_rate,
                               "failed": [(jobs[k][0], jobs[k][4], jobs[k][1], res[k]["status"])
                                          for k in range(len(jobs)) if k not in ok],
                               "sigma_f": hv["sigma_f"], "ell": hv["ell"], "sigma_n": sigma_n,
                               "sigma_n_over_sigma_f": sigma_n / hv["sigma_f"], "lml": lml}
        log(f"flux database: {len(ok)}/{len(jobs)} runs in {wall:.1f} s; sigma_f {hv['sigma_f']:.4g}, "
            f"ell {hv['ell']:.3g}, sigma_n {sigma_n:.3g}")

    def db_union(self, which):
        parts = [self.db[t] for t in which]
        if not parts:
            return np.zeros((0, 3)), np.zeros(0), np.zeros(0)
        return tuple(np.concatenate([p[i] for p in parts]) for i in range(3))

    def macro_dt(self):
        """Explicit-diffusion limit of the march at N = 5 from the D5
        surrogates, D = |dq/dg| |dp/drho| / (rho h), taken over the whole
        database box (the three heights, its densities, forces up to F_A):
        the liquid's dp/drho steepens fast with density, and sections that
        compress past the initial state must stay within the limit;
        dt = 0.4 ds^2 / max D."""
        X5, y5, s5 = self.db_union((0, 1, 2))
        qg = self.B.GP(self.ctx, X5, y5, s5, self.hp_q)
        pg = self.B.GP(self.ctx, self.Xp, self.pp, self.pse, self.hp_p)
        hh, rr, gg = np.meshgrid(np.array(self.h123), np.linspace(DB_RHOS[0], DB_RHOS[-1], 9),
                                 np.linspace(0.1 * F_A, F_A, 4), indexing="ij")
        h, r, g = hh.ravel(), rr.ravel(), gg.ravel()
        d = 1e-3
        qa, _ = qg.predict(np.column_stack([h, r, g + d]))
        qb, _ = qg.predict(np.column_stack([h, r, g - d]))
        pa, _ = pg.predict(np.column_stack([h, r + d]))
        pb, _ = pg.predict(np.column_stack([h, r - d]))
        qg.close()
        pg.close()
        D = np.abs((qa - qb) / (2 * d)) * np.abs((pa - pb) / (2 * d)) / (r * h)
        ds = CH["L"] / N0
        self.dt5 = float(0.4 * ds * ds / D.max())
        self.out["setup"]["dt_macro_at_n5"] = self.dt5

    # -- marches ------------------------------------------------------------
    def march(self, name, n, flux_db, p_db, tau, forcing=None, all_md=False):
        """One march of STEPS (N / 5)^2 macro steps at dt (5 / N)^2, the
        forcing period scaled alike (the same physical time)."""
        B, HB = self.B, self.HB
        scale = (n // N0) ** 2
        steps, period, dt = STEPS * scale, PERIOD * scale, self.dt5 / scale
        Xq, yq, sq = flux_db
        hp_q = self.hp_q
        if all_md:  # a flux surrogate that is never certain: MD everywhere
            hp_q = B.gp_hyper(ranges=(4.0, 0.212, G_SPAN), scale_mode=1, out_scale=0, sigma_n=1e6, sigma_f=1e6)
        qg = B.GP(self.ctx, Xq, yq, sq, hp_q)
        pg = B.GP(self.ctx, p_db[0], p_db[1], p_db[2], self.hp_p)
        self.seed += 1
        cfg = HB.hybrid_cfg(surrogate=0, eos=1, n_sections=n, tau_rel=0.0, tau_abs=tau, md_sample=MD[1],
                            dt_macro=dt, audit_every=0, f_amp=F_A, f_period=float(period), rho_ref=0.78,
                            seed=self.seed, **CH)
        hy = HB.Hybrid(self.ctx, cfg, gp=qg, pgp=pg)
        hy.set_rho(initial_rho(n))
        if forcing is not None:
            hy.set_forcing(forcing_table(forcing, steps, period, F_A))
        qbar, calls = np.zeros(steps), np.zeros(steps, dtype=np.int64)
        rho_hist = []
        g_lo, g_hi = np.inf, -np.inf
        t0 = time.perf_counter()
        last = time.perf_counter()
        for k in range(steps):
            st = hy.step()
            r = hy.get()
            qbar[k] = r["q"].mean()
            calls[k] = st["md_calls"]
            g_lo, g_hi = min(g_lo, float(r["g"].min())), max(g_hi, float(r["g"].max()))
            if scale == 1 or k % scale == scale - 1:
                rho_hist.append(r["rho"].copy())
            if time.perf_counter() - last > 30.0:
                log(f"  {name}: step {k + 1}/{steps}, {st['md_calls']} MD runs")
                last = time.perf_counter()
        wall = time.perf_counter() - t0
        m0 = float((initial_rho(n) * heights(n)).sum())
        rho = np.array(rho_hist)
        res = {"n_sections": n, "steps": steps, "dt_macro": dt, "tau_abs": tau, "forcing": forcing or "sine",
               "md_calls": int(st["md_calls"]), "md_failed": int(st["md_failed"]), "p_appends": int(st["p_appends"]),
               "md_atom_steps": float(st["md_atom_steps"]), "wall_s": wall, "md_wall_s": float(st["md_wall_s"]),
               "calls_by_first_peak": int(calls[min(steps, period // 4) - 1]),
               "calls_first_tenth": int(calls[max(1, steps // 10) - 1]),
               "last_call_step": int(np.nonzero(np.diff(np.concatenate([[0], calls])))[0].max())
               if calls[-1] > 0 else None,
               "mass_drift": float((rho[-1] * heights(n)).sum() / m0 - 1.0),
               "rho_range": [float(rho.min()), float(rho.max())], "g_range": [g_lo, g_hi],
               "rho_final": [float(v) for v in rho[-1]],
               # the two-cell (odd-even) component of the density profile,
               # which the march's central differences leave undamped
               "rho_odd_even": float(np.abs(np.sum(rho[-1] * (-1.0) ** np.arange(n))) / n) if n % 2 == 0 else None,
               "db_start": int(len(yq)), "db_end": len(qg)}
        final = (qg.data(), pg.data())
        hy.close()
        qg.close()
        pg.close()
        log(f"{name}: N={n}, {steps} steps in {wall:.1f} s, {res['md_calls']} MD runs "
            f"({res['calls_by_first_peak']} by the first peak)")
        return res, qbar[scale - 1::scale], calls, final

    def reference_march(self, name, forcing=None):
        """An all-MD march and its subdomain-mean flux smoothed over time by
        GP regression, the hyperparameters maximising the evidence: the
        App. B periodic kernel for Eq. extForcing1, a squared-exponential
        kernel in time for a forcing table that is not periodic."""
        p_db = (self.Xp, self.pp, self.pse)
        res, q, _, _ = self.march(name, N0, (np.zeros((0, 3)), np.zeros(0), np.zeros(0)), p_db, 0.0,
                                  forcing=forcing, all_md=True)
        t = np.arange(len(q), dtype=np.float64)
        B = self.B
        if forcing is None:
            hp = B.gp_hyper(kernel=1, period=float(PERIOD), out_scale=1, sigma_n=0.1 * float(np.std(q)),
                            ranges=(float(len(q)),))
        else:
            hp = B.gp_hyper(kernel=0, scale_mode=1, out_scale=1, sigma_n=0.1 * float(np.std(q)),
                            ranges=(float(len(q)),))
        g = B.GP(self.ctx, t[:, None], q, None, hp)
        lml = g.optimize(("sigma_f", "ell", "sigma_n"))
        Q, _ = g.predict(t[:, None])
        hv = g.hyper()
        g.close()
        res.update({"smoother": {"kernel": "periodic" if forcing is None else "squared exponential",
                                 "sigma_f": hv["sigma_f"], "ell": hv["ell"], "sigma_n": hv["sigma_n"], "lml": lml},
                    "raw_error_pct": eq_error(q, Q), "Q_peak": float(np.abs(Q).max())})
        log(f"{name}: raw series vs its smoothing, Eq. error {res['raw_error_pct']:.1f}%")
        return res, q, Q

    def reference(self):
        """The all-MD march of Eq. extForcing1: the reference of Cases T, D, S."""
        res, q, Q = self.reference_march("reference (all-MD)")
        self.Q, self.Qraw = Q, q
        self.ref_atom_steps = res["md_atom_steps"]
        self.ref_wall = res["wall_s"]
        self.out["reference"] = res

    def score(self, res, qbar):
        res["error_pct"] = eq_error(qbar, self.Q)
        res["error_pct_at_first_peak"] = float(eq_error_series(qbar, self.Q)[PERIOD // 4 - 1])
        res["speedup_atom_steps"] = self.ref_atom_steps / res["md_atom_steps"] if res["md_atom_steps"] > 0 else None
        res["speedup_wall"] = self.ref_wall / res["wall_s"]
        return res

    # -- the studies ----------------------------------------------------------
    def run(self, cases):
        t_all = time.perf_counter()
        self.presimulate()
        self.flux_database()
        self.macro_dt()
        self.reference()
        p_db = (self.Xp, self.pp, self.pse)
        empty = (np.zeros((0, 3)), np.zeros(0), np.zeros(0))
        case1 = None
        if "T" in cases or "S" in cases or "F" in cases:
            self.out["T"] = {}
            for k, c in enumerate(THRESH):
                if k > 0 and "T" not in cases:
                    break
                res, q, _, final = self.march(f"T{k + 1}", N0, empty, p_db, c * self.sigma_f)
                res["tau_over_sigma_f"] = c
                self.out["T"][f"T{k + 1}"] = self.score(res, q)
                if k == 0:
                    case1 = final
        if "D" in cases:
            self.out["D"] = {"D1": dict(self.out["T"]["T1"], note="Case T1")} if "T1" in self.out.get("T", {}) else {}
            for name, which in (("D2", (0,)), ("D3", (2,)), ("D4", (0, 2)), ("D5", (0, 1, 2))):
                res, q, _, _ = self.march(name, N0, self.db_union(which), p_db, THRESH[0] * self.sigma_f)
                res["initial_heights"] = [self.h123[t] for t in which]
                self.out["D"][name] = self.score(res, q)
        if "S" in cases and case1 is not None:
            self.out["S"] = {"S1": {"n_sections": N0, "md_calls": self.out["T"]["T1"]["md_calls"], "note": "Case T1"}}
            fdb, pdb = case1
            for k, n in enumerate((10, 20, 40)):
                res, q, _, (fdb, pdb) = self.march(f"S{k + 2}", n, fdb, pdb, THRESH[0] * self.sigma_f)
                self.out["S"][f"S{k + 2}"] = self.score(res, q)
        if "F" in cases and case1 is not None:
            self.out["F"] = {}
            # Case F1 has an all-MD march of its own forcing as reference
            # (Case F2 has none, as in the paper)
            jres, _, QF1 = self.reference_march("reference F1 (all-MD)", forcing="chirp")
            self.out["reference_F1"] = jres
            for name, kind in (("F1", "chirp"), ("F2", "ramp")):
                res, q, _, _ = self.march(name, N0, case1[0], case1[1], THRESH[0] * self.sigma_f, forcing=kind)
                if name == "F1":
                    res["error_pct"] = eq_error(q, QF1)
                    res["speedup_atom_steps"] = (jres["md_atom_steps"] / res["md_atom_steps"]
                                                 if res["md_atom_steps"] > 0 else None)
                    res["speedup_wall"] = jres["wall_s"] / res["wall_s"]
                self.out["F"][name] = res
        self.out["wall_s"] = time.perf_counter() - t_all
        return self.out


def markdown(out):
    lines = ["| case | N | threshold / sigma_f | initial DB | MD runs | by first peak | Eq. error % | "
             "speed-up (atom-steps) | wall s |", "|---|---|---|---|---|---|---|---|---|"]
    for grp in ("T", "D", "S", "F"):
        for name, r in out.get(grp, {}).items():
            if "steps" not in r:
                continue
            tau = r["tau_abs"] / out["flux_db"]["sigma_f"]
            sp = r.get("speedup_atom_steps")
            err = r.get("error_pct")
            lines.append(f"| {name} | {r['n_sections']} | {tau:.2f} | {r['db_start']} | {r['md_calls']} | "
                         f"{r['calls_by_first_peak']} | {'' if err is None else f'{err:.1f}'} | "
                         f"{'inf' if sp is None else f'{sp:.1f}'} | {r['wall_s']:.1f} |")
    for key, label in (("reference", "reference (all-MD)"), ("reference_F1", "reference F1 (all-MD, F1's forcing)")):
        if key not in out:
            continue
        j = out[key]
        lines.append(f"| {label} | {j['n_sections']} | - | 0 | {j['md_calls']} | {j['calls_by_first_peak']} | "
                     f"{j['raw_error_pct']:.1f} (raw vs smoothed) | 1 | {j['wall_s']:.1f} |")
    return "\n".join(lines) + "\n"


def main():
    global STEPS, PERIOD, MD
    ap = argparse.ArgumentParser()
    ap.add_argument("--cases", default="T,D,S,F", help="comma-separated groups of cases: T, D, S, F")
    ap.add_argument("--markdown", default="", help="also write a summary table to this file")
    ap.add_argument("--steps", type=int, default=STEPS, help="macro steps at N = 5 (two forcing periods)")
    ap.add_argument("--md", default=f"{MD[0]},{MD[1]}", help="MD protocol: equilibration,sampling steps")
    args = ap.parse_args()
    STEPS = args.steps
    PERIOD = max(4, STEPS // 2)
    MD = tuple(int(v) for v in args.md.split(","))
    cases = set(args.cases.split(","))
    out = Study(args).run(cases)
    print(json.dumps(out))
    if args.markdown:
        with open(args.markdown, "w") as f:
            f.write(markdown(out))


if __name__ == "__main__":
    main()
