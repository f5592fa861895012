"""Hybrid macro-march oracle (Alg. 1 of the paper), FP64 numpy.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

Per macro step (Alg. 1, time-evolution loop):
  1. pressure from the density: a linear equation of state
     p = p_out + c2 (rho - rho_ref) (eos = 0, a reading standing in for the
     pressure GP), or the pressure surrogate p(h, rho) (eos = 1, below);
  2. pressure gradient by central differences (Alg. 1, p' = dp/ds), ghost
     values p_in(t) before the first and p_out after the last section;
  3. body force per section, Eq. momentumEq: g = F_ext/m - (1/rho) dp/ds
     (F_ext = 0: the flow is driven by the oscillating inlet pressure);
  4. surrogate mean and standard deviation at (h, g) (Eqs. predMeanEq,
     predVarEq for the GP); with `mirror` the query is made at (h, |g|) and
     the answer takes the sign of g, since the channel is symmetric under
     s -> -s and the flux is odd in the body force (a reading: the paper's
     database holds both signs of the force instead);
  5. sections whose standard deviation exceeds max(tau_rel |mean|, tau_abs)
     take the flux from the micro-solver and are added to the database
     (Alg. 1 MD branch; tau_abs alone is the paper's absolute threshold
     sigma_t, tau_rel alone a relative one); every `audit_every`-th surrogate
     answer is also checked against the micro-solver;
  6. mass conservation, Eq. continuityEq per unit span:
     d(rho h)/dt = -(q'_{i+1/2} - q'_{i-1/2}) / ds with face fluxes the mean
     of the two neighbouring sections and the boundary faces carrying the
     boundary section's own flux.
The flagged sections of one step are solved together (one batch) and the
database grows after the step, where Alg. 1 walks the sections one by one.

Geometry 1 is the paper's benchmark channel (Sec. 2.1): periodic in s
(the first section sits at inlet and outlet), sections at s_i = (i - 1) L / N
(Eq. subsEq), h = a [cos(2 pi s / L) - 1] + h_1 (Eq. heightEq, with h_1 = h0
and a = amp h0), driven by a uniform external force
F_ext(t) = F_A sin(2 pi t / T) (Eq. extForcing1, t in macro steps); the
pressure gradient and the face fluxes wrap around the ring.

Pressure from a surrogate (eos = 1, Alg. 1 with the paper's full input
set): step 1 takes the mean pressure p(h, rho) of each section from the
pressure surrogate (Alg. 1 GPreg on C_p; inputs h and rho); the flux query
is x* = (h, rho, F) (three inputs, F = g per unit mass); the micro-solver
returns flux and pressure with their standard errors, the flux joins the flux
database and the pressure joins the pressure database when its (h, rho) is
not there yet (both within a relative 1e-9 of an entry count as present).  The boundary pressures p_in(t) and p_out are then absolute.
The pressure database comes from pre-simulations (``presimulate``): per
distinct section height, runs at rest over a sweep of densities (the paper
removes atoms progressively from one run; here each density is its own run,
so that the sweep is one batch).  Warm starts are not combined with it (a
stored state fits only a run of the same atom count).

With warm starts (Alg. 1 "find nearest prior input", "pseudoMD"), each
flagged section's run starts from the recorded fallback run of the same
height whose input is nearest (``startup.nearest_prior``; with the height
fixed only the body force differs), else from the lattice, and equilibrates
for the pseudoMD start-up of the 1-D channel flow (``startup.startup_time``),
at least n_min_warm (n_min_cold from the lattice) steps; the step's batch
equilibrates for the longest of them.
"""
from dataclasses import dataclass

import numpy as np

from . import startup


@dataclass
class HybridCfg:
    n_sections: int = 200
    h0: float = 10.0
    amp: float = 0.5
    L: float = 2000.0
    dt_macro: float = 0.02
    rho_ref: float = 0.8
    p_out: float = 0.0
    dp_mean: float = 10.0
    dp_amp: float = 0.3
    period: float = 250.0     # in macro steps
    c2: float = 200.0
    tau_rel: float = 0.05
    tau_abs: float = 0.0      # absolute threshold sigma_t of Sec. 2.2 (0: off)
    audit_every: int = 0
    mirror: bool = True       # q(h, -g) = -q(h, g): query at |g|, answer with the sign of g
    warm_start: bool = False  # warm starts and pseudoMD start-up lengths
    pseudo_nu: float = 2.5
    pseudo_slip: float = 0.5
    pseudo_tol: float = 0.01
    n_min_warm: int = 1000
    n_min_cold: int = 2000
    md_dt: float = 0.005      # MD time step (start-up time -> steps)
    geometry: int = 0         # 0 inlet/outlet channel, 1 the paper's periodic channel
    f_amp: float = 0.0        # F_A / m of Eq. extForcing1 (geometry 1)
    f_period: float = 250.0   # T of Eq. extForcing1, in macro steps
    eos: int = 0              # 0 linear p = p_out + c2 (rho - rho_ref); 1 pressure surrogate p(h, rho)


class Hybrid:
    """micro(h, g) -> (q, se) arrays (eos = 1: micro(h, rho, g) -> (q, se, p,
    p_se)); surrogate has predict(X) -> (mean, var) and append(x, y, se),
    with X rows (h, g) (eos = 1: (h, rho, g)); psur (eos = 1) is the
    pressure surrogate over (h, rho), a GP with its inputs in .X.
    `var_is_std` selects whether the flux surrogate's second output is a
    standard deviation (ensemble) or a variance (GP)."""

    def __init__(self, cfg: HybridCfg, surrogate, micro, var_is_std=False, rho0=None, psur=None):
        if cfg.eos == 1 and (psur is None or cfg.warm_start):
            raise ValueError("eos = 1 needs a pressure surrogate and no warm starts")
        self.c = cfg
        n = cfg.n_sections
        self.ds = cfg.L / n
        if cfg.geometry == 1:
            self.s = np.arange(n) * self.ds  # Eq. subsEq: s_i = (i - 1) L / N
            self.h = cfg.amp * cfg.h0 * (np.cos(2.0 * np.pi * self.s / cfg.L) - 1.0) + cfg.h0  # Eq. heightEq
        else:
            self.s = (np.arange(n) + 0.5) * self.ds
            self.h = cfg.h0 * (1.0 + cfg.amp * np.cos(2.0 * np.pi * self.s / cfg.L))
        self.rho = np.full(n, cfg.rho_ref) if rho0 is None else np.asarray(rho0, dtype=np.float64).copy()
        self.sur = surrogate
        self.micro = micro
        self.var_is_std = var_is_std
        self.step_no = 0
        self.md_calls = 0
        self.audited = 0
        self.audit_pass = 0
        self.audit_pass_cal = 0   # passes of |mean - q_MD| <= 2 sqrt(std^2 + SE^2)
        self.answers = 0
        self.q = np.zeros(n)
        self.q_std = np.zeros(n)
        self.from_md = np.zeros(n, dtype=bool)
        self.warm = []            # (h, g) of the recorded fallback runs
        self.plan_prior = np.full(n, -2)
        self.plan_equil = np.zeros(n, dtype=np.int64)
        self.plan_batch_equil = 0
        self.psur = psur
        self.p_db = np.zeros((0, 2)) if psur is None else np.asarray(psur.X, dtype=np.float64).reshape(-1, 2).copy()
        self.p_appends = 0
        self.p = np.zeros(n)
        self.p_std = np.zeros(n)
        self.forcing = None       # geometry 1: F_ext / m per macro step (Sec. 3.4 forcing variants)

    def set_forcing(self, f):
        """Macro step k takes f[k] in place of Eq. extForcing1 (the
        variable-frequency and variable-amplitude cases of Sec. 3.4)."""
        if self.c.geometry != 1:
            raise ValueError("a forcing table needs the periodic channel")
        f = np.asarray(f, dtype=np.float64)
        self.forcing = f.copy() if len(f) else None

    def p_known(self, xp):
        """Whether (h, rho) is in the pressure database: both inputs equal
        within a relative 1e-9 (a reading of Alg. 1's test; section heights
        computed with two libraries' cosines can differ in the last bits)."""
        d = np.abs(self.p_db - xp) <= 1e-9 * np.maximum(np.abs(self.p_db), np.abs(xp))
        return bool(np.any(d[:, 0] & d[:, 1]))

    def p_in(self, t_steps):
        c = self.c
        return c.p_out + c.dp_mean * (1.0 + c.dp_amp * np.sin(2.0 * np.pi * t_steps / c.period))

    def f_ext(self, t_steps):
        """Eq. extForcing1 (geometry 1), per unit mass, or the step's entry
        of the forcing table."""
        c = self.c
        if self.forcing is not None:
            if t_steps >= len(self.forcing):
                raise ValueError("the march has reached the end of its forcing table")
            return float(self.forcing[t_steps])
        return c.f_amp * np.sin(2.0 * np.pi * t_steps / c.f_period) if c.geometry == 1 else 0.0

    def pressure(self):
        """Section pressures: the linear law, or (eos = 1) the pressure
        surrogate's mean at (h, rho) with its standard deviation."""
        c = self.c
        if c.eos == 1:
            mean, var = self.psur.predict(np.column_stack([self.h, self.rho]))
            return mean, np.sqrt(np.maximum(var, 0.0))
        return c.p_out + c.c2 * (self.rho - c.rho_ref), np.zeros(len(self.rho))

    def forces(self):
        """Eq. momentumEq per unit mass: F_ext/m - (1/rho) dp/ds."""
        c = self.c
        p, self.p_std = self.pressure()
        self.p = p
        if c.geometry == 1:
            pl, pr = np.roll(p, 1), np.roll(p, -1)
        else:
            pl = np.concatenate([[self.p_in(self.step_no)], p[:-1]])
            pr = np.concatenate([p[1:], [c.p_out]])
        dpds = (pr - pl) / (2.0 * self.ds)
        return self.f_ext(self.step_no) - dpds / self.rho

    def step(self):
        c = self.c
        g = self.forces()
        # mirror symmetry s -> -s of the channel: the flux is odd in the body
        # force, so the query is made at |g| and the answer takes g's sign
        sgn = np.where(g < 0.0, -1.0, 1.0) if c.mirror else np.ones_like(g)
        gq = sgn * g
        X = np.column_stack([self.h, self.rho, gq]) if c.eos == 1 else np.column_stack([self.h, gq])
        mean, second = self.sur.predict(X)
        std = second if self.var_is_std else np.sqrt(np.maximum(second, 0.0))
        flag = std > np.maximum(c.tau_rel * np.abs(mean), c.tau_abs)
        audit = np.zeros_like(flag)
        if c.audit_every > 0:
            for i in np.nonzero(~flag)[0]:
                self.answers += 1
                if self.answers % c.audit_every == 0:
                    audit[i] = True
        run = flag | audit
        q = sgn * mean
        self.plan_prior = np.full(len(g), -2)
        self.plan_equil = np.zeros(len(g), dtype=np.int64)
        self.plan_batch_equil = 0
        if c.warm_start:
            Xw = np.array(self.warm).reshape(-1, 2)
            for i in np.nonzero(flag)[0]:
                x_star = np.array([self.h[i], gq[i]])
                prior = startup.nearest_prior(Xw, x_star, np.ones(2), np.ones(len(Xw), dtype=bool))
                g_in = Xw[prior, 1] if prior >= 0 else 0.0
                ts = startup.startup_time(self.h[i], g_in, gq[i], c.pseudo_nu, c.pseudo_slip, c.pseudo_tol)
                ne = startup.startup_steps(ts, c.md_dt, c.n_min_warm if prior >= 0 else c.n_min_cold)
                self.plan_prior[i] = prior
                self.plan_equil[i] = ne
                self.plan_batch_equil = max(self.plan_batch_equil, ne)
        if run.any():
            idx = np.nonzero(run)[0]
            if c.eos == 1:
                qm, se, pm, pse = self.micro(self.h[idx], self.rho[idx], gq[idx])
            else:
                qm, se = self.micro(self.h[idx], gq[idx])
            self.md_calls += int(flag.sum())  # audits are counted apart
            for k, i in enumerate(idx):
                if flag[i]:
                    q[i] = sgn[i] * qm[k]
                else:
                    self.audited += 1
                    self.audit_pass += int(abs(mean[i] - qm[k]) <= 2.0 * se[k])
                    self.audit_pass_cal += int(abs(mean[i] - qm[k]) <= 2.0 * np.sqrt(std[i] ** 2 + se[k] ** 2))
            for k, i in enumerate(idx):
                if flag[i]:
                    self.sur.append(X[i], qm[k], se[k])
                    if c.warm_start:
                        self.warm.append((self.h[i], gq[i]))
                    # Alg. 1: the run's pressure joins the pressure database
                    # when its (h, rho) is not there yet
                    xp = np.array([self.h[i], self.rho[i]])
                    if c.eos == 1 and not self.p_known(xp):
                        self.psur.append(xp, pm[k], pse[k])
                        self.p_db = np.vstack([self.p_db, xp])
                        self.p_appends += 1
        self.q, self.q_std, self.from_md = q, std, flag
        if c.geometry == 1:  # periodic faces: the last one closes the ring
            face = 0.5 * (q + np.roll(q, -1))
            flux = np.concatenate([[face[-1]], face])
        else:
            face = 0.5 * (q[:-1] + q[1:])
            flux = np.concatenate([[q[0]], face, [q[-1]]])
        m = self.rho * self.h - c.dt_macro * (flux[1:] - flux[:-1]) / self.ds
        self.rho = m / self.h
        self.step_no += 1

    def mass(self):
        return float((self.rho * self.h).sum() * self.ds)


def presimulate(micro_p, heights, rhos):
    """Pressure database of the pre-simulations (Sec. 2.4): every distinct
    height at every density of the sweep, the fluid at rest;
    micro_p(h, rho) -> (p, p_se) arrays.  Returns (X_p rows (h, rho), p,
    p_se)."""
    hs = np.unique(np.asarray(heights, dtype=np.float64))
    H, R = np.meshgrid(hs, np.asarray(rhos, dtype=np.float64), indexing="ij")
    Xp = np.column_stack([H.ravel(), R.ravel()])
    p, pse = micro_p(Xp[:, 0], Xp[:, 1])
    return Xp, np.asarray(p, dtype=np.float64), np.asarray(pse, dtype=np.float64)


def poiseuille_flux(h, g, rho=0.8, eta=2.0, slip=0.0):
    """Continuum flux per unit span of a planar channel with Navier slip:
    q' = rho^2 g h^3 (1 + 6 b / h) / (12 eta)."""
    h = np.asarray(h, dtype=np.float64)
    return rho * rho * np.asarray(g) * h ** 3 * (1.0 + 6.0 * slip / h) / (12.0 * eta)


def lubrication_integral(h0, amp, L, n=200000):
    """int_0^L h(s)^-3 ds for h = h0 (1 + amp cos(2 pi s / L)) (midpoint rule)."""
    s = (np.arange(n) + 0.5) * L / n
    return float(np.sum((h0 * (1 + amp * np.cos(2 * np.pi * s / L))) ** -3) * L / n)
