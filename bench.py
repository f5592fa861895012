"""Benchmark of the batched NEMD micro-solve on one MI355X.

Workload (one "step" = one velocity-Verlet step of every system in the batch,
all hot-path kernels): 64 independent channels in the 57.1 x 57.1 sigma box,
h_k = 4 + 16 u_0(k), g_k = 0.001 + 0.049 u_1(k), seeds 0..63, LJ fluid at
density 0.8 between frozen FCC walls; 10,000 equilibration + 20,000 sampling
steps (30,000 in total).  Inputs are generated on the host and uploaded before
the timed region; the timed region is the step loop (HIP-graph replays).

Prints one JSON line: MD atom-steps/s of the batched path, the same jobs on
the plain path (one system at a time, direct launches), the force kernel's
roofline position from clock stamps around the kernels of the timed graph
replays, the surrogates and the hybrid solve, and the CPU oracle on a bounded
sample.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import workloads  # noqa: E402

METRIC = "MD atom-steps/s (batched FP32 vs plain) + hybrid solve wall-time at flux err<2 SE"
# MI355X published FP32 vector peak (TFLOP/s); the build disables packed-FP32
# instruction selection, which halves the issue rate to 78.6 TFLOP/s.
PEAK_FP32 = 157.3
# FLOPs per in-cutoff ordered pair (FMA = 2, reciprocal = 1): separation 3,
# r^2 5, 1/r^2 1, r^-6 2, force factor 4, accumulation 6.
FLOP_PER_PAIR = 21
N_EQUIL, N_SAMPLE = 10000, 20000
PATH_NAMES = {0: "cell list", 1: "pair list", 2: "pair list, LDS-staged tiles"}
# force kernel of a sampling step on this workload (square box, wall parameters = fluid)
FORCE_KERNELS = {0: "k_force_cell<1>", 1: "k_force_list<1, 0, 1, 1, 0>", 2: "k_force_tiles<1, 0, 1, 1, 0>"}


COUNTERS = os.path.join(ROOT, "profiles", "force_tiles_batch64_counters.md")
KERNEL_SRC = os.path.join(ROOT, "paper_1603_04628_amd", "csrc", "md_kernels.hip")


def committed_counters(kernel):
    """Per-launch HBM traffic and counter FLOPs of the force kernel from the
    committed rocprofv3 summary, or None when that summary covers another
    kernel or the kernel source has changed since the counters were taken."""
    import hashlib
    try:
        vals = {}
        for line in open(COUNTERS):
            if ":" in line and not line.startswith(("|", "#", "`")):
                k, v = line.split(":", 1)
                vals[k.strip()] = v.strip()
        sha = hashlib.sha256(open(KERNEL_SRC, "rb").read()).hexdigest()
    except OSError:
        return None
    if vals.get("source_sha256") != sha or vals.get("kernel") != kernel:
        return None
    return {"traffic": float(vals["traffic_bytes_per_launch"]), "flop": float(vals["counter_flop_per_launch"])}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def advance(batch, n, chunk):
    """n steps as graph replays of `chunk` steps, then one replay of the even
    remainder and, for an odd n, one direct step (chunk 0: direct launches,
    for counter runs)."""
    if chunk == 0:
        batch.run(n, graph_chunk=0)
        return
    full = (n // chunk) * chunk
    if full:
        batch.run(full, graph_chunk=chunk)
    rest = n - full
    if rest >= 2:
        batch.run(rest - rest % 2, graph_chunk=rest - rest % 2)
    if rest % 2:
        batch.run(1, graph_chunk=0)


def timed_plan(steps, warmup, chunk):
    """Which steps of the 10k + 20k protocol are timed.  The timed steps split
    1 : 2 between equilibrating and sampling steps (the protocol's own
    proportion); when they are fewer than the protocol, the rest of the
    equilibration runs untimed between the two timed stretches.  Returns the
    warm-up, the timed stretches, the untimed skip, the graph chunk and the
    graph sizes to capture during the warm-up."""
    total = N_EQUIL + N_SAMPLE
    if warmup + steps >= total:
        eq = max(0, N_EQUIL - warmup)
    else:
        eq = min(max(0, N_EQUIL - warmup), 2 * int(round(steps / 6.0)))
    eq = min(eq, steps)
    sa = steps - eq
    skip = max(0, N_EQUIL - warmup - eq) if sa > 0 else 0
    if chunk == 0:  # direct launches: no graphs to capture
        return {"warmup": warmup, "eq": eq, "sa": sa, "skip": skip, "chunk": 0, "chunks": []}
    c = max(2, min(chunk, eq if eq >= 2 else chunk, sa if sa >= 2 else chunk))
    c -= c % 2
    sizes = set()
    for n in (eq, sa):
        if n >= c:
            sizes.add(c)
        rest = n % c
        if rest >= 2:
            sizes.add(rest - rest % 2)
    return {"warmup": warmup, "eq": eq, "sa": sa, "skip": skip, "chunk": c, "chunks": sorted(sizes)}


def cpu_baseline(budget_s: float):
    """The oracle as it stands on the host cores: one system of the batch
    (seed 0), timed for a bounded number of steps."""
    from oracle import md as omd
    job = workloads.batch_jobs(1)[0]
    s = omd.System(job.h, job.g, job.seed, omd.Params(**workloads.batch_box()))
    s.run(20)  # warm caches and threads
    steps, t0 = 0, time.perf_counter()
    chunk = 20
    while time.perf_counter() - t0 < budget_s:
        s.run(chunk)
        steps += chunk
    dt = time.perf_counter() - t0
    return {"value": s.n_fluid * steps / dt, "unit": "atom-steps/s", "cores": omd.num_threads(),
            "kind": "oracle",
            "sample": f"system 0 of the batch (h={job.h:.2f}, {s.n_fluid} fluid atoms), {steps} steps "
                      f"in {dt:.1f} s, FP64, OpenMP over atoms"}


def copy_calibration(mib: int):
    """A plain device copy of known size (mib MiB read, mib MiB written),
    three times: what a hardware byte counter reads for it calibrates the
    same counter on the force kernel."""
    import torch
    n = mib * (1 << 20) // 4
    src = torch.ones(n, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    log(f"copied {mib} MiB three times")


def summarize_pmc(path: str, kernel: str):
    """Mean per-dispatch value of each counter in a rocprofv3 counter
    collection CSV, over the dispatches whose kernel name contains `kernel`."""
    import csv
    sums, counts = {}, {}
    with open(path, newline="") as fh:
        for row in csv.DictReader(fh):
            if kernel not in row["Kernel_Name"]:
                continue
            k = row["Counter_Name"]
            sums[k] = sums.get(k, 0.0) + float(row["Counter_Value"])
            counts[k] = counts.get(k, 0) + 1
    for k in sorted(sums):
        print(f"{kernel}\t{k}\tdispatches={counts[k]}\tmean={sums[k] / counts[k]:.6g}")


# Macro problem of the hybrid solve: converging-diverging channel
# h(s) = h0 (1 + 0.5 cos 2 pi s / L), 200 cross-sections of 10 sigma, linear
# equation of state with an artificial stiffness c^2 (weakly compressible),
# inlet pressure oscillating by 10% with a period of 250 macro steps, mean
# pressure drop set so the steady lubrication solution has g = 0.038 at the
# throat (h = 5): with the oscillation every g stays inside the training
# range [0.001, 0.05] of the surrogates.
HY = dict(n_sections=200, h0=10.0, amp=0.5, L=2000.0, rho_ref=0.8, p_out=0.0, dp_amp=0.1, period=250.0,
          c2=200.0)
HY_G_THROAT = 0.038
# MD protocol of a fallback or audit call: the batch protocol, long enough
# for the start-up flow of the widest section (h = 15) to settle
HY_EQUIL, HY_SAMPLE = N_EQUIL, N_SAMPLE
HY_STEPS = 500


def _sections():
    n, L = HY["n_sections"], HY["L"]
    s = (np.arange(n) + 0.5) * L / n
    return s, HY["h0"] * (1.0 + HY["amp"] * np.cos(2.0 * np.pi * s / L))


def _lubrication_start(dp):
    """Steady lubrication profile (q' ~ h^3 g constant): g = C / h^3 with the
    integral of g over the channel equal to dp / rho_ref; the density follows
    from the linear equation of state."""
    s, h = _sections()
    ds = HY["L"] / HY["n_sections"]
    w = h ** -3
    C = dp / (HY["rho_ref"] * w.sum() * ds)
    g = C * w
    p = HY["p_out"] + dp - HY["rho_ref"] * (np.cumsum(g) - 0.5 * g) * ds
    return HY["rho_ref"] + (p - HY["p_out"]) / HY["c2"], C


def hybrid_bench(args, hmd, first_results):
    """Surrogate data and fits (training 256 + held-out 64 batched MD runs of
    the batch protocol), then the hybrid march with the GP and with the MLP
    ensemble, and two all-MD macro steps that price the all-MD march."""
    import torch
    from paper_1603_04628_amd import binding as B
    from paper_1603_04628_amd import hybrid_binding as HB
    out = {}
    ctx = hmd.Context(hmd.Params(n_equil=N_EQUIL, **workloads.batch_box()))
    train, test = workloads.surrogate_training_jobs(args.train_points, 64)
    # the timed batch already ran seeds 0..63 with this protocol: reuse them
    reuse = len(first_results) if len(first_results) <= len(train) else 0
    todo = train[reuse:] + test
    t0 = time.perf_counter()
    rnew = hmd.md_flux_batch(ctx, [(j.h, j.g, j.seed, N_SAMPLE) for j in todo])
    t_data = time.perf_counter() - t0
    rtr = list(first_results[:reuse]) + rnew[:len(train) - reuse]
    rte = rnew[len(train) - reuse:]
    ok_tr = [k for k, r in enumerate(rtr) if r["status"] == 0]
    ok_te = [k for k, r in enumerate(rte) if r["status"] == 0]
    X = np.array([[train[k].h, train[k].g] for k in ok_tr])
    y = np.array([rtr[k]["flux"] for k in ok_tr])
    se = np.array([rtr[k]["flux_se"] for k in ok_tr])
    Xt = np.array([[test[k].h, test[k].g] for k in ok_te])
    yt = np.array([rte[k]["flux"] for k in ok_te])
    set_ = np.array([rte[k]["flux_se"] for k in ok_te])
    log(f"surrogate data: {len(ok_tr)} + {len(ok_te)} MD runs in {t_data:.1f} s")
    hyper = B.gp_hyper(ranges=(16.0, 0.049))
    hyper_info = {"rule": args.gp_hyper, "sigma_f": 1.0, "ell": 1.0}
    if args.gp_hyper == "evidence":
        # Sec. 2.3: sigma_f and l maximise the log marginal likelihood of the
        # training data (sigma_n from the runs' own standard errors)
        t0 = time.perf_counter()
        g_opt = B.GP(ctx, X, y, se, hyper)
        lml0 = g_opt.log_marginal()
        lml = g_opt.optimize(("sigma_f", "ell"))
        hp = g_opt.hyper()
        g_opt.close()
        hyper = B.gp_hyper(ranges=(16.0, 0.049), sigma_f=hp["sigma_f"], ell=hp["ell"])
        hyper_info.update(sigma_f=hp["sigma_f"], ell=hp["ell"], lml_at_1_1=lml0, lml=lml,
                          optimize_s=time.perf_counter() - t0)
        log(f"gp hyperparameters by evidence: {hyper_info}")
    ecfg = B.ens_cfg(members=5, hidden=64, iters=args.ens_iters, lr=1e-3)
    Xq = Xt[np.arange(200) % len(Xt)]
    fits = {}
    # the bootstrap ensemble: each member on its own resample of the data
    ecfg_boot = B.ens_cfg(members=5, hidden=64, iters=args.ens_iters, lr=1e-3, bootstrap=1)
    variants = (("gp", 0), ("gp_per_point_noise", 0), ("ensemble", 1), ("ensemble_bootstrap", 2))
    for name, kind in variants:
        t0 = time.perf_counter()
        if kind == 0:
            hp_v = hyper
            if name == "gp_per_point_noise":
                hp_v = B.gp_hyper(ranges=(16.0, 0.049), sigma_f=hyper.sigma_f, ell=hyper.ell, noise_mode=1)
            sur = B.GP(ctx, X, y, se, hp_v)
        else:
            sur = B.Ensemble(ctx, X, y, ecfg if kind == 1 else ecfg_boot)
        torch.cuda.synchronize()
        t_fit = time.perf_counter() - t0
        sur.predict(Xq)
        t0 = time.perf_counter()
        for _ in range(20):
            m, v = sur.predict(Xq)
        t_pred = (time.perf_counter() - t0) / 20
        m, v = sur.predict(Xt)
        sd = np.sqrt(v) if kind == 0 else v
        inside = np.abs(m - yt) <= 2.0 * np.sqrt(sd ** 2 + set_ ** 2)
        fits[name] = {"fit_s": t_fit, "predict_200_ms": 1e3 * t_pred, "heldout_within_2sigma": float(inside.mean()),
                      "heldout_rmse_over_rms": float(np.sqrt(np.mean((m - yt) ** 2)) / np.sqrt(np.mean(yt ** 2))),
                      "heldout_median_se_over_rms": float(np.median(set_) / np.sqrt(np.mean(yt ** 2))),
                      "heldout_median_std_over_rms": float(np.median(sd) / np.sqrt(np.mean(yt ** 2)))}
        log(f"{name}: {fits[name]}")
        sur.close()
    out["surrogate"] = {"train_points": len(ok_tr), "heldout_points": len(ok_te), "md_data_s": t_data,
                        "gp_hyperparameters": hyper_info,
                        "reused_from_timed_batch": reuse,
                        "protocol": f"{N_EQUIL} + {N_SAMPLE} steps per point, 57.1 x 57.1 sigma box", **fits}

    # macro constants: pressure drop from the throat condition, macro step
    # from the explicit diffusion limit with the surrogate's dq'/dg
    _, C0 = _lubrication_start(1.0)
    dp = HY_G_THROAT / (C0 / 5.0 ** 3)
    rho0, _ = _lubrication_start(dp)
    _, hs = _sections()
    gp0 = B.GP(ctx, X, y, se, hyper)
    dg = 1e-3
    qp, _ = gp0.predict(np.column_stack([hs, np.full_like(hs, 0.025 + dg)]))
    qm, _ = gp0.predict(np.column_stack([hs, np.full_like(hs, 0.025 - dg)]))
    dqdg = (qp - qm) / (2 * dg)
    ds = HY["L"] / HY["n_sections"]
    d_max = float(np.max(HY["c2"] * dqdg / (HY["rho_ref"] * hs)))
    dt_macro = 0.4 * ds * ds / d_max
    gp0.close()
    base = dict(HY, dt_macro=dt_macro, dp_mean=dp, md_sample=HY_SAMPLE, refit_every=args.refit_every)
    hctx = hmd.Context(hmd.Params(n_equil=HY_EQUIL, **workloads.batch_box()))

    # absolute floor of the flagging threshold: the typical standard error of
    # the training MD itself (a surrogate this certain is not improved on by
    # a fresh MD call)
    tau_abs = float(np.median(se))

    def run(surrogate, tau, steps, audit_every, budget_s=None, floor=tau_abs, warm=1):
        # surrogate 0: GP; 1: ensemble; 2: bootstrap ensemble (the march's kind 1)
        sur = B.GP(hctx, X, y, se, hyper) if surrogate == 0 else B.Ensemble(hctx, X, y,
                                                                            ecfg if surrogate == 1 else ecfg_boot)
        surrogate = min(surrogate, 1)
        cfg = HB.hybrid_cfg(surrogate=surrogate, tau_rel=tau, tau_abs=floor, audit_every=audit_every,
                            audit_batch=64, warm_start=warm, **base)
        hy = HB.Hybrid(hctx, cfg, gp=sur if surrogate == 0 else None, ens=sur if surrogate == 1 else None)
        hy.set_rho(rho0)
        t0 = time.perf_counter()
        for _ in range(steps):
            st = hy.step()
            if budget_s is not None and time.perf_counter() - t0 > budget_s:
                break
        st = hy.flush_audits()
        wall = time.perf_counter() - t0
        r = hy.get()
        hy.close()
        sur.close()
        st["wall_s"] = wall
        st["rho_range"] = [float(r["rho"].min()), float(r["rho"].max())]
        st["g_range"] = [float(r["g"].min()), float(r["g"].max())]
        return st

    # all-MD: every query answered by batched MD from the lattice with the
    # full protocol (threshold 0, no warm starts) for the first macro steps;
    # the whole march is priced at the rate measured here
    nv = args.all_md_steps
    allmd = run(0, 0.0, nv, 0, floor=0.0, warm=0)
    per_step_atom_steps = allmd["md_atom_steps"] / nv
    md_rate = allmd["md_atom_steps"] / allmd["md_wall_s"]
    all_md_s = args.hybrid_steps * per_step_atom_steps / md_rate
    # training data as MD cost: the atom-steps of the training runs at the
    # measured batched rate (the held-out runs are measurement, not method)
    train_atom_steps = float(sum(rtr[k]["n_fluid"] for k in ok_tr)) * (N_EQUIL + N_SAMPLE)
    train_md_s = train_atom_steps / md_rate
    log(f"all-MD: {nv} steps in {allmd['wall_s']:.1f} s, {md_rate:.3e} atom-steps/s -> {all_md_s:.0f} s for "
        f"{args.hybrid_steps} steps; training MD {train_md_s:.1f} s")
    runs = []
    # the GP under both rules (the plain one only at the thresholds of
    # --plain-taus: elsewhere it falls back at nearly every section and a run
    # stops at its time budget after a step or two), the ensembles under the
    # floor rule at --ens-taus
    plan = [(name, sid, tau, rule) for name, sid in (("gp", 0), ("ensemble", 1), ("ensemble_bootstrap", 2))
            for tau in args.taus for rule in args.rules
            if (name == "gp" and (rule != "plain" or tau in args.plain_taus))
            or (name != "gp" and tau in args.ens_taus and rule != "plain")]
    for name, sid, tau, rule in plan:
        floor = tau_abs if rule == "floor" else 0.0
        st = run(sid, tau, args.hybrid_steps, args.audit_every, budget_s=args.hybrid_budget, floor=floor)
        done = st["steps"]
        method_s = st["wall_s"] - st["audit_wall_s"]  # audits are measurement, not method
        all_md_done = done * per_step_atom_steps
        st.update(surrogate=name, tau=tau, rule=rule, tau_abs=floor, method_wall_s=method_s,
                  speedup_vs_all_md=all_md_done / md_rate / method_s,
                  speedup_vs_all_md_incl_training=all_md_done / md_rate / (method_s + train_md_s * done /
                                                                           args.hybrid_steps),
                  audit_pass_rate=st["audit_pass"] / st["audited"] if st["audited"] else None,
                  audit_pass_rate_with_surrogate_std=st["audit_pass_cal"] / st["audited"] if st["audited"] else None,
                  md_atom_steps_ratio=all_md_done / max(st["md_atom_steps"], 1.0),
                  md_atom_steps_ratio_incl_training=all_md_done / max(
                      st["md_atom_steps"] + train_atom_steps * done / args.hybrid_steps, 1.0),
                  warm_start_atom_steps_saved=st["md_atom_steps_cold"] - st["md_atom_steps"])
        log(f"hybrid {name} tau={tau} {rule}: {done} steps, {method_s:.1f} s (+{st['audit_wall_s']:.1f} s audits), "
            f"md_calls {st['md_calls']} ({st['warm_starts']} warm), audits {st['audit_pass']}/{st['audited']} "
            f"({st['audit_pass_cal']} with the surrogate's std), "
            f"speedup {st['speedup_vs_all_md']:.0f}x ({st['speedup_vs_all_md_incl_training']:.0f}x with training)")
        runs.append(st)
    out["hybrid"] = {"macro": dict(base, steps=args.hybrid_steps, md_protocol=f"{HY_EQUIL} + {HY_SAMPLE} steps",
                                   warm_start="Alg. 1 nearest prior + pseudoMD start-up (1-D N-S, Navier slip)"),
                     "all_md": {"validated_steps": nv, "wall_s_validated": allmd["wall_s"],
                                "atom_steps_per_macro_step": per_step_atom_steps,
                                "md_atom_steps_per_s": md_rate, "estimated_wall_s": all_md_s},
                     "training_md": {"runs": len(ok_tr), "atom_steps": train_atom_steps, "wall_s": train_md_s,
                                     "counted_per": "march steps done / march steps, like the all-MD price"},
                     "runs": runs}
    return out


# The paper's benchmark channel with its full input set (Sec. 2.2; Alg. 1
# with both GPs): 40 sections on a periodic ring (Eqs. subsEq, heightEq:
# h from 6 to 10 sigma), driven by the external force of Eq. extForcing1
# (amplitude 0.01 per unit mass, period 400 macro steps: the narrowest
# sections then see body forces up to about 0.045, the top of the flux
# database).  The pressure GP p(h, rho) comes from pre-simulations at rest
# over a density sweep of every section height (0.025 apart: the pressure
# rises from about 1 to 17 between densities 0.70 and 0.95); the flux GP over
# (h, rho, g) from batched runs at the march's protocol.
EG = dict(n_sections=40, h0=10.0, amp=0.2, L=400.0, geometry=1, f_amp=0.01, f_period=400.0, rho_ref=0.8)
EG_RHOS = tuple(round(0.70 + 0.025 * k, 3) for k in range(11))
EG_PRE = (2000, 4000)     # pre-simulation equilibration and sampling steps
EG_TRAIN = 96             # flux database runs
EG_STEPS = 300            # macro steps


def eos_gp_bench(args, hmd):
    """The hybrid solve with the pressure GP and the 3-input flux GP on the
    paper's periodic channel: pre-simulations, flux database, march, and the
    all-MD price of the same march."""
    from paper_1603_04628_amd import binding as B
    from paper_1603_04628_amd import hybrid_binding as HB
    box = workloads.batch_box()
    n, L, h0, a = EG["n_sections"], EG["L"], EG["h0"], EG["amp"] * EG["h0"]
    heights = a * (np.cos(2.0 * np.pi * (np.arange(n) * L / n) / L) - 1.0) + h0  # the march's sections
    hu = np.unique(np.round(heights, 9))  # mirrored sections agree to the last bits: one run per height
    ctx = hmd.Context(hmd.Params(n_equil=EG_PRE[0], pressure=1, **box))
    t0 = time.perf_counter()
    pre = [(h, 0.0, 200000 + k, EG_PRE[1], r) for k, (h, r) in enumerate((h, r) for h in hu for r in EG_RHOS)]
    rp = hmd.md_flux_batch(ctx, pre)
    t_pre = time.perf_counter() - t0
    okp = [k for k, r in enumerate(rp) if r["status"] == 0]
    Xp = np.array([[pre[k][0], pre[k][4]] for k in okp])
    pp = np.array([rp[k]["p"] for k in okp])
    pse = np.array([rp[k]["p_se"] for k in okp])
    pre_atom_steps = float(sum(rp[k]["n_fluid"] for k in okp)) * sum(EG_PRE)
    log(f"eos-gp: {len(okp)} pre-simulations in {t_pre:.1f} s; p from {pp.min():.3f} to {pp.max():.3f}")
    # flux database at the march's protocol, (h, rho, g) drawn over the ring's
    # heights, densities around the reference and forces up to 0.045
    ctx.set_params(hmd.Params(n_equil=N_EQUIL, pressure=1, **box))
    jobs = workloads.density_jobs(EG_TRAIN, 0, float(hu.min()), float(hu.max()), 0.72, 0.92, 0.001, 0.045)
    t0 = time.perf_counter()
    rq = hmd.md_flux_batch(ctx, [(j.h, j.g, j.seed, N_SAMPLE, j.rho) for j in jobs])
    t_train = time.perf_counter() - t0
    okq = [k for k, r in enumerate(rq) if r["status"] == 0]
    X = np.array([[jobs[k].h, jobs[k].rho, jobs[k].g] for k in okq])
    y = np.array([rq[k]["flux"] for k in okq])
    se = np.array([rq[k]["flux_se"] for k in okq])
    train_atom_steps = float(sum(rq[k]["n_fluid"] for k in okq)) * (N_EQUIL + N_SAMPLE)
    md_rate = train_atom_steps / t_train
    # hyperparameters by the evidence (Sec. 2.3), as for the 2-input GP
    hp_p = B.gp_hyper(ranges=(float(np.ptp(hu)), 0.25))
    hp_q = B.gp_hyper(ranges=(float(np.ptp(hu)), 0.2, 0.044))
    hyp = {}
    for name, Xd, yd, sd, hp in (("p", Xp, pp, pse, hp_p), ("q", X, y, se, hp_q)):
        g = B.GP(ctx, Xd, yd, sd, hp)
        lml = g.optimize(("sigma_f", "ell"))
        hv = g.hyper()
        g.close()
        hyp[name] = {"sigma_f": hv["sigma_f"], "ell": hv["ell"], "lml": lml}
    hp_p = B.gp_hyper(ranges=(float(np.ptp(hu)), 0.25), sigma_f=hyp["p"]["sigma_f"], ell=hyp["p"]["ell"])
    hp_q = B.gp_hyper(ranges=(float(np.ptp(hu)), 0.2, 0.044), sigma_f=hyp["q"]["sigma_f"], ell=hyp["q"]["ell"])
    hctx = hmd.Context(hmd.Params(n_equil=N_EQUIL, **box))
    pg = B.GP(hctx, Xp, pp, pse, hp_p)
    qg = B.GP(hctx, X, y, se, hp_q)
    # macro step from the explicit diffusion limit, D = (dq/dg)(dp/drho) / (rho h),
    # over the flux database's box (every section height, its densities and
    # forces): the liquid's dp/drho steepens fast with density, and sections
    # that compress past the reference must stay within the limit
    dg, dr = 1e-3, 1e-3
    hh, rr, gg = (a.ravel() for a in np.meshgrid(hu, np.linspace(0.72, 0.92, 9), np.linspace(0.0045, 0.045, 4),
                                                  indexing="ij"))
    qa, _ = qg.predict(np.column_stack([hh, rr, gg + dg]))
    qb, _ = qg.predict(np.column_stack([hh, rr, gg - dg]))
    pa, _ = pg.predict(np.column_stack([hh, rr + dr]))
    pb, _ = pg.predict(np.column_stack([hh, rr - dr]))
    D = np.abs((qa - qb) / (2 * dg)) * np.abs((pa - pb) / (2 * dr)) / (rr * hh)
    dt = 0.4 * (L / n) ** 2 / float(D.max())
    cfg = HB.hybrid_cfg(surrogate=0, eos=1, tau_rel=0.05, tau_abs=float(np.median(se)), md_sample=N_SAMPLE,
                        dt_macro=dt, audit_every=0, **EG)
    hy = HB.Hybrid(hctx, cfg, gp=qg, pgp=pg)
    t0 = time.perf_counter()
    for _ in range(EG_STEPS):
        st = hy.step()
        if time.perf_counter() - t0 > args.hybrid_budget:
            break
    wall = time.perf_counter() - t0
    r = hy.get()
    p, p_sd = hy.pressure()
    # all-MD: every section every step at the march's protocol, atoms at each
    # section's height from the pre-simulations at the reference density
    n_at = {round(pre[k][0], 9): rp[k]["n_fluid"] for k in okp if abs(pre[k][4] - 0.80) < 1e-12}
    per_step = float(sum(n_at.get(round(h, 9), 0) for h in heights)) * (N_EQUIL + N_SAMPLE)
    done = st["steps"]
    method_s = wall
    all_md_s = done * per_step / md_rate
    out = {"macro": dict(EG, dt_macro=dt, steps_done=done, tau_rel=0.05, tau_abs=float(np.median(se)),
                         md_protocol=f"{N_EQUIL} + {N_SAMPLE} steps", eos="pressure GP p(h, rho)",
                         flux_inputs="(h, rho, g)"),
           "pre_simulations": {"runs": len(okp), "densities": list(EG_RHOS), "heights": len(hu),
                               "protocol": f"{EG_PRE[0]} + {EG_PRE[1]} steps at rest", "wall_s": t_pre,
                               "atom_steps": pre_atom_steps, "p_range": [float(pp.min()), float(pp.max())],
                               "p_se_median": float(np.median(pse))},
           "flux_database": {"runs": len(okq), "wall_s": t_train, "md_atom_steps_per_s": md_rate},
           "hyperparameters": hyp,
           "march": {"wall_s": method_s, "md_calls": st["md_calls"], "md_failed": st["md_failed"],
                     "p_appends": st["p_appends"], "md_wall_s": st["md_wall_s"],
                     "surrogate_wall_s": st["surrogate_wall_s"],
                     "rho_range": [float(r["rho"].min()), float(r["rho"].max())],
                     "g_range": [float(r["g"].min()), float(r["g"].max())],
                     "p_range": [float(p.min()), float(p.max())], "p_std_max": float(p_sd.max())},
           "all_md_estimated_s": all_md_s,
           "speedup_vs_all_md": all_md_s / method_s,
           "speedup_vs_all_md_incl_presim_and_database": all_md_s / (
               method_s + (t_pre + t_train) * done / EG_STEPS)}
    log(f"eos-gp: {done} steps in {method_s:.1f} s, md_calls {st['md_calls']}, p appends {st['p_appends']}, "
        f"rho {out['march']['rho_range']}, speedup {out['speedup_vs_all_md']:.0f}x "
        f"({out['speedup_vs_all_md_incl_presim_and_database']:.0f}x with pre-simulations and database)")
    hy.close()
    pg.close()
    qg.close()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=N_EQUIL + N_SAMPLE - 200)
    ap.add_argument("--warmup", type=int, default=200)
    ap.add_argument("--chunk", type=int, default=100,
                    help="steps per graph replay; 0: direct launches (for hardware-counter runs)")
    ap.add_argument("--plain-sims", type=int, default=8)
    ap.add_argument("--plain-steps", type=int, default=1000)
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--skin", type=float, default=0.35, help="pair-list skin (sigma); 0.35 is the best of a 0.25-0.45 sweep on this workload")
    ap.add_argument("--force-path", type=int, default=-1, help="0 cell lists, 1 pair lists, -1 library choice")
    ap.add_argument("--no-hybrid", action="store_true", help="skip the surrogate and hybrid-solve measurement")
    ap.add_argument("--train-points", type=int, default=256)
    ap.add_argument("--taus", type=lambda t: [float(x) for x in t.split(",")], default=[0.01, 0.05, 0.10],
                    help="relative uncertainty thresholds of the GP hybrid runs, comma separated")
    ap.add_argument("--ens-taus", type=lambda t: [float(x) for x in t.split(",")], default=[0.05],
                    help="thresholds at which the ensemble also marches")
    ap.add_argument("--rules", type=lambda t: t.split(","), default=["plain", "floor"],
                    help="threshold rules: plain (std > tau |mean|) and floor (std > max(tau |mean|, median "
                         "training SE))")
    ap.add_argument("--audit-every", type=int, default=1009,
                    help="audit every k-th surrogate answer; a k coprime with the 200 sections makes successive "
                         "audits visit different sections (k = 1000 audits one section only)")
    ap.add_argument("--hybrid-steps", type=int, default=HY_STEPS)
    ap.add_argument("--refit-every", type=int, default=1, help="ensemble retrains after this many new MD points")
    ap.add_argument("--ens-iters", type=int, default=20000,
                    help="Adam iterations of each ensemble member (5000 leaves the members short of convergence)")
    ap.add_argument("--gp-hyper", choices=("evidence", "paper"), default="evidence",
                    help="GP sigma_f and l: maximise the evidence on the training data (Sec. 2.3's procedure), or "
                         "the paper's values 1, 1")
    ap.add_argument("--all-md-steps", type=int, default=1, help="macro steps run all-MD to price the all-MD march")
    ap.add_argument("--plain-taus", type=lambda t: [float(x) for x in t.split(",")], default=[0.10],
                    help="thresholds at which the GP also runs under the plain relative rule")
    ap.add_argument("--hybrid-budget", type=float, default=40.0,
                    help="wall-clock cap (s) of one hybrid run; the speed-up is then taken over the steps done")
    ap.add_argument("--no-eos-gp", action="store_true",
                    help="skip the hybrid solve with the pressure GP and the 3-input flux GP")
    ap.add_argument("--no-finish", action="store_true",
                    help="stop after the timed steps (no flux results): for short profiled runs")
    ap.add_argument("--no-autotune", action="store_true",
                    help="skip the autotuner (by default it times its candidates on the batch, outside the timed "
                         "region, and the batch uses the fastest)")
    ap.add_argument("--tune-steps", type=int, default=200, help="probe steps per autotuner candidate")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of MIB MiB (counter calibration)")
    ap.add_argument("--summarize-pmc", default="", metavar="CSV",
                    help="only print per-dispatch counter means of --kernel from a rocprofv3 CSV")
    ap.add_argument("--kernel", default="k_force_list")
    args = ap.parse_args()
    if args.summarize_pmc:
        summarize_pmc(args.summarize_pmc, args.kernel)
        return
    if args.copy_calibration:
        copy_calibration(args.copy_calibration)
        return
    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported (independent micro-solves "
              "would shard by bin-packing systems across GPUs with no communication during MD)", file=sys.stderr)
        sys.exit(2)

    import torch  # device memory / stream plumbing only
    assert torch.cuda.is_available(), "no GPU"
    import paper_1603_04628_amd as hmd

    jobs = workloads.batch_jobs(64)
    params = hmd.Params(n_equil=N_EQUIL, skin=args.skin, force_path=args.force_path, **workloads.batch_box())
    ctx = hmd.Context(params)
    tune_table, tune_s = None, None
    if not args.no_autotune and args.force_path < 0:
        t0 = time.perf_counter()
        tune_table = hmd.md_autotune(ctx, [(j.h, j.g, j.seed, N_SAMPLE) for j in jobs], probe_steps=args.tune_steps)
        tune_s = time.perf_counter() - t0
        log(f"autotune in {tune_s:.1f} s: {tune_table.tolist()}")
    t0 = time.perf_counter()
    batch = hmd.Batch(ctx, [(j.h, j.g, j.seed, N_SAMPLE) for j in jobs])
    log(f"batch set up in {time.perf_counter() - t0:.1f} s: {batch.atoms} fluid atoms")
    ff, wf = batch.pair_count()
    pairs_per_launch = ff + wf
    plan = timed_plan(args.steps, args.warmup, args.chunk)
    log(f"timed plan: {plan}")
    names = ("integrate", "keys", "scan", "scatter", "reorder", "list", "force")
    # warm-up: capture the timed graphs (their first replays are warm-up
    # steps), then the rest of the warm-up untimed
    done = 0
    for cs in plan["chunks"]:
        batch.set_timing(True)
        batch.run(cs, graph_chunk=cs)
        done += cs
    batch.set_timing(False)
    if plan["warmup"] > done:
        advance(batch, plan["warmup"] - done, args.chunk)
        done = plan["warmup"]
    warm_steps = done
    builds = 0
    wall, windows = 0.0, []
    for phase, n_timed in (("equilibrating", plan["eq"]), ("sampling", plan["sa"])):
        if n_timed > 0:
            batch.set_timing(True)
            b0 = batch.list_builds()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            advance(batch, n_timed, plan["chunk"])
            torch.cuda.synchronize()
            wall += time.perf_counter() - t0
            nb = batch.list_builds() - b0
            builds += nb
            km = {k: batch.kernel_ms(k) for k in names + ("graph_step", "list_rebuild", "list_idle")}
            # the list build per step: its time on stamped rebuild and idle
            # steps, weighted by this stretch's exact rebuild rate (the
            # stamped steps hold too few rebuilds for a steady mean)
            rate = nb / n_timed
            if km["list_rebuild"][1] > 0 and km["list_idle"][1] > 0:
                km["list_sampled"] = km["list"]
                km["list"] = (rate * km["list_rebuild"][0] + (1.0 - rate) * km["list_idle"][0], km["list"][1])
            km["rebuilds_per_step"] = (rate, nb)
            windows.append((phase, n_timed, km))
            batch.set_timing(False)
            done += n_timed
        if phase == "equilibrating" and plan["sa"] > 0 and done < N_EQUIL:  # untimed: the rest of it
            advance(batch, N_EQUIL - done, args.chunk)
            done = N_EQUIL
    ms_step = 1e3 * wall / args.steps
    value = batch.atoms * args.steps / wall
    # per-kernel averages (ms per launch, one launch of each per step) from the
    # clock stamps around each kernel of the stamped steps in the timed graph
    # replays, weighted like the protocol: one third of the steps
    # equilibrating, two thirds sampling
    w_phase = {"equilibrating": N_EQUIL / (N_EQUIL + N_SAMPLE), "sampling": N_SAMPLE / (N_EQUIL + N_SAMPLE)}
    present = [w for w in windows if w[1] > 0]
    wsum = sum(w_phase[p] for p, _, _ in present)
    kern = {k: float(sum(w_phase[p] * km[k][0] for p, _, km in present) / wsum) for k in names}
    kern["graph_step"] = float(sum(w_phase[p] * km["graph_step"][0] for p, _, km in present) / wsum)
    kern_windows = {p: {"timed_steps": n, "launches_timed": int(km["force"][1]),
                        **{k: float(v[0]) for k, v in km.items()},
                        "stamped_rebuild_steps": int(km["list_rebuild"][1])} for p, n, km in windows}
    cfg = batch.config()
    tuning = batch.tuning()
    if done < N_EQUIL + N_SAMPLE and not args.no_finish:  # the rest of the sampling window (untimed): flux results
        advance(batch, N_EQUIL + N_SAMPLE - done, args.chunk)
    res = batch.results() if not args.no_finish else []
    log(f"batched: {value:.3e} atom-steps/s, {ms_step:.3f} ms/step, kernels {kern}")
    n_atoms = int(batch.atoms)
    batch.close()

    # plain path: the same jobs one system at a time with direct launches
    plain_atoms, plain_time = 0, 0.0
    stride = max(1, len(jobs) // max(1, args.plain_sims))
    plain_jobs = jobs[::stride][:args.plain_sims]  # spread over the batch's heights
    for j in plain_jobs:
        single = hmd.Batch(ctx, [(j.h, j.g, j.seed, N_SAMPLE)])
        single.run(50, graph_chunk=0)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        single.run(args.plain_steps, graph_chunk=0)
        torch.cuda.synchronize()
        plain_time += time.perf_counter() - t0
        plain_atoms += single.atoms * args.plain_steps
        single.close()
    plain = plain_atoms / plain_time if plain_time > 0 else None
    log(f"plain: {plain} atom-steps/s")

    # achievable device rates (outside the timed region), beside the
    # published peaks the roofline divides by
    from paper_1603_04628_amd import binding as B
    peaks = B.measure_peaks(ctx)
    log(f"achievable: {peaks}")
    force_ms = kern["force"]
    achieved = pairs_per_launch * FLOP_PER_PAIR / (force_ms * 1e-3) / 1e12
    cnt = committed_counters(FORCE_KERNELS[cfg["path"]])
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "atom-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": warm_steps,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "batched uneven NEMD channels: 64 systems, h=4+16u, g=0.001+0.049u, "
                               "57.1x57.1 sigma box, rho 0.8, T 1, rc 2.5, dt 0.005, protocol 10k+20k steps, "
                               f"FP32 forces / FP64 state and sums; timed: {plan['eq']} equilibrating + "
                               f"{plan['sa']} sampling steps as "
                               + (f"graph replays of {plan['chunk']} steps" if plan['chunk'] else "direct launches")
                               + (f" (the other equilibration steps untimed)" if plan['skip'] else ""),
                   "systems": len(jobs), "fluid_atoms": n_atoms, "graph_chunk": plan["chunk"],
                   "force_path": PATH_NAMES[cfg["path"]], "skin": cfg["skin"],
                   "threads_per_block": cfg["tpb"], "tile_alpha": tuning["tile_alpha"],
                   "cell_width": tuning["cell_width"], "whole_run_graph_chunk": tuning["graph_chunk"],
                   "tiles": tuning["tiles"],
                   "autotuned": tune_table is not None,
                   "list_builds_per_step": builds / args.steps},
        "roofline": {"bound": "alu", "achieved": achieved, "peak": PEAK_FP32, "unit": "TFLOP/s",
                     "frac": achieved / PEAK_FP32, "traffic": cnt["traffic"] if cnt else None,
                     "achievable_peak": peaks["fp32_fma_tflops"],
                     "frac_of_achievable": achieved / peaks["fp32_fma_tflops"],
                     "counter_tflops": cnt["flop"] / (force_ms * 1e-3) / 1e12 if cnt else None,
                     "kernel": FORCE_KERNELS[cfg["path"]], "avg_ms": force_ms,
                     "pairs_per_launch": pairs_per_launch, "flop_per_pair": FLOP_PER_PAIR},
        "achievable_peaks": peaks,
        "plain_atom_steps_per_s": plain,
        "batched_over_plain": value / plain if plain else None,
        "plain_sample": f"{len(plain_jobs)} systems of the batch (every {stride}th: h = "
                        f"{', '.join(f'{j.h:.1f}' for j in plain_jobs)}), one at a time, {args.plain_steps} "
                        "steps each, direct launches",
        "kernel_ms": kern,
        "kernel_ms_windows": kern_windows,
        "autotune": None if tune_table is None else {
            "seconds": tune_s, "probe_steps": args.tune_steps,
            "candidates": [dict(zip(("path", "skin", "tpb", "tile_alpha", "cell_w", "chunk", "ms_per_step"),
                                    [float(v) for v in row])) for row in tune_table]},
    }
    if res:
        st = [r["status"] for r in res]
        out["flux_status_ok"] = int(sum(1 for s in st if s == 0))
        out["flux_rel_se_median"] = float(np.median([r["flux_se"] / abs(r["flux"]) for r in res if r["flux"]]))
    if not args.no_hybrid:
        out.update(hybrid_bench(args, hmd, res))
    if not args.no_hybrid and not args.no_eos_gp:
        out["hybrid_eos_gp"] = eos_gp_bench(args, hmd)
    if not args.no_cpu:
        cb = cpu_baseline(args.cpu_seconds)
        out["cpu_baseline"] = cb
        log(f"cpu oracle: {cb['value']:.3e} atom-steps/s on {cb['cores']} threads")
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
