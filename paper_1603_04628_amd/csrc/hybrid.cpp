// hybrid.cpp -- the macro march of the hybrid scheme (paper Alg. 1): 1-D
// mass conservation over the channel sections, body force from the pressure
// gradient, flux from the surrogate (device GP or MLP ensemble) or, where the
// surrogate is too uncertain, from one batched MD launch for every such
// section; new MD results grow the surrogate's database.
//
// Host code (the section arrays are a few hundred doubles); built without
// floating-point contraction so the march rounds as written.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <string>
#include <utility>
#include <vector>

#include "hmd.h"
#include "startup.h"

struct hmd_ctx;  // opaque here

namespace {
// One recorded fallback run: its input and, with real MD, its final state.
struct Warm {
  double h, g;
  std::vector<double> x, v;
};
}  // namespace

struct hmd_hybrid {
  hmd_ctx* ctx = nullptr;
  hmd_hybrid_cfg cfg{};
  hmd_gp* gp = nullptr;
  hmd_ens* ens = nullptr;
  hmd_micro_fn micro = nullptr;
  void* micro_user = nullptr;
  hmd_micro_p_fn micro_p = nullptr;  // eos 1 replacement micro-solver
  void* micro_p_user = nullptr;
  hmd_gp* pgp = nullptr;             // eos 1: pressure GP over (h, rho)
  std::vector<std::pair<double, double>> p_db;  // eos 1: (h, rho) inputs in the pressure GP
  std::vector<double> forcing;       // geometry 1: F_ext / m per macro step, in place of the sinusoid
  double ds = 0.0;
  std::vector<double> h, rho, q, q_std, g, p, p_std;
  std::vector<uint8_t> from_md;
  int64_t step_no = 0, answers = 0, pending_refit = 0;
  uint64_t next_seed = 0;
  hmd_hybrid_stats st{};
  // audits waiting for their batch: (h, rho, |g|) and the surrogate's answer
  std::vector<double> audit_h, audit_rho, audit_g, audit_mean, audit_sd;
  // warm starts: the recorded fallback runs and the last step's plan
  std::vector<Warm> warm;
  std::vector<int> plan_prior;
  std::vector<int64_t> plan_equil;
  int64_t plan_batch_equil = 0;
};

namespace {

constexpr double kTwoPi = 6.283185307179586;

// Whether (h, rho) is among the pressure GP's inputs: both equal within a
// relative 1e-9 (section heights computed with different libraries'
// cosines can differ in the last bits).
bool p_known(const std::vector<std::pair<double, double>>& db, double h, double rho) {
  auto near = [](double a, double b) { return std::fabs(a - b) <= 1e-9 * std::fmax(std::fabs(a), std::fabs(b)); };
  for (const auto& e : db)
    if (near(e.first, h) && near(e.second, rho)) return true;
  return false;
}

using clock_t_ = std::chrono::steady_clock;

double seconds_since(clock_t_::time_point t0) {
  return std::chrono::duration<double>(clock_t_::now() - t0).count();
}

// Fluxes for the listed sections from the micro-solver (callback or batched
// MD).  Audits run from the lattice with params.n_equil; fallback runs with
// warm starts use `prior` (index into hy->warm, -1: lattice) and equilibrate
// for n_equil steps, and return their final states in xs, vs.  With eos 1
// every run takes its section's density rr[k] and also returns the wall
// pressure pm, its SE pse.
int solve_micro(hmd_hybrid* hy, std::vector<double> hh, std::vector<double> gg, std::vector<double>& qm,
                std::vector<double>& se, std::vector<int>& ok, bool audit, const std::vector<int>* prior = nullptr,
                int64_t n_equil = -1, std::vector<std::vector<double>>* xs = nullptr,
                std::vector<std::vector<double>>* vs = nullptr, const std::vector<double>* rr = nullptr,
                std::vector<double>* pm = nullptr, std::vector<double>* pse = nullptr) {
  double& wall = audit ? hy->st.audit_wall_s : hy->st.md_wall_s;
  double& atom_steps = audit ? hy->st.audit_atom_steps : hy->st.md_atom_steps;
  const int n = int(hh.size());
  const bool press = hy->cfg.eos == 1;
  qm.assign(n, 0.0);
  se.assign(n, 0.0);
  ok.assign(n, 1);
  if (pm) pm->assign(n, 0.0);
  if (pse) pse->assign(n, 0.0);
  const auto t0 = clock_t_::now();
  if (press && hy->micro_p) {
    const int rc = hy->micro_p(hy->micro_p_user, n, hh.data(), rr->data(), gg.data(), qm.data(), se.data(),
                               pm->data(), pse->data());
    wall += seconds_since(t0);
    return rc == 0 ? HMD_OK : HMD_EINVAL;
  }
  if (!press && hy->micro) {
    const int rc = hy->micro(hy->micro_user, n, hh.data(), gg.data(), qm.data(), se.data());
    wall += seconds_since(t0);
    return rc == 0 ? HMD_OK : HMD_EINVAL;
  }
  std::vector<hmd_md_job> jobs(n);
  for (int k = 0; k < n; ++k)
    jobs[k] = hmd_md_job{hh[k], gg[k], hy->next_seed++, hy->cfg.md_sample, press ? (*rr)[k] : 0.0};
  std::vector<hmd_md_result> res(n);
  hmd_md_params P;
  hmd_get_params(hy->ctx, &P);
  const int64_t cold_equil = P.n_equil;
  int rc = HMD_OK;
  if (press) {  // the runs also record the wall pressure
    hmd_md_params Q = P;
    Q.pressure = 1;
    rc = hmd_set_params(hy->ctx, &Q);
    if (rc == HMD_OK) rc = md_flux_batch(hy->ctx, jobs.data(), n, res.data());
    hmd_set_params(hy->ctx, &P);
  } else if (!prior) {
    rc = md_flux_batch(hy->ctx, jobs.data(), n, res.data());
  } else {
    // the batch's own equilibration, warm states set after creation
    hmd_md_params Q = P;
    Q.n_equil = n_equil;
    rc = hmd_set_params(hy->ctx, &Q);
    hmd_batch* b = nullptr;
    if (rc == HMD_OK) rc = md_batch_create(hy->ctx, jobs.data(), n, &b);
    hmd_set_params(hy->ctx, &P);
    if (rc == HMD_OK) {
      std::vector<int> sims;
      std::vector<const double*> px, pv;
      for (int k = 0; k < n; ++k)
        if ((*prior)[k] >= 0) {
          sims.push_back(k);
          px.push_back(hy->warm[(*prior)[k]].x.data());
          pv.push_back(hy->warm[(*prior)[k]].v.data());
        }
      rc = md_batch_set_states(b, int(sims.size()), sims.data(), px.data(), pv.data());
      if (rc == HMD_OK) rc = md_batch_run(b, n_equil + hy->cfg.md_sample, P.graph_chunk > 0 ? P.graph_chunk : 100);
      if (rc == HMD_OK) rc = md_batch_results(b, res.data());
      if (rc == HMD_OK) {
        xs->assign(n, {});
        vs->assign(n, {});
        std::vector<double*> ox(n), ov(n);
        for (int k = 0; k < n; ++k) {
          (*xs)[k].resize(3 * size_t(res[k].n_fluid));
          (*vs)[k].resize(3 * size_t(res[k].n_fluid));
          ox[k] = (*xs)[k].data();
          ov[k] = (*vs)[k].data();
        }
        rc = md_batch_get_states(b, ox.data(), ov.data());
      }
    }
    if (b) md_batch_free(b);
  }
  wall += seconds_since(t0);
  if (rc != HMD_OK) return rc;
  const int64_t equil = prior ? n_equil : cold_equil;
  for (int k = 0; k < n; ++k) {
    qm[k] = res[k].flux;
    se[k] = res[k].flux_se;
    if (pm) (*pm)[k] = res[k].p;
    if (pse) (*pse)[k] = res[k].p_se;
    ok[k] = res[k].status == HMD_OK;
    hy->st.md_failed += ok[k] || audit ? 0 : 1;
    atom_steps += double(res[k].n_fluid) * double(equil + hy->cfg.md_sample);
    if (!audit) {
      hy->st.md_equil_atom_steps += double(res[k].n_fluid) * double(equil);
      hy->st.md_atom_steps_cold += double(res[k].n_fluid) * double(cold_equil + hy->cfg.md_sample);
    }
  }
  return HMD_OK;
}

// Runs the pending audits as one batch and scores them.
int flush_audits(hmd_hybrid* hy) {
  if (hy->audit_h.empty()) return HMD_OK;
  std::vector<double> qm, se, pm, pse;
  std::vector<int> ok;
  const int rc = solve_micro(hy, hy->audit_h, hy->audit_g, qm, se, ok, true, nullptr, -1, nullptr, nullptr,
                             &hy->audit_rho, &pm, &pse);
  if (rc != HMD_OK) return rc;
  for (size_t k = 0; k < qm.size(); ++k) {
    if (!ok[k]) continue;
    hy->st.audited += 1;
    const double dev = std::fabs(hy->audit_mean[k] - qm[k]);
    hy->st.audit_pass += dev <= 2.0 * se[k] ? 1 : 0;
    hy->st.audit_pass_cal +=
        dev <= 2.0 * std::sqrt(hy->audit_sd[k] * hy->audit_sd[k] + se[k] * se[k]) ? 1 : 0;
  }
  hy->audit_h.clear();
  hy->audit_rho.clear();
  hy->audit_g.clear();
  hy->audit_mean.clear();
  hy->audit_sd.clear();
  return HMD_OK;
}

}  // namespace

extern "C" {

void hmd_hybrid_cfg_default(hmd_hybrid_cfg* c) {
  if (!c) return;
  c->n_sections = 200;
  c->h0 = 10.0;
  c->amp = 0.5;
  c->L = 2000.0;
  c->dt_macro = 0.02;
  c->rho_ref = 0.8;
  c->p_out = 0.0;
  c->dp_mean = 10.0;
  c->dp_amp = 0.3;
  c->period = 250.0;
  c->c2 = 200.0;
  c->tau_rel = 0.05;
  c->tau_abs = 0.0;
  c->surrogate = 0;
  c->audit_every = 0;
  c->md_sample = 4000;
  c->refit_every = 16;
  c->seed = 1000000;
  c->mirror = 1;
  c->audit_batch = 0;
  c->warm_start = 0;
  c->pseudo_nu = 2.5;
  c->pseudo_slip = 0.5;
  c->pseudo_tol = 0.01;
  c->n_min_warm = 1000;
  c->n_min_cold = 2000;
  c->geometry = 0;
  c->f_amp = 0.0;
  c->f_period = 250.0;
  c->eos = 0;
}

int hybrid_create(hmd_ctx* ctx, const hmd_hybrid_cfg* cfg, hmd_gp* gp, hmd_ens* ens, hmd_hybrid** out) {
  if (!ctx || !cfg || !out) return HMD_EINVAL;
  const hmd_hybrid_cfg& c = *cfg;
  if (c.n_sections < 2 || !(c.L > 0.0) || !(c.h0 > 0.0) || !(c.dt_macro > 0.0) || !(c.rho_ref > 0.0) ||
      c.tau_rel < 0.0 || c.tau_abs < 0.0 || (c.surrogate == 0 && !gp) || (c.surrogate == 1 && !ens) ||
      c.surrogate < 0 || c.surrogate > 1 || c.md_sample < 0 || c.refit_every < 1 || !(c.period > 0.0) ||
      (c.warm_start && (!(c.pseudo_nu > 0.0) || !(c.pseudo_slip >= 0.0) || !(c.pseudo_tol > 0.0) ||
                        c.n_min_warm < 0 || c.n_min_cold < 0)) ||
      c.geometry < 0 || c.geometry > 1 || (c.geometry == 1 && !(c.f_period > 0.0)) || c.eos < 0 || c.eos > 1 ||
      (c.eos == 1 && (c.surrogate != 0 || c.warm_start)))
    return HMD_EINVAL;
  auto* hy = new hmd_hybrid();
  hy->ctx = ctx;
  hy->cfg = c;
  hy->gp = gp;
  hy->ens = ens;
  hy->next_seed = c.seed;
  const int n = c.n_sections;
  hy->ds = c.L / double(n);
  hy->h.resize(n);
  for (int i = 0; i < n; ++i) {
    if (c.geometry == 1) {  // Eqs. subsEq and heightEq
      const double s = double(i) * hy->ds;
      hy->h[i] = c.amp * c.h0 * (std::cos(kTwoPi * s / c.L) - 1.0) + c.h0;
    } else {
      const double s = (double(i) + 0.5) * hy->ds;
      hy->h[i] = c.h0 * (1.0 + c.amp * std::cos(kTwoPi * s / c.L));
    }
  }
  hy->rho.assign(n, c.rho_ref);
  hy->q.assign(n, 0.0);
  hy->q_std.assign(n, 0.0);
  hy->g.assign(n, 0.0);
  hy->p.assign(n, 0.0);
  hy->p_std.assign(n, 0.0);
  hy->from_md.assign(n, 0);
  hy->plan_prior.assign(n, -2);
  hy->plan_equil.assign(n, 0);
  *out = hy;
  return HMD_OK;
}

int hybrid_set_micro(hmd_hybrid* hy, hmd_micro_fn fn, void* user) {
  if (!hy) return HMD_EINVAL;
  hy->micro = fn;
  hy->micro_user = user;
  return HMD_OK;
}

int hybrid_set_micro_p(hmd_hybrid* hy, hmd_micro_p_fn fn, void* user) {
  if (!hy) return HMD_EINVAL;
  hy->micro_p = fn;
  hy->micro_p_user = user;
  return HMD_OK;
}

int hybrid_set_pressure_gp(hmd_hybrid* hy, hmd_gp* pgp) {
  if (!hy || !pgp) return HMD_EINVAL;
  int n = 0, d = 0;
  int rc = gp_inputs(pgp, nullptr, &n, &d);
  if (rc != HMD_OK) return rc;
  if (d != 2) return HMD_EINVAL;
  std::vector<double> X(2 * size_t(n));
  rc = gp_inputs(pgp, X.data(), nullptr, nullptr);
  if (rc != HMD_OK) return rc;
  hy->pgp = pgp;
  hy->p_db.clear();
  for (int k = 0; k < n; ++k) hy->p_db.push_back({X[2 * size_t(k)], X[2 * size_t(k) + 1]});
  return HMD_OK;
}

int hybrid_set_forcing(hmd_hybrid* hy, const double* f, int64_t n) {
  if (!hy || n < 0 || (n > 0 && !f)) return HMD_EINVAL;
  if (n > 0 && hy->cfg.geometry != 1) return HMD_EINVAL;  // a table needs the periodic channel
  for (int64_t k = 0; k < n; ++k)
    if (!std::isfinite(f[k])) return HMD_EINVAL;
  hy->forcing.assign(f, f + n);
  return HMD_OK;
}

int hybrid_get_pressure(hmd_hybrid* hy, double* p, double* p_std) {
  if (!hy) return HMD_EINVAL;
  const int n = hy->cfg.n_sections;
  if (p) std::copy(hy->p.begin(), hy->p.begin() + n, p);
  if (p_std) std::copy(hy->p_std.begin(), hy->p_std.begin() + n, p_std);
  return HMD_OK;
}

int hybrid_set_rho(hmd_hybrid* hy, const double* rho) {
  if (!hy || !rho) return HMD_EINVAL;
  for (int i = 0; i < hy->cfg.n_sections; ++i)
    if (!(rho[i] > 0.0)) return HMD_EINVAL;
  hy->rho.assign(rho, rho + hy->cfg.n_sections);
  return HMD_OK;
}

int hybrid_step(hmd_hybrid* hy, hmd_hybrid_stats* out) {
  if (!hy) return HMD_EINVAL;
  const auto t0 = clock_t_::now();
  const hmd_hybrid_cfg& c = hy->cfg;
  const int n = c.n_sections;
  const bool press = c.eos == 1;
  if (press && !hy->pgp) return HMD_EINVAL;  // eos 1 needs hybrid_set_pressure_gp first
  // the march has reached the end of its forcing table
  if (!hy->forcing.empty() && hy->step_no >= int64_t(hy->forcing.size())) return HMD_EINVAL;
  // pressure (linear law, or eos 1: the pressure GP at (h, rho)),
  // central-difference gradient with ghost pressures, body force
  std::vector<double> p(n);
  if (press) {
    std::vector<double> Xp(2 * size_t(n)), pv(n);
    for (int i = 0; i < n; ++i) {
      Xp[2 * i] = hy->h[i];
      Xp[2 * i + 1] = hy->rho[i];
    }
    const auto tp = clock_t_::now();
    const int rcp = gp_predict(hy->pgp, Xp.data(), n, p.data(), pv.data());
    hy->st.surrogate_wall_s += seconds_since(tp);
    if (rcp != HMD_OK) return rcp;
    for (int i = 0; i < n; ++i) hy->p_std[i] = std::sqrt(pv[i] > 0.0 ? pv[i] : 0.0);
  } else {
    for (int i = 0; i < n; ++i) {
      p[i] = c.p_out + c.c2 * (hy->rho[i] - c.rho_ref);
      hy->p_std[i] = 0.0;
    }
  }
  hy->p = p;
  const double p_in = c.p_out + c.dp_mean * (1.0 + c.dp_amp * std::sin(kTwoPi * double(hy->step_no) / c.period));
  // Eq. extForcing1 on the periodic channel, or the step's entry of a
  // forcing table (the variable-frequency and variable-amplitude cases of
  // Sec. 3.4)
  const double f_ext = !hy->forcing.empty() ? hy->forcing[size_t(hy->step_no)]
                       : c.geometry == 1   ? c.f_amp * std::sin(kTwoPi * double(hy->step_no) / c.f_period)
                                           : 0.0;
  for (int i = 0; i < n; ++i) {
    double pl, pr;
    if (c.geometry == 1) {
      pl = p[(i + n - 1) % n];
      pr = p[(i + 1) % n];
    } else {
      pl = i > 0 ? p[i - 1] : p_in;
      pr = i < n - 1 ? p[i + 1] : c.p_out;
    }
    const double dpds = (pr - pl) / (2.0 * hy->ds);
    hy->g[i] = f_ext - dpds / hy->rho[i];
  }
  // surrogate query for every section (at |g| with the sign restored after,
  // when mirror is on)
  const int dx = press ? 3 : 2;  // flux inputs: (h, |g|), or (h, rho, |g|)
  std::vector<double> X(dx * size_t(n)), mean(n), second(n), sd(n), gq(n), sgn(n, 1.0);
  for (int i = 0; i < n; ++i) {
    const bool neg = c.mirror && hy->g[i] < 0.0;
    gq[i] = neg ? -hy->g[i] : hy->g[i];
    sgn[i] = neg ? -1.0 : 1.0;
    X[dx * i] = hy->h[i];
    if (press) X[dx * i + 1] = hy->rho[i];
    X[dx * i + dx - 1] = gq[i];
  }
  const auto ts = clock_t_::now();
  int rc = c.surrogate == 0 ? gp_predict(hy->gp, X.data(), n, mean.data(), second.data())
                            : ens_predict(hy->ens, X.data(), n, mean.data(), second.data());
  hy->st.surrogate_wall_s += seconds_since(ts);
  if (rc != HMD_OK) return rc;
  for (int i = 0; i < n; ++i) sd[i] = c.surrogate == 0 ? std::sqrt(second[i] > 0.0 ? second[i] : 0.0) : second[i];
  hy->st.queries += n;
  // threshold test and audits
  std::vector<int> run;
  std::vector<uint8_t> flag(n, 0), audit(n, 0);
  for (int i = 0; i < n; ++i) {
    const double thr = std::fmax(c.tau_rel * std::fabs(mean[i]), c.tau_abs);
    flag[i] = sd[i] > thr;
  }
  for (int i = 0; i < n; ++i)
    if (!flag[i] && c.audit_every > 0) {
      hy->answers += 1;
      if (hy->answers % c.audit_every == 0) audit[i] = 1;
    }
  for (int i = 0; i < n; ++i)
    if (flag[i] || audit[i]) run.push_back(i);
  std::vector<double> qv(n);
  for (int i = 0; i < n; ++i) qv[i] = sgn[i] * mean[i];
  std::vector<int> fl, au;
  for (int i : run) (flag[i] ? fl : au).push_back(i);
  std::fill(hy->plan_prior.begin(), hy->plan_prior.end(), -2);
  std::fill(hy->plan_equil.begin(), hy->plan_equil.end(), int64_t(0));
  hy->plan_batch_equil = 0;
  if (!fl.empty()) {
    std::vector<double> qm, se, hh, gg, rr, pm, pse;
    std::vector<int> ok, prior;
    for (int i : fl) {
      hh.push_back(hy->h[i]);
      gg.push_back(gq[i]);
      rr.push_back(hy->rho[i]);
    }
    std::vector<std::vector<double>> xs, vs;
    if (c.warm_start) {
      // nearest prior of the same height (within a relative 1e-9: mirrored
      // sections' heights can differ in the last bits): the largest
      // covariance of the inputs is the smallest distance between them;
      // ties go to the earliest
      hmd_md_params P;
      hmd_get_params(hy->ctx, &P);
      for (size_t k = 0; k < fl.size(); ++k) {
        int best = -1;
        double bd = 0.0;
        for (size_t j = 0; j < hy->warm.size(); ++j) {
          if (std::fabs(hy->warm[j].h - hh[k]) > 1e-9 * std::fmax(hy->warm[j].h, hh[k]) ||
              (!hy->micro && hy->warm[j].x.empty()))
            continue;
          const double dh = hy->warm[j].h - hh[k], dg = hy->warm[j].g - gg[k];
          const double d = dh * dh + dg * dg;  // squared distance of the inputs (unit scales)
          if (best < 0 || d < bd) {
            best = int(j);
            bd = d;
          }
        }
        const double g_in = best >= 0 ? hy->warm[best].g : 0.0;
        const double ts = hmd::startup_time(hh[k], g_in, gg[k], c.pseudo_nu, c.pseudo_slip, c.pseudo_tol);
        const int64_t ne = hmd::startup_steps(ts, P.dt, best >= 0 ? c.n_min_warm : c.n_min_cold);
        prior.push_back(best);
        hy->plan_prior[fl[k]] = best;
        hy->plan_equil[fl[k]] = ne;
        hy->plan_batch_equil = std::max(hy->plan_batch_equil, ne);
        hy->st.warm_starts += best >= 0 ? 1 : 0;
      }
    }
    rc = c.warm_start ? solve_micro(hy, hh, gg, qm, se, ok, false, &prior, hy->plan_batch_equil, &xs, &vs)
                      : solve_micro(hy, hh, gg, qm, se, ok, false, nullptr, -1, nullptr, nullptr, &rr, &pm, &pse);
    if (rc != HMD_OK) return rc;
    hy->st.md_calls += int64_t(fl.size());
    for (size_t k = 0; k < fl.size(); ++k) qv[fl[k]] = sgn[fl[k]] * qm[k];
    // database growth (runs that failed to converge are left out, Sec. 3.2);
    // with warm starts each converged run is recorded with its final state
    const auto tg = clock_t_::now();
    for (size_t k = 0; k < fl.size(); ++k) {
      const int i = fl[k];
      if (!ok[k]) continue;
      const double x[3] = {hy->h[i], press ? hy->rho[i] : gq[i], gq[i]};
      if (c.surrogate == 0) {
        rc = gp_append(hy->gp, x, qm[k], se[k]);
        // Alg. 1: the run's pressure joins the pressure GP when its
        // (h, rho) is not there yet
        if (rc == HMD_OK && press && !p_known(hy->p_db, hy->h[i], hy->rho[i])) {
          hy->p_db.push_back({hy->h[i], hy->rho[i]});
          const double xp[2] = {hy->h[i], hy->rho[i]};
          rc = gp_append(hy->pgp, xp, pm[k], pse[k]);
          hy->st.p_appends += 1;
        }
      } else {
        rc = ens_append(hy->ens, x, qm[k]);
        hy->pending_refit += 1;
      }
      if (rc != HMD_OK) return rc;
      if (c.warm_start) {
        Warm w{hh[k], gg[k], {}, {}};
        if (!xs.empty()) {
          w.x.swap(xs[k]);
          w.v.swap(vs[k]);
        }
        hy->warm.push_back(std::move(w));
      }
    }
    if (c.surrogate == 1 && hy->pending_refit >= c.refit_every) {
      rc = ens_refit(hy->ens);
      if (rc != HMD_OK) return rc;
      hy->pending_refit = 0;
    }
    hy->st.surrogate_wall_s += seconds_since(tg);
  }
  // audits do not feed back into the march: they wait and run as batches of
  // their own (audit_batch at a time, 0: at once), timed apart from the method
  for (int i : au) {
    hy->audit_h.push_back(hy->h[i]);
    hy->audit_rho.push_back(hy->rho[i]);
    hy->audit_g.push_back(gq[i]);
    hy->audit_mean.push_back(mean[i]);
    hy->audit_sd.push_back(sd[i]);
  }
  if (!hy->audit_h.empty() && int(hy->audit_h.size()) >= std::max(c.audit_batch, 1)) {
    rc = flush_audits(hy);
    if (rc != HMD_OK) return rc;
  }
  // conservative update of rho h
  std::vector<double> flux(n + 1);
  for (int i = 0; i + 1 < n; ++i) flux[i + 1] = 0.5 * (qv[i] + qv[i + 1]);
  if (c.geometry == 1) {  // the face between the last and first section closes the ring
    flux[n] = 0.5 * (qv[n - 1] + qv[0]);
    flux[0] = flux[n];
  } else {
    flux[0] = qv[0];
    flux[n] = qv[n - 1];
  }
  for (int i = 0; i < n; ++i) {
    const double m = hy->rho[i] * hy->h[i] - c.dt_macro * (flux[i + 1] - flux[i]) / hy->ds;
    hy->rho[i] = m / hy->h[i];
  }
  hy->q = qv;
  hy->q_std = sd;
  hy->from_md = flag;
  hy->step_no += 1;
  hy->st.steps = hy->step_no;
  hy->st.wall_s += seconds_since(t0);
  if (out) *out = hy->st;
  return HMD_OK;
}

int hybrid_get(hmd_hybrid* hy, double* rho, double* q, double* q_std, double* g, uint8_t* from_md) {
  if (!hy) return HMD_EINVAL;
  const size_t n = size_t(hy->cfg.n_sections);
  if (rho) std::memcpy(rho, hy->rho.data(), 8 * n);
  if (q) std::memcpy(q, hy->q.data(), 8 * n);
  if (q_std) std::memcpy(q_std, hy->q_std.data(), 8 * n);
  if (g) std::memcpy(g, hy->g.data(), 8 * n);
  if (from_md) std::memcpy(from_md, hy->from_md.data(), n);
  return HMD_OK;
}

int hybrid_last_plan(hmd_hybrid* hy, int* prior, int64_t* n_equil, int64_t* batch_equil) {
  if (!hy) return HMD_EINVAL;
  const size_t n = size_t(hy->cfg.n_sections);
  if (prior) std::memcpy(prior, hy->plan_prior.data(), sizeof(int) * n);
  if (n_equil) std::memcpy(n_equil, hy->plan_equil.data(), sizeof(int64_t) * n);
  if (batch_equil) *batch_equil = hy->plan_batch_equil;
  return HMD_OK;
}

int hybrid_flush_audits(hmd_hybrid* hy, hmd_hybrid_stats* out) {
  if (!hy) return HMD_EINVAL;
  const auto t0 = clock_t_::now();
  const int rc = flush_audits(hy);
  hy->st.wall_s += seconds_since(t0);
  if (out) *out = hy->st;
  return rc;
}

void hybrid_free(hmd_hybrid* hy) { delete hy; }

}  // extern "C"
