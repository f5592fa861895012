"""Mass-flux parity against oracle runs at three configurations:

* the batch's own (density 0.8, 57.15 x 57.15 sigma box, 10,000 equilibration
  + 20,000 sampling steps): two channels of the batch (h = 4.53, g = 0.0165
  and h = 9.87, g = 0.0256);
* the 2,048-atom channel (h = 6, g = 0.02) at a long protocol, 10,000 +
  40,000 steps;
* the 39,189-atom channel (h = 15, g = 0.0288), 20,000 + 50,000 steps.

The oracle values are tests/golden/flux_*.txt, written by
tests/golden/make_flux_golden.py (oracle only, seeds from 1000).  The GPU runs
its own seeds (from 2000) in one batch.  The two sides are independent
estimates of the same mean flux, so the bar is |mean_gpu - mean_oracle| <=
2 sqrt(se_gpu^2 + se_oracle^2), each standard error taken from the
seed-to-seed spread of that side's runs (independent runs; a run's own
time-series error can misjudge a flux that oscillates or relaxes slowly).
"""
import os

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

hmd = pytest.importorskip("paper_1603_04628_amd")
import workloads  # noqa: E402

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _golden(name):
    rows = {}
    with open(os.path.join(GOLDEN, name)) as fh:
        for line in fh:
            if line.startswith("#") or not line.strip():
                continue
            job, h, g, seed, nf, flux, se, ty, st = line.split()
            rows.setdefault(int(job), []).append((float(h), float(g), int(seed), int(nf), float(flux), float(se),
                                                  float(ty), int(st)))
    return rows


def _compare(gold, cases, params, n_sample, gpu_seeds):
    """cases: job number -> (h, g) of the golden rows; runs every case with
    every GPU seed in one batch and applies the 2-standard-error bar."""
    assert sorted(gold) == sorted(cases)
    order = sorted(cases)
    for c in order:
        assert all((r[0], r[1]) == cases[c] for r in gold[c])
        assert all(r[7] == 0 for r in gold[c])
    ctx = hmd.Context(params)
    res = hmd.md_flux_batch(ctx, [(*cases[c], s, n_sample) for c in order for s in gpu_seeds])
    n = len(gpu_seeds)
    for k, c in enumerate(order):
        rows = gold[c]
        h, g = cases[c]
        r_g = res[k * n:(k + 1) * n]
        assert all(r["status"] == 0 for r in r_g), c
        assert all(r["n_fluid"] == rows[0][3] for r in r_g)
        fg = np.array([r["flux"] for r in r_g])
        fo = np.array([r[4] for r in rows])
        se_g = fg.std(ddof=1) / np.sqrt(len(fg))
        se_o = fo.std(ddof=1) / np.sqrt(len(fo))
        z = (fg.mean() - fo.mean()) / np.sqrt(se_g ** 2 + se_o ** 2)
        print(f"job {c}: h={h:.3f} g={g:.4f} n_fluid {rows[0][3]}: gpu {fg.mean():.6f} +- {se_g:.6f} ({n} runs), "
              f"oracle {fo.mean():.6f} +- {se_o:.6f} ({len(fo)} runs), z = {z:.2f}; mean run SE gpu "
              f"{np.mean([r['flux_se'] for r in r_g]):.6f} oracle {np.mean([r[5] for r in rows]):.6f}")
        assert abs(z) <= 2.0, (c, z)
        # the thermostatted component holds T0 on both sides
        assert np.mean([r["T"][1] for r in r_g]) == pytest.approx(np.mean([r[6] for r in rows]), abs=0.005)


def test_flux_matches_oracle_in_the_batch_box():
    jobs = workloads.batch_jobs(64)
    _compare(_golden("flux_batch_box.txt"), {c: (jobs[c].h, jobs[c].g) for c in (5, 8)},
             hmd.Params(n_equil=10000, skin=0.35, **workloads.batch_box()), 20000, range(2000, 2064))


def test_flux_matches_oracle_small_channel_long_protocol():
    box, job, _ = workloads.small_channel()
    _compare(_golden("flux_small_long.txt"), {0: (job.h, job.g)}, hmd.Params(n_equil=10000, **box), 40000,
             range(2000, 2064))


def test_flux_matches_oracle_paper_scale_channel():
    box, job, (n_equil, n_sample) = workloads.paper_scale_channel()
    _compare(_golden("flux_paper_scale.txt"), {0: (job.h, job.g)}, hmd.Params(n_equil=n_equil, **box), n_sample,
             range(2000, 2032))
