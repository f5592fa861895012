"""Mass-flux parity at the batch's own configuration (density 0.8, 57.15 x
57.15 sigma box, 10,000 equilibration + 20,000 sampling steps, body forces in
the batch's range): GPU runs against oracle runs of the same two channels of
the batch (h = 4.53, g = 0.0165 and h = 9.87, g = 0.0256).

The oracle values are tests/golden/flux_batch_box.txt, written by
tests/golden/make_flux_golden.py (oracle only, seeds 1000..1007).  The GPU
runs its own seeds (2000..2063) in one batch.  The two sides are independent
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

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "flux_batch_box.txt")
N_EQUIL, N_SAMPLE = 10000, 20000
GPU_SEEDS = range(2000, 2064)


def _golden():
    rows = {}
    with open(GOLDEN) as fh:
        for line in fh:
            if line.startswith("#") or not line.strip():
                continue
            job, h, g, seed, nf, flux, se, ty, st = line.split()
            rows.setdefault(int(job), []).append((float(h), float(g), int(seed), int(nf), float(flux), float(se),
                                                  float(ty), int(st)))
    return rows


def test_flux_matches_oracle_in_the_batch_box():
    gold = _golden()
    assert sorted(gold) == [5, 8]
    jobs = workloads.batch_jobs(64)
    ctx = hmd.Context(hmd.Params(n_equil=N_EQUIL, skin=0.35, **workloads.batch_box()))
    cases = sorted(gold)
    batch = [(jobs[c].h, jobs[c].g, s, N_SAMPLE) for c in cases for s in GPU_SEEDS]
    res = hmd.md_flux_batch(ctx, batch)
    n = len(GPU_SEEDS)
    for k, c in enumerate(cases):
        rows = gold[c]
        h, g = rows[0][0], rows[0][1]
        assert (h, g) == (jobs[c].h, jobs[c].g)
        assert all(r[7] == 0 for r in rows)
        r_g = res[k * n:(k + 1) * n]
        assert all(r["status"] == 0 for r in r_g), c
        assert all(r["n_fluid"] == rows[0][3] for r in r_g)
        fg = np.array([r["flux"] for r in r_g])
        fo = np.array([r[4] for r in rows])
        se_g = fg.std(ddof=1) / np.sqrt(len(fg))
        se_o = fo.std(ddof=1) / np.sqrt(len(fo))
        z = (fg.mean() - fo.mean()) / np.sqrt(se_g ** 2 + se_o ** 2)
        print(f"job {c}: h={h:.3f} g={g:.4f} gpu {fg.mean():.6f} +- {se_g:.6f} ({n} runs), oracle "
              f"{fo.mean():.6f} +- {se_o:.6f} ({len(fo)} runs), z = {z:.2f}; mean run SE gpu "
              f"{np.mean([r['flux_se'] for r in r_g]):.6f} oracle {np.mean([r[5] for r in rows]):.6f}")
        assert abs(z) <= 2.0, (c, z)
        # the thermostatted component holds T0 on both sides
        assert np.mean([r["T"][1] for r in r_g]) == pytest.approx(np.mean([r[6] for r in rows]), abs=0.005)
