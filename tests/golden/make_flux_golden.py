"""Write the oracle mass flow rates that the statistical flux-parity tests
compare with, one file per set of channels:

* ``batch_box`` -> flux_batch_box.txt: two channels of the 64-channel batch
  (workloads.batch_jobs: job 5, h = 4.53, and job 8, h = 9.87), density 0.8 in
  the 57.15 x 57.15 sigma box, 10,000 equilibration + 20,000 sampling steps.
* ``small_long`` -> flux_small_long.txt: the 2,048-atom channel (h = 6,
  g = 0.02, 20.64 sigma box) at a long protocol, 10,000 + 40,000 steps.
* ``paper_scale`` -> flux_paper_scale.txt: the 39,189-atom channel (h = 15,
  g = 0.001 + 0.049 u, 57.15 sigma box), 20,000 + 50,000 steps.

Only the CPU oracle runs here (oracle/, FP64), one independent run per seed.
Per run a file holds the mean flux q' = sum(m v_x) / (Lx Lz) over the sampled
steps (Sec. 2.1), its standard error by Geyer's initial monotone sequence
estimator over the per-step series (Sec. 2.3: from the raw time-instantaneous
data), the thermostatted temperature and the status.

    python tests/golden/make_flux_golden.py [set] [seeds_per_case]
"""
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import workloads  # noqa: E402
from oracle import md  # noqa: E402

FIRST_SEED = 1000        # oracle seeds; the GPU tests draw their own


def _batch_box():
    jobs = workloads.batch_jobs(64)
    return [(c, jobs[c].h, jobs[c].g) for c in (5, 8)], workloads.batch_box(), 10000, 20000


def _small_long():
    box, job, _ = workloads.small_channel()
    return [(0, job.h, job.g)], box, 10000, 40000


def _paper_scale():
    box, job, (n_equil, n_sample) = workloads.paper_scale_channel()
    return [(0, job.h, job.g)], box, n_equil, n_sample


# set name -> (output file, cases, default seeds per case, header description)
SETS = {
    "batch_box": ("flux_batch_box.txt", _batch_box, 8, "density 0.8, 57.146 sigma box"),
    "small_long": ("flux_small_long.txt", _small_long, 16, "2,048 fluid atoms, 20.636 sigma box"),
    "paper_scale": ("flux_paper_scale.txt", _paper_scale, 6, "density 0.8, 57.146 sigma box"),
}


def main():
    name = sys.argv[1] if len(sys.argv) > 1 else "batch_box"
    fname, cases_of, nseeds, desc = SETS[name]
    nseeds = int(sys.argv[2]) if len(sys.argv) > 2 else nseeds
    cases, box, n_equil, n_sample = cases_of()
    out = os.path.join(HERE, fname)
    # finished runs are kept in out + ".partial" (one row per line, the final
    # file's format) so that an interrupted set resumes where it stopped
    partial = out + ".partial"
    done = {}
    if os.path.exists(partial):
        with open(partial) as fh:
            for line in fh:
                f = line.split()
                if len(f) == 9:
                    done[(int(f[0]), int(f[3]))] = (int(f[0]), float(f[1]), float(f[2]), int(f[3]), int(f[4]),
                                                    float(f[5]), float(f[6]), float(f[7]), int(f[8]))
    rows = []
    for c, h, g in cases:
        for s in range(FIRST_SEED, FIRST_SEED + nseeds):
            if (c, s) in done and done[(c, s)][1:3] == (h, g):
                rows.append(done[(c, s)])
                continue
            t0 = time.time()
            p = md.Params(n_equil=n_equil, **box)
            r = md.md_flux(h, g, s, n_sample, p)
            row = (c, h, g, s, r["n_fluid"], r["flux"], r["flux_se"], r["T"][1], r["status"])
            rows.append(row)
            with open(partial, "a") as fh:
                fh.write("%d %.17g %.17g %d %d %.17g %.17g %.17g %d\n" % row)
            print(f"job {c} h={h:.4f} g={g:.5f} seed {s}: flux {r['flux']:.6f} +- {r['flux_se']:.6f} "
                  f"T_y {r['T'][1]:.4f} status {r['status']} ({time.time() - t0:.0f} s)", flush=True)
    with open(out, "w") as fh:
        fh.write("# oracle (FP64 CPU) mass flow rate per unit span, written by make_flux_golden.py\n")
        fh.write(f"# {desc}, {n_equil} + {n_sample} steps, dt 0.005, rc 2.5, T 1 (Berendsen "
                 "on v_y); SE: Geyer initial monotone sequence over the per-step series\n")
        fh.write("# job h g seed n_fluid flux flux_se T_y status\n")
        for row in rows:
            fh.write("%d %.17g %.17g %d %d %.17g %.17g %.17g %d\n" % row)
    if os.path.exists(partial):
        os.remove(partial)
    print("wrote", out)


if __name__ == "__main__":
    main()
