"""Write tests/golden/flux_batch_box.txt: oracle mass flow rates of two
channels of the 64-channel batch at its own protocol, for the statistical
flux-parity test.

Only the CPU oracle runs here (oracle/, FP64).  Each case is one (h, g) of the
batch (workloads.batch_jobs: job 5, h = 4.53, and job 8, h = 9.87), density
0.8 in the 57.15 x 57.15 sigma box, 10,000 equilibration + 20,000 sampling
steps, one independent run per seed.  Per run the file holds the mean flux
q' = sum(m v_x) / (Lx Lz) over the sampled steps (Sec. 2.1), its standard
error by Geyer's initial monotone sequence estimator over the per-step series
(Sec. 2.3: from the raw time-instantaneous data), the thermostatted
temperature and the status.

    python tests/golden/make_flux_golden.py [seeds_per_case]
"""
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import workloads  # noqa: E402
from oracle import md  # noqa: E402

N_EQUIL, N_SAMPLE = 10000, 20000
CASES = (5, 8)           # jobs of the batch
FIRST_SEED = 1000        # oracle seeds; the GPU test draws its own
OUT = os.path.join(HERE, "flux_batch_box.txt")


def main():
    nseeds = int(sys.argv[1]) if len(sys.argv) > 1 else 8
    jobs = workloads.batch_jobs(64)
    rows = []
    for c in CASES:
        j = jobs[c]
        for s in range(FIRST_SEED, FIRST_SEED + nseeds):
            t0 = time.time()
            p = md.Params(n_equil=N_EQUIL, **workloads.batch_box())
            r = md.md_flux(j.h, j.g, s, N_SAMPLE, p)
            rows.append((c, j.h, j.g, s, r["n_fluid"], r["flux"], r["flux_se"], r["T"][1], r["status"]))
            print(f"job {c} h={j.h:.4f} g={j.g:.5f} seed {s}: flux {r['flux']:.6f} +- {r['flux_se']:.6f} "
                  f"T_y {r['T'][1]:.4f} status {r['status']} ({time.time() - t0:.0f} s)", flush=True)
    with open(OUT, "w") as fh:
        fh.write("# oracle (FP64 CPU) mass flow rate per unit span, written by make_flux_golden.py\n")
        fh.write(f"# density 0.8, 57.146 sigma box, {N_EQUIL} + {N_SAMPLE} steps, dt 0.005, rc 2.5, T 1 (Berendsen "
                 "on v_y); SE: Geyer initial monotone sequence over the per-step series\n")
        fh.write("# job h g seed n_fluid flux flux_se T_y status\n")
        for row in rows:
            fh.write("%d %.17g %.17g %d %d %.17g %.17g %.17g %d\n" % row)
    print("wrote", OUT)


if __name__ == "__main__":
    main()
