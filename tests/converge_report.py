"""Scores the ln g saved by ``bench.py --converge --save FILE`` against exact
results (CPU).

Ising: the exact density of states of the periodic L x L lattice (the golden
tables under tests/golden, written from the oracle's exact routines); the
error of an instance is max_E |ln g(E) - ln g_exact(E)| after the sum rule
sum g = 2^N.  Potts: the sum rule sum g = q^N (normalisation is g(E_min) =
q) and the exact counts of the lowest excitations.  Where jackknife errors
were saved, the report also gives their size next to the true error.

    python -m tests.converge_report FILE.npz
"""
import json
import sys

import numpy as np

from oracle import exact_dos
from tests.test_oracle_exact import load_ising_table


def report(path):
    z = np.load(path, allow_pickle=False)
    model, L, q = int(z["model"]), int(z["L"]), int(z["q"])
    N = L * L
    out = {"file": path, "config": str(z["config"]), "runs": {}}
    for tag in ("fp64", "fp32c"):
        if f"{tag}_lng" not in z:
            continue
        lng = z[f"{tag}_lng"]
        jk = z[f"{tag}_jk_err"] if f"{tag}_jk_err" in z else None
        r = {"instances": int(len(lng))}
        if model == 0:
            exact = exact_dos.ln_g(load_ising_table(L))
            fin = np.isfinite(exact)
            errs = np.array([np.max(np.abs(v[fin] - exact[fin])) for v in lng])
            r.update({"max_abs_err_vs_exact": [float(e) for e in errs],
                      "median_max_abs_err": float(np.median(errs)),
                      "rms_err_per_bin": float(np.sqrt(np.mean((lng[:, fin] - exact[fin]) ** 2)))})
            if len(lng) > 1:
                # spread between instances: the statistical error per bin
                r["instance_std_per_bin_median"] = float(np.median(lng[:, fin].std(0, ddof=1)))
        else:
            low = exact_dos.potts_low_energy(q, L)
            sums, lows = [], []
            for v in lng:
                fin = np.isfinite(v)
                mx = np.max(v[fin])
                sums.append(float(mx + np.log(np.sum(np.exp(v[fin] - mx))) - N * np.log(q)))
                lows.append(float(max(abs(v[j] - np.log(c)) for j, c in low.items() if c)))
            r.update({"lse_minus_N_ln_q": sums, "max_abs_err_low_energy_counts": lows})
        if jk is not None:
            pos = jk[jk > 0]
            r["jackknife_err_median"] = float(np.median(pos)) if pos.size else 0.0
            r["jackknife_err_max"] = float(jk.max())
        out["runs"][tag] = r
    return out


if __name__ == "__main__":
    print(json.dumps(report(sys.argv[1])))
