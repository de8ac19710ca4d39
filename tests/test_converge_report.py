"""The convergence scorer (tests/converge_report.py) on synthetic input:
exact ln g scores zero, a known offset scores that offset (CPU)."""
import numpy as np

from oracle import exact_dos as X
from tests import converge_report
from tests.test_oracle_exact import load_ising_table


def test_exact_input_scores_zero_and_offsets_are_seen(tmp_path):
    exact = X.ln_g(load_ising_table(8))
    bumped = exact.copy()
    fin = np.isfinite(exact)
    k = np.nonzero(fin)[0][5]
    bumped[k] += 0.03
    f = tmp_path / "run.npz"
    np.savez(f, config="ising8", model=0, L=8, q=2,
             fp64_instances=np.array([0, 1]), fp64_lng=np.array([exact, bumped]),
             fp64_jk_err=np.array([np.zeros_like(exact), np.zeros_like(exact)]))
    r = converge_report.report(str(f))["runs"]["fp64"]
    assert r["max_abs_err_vs_exact"][0] == 0.0
    assert abs(r["max_abs_err_vs_exact"][1] - 0.03) < 1e-12
    assert r["jackknife_err_median"] == 0.0
