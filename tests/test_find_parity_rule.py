"""The finder parity rule of the GPU tests, checked on the CPU with a planted
difference: the oracle stands in for the GPU with its chi2 cut moved by 0.5 (a
mistake planted in a copy of the oracle's call, never in the library).  Where the
flagging tolerance covers that shift, every seed whose candidates differ must first
part at a layer the reference oracle flags; where it does not, the rule must report
unexplained differences (a rule that accepted a flag on any layer would pass most of
them)."""
import numpy as np
import pytest

import oracle
import synth
import test_gpu_find as rule


def _planted(geom, ev, keep=6, max_miss=3, chi2_cut=30.0, nsigma=3.0, refit=False, graph=False, material=None,
             field=None):
    r = oracle.find(geom, ev, keep=keep, max_miss=max_miss, chi2_cut=chi2_cut - 0.5, nsigma=nsigma)
    return {k: (v.astype(np.float32) if v.dtype == np.float64 else v) for k, v in r.items()}


@pytest.mark.parametrize("tol,covers", [(0.6, True), (0.3, False)])
def test_first_divergence_rule(oracle_lib, monkeypatch, tol, covers):
    monkeypatch.setattr(rule, "run_gpu", _planted)
    monkeypatch.setattr(rule, "TOL_CHI2", tol)
    geom, ev = synth.find_workload(3, n_tracks=600)
    g = _planted(geom, ev, chi2_cut=8.0)
    r = rule.oracle_find(geom, ev, chi2_cut=8.0)
    if covers:
        st = rule.compare(geom, ev, g, r, f"planted cut shift, flag tolerance {tol}", chi2_cut=8.0)
        assert st["ambiguous"] > 20            # the planted shift does change candidates
    else:
        with pytest.raises(AssertionError, match="first divergent layer"):
            rule.compare(geom, ev, g, r, f"planted cut shift, flag tolerance {tol}", chi2_cut=8.0)
