"""Host logic of the significance threshold (gmgm_significance_threshold, no
device work) against the oracle: Theorem 3's statistic with the normal
quantile taken from scipy, and the library's argument checks."""
import numpy as np
import pytest

from oracle import significance as SG
from tests import _libs


@pytest.fixture(scope="module")
def g():
    _libs.ensure_built()
    import paper_2407_19892_amd as pkg
    pkg.load()
    return pkg


@pytest.mark.parametrize("d_l,d_all,trace_s,alpha,m", [
    (1000, [2e7], [3e7], 0.05, None),                        # one modality, default Bonferroni count
    (20000, [2e10, 5e10], [1e9, 3e10], 0.01, None),          # an axis shared by two modalities
    (50, [5e6], [7e5], 0.2, 10.0),                           # explicit test count
    (1_000_000, [2e10, 5e10], [4e9, 1e9], 0.05, None),       # million-cell axis: p ~ 5e-14
    (2, [4.0], [4.0], 0.5, 1.0),                             # smallest axis, p = 0.25
])
def test_threshold_matches_oracle(g, d_l, d_all, trace_s, alpha, m):
    got = g.significance_threshold(d_l, d_all, trace_s, alpha, m or 0.0)
    want = SG.significance_threshold(d_l, d_all, trace_s, alpha, m)
    assert abs(got - want) <= 1e-12 * want


@pytest.mark.parametrize("args", [
    (1, [1.0], [1.0], 0.05),        # axis too small
    (10, [1.0], [0.0], 0.05),       # zero variance
    (10, [1.0], [1.0], 0.0),        # alpha out of range
    (10, [1.0], [1.0], 1.0),
    (10, [-1.0], [1.0], 0.05),
    (10, [1.0], [float("nan")], 0.05),
])
def test_threshold_rejects_bad_arguments(g, args):
    with pytest.raises(g.GmgmError):
        g.significance_threshold(*args)
