"""The library's grid stretching (host code behind the C ABI) against the
oracle: same nodes to 1e-13 of the axis length and the same number of
sweeps, for one to three transition zones; bad arguments are refused.  Runs
without a GPU: the routine does no device work."""
import numpy as np
import pytest

from oracle import gridgen

CASES = [
    (-0.75, 0.75, 96, (1.0, 8.0, 1.0), ((-0.3, -0.2), (0.2, 0.3))),          # bow and stern clusters
    (-0.25, 0.25, 64, (8.0, 1.0), ((0.02, 0.1),)),                          # centre-line cluster
    (-0.5, 0.25, 80, (1.0, 6.0, 6.0, 1.0), ((-0.2, -0.05), (-0.05, 0.0), (0.0, 0.12))),
    (0.0, 1.0, 1, (2.0,), ()),
    (0.0, 1.0, 7, (1.0, 3.0), ((-1.0, 2.0),)),                               # zone wider than the axis
]


@pytest.mark.parametrize("a,b,n,levels,zones", CASES)
def test_stretching_matches_the_oracle(a, b, n, levels, zones):
    from paper_1410_1937_amd import nfa
    ref, it_ref = gridgen.stretch(a, b, n, levels, zones)
    got, it = nfa.stretch_axis(a, b, n, levels, zones)
    assert np.max(np.abs(got - ref)) <= 1e-13 * (b - a)
    assert abs(it - it_ref) <= 1
    assert got[0] == a and got[-1] == b and np.all(np.diff(got) > 0)


def test_bad_arguments_are_refused():
    from paper_1410_1937_amd import nfa
    with pytest.raises(nfa.NFAError, match="levels"):
        nfa.stretch_axis(0.0, 1.0, 8, (1.0, -2.0), ((0.2, 0.4),))
    with pytest.raises(nfa.NFAError, match="zones"):
        nfa.stretch_axis(0.0, 1.0, 8, (1.0, 2.0, 1.0), ((0.2, 0.6), (0.5, 0.8)))
    with pytest.raises(nfa.NFAError, match="a < b"):
        nfa.stretch_axis(1.0, 0.0, 8, (1.0,), ())
    with pytest.raises(nfa.NFAError, match="converge"):
        nfa.stretch_axis(0.0, 1.0, 64, (1.0, 50.0), ((0.4, 0.45),), max_iter=2)
