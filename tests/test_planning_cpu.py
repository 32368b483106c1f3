"""Plan decisions of the planning workload (host logic, no GPU): push-down
of a build-side selection below tau on a large enough table (Section 2.1),
the smaller filtered build relation joined first (Section 2.2), and plan
agreement with join-order ties (both build relations kept at most tie_sel
of their rows: either order costs the same)."""
from paper_1901_01488_amd import planning

G = planning.GateConfig(tau=0.05, min_rows=1_000_000, beta=1.5, tie_sel=1e-3)


def test_decide():
    # R: 10M rows at 1 % -> pushed; S: 100M rows at 10 % -> not pushed
    push_r, push_s, r_first = planning.decide(0.01, 0.10, 10**7, 10**8, G)
    assert (push_r, push_s, r_first) == (True, False, True)
    # a table below min_rows is never pushed down, however selective
    assert planning.decide(0.001, 0.5, 10**5, 10**8, G)[0] is False
    # the boundary: exactly tau is not below tau
    assert planning.decide(0.05, 0.5, 10**7, 10**8, G)[0] is False
    # join order by filtered size: 10M * 0.5 = 5M against 100M * 0.01 = 1M
    assert planning.decide(0.5, 0.01, 10**7, 10**8, G)[2] is False
    # equal filtered sizes: R first
    assert planning.decide(0.1, 0.01, 10**7, 10**8, G)[2] is True


def test_agree_with_ties():
    exact = planning.decide(1e-4, 2e-5, 10**7, 10**8, G)        # both tiny: a tied order
    other = (exact[0], exact[1], not exact[2])
    assert planning.agree(exact, other, (1e-4, 2e-5), G)
    strict = planning.GateConfig(tau=0.05, min_rows=1_000_000, beta=1.5, tie_sel=0.0)
    assert not planning.agree(exact, other, (1e-4, 2e-5), strict)
    # above tie_sel the order counts
    exact2 = planning.decide(0.02, 0.001, 10**7, 10**8, G)
    flipped = (exact2[0], exact2[1], not exact2[2])
    assert not planning.agree(exact2, flipped, (0.02, 0.001), G)
    # a push-down decision that differs never agrees, tie or not
    assert not planning.agree(exact, (not exact[0], exact[1], exact[2]), (1e-4, 2e-5), G)


def test_plans_of_a_selectivity_array():
    import numpy as np
    sel = np.array([[0.01, 0.1, 0.5], [0.5, 0.001, 0.2]])
    ps = planning.plans(sel, [10**7, 10**8, 10**9], G)
    assert ps == [planning.decide(0.01, 0.1, 10**7, 10**8, G), planning.decide(0.5, 0.001, 10**7, 10**8, G)]
