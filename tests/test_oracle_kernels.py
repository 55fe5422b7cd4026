"""Pins of the oracle's delta kernels (cited Roma 1999 3-point, Peskin 2002 4-point).

The moment conditions below determine each kernel uniquely (that is how both
were constructed): support, partition of unity (with the even/odd split for
the 4-point kernel), vanishing first moment and a constant sum of squares.
A kernel that passes all of them is the published one.
"""
import numpy as np
import pytest

SUPPORT = {3: 1.5, 4: 2.0}
SUMSQ = {3: 0.5, 4: 0.375}


def _shifts(P):
    return np.arange(-4, 5)


@pytest.mark.parametrize("P", [3, 4])
def test_partition_of_unity_and_first_moment(oracle_mod, P):
    rng = np.random.default_rng(1)
    for r in np.concatenate([rng.uniform(-1, 1, 200), [0.0, 0.5, -0.5, 0.25, 1.0]]):
        j = _shifts(P)
        w = oracle_mod.phi(P, r - j)
        assert abs(w.sum() - 1.0) <= 4.5e-16 * 4
        assert abs(((r - j) * w).sum()) <= 4.5e-16 * 8
        assert abs((w * w).sum() - SUMSQ[P]) <= 1e-15


def test_four_point_even_odd_sums(oracle_mod):
    rng = np.random.default_rng(2)
    for r in rng.uniform(-1, 1, 100):
        j = _shifts(4)
        w = oracle_mod.phi(4, r - j)
        assert abs(w[j % 2 == 0].sum() - 0.5) <= 1e-15
        assert abs(w[j % 2 != 0].sum() - 0.5) <= 1e-15


@pytest.mark.parametrize("P", [3, 4])
def test_support_and_symmetry(oracle_mod, P):
    r = np.linspace(-3, 3, 601)
    w = oracle_mod.phi(P, r)
    assert np.all(w[np.abs(r) >= SUPPORT[P]] == 0.0)
    assert np.all(w[np.abs(r) < SUPPORT[P]] > 0.0)
    assert np.array_equal(w, oracle_mod.phi(P, -r))


def test_spot_values(oracle_mod):
    v3 = oracle_mod.phi(3, [0.0, 0.5, 1.0, 1.5])
    assert np.allclose(v3, [2 / 3, 0.5, 1 / 6, 0.0], atol=1e-16, rtol=0)
    v4 = oracle_mod.phi(4, [0.0, 1.0, 2.0])
    assert np.allclose(v4, [0.5, 0.25, 0.0], atol=1e-16, rtol=0)


@pytest.mark.parametrize("P", [3, 4])
def test_derivative_matches_finite_differences(oracle_mod, P):
    rng = np.random.default_rng(3)
    r = rng.uniform(-SUPPORT[P] - 0.2, SUPPORT[P] + 0.2, 300)
    eps = 1e-6
    fd = (oracle_mod.phi(P, r + eps) - oracle_mod.phi(P, r - eps)) / (2 * eps)
    an = oracle_mod.dphi(P, r)
    assert np.max(np.abs(fd - an)) < 2e-8


@pytest.mark.parametrize("P,joins", [(3, [0.5, 1.5]), (4, [1.0, 2.0])])
def test_c1_at_branch_joins(oracle_mod, P, joins):
    for x in joins:
        lo, hi = x - 1e-12, x + 1e-12
        assert abs(oracle_mod.phi(P, lo) - oracle_mod.phi(P, hi)) < 1e-10
        assert abs(oracle_mod.dphi(P, lo) - oracle_mod.dphi(P, hi)) < 1e-5
    # derivative vanishes at the origin and at the support edge
    assert abs(oracle_mod.dphi(P, 0.0)) == 0.0
    assert abs(oracle_mod.dphi(P, SUPPORT[P])) < 1e-15
