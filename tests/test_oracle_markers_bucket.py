"""Pins of the oracle's markers (a1) and bucketing (a2)."""
import math

import numpy as np
import pytest

import workloads as W


def test_marker_counts_match_configured_formula(oracle_mod):
    h = 1.0 / 64
    # round(pi (D/h)^2): 804 markers at D = 16h, 1810 at D = 24h
    assert oracle_mod.count_markers([16 * h], h)[-1] == 804
    assert oracle_mod.count_markers([24 * h], h)[-1] == 1810
    assert oracle_mod.count_markers([24 * h] * 8, h)[-1] == 14480


def test_markers_on_sphere_with_shell_volume(oracle_mod):
    h = 1.0 / 128
    d = np.array([16.0, 9.5, 31.0]) * h
    xc = np.array([[0.3, 0.4, 0.5], [0.9, 0.1, 0.2], [0.5, 0.5, 0.99]])
    m = oracle_mod.build_markers(xc, d, h)
    X = m.xyz()
    for p in range(3):
        sl = slice(m.offs[p], m.offs[p + 1])
        R = X[sl] - xc[p]
        rad = np.linalg.norm(R, axis=1)
        assert np.max(np.abs(rad / (0.5 * d[p]) - 1.0)) < 4e-16 * 8
        N = m.offs[p + 1] - m.offs[p]
        # equal-area bands: z offsets are the band midpoints 1 - (2l+1)/N
        zl = R[:, 2] / (0.5 * d[p])
        assert np.allclose(zl, 1.0 - (2 * np.arange(N) + 1) / N, atol=1e-15)
        assert abs(zl.sum()) < 1e-12
        # N dV equals the volume of the shell of thickness h around the surface
        Rp = 0.5 * d[p]
        shell = 4 * math.pi / 3 * ((Rp + h / 2) ** 3 - (Rp - h / 2) ** 3)
        assert abs(N * m.dv[p] / shell - 1.0) < 1e-14
        assert np.all(m.pid[sl] == p)


def _small_level(n=32, box=16, ngrow=2, covered=None):
    return W.make_level((n, n, n), 1.0 / n, box=box, ngrow=ngrow, covered=covered)


@pytest.mark.parametrize("P", [3, 4])
def test_bucket_sort_is_stable_and_complete(oracle_mod, P):
    rng = np.random.default_rng(5)
    lev = _small_level()
    m = oracle_mod.build_markers(rng.uniform(0, 1, (5, 3)), rng.uniform(4, 10, 5) / 32, 1 / 32)
    b = oracle_mod.bucket(lev, P, m)
    assert b["flagged"] == 0
    perm, t = b["perm"], b["tile"]
    assert np.array_equal(np.sort(perm), np.arange(m.nl))
    ts = t[perm]
    assert np.all(np.diff(ts) >= 0)
    for tt in np.unique(ts):
        seg = perm[ts == tt]
        assert np.all(np.diff(seg) > 0)              # stable: original order kept
    T = (32 // 8) ** 3
    assert np.array_equal(b["tile_offs"], np.searchsorted(ts, np.arange(T + 1)))


@pytest.mark.parametrize("P", [3, 4])
def test_owning_cell_and_stencil_cover_kernel_support(oracle_mod, P):
    """Owning cell found by edge search; every cell with a nonzero weight is in the stencil."""
    rng = np.random.default_rng(6)
    n = 32
    h = 1.0 / n
    lev = _small_level(n)
    m = oracle_mod.build_markers(rng.uniform(0, 1, (4, 3)), rng.uniform(4, 9, 4) * h, h)
    b = oracle_mod.bucket(lev, P, m)
    X = m.xyz()
    edges = np.arange(n + 1) * h
    for l in range(m.nl):
        owning = []
        for d in range(3):
            xw = X[l, d] % 1.0
            owning.append(int(np.searchsorted(edges, xw, side="right") - 1))
        assert b["cell"][l] == owning[0] + n * (owning[1] + n * owning[2])
        for d in range(3):
            centres = (np.arange(-8, n + 8) + 0.5) * h
            wts = oracle_mod.phi(P, (X[l, d] - centres) / h)
            nz = np.arange(-8, n + 8)[wts > 0]
            base = b["base"][l, d]
            assert nz.min() >= base and nz.max() <= base + P - 1


def test_source_lists_hold_every_touching_marker(oracle_mod):
    """src(tile) = sorted positions whose stencil reaches the tile, ascending."""
    rng = np.random.default_rng(7)
    n, P, tile = 32, 4, 8
    lev = _small_level(n)
    m = oracle_mod.build_markers(rng.uniform(0, 1, (6, 3)), rng.uniform(4, 9, 6) / n, 1 / n)
    b = oracle_mod.bucket(lev, P, m)
    nt = n // tile
    so, si = b["src_offs"], b["src_idx"]
    for t in range(nt ** 3):
        lst = si[so[t]:so[t + 1]]
        assert np.all(np.diff(lst) > 0)
    # brute force: enumerate stencil cells of each marker and their tiles
    expect = {t: set() for t in range(nt ** 3)}
    inv = np.argsort(b["perm"])
    for l in range(m.nl):
        base = b["base"][l]
        for k in range(P):
            for j in range(P):
                for i in range(P):
                    c = (base + np.array([i, j, k])) % n
                    t = (c[0] // tile) + nt * ((c[1] // tile) + nt * (c[2] // tile))
                    expect[int(t)].add(int(inv[l]))
    for t in range(nt ** 3):
        assert set(si[so[t]:so[t + 1]].tolist()) == expect[t]


def test_flag_marks_markers_next_to_uncovered_boxes(oracle_mod):
    n, box = 32, 16
    cov = np.ones((2, 2, 2), bool)
    cov[0, 0, 1] = False                 # box (x=1, y=0, z=0) uncovered
    lev = _small_level(n, box, covered=cov)
    h = 1.0 / n
    m_in = oracle_mod.build_markers([[0.25, 0.25, 0.25]], [6 * h], h)
    assert oracle_mod.bucket(lev, 4, m_in)["flagged"] == 0
    m_edge = oracle_mod.build_markers([[0.45, 0.25, 0.25]], [6 * h], h)
    assert oracle_mod.bucket(lev, 4, m_edge)["flagged"] > 0
