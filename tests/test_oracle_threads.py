"""The OpenMP build of the oracle against the single-threaded build.

Both come from the same C source.  The parallel build splits interpolation per
marker, the velocity correction per cell and spreading by slabs of z planes
(each thread visits every marker in index order and adds only into its own
planes), so every sum keeps its serial order and the results must agree bit
for bit -- also with more threads than planes and across periodic wraps."""
import numpy as np
import pytest

import workloads as W


def _case(n, delta, ns, seed, k=4, periodic=(1, 1, 1)):
    rng = np.random.default_rng(300 + seed)
    diam = rng.uniform(5.0, 9.0, k)
    return W.make_workload(f"omp{n}_{delta}_{seed}", n, 16, 2, delta, ns, diam, seed=seed,
                           nmodes=8, K=4, cover_all=True)


@pytest.mark.parametrize("P,threads", [(3, 3), (4, 5), (4, 64)])
def test_openmp_loop_identical(oracle_mod, P, threads):
    wl = _case(32, P, 3, P + threads)
    lev = wl.level
    g = oracle_mod.grid_of(lev)
    m = oracle_mod.build_markers(wl.xc, wl.d, lev.h)
    args = (g, P, wl.ns, wl.dt, m, wl.xc, wl.up, wl.om, wl.u0)
    a = oracle_mod.multidirect(*args, history=True)
    b = oracle_mod.multidirect(*args, history=True, threads=threads)
    for k in ("ustar", "f", "F", "resid", "Fhist"):
        assert np.array_equal(a[k], b[k]), k
    # the particle-by-particle order goes through the same loop
    a = oracle_mod.multidirect(*args, order="sequential")
    b = oracle_mod.multidirect(*args, order="sequential", threads=threads)
    for k in ("ustar", "f", "F"):
        assert np.array_equal(a[k], b[k]), k


@pytest.mark.parametrize("P", [3, 4])
def test_openmp_interp_spread_identical(oracle_mod, P):
    wl = _case(32, P, 2, 7 + P)
    lev = wl.level
    g = oracle_mod.grid_of(lev)
    m = oracle_mod.build_markers(wl.xc, wl.d, lev.h)
    F = np.random.default_rng(5).normal(size=(m.nl, 3))
    assert np.array_equal(oracle_mod.spread(g, P, m, F), oracle_mod.spread(g, P, m, F, threads=6))
    assert np.array_equal(oracle_mod.interp(g, P, m, wl.u0),
                          oracle_mod.interp(g, P, m, wl.u0, threads=6))


def test_openmp_thread_count(oracle_mod):
    assert oracle_mod.threads_available() >= 1
    oracle_mod._load(3)
    assert oracle_mod.threads_available() == 3
