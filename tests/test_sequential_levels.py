"""Host checks of the conflict levels behind the particle-by-particle order
(Sec. 3.1, the remarks after Algorithm 1): the conservative support test never
misses two particles whose stencils share a cell, and running particles in
(level, index) order gives the oracle's index-order sweep."""
import numpy as np
import pytest

import workloads as W
from seq_ref import chain_workload, ref_levels, support_cells


def _L(lev):
    return [lev.n[a] * lev.h if lev.periodic[a] else 0.0 for a in range(3)]


@pytest.mark.parametrize("which", ["chain4", "chain3", "spheres64_128"])
def test_support_test_covers_every_shared_cell(oracle_mod, which):
    if which == "spheres64_128":
        wl = W.config(5, 0, with_field=False)
    else:
        wl = chain_workload(delta=4 if which == "chain4" else 3)
    lev = wl.level
    h, n, P = lev.h, lev.n[0], wl.delta
    m = oracle_mod.build_markers(wl.xc, wl.d, h)
    sup = []
    for p in range(wl.npart):
        a, z = int(m.offs[p]), int(m.offs[p + 1])
        sup.append(support_cells(m.x[a:z], m.y[a:z], m.z[a:z], n, h, P))
    L = _L(lev)
    reach = 2.0 * P * h
    shared = 0
    for j in range(wl.npart):
        for i in range(j):
            dx = wl.xc[i] - wl.xc[j]
            dx -= np.array(L) * np.floor(dx / np.array(L) + 0.5)
            flagged = (dx @ dx) < (0.5 * (wl.d[i] + wl.d[j]) + reach) ** 2
            meet = np.intersect1d(sup[i], sup[j]).size > 0
            shared += meet
            assert flagged or not meet, (i, j)
    if which != "spheres64_128":
        assert shared >= 5
    lv = ref_levels(wl.xc, wl.d, h, P, L)
    if which != "spheres64_128":
        assert lv.max() >= 2
        assert not np.array_equal(np.argsort(lv, kind="stable"), np.arange(wl.npart))


def test_level_order_reproduces_index_order(oracle_mod):
    """The oracle's sweep over the particles permuted into (level, index)
    order equals its sweep in index order."""
    wl = chain_workload(n=48, box=16, k=6, extra=2, seed=1)
    lev = wl.level
    g = oracle_mod.grid_of(lev)
    lv = ref_levels(wl.xc, wl.d, lev.h, wl.delta, _L(lev))
    perm = np.argsort(lv, kind="stable")
    assert lv.max() >= 2 and not np.array_equal(perm, np.arange(wl.npart))
    m = oracle_mod.build_markers(wl.xc, wl.d, lev.h)
    a = oracle_mod.multidirect(g, wl.delta, wl.ns, wl.dt, m, wl.xc, wl.up, wl.om, wl.u0,
                               order="sequential")
    mp = oracle_mod.build_markers(wl.xc[perm], wl.d[perm], lev.h)
    b = oracle_mod.multidirect(g, wl.delta, wl.ns, wl.dt, mp, wl.xc[perm], wl.up[perm],
                               wl.om[perm], wl.u0, order="sequential")
    # markers of particle perm[k] sit at mp.offs[k] in the permuted run
    Fb = np.zeros_like(a["F"])
    for k, p in enumerate(perm):
        Fb[m.offs[p]:m.offs[p + 1]] = b["F"][mp.offs[k]:mp.offs[k + 1]]
    assert np.max(np.abs(Fb - a["F"])) <= 1e-13 * np.abs(a["F"]).max()
    assert np.max(np.abs(b["ustar"] - a["ustar"])) <= 1e-13 * np.abs(a["ustar"]).max()
    assert np.max(np.abs(b["f"] - a["f"])) <= 1e-13 * np.abs(a["f"]).max()
    # and the index order matters for this workload
    jac = oracle_mod.multidirect(g, wl.delta, wl.ns, wl.dt, m, wl.xc, wl.up, wl.om, wl.u0)
    assert np.max(np.abs(jac["F"] - a["F"])) > 1e-6 * np.abs(a["F"]).max()
