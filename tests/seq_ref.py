"""Test-side definitions for the particle-by-particle order of the loop.

``ref_levels`` is the conflict level written out as its definition (the
longest chain of conflicting earlier particles ending at each particle, in
index order), with the same conservative support test the library states;
``support_cells`` is the set of cells a particle's markers reach, from the
stencil rule (base cell and P cells per axis, wrapped), with no index logic
shared with either side.  ``chain_workload`` places spheres whose supports
overlap along a periodic chain, in shuffled index order, so that the levels
are neither trivial nor equal to the index order.
"""
import numpy as np

import workloads as W


def ref_levels(xc, d, h, P, L):
    n = d.shape[0]
    lev = np.zeros(n, dtype=np.int64)
    reach = 2.0 * P * h
    for j in range(n):
        if j == 0:
            continue
        dx = xc[:j] - xc[j]
        for c in range(3):
            if L[c] > 0:
                dx[:, c] -= L[c] * np.floor(dx[:, c] / L[c] + 0.5)
        r2 = dx[:, 0] * dx[:, 0] + dx[:, 1] * dx[:, 1] + dx[:, 2] * dx[:, 2]
        lim = 0.5 * (d[:j] + d[j]) + reach
        hit = r2 < lim * lim
        lev[j] = lev[:j][hit].max() + 1 if hit.any() else 0
    return lev


def support_cells(x, y, z, n, h, P):
    """Linear indices of every cell in the union of the markers' stencils."""
    cells = []
    for s_ax, arr in enumerate((x, y, z)):
        s = arr / h
        base = np.floor(s).astype(np.int64) - 1 if P == 3 else \
            np.floor(s - 0.5).astype(np.int64) - 1
        cells.append(np.mod(base[:, None] + np.arange(P)[None, :], n))
    cx, cy, cz = cells
    lin = cx[:, None, None, :] + n * (cy[:, None, :, None] + n * cz[:, :, None, None])
    return np.unique(lin.reshape(-1))


def chain_workload(n=64, box=16, delta=4, ns=3, seed=0, k=7, extra=3):
    """k spheres along x with gaps of 0.5-3 cells (the chain closes across the
    periodic face), plus ``extra`` isolated spheres; indices shuffled."""
    rng = np.random.default_rng(500 + seed)
    h = 1.0 / n
    dcell = rng.uniform(5.5, 7.5, k)
    xs = [0.05]
    for i in range(1, k):
        xs.append(xs[-1] + (0.5 * (dcell[i - 1] + dcell[i]) + rng.uniform(0.5, 3.0)) * h)
    cen = np.stack([np.mod(np.array(xs), 1.0),
                    0.5 + rng.uniform(-1.0, 1.0, k) * h,
                    0.5 + rng.uniform(-1.0, 1.0, k) * h], axis=1)
    iso_d = rng.uniform(5.0, 7.0, extra)
    iso = np.stack([rng.uniform(0.1, 0.9, extra), np.full(extra, 0.12),
                    np.linspace(0.15, 0.85, extra)], axis=1)
    allc = np.concatenate([cen, iso])
    alld = np.concatenate([dcell, iso_d])
    order = rng.permutation(allc.shape[0])
    return W.make_workload(f"chain{n}_{delta}_{seed}", n, box, 2, delta, ns, alld[order],
                           seed=seed, centres=allc[order], nmodes=8, K=4, cover_all=True)
