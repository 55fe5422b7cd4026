"""Dense brute-force form of the IB operators, used to pin the oracle.

The interpolation operator is built as a dense matrix over every cell of a
small periodic grid, with the minimum-image distance from each cell centre to
each marker and no stencil at all: the compact support of the kernel alone
decides which cells take part.  This shares no index logic with the oracle
(base cells, wrapping, stencil loops); only the 1-D kernel is taken from it.
"""
import numpy as np


def dense_weights(n, h, X, phi_vec):
    """Dense matrix W[l, cell] = prod_d phi((X_ld - x_d)/h), cell x fastest."""
    xs = (np.arange(n) + 0.5) * h
    L = n * h
    ws = []
    for d in range(3):
        dist = X[:, d, None] - xs[None, :]
        dist = dist - L * np.round(dist / L)          # minimum image
        ws.append(phi_vec(dist / h))                  # (nl, n)
    W = np.einsum("lk,lj,li->lkji", ws[2], ws[1], ws[0])
    return W.reshape(X.shape[0], n ** 3)


def dense_multidirect(W, dv_l, h, ns, dt, Ud, u0):
    """Algorithm 1 with dense operators; u0 is (3, n^3)."""
    F = np.zeros_like(Ud)
    u = u0.copy()
    resid = [np.sqrt((dv_l[:, None] * (Ud - (W @ u.T)) ** 2).sum())]
    f = np.zeros_like(u0)
    for _ in range(ns):
        U = (W @ u.T)                                # (nl, 3)
        F = F + (Ud - U) / dt
        f = (W.T @ (F * (dv_l / h ** 3)[:, None])).T
        u = u0 + dt * f
        resid.append(np.sqrt((dv_l[:, None] * (Ud - (W @ u.T)) ** 2).sum()))
    return u, f, F, np.array(resid)
