"""Error bound of a central difference quotient of an FP64 loss."""


def fd_bound(L_at, eps, eps_mach=2.0 ** -52):
    """Bound on |(L(eps) - L(-eps))/(2 eps) - dL/dt(0)| for a loss evaluated in
    FP64 along a direction; L_at(t) returns (L, sum of |terms of L|).

    Rounding: each evaluation is off by at most eps_mach S (S = the sum of the
    magnitudes of the loss's terms), which the difference quotient divides by
    eps.  Truncation: the central difference is off by eps^2/6 d3 + O(eps^4),
    d3 the third derivative along the direction, estimated by the four-point
    formula with step eta = 10 eps,
    d3 = (L(2 eta) - 2 L(eta) + 2 L(-eta) - L(-2 eta)) / (2 eta^3),
    whose own rounding (3 eps_mach S / eta^3, times eps^2/6: 5e-4 of the
    rounding term) is negligible.  The factor 2 covers the neglected higher
    order terms of both formulas and the rounding of the analytic gradient."""
    Lp, Sp = L_at(eps)
    Lm, Sm = L_at(-eps)
    eta = 10 * eps
    L2 = [L_at(t)[0] for t in (2 * eta, eta, -eta, -2 * eta)]
    d3 = (L2[0] - 2 * L2[1] + 2 * L2[2] - L2[3]) / (2 * eta ** 3)
    fd = (Lp - Lm) / (2 * eps)
    return fd, 2.0 * (eps_mach * max(Sp, Sm) / eps + eps ** 2 / 6 * abs(d3))
