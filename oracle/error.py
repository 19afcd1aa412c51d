"""FP64 oracle -- the global error of a product (test infrastructure only;
see oracle/tree.py for the usage rule).

The experiments of Section 6 report the relative spectral error
||XY - C||_2 / ||XY||_2 of a computed product C, each norm estimated by ten
steps of the power iteration.  The steps taken here, on E^* E for a linear
map E given by its action and the action of its adjoint:
    z = z0 / ||z0||;  repeat: w = E z,  sigma = ||w||,  z = E^* w / ||E^* w||
and the estimate is the sigma of the last step (the Rayleigh value
sqrt(z^* E^* E z) for a unit z, hence a lower bound of ||E||_2).  E z for
E = XY - C is X(Y z) - C z with the H2 matrix-vector products of Section 2
(H2Matrix.matvec / rmatvec).
"""
from __future__ import annotations

import math

import numpy as np


def power_norm(apply, apply_adj, z0, iters: int) -> float:
    """Estimate of ||E||_2 after `iters` steps from the start vector z0."""
    z = np.array(z0, dtype=np.float64)
    n0 = math.sqrt(float(z @ z))
    if n0 == 0.0:
        raise ValueError("zero start vector")
    z = z / n0
    sigma = 0.0
    for _ in range(iters):
        w = apply(z)
        sigma = math.sqrt(float(w @ w))
        zt = apply_adj(w)
        nz = math.sqrt(float(zt @ zt))
        if nz == 0.0:
            break
        z = zt / nz
    return sigma


def product_error(X, Y, c_apply, c_apply_adj, z0, iters: int = 10):
    """(estimate of ||XY - C||_2, estimate of ||XY||_2) for oracle H2 matrices
    X, Y and a product C given by its action (c_apply, c_apply_adj; None for
    C = 0), original index order."""
    def xy(z):
        return X.matvec(Y.matvec(z))

    def xy_adj(w):
        return Y.rmatvec(X.rmatvec(w))

    if c_apply is None:
        err = 0.0
    else:
        err = power_norm(lambda z: xy(z) - c_apply(z), lambda w: xy_adj(w) - c_apply_adj(w), z0, iters)
    return err, power_norm(xy, xy_adj, z0, iters)
