"""Residual of one grid point of a dimension-by-dimension scheme as the sum
of its line contributions, each evaluated by the oracle on the line alone
(a grid whose other axes hold nine periodic copies of the line: their flux
differences vanish exactly).  Used to check full-size GPU residuals on
sampled points."""
import numpy as np

COPIES = 9


def bc_tuple(prob, ndim):
    bc = prob["bc"]
    return tuple(bc for _ in range(ndim)) if isinstance(bc, str) else tuple(bc)


def line_contribution(ora, prob, U, axis, idx, kw):
    """Residual contribution of direction `axis` along the line through the
    node idx (a tuple in array order z, y, x / y, x), from the oracle."""
    ndim = prob["ndim"]
    n = list(prob["n"])           # (nx, ny[, nz])
    h = list(prob["h"])
    bc = list(bc_tuple(prob, ndim))
    sl = [slice(None)] + [slice(i, i + 1) for i in idx]
    ax_arr = ndim - axis          # array axis of `axis` (array order is reversed, after nv)
    sl[ax_arr] = slice(None)
    line = U[tuple(sl)]           # (nv, 1.., n_axis, 1..)
    reps = [1] + [COPIES] * ndim
    reps[ax_arr] = 1
    Ul = np.ascontiguousarray(np.tile(line, reps))
    nl = [COPIES] * ndim
    nl[axis] = n[axis]
    bl = ["periodic"] * ndim
    bl[axis] = bc[axis]
    P = ora.Problem(system="euler", ndim=ndim, n=tuple(nl), h=tuple(h), bc=tuple(bl),
                    gamma=prob.get("gamma", 1.4), **kw)
    R = P.residual(Ul)
    pos = [0] * ndim
    pos[ndim - 1 - axis] = idx[ndim - 1 - axis]
    return R[(slice(None),) + tuple(pos)]
