"""The D2Q9 lattice as the tests define it, independently of both the oracle
and the GPU library: velocities, weights, reverse directions, and moment
helpers over arrays shaped [9, ...]."""
import numpy as np

# 0 rest, 1 E, 2 N, 3 W, 4 S, 5 NE, 6 NW, 7 SW, 8 SE
C = np.array([(0, 0), (1, 0), (0, 1), (-1, 0), (0, -1),
              (1, 1), (-1, 1), (-1, -1), (1, -1)], dtype=np.int64)
W = np.array([4 / 9] + [1 / 9] * 4 + [1 / 36] * 4)
OPP = np.array([0, 3, 4, 1, 2, 7, 8, 5, 6])
CS2 = 1.0 / 3.0


def density(f):
    return f.sum(axis=0)


def momentum(f):
    cx = C[:, 0].astype(float).reshape((9,) + (1,) * (f.ndim - 1))
    cy = C[:, 1].astype(float).reshape((9,) + (1,) * (f.ndim - 1))
    return (f * cx).sum(axis=0), (f * cy).sum(axis=0)


def second_moment(f):
    shp = (9,) + (1,) * (f.ndim - 1)
    cx = C[:, 0].astype(float).reshape(shp)
    cy = C[:, 1].astype(float).reshape(shp)
    return (f * cx * cx).sum(0), (f * cx * cy).sum(0), (f * cy * cy).sum(0)


def equilibrium(rho, ux, uy):
    """Textbook second-order D2Q9 equilibrium (Kruger et al. 2016), with
    numpy broadcasting over rho/ux/uy."""
    rho = np.asarray(rho, float)
    ux = np.asarray(ux, float)
    uy = np.asarray(uy, float)
    out = []
    for i in range(9):
        cu = C[i, 0] * ux + C[i, 1] * uy
        out.append(W[i] * rho * (1 + cu / CS2 + cu * cu / (2 * CS2 * CS2)
                                 - (ux * ux + uy * uy) / (2 * CS2)))
    return np.stack(out)


def stream_pull(f, ybc="fixed"):
    """Streaming by array shifts: f*_i(x, y) = f_i(x - c_ix, y - c_iy), x
    periodic; y periodic, or a bounce-back wall below row 0 and nothing above
    the top row.  f is [9, H, L]."""
    out = np.zeros_like(f)
    H = f.shape[1]
    for i in range(9):
        cx, cy = int(C[i, 0]), int(C[i, 1])
        g = np.roll(f[i], shift=cx, axis=1)          # x - cx, periodic
        if ybc == "periodic":
            out[i] = np.roll(g, shift=cy, axis=0)
            continue
        if cy == 0:
            out[i] = g
        elif cy == 1:                                  # from the row below
            out[i, 1:] = g[:-1]
            out[i, 0] = f[OPP[i], 0]                   # wall: reflected in place
        else:                                          # from the row above
            out[i, :H - 1] = g[1:]
            out[i, H - 1] = 0.0
    return out
