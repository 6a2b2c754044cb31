"""The paper's triangular D2Q7 lattice (Sec. II) from its geometry, for the
tests: directions e_i = (cos, sin)((i - 1) pi/3), weights 1/2 and 1/12,
c_s^2 = 1/4, and site (x, y) at (x + (y mod 2)/2, y sqrt(3)/2).  Nothing here
is taken from the oracle or the GPU library."""
import numpy as np

ANG = np.array([0.0] + [(i - 1) * np.pi / 3.0 for i in range(1, 7)])
EX = np.where(np.arange(7) == 0, 0.0, np.cos(ANG))
EY = np.where(np.arange(7) == 0, 0.0, np.sin(ANG))
W = np.array([1.0 / 2.0] + [1.0 / 12.0] * 6)
CS2 = 0.25
# reverse direction: the one whose vector is -e_i
OPP = np.array([0] + [int(np.argmin((EX + EX[i]) ** 2 + (EY + EY[i]) ** 2 + (np.arange(7) == 0)))
                      for i in range(1, 7)])


def equilibrium(rho, ux, uy):
    """Eq. 3 on D2Q7: w_i rho (1 + e.u / c_s^2 + (e.u)^2 / (2 c_s^4) - u^2 / (2 c_s^2))."""
    rho, ux, uy = np.broadcast_arrays(*(np.asarray(a, dtype=np.float64) for a in (rho, ux, uy)))
    cu = EX[:, None, None] * ux[None] + EY[:, None, None] * uy[None]
    usq = ux * ux + uy * uy
    return W[:, None, None] * rho[None] * (1.0 + cu / CS2 + cu * cu / (2 * CS2 ** 2)
                                           - usq[None] / (2 * CS2))


def momentum(f):
    return (EX[:, None, None] * f).sum(0), (EY[:, None, None] * f).sum(0)


def position(x, y):
    return x + 0.5 * (y % 2), y * np.sqrt(3.0) / 2.0


def site_at(px, py, L):
    """(x, y_raw) of the site at position (px, py), x taken modulo L (y_raw
    may lie outside the lattice); None if no site is there."""
    y = int(round(py / (np.sqrt(3.0) / 2.0)))
    if abs(y * np.sqrt(3.0) / 2.0 - py) > 1e-9:
        return None
    xf = px - 0.5 * (y % 2)
    x = int(round(xf))
    if abs(xf - x) > 1e-9:
        return None
    return x % L, y
