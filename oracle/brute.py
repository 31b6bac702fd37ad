"""Scalar brute-force DAS in pure Python (``math`` only).  TEST INFRASTRUCTURE.

A second, independently written form of the same defining sum as
``das_oracle.das`` (paper Sec. 2.1 / 4.1 / 4.3): one voxel, one frame, one
element, one transmit at a time, with the interpolation done by reading the
two neighbouring samples explicitly and the phasor built from cos/sin.  It is
meant for tiny inputs only (it is thousands of times slower), to pin the
vectorised oracle by brute force.
"""

import math


def _window(rho, alpha):
    if rho >= 1.0:
        return 0.0
    if alpha <= 0.0:
        return 1.0
    edge = 1.0 - alpha
    if rho <= edge:
        return 1.0
    return 0.5 + 0.5 * math.cos(math.pi * (rho - edge) / alpha)


def das_scalar(iq, elem, vox, tx, c, fs, fd, t0, f_number, alpha):
    """``iq`` nested lists/arrays [T][E][S][F] of complex; returns list [V][F] complex."""
    T = len(iq)
    E = len(iq[0])
    S = len(iq[0][0])
    F = len(iq[0][0][0])
    out = []
    for v in range(len(vox)):
        xv, yv, zv = (float(a) for a in vox[v])
        row = [0j] * F
        for e in range(E):
            xe, ye, ze = (float(a) for a in elem[e])
            if f_number == 0.0:
                w = 1.0
            else:
                depth = zv - ze
                if depth <= 0.0:
                    w = 0.0
                else:
                    lateral = math.sqrt((xv - xe) * (xv - xe) + (yv - ye) * (yv - ye))
                    w = _window(2.0 * f_number * lateral / depth, alpha)
            dist = math.sqrt((xv - xe) ** 2 + (yv - ye) ** 2 + (zv - ze) ** 2)
            for t in range(T):
                delay = float(tx[t][v]) + dist / c
                pos = (delay - t0) * fs
                left = math.floor(pos)
                frac = pos - left
                cyc = 2.0 * math.pi * fd * delay
                phasor = complex(math.cos(cyc), math.sin(cyc))
                for f in range(F):
                    a = complex(iq[t][e][left][f]) if 0 <= left < S else 0j
                    b = complex(iq[t][e][left + 1][f]) if 0 <= left + 1 < S else 0j
                    row[f] += w * phasor * (a + frac * (b - a))
        out.append(row)
    return out
