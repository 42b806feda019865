"""Ray-path gradient of a travel time with respect to the orientation of every node (a check
of the adjoint by a different discretisation, not part of the method).

A ray's time is stationary in its path (Fermat), so to first order a change of the medium
changes the time only through the slowness along the path held fixed.  Each straight piece
of the polyline is cut at the nearest-node cell boundaries, as the dense-graph reference
cuts its segments; a piece of length l (grid units) in the cell of node p, travelled in
direction a, takes l h / V(phi) with phi = a - (theta_p + 90 deg), V the group speed of the
node's material (Section 5.1), so its derivative in theta_p is l h V'(phi) / V(phi)^2.
"""
import math

import numpy as np


def ray_path_gradient(orc, h, mats, mat_id, orient, pts):
    """d(time along the polyline pts [n, 2] of grid coordinates (x, z)) / d(orientation of
    every node) [nz, nx], the path held fixed."""
    mat_id, orient = np.asarray(mat_id), np.asarray(orient, np.float64)
    nz, nx = mat_id.shape
    G = np.zeros((nz, nx))
    pts = np.asarray(pts, np.float64)
    for (x0, z0), (x1, z1) in zip(pts[:-1], pts[1:]):
        dx, dz = x1 - x0, z1 - z0
        length = math.hypot(dx, dz)
        if length == 0.0:
            continue
        ang = math.atan2(dz, dx)
        cuts = [0.0, 1.0]
        for start, d in ((x0, dx), (z0, dz)):
            if d == 0.0:
                continue
            lo, hi = min(start, start + d), max(start, start + d)
            b = math.floor(lo - 0.5) + 0.5
            while b <= hi:
                t = (b - start) / d
                if 0.0 < t < 1.0:
                    cuts.append(t)
                b += 1.0
        cuts.sort()
        for ta, tb in zip(cuts[:-1], cuts[1:]):
            if tb <= ta:
                continue
            tm = 0.5 * (ta + tb)
            ci = min(max(int(math.floor(x0 + tm * dx + 0.5)), 0), nx - 1)
            cj = min(max(int(math.floor(z0 + tm * dz + 0.5)), 0), nz - 1)
            m = mats[int(mat_id[cj, ci])]
            phi = ang - (orient[cj, ci] + 0.5 * math.pi)
            V, dV = orc.group_speed(m, phi), orc.group_speed_deriv(m, phi)
            G[cj, ci] += (tb - ta) * length * h * dV / (V * V)
    return G


def cosine(a, b):
    a, b = np.ravel(a), np.ravel(b)
    return float(a @ b / (np.linalg.norm(a) * np.linalg.norm(b)))
