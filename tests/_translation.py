"""Shape measures of a drop in a periodic box (translation test helpers).

The centre is the circular mean of the heavy-phase indicator per axis (exact
for a drop that does not wrap onto itself), the eccentricity comes from the
second moments about that centre: sqrt(1 - lambda_min / lambda_max), 0 for a
circle.  Nodes of the jittered grids carry equal area on average, so the
indicator is not mass-weighted.
"""
import numpy as np


def drop_centre(xyz, box, C):
    w = np.clip(C, 0.0, 1.0)
    c = np.empty(xyz.shape[1])
    for a in range(xyz.shape[1]):
        th = 2.0 * np.pi * xyz[:, a] / box[a]
        c[a] = (np.arctan2((w * np.sin(th)).sum(), (w * np.cos(th)).sum()) / (2.0 * np.pi) * box[a]) % box[a]
    return c


def min_image(d, box):
    return d - box * np.round(d / box)


def drop_shape(xyz, box, C):
    """(centre, eccentricity) of the heavy phase."""
    c = drop_centre(xyz, box, C)
    w = np.clip(C, 0.0, 1.0)
    d = min_image(xyz - c, box)
    I = np.einsum("n,ni,nj->ij", w, d, d) / w.sum()
    ev = np.linalg.eigvalsh(I)
    return c, float(np.sqrt(max(0.0, 1.0 - ev[0] / ev[-1])))
