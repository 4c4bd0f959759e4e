"""Local interaction zone (LIZ) of every atom, by brute force.

Part of the test oracle (test infrastructure only; see ``oracle/__init__``).

Sec. II.A and Fig. 1: for atom m only sites n closer than the LIZ radius
scatter (tau^{mn} = 0 beyond it); Sec. II.B restricts the inner sum of
Eq. (10) to n in LIZ_m.  Reading used here (the paper does not fix these
details): a member is any periodic image R_j + T of any atom j with
|R_j + T - R_m| < r_LIZ (strict), images of the same atom may appear more than
once, the central atom (zero displacement) comes first and the others follow
in increasing distance, ties broken by the displacement's x, then y, then z,
all compared after rounding to 1e-9 (bohr^2 for the squared distance).
"""

import math

import numpy as np

_Q = 1e9


def _quant(v):
    return np.floor(v * _Q + 0.5).astype(np.int64)


def image_range(cell, r_liz):
    """Number of periodic images needed along each cell vector."""
    c = np.asarray(cell, dtype=np.float64)
    vol = abs(np.linalg.det(c))
    K = []
    for d in range(3):
        e, f = c[(d + 1) % 3], c[(d + 2) % 3]
        height = vol / np.linalg.norm(np.cross(e, f))
        K.append(int(math.ceil(r_liz / height)) + 1)
    return K


def build_liz(pos, cell, r_liz, centres=None):
    """LIZ lists for every atom (or only for the listed centres).

    pos     : [N, 3] atom positions (bohr)
    cell    : [3, 3] lattice vectors as rows, or None for an open cluster
    centres : None (every atom) or an iterable of atom indices; every other atom
              gets an empty LIZ (liz_ptr[m + 1] == liz_ptr[m]), the members of a
              listed centre's LIZ are the same as in the full build
    Returns (liz_ptr [N+1] int64, liz_atom [S] int32, liz_pos [S, 3] float64)
    where liz_pos holds displacements (R_j + T) - R_m.
    """
    pos = np.asarray(pos, dtype=np.float64)
    N = pos.shape[0]
    if cell is None:
        shifts = np.zeros((1, 3))
    else:
        c = np.asarray(cell, dtype=np.float64)
        K = image_range(c, r_liz)
        rng = [np.arange(-k, k + 1) for k in K]
        g = np.stack(np.meshgrid(*rng, indexing="ij"), axis=-1).reshape(-1, 3).astype(np.float64)
        # T = n1*a1 + n2*a2 + n3*a3, accumulated in this order (componentwise)
        shifts = g[:, 0:1] * c[0] + g[:, 1:2] * c[1]
        shifts = shifts + g[:, 2:3] * c[2]
    ptr = [0]
    atoms = [np.zeros(0, dtype=np.int32)]
    disps = [np.zeros((0, 3))]
    r2max = r_liz * r_liz
    wanted = None if centres is None else set(int(c) for c in centres)
    for m in range(N):
        if wanted is not None and m not in wanted:
            ptr.append(ptr[-1])
            continue
        img = pos[None, :, :] + shifts[:, None, :]  # [nshift, N, 3]
        d = img - pos[m]
        d2 = d[..., 0] * d[..., 0] + d[..., 1] * d[..., 1]
        d2 = d2 + d[..., 2] * d[..., 2]
        sel = d2 < r2max
        j_idx = np.nonzero(sel)[1]
        dd = d[sel]
        q2 = d2[sel]
        keys = np.stack([_quant(q2), _quant(dd[:, 0]), _quant(dd[:, 1]), _quant(dd[:, 2])], axis=1)
        order = np.lexsort(keys.T[::-1])
        j_sorted = j_idx[order]
        d_sorted = dd[order]
        if q2[order][0] != 0.0 or j_sorted[0] != m:
            raise ValueError("central atom missing from its own LIZ")
        if len(q2) > 1 and np.sort(q2)[1] < 1e-16:
            raise ValueError("coincident sites: two LIZ members at zero distance")
        atoms.append(j_sorted.astype(np.int32))
        disps.append(d_sorted)
        ptr.append(ptr[-1] + len(j_sorted))
    return (np.asarray(ptr, dtype=np.int64), np.concatenate(atoms).astype(np.int32),
            np.concatenate(disps, axis=0))
