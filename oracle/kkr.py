"""Multiple-scattering matrices of one LIZ: t, g, 1 - t g and the tau blocks.

Part of the test oracle (test infrastructure only; see ``oracle/__init__``).

Units: Rydberg atomic units (hbar = 1, 2 m_e = 1), so the wavenumber of
Sec. II.C is kappa = sqrt(z).  Lengths in bohr, energies in Ry.

Readings of points the paper leaves open (each is pinned by a test):

* Energies z+- = eF +- i eta (Eq. (7)); kappa+ = principal sqrt(z+)
  (Im > 0) and kappa- = -conj(kappa+) (the same physical sheet).
* t-matrix of a spherical scatterer from its phase shifts:
  t_l(z+) = -sin(delta_l) e^{i delta_l} / kappa+ and t(z-) = conj(t(z+)); T is
  diagonal in L (Eq. (4)).
* Free-electron structure constants g^{ab} (the propagator of Eq. (3)) for
  two LIZ members a != b with R = p_a - p_b:
      g^{ab}_{LL'} = -4 pi i kappa sum_{L''} i^{l - l' + l''} C_{L L' L''}
                     h_{l''}(kappa |R|) Y_{L''}(R^)
  and g^{aa} = 0.  This is the two-centre expansion of the free outgoing
  Green function -exp(i kappa |r - r'|) / (4 pi |r - r'|) in regular solutions
  j_l(kappa r) Y_L(r^) about the two sites.
* tau = (T^-1 - g)^-1 (Eq. (3)) is evaluated as (1 - T g)^-1 T, which avoids
  T^-1 for small phase shifts.
"""

import numpy as np
import scipy.linalg

from . import special

LMAX = 3
NL = (LMAX + 1) ** 2


def energies(e_fermi, eta):
    """Return (z+, z-, kappa+, kappa-)."""
    zp = complex(e_fermi, eta)
    zm = complex(e_fermi, -eta)
    kp = np.sqrt(zp)
    if kp.imag < 0:
        kp = -kp
    km = -np.conj(kp)
    return zp, zm, complex(kp), complex(km)


def t_matrix(phase, kappa_plus):
    """Single-site t_l at z+ and z- from phase shifts delta_l (radians).

    phase: [..., lmax+1].  Returns (t_plus, t_minus), same shape, complex.
    """
    d = np.asarray(phase, dtype=np.float64)
    tp = -np.sin(d) * np.exp(1j * d) / kappa_plus
    return tp, np.conj(tp)


def expand_t(t_l, lmax=LMAX):
    """Broadcast t_l over the 2l+1 channels m of each shell: [..., (lmax+1)^2]."""
    idx = np.array([special.lm_of(L)[0] for L in range((lmax + 1) ** 2)])
    return np.asarray(t_l)[..., idx]


_GAUNT_CACHE = {}


def _gaunt(lmax):
    if lmax not in _GAUNT_CACHE:
        _GAUNT_CACHE[lmax] = special.gaunt_table(lmax, lmax, 2 * lmax)
    return _GAUNT_CACHE[lmax]


def g0_blocks(R, kappa, lmax=LMAX):
    """Structure-constant blocks g^{ab}_{LL'} for displacements R[..., 3] = p_a - p_b (R != 0).

    Returns [..., NL, NL] complex.
    """
    R = np.asarray(R, dtype=np.float64)
    l3max = 2 * lmax
    nl3 = (l3max + 1) ** 2
    C = _gaunt(lmax)  # [NL, NL, NL3]
    nl = C.shape[0]
    l_of = np.array([special.lm_of(L)[0] for L in range(nl3)])
    # phase i^{l - l' + l''} times the Gaunt coefficient
    expo = (l_of[:nl, None, None] - l_of[None, :nl, None] + l_of[None, None, :]) % 4
    PC = np.array([1.0, 1j, -1.0, -1j])[expo] * C
    dist = np.sqrt(np.sum(R * R, axis=-1))
    h = special.hankel1(l3max, kappa * dist)  # [l3max+1, ...]
    Y = special.real_ylm(l3max, R)  # [..., NL3]
    hY = np.moveaxis(h[l_of], 0, -1) * Y  # [..., NL3]
    return -4.0 * np.pi * 1j * kappa * np.einsum("xyz,...z->...xy", PC, hY)


def g0_block(R, kappa, lmax=LMAX):
    """Single block g^{ab} for R = p_a - p_b."""
    return g0_blocks(np.asarray(R, dtype=np.float64)[None, :], kappa, lmax)[0]


def g0_matrix(liz_pos, kappa, lmax=LMAX):
    """Full structure-constant matrix g over one LIZ (n = NL * members)."""
    P = np.asarray(liz_pos, dtype=np.float64)
    nm = P.shape[0]
    nl = (lmax + 1) ** 2
    a, b = np.nonzero(~np.eye(nm, dtype=bool))
    blocks = g0_blocks(P[a] - P[b], kappa, lmax)
    G = np.zeros((nm, nl, nm, nl), dtype=np.complex128)
    G[a, :, b, :] = blocks
    return G.reshape(nm * nl, nm * nl)


def kkr_matrix(liz_pos, t_members, kappa, lmax=LMAX):
    """M = 1 - T g for one LIZ.  t_members: [members, lmax+1] complex t_l."""
    G = g0_matrix(liz_pos, kappa, lmax)
    tdiag = expand_t(np.asarray(t_members), lmax).reshape(-1)
    return np.eye(G.shape[0], dtype=np.complex128) - tdiag[:, None] * G


def tau_blocks(M, t_members, lmax=LMAX):
    """Column and row of tau touching the central member 0.

    tau = (1 - T g)^-1 T.  Column:  X = M^-1 T E0, block a is tau^{a0}.
    Row:  tau^{0.} = E0^T M^-1 T, obtained from the transposed system
    M^T y = E0, block a of the row is (y^T T)[:, a-block] = tau^{0a}.
    Returns (col [members, NL, NL], row [members, NL, NL]).
    """
    nl = (lmax + 1) ** 2
    tdiag = expand_t(np.asarray(t_members), lmax).reshape(-1)
    n = M.shape[0]
    nm = n // nl
    lu = scipy.linalg.lu_factor(M)
    E0 = np.zeros((n, nl), dtype=np.complex128)
    E0[np.arange(nl), np.arange(nl)] = 1.0
    X = scipy.linalg.lu_solve(lu, E0 * tdiag[None, :nl])  # B = E0 t_center
    Yt = scipy.linalg.lu_solve(lu, E0, trans=1)  # M^T Yt = E0
    row = (Yt.T * tdiag[None, :])  # [NL, n] = E0^T M^-1 T
    col = X.reshape(nm, nl, nl)
    rowb = row.reshape(nl, nm, nl).transpose(1, 0, 2)
    return col, rowb


def atom_tau(liz_pos, t_plus_members, t_minus_members, kappa_plus, kappa_minus, lmax=LMAX):
    """tau column/row blocks of one LIZ at both energies.

    Returns dict with 'col+', 'row+', 'col-', 'row-' ([members, NL, NL] each).
    """
    out = {}
    for tag, tm, k in (("+", t_plus_members, kappa_plus), ("-", t_minus_members, kappa_minus)):
        M = kkr_matrix(liz_pos, tm, k, lmax)
        col, row = tau_blocks(M, tm, lmax)
        out["col" + tag] = col
        out["row" + tag] = row
    return out
