"""Derivative of the conductivity with respect to the phase shifts.

Part of the test oracle (test infrastructure only; see ``oracle/__init__``).

Differentiating Eq. (3): with W = (1 - T g)^-1 one has tau = W T = T W^T and
d tau = W dT W^T (no T^-1 appears).  T is diagonal, so perturbing the
t-matrix of LIZ member b in shell l changes every block by
    d tau^{pq}_{L1 L2} = sum_{m} W_{(p,L1),(b,lm)} W_{(q,L2),(b,lm)} dt_l.
This module forms those derivatives explicitly (forward mode, one dense
inverse per LIZ and energy), propagates them through Eq. (10) and Eq. (7),
and applies the chain rule dt_l(z+)/d delta_l = -e^{2 i delta_l}/kappa+ and
dt(z-)/d delta = conj(dt(z+)/d delta) (t(z-) = conj t(z+)).  Contributions of
every LIZ image of a site are summed into that site's entry.
"""

import numpy as np

from . import kkr, kubo, liz


def dsigma_dphase(pos, cell, r_liz, species, phase, J, e_fermi, eta, dsigma, volume=None, liz_lists=None,
                  pairs=None):
    """Gradient of L = sum_mu dsigma[mu] * sigma_mu with respect to phase[N, 4].

    ``pairs`` (None: all) restricts the result to the listed (site, l) entries: only the
    atoms whose LIZ holds an image of a listed site contribute to them, so only those LIZ are
    inverted; every other entry of the result is left zero.
    Returns complex [N, 4]; the imaginary part vanishes analytically.
    """
    pos = np.asarray(pos, dtype=np.float64)
    N = pos.shape[0]
    nl = kkr.NL
    if volume is None:
        volume = kubo.supercell_volume(cell)
    if liz_lists is None:
        liz_lists = liz.build_liz(pos, cell, r_liz)
    ptr, latom, lpos = liz_lists
    zp, zm, kp, km = kkr.energies(e_fermi, eta)
    phase = np.asarray(phase, dtype=np.float64)
    tp, tm = kkr.t_matrix(phase, kp)
    dtp = -np.exp(2j * phase) / kp  # dt(z+)/d delta
    dtm = np.conj(dtp)
    species = np.asarray(species)
    dsigma = np.asarray(dsigma, dtype=np.float64)
    # weight of s[c, mu] in L
    w = np.zeros((4, 3))
    for c in range(4):
        w[c] = dsigma * 0.25 * kubo.SIGNS[c] * (-1.0 / (np.pi * volume))
    lshell = np.array([0, 1, 1, 1, 2, 2, 2, 2, 2, 3, 3, 3, 3, 3, 3, 3])
    grad = np.zeros((N, 4), dtype=np.complex128)
    wanted = None
    if pairs is not None:
        wanted = {}
        for k, l in pairs:
            wanted.setdefault(int(k), set()).add(int(l))
    for i in range(N):
        mem = latom[ptr[i]:ptr[i + 1]]
        nm = len(mem)
        if nm == 0 or (wanted is not None and not any(int(k) in wanted for k in mem)):
            continue
        P = lpos[ptr[i]:ptr[i + 1]]
        Wd, col, row = {}, {}, {}
        for tag, t, k in (("+", tp[mem], kp), ("-", tm[mem], km)):
            M = kkr.kkr_matrix(P, t, k)
            W = np.linalg.inv(M)
            tdiag = kkr.expand_t(t).reshape(-1)
            tau = W * tdiag[None, :]
            Wd[tag] = W.reshape(nm, nl, nm, nl)
            col[tag] = tau.reshape(nm, nl, nm, nl)[:, :, 0, :]   # tau^{a0}
            row[tag] = tau.reshape(nm, nl, nm, nl)[0, :, :, :].transpose(1, 0, 2)  # tau^{0a}
        Jc = J[species[i]]
        Jm = J[species[mem]]
        for e in ("+", "-"):
            W4 = Wd[e]
            for b in range(nm):
                for l in range(4):
                    if wanted is not None and l not in wanted.get(int(mem[b]), ()):
                        continue
                    chans = np.nonzero(lshell == l)[0]
                    # d tau^{a0} and d tau^{0a} for unit dt at (b, l), energy e
                    Wab = W4[:, :, b, chans]          # [a, L1, p]
                    W0b = W4[0, :, b, chans]          # [p, L2]  (fancy index moves p first)
                    dcol = np.einsum("aip,pj->aij", Wab, W0b)       # sum_p W_{(a,L1),p} W_{(0,L2),p}
                    drow = np.einsum("pi,ajp->aij", W0b, Wab)       # sum_p W_{(0,L1),p} W_{(a,L2),p}
                    dL = 0.0 + 0.0j
                    for c, (z1, z2) in enumerate(kubo.COMBOS):
                        c_rev = kubo.COMBO_INDEX[(z2, z1)]
                        for mu in range(3):
                            if w[c, mu] == 0.0:
                                continue
                            J0 = Jc[c_rev, mu]
                            Ja = Jm[:, c, mu]
                            ds = 0.0 + 0.0j
                            if z1 == e:
                                ds += np.trace(J0[None] @ drow @ Ja @ col[z2], axis1=1, axis2=2).sum()
                            if z2 == e:
                                ds += np.trace(J0[None] @ row[z1] @ Ja @ dcol, axis1=1, axis2=2).sum()
                            dL += w[c, mu] * ds
                    site = mem[b]
                    chain = dtp[site, l] if e == "+" else dtm[site, l]
                    grad[site, l] += dL * chain
    return grad
