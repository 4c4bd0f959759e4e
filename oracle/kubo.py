"""Kubo-Greenwood conductivity in multiple-scattering form.

Part of the test oracle (test infrastructure only; see ``oracle/__init__``).

Eq. (10) (LSMS form): for every atom m and every member n of its LIZ,
    sum_{L1..L4} J^{m mu}_{L4 L1}(z2, z1) tau^{mn}_{L1 L2}(z1)
                 J^{n nu}_{L2 L3}(z1, z2) tau^{nm}_{L3 L4}(z2)
  = Tr[ J^{m mu}(z2, z1) tau^{mn}(z1) J^{n nu}(z1, z2) tau^{nm}(z2) ],
and sigma~(z1, z2) = -(4 m_e^2 / (pi N Omega hbar^3)) * (sum over m, n).
Eq. (7): sigma = 1/4 [sigma~(+,+) - sigma~(+,-) - sigma~(-,+) + sigma~(-,-)].

Readings (the paper gives no numbers for these): Rydberg units make
4 m_e^2 / hbar^3 = 1, N Omega is the supercell volume V, the limit
delta -> 0 of Eq. (7) is replaced by the finite broadening eta of the inputs,
the ensemble average is the single seeded structure (as Sec. II.B does).
``atom_traces`` forms the diagonal mu = nu; ``atom_traces_tensor`` all nine
(mu, nu), with mu on the centre atom's current J^{m mu}(z2, z1) and nu on the
member's J^{n nu}(z1, z2), as Eq. (10) places them.

Index conventions: combo c enumerates (z1, z2) as (+,+), (+,-), (-,+), (-,-);
J[s, c, mu] holds J^{s mu}(zA, zB) for the pair (zA, zB) of combo c; mu = x, y, z.
"""

import numpy as np

from . import kkr, liz

COMBOS = (("+", "+"), ("+", "-"), ("-", "+"), ("-", "-"))
COMBO_INDEX = {c: i for i, c in enumerate(COMBOS)}
SIGNS = (1.0, -1.0, -1.0, 1.0)


def atom_traces(tau, J, sp_center, sp_members):
    """Per-atom sums s[c, mu] = sum_a Tr[J^0(z2,z1) tau^{0a}(z1) J^a(z1,z2) tau^{a0}(z2)].

    tau: dict from ``kkr.atom_tau`` (row/col blocks at both energies, read directly,
    no symmetry used).  Returns complex [4, 3].
    """
    s = np.zeros((4, 3), dtype=np.complex128)
    for c, (z1, z2) in enumerate(COMBOS):
        c_rev = COMBO_INDEX[(z2, z1)]
        row1 = tau["row" + z1]  # tau^{0a}(z1), [members, NL, NL]
        col2 = tau["col" + z2]  # tau^{a0}(z2)
        for mu in range(3):
            J0 = J[sp_center, c_rev, mu]
            Ja = J[sp_members, c, mu]  # [members, NL, NL]
            prod = J0[None, :, :] @ row1 @ Ja @ col2
            s[c, mu] = np.trace(prod, axis1=1, axis2=2).sum()
    return s


def atom_traces_tensor(tau, J, sp_center, sp_members):
    """Per-atom sums s[c, mu, nu] = sum_a Tr[J^{0 mu}(z2,z1) tau^{0a}(z1) J^{a nu}(z1,z2) tau^{a0}(z2)].

    Same inputs as ``atom_traces``; returns complex [4, 3, 3].
    """
    s = np.zeros((4, 3, 3), dtype=np.complex128)
    for c, (z1, z2) in enumerate(COMBOS):
        c_rev = COMBO_INDEX[(z2, z1)]
        row1 = tau["row" + z1]
        col2 = tau["col" + z2]
        for mu in range(3):
            J0 = J[sp_center, c_rev, mu]
            for nu in range(3):
                Ja = J[sp_members, c, nu]
                prod = J0[None, :, :] @ row1 @ Ja @ col2
                s[c, mu, nu] = np.trace(prod, axis1=1, axis2=2).sum()
    return s


def sigma_tilde(trace_sum, volume):
    """sigma~[c, mu] = -(1 / (pi V)) * sum over atoms of s[c, mu]."""
    return -np.asarray(trace_sum) / (np.pi * volume)


def combine(st):
    """Eq. (7) at finite eta: sigma[...] = 1/4 sum_c sign_c sigma~[c, ...] (complex; any trailing shape)."""
    st = np.asarray(st)
    return 0.25 * (st[0] - st[1] - st[2] + st[3])


def supercell_volume(cell):
    return abs(float(np.linalg.det(np.asarray(cell, dtype=np.float64))))


def sigma(pos, cell, r_liz, species, phase, J, e_fermi, eta, volume=None, atoms=None, liz_lists=None,
          tensor=False):
    """Conductivity of a structure from Eq. (10) and Eq. (7).

    pos [N,3], cell [3,3] or None, species [N] int, phase [N, 4] radians,
    J [n_species, 4, 3, NL, NL] complex.  ``atoms`` restricts the outer sum
    (per-atom results are still returned for those atoms only).
    Returns dict: sigma [3] complex, sigma_tilde [4,3], per_atom {i: s[4,3]},
    and the tau blocks per atom under 'tau'.  With ``tensor`` the trailing
    [3] becomes [3, 3] (mu, nu).
    """
    pos = np.asarray(pos, dtype=np.float64)
    N = pos.shape[0]
    if volume is None:
        volume = supercell_volume(cell)
    if liz_lists is None:
        liz_lists = liz.build_liz(pos, cell, r_liz, centres=atoms)
    ptr, latom, lpos = liz_lists
    zp, zm, kp, km = kkr.energies(e_fermi, eta)
    tp, tm = kkr.t_matrix(phase, kp)
    species = np.asarray(species)
    per_atom = {}
    taus = {}
    total = np.zeros((4, 3, 3) if tensor else (4, 3), dtype=np.complex128)
    for i in (range(N) if atoms is None else atoms):
        mem = latom[ptr[i]:ptr[i + 1]]
        P = lpos[ptr[i]:ptr[i + 1]]
        tau = kkr.atom_tau(P, tp[mem], tm[mem], kp, km)
        s = (atom_traces_tensor if tensor else atom_traces)(tau, J, species[i], species[mem])
        per_atom[i] = s
        taus[i] = tau
        total += s
    st = sigma_tilde(total, volume)
    return {"sigma": combine(st), "sigma_tilde": st, "per_atom": per_atom, "tau": taus,
            "liz": liz_lists, "volume": volume}


def sigma_all_sites(pos, species, phase, J, e_fermi, eta, volume, tensor=False):
    """Eq. (9) for an open cluster: one inverse over all sites, sum over all m, n.

    tau = (T^-1 - g)^-1 over the whole cluster (evaluated as (1 - T g)^-1 T) and
    sigma~ = -(1/(pi V)) sum_{m,n} Tr[J^{m mu}(z2,z1) tau^{mn}(z1) J^{n nu}(z1,z2) tau^{nm}(z2)],
    for mu = nu, or for all (mu, nu) with ``tensor``.
    """
    pos = np.asarray(pos, dtype=np.float64)
    N = pos.shape[0]
    nl = kkr.NL
    zp, zm, kp, km = kkr.energies(e_fermi, eta)
    tp, tm = kkr.t_matrix(phase, kp)
    full = {}
    for tag, t, k in (("+", tp, kp), ("-", tm, km)):
        M = kkr.kkr_matrix(pos, t, k)
        tdiag = kkr.expand_t(t).reshape(-1)
        tau = np.linalg.inv(M) * tdiag[None, :]
        full[tag] = tau.reshape(N, nl, N, nl)
    pairs = [(mu, nu) for mu in range(3) for nu in range(3)] if tensor else [(mu, mu) for mu in range(3)]
    total = np.zeros((4, 3, 3) if tensor else (4, 3), dtype=np.complex128)
    for c, (z1, z2) in enumerate(COMBOS):
        c_rev = COMBO_INDEX[(z2, z1)]
        for mu, nu in pairs:
            acc = 0.0 + 0.0j
            for m in range(N):
                for n in range(N):
                    acc += np.trace(J[species[m], c_rev, mu] @ full[z1][m, :, n, :]
                                    @ J[species[n], c, nu] @ full[z2][n, :, m, :])
            total[(c, mu, nu) if tensor else (c, mu)] = acc
    st = sigma_tilde(total, volume)
    return {"sigma": combine(st), "sigma_tilde": st}
