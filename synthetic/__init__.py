"""Seeded synthetic inputs shaped like the paper's workloads.

This module only builds INPUT arrays (structures, species, phase shifts,
current matrix elements).  It holds none of the method's arithmetic: no
structure constants, no t-matrices, no solves, no traces.  Both the HIP
library's callers and the CPU oracle receive the same arrays from here.

The paper's own inputs (self-consistent potentials of Ag, Al, Li, V, AlV and
FeSi, 16,000-atom bcc / 16,384-atom fcc supercells, LIZ of ~1000 atoms) are
not available; these structures stand in for their shape: pure and random
binary fcc/bcc crystals, and a displaced, vacancy-bearing three-species bcc.

Units: bohr, Ry, radians.  Angular-momentum channels L = l*l + l + m, l <= 3.
"""

import math

import numpy as np
import scipy.special

LMAX = 3
NL = 16
BASE_SEED = 2311012134

FCC_BASIS = np.array([[0.0, 0.0, 0.0], [0.5, 0.5, 0.0], [0.5, 0.0, 0.5], [0.0, 0.5, 0.5]])
BCC_BASIS = np.array([[0.0, 0.0, 0.0], [0.5, 0.5, 0.5]])


def cubic_supercell(a, ncell, basis):
    """Positions of a cubic crystal: ncell^3 conventional cells of side a."""
    pos = []
    for i in range(ncell):
        for j in range(ncell):
            for k in range(ncell):
                for b in basis:
                    pos.append((np.array([i, j, k], dtype=np.float64) + b) * a)
    cell = np.eye(3) * (a * ncell)
    return np.asarray(pos), cell


def fcc_supercell(a, ncell):
    return cubic_supercell(a, ncell, FCC_BASIS)


def bcc_supercell(a, ncell):
    return cubic_supercell(a, ncell, BCC_BASIS)


def species_iid(n, probs, rng):
    """Each site draws its species independently with the given probabilities."""
    return rng.choice(len(probs), size=n, p=np.asarray(probs)).astype(np.int32)


def species_exact(counts, rng):
    """Exact species counts, placed by a seeded permutation."""
    lab = np.concatenate([np.full(c, s, dtype=np.int32) for s, c in enumerate(counts)])
    return lab[rng.permutation(len(lab))]


def _real_sph(lmax, theta, phi):
    """Real spherical harmonics (no Condon-Shortley phase) from scipy's complex ones."""
    out = np.zeros(theta.shape + ((lmax + 1) ** 2,))
    for l in range(lmax + 1):
        for m in range(-l, l + 1):
            am = abs(m)
            y = scipy.special.sph_harm_y(l, am, theta, phi)
            if m == 0:
                v = y.real
            elif m > 0:
                v = math.sqrt(2.0) * (-1) ** am * y.real
            else:
                v = math.sqrt(2.0) * (-1) ** am * y.imag
            out[..., l * l + l + m] = v
    return out


def dipole_angular(lmax=LMAX):
    """D[mu, L, L'] = integral of Y_L (r^_mu) Y_L' over the unit sphere, mu = x, y, z.

    Nonzero only for l' = l +- 1 (dipole selection rule).  Evaluated with a
    Gauss-Legendre x uniform product rule that is exact at these degrees.
    """
    nt, npp = lmax + 4, 2 * lmax + 6
    xt, wt = np.polynomial.legendre.leggauss(nt)
    th = np.arccos(xt)
    ph = 2.0 * math.pi * np.arange(npp) / npp
    TH, PH = np.meshgrid(th, ph, indexing="ij")
    W = np.outer(wt, np.full(npp, 2.0 * math.pi / npp))
    Y = _real_sph(lmax, TH, PH)
    rhat = np.stack([np.sin(TH) * np.cos(PH), np.sin(TH) * np.sin(PH), np.cos(TH)])
    D = np.einsum("tp,mtp,tpa,tpb->mab", W, rhat, Y, Y)
    D[np.abs(D) < 1e-14] = 0.0
    return D


DIPOLE_PAIRS = ((0, 1), (1, 0), (1, 2), (2, 1), (2, 3), (3, 2))


def current_matrices(n_species, rng, lmax=LMAX):
    """Synthetic current matrix elements J[s, c, mu, L, L'] (complex128).

    c enumerates the energy pair (zA, zB) as (+,+), (+,-), (-,+), (-,-).  For
    c in {(+,+), (+,-)} the block (l, l') of J^{s mu} is a seeded complex
    Gaussian amplitude a_{ll'} = (g1 + i g2)/sqrt(2) times the dipole angular
    factor sqrt(4 pi / 3) * D[mu] (so J is a vector operator obeying
    l' = l +- 1); amplitudes are drawn in the order species, c, (l, l') pair.
    The other two pairs follow by conjugation: J(-,-) = conj J(+,+) and
    J(-,+) = conj J(+,-).
    """
    D = dipole_angular(lmax) * math.sqrt(4.0 * math.pi / 3.0)
    lsh = np.array([int(math.isqrt(L)) for L in range((lmax + 1) ** 2)])
    J = np.zeros((n_species, 4, 3, NL, NL), dtype=np.complex128)
    for s in range(n_species):
        for c in (0, 1):
            amp = np.zeros((lmax + 1, lmax + 1), dtype=np.complex128)
            for (l1, l2) in DIPOLE_PAIRS:
                g = rng.standard_normal(2)
                amp[l1, l2] = (g[0] + 1j * g[1]) / math.sqrt(2.0)
            A = amp[lsh[:, None], lsh[None, :]]
            J[s, c] = A[None, :, :] * D
        J[s, 3] = np.conj(J[s, 0])
        J[s, 2] = np.conj(J[s, 1])
    return J


def _workload(name):
    """Definitions of the synthetic workloads (sizes follow the paper's kinds of systems)."""
    if name == "fcc32":
        idx = 1
        rng = np.random.default_rng(BASE_SEED + idx)
        a = 7.7
        pos, cell = fcc_supercell(a, 2)
        species = np.zeros(len(pos), dtype=np.int32)
        phase_sp = np.array([[0.9, 0.3, 0.05, 0.005]])
        J = current_matrices(1, rng)
        return dict(name=name, pos=pos, cell=cell, species=species, phase_species=phase_sp, J=J,
                    r_liz=1.1 * a, e_fermi=0.7, etas=(0.005,), lattice="fcc", a=a,
                    r_liz_literal="first 2 shells")
    if name in ("bcc250", "bcc250grad"):
        idx = 2 if name == "bcc250" else 5
        rng = np.random.default_rng(BASE_SEED + 2)
        a = 5.7
        pos, cell = bcc_supercell(a, 5)
        species = species_iid(len(pos), [0.5, 0.5], rng)
        phase_sp = np.array([[0.8, 0.2, 0.6, 0.01], [0.7, 0.25, 0.3, 0.01]])
        J = current_matrices(2, rng)
        return dict(name=name, pos=pos, cell=cell, species=species, phase_species=phase_sp, J=J,
                    r_liz=2.2 * a, e_fermi=0.65, etas=(0.002,), lattice="bcc", a=a,
                    r_liz_literal="1.5a", config_index=idx)
    if name == "fcc4000":
        rng = np.random.default_rng(BASE_SEED + 3)
        a = 7.6
        pos, cell = fcc_supercell(a, 10)
        species = species_exact([1000, 3000], rng)
        phase_sp = np.array([[0.8, 0.2, 0.6, 0.01], [0.7, 0.25, 0.3, 0.01]])
        J = current_matrices(2, rng)
        return dict(name=name, pos=pos, cell=cell, species=species, phase_species=phase_sp, J=J,
                    r_liz=1.95 * a, e_fermi=0.7, etas=(0.005, 0.002, 0.001), lattice="fcc", a=a,
                    r_liz_literal="LIZ 135 atoms")
    if name == "bcc1940":
        rng = np.random.default_rng(BASE_SEED + 4)
        a = 5.7
        pos, cell = bcc_supercell(a, 10)
        pos = pos + rng.normal(0.0, 0.05 * a, size=pos.shape)
        keep = np.sort(rng.permutation(len(pos))[60:])
        pos = pos[keep]
        species = species_exact([776, 776, 388], rng)
        lo = np.array([0.6, 0.15, 0.05, 0.002])
        hi = np.array([1.0, 0.35, 0.7, 0.02])
        phase_sp = lo + (hi - lo) * rng.random((3, 4))
        J = current_matrices(3, rng)
        return dict(name=name, pos=pos, cell=cell, species=species, phase_species=phase_sp, J=J,
                    r_liz=2.2 * a, e_fermi=0.7, etas=(0.003,), lattice="bcc-disordered", a=a,
                    r_liz_literal="1.6a")
    if name == "bcc16000":
        # the paper's large-LIZ setting (Sec. III: 16,000-atom bcc, ~1000-atom LIZ): random
        # binary bcc alloy, 20x20x20 cells, LIZ radius 4.9a (965 members, n = 15440)
        rng = np.random.default_rng(BASE_SEED + 7)
        a = 5.7
        pos, cell = bcc_supercell(a, 20)
        species = species_iid(len(pos), [0.5, 0.5], rng)
        phase_sp = np.array([[0.8, 0.2, 0.6, 0.01], [0.7, 0.25, 0.3, 0.01]])
        J = current_matrices(2, rng)
        return dict(name=name, pos=pos, cell=cell, species=species, phase_species=phase_sp, J=J,
                    r_liz=4.9 * a, e_fermi=0.65, etas=(0.002,), lattice="bcc", a=a,
                    r_liz_literal="approximately a 1000-atom LIZ")
    if name == "bcc16":
        # small random binary bcc alloy for exhaustive checks (2x2x2 cells, LIZ 27)
        rng = np.random.default_rng(BASE_SEED + 6)
        a = 5.7
        pos, cell = bcc_supercell(a, 2)
        species = species_iid(len(pos), [0.5, 0.5], rng)
        phase_sp = np.array([[0.8, 0.2, 0.6, 0.01], [0.7, 0.25, 0.3, 0.01]])
        J = current_matrices(2, rng)
        return dict(name=name, pos=pos, cell=cell, species=species, phase_species=phase_sp, J=J,
                    r_liz=1.5 * a, e_fermi=0.65, etas=(0.002,), lattice="bcc", a=a,
                    r_liz_literal="1.5a")
    raise KeyError(name)


WORKLOADS = ("fcc32", "bcc250", "fcc4000", "bcc1940", "bcc250grad", "bcc16", "bcc16000")


def workload(name):
    """Return the seeded workload dict; ``phase`` is per atom [N, 4] (from its species)."""
    w = _workload(name)
    w["phase"] = w["phase_species"][w["species"]]
    w["volume"] = abs(float(np.linalg.det(w["cell"])))
    return w


def fingerprint(w, keys=("pos", "cell", "species", "phase", "J", "r_liz", "e_fermi", "etas")):
    """sha256 over a workload's input arrays, so a stored expected value can tell whether it
    still belongs to the inputs these generators produce."""
    import hashlib
    h = hashlib.sha256()
    for k in keys:
        v = np.ascontiguousarray(np.asarray(w[k]))
        h.update(k.encode())
        h.update(str(v.dtype).encode())
        h.update(str(v.shape).encode())
        h.update(v.tobytes())
    return h.hexdigest()
