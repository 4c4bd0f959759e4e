"""Resistivity and the LIZ-convergence workflow around the tau-solve + Kubo path.

* ``liz_sweep`` runs the whole GPU path (LIZ, tau solve, Kubo tensor) for each LIZ
  radius and inverts the conductivity tensor, rho = sigma^-1 (Sec. II.C).  With a
  second set of phase shifts (and currents) it treats the two channels of a
  collinear spin-polarized calculation separately and adds their conductivities
  before the inversion (Sec. IV, Fe-Si).
* ``fit_linear`` is Eq. (31) (rho linear in k = 1/(r_LIZ - r_c)); with r_c = 0 it is
  the lower-bound form of Eq. (34), and c1 is the value extrapolated to 1/r_LIZ -> 0.
* ``fit_upper`` is Eq. (32) / (33), rho = b0 / (1 + b1 exp(-2 alpha r_LIZ)) at a
  fixed 2 alpha (0.15 per angstrom for the upper bound); b0 is the extrapolated value.

Both fits minimise the squared error in rho.  The exponential one starts from the
least-squares line of sigma = 1/rho against exp(-2 alpha r) (Eq. (24)'s form, with
a1 = 1/b0 and a0 = b1/b0) and then takes damped Gauss-Newton steps.  Eq. (33) has
a plus sign before b1; figure captions that print b0 / (1 - b1 e^{-0.15 r}) give b1
with the opposite sign.  These are host computations on a handful of numbers.
"""

import math

import numpy as np

ANGSTROM_IN_BOHR = 1.0 / 0.529177210903
TWO_ALPHA_UPPER = 0.15 / ANGSTROM_IN_BOHR  # 2 alpha_max = 0.15 / angstrom, in 1 / bohr


def invert3(sigma):
    """rho = sigma^-1 for a 3 x 3 tensor, from the adjugate (cofactors / determinant)."""
    s = [[float(sigma[i][j]) for j in range(3)] for i in range(3)]
    cof = [[0.0] * 3 for _ in range(3)]
    for i in range(3):
        for j in range(3):
            r = [x for x in range(3) if x != i]
            c = [y for y in range(3) if y != j]
            minor = s[r[0]][c[0]] * s[r[1]][c[1]] - s[r[0]][c[1]] * s[r[1]][c[0]]
            cof[i][j] = minor if (i + j) % 2 == 0 else -minor
    det = s[0][0] * cof[0][0] + s[0][1] * cof[0][1] + s[0][2] * cof[0][2]
    if det == 0.0 or not math.isfinite(det):
        raise ValueError("conductivity tensor is singular")
    return np.array([[cof[j][i] / det for j in range(3)] for i in range(3)])


def _line(x, y):
    """Least-squares slope and intercept of y against x (centred sums)."""
    x = np.asarray(x, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    if x.size < 2:
        raise ValueError("a fit needs at least two LIZ radii")
    xm, ym = x.mean(), y.mean()
    sxx = float(((x - xm) ** 2).sum())
    if sxx == 0.0:
        raise ValueError("a fit needs two distinct LIZ radii")
    slope = float(((x - xm) * (y - ym)).sum()) / sxx
    return slope, float(ym - slope * xm)


def fit_linear(r_liz, rho, r_c=0.0):
    """Eq. (31) / (34): (c0, c1) with rho ~ c0 / (r_LIZ - r_c) + c1."""
    r = np.asarray(r_liz, dtype=np.float64)
    if np.any(r <= r_c):
        raise ValueError("every LIZ radius must exceed r_c")
    return _line(1.0 / (r - r_c), rho)


def upper_model(r_liz, b0, b1, two_alpha=TWO_ALPHA_UPPER):
    return b0 / (1.0 + b1 * np.exp(-two_alpha * np.asarray(r_liz, dtype=np.float64)))


def fit_upper(r_liz, rho, two_alpha=TWO_ALPHA_UPPER, max_iter=200):
    """Eq. (32) / (33): (b0, b1) with rho ~ b0 / (1 + b1 exp(-2 alpha r_LIZ))."""
    r = np.asarray(r_liz, dtype=np.float64)
    rho = np.asarray(rho, dtype=np.float64)
    e = np.exp(-two_alpha * r)
    a0, a1 = _line(e, 1.0 / rho)  # sigma = a1 + a0 e
    b = np.array([1.0 / a1, a0 / a1])

    def resid(b):
        return b[0] / (1.0 + b[1] * e) - rho

    f = resid(b)
    cost = float(f @ f)
    lam = 1e-3
    for _ in range(max_iter):
        d = 1.0 + b[1] * e
        Jm = np.stack([1.0 / d, -b[0] * e / d ** 2], axis=1)
        JtJ = Jm.T @ Jm
        g = Jm.T @ f
        step = None
        while lam < 1e12:
            A = JtJ + lam * np.diag(np.diag(JtJ))
            det = A[0, 0] * A[1, 1] - A[0, 1] * A[1, 0]
            cand = b - np.array([A[1, 1] * g[0] - A[0, 1] * g[1], A[0, 0] * g[1] - A[1, 0] * g[0]]) / det
            fc = resid(cand)
            cc = float(fc @ fc)
            if np.all(1.0 + cand[1] * e > 0) and cc <= cost:
                step = cand
                break
            lam *= 10.0
        if step is None:
            break
        done = np.all(np.abs(step - b) <= 1e-15 * np.maximum(np.abs(step), 1.0)) or cost - cc <= 1e-30 * max(cost, 1e-300)
        b, f, cost = step, fc, cc
        lam = max(lam / 10.0, 1e-12)
        if done:
            break
    return float(b[0]), float(b[1])


def liz_sweep(ctx, pos, cell, species, phase, J, e_fermi, eta, radii, volume, precision="fp64",
              phase_down=None, J_down=None):
    """Conductivity tensor and resistivity for each LIZ radius.

    pos [N,3], cell [3,3] or None, species [N], phase [N,4] (radians), J
    [n_species,4,3,16,16] complex, as for the Kubo entry points.  With ``phase_down``
    (and optionally ``J_down``, default ``J``) the second spin channel is solved too
    and sigma = sigma_up + sigma_down.  Returns one dict per radius: r_liz, liz_max,
    sigma [3,3], rho [3,3] and, spin-polarized, sigma_up and sigma_down.
    """
    import torch

    from .api import build_liz

    dev = ctx.device
    sp = torch.from_numpy(np.asarray(species, dtype=np.int32)).to(dev)
    channels = [(phase, J)]
    if phase_down is not None:
        channels.append((phase_down, J if J_down is None else J_down))
    channels = [(torch.from_numpy(np.ascontiguousarray(p, dtype=np.float64)).to(dev),
                 torch.from_numpy(np.ascontiguousarray(j, dtype=np.complex128)).to(dev)) for p, j in channels]
    out = []
    for r in radii:
        liz = build_liz(pos, cell, float(r))
        la, lp = liz.to_device(dev)
        sig_ch = []
        for ph, Jd in channels:
            tp, tm, info, _ = ctx.tau_solve(liz, la, lp, ph, e_fermi, eta, precision=precision)
            sig, _, _ = ctx.kubo_sigma_tensor(liz, la, tp, tm, sp, Jd, volume)
            if int((info != 0).sum()) != 0:
                raise RuntimeError("tau solve reported a singular KKR matrix at r_LIZ = %g" % r)
            sig_ch.append(sig.cpu().numpy())
            del tp, tm
        total = sig_ch[0] if len(sig_ch) == 1 else sig_ch[0] + sig_ch[1]
        rec = {"r_liz": float(r), "liz_max": int(np.diff(liz.ptr).max()), "sigma": total, "rho": invert3(total)}
        if len(sig_ch) == 2:
            rec["sigma_up"], rec["sigma_down"] = sig_ch
        out.append(rec)
    return out


def main(argv=None):
    """Command line: LIZ-radius sweep of one synthetic workload with both fits, one JSON line."""
    import argparse
    import json
    import time

    import torch

    from .api import Context

    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--workload", default="bcc250")
    ap.add_argument("--radii", default="0.95,1.2,1.5,1.7,1.9,2.2",
                    help="LIZ radii in units of the lattice constant (between shells)")
    ap.add_argument("--precision", default="split", choices=["split", "fp64"])
    ap.add_argument("--spin-scale", type=float, default=0.0,
                    help="if > 0, a second spin channel with phase shifts scaled by this factor")
    args = ap.parse_args(argv)
    import synthetic  # seeded inputs (repository root on the path)

    w = synthetic.workload(args.workload)
    radii = [float(x) * w["a"] for x in args.radii.split(",")]
    ctx = Context(0)
    t0 = time.perf_counter()
    recs = liz_sweep(ctx, w["pos"], w["cell"], w["species"], w["phase"], w["J"], w["e_fermi"], w["etas"][0], radii,
                     w["volume"], precision=args.precision,
                     phase_down=w["phase"] * args.spin_scale if args.spin_scale > 0 else None)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    ctx.close()
    r = [x["r_liz"] for x in recs]
    rho = [x["rho"][0][0] for x in recs]
    out = {"workload": args.workload, "precision": args.precision, "seconds": el,
           "radii_bohr": r, "liz_sites": [x["liz_max"] for x in recs], "rho_xx": rho,
           "sigma_xx": [x["sigma"][0][0] for x in recs]}
    if len(r) >= 2:
        out["lower_bound_fit"] = dict(zip(("c0", "c1"), fit_linear(r, rho)))
    if len(r) >= 3:
        out["upper_bound_fit"] = dict(zip(("b0", "b1"), fit_upper(r, rho)))
    print(json.dumps(out))


if __name__ == "__main__":
    main()
