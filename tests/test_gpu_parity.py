"""GPU parity of the HIP path (through the C ABI) against the FP64 CPU oracle.

Tolerances: FP64 mode 1e-10 relative (tau per atom in Frobenius norm, sigma and the
per-atom Kubo sums); split mode (FP32 trailing updates + FP64 refinement) 1e-8.
"""

import numpy as np
import pytest

import synthetic
from oracle import kkr, kubo
from oracle import liz as oliz

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL64 = 1e-10
TOL_SPLIT = 1e-8


@pytest.fixture(scope="module")
def lctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2311_12134_amd as P
    c = P.Context(0)
    yield c
    c.close()


def _run(lctx, w, eta, precision="fp64", per_atom=True, refine_tol=1e-14, max_refine=10):
    import paper_2311_12134_amd as P
    print("[gpu] workload=%s eta=%g precision=%s" % (w["name"], eta, precision), flush=True)
    liz = P.build_liz(w["pos"], w["cell"], w["r_liz"])
    dev = torch.device("cuda", 0)
    la, lp = liz.to_device(dev)
    phase = torch.from_numpy(np.ascontiguousarray(w["phase"])).to(dev)
    species = torch.from_numpy(w["species"].astype(np.int32)).to(dev)
    J = torch.from_numpy(np.ascontiguousarray(w["J"])).to(dev)
    tp, tm, info, berr = lctx.tau_solve(liz, la, lp, phase, w["e_fermi"], eta, precision=precision,
                                        refine_tol=refine_tol, max_refine=max_refine)
    sig, st, pa = lctx.kubo_sigma(liz, la, tp, tm, species, J, w["volume"], per_atom=per_atom)
    torch.cuda.synchronize()
    return dict(liz=liz, tau_plus=tp.cpu().numpy(), tau_minus=tm.cpu().numpy(), info=info.cpu().numpy(),
                berr=berr.cpu().numpy(), sigma=sig.cpu().numpy(), sigma_tilde=st.cpu().numpy(),
                per_atom=None if pa is None else pa.cpu().numpy())


def _oracle_liz(w, liz, centres=None, r_liz=None):
    """The oracle's own LIZ lists (Sec. II.A, Fig. 1), built from the structure alone for the
    checked centres (None: every atom).  The library's lists must be identical for those
    centres -- the same members in the same order with the same displacements -- because the
    tau blocks are compared member by member; the oracle never sees the library's lists."""
    r = w["r_liz"] if r_liz is None else r_liz
    o = oliz.build_liz(w["pos"], w["cell"], r, centres=centres)
    optr, oatom, opos = o
    for i in (range(liz.n_atoms) if centres is None else centres):
        a, b, c, d = int(liz.ptr[i]), int(liz.ptr[i + 1]), int(optr[i]), int(optr[i + 1])
        assert b - a == d - c, "LIZ of atom %d: %d members, oracle %d" % (i, b - a, d - c)
        assert np.array_equal(liz.atom[a:b], oatom[c:d]), "LIZ of atom %d: member atoms differ" % i
        assert np.array_equal(liz.pos[a:b], opos[c:d]), "LIZ of atom %d: displacements differ" % i
    return o


def _oracle_atoms(w, eta, atoms, liz, tensor=False):
    return kubo.sigma(w["pos"], w["cell"], w["r_liz"], w["species"], w["phase"], w["J"], w["e_fermi"], eta,
                      atoms=atoms, liz_lists=_oracle_liz(w, liz, atoms), tensor=tensor)


def _check_atoms(g, o, atoms, tol):
    ptr = g["liz"].ptr
    worst = 0.0
    for i in atoms:
        sl = slice(ptr[i], ptr[i + 1])
        for tag, key in (("+", "tau_plus"), ("-", "tau_minus")):
            ref = o["tau"][i]["col" + tag]
            got = g[key][sl]
            err = np.linalg.norm(got - ref) / np.linalg.norm(ref)
            worst = max(worst, err)
            assert err <= tol, "atom %d tau%s rel err %.3e" % (i, tag, err)
        ref = o["per_atom"][i]
        got = g["per_atom"][i]
        err = np.abs(got - ref).max() / np.abs(ref).max()
        assert err <= tol, "atom %d Kubo sum rel err %.3e" % (i, err)
    return worst


def test_fcc32_fp64_full(lctx):
    w = synthetic.workload("fcc32")
    eta = w["etas"][0]
    g = _run(lctx, w, eta)
    assert (g["info"] == 0).all()
    atoms = list(range(32))
    o = _oracle_atoms(w, eta, atoms, g["liz"])
    _check_atoms(g, o, atoms, TOL64)
    ref_sig = o["sigma"].real
    assert np.allclose(g["sigma"], ref_sig, rtol=TOL64, atol=0)
    assert np.allclose(g["sigma_tilde"], o["sigma_tilde"], rtol=TOL64, atol=TOL64 * np.abs(o["sigma_tilde"]).max())


def test_bcc16_fp64_full(lctx):
    w = synthetic.workload("bcc16")
    eta = w["etas"][0]
    g = _run(lctx, w, eta)
    assert (g["info"] == 0).all()
    atoms = list(range(16))
    o = _oracle_atoms(w, eta, atoms, g["liz"])
    _check_atoms(g, o, atoms, TOL64)
    assert np.allclose(g["sigma"], o["sigma"].real, rtol=TOL64, atol=0)


def test_bcc16_split_full(lctx):
    w = synthetic.workload("bcc16")
    eta = w["etas"][0]
    g = _run(lctx, w, eta, precision="split")
    assert (g["info"] == 0).all(), g["info"]
    assert (g["berr"] <= 1e-14).all()
    atoms = list(range(16))
    o = _oracle_atoms(w, eta, atoms, g["liz"])
    _check_atoms(g, o, atoms, TOL_SPLIT)
    assert np.allclose(g["sigma"], o["sigma"].real, rtol=TOL_SPLIT, atol=0)


@pytest.mark.parametrize("precision,tol", [("fp64", TOL64), ("split", TOL_SPLIT)])
def test_bcc250_sampled(lctx, precision, tol):
    w = synthetic.workload("bcc250")
    eta = w["etas"][0]
    g = _run(lctx, w, eta, precision=precision)
    assert (g["info"] == 0).all()
    atoms = [0, 77, 249]
    o = _oracle_atoms(w, eta, atoms, g["liz"])
    _check_atoms(g, o, atoms, tol)


def test_bcc1940_uneven_sampled(lctx):
    w = synthetic.workload("bcc1940")
    eta = w["etas"][0]
    g = _run(lctx, w, eta)
    assert (g["info"] == 0).all()
    sizes = np.diff(g["liz"].ptr)
    atoms = [int(np.argmin(sizes)), int(np.argmax(sizes)), 1000]
    o = _oracle_atoms(w, eta, atoms, g["liz"])
    _check_atoms(g, o, atoms, TOL64)


def test_deterministic(lctx):
    w = synthetic.workload("bcc16")
    a = _run(lctx, w, w["etas"][0])
    b = _run(lctx, w, w["etas"][0])
    assert np.array_equal(a["tau_plus"], b["tau_plus"]) and np.array_equal(a["sigma"], b["sigma"])


def test_nan_phase_flags_input(lctx):
    w = dict(synthetic.workload("bcc16"))
    ph = w["phase"].copy()
    ph[3, 2] = np.nan
    w["phase"] = ph
    g = _run(lctx, w, w["etas"][0], per_atom=False)
    # every LIZ that contains atom 3 is flagged
    ptr, atom = g["liz"].ptr, g["liz"].atom
    for i in range(16):
        has = 3 in atom[ptr[i]:ptr[i + 1]]
        assert (g["info"][i] == -2).all() == has


def test_batched_lu_solve_random_and_singular(lctx):
    rng = np.random.default_rng(7)
    dev = torch.device("cuda", 0)
    sizes = [1, 17, 64, 100, 300, 129]
    mats, rhs, refs = [], [], []
    for n in sizes:
        A = rng.normal(size=(n, n)) + 1j * rng.normal(size=(n, n)) + 2 * np.eye(n)
        B = rng.normal(size=(n, 5)) + 1j * rng.normal(size=(n, 5))
        refs.append(np.linalg.solve(A, B))
        mats.append(torch.from_numpy(A).to(dev))
        rhs.append(torch.from_numpy(B).to(dev))
    # a singular system: column 40 of a 100 x 100 matrix is zero
    S = rng.normal(size=(100, 100)) + 0j
    S[:, 40] = 0.0
    mats.append(torch.from_numpy(S).to(dev))
    rhs.append(torch.from_numpy(np.ones((100, 5), dtype=complex)).to(dev))
    info = lctx.batched_lu_solve(mats, rhs).cpu().numpy()
    torch.cuda.synchronize()
    for k, ref in enumerate(refs):
        got = rhs[k].cpu().numpy()
        assert info[k] == 0
        assert np.abs(got - ref).max() <= 1e-10 * np.abs(ref).max(), (sizes[k], np.abs(got - ref).max())
    assert info[-1] > 0


@pytest.mark.parametrize("tiling", list(range(21)))
def test_split_lu_every_gemm_tiling(lctx, tiling):
    """FP32 factors without refinement, uneven batch whose trailing blocks end on 64-row and
    64-column halves of the 128-wide tiles: every tiling of the split-mode update must give
    a solve accurate to FP32 rounding (refinement would otherwise hide a wrong update)."""
    rng = np.random.default_rng(11)
    dev = torch.device("cuda", 0)
    sizes = [1000, 700, 450, 129, 1]
    mats, rhs, refs = [], [], []
    for n in sizes:
        A = (rng.normal(size=(n, n)) + 1j * rng.normal(size=(n, n))) / np.sqrt(n) + 2 * np.eye(n)
        B = rng.normal(size=(n, 3)) + 1j * rng.normal(size=(n, 3))
        refs.append(np.linalg.solve(A, B))
        mats.append(torch.from_numpy(A).to(dev))
        rhs.append(torch.from_numpy(B).to(dev))
    lctx.set_gemm_tiling(tiling)
    try:
        assert lctx.gemm_tiling() == tiling
        info = lctx.batched_lu_solve(mats, rhs, precision="split").cpu().numpy()
    finally:
        lctx.set_gemm_tiling(-1)
    torch.cuda.synchronize()
    for k, ref in enumerate(refs):
        got = rhs[k].cpu().numpy()
        assert info[k] == 0
        err = np.abs(got - ref).max() / np.abs(ref).max()
        assert err <= 2e-5, (tiling, sizes[k], err)


def _random_systems(seed, sizes, scale_diag=2.0):
    rng = np.random.default_rng(seed)
    dev = torch.device("cuda", 0)
    mats, rhs, refs = [], [], []
    for n in sizes:
        A = (rng.normal(size=(n, n)) + 1j * rng.normal(size=(n, n))) / np.sqrt(n) + scale_diag * np.eye(n)
        B = rng.normal(size=(n, 3)) + 1j * rng.normal(size=(n, 3))
        refs.append(np.linalg.solve(A, B))
        mats.append(torch.from_numpy(A).to(dev))
        rhs.append(torch.from_numpy(B).to(dev))
    return mats, rhs, refs


@pytest.mark.parametrize("knob,nv", [("f64_wide", 6), ("f64_narrow", 6), ("f32_narrow", 21)])
def test_lu_every_update_tiling(lctx, knob, nv):
    """Every tiling of the FP64 wide and narrow trailing updates (FP64 solve to 1e-10) and of
    the split-mode narrow update (FP32 factors without refinement, to FP32 rounding) on an
    uneven batch whose trailing blocks end on 64-row halves of the 128-wide tiles."""
    sizes = [1000, 700, 450, 129, 1]
    precision = "split" if knob.startswith("f32") else "fp64"
    tol = 2e-5 if precision == "split" else 1e-10
    print("[gpu] every tiling of %s" % knob, flush=True)
    for v in range(nv):
        mats, rhs, refs = _random_systems(13 + v, sizes)
        lctx.set_knob(knob, v)
        try:
            assert lctx.knob(knob) == v
            info = lctx.batched_lu_solve(mats, rhs, precision=precision).cpu().numpy()
        finally:
            lctx.set_knob(knob, -1)
        torch.cuda.synchronize()
        for k, ref in enumerate(refs):
            assert info[k] == 0
            err = np.abs(rhs[k].cpu().numpy() - ref).max() / np.abs(ref).max()
            assert err <= tol, (knob, v, sizes[k], err)


class _groups:
    """Panels per group of both LUs set for a block (restored to the defaults after)."""

    def __init__(self, lctx, group):
        self.lctx, self.group = lctx, group

    def __enter__(self):
        self.lctx.set_knob("group_f32", self.group)
        self.lctx.set_knob("group_f64", self.group)
        assert self.lctx.knob("group_f32") == self.group and self.lctx.knob("group_f64") == self.group

    def __exit__(self, *exc):
        self.lctx.set_knob("group_f32", -1)
        self.lctx.set_knob("group_f64", -1)


@pytest.mark.parametrize("group", [2, 3, 4])
@pytest.mark.parametrize("precision", ["fp64", "split"])
def test_lu_groups_random_systems(lctx, precision, group):
    """Two, three and four panels per group on one uneven batch whose matrices end on every
    panel of a last group (1024, 960, 896, 832 rows and sizes off the 64 grid), against numpy:
    FP64 to 1e-10, FP32 factors without refinement to FP32 rounding; and a singular system
    (zero column 200) reported at its column."""
    sizes = [1024, 960, 896, 832, 700, 450, 129, 1]
    tol = 2e-5 if precision == "split" else 1e-10
    print("[gpu] groups of %d panels, %s" % (group, precision), flush=True)
    mats, rhs, refs = _random_systems(23 + group, sizes)
    S = np.random.default_rng(5).normal(size=(300, 300)) + 0j
    S[:, 200] = 0.0
    mats.append(torch.from_numpy(S).to("cuda"))
    rhs.append(torch.from_numpy(np.ones((300, 3), dtype=complex)).to("cuda"))
    with _groups(lctx, group):
        info = lctx.batched_lu_solve(mats, rhs, precision=precision).cpu().numpy()
    torch.cuda.synchronize()
    for k, ref in enumerate(refs):
        assert info[k] == 0
        err = np.abs(rhs[k].cpu().numpy() - ref).max() / np.abs(ref).max()
        assert err <= tol, (precision, group, sizes[k], err)
    assert info[-1] == 201


@pytest.mark.parametrize("case", ["bcc16_split", "fcc32_fp64", "bcc1940_split", "tournament_bcc250_split",
                                  "tournament_bcc1940_split", "adjoint_bcc16", "lookahead_bcc250_split",
                                  "graph_fcc32_split", "ldlt_bcc250", "conj_fcc32_split"])
@pytest.mark.parametrize("group", [3, 4])
def test_groups_end_to_end(lctx, group, case):
    """The end-to-end parity tests against the oracle (and the bitwise schedule tests) with
    three and four panels per group in both LUs: tau solves, tournament panels (whose left
    columns then span up to three panels), the adjoint's transposed solves, the look-ahead
    stream, graph replay, the symmetric form and the z+/z- symmetry."""
    print("[gpu] groups of %d panels: %s" % (group, case), flush=True)
    run = {
        "bcc16_split": lambda: test_bcc16_split_full(lctx),
        "fcc32_fp64": lambda: test_fcc32_fp64_full(lctx),
        "bcc1940_split": lambda: test_bcc1940_uneven_sampled(lctx),
        "tournament_bcc250_split": lambda: test_tournament_panels_vs_oracle(lctx, "bcc250", "split", 128, TOL_SPLIT),
        "tournament_bcc1940_split": lambda: test_tournament_panels_vs_oracle(lctx, "bcc1940", "split", 192,
                                                                             TOL_SPLIT),
        "adjoint_bcc16": lambda: test_adjoint_bcc16_vs_oracle_and_fd(lctx),
        "lookahead_bcc250_split": lambda: test_lookahead_matches_single_stream(lctx, "bcc250", "split", 2048),
        "graph_fcc32_split": lambda: test_graph_replay_matches_eager(lctx, "fcc32", "split"),
        "ldlt_bcc250": lambda: test_symmetric_ldlt_vs_oracle(lctx, "bcc250", 2048),
        "conj_fcc32_split": lambda: test_conj_symmetry_mode(lctx, "fcc32", "split", TOL_SPLIT),
    }[case]
    with _groups(lctx, group):
        run()


@pytest.mark.parametrize("rows", [0, 256, 512, 768])
def test_split_panel_variant_threshold(lctx, rows):
    """The split-mode panel's small-workgroup variant used up to 0, 256, 512 or 768 rows on a
    batch of sizes up to 2300 (its panels run through every row-slot count of both variants):
    the same solves to FP32 rounding."""
    mats, rhs, refs = _random_systems(17, [2300, 1800, 1000, 450, 129])
    lctx.set_knob("panel_small_rows", rows)
    try:
        info = lctx.batched_lu_solve(mats, rhs, precision="split").cpu().numpy()
    finally:
        lctx.set_knob("panel_small_rows", -1)
    torch.cuda.synchronize()
    for k, ref in enumerate(refs):
        assert info[k] == 0
        assert np.abs(rhs[k].cpu().numpy() - ref).max() <= 2e-5 * np.abs(ref).max(), (rows, k)


def test_autotuned_choices_per_bucket_at_parity(tmp_path):
    """The autotuner on the disordered 1940-atom bcc workload's two npad buckets (LIZ of
    74-94 sites: padded sizes 1216-1536) for every target; the waves then take each bucket's
    choices, and sampled atoms of every size in both precisions match the oracle.  The table
    survives a save / load round trip through the tuning cache, and a fresh context reads it
    from LSMS_TUNE_CACHE."""
    import os
    import paper_2311_12134_amd as P
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    ctx = P.Context(0)
    try:
        w = synthetic.workload("bcc1940")
        eta = w["etas"][0]
        liz = P.build_liz(w["pos"], w["cell"], w["r_liz"])
        npads = sorted({int(-(-16 * n // 64) * 64) for n in np.diff(liz.ptr)})
        buckets = sorted({(n - 1) // 256 for n in npads})
        assert len(buckets) == 2
        print("[gpu] autotune bcc1940 buckets %s" % buckets, flush=True)
        for b in buckets:
            npad = max(n for n in npads if (n - 1) // 256 == b)
            for what in ("f32_wide", "f32_narrow", "f64_wide", "f64_narrow"):
                best, ms = ctx.autotune_kernel(what, npad, batch=64)
                # the fastest, or the default within 1 % of it
                assert ms[best] <= 1.01 * min(ms) and ctx.tuning_table(what)[b] == best
        thr, ms = ctx.autotune_kernel("f32_panel", batch=64)
        assert thr in (0, 256, 512, 768) and ctx.tuning_table("f32_panel") == thr
        assert len(ms) == 6 and all(m > 0 for m in ms)
        la, lp, phase, species, J = _device_inputs(w, liz)
        sizes = np.diff(liz.ptr)
        atoms = sorted({int(np.argmin(sizes)), int(np.argmax(sizes)), 1000,
                        int(np.nonzero(sizes == np.median(sizes))[0][0])})
        o = _oracle_atoms(w, eta, atoms, liz)
        for precision, tol in (("split", TOL_SPLIT), ("fp64", TOL64)):
            tp, tm, info, _ = ctx.tau_solve(liz, la, lp, phase, w["e_fermi"], eta, precision=precision)
            _, _, pa = ctx.kubo_sigma(liz, la, tp, tm, species, J, w["volume"], per_atom=True)
            torch.cuda.synchronize()
            assert (info.cpu().numpy() == 0).all()
            pa = pa.cpu().numpy()
            for i in atoms:
                sl = slice(int(liz.ptr[i]), int(liz.ptr[i + 1]))
                for tag, t in (("+", tp), ("-", tm)):
                    ref = o["tau"][i]["col" + tag]
                    err = np.linalg.norm(t[sl].cpu().numpy() - ref) / np.linalg.norm(ref)
                    assert err <= tol, (precision, i, tag, err)
                assert np.abs(pa[i] - o["per_atom"][i]).max() <= tol * np.abs(o["per_atom"][i]).max()
        path = tmp_path / "tune.txt"
        ctx.tuning_save(path)
        tables = {what: ctx.tuning_table(what) for what in ("f32_wide", "f32_narrow", "f64_wide", "f64_narrow")}
        os.environ["LSMS_TUNE_CACHE"] = str(path)
        try:
            ctx2 = P.Context(0)
        finally:
            del os.environ["LSMS_TUNE_CACHE"]
        try:
            for what, tab in tables.items():
                assert np.array_equal(ctx2.tuning_table(what), tab), what
            assert ctx2.tuning_table("f32_panel") == thr
        finally:
            ctx2.close()
    finally:
        ctx.close()


def _grad_setup(w):
    import paper_2311_12134_amd as P
    dev = torch.device("cuda", 0)
    liz = P.build_liz(w["pos"], w["cell"], w["r_liz"])
    la, lp = liz.to_device(dev)
    species = torch.from_numpy(w["species"].astype(np.int32)).to(dev)
    J = torch.from_numpy(np.ascontiguousarray(w["J"])).to(dev)
    return liz, la, lp, species, J


def _gpu_sigma(lctx, w, liz, la, lp, species, J, phase_np, eta):
    dev = torch.device("cuda", 0)
    ph = torch.from_numpy(np.ascontiguousarray(phase_np)).to(dev)
    tp, tm, info, _ = lctx.tau_solve(liz, la, lp, ph, w["e_fermi"], eta)
    sig, _, _ = lctx.kubo_sigma(liz, la, tp, tm, species, J, w["volume"])
    return sig.cpu().numpy()


def test_adjoint_bcc16_vs_oracle_and_fd(lctx):
    import paper_2311_12134_amd as P
    from oracle import adjoint
    w = synthetic.workload("bcc16")
    eta = w["etas"][0]
    liz, la, lp, species, J = _grad_setup(w)
    dsig = np.array([1.0, -0.5, 0.25])
    ph = torch.from_numpy(np.ascontiguousarray(w["phase"])).to(torch.device("cuda", 0)).requires_grad_(True)
    sig = P.KuboSigma.apply(ph, lctx, liz, la, lp, species, J, w["volume"], w["e_fermi"], eta)
    sig.backward(torch.from_numpy(dsig).to(sig.device))
    g = ph.grad.cpu().numpy()
    ref = adjoint.dsigma_dphase(w["pos"], w["cell"], w["r_liz"], w["species"], w["phase"], w["J"], w["e_fermi"], eta,
                                dsig, liz_lists=_oracle_liz(w, liz))
    assert np.abs(g - ref.real).max() <= 1e-9 * np.abs(ref.real).max()
    h = 1e-6
    for (k, l) in [(0, 0), (3, 2), (9, 1), (15, 3)]:
        p1 = w["phase"].copy()
        p1[k, l] += h
        p2 = w["phase"].copy()
        p2[k, l] -= h
        fd = (np.dot(dsig, _gpu_sigma(lctx, w, liz, la, lp, species, J, p1, eta))
              - np.dot(dsig, _gpu_sigma(lctx, w, liz, la, lp, species, J, p2, eta))) / (2 * h)
        assert abs(fd - g[k, l]) <= 1e-6 * np.abs(g).max(), (k, l, fd, g[k, l])


def test_adjoint_bcc250_vs_oracle_and_fd(lctx):
    """Gradient workload (250-atom bcc A0.5B0.5, LIZ 89, FP64): d sigma_xx / d delta_l for all
    250 x 4 phase shifts through the adjoint, against the oracle's forward-mode gradient at 40
    seeded (site, l) entries (stored by tests/golden/make_bcc250grad_oracle.py, which calls only
    the oracle) to 1e-9, and against central finite differences (h = 1e-6 rad) of the library's
    own FP64 forward at the same entries."""
    import json
    import os
    import paper_2311_12134_amd as P
    w = synthetic.workload("bcc250grad")
    eta = w["etas"][0]
    with open(os.path.join(os.path.dirname(__file__), "golden", "bcc250grad_oracle_gradient.json")) as f:
        gold = json.load(f)
    assert gold["fingerprint"] == synthetic.fingerprint(w) and gold["eta"] == eta, "stale golden gradient"
    liz, la, lp, species, J = _grad_setup(w)
    _oracle_liz(w, liz, sorted({k for k, _ in gold["pairs"]}))
    dsig = np.array(gold["dsigma"])
    print("[gpu] adjoint bcc250grad vs oracle at %d entries" % len(gold["pairs"]), flush=True)
    ph = torch.from_numpy(np.ascontiguousarray(w["phase"])).to(torch.device("cuda", 0)).requires_grad_(True)
    sig = P.KuboSigma.apply(ph, lctx, liz, la, lp, species, J, w["volume"], w["e_fermi"], eta)
    sig.backward(torch.from_numpy(dsig).to(sig.device))
    g = ph.grad.cpu().numpy()
    assert g.shape == (250, 4) and np.isfinite(g).all()
    ref = np.array(gold["values"])
    got = np.array([g[k, l] for k, l in gold["pairs"]])
    scale = np.abs(ref).max()
    assert np.abs(got - ref).max() <= 1e-9 * scale, np.abs(got - ref).max() / scale
    h = 1e-6
    for (k, l), gk in zip(gold["pairs"], got):
        p1 = w["phase"].copy()
        p1[k, l] += h
        p2 = w["phase"].copy()
        p2[k, l] -= h
        fd = (np.dot(dsig, _gpu_sigma(lctx, w, liz, la, lp, species, J, p1, eta))
              - np.dot(dsig, _gpu_sigma(lctx, w, liz, la, lp, species, J, p2, eta))) / (2 * h)
        assert abs(fd - gk) <= 1e-6 * scale, (k, l, fd, gk)


def test_split_fallback_to_fp64_when_refinement_cannot_converge(lctx):
    """With no refinement budget every job is flagged NOCONV and recomputed in FP64."""
    w = synthetic.workload("bcc16")
    eta = w["etas"][0]
    g = _run(lctx, w, eta, precision="split", refine_tol=1e-300, max_refine=0)
    assert (g["info"] == -1).all()
    assert (g["berr"] == -1.0).all()  # no split-mode residual describes the recomputed solution
    atoms = list(range(16))
    o = _oracle_atoms(w, eta, atoms, g["liz"])
    _check_atoms(g, o, atoms, TOL64)


def _split_job_bytes(npad):
    """Workspace of one split-mode system (the wave layout: FP32 matrix, packed FP64
    contractions of the member pairs, solution and residual blocks, pivots and their
    per-panel interchange lists), each part rounded to 256 bytes."""
    def al(v):
        return (v + 255) // 256 * 256
    nb = npad // 16
    return (al(npad * npad * 8) + al(nb * (nb + 1) // 2 * 136 * 16) + 2 * al(npad * 32 * 16)
            + al((npad + npad // 64 * 258) * 4))


def test_split_fallback_in_one_job_waves():
    """A workspace that holds one system per wave: the FP64 recomputation of a system whose
    refinement cannot converge does not fit in the wave's FP32 matrix area and takes a buffer
    of its own; FP64 parity as with the shared area."""
    import paper_2311_12134_amd as P
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    w = synthetic.workload("bcc16")
    eta = w["etas"][0]
    liz = P.build_liz(w["pos"], w["cell"], w["r_liz"])
    nl = np.diff(liz.ptr)
    npad = int(((16 * nl.max() + 63) // 64) * 64)
    small = P.Context(0, workspace_limit=int(1.5 * _split_job_bytes(npad)))
    try:
        g = _run(small, w, eta, precision="split", refine_tol=1e-300, max_refine=0)
    finally:
        small.close()
    assert (g["info"] == -1).all()
    assert (g["berr"] == -1.0).all()
    atoms = list(range(16))
    o = _oracle_atoms(w, eta, atoms, g["liz"])
    _check_atoms(g, o, atoms, TOL64)


def test_split_refinement_reaches_tolerance_quickly(lctx):
    w = synthetic.workload("bcc250")
    g = _run(lctx, w, w["etas"][0], precision="split", refine_tol=1e-14, max_refine=3, per_atom=False)
    assert (g["info"] == 0).all() and (g["berr"] <= 1e-14).all()


@pytest.mark.parametrize("name,precision", [("fcc32", "fp64"), ("fcc32", "split"), ("bcc1940", "split")])
def test_graph_replay_matches_eager(lctx, name, precision):
    """Graph-captured factorization + first solve, replayed three times with eager work and
    synchronizations in between, gives bitwise the eager result every time."""
    import paper_2311_12134_amd as P
    w = synthetic.workload(name)
    eta = w["etas"][0]
    dev = torch.device("cuda", 0)
    liz = P.build_liz(w["pos"], w["cell"], w["r_liz"])
    la, lp = liz.to_device(dev)
    phase = torch.from_numpy(np.ascontiguousarray(w["phase"])).to(dev)
    species = torch.from_numpy(w["species"].astype(np.int32)).to(dev)
    J = torch.from_numpy(np.ascontiguousarray(w["J"])).to(dev)
    print("[gpu] graphs %s %s" % (name, precision), flush=True)

    def solve():
        tp, tm, info, berr = lctx.tau_solve(liz, la, lp, phase, w["e_fermi"], eta, precision=precision)
        sig, _, _ = lctx.kubo_sigma(liz, la, tp, tm, species, J, w["volume"])
        torch.cuda.synchronize()
        return tp.cpu().numpy(), tm.cpu().numpy(), info.cpu().numpy(), sig.cpu().numpy()

    ref = solve()
    assert (ref[2] == 0).all()
    lctx.set_graphs(True)
    try:
        for rep in range(3):
            got = solve()
            for a, b in zip(ref, got):
                assert np.array_equal(a, b), (name, precision, rep)
    finally:
        lctx.set_graphs(False)


def test_autotune_picks_fastest_tiling(lctx):
    best, ms = lctx.autotune(npad=448, batch=32)
    assert 0 <= best < 21 and len(ms) == 21
    assert all(np.isfinite(m) and m > 0 for m in ms)
    assert ms[best] == min(ms) or (best == 19 and ms[19] <= 1.01 * min(ms))  # the default within 1 %
    try:
        assert lctx.gemm_tiling() == best
    finally:
        lctx.set_gemm_tiling(-1)


def _device_inputs(w, liz):
    dev = torch.device("cuda", 0)
    la, lp = liz.to_device(dev)
    phase = torch.from_numpy(np.ascontiguousarray(w["phase"])).to(dev)
    species = torch.from_numpy(w["species"].astype(np.int32)).to(dev)
    J = torch.from_numpy(np.ascontiguousarray(w["J"])).to(dev)
    return la, lp, phase, species, J


@pytest.mark.parametrize("name,precision,tol", [("bcc16", "fp64", TOL64), ("fcc32", "split", TOL_SPLIT)])
def test_tensor_full_vs_oracle(lctx, name, precision, tol):
    """All nine sigma_{mu nu} (Eq. (10) + Eq. (7)) against the oracle; the diagonal also
    against lsms_kubo_sigma on the same tau."""
    import paper_2311_12134_amd as P
    w = synthetic.workload(name)
    eta = w["etas"][0]
    print("[gpu] tensor %s %s" % (name, precision), flush=True)
    liz = P.build_liz(w["pos"], w["cell"], w["r_liz"])
    la, lp, phase, species, J = _device_inputs(w, liz)
    tp, tm, info, _ = lctx.tau_solve(liz, la, lp, phase, w["e_fermi"], eta, precision=precision)
    sig, st, pa = lctx.kubo_sigma_tensor(liz, la, tp, tm, species, J, w["volume"], per_atom=True)
    sd, std, _ = lctx.kubo_sigma(liz, la, tp, tm, species, J, w["volume"])
    torch.cuda.synchronize()
    assert (info.cpu().numpy() == 0).all()
    sig, st, pa, sd = sig.cpu().numpy(), st.cpu().numpy(), pa.cpu().numpy(), sd.cpu().numpy()
    o = kubo.sigma(w["pos"], w["cell"], w["r_liz"], w["species"], w["phase"], w["J"], w["e_fermi"], eta,
                   liz_lists=_oracle_liz(w, liz), tensor=True)
    scale = np.abs(o["sigma"].real).max()
    assert np.abs(sig - o["sigma"].real).max() <= tol * scale
    assert np.abs(st - o["sigma_tilde"]).max() <= tol * np.abs(o["sigma_tilde"]).max()
    for i in range(liz.n_atoms):
        ref = o["per_atom"][i]
        assert np.abs(pa[i] - ref).max() <= tol * np.abs(ref).max(), i
    assert np.allclose(np.diag(sig), sd, rtol=1e-13, atol=0)


@pytest.mark.parametrize("eta", [0.005, 0.002, 0.001])
def test_fcc4000_split_sampled(lctx, eta):
    """The 4000-atom fcc alloy in the configuration the benchmark times (split precision, the
    library's default tiling, all atoms batched), at each of its three broadenings: sampled
    atoms plus the atom whose refined solution has the largest backward error, tau and Kubo
    tensor sums against the oracle to 1e-8; sigma's diagonal from both Kubo entry points."""
    import paper_2311_12134_amd as P
    w = synthetic.workload("fcc4000")
    assert eta in w["etas"]
    print("[gpu] fcc4000 split sampled eta %g" % eta, flush=True)
    liz = P.build_liz(w["pos"], w["cell"], w["r_liz"])
    la, lp, phase, species, J = _device_inputs(w, liz)
    tp, tm, info, berr = lctx.tau_solve(liz, la, lp, phase, w["e_fermi"], eta, precision="split")
    sig, st, pa = lctx.kubo_sigma_tensor(liz, la, tp, tm, species, J, w["volume"], per_atom=True)
    sd, _, _ = lctx.kubo_sigma(liz, la, tp, tm, species, J, w["volume"])
    torch.cuda.synchronize()
    berr = berr.cpu().numpy()
    assert (info.cpu().numpy() == 0).all() and (berr <= 1e-14).all()
    assert np.allclose(np.diag(sig.cpu().numpy()), sd.cpu().numpy(), rtol=1e-13, atol=0)
    worst = int(np.argmax(berr.max(axis=1)))
    atoms = sorted({0, 1777, 3999, worst})
    print("[gpu] fcc4000 eta %g: largest berr %.2e at atom %d" % (eta, berr.max(), worst), flush=True)
    o = _oracle_atoms(w, eta, atoms, liz, tensor=True)
    for i in atoms:
        sl = slice(int(liz.ptr[i]), int(liz.ptr[i + 1]))
        for tag, t in (("+", tp), ("-", tm)):
            ref = o["tau"][i]["col" + tag]
            got = t[sl].cpu().numpy()
            err = np.linalg.norm(got - ref) / np.linalg.norm(ref)
            assert err <= TOL_SPLIT, "atom %d tau%s rel err %.3e" % (i, tag, err)
            # element by element, against the largest block entry of that atom
            assert np.abs(got - ref).max() <= TOL_SPLIT * np.abs(ref).max(), (i, tag)
        ref = o["per_atom"][i]
        err = np.abs(pa[i].cpu().numpy() - ref).max() / np.abs(ref).max()
        assert err <= TOL_SPLIT, "atom %d Kubo tensor rel err %.3e" % (i, err)


def test_liz_sweep_and_spin_vs_oracle(lctx):
    """The LIZ-radius sweep (Sec. II.C, Sec. IV): sigma tensor and rho = sigma^-1 at three
    radii of the pure fcc crystal, spin-polarized with two phase-shift sets, against the
    oracle's per-channel sums; then both fits on the three points."""
    from paper_2311_12134_amd import resistivity as R
    from oracle import resistivity as O
    w = synthetic.workload("fcc32")
    eta = w["etas"][0]
    a = w["a"]
    radii = [0.75 * a, 1.1 * a, 1.3 * a]
    phase_dn = np.ascontiguousarray(w["phase"] * 0.8)
    print("[gpu] liz sweep fcc32 radii %s" % radii, flush=True)
    got = R.liz_sweep(lctx, w["pos"], w["cell"], w["species"], w["phase"], w["J"], w["e_fermi"], eta, radii,
                      w["volume"], precision="fp64", phase_down=phase_dn)
    assert [g["liz_max"] for g in got] == [13, 19, 43]
    for g, r in zip(got, radii):
        up = kubo.sigma(w["pos"], w["cell"], r, w["species"], w["phase"], w["J"], w["e_fermi"], eta,
                        volume=w["volume"], tensor=True)["sigma"].real
        dn = kubo.sigma(w["pos"], w["cell"], r, w["species"], phase_dn, w["J"], w["e_fermi"], eta,
                        volume=w["volume"], tensor=True)["sigma"].real
        tot = O.spin_sum(up, dn)
        scale = np.abs(tot).max()
        assert np.abs(g["sigma_up"] - up).max() <= TOL64 * np.abs(up).max()
        assert np.abs(g["sigma_down"] - dn).max() <= TOL64 * np.abs(dn).max()
        assert np.abs(g["sigma"] - tot).max() <= TOL64 * scale
        rho = O.resistivity(tot)
        assert np.abs(g["rho"] - rho).max() <= 1e-9 * np.abs(rho).max()
    rx = np.array([g["rho"][0, 0] for g in got])
    assert np.allclose(R.fit_linear(radii, rx), O.fit_linear(radii, rx), rtol=1e-9)


@pytest.mark.parametrize("name,precision,tol", [("bcc16", "fp64", TOL64), ("fcc32", "split", TOL_SPLIT),
                                                ("bcc1940", "split", TOL_SPLIT)])
def test_conj_symmetry_mode(lctx, name, precision, tol):
    """z+ solved alone, z- derived as P conj(tau(z+)) P: z+ blocks bitwise those of the full
    solve, z- blocks and the Kubo sums against the oracle (which solves both energies)."""
    import paper_2311_12134_amd as P
    w = synthetic.workload(name)
    eta = w["etas"][0]
    print("[gpu] conj symmetry %s %s" % (name, precision), flush=True)
    liz = P.build_liz(w["pos"], w["cell"], w["r_liz"])
    la, lp, phase, species, J = _device_inputs(w, liz)
    full = lctx.tau_solve(liz, la, lp, phase, w["e_fermi"], eta, precision=precision)
    lctx.set_conj_symmetry(True)
    try:
        assert lctx.conj_symmetry()
        tp, tm, info, berr = lctx.tau_solve(liz, la, lp, phase, w["e_fermi"], eta, precision=precision)
    finally:
        lctx.set_conj_symmetry(False)
    _, _, pa = lctx.kubo_sigma(liz, la, tp, tm, species, J, w["volume"], per_atom=True)
    torch.cuda.synchronize()
    info = info.cpu().numpy()
    assert (info == 0).all() and np.array_equal(info[:, 0], info[:, 1])
    assert np.array_equal(berr.cpu().numpy()[:, 0], berr.cpu().numpy()[:, 1])
    if np.ptp(np.diff(liz.ptr)) == 0:  # uniform sizes: identical waves for z+, so bitwise
        assert torch.equal(tp, full[0])
    sizes = np.diff(liz.ptr)
    atoms = [0, 5] if liz.n_atoms < 100 else [int(np.argmin(sizes)), int(np.argmax(sizes)), 1000]
    o = _oracle_atoms(w, eta, atoms, liz)
    pa = pa.cpu().numpy()
    for i in atoms:
        sl = slice(int(liz.ptr[i]), int(liz.ptr[i + 1]))
        for tag, t in (("+", tp), ("-", tm)):
            ref = o["tau"][i]["col" + tag]
            err = np.linalg.norm(t[sl].cpu().numpy() - ref) / np.linalg.norm(ref)
            assert err <= tol, "atom %d tau%s rel err %.3e" % (i, tag, err)
        err = np.abs(pa[i] - o["per_atom"][i]).max() / np.abs(o["per_atom"][i]).max()
        assert err <= tol, "atom %d Kubo rel err %.3e" % (i, err)


@pytest.mark.parametrize("name,precision,chunk,tol", [("bcc250", "fp64", 256, TOL64), ("bcc250", "split", 128, TOL_SPLIT),
                                                      ("bcc1940", "split", 192, TOL_SPLIT)])
def test_tournament_panels_vs_oracle(lctx, name, precision, chunk, tol):
    """Panels taller than 2 chunk rows take the tournament-pivoting path (on LIZ of a few
    hundred sites with the default chunk; forced here with small chunks): sampled atoms
    against the oracle; bcc1940 mixes LIZ sizes, so jobs of one wave have different chunk
    counts."""
    import paper_2311_12134_amd as P
    w = synthetic.workload(name)
    eta = w["etas"][0]
    print("[gpu] tournament %s %s chunk %d" % (name, precision, chunk), flush=True)
    liz = P.build_liz(w["pos"], w["cell"], w["r_liz"])
    la, lp, phase, species, J = _device_inputs(w, liz)
    lctx.set_tslu_chunk(chunk)
    try:
        assert lctx.tslu_chunk() == chunk
        tp, tm, info, berr = lctx.tau_solve(liz, la, lp, phase, w["e_fermi"], eta, precision=precision)
        _, _, pa = lctx.kubo_sigma(liz, la, tp, tm, species, J, w["volume"], per_atom=True)
        torch.cuda.synchronize()
    finally:
        lctx.set_tslu_chunk(2048)
    assert (info.cpu().numpy() == 0).all()
    sizes = np.diff(liz.ptr)
    atoms = [0, 77, 249] if name == "bcc250" else [int(np.argmin(sizes)), int(np.argmax(sizes)), 1000]
    o = _oracle_atoms(w, eta, atoms, liz)
    pa = pa.cpu().numpy()
    for i in atoms:
        sl = slice(int(liz.ptr[i]), int(liz.ptr[i + 1]))
        for tag, t in (("+", tp), ("-", tm)):
            ref = o["tau"][i]["col" + tag]
            err = np.linalg.norm(t[sl].cpu().numpy() - ref) / np.linalg.norm(ref)
            assert err <= tol, "atom %d tau%s rel err %.3e" % (i, tag, err)
        err = np.abs(pa[i] - o["per_atom"][i]).max() / np.abs(o["per_atom"][i]).max()
        assert err <= tol, "atom %d Kubo rel err %.3e" % (i, err)


def test_batched_lu_solve_tall_panels(lctx):
    """The diagnostic batched solve with tournament panels on random systems (FP64),
    against numpy; sizes not multiples of 64, uneven in one batch."""
    rng = np.random.default_rng(12)
    ns = [700, 1100, 333]
    print("[gpu] batched tall panels %s" % ns, flush=True)
    A = [rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n)) for n in ns]
    B = [rng.standard_normal((n, 3)) + 1j * rng.standard_normal((n, 3)) for n in ns]
    Ad = [torch.from_numpy(a).to("cuda") for a in A]
    Bd = [torch.from_numpy(b).to("cuda") for b in B]
    lctx.set_tslu_chunk(128)
    try:
        info = lctx.batched_lu_solve(Ad, Bd, precision="fp64")
        torch.cuda.synchronize()
    finally:
        lctx.set_tslu_chunk(2048)
    assert (info.cpu().numpy() == 0).all()
    for a, b, x in zip(A, B, Bd):
        ref = np.linalg.solve(a, b)
        assert np.abs(x.cpu().numpy() - ref).max() <= 1e-9 * np.abs(ref).max()


def test_paper_scale_liz_bcc16000(lctx):
    """The paper's large-LIZ setting (16,000-atom bcc alloy, 965-site LIZ, n = 15440) in split
    precision with the default tournament chunk: two sampled centres (empty LIZ for the other
    atoms); the refined solution's backward error, and the oracle's own block rows of
    M = 1 - t g applied to the GPU's tau column (residual of the oracle's system) for
    sampled members."""
    import paper_2311_12134_amd as P
    w = synthetic.workload("bcc16000")
    eta = w["etas"][0]
    centres = [0, 12345]
    print("[gpu] paper-scale LIZ bcc16000 centres %s" % centres, flush=True)
    liz = P.build_liz(w["pos"], w["cell"], w["r_liz"], centres=centres)
    assert list(np.diff(liz.ptr)[centres]) == [965, 965] and liz.total == 2 * 965
    la, lp, phase, species, J = _device_inputs(w, liz)
    tp, tm, info, berr = lctx.tau_solve(liz, la, lp, phase, w["e_fermi"], eta, precision="split")
    sig, _, pa = lctx.kubo_sigma(liz, la, tp, tm, species, J, w["volume"], per_atom=True)
    torch.cuda.synchronize()
    info, berr, pa = info.cpu().numpy(), berr.cpu().numpy(), pa.cpu().numpy()
    assert (info == 0).all() and (berr[centres] <= 1e-14).all()
    others = np.setdiff1d(np.arange(liz.n_atoms), centres)
    assert (berr[others] == 0).all() and not pa[others].any() and np.isfinite(sig.cpu().numpy()).all()
    _, _, kp, km = kkr.energies(w["e_fermi"], eta)
    tpl, tmi = kkr.t_matrix(w["phase"], kp)
    rng = np.random.default_rng(4)
    optr, oatom, opos = _oracle_liz(w, liz, centres)
    for m in centres:
        sl = slice(int(liz.ptr[m]), int(liz.ptr[m + 1]))
        P_ = opos[optr[m]:optr[m + 1]]
        mem = oatom[optr[m]:optr[m + 1]]
        for tag, tt, kap, tau in (("+", tpl, kp, tp), ("-", tmi, km, tm)):
            X = tau[sl].cpu().numpy()  # [members, 16, 16]
            tdiag = np.stack([kkr.expand_t(tt[a]) for a in mem])  # [members, 16]
            for a in [0, 1] + list(rng.choice(np.arange(2, len(mem)), 4, replace=False)):
                others_b = np.array([b for b in range(len(mem)) if b != a])
                g = kkr.g0_blocks(P_[a] - P_[others_b], kap)  # [n-1, 16, 16]
                tg = tdiag[a][None, :, None] * g
                r = X[a] - np.einsum("bij,bjk->ik", tg, X[others_b])
                if a == 0:
                    r = r - np.diag(tdiag[0])
                scale = (np.linalg.norm(X[a]) + sum(np.linalg.norm(tg[q]) * np.linalg.norm(X[b])
                                                    for q, b in enumerate(others_b)) + (a == 0) * np.linalg.norm(tdiag[0]))
                assert np.linalg.norm(r) <= 1e-12 * scale, (m, tag, a, np.linalg.norm(r) / scale)


@pytest.mark.parametrize("name,precision,chunk", [("fcc32", "fp64", 2048), ("bcc250", "split", 2048),
                                                  ("bcc1940", "split", 2048), ("bcc250", "split", 256)])
def test_lookahead_matches_single_stream(lctx, name, precision, chunk):
    """The look-ahead schedule (next first panel on a second stream) gives bitwise the
    single-stream result, also with tournament panels."""
    import paper_2311_12134_amd as P
    w = synthetic.workload(name)
    eta = w["etas"][0]
    print("[gpu] look-ahead %s %s chunk %d" % (name, precision, chunk), flush=True)
    liz = P.build_liz(w["pos"], w["cell"], w["r_liz"])
    la, lp, phase, species, J = _device_inputs(w, liz)
    lctx.set_tslu_chunk(chunk)
    # the look-ahead stream turns wave pipelining off; keep it off in both runs so the waves
    # group the (uneven) systems alike (it is off by default too)
    lctx.set_pipeline(False)
    try:
        lctx.set_lookahead(False)
        a = lctx.tau_solve(liz, la, lp, phase, w["e_fermi"], eta, precision=precision)
        lctx.set_lookahead(True)
        b = lctx.tau_solve(liz, la, lp, phase, w["e_fermi"], eta, precision=precision)
        torch.cuda.synchronize()
    finally:
        lctx.set_lookahead(False)
        lctx.set_tslu_chunk(2048)
    for x, y in zip(a, b):
        assert torch.equal(x, y)
    assert (a[2].cpu().numpy() == 0).all()


@pytest.mark.parametrize("precision,tol", [("fp64", TOL64), ("split", TOL_SPLIT)])
def test_single_site_and_small_open_clusters(lctx, precision, tol):
    """Degenerate sizes: an isolated atom (LIZ of 1 site, n = 16 padded to 64: tau = t
    exactly), a pair and a triangle of an open cluster, in one batch, against the oracle."""
    import paper_2311_12134_amd as P
    pos = np.array([[0.0, 0.0, 0.0], [4.2, 0.3, 0.1], [0.4, 4.1, -0.3], [40.0, 0.0, 0.0], [47.0, 1.0, 0.0]])
    species = np.array([0, 1, 0, 1, 0], dtype=np.int32)
    phase = np.array([[0.8, 0.2, 0.6, 0.01], [0.7, 0.25, 0.3, 0.01]])[species]
    J = synthetic.current_matrices(2, np.random.default_rng(31))
    w = dict(pos=pos, cell=None, r_liz=7.5, species=species, phase=phase, J=J, e_fermi=0.65, volume=900.0)
    print("[gpu] small open clusters %s" % precision, flush=True)
    liz = P.build_liz(pos, None, w["r_liz"])
    assert list(np.diff(liz.ptr)) == [3, 3, 3, 2, 2]
    iso = P.build_liz(pos, None, 5.0)
    assert np.diff(iso.ptr)[3] == 1
    for L in (liz, iso):
        la, lp, ph, sp, Jd = _device_inputs(w, L)
        tp, tm, info, _ = lctx.tau_solve(L, la, lp, ph, w["e_fermi"], 0.004, precision=precision)
        _, _, pa = lctx.kubo_sigma(L, la, tp, tm, sp, Jd, w["volume"], per_atom=True)
        torch.cuda.synchronize()
        assert (info.cpu().numpy() == 0).all()
        o = kubo.sigma(pos, None, w["r_liz"], species, phase, J, w["e_fermi"], 0.004, volume=w["volume"],
                       liz_lists=_oracle_liz(w, L, r_liz=w["r_liz"] if L is liz else 5.0))
        for i in range(5):
            sl = slice(int(L.ptr[i]), int(L.ptr[i + 1]))
            for tag, t in (("+", tp), ("-", tm)):
                ref = o["tau"][i]["col" + tag]
                err = np.linalg.norm(t[sl].cpu().numpy() - ref) / np.linalg.norm(ref)
                assert err <= tol, (i, tag, err)
            ref = o["per_atom"][i]
            assert np.abs(pa[i].cpu().numpy() - ref).max() <= tol * np.abs(ref).max(), i
    # the isolated atom: tau^{00} = t exactly (diagonal, no scattering partners)
    _, _, kp, _ = kkr.energies(w["e_fermi"], 0.004)
    t3 = kkr.expand_t(kkr.t_matrix(phase, kp)[0][3])
    la, lp, ph, sp, Jd = _device_inputs(w, iso)
    tp = lctx.tau_solve(iso, la, lp, ph, w["e_fermi"], 0.004, precision=precision)[0]
    got = tp[int(iso.ptr[3])].cpu().numpy()
    assert np.abs(got - np.diag(t3)).max() <= 1e-15 * np.abs(t3).max() * 16


def test_one_centre_subset(lctx):
    """Only one centre of a structure solved (every other atom's LIZ empty): its tau and
    Kubo sum equal those of the full run, the skipped atoms report zeros."""
    import paper_2311_12134_amd as P
    w = synthetic.workload("bcc250")
    eta = w["etas"][0]
    print("[gpu] one-centre subset bcc250", flush=True)
    full = P.build_liz(w["pos"], w["cell"], w["r_liz"])
    sub = P.build_liz(w["pos"], w["cell"], w["r_liz"], centres=[77])
    res = []
    for L in (full, sub):
        la, lp, ph, sp, Jd = _device_inputs(w, L)
        tp, tm, info, berr = lctx.tau_solve(L, la, lp, ph, w["e_fermi"], eta, precision="fp64")
        _, st, pa = lctx.kubo_sigma(L, la, tp, tm, sp, Jd, w["volume"], per_atom=True)
        torch.cuda.synchronize()
        res.append((L, tp.cpu().numpy(), info.cpu().numpy(), pa.cpu().numpy(), st.cpu().numpy()))
    (F, tpf, _, paf, _), (S, tps, infos, pas, sts) = res
    a, b = slice(F.ptr[77], F.ptr[78]), slice(S.ptr[77], S.ptr[78])
    assert np.allclose(tps[b], tpf[a], rtol=0, atol=1e-13 * np.abs(tpf[a]).max())
    assert np.allclose(pas[77], paf[77], rtol=1e-12)
    assert (infos == 0).all() and not np.delete(pas, 77, axis=0).any()
    assert np.allclose(sts, -pas[77] / (np.pi * w["volume"]), rtol=1e-14)


def test_adjoint_with_tournament_panels(lctx):
    """The adjoint's transposed solves reuse factors whose panels came from the tournament
    (250-atom alloy, 256-row chunks): the gradient equals the one from register panels
    (itself checked against the oracle and finite differences) to 1e-9."""
    import paper_2311_12134_amd as P
    w = synthetic.workload("bcc250grad")
    eta = w["etas"][0]
    liz, la, lp, species, J = _grad_setup(w)
    dsig = torch.tensor([1.0, 0.0, 0.0], dtype=torch.float64, device="cuda")
    print("[gpu] adjoint with tournament panels bcc250", flush=True)

    def grad():
        ph = torch.from_numpy(np.ascontiguousarray(w["phase"])).to(torch.device("cuda", 0)).requires_grad_(True)
        sig = P.KuboSigma.apply(ph, lctx, liz, la, lp, species, J, w["volume"], w["e_fermi"], eta)
        sig.backward(dsig)
        return ph.grad.cpu().numpy()

    ref = grad()
    lctx.set_tslu_chunk(256)
    try:
        g = grad()
    finally:
        lctx.set_tslu_chunk(2048)
    assert np.abs(g - ref).max() <= 1e-9 * np.abs(ref).max()


def test_graph_replay_with_tournament_panels(lctx):
    """Captured factorization + first solve with tournament panels (chunk 256), replayed three
    times with eager work in between: bitwise the eager result."""
    import paper_2311_12134_amd as P
    w = synthetic.workload("bcc250")
    eta = w["etas"][0]
    print("[gpu] graphs with tournament panels bcc250", flush=True)
    liz = P.build_liz(w["pos"], w["cell"], w["r_liz"])
    la, lp, phase, species, J = _device_inputs(w, liz)
    lctx.set_tslu_chunk(256)
    try:
        def solve():
            tp, tm, info, _ = lctx.tau_solve(liz, la, lp, phase, w["e_fermi"], eta, precision="split")
            torch.cuda.synchronize()
            return tp.cpu().numpy(), tm.cpu().numpy(), info.cpu().numpy()
        ref = solve()
        assert (ref[2] == 0).all()
        lctx.set_graphs(True)
        for rep in range(3):
            got = solve()
            for a, b in zip(ref, got):
                assert np.array_equal(a, b), rep
    finally:
        lctx.set_graphs(False)
        lctx.set_tslu_chunk(2048)


@pytest.mark.parametrize("name,chunk", [("fcc32", 2048), ("bcc250", 2048), ("bcc1940", 2048), ("bcc250", 256)])
def test_symmetric_ldlt_vs_oracle(lctx, name, chunk):
    """Split mode on the symmetric form 1 - T^1/2 g T^1/2 with L D L^T (no pivoting), FP64
    refinement of S (residuals from the FP64 pair contractions): sampled atoms' tau and Kubo
    sums against the oracle (which solves M X = T E0 by LU), and the backward error reached.  With 256-row
    chunks the panels taller than 512 rows take the diagonal-block path of tall panels."""
    import paper_2311_12134_amd as P
    w = synthetic.workload(name)
    eta = w["etas"][0]
    print("[gpu] symmetric LDLT %s chunk %d" % (name, chunk), flush=True)
    liz = P.build_liz(w["pos"], w["cell"], w["r_liz"])
    la, lp, phase, species, J = _device_inputs(w, liz)
    lctx.set_symmetric(True)
    lctx.set_tslu_chunk(chunk)
    try:
        tp, tm, info, berr = lctx.tau_solve(liz, la, lp, phase, w["e_fermi"], eta, precision="split")
        _, _, pa = lctx.kubo_sigma(liz, la, tp, tm, species, J, w["volume"], per_atom=True)
        torch.cuda.synchronize()
    finally:
        lctx.set_symmetric(False)
        lctx.set_tslu_chunk(2048)
    assert (info.cpu().numpy() == 0).all() and (berr.cpu().numpy() <= 1e-14).all()
    sizes = np.diff(liz.ptr)
    atoms = ([0, 5, 31] if name == "fcc32" else [0, 77, 249] if name == "bcc250"
             else [int(np.argmin(sizes)), int(np.argmax(sizes)), 1000])
    o = _oracle_atoms(w, eta, atoms, liz)
    pa = pa.cpu().numpy()
    for i in atoms:
        sl = slice(int(liz.ptr[i]), int(liz.ptr[i + 1]))
        for tag, t in (("+", tp), ("-", tm)):
            ref = o["tau"][i]["col" + tag]
            err = np.linalg.norm(t[sl].cpu().numpy() - ref) / np.linalg.norm(ref)
            assert err <= TOL_SPLIT, "atom %d tau%s rel err %.3e" % (i, tag, err)
        err = np.abs(pa[i] - o["per_atom"][i]).max() / np.abs(o["per_atom"][i]).max()
        assert err <= TOL_SPLIT, "atom %d Kubo rel err %.3e" % (i, err)


def test_symmetric_ldlt_with_conj_symmetry(lctx):
    """Both algorithmic savings at once (z+ only, tau(z-) by conjugation; symmetric form with
    L D L^T): sampled atoms of the 250-atom alloy against the oracle."""
    import paper_2311_12134_amd as P
    w = synthetic.workload("bcc250")
    eta = w["etas"][0]
    print("[gpu] symmetric LDLT + conj symmetry bcc250", flush=True)
    liz = P.build_liz(w["pos"], w["cell"], w["r_liz"])
    la, lp, phase, species, J = _device_inputs(w, liz)
    lctx.set_symmetric(True)
    lctx.set_conj_symmetry(True)
    try:
        tp, tm, info, berr = lctx.tau_solve(liz, la, lp, phase, w["e_fermi"], eta, precision="split")
        torch.cuda.synchronize()
    finally:
        lctx.set_symmetric(False)
        lctx.set_conj_symmetry(False)
    assert (info.cpu().numpy() == 0).all() and (berr.cpu().numpy() <= 1e-14).all()
    atoms = [0, 77, 249]
    o = _oracle_atoms(w, eta, atoms, liz)
    for i in atoms:
        sl = slice(int(liz.ptr[i]), int(liz.ptr[i + 1]))
        for tag, t in (("+", tp), ("-", tm)):
            ref = o["tau"][i]["col" + tag]
            err = np.linalg.norm(t[sl].cpu().numpy() - ref) / np.linalg.norm(ref)
            assert err <= TOL_SPLIT, "atom %d tau%s rel err %.3e" % (i, tag, err)


def test_argument_errors_are_reported(lctx):
    """Bad arguments fail synchronously with the library's message, before any device work;
    a context whose workspace cannot hold one system reports LSMS_E_NOMEM."""
    import paper_2311_12134_amd as P
    from paper_2311_12134_amd._lib import LsmsError
    w = synthetic.workload("bcc16")
    liz = P.build_liz(w["pos"], w["cell"], w["r_liz"])
    la, lp, phase, species, J = _device_inputs(w, liz)
    print("[gpu] argument errors", flush=True)
    for knob_call in (lambda: lctx.set_tslu_chunk(100), lambda: lctx.set_tslu_chunk(4096),
                      lambda: lctx.set_gemm_tiling(99), lambda: lctx.set_knob("group_f32", 5),
                      lambda: lctx.set_knob("group_f64", 1)):
        with pytest.raises(LsmsError):
            knob_call()
    with pytest.raises(LsmsError):
        lctx.tau_solve(liz, la, lp, phase, w["e_fermi"], 0.0)
    with pytest.raises(LsmsError):
        lctx.tau_solve(liz, la, lp, phase, w["e_fermi"], 0.002, precision="split", refine_tol=-1.0)
    tp, tm, info, _ = lctx.tau_solve(liz, la, lp, phase, w["e_fermi"], 0.002)
    with pytest.raises(LsmsError):
        lctx.kubo_sigma(liz, la, tp, tm, species, J, -1.0)
    with pytest.raises(LsmsError):
        lctx.autotune(npad=100, batch=4)
    small = P.Context(0, workspace_limit=1 << 20)
    try:
        with pytest.raises(LsmsError, match="workspace|bytes"):
            small.tau_solve(liz, la, lp, phase, w["e_fermi"], 0.002)
    finally:
        small.close()
    torch.cuda.synchronize()
    assert (info.cpu().numpy() == 0).all()  # the context still works after the refused calls


def test_symmetric_fallback_to_fp64_lu(lctx):
    """Symmetric form with no refinement budget: every system is flagged and recomputed by
    the FP64 LU with partial pivoting of S, then scaled back (tau = T^1/2 Y): FP64 parity."""
    w = synthetic.workload("bcc16")
    eta = w["etas"][0]
    lctx.set_symmetric(True)
    try:
        g = _run(lctx, w, eta, precision="split", refine_tol=1e-300, max_refine=0)
    finally:
        lctx.set_symmetric(False)
    assert (g["info"] == -1).all() and (g["berr"] == -1.0).all()
    atoms = list(range(16))
    o = _oracle_atoms(w, eta, atoms, g["liz"])
    _check_atoms(g, o, atoms, TOL64)


def test_graph_replay_symmetric(lctx):
    """Captured symmetric factorization + first solve, replayed three times: bitwise the eager
    result."""
    import paper_2311_12134_amd as P
    w = synthetic.workload("bcc250")
    eta = w["etas"][0]
    print("[gpu] graphs with the symmetric form bcc250", flush=True)
    liz = P.build_liz(w["pos"], w["cell"], w["r_liz"])
    la, lp, phase, species, J = _device_inputs(w, liz)
    lctx.set_symmetric(True)
    try:
        def solve():
            tp, tm, info, _ = lctx.tau_solve(liz, la, lp, phase, w["e_fermi"], eta, precision="split")
            torch.cuda.synchronize()
            return tp.cpu().numpy(), tm.cpu().numpy(), info.cpu().numpy()
        ref = solve()
        assert (ref[2] == 0).all()
        lctx.set_graphs(True)
        for rep in range(3):
            got = solve()
            for a, b in zip(ref, got):
                assert np.array_equal(a, b), rep
    finally:
        lctx.set_graphs(False)
        lctx.set_symmetric(False)


@pytest.mark.parametrize("precision", ["split", "fp64"])
def test_pipelined_waves_bitwise(lctx, precision):
    """Waves alternating between two streams (LSMS_TUNE_PIPELINE) give bitwise
    the results of one stream and of a single wave when all systems share one padded size:
    a 4 GiB workspace cuts bcc250 into many waves.  Also with captured graphs replayed on
    both streams."""
    import paper_2311_12134_amd as P
    w = synthetic.workload("bcc250")
    eta = w["etas"][0]
    print("[gpu] pipelined waves bcc250 %s" % precision, flush=True)
    liz = P.build_liz(w["pos"], w["cell"], w["r_liz"])
    la, lp, phase, species, J = _device_inputs(w, liz)

    def solve(ctx):
        tp, tm, info, berr = ctx.tau_solve(liz, la, lp, phase, w["e_fermi"], eta, precision=precision)
        sig, _, _ = ctx.kubo_sigma(liz, la, tp, tm, species, J, w["volume"])
        torch.cuda.synchronize()
        return [a.cpu().numpy() for a in (tp, tm, info, berr, sig)]

    one = solve(lctx)  # the whole batch is one wave in the default workspace
    small = P.Context(0, workspace_limit=4 << 30)
    try:
        assert not small.pipeline()
        small.set_pipeline(True)
        got = solve(small)
        small.set_graphs(True)
        replays = [solve(small) for _ in range(2)]
        small.set_graphs(False)
        small.set_pipeline(False)
        ref = solve(small)
    finally:
        small.close()
    assert (one[2] == 0).all()
    for i, (a, b, c) in enumerate(zip(got, ref, one)):
        assert np.array_equal(a, b) and np.array_equal(a, c), i
    for r in replays:
        for i, (a, b) in enumerate(zip(got, r)):
            assert np.array_equal(a, b), i
