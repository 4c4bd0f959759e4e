"""The allocation-free Kubo sum (lsms_kubo_sigma_noalloc) through the C ABI against
lsms_kubo_sigma on the same tau: two calls in a row on one GPU, the second with fewer atoms,
so the second reads a fixed scratch that still holds the first call's partial sums."""

import numpy as np
import pytest

import synthetic

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _inputs(P, name, dev):
    w = synthetic.workload(name)
    liz = P.build_liz(w["pos"], w["cell"], w["r_liz"])
    la, lp = liz.to_device(dev)
    phase = torch.from_numpy(np.ascontiguousarray(w["phase"])).to(dev)
    species = torch.from_numpy(w["species"].astype(np.int32)).to(dev)
    J = torch.from_numpy(np.ascontiguousarray(w["J"])).to(dev)
    return w, liz, la, lp, phase, species, J


def test_noalloc_kubo_sum_matches_allocating_entry_twice():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2311_12134_amd as P
    from paper_2311_12134_amd._lib import LsmsError
    dev = torch.device("cuda", 0)
    ctx = P.Context(0)
    try:
        for name, precision in (("bcc250", "split"), ("fcc32", "fp64")):
            print("[gpu] no-alloc Kubo sum %s %s" % (name, precision), flush=True)
            w, liz, la, lp, phase, species, J = _inputs(P, name, dev)
            eta = w["etas"][0]
            tp, tm, info, _ = ctx.tau_solve(liz, la, lp, phase, w["e_fermi"], eta, precision=precision)
            ref_sig, ref_st, ref_pa = ctx.kubo_sigma(liz, la, tp, tm, species, J, w["volume"], per_atom=True)
            ptr_dev = torch.from_numpy(liz.ptr).to(dev)
            sig = torch.full((3,), np.nan, dtype=torch.float64, device=dev)
            st = torch.full((4, 3), np.nan, dtype=torch.complex128, device=dev)
            ctx.kubo_sigma_noalloc(ptr_dev, la, tp, tm, species, J, w["volume"], sig, st)
            torch.cuda.synchronize()
            assert (info.cpu().numpy() == 0).all()
            # same kernels and the same fixed reduction order: bitwise equal
            assert torch.equal(sig, ref_sig), (name, sig, ref_sig)
            assert torch.equal(st, ref_st), name
            # and with a caller-provided per-atom array
            pa = torch.empty_like(ref_pa)
            ctx.kubo_sigma_noalloc(ptr_dev, la, tp, tm, species, J, w["volume"], sig, st, per_atom=pa)
            torch.cuda.synchronize()
            assert torch.equal(pa, ref_pa) and torch.equal(sig, ref_sig), name
        # more atoms than the fixed scratch holds: refused before any device work
        big = torch.zeros(32768 + 2, dtype=torch.int64, device=dev)
        with pytest.raises(LsmsError) as e:
            ctx.kubo_sigma_noalloc(big, la, tp, tm, species, J, w["volume"], sig, st)
        assert e.value.code == -1
    finally:
        ctx.close()
