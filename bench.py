"""Benchmark of the LSMS tau-solve + Kubo-Greenwood hot path on one MI355X.

Workload: random binary fcc alloy A0.25B0.75, a = 7.6 bohr, 10x10x10 conventional cells
(4000 atoms), lmax = 3, LIZ of 135 atoms (n = 2160 complex per system), both energies
eF +- i eta with eta cycling over (0.005, 0.002, 0.001) Ry step by step.  A step is the
whole hot path for all 4000 atoms at one eta: assembly of 1 - t g, 8000 complex LU
factorizations with partial pivoting, the tau solves (split precision: FP32 trailing
updates + FP64 refinement), the Kubo-Greenwood traces and the reduction to sigma.
Inputs are synthetic and seeded (no dataset); they live in HBM before the timed region.

Prints one JSON line.  `roofline` is the wide trailing update's achieved algorithmic
TFLOP/s (8 m c K complex flops per job and launch, over its HIP-event launch time on its own
stream) against the 157.3 TFLOP/s FP32 MFMA peak, with the HBM traffic recorded for that
kernel source and launch shape; `cpu_baseline` is the oracle's rate on a bounded sample of
the same workload on the host cores.
"""

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

METRIC = "atoms/sec through LIZ τ-solve + Kubo trace; % MFMA peak; split vs FP64 at 1e-8"
PEAK_FP32_MFMA = 157.3e12
PEAK_FP64_MFMA = 78.6e12
CSRC = os.path.join(ROOT, "paper_2311_12134_amd", "csrc")


def gemm_source(precision, tiling):
    """The source file that holds a trailing-update tiling's kernel."""
    if precision == "split":
        name = "gemm.hip" if tiling < 10 or tiling == 19 else (
            "gemm_wide.hip" if 12 <= tiling <= 16 or tiling == 20 else "gemm_persist.hip")
    else:
        name = "gemm.hip" if tiling == 0 else "gemm64.hip"
    return os.path.join(CSRC, name)

# HBM bytes per launch of the trailing-update kernel on this workload, from two rocprofv3
# counter runs (FETCH_SIZE, WRITE_SIZE) over one step, each scaled by what the same counter
# read for a 1 GiB device-to-device copy in the same run (--copy-calibration).  Keyed by
# (precision, workload, tiling) and tied to the sha256 of the kernel's source file (gemm_source)
# when the counters were taken and to the launches' algorithmic bytes (the wave size, which follows the free HBM):
# any later change to that source, or launches of another shape, make the figure stale and
# it is reported as null.
TRAFFIC = {
    ("split", "fcc4000", 1): {"sha256": "2e3078da84b18709ee1905d4151e5884815da676e36d9ca16b6e12f1ce630b8a",
                              "alg_bytes_per_launch": 6.9042e10, "bytes_per_launch": 1.3337e11},
    ("split", "fcc4000", 2): {"sha256": "2e3078da84b18709ee1905d4151e5884815da676e36d9ca16b6e12f1ce630b8a",
                              "alg_bytes_per_launch": 6.9042e10, "bytes_per_launch": 1.2319e11},
    ("split", "fcc4000", 13): {"sha256": "9001bedb113c858cbd9ba443f681c5ea7cc9357d9d5376fc8cf357fbb44d05b4",
                               "alg_bytes_per_launch": 6.9042e10, "bytes_per_launch": 1.1088e11},
    ("split", "fcc4000", 19): {"sha256": "2e3078da84b18709ee1905d4151e5884815da676e36d9ca16b6e12f1ce630b8a",
                               "alg_bytes_per_launch": 6.9042e10, "bytes_per_launch": 8.2470e10},
    ("split", "fcc4000", 20): {"sha256": "9001bedb113c858cbd9ba443f681c5ea7cc9357d9d5376fc8cf357fbb44d05b4",
                               "alg_bytes_per_launch": 6.9042e10, "bytes_per_launch": 8.4043e10},
}


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def cpu_baseline(w, etas, n_sample, n_single=3):
    """The oracle as it stands on a seeded sample of atoms of the same workload (host cores),
    split evenly over the broadenings the timed region cycles through, and a smaller sample
    with its BLAS held to one thread.  The oracle builds its own LIZ for the sampled centres
    (outside the timer, as the library's LIZ build is outside the GPU's timed region); its
    per-atom Kubo sums are returned for the error report."""
    from oracle import kubo
    from oracle import liz as oliz
    try:
        from threadpoolctl import threadpool_info, threadpool_limits
        threads = max([d.get("num_threads", 1) for d in threadpool_info()] or [1])
    except Exception:
        threadpool_limits = None
        threads = os.cpu_count()
    rng = np.random.default_rng(2311012134 + 30)
    sample = rng.choice(len(w["pos"]), n_sample, replace=False)
    groups = {eta: sorted(int(a) for a in sample[k::len(etas)]) for k, eta in enumerate(etas)}
    lists = oliz.build_liz(w["pos"], w["cell"], w["r_liz"], centres=sorted(int(a) for a in sample))

    def run(atoms, eta):
        t0 = time.perf_counter()
        r = kubo.sigma(w["pos"], w["cell"], w["r_liz"], w["species"], w["phase"], w["J"], w["e_fermi"], eta,
                       atoms=atoms, liz_lists=lists)
        return time.perf_counter() - t0, r

    dt = 0.0
    per_atom = {}
    for eta, atoms in groups.items():
        d, r = run(atoms, eta)
        dt += d
        per_atom[eta] = r["per_atom"]
    what = "of the %s workload, %s atoms at eta %s Ry (both energies, assembly + LU + both tau blocks + Kubo " \
           "traces)" % (w["name"], "/".join(str(len(a)) for a in groups.values()), "/".join("%g" % e for e in etas))
    res = {"value": n_sample / dt, "unit": "atoms/s", "cores": int(threads), "kind": "oracle",
           "sample": "%d atoms %s, %.1f s" % (n_sample, what, dt), "cpu_model": cpu_model()}
    if threadpool_limits is not None and n_single > 0:
        atoms1 = groups[etas[0]][:n_single]
        with threadpool_limits(limits=1):
            d1, _ = run(atoms1, etas[0])
        res["single_thread"] = {"value": len(atoms1) / d1, "unit": "atoms/s", "cores": 1,
                                "sample": "%d atoms of the same sample at eta %g, %.1f s" % (len(atoms1), etas[0], d1)}
    return res, lists, groups, per_atom


def oracle_errors(groups, oracle_pa, gpu_pa):
    """Largest relative error of the GPU's per-atom Kubo sums (all 4 x 3 entries) against the
    oracle's, per broadening, over the sampled atoms."""
    out = {}
    for eta, atoms in groups.items():
        if eta not in gpu_pa:
            continue
        errs = [float(np.abs(gpu_pa[eta][a] - oracle_pa[eta][a]).max() / np.abs(oracle_pa[eta][a]).max())
                for a in atoms]
        out[eta] = max(errs)
    return out


def adjoint_leg(P, torch, ctx):
    """The gradient configuration (250-atom bcc A0.5B0.5 alloy, LIZ 89 sites, FP64):
    sigma with its factors kept, then d sigma_xx / d delta_l for all 250 x 4 phase shifts
    through the hand-written adjoint; one warm-up and one timed forward + backward."""
    import synthetic
    w = synthetic.workload("bcc250grad")
    dev = torch.device("cuda", 0)
    liz = P.build_liz(w["pos"], w["cell"], w["r_liz"])
    la, lp = liz.to_device(dev)
    species = torch.from_numpy(w["species"].astype(np.int32)).to(dev)
    J = torch.from_numpy(np.ascontiguousarray(w["J"])).to(dev)
    eta = w["etas"][0]
    dsig = torch.tensor([1.0, 0.0, 0.0], dtype=torch.float64, device=dev)

    def run():
        ph = torch.from_numpy(np.ascontiguousarray(w["phase"])).to(dev).requires_grad_(True)
        t0 = time.perf_counter()
        sig = P.KuboSigma.apply(ph, ctx, liz, la, lp, species, J, w["volume"], w["e_fermi"], eta)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        sig.backward(dsig)
        torch.cuda.synchronize()
        return t1 - t0, time.perf_counter() - t1, ph.grad

    run()
    tf, tb, g = run()
    log("adjoint leg: forward %.1f ms, backward %.1f ms" % (1e3 * tf, 1e3 * tb))
    return {"workload": "bcc250grad: random bcc A0.5B0.5, 250 atoms, LIZ 89 sites (n = 1424), FP64, "
                        "d sigma_xx / d delta_l for 250 x 4 phase shifts",
            "forward_ms": 1e3 * tf, "backward_ms": 1e3 * tb, "backward_over_forward": tb / tf,
            "grad_finite": bool(torch.isfinite(g).all().item())}


def paper_scale_leg(P, torch, ctx, n_sample, precision, ldlt=False):
    """The paper's large-LIZ setting (16,000-atom bcc alloy, LIZ of 965 sites, n = 15440):
    a seeded sample of centre atoms (the others get empty LIZ and are skipped), one warm-up
    and one timed step of tau solve + Kubo sums; reported apart from the headline value."""
    import synthetic
    w = synthetic.workload("bcc16000")
    rng = np.random.default_rng(2311012134)
    centres = np.sort(rng.choice(len(w["pos"]), n_sample, replace=False))
    liz = P.build_liz(w["pos"], w["cell"], w["r_liz"], centres=centres)
    dev = torch.device("cuda", 0)
    la, lp = liz.to_device(dev)
    phase = torch.from_numpy(np.ascontiguousarray(w["phase"])).to(dev)
    species = torch.from_numpy(w["species"].astype(np.int32)).to(dev)
    J = torch.from_numpy(np.ascontiguousarray(w["J"])).to(dev)
    eta = w["etas"][0]

    def step():
        tp, tm, info, berr = ctx.tau_solve(liz, la, lp, phase, w["e_fermi"], eta, precision=precision)
        sig, _, _ = ctx.kubo_sigma(liz, la, tp, tm, species, J, w["volume"])
        return info, berr, sig

    step()
    torch.cuda.synchronize()
    ctx.set_profiling(True)
    t0 = time.perf_counter()
    info, berr, sig = step()
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    gms, gl, gf, _ = ctx.kernel_stats(kind=1)
    ctx.set_profiling(False)
    n = 16 * int(np.diff(liz.ptr).max())
    alg = n_sample * 2.0 * ((8.0 / 3.0) * n**3 + 128.0 * n**2)
    peak = PEAK_FP32_MFMA if precision == "split" else PEAK_FP64_MFMA
    res = {"workload": "bcc16000: random bcc A0.5B0.5, 16000 atoms, LIZ 965 sites (n = %d), %d seeded centres, "
                       "both energies, eta %g Ry" % (n, n_sample, eta),
           "value": n_sample / el, "unit": "atoms/s", "ms_per_step": 1e3 * el, "precision": precision,
           "path_tflops_alg": alg / el / 1e12, "path_frac_of_peak": alg / el / peak,
           "info_nonzero": int((info.cpu().numpy()[centres] != 0).sum()),
           "berr_max": float(berr.cpu().numpy()[centres].max())}
    if gl:
        res["trailing_update"] = {"launches": gl, "avg_launch_ms": gms / gl,
                                  "achieved_tflops": gf / (gms / 1e3) / 1e12, "frac": gf / (gms / 1e3) / peak}
    log("paper-scale leg: %d atoms of bcc16000 (n = %d) in %.2f s: %.2f atoms/s" % (n_sample, n, el, n_sample / el))
    if ldlt and precision == "split":
        # the same sample through the symmetric form and L D L^T (reported apart from the LU)
        ctx.set_symmetric(True)
        step()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        info_l, berr_l, _ = step()
        torch.cuda.synchronize()
        el_l = time.perf_counter() - t0
        ctx.set_symmetric(False)
        res["symmetric_ldlt"] = {"value": n_sample / el_l, "unit": "atoms/s", "ms_per_step": 1e3 * el_l,
                                 "info_nonzero": int((info_l.cpu().numpy()[centres] != 0).sum()),
                                 "berr_max": float(berr_l.cpu().numpy()[centres].max())}
        log("paper-scale L D L^T: %.2f s, %.2f atoms/s" % (el_l, n_sample / el_l))
    return res


F32_TILINGS = {0: "gemm_f32_3m_kernel", 1: "gemm_f32_3m_tiled<64,64,32,32>", 2: "gemm_f32_3m_tiled<64,64,32,32,xcd>",
               3: "gemm_f32_3m_tiled<128,64,32,64,xcd>", 4: "gemm_f32_3m_tiled<64,128,64,32,xcd>",
               5: "gemm_f32_3m_tiled<128,128,64,64,xcd>", 6: "gemm_f32_3m_tiled<128,128,64,64>",
               7: "gemm_f32_3m_tiled<64,64,32,32,xcd,C prefetch>", 8: "gemm_f32_3m_tiled<64,64,32,32,xcd,K32>",
               9: "gemm_f32_3m_tiled<64,64,32,32,xcd,32x32x2>", 10: "gemm_f32_3m_persist<64,64,32,32,xcd>",
               11: "gemm_f32_3m_persist<64,64,32,32,xcd,C prefetch>", 12: "gemm_f32_3m_big<128,64>",
               13: "gemm_f32_3m_big<64,128>", 14: "gemm_f32_3m_big<128,128>",
               15: "gemm_f32_3m_big<64,64,prefetch 2>", 16: "gemm_f32_3m_big<64,128,prefetch 2>",
               17: "gemm_f32_3m_stream", 18: "gemm_f32_3m_stream<C prefetch>",
               19: "gemm_f32_3m_tiled<64,64,32,32,xcd,bands of 8>", 20: "gemm_f32_3m_big<64,128,bands of 8>"}
F64_TILINGS = {0: "gemm_f64_kernel", 1: "gemm_f64_tiled<64,64,32,32,xcd,K8>", 2: "gemm_f64_tiled<32,64,16,32,xcd,K8>",
               3: "gemm_f64_tiled<128,64,64,32,xcd,K8>", 4: "gemm_f64_tiled<64,128,32,64,xcd,K8>",
               5: "gemm_f64_tiled<64,64,32,32,K8>"}


def tune_all(ctx, npads, batch=256):
    """The autotuner over every kernel choice of the LU for each padded-size bucket the workload
    has (the largest npad of the bucket), and the split-mode panel threshold; the context keeps
    the fastest per bucket.  Returns the per-bucket record for the JSON line."""
    buckets = {}
    for n in npads:
        b = (n - 1) // 256
        buckets[b] = max(buckets.get(b, 0), n)
    rec = []
    for b, n in sorted(buckets.items()):
        entry = {"bucket": b, "npad_range": [256 * b + 1, 256 * (b + 1)], "tuned_at_npad": n}
        for what in ("f32_wide", "f32_narrow", "f64_wide", "f64_narrow"):
            if n <= 64 * ctx.knob("group_f32" if what.startswith("f32") else "group_f64"):
                continue  # matrices this small have no update of the autotuner's shapes
            best, ms = ctx.autotune_kernel(what, n, batch=batch)
            entry[what] = {"best": best, "ms": [round(m, 3) for m in ms]}
        rec.append(entry)
        log("autotuned bucket %d (npad %d): %s" % (b, n, {k: entry[k]["best"] for k in
                                                         ("f32_wide", "f32_narrow", "f64_wide", "f64_narrow")
                                                         if k in entry}))
    # the panel runs one workgroup per system, so its batch must fill the chip several times over
    thr, ms = ctx.autotune_kernel("f32_panel", batch=8 * batch)
    log("autotuned split-mode panel threshold: %d rows %s" % (thr, [round(m, 3) for m in ms]))
    return {"batch": batch, "buckets": rec,
            "panel_small_rows": {"best": thr, "heights": [256, 512, 768],
                                 "ms_small_large_per_height": [round(m, 3) for m in ms]}}


def gemm_roofline(ctx, precision, workload, tiling, timed_in):
    """The wide trailing update's roofline entry from the launches recorded while profiling."""
    gemm_ms, launches, flops, alg_bytes = ctx.kernel_stats(kind=1)
    if not launches:
        return None
    avg_s = gemm_ms / launches / 1e3
    achieved = flops / launches / avg_s
    peak = PEAK_FP32_MFMA if precision == "split" else PEAK_FP64_MFMA
    kname = (F32_TILINGS if precision == "split" else F64_TILINGS).get(tiling, "tiling %d" % tiling)
    with open(gemm_source(precision, tiling), "rb") as f:
        digest = hashlib.sha256(f.read()).hexdigest()
    rec = TRAFFIC.get((precision, workload, tiling))
    same_shape = rec is not None and abs(alg_bytes / launches / rec["alg_bytes_per_launch"] - 1) < 1e-3
    traffic = rec["bytes_per_launch"] if rec is not None and rec["sha256"] == digest and same_shape else None
    return {"kernel": kname, "bound": "mfma", "achieved": achieved / 1e12, "peak": peak / 1e12,
            "timed_in": timed_in, "unit": "TFLOP/s", "frac": achieved / peak, "traffic": traffic,
            "launches": launches, "avg_launch_ms": 1e3 * avg_s, "alg_flops_per_launch": flops / launches,
            "alg_bytes_per_launch": alg_bytes / launches}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="fcc4000")
    ap.add_argument("--precision", default="split", choices=["split", "fp64"])
    ap.add_argument("--no-fp64-compare", action="store_true")
    ap.add_argument("--cpu-sample", type=int, default=30)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--gemm-tiling", type=int, default=-1,
                    help="explicit tiling of the split-mode wide trailing update (-1: the autotuned one)")
    ap.add_argument("--group-f32", type=int, default=-1,
                    help="panels per group of the split-mode LU, 2 .. 4 (-1: the library default or the tuning cache's)")
    ap.add_argument("--group-f64", type=int, default=-1,
                    help="panels per group of the FP64 LU, 2 .. 4 (-1: the library default or the tuning cache's)")
    ap.add_argument("--no-autotune", action="store_true",
                    help="no autotuning: the library's defaults, or the tuning cache named by LSMS_TUNE_CACHE")
    ap.add_argument("--save-tuning", default=None,
                    help="write the autotuned kernel choices to this tuning cache (lsms_tuning_save)")
    ap.add_argument("--graphs", action=argparse.BooleanOptionalAction, default=True,
                    help="time the steps with each wave's factorization + first solve replayed from HIP graphs "
                         "(default); the trailing update's launch times then come from a second, eager timed "
                         "region over the same steps, which is reported too")
    ap.add_argument("--no-conj-leg", action="store_true",
                    help="skip the separately reported run that solves z+ only and derives tau(z-)")
    ap.add_argument("--paper-scale-atoms", type=int, default=26,
                    help="atoms of the 16,000-atom bcc alloy (965-site LIZ) timed in the separately reported "
                         "paper-scale leg (0: skip)")
    ap.add_argument("--no-ldlt-leg", action="store_true",
                    help="skip the separately reported run with the symmetric form and L D L^T")
    ap.add_argument("--no-adjoint-leg", action="store_true",
                    help="skip the separately reported gradient run (250-atom bcc alloy, d sigma_xx / d delta)")
    ap.add_argument("--paper-scale-only", action="store_true",
                    help="run only the paper-scale leg (for profiling it) and print its JSON object")
    ap.add_argument("--pipeline", action="store_true",
                    help="alternate the waves between two streams (LSMS_TUNE_PIPELINE)")
    ap.add_argument("--workspace-frac", type=float, default=0.8,
                    help="wave workspace as a fraction of free HBM after the inputs are allocated "
                         "(the library's own default is 0.6, which leaves more room for the caller)")
    ap.add_argument("--peak-probe", action="store_true",
                    help="print the device's sustained MFMA, FP64 FMA and HBM rates (lsms_peak_probe) as one "
                         "JSON line and exit")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="run one 1 GiB device-to-device copy before the timed region (scale for HBM counters)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on exactly one GPU: the library has no multi-GPU path "
              "(atoms are independent and shard across GPUs with one process per GPU)", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_2311_12134_amd as P
    import synthetic

    if args.peak_probe:
        ctx = P.Context(0)
        units = {"mfma_f64": "TFLOP/s", "mfma_f32": "TFLOP/s", "mfma_f32_32x32x2": "TFLOP/s", "fma_f64": "TFLOP/s",
                 "copy": "GB/s (read + written)", "write": "GB/s", "read": "GB/s"}
        res = {k: {"value": ctx.peak_probe(k), "unit": u} for k, u in units.items()}
        ctx.close()
        print(json.dumps(res), flush=True)
        return

    if args.paper_scale_only:
        ctx = P.Context(0)
        res = paper_scale_leg(P, torch, ctx, max(args.paper_scale_atoms, 1), args.precision,
                              ldlt=not args.no_ldlt_leg)
        ctx.close()
        print(json.dumps(res), flush=True)
        return

    w = synthetic.workload(args.workload)
    etas = list(w["etas"])
    dev = torch.device("cuda", 0)
    t0 = time.perf_counter()
    liz = P.build_liz(w["pos"], w["cell"], w["r_liz"])
    log("LIZ built in %.2f s: %d atoms, members %d..%d" % (time.perf_counter() - t0, liz.n_atoms,
                                                             np.diff(liz.ptr).min(), np.diff(liz.ptr).max()))
    la, lp = liz.to_device(dev)
    phase = torch.from_numpy(np.ascontiguousarray(w["phase"])).to(dev)
    species = torch.from_numpy(w["species"].astype(np.int32)).to(dev)
    J = torch.from_numpy(np.ascontiguousarray(w["J"])).to(dev)
    n_atoms = liz.n_atoms
    tp = torch.empty((liz.total, 16, 16), dtype=torch.complex128, device=dev)
    tm = torch.empty_like(tp)

    def outputs():
        # one set per broadening, so every eta's status and sums survive the timed region
        return {eta: {"info": torch.empty((n_atoms, 2), dtype=torch.int32, device=dev),
                      "berr": torch.empty((n_atoms, 2), dtype=torch.float64, device=dev),
                      "sig": torch.empty(3, dtype=torch.float64, device=dev),
                      "st": torch.empty((4, 3), dtype=torch.complex128, device=dev),
                      "pa": torch.empty((n_atoms, 4, 3), dtype=torch.complex128, device=dev)} for eta in etas}

    main_out = outputs()
    fp64_out = outputs() if (not args.no_fp64_compare and args.precision == "split") else None
    side_out = outputs()
    ws = int(args.workspace_frac * torch.cuda.mem_get_info()[0]) if args.workspace_frac > 0 else 0
    ctx = P.Context(0, workspace_limit=ws)
    ctx.set_pipeline(args.pipeline)
    ctx.set_gemm_tiling(args.gemm_tiling)
    if args.group_f32 > 0:
        ctx.set_knob("group_f32", args.group_f32)
    if args.group_f64 > 0:
        ctx.set_knob("group_f64", args.group_f64)
    tune = None
    npads = sorted({int(-(-16 * int(m) // 64) * 64) for m in np.diff(liz.ptr) if m > 0})
    if not args.no_autotune:
        tune = tune_all(ctx, npads)
        if args.save_tuning:
            ctx.tuning_save(args.save_tuning)

    def tiling_in_effect(precision):
        """The wide-update tiling the library picks for the workload's largest systems."""
        if precision == "split" and args.gemm_tiling >= 0:
            return args.gemm_tiling
        b = (npads[-1] - 1) // 256
        t = int(ctx.tuning_table("f32_wide" if precision == "split" else "f64_wide")[b])
        return t if t >= 0 else (19 if precision == "split" else 1)  # the library's defaults

    def step(i, precision, out):
        eta = etas[i % len(etas)]
        b = out[eta]
        ctx.tau_solve(liz, la, lp, phase, w["e_fermi"], eta, precision=precision, out=(tp, tm, b["info"], b["berr"]))
        ctx.kubo_sigma(liz, la, tp, tm, species, J, w["volume"], out=(b["sig"], b["st"], b["pa"]))

    def timed(precision, out, steps, graphs, profile):
        ctx.set_graphs(graphs)
        ctx.set_profiling(profile)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for i in range(steps):
            step(i, precision, out)
        torch.cuda.synchronize()
        return time.perf_counter() - t0

    if args.copy_calibration:
        src = torch.ones(1 << 28, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        log("copy calibration: %d bytes read, %d bytes written" % (src.numel() * 4, dst.numel() * 4))
        del src, dst

    ctx.set_graphs(args.graphs)
    for i in range(args.warmup):
        step(i, args.precision, main_out)
        torch.cuda.synchronize()
        log("warmup step %d done" % i)
    # The trailing update's launches are timed with HIP events on the stream they run on.  The
    # library records no events inside replayed graphs, so with graphs the headline region runs
    # unprofiled and a second, eager region over the same steps supplies the launch times.
    elapsed = timed(args.precision, main_out, args.steps, args.graphs, not args.graphs)
    eager = None
    if args.graphs:
        el_e = timed(args.precision, main_out, args.steps, False, True)
        eager = {"value": n_atoms * args.steps / el_e, "unit": "atoms/s", "ms_per_step": 1e3 * el_e / args.steps,
                 "what": "the same steps with every launch issued eagerly (trailing-update launches timed)"}
        log("eager region: %.1f ms/step" % (1e3 * el_e / args.steps))
    tiling = tiling_in_effect(args.precision)
    roof = gemm_roofline(ctx, args.precision, args.workload, tiling,
                         "the eager timed region" if args.graphs else "the timed region")
    narrow_ms, narrow_launches, narrow_flops, _ = ctx.kernel_stats(kind=0)
    ctx.set_profiling(False)
    ctx.set_graphs(False)
    ms_per_step = 1e3 * elapsed / args.steps
    value = n_atoms * args.steps / elapsed
    log("timed %d steps: %.1f ms/step, %.1f atoms/s%s" % (args.steps, ms_per_step, value,
                                                         " (graph replay)" if args.graphs else ""))

    n_true = 16 * np.diff(liz.ptr).astype(np.float64)
    alg_flops_step = float(np.sum(2.0 * ((8.0 / 3.0) * n_true**3 + 128.0 * n_true**2)))
    peak = PEAK_FP32_MFMA if args.precision == "split" else PEAK_FP64_MFMA
    timed_etas = sorted({etas[i % len(etas)] for i in range(max(args.steps, 1))}, reverse=True)
    out = {"metric": METRIC, "value": value, "unit": "atoms/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": ms_per_step, "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None,
           "dtype": "fp32 LU updates and refinement solves + fp64 pivot keys/residuals/solution" if args.precision == "split" else "f64",
           "data": "synthetic (seeded structure, phase shifts and current matrices)",
           "config": {"workload": "%s: %s, %d atoms, LIZ %d-%d atoms, lmax 3, eF %.2f Ry, eta cycling %s Ry"
                      % (w["name"], w["lattice"], n_atoms, int(n_true.min() / 16), int(n_true.max() / 16),
                         w["e_fermi"], etas),
                      "precision": args.precision, "gemm_tiling": tiling, "graphs": args.graphs,
                      "panels_per_group": ctx.knob("group_f32" if args.precision == "split" else "group_f64"),
                      "pipeline": args.pipeline, "workspace_frac": args.workspace_frac or 0.6,
                      "parallelism": "single GPU, all atoms batched"},
           "path_tflops_alg": alg_flops_step * args.steps / elapsed / 1e12,
           "path_frac_of_peak": alg_flops_step * args.steps / elapsed / peak}
    if eager is not None:
        eager["path_frac_of_peak"] = alg_flops_step * args.steps / (1e-3 * eager["ms_per_step"] * args.steps) / peak
        out["eager"] = eager
    if tune is not None:
        out["autotune"] = tune
    if roof is not None:
        out["roofline"] = roof
    if narrow_launches:
        out["narrow_update"] = {"launches": narrow_launches, "avg_launch_ms": narrow_ms / narrow_launches,
                                "achieved_tflops": narrow_flops / (narrow_ms / 1e3) / 1e12}
    per_eta = {}
    for eta in timed_etas:
        b = main_out[eta]
        info_np, berr_np = b["info"].cpu().numpy(), b["berr"].cpu().numpy()
        per_eta[eta] = {"eta": eta, "info_nonzero": int((info_np != 0).sum()), "berr_max": float(berr_np.max()),
                        "sigma": b["sig"].cpu().numpy().tolist()}
    out["info_nonzero"] = sum(v["info_nonzero"] for v in per_eta.values())
    if fp64_out is not None:
        # the plain FP64 GPU path, one step per broadening after one warm-up step, its wide
        # trailing update timed like the split mode's
        step(0, "fp64", fp64_out)
        torch.cuda.synchronize()
        t64 = timed("fp64", fp64_out, len(etas), False, True)
        roof64 = gemm_roofline(ctx, "fp64", args.workload, tiling_in_effect("fp64"), "the FP64 steps")
        ctx.set_profiling(False)
        fp64_ms = 1e3 * t64 / len(etas)
        out["fp64_ms_per_step"] = fp64_ms
        out["fp64_atoms_per_s"] = n_atoms / (1e-3 * fp64_ms)
        out["split_speedup_vs_fp64"] = value / out["fp64_atoms_per_s"]
        if roof64 is not None:
            out["fp64_roofline"] = roof64
        errs = []
        for eta in timed_etas:
            s64 = fp64_out[eta]["sig"].cpu().numpy()
            e = float(np.abs(np.array(per_eta[eta]["sigma"]) - s64).max() / np.abs(s64).max())
            per_eta[eta]["sigma_fp64"] = s64.tolist()
            per_eta[eta]["sigma_rel_err_split_vs_fp64"] = e
            per_eta[eta]["fp64_info_nonzero"] = int((fp64_out[eta]["info"].cpu().numpy() != 0).sum())
            errs.append(e)
        out["sigma_rel_err_split_vs_fp64"] = max(errs)
        log("fp64 step %.1f ms; max sigma rel err split vs fp64 %.2e" % (fp64_ms, max(errs)))
    if not args.no_conj_leg:
        # Algorithmic saving, reported apart from the like-for-like value above: solve z+ only
        # and write tau(z-) = P conj tau(z+) P (exact for real phase shifts).
        ctx.set_conj_symmetry(True)
        step(0, args.precision, side_out)
        torch.cuda.synchronize()
        tc = timed(args.precision, side_out, args.steps, False, False)
        errs = [float(np.abs(side_out[e]["sig"].cpu().numpy() - main_out[e]["sig"].cpu().numpy()).max()
                      / np.abs(main_out[e]["sig"].cpu().numpy()).max()) for e in timed_etas]
        combined = None
        if not args.no_ldlt_leg and args.precision == "split":
            # both savings together: z+ only, factored through the symmetric form
            ctx.set_symmetric(True)
            step(0, args.precision, side_out)
            torch.cuda.synchronize()
            combined = n_atoms * args.steps / timed(args.precision, side_out, args.steps, False, False)
            ctx.set_symmetric(False)
        ctx.set_conj_symmetry(False)
        out["conj_symmetry"] = {"value": n_atoms * args.steps / tc, "unit": "atoms/s",
                                "ms_per_step": 1e3 * tc / args.steps,
                                "speedup_vs_full_solve": (n_atoms * args.steps / tc) / value,
                                "sigma_rel_err_vs_full_solve": max(errs),
                                "what": "z+ systems only; tau(z-)_{LL'} = (-1)^(l+l') conj tau(z+)_{LL'}",
                                "with_symmetric_ldlt": combined}
        log("conj-symmetry leg: %.1f ms/step, %.1f atoms/s" % (1e3 * tc / args.steps, n_atoms * args.steps / tc))
    if not args.no_ldlt_leg and args.precision == "split":
        # Algorithmic saving, reported apart: the complex-symmetric form 1 - T^1/2 g T^1/2 factored
        # by L D L^T without pivoting (half the trailing-update work), FP64 refinement as before.
        ctx.set_symmetric(True)
        step(0, args.precision, side_out)
        torch.cuda.synchronize()
        tl = timed(args.precision, side_out, args.steps, False, False)
        ctx.set_symmetric(False)
        errs = [float(np.abs(side_out[e]["sig"].cpu().numpy() - main_out[e]["sig"].cpu().numpy()).max()
                      / np.abs(main_out[e]["sig"].cpu().numpy()).max()) for e in timed_etas]
        out["symmetric_ldlt"] = {"value": n_atoms * args.steps / tl, "unit": "atoms/s",
                                 "ms_per_step": 1e3 * tl / args.steps,
                                 "speedup_vs_lu": (n_atoms * args.steps / tl) / value,
                                 "sigma_rel_err_vs_lu": max(errs),
                                 "info_nonzero": sum(int((side_out[e]["info"].cpu().numpy() != 0).sum())
                                                     for e in timed_etas),
                                 "what": "S = 1 - T^1/2 g T^1/2, unpivoted L D L^T in FP32 (lower-triangle updates), "
                                         "FP64 refinement and fallback; not the paper's LU"}
        log("symmetric L D L^T leg: %.1f ms/step, %.1f atoms/s" % (1e3 * tl / args.steps, n_atoms * args.steps / tl))
    if args.paper_scale_atoms > 0:
        out["paper_scale_liz"] = paper_scale_leg(P, torch, ctx, args.paper_scale_atoms, args.precision,
                                                 ldlt=not args.no_ldlt_leg)
    if not args.no_adjoint_leg:
        out["adjoint"] = adjoint_leg(P, torch, ctx)
    main_pa = {e: main_out[e]["pa"].cpu().numpy() for e in timed_etas}
    fp64_pa = {e: fp64_out[e]["pa"].cpu().numpy() for e in timed_etas} if fp64_out is not None else None
    ctx.close()
    if not args.no_cpu_baseline:
        cb, _, groups, oracle_pa = cpu_baseline(w, timed_etas, args.cpu_sample)
        out["cpu_baseline"] = cb
        for eta, e in oracle_errors(groups, oracle_pa, main_pa).items():
            per_eta[eta]["kubo_per_atom_rel_err_vs_oracle"] = e
            per_eta[eta]["oracle_atoms"] = groups[eta]
        if fp64_pa is not None:
            for eta, e in oracle_errors(groups, oracle_pa, fp64_pa).items():
                per_eta[eta]["kubo_per_atom_rel_err_vs_oracle_fp64"] = e
    out["per_eta"] = [per_eta[e] for e in timed_etas]
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
