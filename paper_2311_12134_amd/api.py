"""Thin PyTorch binding of the C ABI (include/lsms_kkr.h).

PyTorch only provides device memory and the current HIP stream; every step of the
path (assembly, LU, solves, refinement, Kubo sums, adjoint) runs in liblsms_kkr.so.
"""

import ctypes
from dataclasses import dataclass

import numpy as np
import torch

from . import _lib
from ._lib import check, lib

NL = 16


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


@dataclass
class Liz:
    """CSR local interaction zones: ptr [N+1] int64 (host), atom [S] int32, pos [S,3] float64."""
    ptr: np.ndarray
    atom: np.ndarray
    pos: np.ndarray

    @property
    def n_atoms(self):
        return len(self.ptr) - 1

    @property
    def total(self):
        return int(self.ptr[-1])

    def to_device(self, device):
        return (torch.from_numpy(np.ascontiguousarray(self.atom)).to(device),
                torch.from_numpy(np.ascontiguousarray(self.pos)).to(device))


def gaunt_table():
    """The library's Gaunt table [16, 16, 49] (host query, no GPU needed)."""
    out = np.zeros((NL, NL, 49), dtype=np.float64)
    check(lib().lsms_gaunt_table(out.ctypes.data_as(ctypes.c_void_p)))
    return out


def build_liz(pos, cell, r_liz, centres=None):
    """LIZ construction in the library (host C++); no context or GPU needed.  With
    ``centres`` only those atoms get their LIZ (the others an empty one, which the solves
    and Kubo sums skip)."""
    pos = np.ascontiguousarray(pos, dtype=np.float64)
    n = pos.shape[0]
    cellp = None
    if cell is not None:
        cell = np.ascontiguousarray(cell, dtype=np.float64)
        cellp = cell.ctypes.data_as(ctypes.c_void_p)
    ptr = np.zeros(n + 1, dtype=np.int64)
    needed = ctypes.c_int64(0)
    if centres is None:
        def call(cap, atom, disp):
            return lib().lsms_build_liz(None, n, pos.ctypes.data_as(ctypes.c_void_p), cellp, float(r_liz), cap,
                                        ptr.ctypes.data_as(ctypes.c_void_p), atom, disp, ctypes.byref(needed))
    else:
        cen = np.ascontiguousarray(centres, dtype=np.int32)

        def call(cap, atom, disp):
            return lib().lsms_build_liz_subset(None, n, pos.ctypes.data_as(ctypes.c_void_p), cellp, float(r_liz),
                                               int(cen.size), cen.ctypes.data_as(ctypes.c_void_p), cap,
                                               ptr.ctypes.data_as(ctypes.c_void_p), atom, disp,
                                               ctypes.byref(needed))
    rc = call(0, None, None)
    if rc not in (_lib.LSMS_OK, _lib.LSMS_E_CAPACITY):
        check(rc)
    cap = needed.value
    atom = np.zeros(cap, dtype=np.int32)
    disp = np.zeros((cap, 3), dtype=np.float64)
    check(call(cap, atom.ctypes.data_as(ctypes.c_void_p), disp.ctypes.data_as(ctypes.c_void_p)))
    return Liz(ptr, atom, disp)


class Factors:
    """Library-owned LU factors kept by a tau solve for the adjoint."""

    def __init__(self, handle, ctx):
        self.handle = handle
        self.ctx = ctx

    def free(self):
        if self.handle is not None and self.handle.value:
            check(lib().lsms_factors_free(self.handle))
        self.handle = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


class Context:
    """A library context on one GPU (lmax = 3)."""

    def __init__(self, device=0, workspace_limit=0):
        if not torch.cuda.is_available():
            raise RuntimeError("the LSMS tau-solve library needs a HIP device")
        self.device = torch.device("cuda", device)
        self._h = ctypes.c_void_p()
        check(lib().lsms_create(device, 3, int(workspace_limit), ctypes.byref(self._h)))

    def close(self):
        if self._h is not None and self._h.value:
            check(lib().lsms_destroy(self._h))
        self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- tau ------------------------------------------------------------------------
    def tau_solve(self, liz, liz_atom_dev, liz_pos_dev, phase, e_fermi, eta, precision="fp64", refine_tol=1e-14,
                  max_refine=10, keep=False, out=None):
        """tau^{a0}(z+-) for every atom: returns (tau_plus, tau_minus, info, berr[, factors])."""
        prec = {"fp64": _lib.LSMS_FP64, "split": _lib.LSMS_SPLIT}[precision]
        n = liz.n_atoms
        assert phase.is_cuda and phase.dtype == torch.float64 and phase.shape == (n, 4) and phase.is_contiguous()
        assert liz_atom_dev.dtype == torch.int32 and liz_pos_dev.dtype == torch.float64
        if out is None:
            tp = torch.empty((liz.total, NL, NL), dtype=torch.complex128, device=self.device)
            tm = torch.empty_like(tp)
            info = torch.empty((n, 2), dtype=torch.int32, device=self.device)
            berr = torch.empty((n, 2), dtype=torch.float64, device=self.device)
        else:
            tp, tm, info, berr = out
        fh = ctypes.c_void_p() if keep else None
        check(lib().lsms_tau_solve(self._h, n, liz.ptr.ctypes.data_as(ctypes.c_void_p), _ptr(liz_atom_dev),
                                   _ptr(liz_pos_dev), _ptr(phase), float(e_fermi), float(eta), prec,
                                   float(refine_tol), int(max_refine), _ptr(tp), _ptr(tm), _ptr(info), _ptr(berr),
                                   ctypes.byref(fh) if keep else None, _stream()))
        if keep:
            return tp, tm, info, berr, Factors(fh, self)
        return tp, tm, info, berr

    # -- Kubo-Greenwood -----------------------------------------------------------------
    def kubo_sigma(self, liz, liz_atom_dev, tau_plus, tau_minus, species, J, volume, per_atom=False, out=None):
        """sigma [3] (float64), sigma_tilde [4,3] (complex128) and optionally per-atom sums [N,4,3]."""
        n = liz.n_atoms
        assert species.dtype == torch.int32 and J.dtype == torch.complex128 and J.is_contiguous()
        n_species = J.shape[0]
        if out is None:
            sig = torch.empty(3, dtype=torch.float64, device=self.device)
            st = torch.empty((4, 3), dtype=torch.complex128, device=self.device)
            pa = torch.empty((n, 4, 3), dtype=torch.complex128, device=self.device) if per_atom else None
        else:
            sig, st, pa = out
        check(lib().lsms_kubo_sigma(self._h, n, liz.ptr.ctypes.data_as(ctypes.c_void_p), _ptr(liz_atom_dev),
                                    _ptr(tau_plus), _ptr(tau_minus), _ptr(species), n_species, _ptr(J),
                                    float(volume), _ptr(sig), _ptr(st), _ptr(pa), _stream()))
        return sig, st, pa

    def kubo_sigma_noalloc(self, liz_ptr_dev, liz_atom_dev, tau_plus, tau_minus, species, J, volume, sigma,
                           sigma_tilde, per_atom=None):
        """lsms_kubo_sigma_noalloc: the caller passes every array (liz_ptr on the device,
        int64 [N+1]); the library allocates nothing and uses its fixed per-GPU scratch for the
        per-atom sums when per_atom is None."""
        n = liz_ptr_dev.numel() - 1
        assert liz_ptr_dev.is_cuda and liz_ptr_dev.dtype == torch.int64
        assert species.dtype == torch.int32 and J.dtype == torch.complex128 and J.is_contiguous()
        check(lib().lsms_kubo_sigma_noalloc(self._h, n, _ptr(liz_ptr_dev), _ptr(liz_atom_dev), _ptr(tau_plus),
                                            _ptr(tau_minus), _ptr(species), J.shape[0], _ptr(J), float(volume),
                                            _ptr(sigma), _ptr(sigma_tilde), _ptr(per_atom), _stream()))
        return sigma, sigma_tilde, per_atom

    def kubo_sigma_tensor(self, liz, liz_atom_dev, tau_plus, tau_minus, species, J, volume, per_atom=False,
                          out=None):
        """sigma [3,3] (float64, row mu, column nu), sigma_tilde [4,3,3] (complex128), per-atom sums [N,4,3,3]."""
        n = liz.n_atoms
        assert species.dtype == torch.int32 and J.dtype == torch.complex128 and J.is_contiguous()
        n_species = J.shape[0]
        if out is None:
            sig = torch.empty((3, 3), dtype=torch.float64, device=self.device)
            st = torch.empty((4, 3, 3), dtype=torch.complex128, device=self.device)
            pa = torch.empty((n, 4, 3, 3), dtype=torch.complex128, device=self.device) if per_atom else None
        else:
            sig, st, pa = out
        check(lib().lsms_kubo_sigma_tensor(self._h, n, liz.ptr.ctypes.data_as(ctypes.c_void_p), _ptr(liz_atom_dev),
                                           _ptr(tau_plus), _ptr(tau_minus), _ptr(species), n_species, _ptr(J),
                                           float(volume), _ptr(sig), _ptr(st), _ptr(pa), _stream()))
        return sig, st, pa

    def kubo_sigma_grad(self, factors, liz, liz_atom_dev, phase, tau_plus, tau_minus, species, J, volume, dsigma):
        n = liz.n_atoms
        dphase = torch.empty((n, 4), dtype=torch.float64, device=self.device)
        dsig = dsigma.to(device=self.device, dtype=torch.float64).contiguous()
        check(lib().lsms_kubo_sigma_grad(self._h, factors.handle, n, liz.ptr.ctypes.data_as(ctypes.c_void_p),
                                         _ptr(liz_atom_dev), _ptr(phase), _ptr(tau_plus), _ptr(tau_minus),
                                         _ptr(species), J.shape[0], _ptr(J), float(volume), _ptr(dsig),
                                         _ptr(dphase), _stream()))
        return dphase

    # -- measurement ---------------------------------------------------------------------
    def set_profiling(self, on=True):
        check(lib().lsms_set_profiling(self._h, 1 if on else 0))

    def set_gemm_tiling(self, variant):
        """Tiling of the split-mode trailing update (-1: library default)."""
        check(lib().lsms_set_tuning(self._h, 0, int(variant)))

    def set_graphs(self, on=True):
        """Replay each wave's factorization and first solve from captured HIP graphs."""
        check(lib().lsms_set_tuning(self._h, 1, 1 if on else 0))

    def set_lookahead(self, on=True):
        """Factor the next group's first panel on a second stream during the trailing update."""
        check(lib().lsms_set_tuning(self._h, 4, 1 if on else 0))

    def set_symmetric(self, on=True):
        """Split mode: symmetric form and L D L^T (no pivoting) with FP64 refinement and
        fallback, instead of the LU (not with kept factors)."""
        check(lib().lsms_set_tuning(self._h, 5, 1 if on else 0))

    def set_pipeline(self, on=True):
        """Alternate waves between two streams so one wave's refinement overlaps the next
        wave's factorization (default off; with one padded size the results are bitwise the
        same)."""
        check(lib().lsms_set_tuning(self._h, 6, 1 if on else 0))

    def pipeline(self):
        v = ctypes.c_int(0)
        check(lib().lsms_get_tuning(self._h, 6, ctypes.byref(v)))
        return bool(v.value)

    def set_tslu_chunk(self, rows=2048):
        """Rows per chunk of the tournament-pivoting panels (used for panels taller than
        2 * rows; a multiple of 64 in [64, 2048])."""
        check(lib().lsms_set_tuning(self._h, 3, int(rows)))

    def tslu_chunk(self):
        v = ctypes.c_int(0)
        check(lib().lsms_get_tuning(self._h, 3, ctypes.byref(v)))
        return v.value

    def set_conj_symmetry(self, on=True):
        """Solve z+ only and derive tau(z-) = P conj tau(z+) P (P = diag((-1)^l)); not used
        when factors are kept for the adjoint."""
        check(lib().lsms_set_tuning(self._h, 2, 1 if on else 0))

    def conj_symmetry(self):
        v = ctypes.c_int(0)
        check(lib().lsms_get_tuning(self._h, 2, ctypes.byref(v)))
        return bool(v.value)

    def autotune(self, npad, batch=256):
        """Time every split-mode tiling for systems of padded size npad on a synthetic batch
        and adopt the fastest; returns (best tiling, [ms per tiling])."""
        best = ctypes.c_int(-1)
        ms = (ctypes.c_float * 21)()
        check(lib().lsms_autotune(self._h, int(npad), int(batch), ctypes.byref(best), ms, _stream()))
        return best.value, [float(x) for x in ms]

    AUTOTUNE_TARGETS = {"f32_wide": 0, "f32_narrow": 1, "f64_wide": 2, "f64_narrow": 3, "f32_panel": 4}
    KNOBS = {"f32_wide": 0, "f32_narrow": 7, "f64_wide": 8, "f64_narrow": 9, "panel_small_rows": 10,
             "group_f32": 11, "group_f64": 12}

    def autotune_kernel(self, what, npad=0, batch=256):
        """lsms_autotune_kernel: time every variant of one LU kernel (see AUTOTUNE_TARGETS) and
        record the fastest for npad's bucket (the panel target: the small-panel threshold).
        Returns (best, [ms per variant])."""
        best = ctypes.c_int(-1)
        ms = (ctypes.c_float * 21)()
        check(lib().lsms_autotune_kernel(self._h, self.AUTOTUNE_TARGETS[what], int(npad), int(batch),
                                         ctypes.byref(best), ms, 21, _stream()))
        n = {"f32_wide": 21, "f32_narrow": 21, "f64_wide": 6, "f64_narrow": 6, "f32_panel": 6}[what]
        return best.value, [float(x) for x in ms[:n]]

    PROBES = {"mfma_f64": 0, "mfma_f32": 1, "mfma_f32_32x32x2": 2, "fma_f64": 3, "copy": 4, "write": 5, "read": 6}

    def peak_probe(self, what):
        """lsms_peak_probe: the device's sustained rate for one instruction stream (TFLOP/s) or
        a 1 GiB copy (GB/s)."""
        v = ctypes.c_double(0)
        check(lib().lsms_peak_probe(self._h, self.PROBES[what], ctypes.byref(v), _stream()))
        return v.value

    def tuning_table(self, what):
        """The autotuned choice per npad bucket (bucket b: npad in (256 b, 256 (b + 1)]), -1 if
        none; for "f32_panel" the panel threshold."""
        out = np.full(64, -1, dtype=np.int32)
        check(lib().lsms_tuning_table(self._h, self.AUTOTUNE_TARGETS[what], out.ctypes.data_as(ctypes.c_void_p)))
        return int(out[0]) if what == "f32_panel" else out

    def tuning_save(self, path):
        check(lib().lsms_tuning_save(self._h, str(path).encode()))

    def tuning_load(self, path):
        check(lib().lsms_tuning_load(self._h, str(path).encode()))

    def set_knob(self, name, value):
        """Explicit kernel choice (see KNOBS); -1 returns to the autotuned choice or the default."""
        check(lib().lsms_set_tuning(self._h, self.KNOBS[name], int(value)))

    def knob(self, name):
        v = ctypes.c_int(0)
        check(lib().lsms_get_tuning(self._h, self.KNOBS[name], ctypes.byref(v)))
        return v.value

    def gemm_tiling(self):
        v = ctypes.c_int(0)
        check(lib().lsms_get_tuning(self._h, 0, ctypes.byref(v)))
        return v.value

    def kernel_stats(self, kind=1):
        """(total ms, launches, algorithmic flops, algorithmic bytes) of the recorded
        trailing-update launches: kind 1 the wide (K = 128) updates, 0 the narrow ones,
        -1 all."""
        ms = ctypes.c_double(0)
        n = ctypes.c_int64(0)
        fl = ctypes.c_double(0)
        by = ctypes.c_double(0)
        check(lib().lsms_kernel_stats(self._h, int(kind), ctypes.byref(ms), ctypes.byref(n), ctypes.byref(fl),
                                      ctypes.byref(by)))
        return ms.value, n.value, fl.value, by.value

    # -- diagnostic batched solve ------------------------------------------------------
    def batched_lu_solve(self, mats, rhs, precision="fp64"):
        """Solve A_b X_b = B_b in place of B_b (lists of CUDA complex128 tensors); returns info [batch]."""
        batch = len(mats)
        ns = np.array([m.shape[0] for m in mats], dtype=np.int32)
        nrhs = rhs[0].shape[1]
        aptr = (ctypes.c_void_p * batch)(*[m.data_ptr() for m in mats])
        bptr = (ctypes.c_void_p * batch)(*[b.data_ptr() for b in rhs])
        info = torch.zeros(batch, dtype=torch.int32, device=self.device)
        prec = {"fp64": _lib.LSMS_FP64, "split": _lib.LSMS_SPLIT}[precision]
        check(lib().lsms_batched_lu_solve(self._h, batch, ns.ctypes.data_as(ctypes.c_void_p), aptr, bptr, nrhs,
                                          prec, _ptr(info), _stream()))
        return info


class KuboSigma(torch.autograd.Function):
    """sigma(phase) through the library, with the hand-written adjoint as backward.

    forward(ctx, phase, lsms_context, liz, liz_atom_dev, liz_pos_dev, species, J, volume, e_fermi, eta)
    """

    @staticmethod
    def forward(ctx, phase, lctx, liz, liz_atom_dev, liz_pos_dev, species, J, volume, e_fermi, eta):
        phase = phase.contiguous()
        tp, tm, info, berr, fac = lctx.tau_solve(liz, liz_atom_dev, liz_pos_dev, phase, e_fermi, eta, keep=True)
        sig, _, _ = lctx.kubo_sigma(liz, liz_atom_dev, tp, tm, species, J, volume)
        ctx.lctx = lctx
        ctx.liz = liz
        ctx.fac = fac
        ctx.volume = volume
        ctx.save_for_backward(phase, liz_atom_dev, tp, tm, species, J)
        return sig

    @staticmethod
    def backward(ctx, gsig):
        phase, liz_atom_dev, tp, tm, species, J = ctx.saved_tensors
        dphase = ctx.lctx.kubo_sigma_grad(ctx.fac, ctx.liz, liz_atom_dev, phase, tp, tm, species, J, ctx.volume,
                                          gsig)
        ctx.fac.free()
        return (dphase,) + (None,) * 9
