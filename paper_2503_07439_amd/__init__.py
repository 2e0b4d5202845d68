"""Event-parallel tree-level matrix elements on AMD MI355X.

The computation lives in libnlome.so (hand-written HIP for gfx950, C ABI in
include/nlome.h).  This package holds the ctypes binding, a torch-facing
convenience layer (torch supplies device memory and streams only), and the
build-time diagram generator."""
from . import _lib
from ._lib import (NLO_FP64, NLO_FP32, NLO_FP16, NLO_BF16, NLO_MIXED, PREC, NloError,  # noqa: F401
                   nlo_abi_version, nlo_create, nlo_destroy, nlo_last_error, nlo_num_processes,
                   nlo_process_info, nlo_set_kernel_config, nlo_get_kernel_config, nlo_me2,
                   nlo_subtracted, nlo_subtracted_static, nlo_set_fks_threshold, nlo_fks_out, nlo_work_item, nlo_batch_plan,
                   nlo_batch_run, nlo_plan_destroy, NLO_ITEM_ME2, NLO_ITEM_SUBTRACTED, nlo_autotune,
                   nlo_uniforms, nlo_phase_space, nlo_fks_variables, nlo_cross_section, nlo_set_fks_mask_mode,
                   nlo_me2_checked, nlo_reserve, nlo_colour_unit, nlo_integrate_subtracted, nlo_fks_config,
                   nlo_set_fks_config, nlo_get_fks_config, nlo_autotune_subtracted, nlo_tuning_cache, nlo_cuts,
                   make_cuts, nlo_cut_mask, nlo_fks_cut_masks, nlo_generate_passing, nlo_virtual_integrated,
                   nlo_fks_buffer_create, nlo_fks_buffer_push, nlo_fks_buffer_flush, nlo_fks_buffer_destroy)

PROCESSES = ["ee_mumu", "ee_uu", "ee_uug", "gg_tt", "uu_tt", "gg_ttg", "uu_ttg", "ug_ttu", "gg_ttgg"]


def proc_id(name):
    return PROCESSES.index(name)


class Context:
    """Owns one nlo_ctx.  Tensors are torch CUDA tensors (HIP device memory);
    launches go on torch's current stream."""

    def __init__(self, alpha=1.0 / 132.507, alpha_s=0.118, m_top=173.0, device=0):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("paper_2503_07439_amd needs a HIP device")
        self.device = device
        self.ctx = nlo_create(alpha, alpha_s, m_top, device)
        self.reserved = 0

    def reserve(self, n):
        """Size the context workspace for evaluation calls of up to n events
        (host side, before the call: the calls themselves never allocate)."""
        if n > self.reserved:
            nlo_reserve(self.ctx, n)
            self.reserved = n

    def close(self):
        if self.ctx is not None:
            nlo_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def info(self, proc):
        return nlo_process_info(self.ctx, proc_id(proc))

    def _stream(self):
        import torch
        return torch.cuda.current_stream(self.device).cuda_stream

    def me2(self, proc, mom, prec="fp64", out=None):
        """mom: float64 CUDA tensor [npart, 4, n] (or [npart, 4, ld] with n
        given by out).  Returns |M|^2 [n] (float64, CUDA)."""
        import torch
        assert mom.dtype == torch.float64 and mom.is_cuda and mom.is_contiguous()
        npart, four, ld = mom.shape
        n = ld if out is None else out.shape[0]
        if out is None:
            out = torch.empty(n, dtype=torch.float64, device=mom.device)
        if prec in ("fp16", "bf16"):
            self.reserve(n)
        nlo_me2(self.ctx, proc_id(proc), n, ld, mom.data_ptr(), out.data_ptr(), PREC[prec], self._stream())
        return out

    def me2_checked(self, proc, mom, prec="fp64"):
        """(|M|^2 [n], status [n] uint8): bit0 non-finite or negative result,
        bit1 non-finite input, bit2 FP32 pass of a half-width evaluation."""
        import torch
        assert mom.dtype == torch.float64 and mom.is_cuda and mom.is_contiguous()
        npart, four, n = mom.shape
        out = torch.empty(n, dtype=torch.float64, device=mom.device)
        st = torch.empty(n, dtype=torch.uint8, device=mom.device)
        if prec in ("fp16", "bf16"):
            self.reserve(n)
        nlo_me2_checked(self.ctx, proc_id(proc), n, n, mom.data_ptr(), out.data_ptr(), st.data_ptr(), PREC[prec],
                        self._stream())
        return out, st

    def colour_unit(self, proc, prec):
        """"valu" or "mfma": the colour-contraction unit (proc, prec) runs on."""
        return {1: "valu", 2: "mfma"}[nlo_colour_unit(self.ctx, proc_id(proc), PREC[prec])]

    FKS_FIELDS = ("W", "xi", "born", "g_R", "g_S", "g_C", "g_Cm", "g_SC", "g_SCm", "dsig", "jac")

    def subtracted(self, real, fks_i, fks_j, born_mom, xi_tilde, y, phi, prec="fp64", mask=None,
                   want_real=False, want_sum=False):
        """FKS-subtracted real emission.  born_mom: float64 CUDA tensor
        [npart_born, 4, n]; xi_tilde, y, phi: float64 CUDA [n]; mask: uint8
        CUDA [4, n] or None.  Returns a dict of CUDA tensors."""
        import torch
        npart, _, n = born_mom.shape
        dev = born_mom.device
        res = {k: torch.empty(n, dtype=torch.float64, device=dev) for k in self.FKS_FIELDS}
        res["status"] = torch.empty(n, dtype=torch.uint8, device=dev)
        out = nlo_fks_out()
        for k in self.FKS_FIELDS:
            setattr(out, k, res[k].data_ptr())
        out.status = res["status"].data_ptr()
        if want_real:
            res["real_mom"] = torch.empty((npart + 1, 4, n), dtype=torch.float64, device=dev)
            out.real_mom = res["real_mom"].data_ptr()
        if want_sum:
            res["w_sum"] = torch.empty(1, dtype=torch.float64, device=dev)
            out.w_sum = res["w_sum"].data_ptr()
        for t in (born_mom, xi_tilde, y, phi):
            assert t.dtype == torch.float64 and t.is_cuda and t.is_contiguous()
        mptr = 0
        if mask is not None:
            assert mask.dtype == torch.uint8 and mask.shape == (4, n) and mask.is_contiguous()
            mptr = mask.data_ptr()
        self.reserve(n)
        nlo_subtracted(self.ctx, proc_id(real), fks_i, fks_j, n, n, born_mom.data_ptr(), xi_tilde.data_ptr(),
                       y.data_ptr(), phi.data_ptr(), mptr, PREC[prec], out, self._stream())
        return res

    def autotune(self, proc, mom, prec="mixed"):
        """Time every launch configuration on this sample and keep the fastest.
        Returns ((block, colour_mode, schedule), ns per event)."""
        import torch
        n = mom.shape[2]
        out = torch.empty(n, dtype=torch.float64, device=mom.device)
        if prec in ("fp16", "bf16"):
            self.reserve(n)
        return nlo_autotune(self.ctx, proc_id(proc), PREC[prec], n, n, mom.data_ptr(), out.data_ptr(),
                            self._stream())

    def autotune_subtracted(self, real, fks_i, fks_j, born_mom, xi_tilde, y, phi, prec="mixed"):
        """Time the launch configurations of one FKS sector on this sample and
        keep the fastest.  Returns ((real_block, colour_mode, ct_block), ns per
        event)."""
        import torch
        n = born_mom.shape[2]
        w = torch.empty(n, dtype=torch.float64, device=born_mom.device)
        self.reserve(n)
        return nlo_autotune_subtracted(self.ctx, proc_id(real), fks_i, fks_j, n, n, born_mom.data_ptr(),
                                       xi_tilde.data_ptr(), y.data_ptr(), phi.data_ptr(), PREC[prec], w.data_ptr(),
                                       self._stream())

    def set_fks_config(self, real, fks_i, fks_j, prec, real_block, colour_mode, ct_block):
        nlo_set_fks_config(self.ctx, proc_id(real), fks_i, fks_j, PREC[prec], real_block, colour_mode, ct_block)

    def fks_config(self, real, fks_i, fks_j, prec):
        """(real_block, colour_mode, ct_block) of one FKS sector and precision."""
        return nlo_get_fks_config(self.ctx, proc_id(real), fks_i, fks_j, PREC[prec])

    def kernel_config(self, proc, prec):
        """(block, colour_mode, schedule) of one process and precision."""
        return nlo_get_kernel_config(self.ctx, proc_id(proc), PREC[prec])

    def fks_buffer(self, real, fks_i, fks_j, prec, threshold, w_out):
        """A buffered evaluator of one FKS sector adding W contributions to
        w_out (float64 CUDA, zeroed by the caller): .push(born, xt, y, phi,
        mask, slot), .flush(), .close()."""
        ctx = self

        class _Buf:
            def __init__(self):
                self.b = nlo_fks_buffer_create(ctx.ctx, proc_id(real), fks_i, fks_j, PREC[prec], threshold,
                                               w_out.data_ptr())

            def push(self, born, xt, y, phi, mask, slot):
                n = born.shape[2]
                nlo_fks_buffer_push(self.b, n, n, born.data_ptr(), xt.data_ptr(), y.data_ptr(), phi.data_ptr(),
                                    mask.data_ptr() if mask is not None else None, slot.data_ptr(), ctx._stream())

            def flush(self):
                nlo_fks_buffer_flush(self.b, ctx._stream())

            def close(self):
                if self.b:
                    nlo_fks_buffer_destroy(self.b)
                    self.b = None

        return _Buf()

    def virtual_integrated(self, born_proc, mom, prec="fp64"):
        """(Born |M|^2, finite virtual + integrated counterterms) per event, CUDA [n] each"""
        import torch
        n = mom.shape[2]
        b = torch.empty(n, dtype=torch.float64, device=mom.device)
        vi = torch.empty(n, dtype=torch.float64, device=mom.device)
        nlo_virtual_integrated(self.ctx, proc_id(born_proc), n, n, mom.data_ptr(), PREC[prec], b.data_ptr(),
                               vi.data_ptr(), self._stream())
        return b, vi

    def cut_mask(self, proc, mom, cuts):
        """uint8 CUDA [n]: 1 where an event passes the cuts (dict of nlo_cuts fields)"""
        import torch
        n = mom.shape[2]
        out = torch.empty(n, dtype=torch.uint8, device=mom.device)
        nlo_cut_mask(self.ctx, proc_id(proc), n, n, mom.data_ptr(), make_cuts(cuts), out.data_ptr(), self._stream())
        return out

    def fks_cut_masks(self, real, fks_i, fks_j, born_mom, xi_tilde, y, phi, cuts):
        """uint8 CUDA [4][n]: the B, R, S, C masks of nlo_subtracted from the cuts"""
        import torch
        n = born_mom.shape[2]
        out = torch.empty((4, n), dtype=torch.uint8, device=born_mom.device)
        nlo_fks_cut_masks(self.ctx, proc_id(real), fks_i, fks_j, n, n, born_mom.data_ptr(), xi_tilde.data_ptr(),
                          y.data_ptr(), phi.data_ptr(), make_cuts(cuts), out.data_ptr(), self._stream())
        return out

    def generate_passing(self, proc, n, sqrt_s, stream, cuts, first=0, seed=7439):
        """n RAMBO points that pass the cuts, in candidate order: (mom CUDA
        [npart][4][n], weight [n], number of candidates used)"""
        import torch
        lo, hi = sqrt_s if isinstance(sqrt_s, tuple) else (sqrt_s, sqrt_s)
        npart = self.info(proc).npart
        mom = torch.empty((npart, 4, n), dtype=torch.float64, device="cuda")
        w = torch.empty(n, dtype=torch.float64, device="cuda")
        self.reserve(1)
        t = nlo_generate_passing(self.ctx, proc_id(proc), n, n, seed, stream, first, float(lo), float(hi),
                                 make_cuts(cuts), mom.data_ptr(), w.data_ptr(), self._stream())
        return mom, w, t

    def tuning_cache(self, path):
        """Apply the matching entries of the JSON tuning cache at path and merge
        later autotune results into it; returns the number applied."""
        return nlo_tuning_cache(self.ctx, path)

    def set_fks_threshold(self, thr):
        nlo_set_fks_threshold(self.ctx, thr)

    def set_fks_mask_mode(self, compact):
        """False: branch-free masks (evaluate everything, zero failed terms);
        True: events failing the R cut skip the real |M|^2."""
        nlo_set_fks_mask_mode(self.ctx, 1 if compact else 0)

    def set_kernel_config(self, proc, prec, block, colour_mode=0, schedule=0):
        nlo_set_kernel_config(self.ctx, proc_id(proc), PREC[prec], block, colour_mode, schedule)

    SEED = 7439

    def uniforms(self, n, stream, slot, first=0, seed=SEED):
        """float64 CUDA [n, 2]: the generator's two uniforms per event."""
        import torch
        out = torch.empty((n, 2), dtype=torch.float64, device="cuda:%d" % self.device)
        nlo_uniforms(self.ctx, n, seed, stream, first, slot, out.data_ptr(), self._stream())
        return out

    def phase_space(self, proc, n, sqrt_s, stream, first=0, seed=SEED):
        """RAMBO points on the device: (mom [npart, 4, n], weight [n]) as float64
        CUDA tensors; sqrt_s is a number or a (lo, hi) range."""
        import torch
        lo, hi = (sqrt_s, sqrt_s) if not isinstance(sqrt_s, (tuple, list)) else sqrt_s
        npart = self.info(proc).npart
        mom = torch.empty((npart, 4, n), dtype=torch.float64, device="cuda:%d" % self.device)
        w = torch.empty(n, dtype=torch.float64, device=mom.device)
        nlo_phase_space(self.ctx, proc_id(proc), n, n, seed, stream, first, float(lo), float(hi), mom.data_ptr(),
                        w.data_ptr(), self._stream())
        return mom, w

    def fks_variables(self, n, stream, initial_state=False, first=0, seed=SEED):
        """(xi_tilde, y, phi), float64 CUDA [n] each."""
        import torch
        dev = "cuda:%d" % self.device
        xt, y, phi = (torch.empty(n, dtype=torch.float64, device=dev) for _ in range(3))
        nlo_fks_variables(self.ctx, n, seed, stream, first, 1 if initial_state else 0, xt.data_ptr(), y.data_ptr(),
                          phi.data_ptr(), self._stream())
        return xt, y, phi

    def integrate_subtracted(self, real, sqrt_s_born, n, niter, nadapt, stream, prec="fp64", seed=SEED):
        """Subtracted real-emission cross section at fixed Born energy, summed
        over the FKS sectors, by VEGAS on the device: (sigma, error, chi2/dof,
        per-iteration [(mean, error)]) in pb."""
        self.reserve(n)
        return nlo_integrate_subtracted(self.ctx, proc_id(real), float(sqrt_s_born), n, niter, nadapt, seed, stream,
                                        PREC[prec], self._stream())

    def cross_section(self, proc, n, sqrt_s, stream, prec="fp64", seed=SEED):
        """(sigma, error) in pb at fixed sqrt(s_hat), plain Monte Carlo on the device."""
        self.reserve(min(n, 1 << 20))
        return nlo_cross_section(self.ctx, proc_id(proc), n, seed, stream, float(sqrt_s), PREC[prec], self._stream())

