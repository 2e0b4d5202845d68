"""Event-parallel tree-level matrix elements on AMD MI355X.

The computation lives in libnlome.so (hand-written HIP for gfx950, C ABI in
include/nlome.h).  This package holds the ctypes binding, a torch-facing
convenience layer (torch supplies device memory and streams only), and the
build-time diagram generator."""
from . import _lib
from ._lib import (NLO_FP64, NLO_FP32, NLO_FP16, NLO_BF16, NLO_MIXED, PREC, NloError,  # noqa: F401
                   nlo_abi_version, nlo_create, nlo_destroy, nlo_last_error, nlo_num_processes,
                   nlo_process_info, nlo_set_kernel_config, nlo_get_kernel_config, nlo_me2)

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
        nlo_me2(self.ctx, proc_id(proc), n, ld, mom.data_ptr(), out.data_ptr(), PREC[prec], self._stream())
        return out

    def set_kernel_config(self, proc, prec, block, colour_mode=0):
        nlo_set_kernel_config(self.ctx, proc_id(proc), PREC[prec], block, colour_mode)
