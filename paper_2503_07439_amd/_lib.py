"""ctypes binding of libnlome.so (include/nlome.h): same names, argument
marshalling only.  Every step of the computation runs in the HIP kernels;
there is no CPU fallback -- a missing library raises."""
import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libnlome.so")

NLO_OK, NLO_EINVAL, NLO_EPROC, NLO_EDEVICE, NLO_ENOMEM, NLO_EUNSUPPORTED = range(6)
NLO_FP64, NLO_FP32, NLO_FP16, NLO_BF16, NLO_MIXED = range(5)
PREC = {"fp64": NLO_FP64, "fp32": NLO_FP32, "fp16": NLO_FP16, "bf16": NLO_BF16, "mixed": NLO_MIXED}


class nlo_params(ctypes.Structure):
    _fields_ = [("alpha", ctypes.c_double), ("alpha_s", ctypes.c_double), ("m_top", ctypes.c_double),
                ("device", ctypes.c_int)]


class nlo_proc_info(ctypes.Structure):
    _fields_ = [("name", ctypes.c_char_p), ("npart", ctypes.c_int), ("ninitial", ctypes.c_int),
                ("ncolour", ctypes.c_int), ("nhel", ctypes.c_int), ("ngood_hel", ctypes.c_int),
                ("ndiagrams", ctypes.c_int), ("nterms", ctypes.c_int), ("ncurrents", ctypes.c_int),
                ("avg_factor", ctypes.c_double), ("ident_factor", ctypes.c_double),
                ("gs_pow", ctypes.c_int), ("e_pow", ctypes.c_int), ("nschedules", ctypes.c_int)]


class nlo_cuts(ctypes.Structure):
    _fields_ = [("jet_r", ctypes.c_double), ("jet_ptmin", ctypes.c_double), ("jet_ymax", ctypes.c_double),
                ("njet_min", ctypes.c_int), ("top_ptmin", ctypes.c_double), ("top_ymax", ctypes.c_double),
                ("lep_ptmin", ctypes.c_double), ("lep_ymax", ctypes.c_double)]


def make_cuts(d):
    """nlo_cuts from a dict with the field names (missing cuts are off)"""
    c = nlo_cuts(0.4, 0.0, 1e300, 0, 0.0, 1e300, 0.0, 1e300)
    for k, v in d.items():
        setattr(c, k, v)
    return c


class nlo_fks_config(ctypes.Structure):
    _fields_ = [("real_block", ctypes.c_int), ("colour_mode", ctypes.c_int), ("ct_block", ctypes.c_int)]


class nlo_kernel_config(ctypes.Structure):
    _fields_ = [("block", ctypes.c_int), ("colour_mode", ctypes.c_int), ("schedule", ctypes.c_int)]


class nlo_fks_out(ctypes.Structure):
    _fields_ = [("W", ctypes.c_void_p), ("xi", ctypes.c_void_p), ("born", ctypes.c_void_p),
                ("g_R", ctypes.c_void_p), ("g_S", ctypes.c_void_p), ("g_C", ctypes.c_void_p),
                ("g_Cm", ctypes.c_void_p), ("g_SC", ctypes.c_void_p), ("g_SCm", ctypes.c_void_p),
                ("status", ctypes.c_void_p), ("real_mom", ctypes.c_void_p), ("w_sum", ctypes.c_void_p),
                ("dsig", ctypes.c_void_p), ("jac", ctypes.c_void_p)]


class nlo_work_item(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int), ("proc_id", ctypes.c_int), ("fks_i", ctypes.c_int), ("fks_j", ctypes.c_int),
                ("n", ctypes.c_int64), ("ld", ctypes.c_int64), ("mom", ctypes.c_void_p),
                ("xi_tilde", ctypes.c_void_p), ("y", ctypes.c_void_p), ("phi", ctypes.c_void_p),
                ("mask", ctypes.c_void_p), ("prec", ctypes.c_int), ("me2", ctypes.c_void_p),
                ("fks_out", nlo_fks_out)]


NLO_ITEM_ME2, NLO_ITEM_SUBTRACTED = 0, 1


class NloError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__("nlome status %d: %s" % (status, msg))
        self.status = status


_lib = None

# exported symbols and their signatures (argtypes, restype)
_VP = ctypes.c_void_p
_I64 = ctypes.c_int64
SIGNATURES = {
    "nlo_abi_version": ([], ctypes.c_uint32),
    "nlo_create": ([ctypes.POINTER(_VP), ctypes.POINTER(nlo_params)], ctypes.c_int),
    "nlo_destroy": ([_VP], ctypes.c_int),
    "nlo_last_error": ([], ctypes.c_char_p),
    "nlo_num_processes": ([], ctypes.c_int),
    "nlo_process_info": ([_VP, ctypes.c_int, ctypes.POINTER(nlo_proc_info)], ctypes.c_int),
    "nlo_set_kernel_config": ([_VP, ctypes.c_int, ctypes.c_int, ctypes.POINTER(nlo_kernel_config)], ctypes.c_int),
    "nlo_get_kernel_config": ([_VP, ctypes.c_int, ctypes.c_int, ctypes.POINTER(nlo_kernel_config)], ctypes.c_int),
    "nlo_set_fks_config": ([_VP, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                            ctypes.POINTER(nlo_fks_config)], ctypes.c_int),
    "nlo_get_fks_config": ([_VP, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                            ctypes.POINTER(nlo_fks_config)], ctypes.c_int),
    "nlo_autotune_subtracted": ([_VP, ctypes.c_int, ctypes.c_int, ctypes.c_int, _I64, _I64, _VP, _VP, _VP, _VP,
                                 ctypes.c_int, _VP, _VP, ctypes.POINTER(nlo_fks_config),
                                 ctypes.POINTER(ctypes.c_double)], ctypes.c_int),
    "nlo_tuning_cache": ([_VP, ctypes.c_char_p, ctypes.POINTER(ctypes.c_int)], ctypes.c_int),
    "nlo_fks_buffer_create": ([_VP, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int, _I64, _VP,
                               ctypes.POINTER(_VP)], ctypes.c_int),
    "nlo_fks_buffer_push": ([_VP, _I64, _I64, _VP, _VP, _VP, _VP, _VP, _VP, _VP], ctypes.c_int),
    "nlo_fks_buffer_flush": ([_VP, _VP], ctypes.c_int),
    "nlo_fks_buffer_destroy": ([_VP], ctypes.c_int),
    "nlo_virtual_integrated": ([_VP, ctypes.c_int, _I64, _I64, _VP, ctypes.c_int, _VP, _VP, _VP], ctypes.c_int),
    "nlo_cut_mask": ([_VP, ctypes.c_int, _I64, _I64, _VP, ctypes.POINTER(nlo_cuts), _VP, _VP], ctypes.c_int),
    "nlo_fks_cut_masks": ([_VP, ctypes.c_int, ctypes.c_int, ctypes.c_int, _I64, _I64, _VP, _VP, _VP, _VP,
                           ctypes.POINTER(nlo_cuts), _VP, _VP], ctypes.c_int),
    "nlo_generate_passing": ([_VP, ctypes.c_int, _I64, _I64, ctypes.c_uint32, ctypes.c_uint32, ctypes.c_uint64,
                              ctypes.c_double, ctypes.c_double, ctypes.POINTER(nlo_cuts), _VP, _VP,
                              ctypes.POINTER(ctypes.c_uint64), _VP], ctypes.c_int),
    "nlo_me2": ([_VP, ctypes.c_int, _I64, _I64, _VP, _VP, ctypes.c_int, _VP], ctypes.c_int),
    "nlo_me2_checked": ([_VP, ctypes.c_int, _I64, _I64, _VP, _VP, _VP, ctypes.c_int, _VP], ctypes.c_int),
    "nlo_reserve": ([_VP, _I64], ctypes.c_int),
    "nlo_integrate_subtracted": ([_VP, ctypes.c_int, ctypes.c_double, _I64, ctypes.c_int, ctypes.c_int,
                                  ctypes.c_uint32, ctypes.c_uint32, ctypes.c_int, ctypes.POINTER(ctypes.c_double),
                                  ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double),
                                  ctypes.POINTER(ctypes.c_double), _VP], ctypes.c_int),
    "nlo_colour_unit": ([_VP, ctypes.c_int, ctypes.c_int, ctypes.POINTER(ctypes.c_int)], ctypes.c_int),
    "nlo_subtracted": ([_VP, ctypes.c_int, ctypes.c_int, ctypes.c_int, _I64, _I64, _VP, _VP, _VP, _VP, _VP,
                        ctypes.c_int, ctypes.POINTER(nlo_fks_out), _VP], ctypes.c_int),
    "nlo_subtracted_static": ([_VP, ctypes.c_int, ctypes.c_int, ctypes.c_int, _I64, _I64, _VP, _VP, _VP, _VP, _VP,
                               ctypes.c_int, ctypes.POINTER(nlo_fks_out), _VP], ctypes.c_int),
    "nlo_set_fks_threshold": ([_VP, ctypes.c_double], ctypes.c_int),
    "nlo_set_fks_mask_mode": ([_VP, ctypes.c_int], ctypes.c_int),
    "nlo_batch_plan": ([_VP, ctypes.POINTER(nlo_work_item), ctypes.c_int, ctypes.c_int, ctypes.POINTER(_VP)],
                       ctypes.c_int),
    "nlo_batch_run": ([_VP, _VP], ctypes.c_int),
    "nlo_autotune": ([_VP, ctypes.c_int, ctypes.c_int, _I64, _I64, _VP, _VP, _VP, ctypes.POINTER(nlo_kernel_config),
                      ctypes.POINTER(ctypes.c_double)], ctypes.c_int),
    "nlo_plan_destroy": ([_VP], ctypes.c_int),
    "nlo_uniforms": ([_VP, _I64, ctypes.c_uint32, ctypes.c_uint32, ctypes.c_uint64, ctypes.c_uint32, _VP, _VP],
                     ctypes.c_int),
    "nlo_phase_space": ([_VP, ctypes.c_int, _I64, _I64, ctypes.c_uint32, ctypes.c_uint32, ctypes.c_uint64,
                         ctypes.c_double, ctypes.c_double, _VP, _VP, _VP], ctypes.c_int),
    "nlo_fks_variables": ([_VP, _I64, ctypes.c_uint32, ctypes.c_uint32, ctypes.c_uint64, ctypes.c_int, _VP, _VP, _VP,
                           _VP], ctypes.c_int),
    "nlo_cross_section": ([_VP, ctypes.c_int, _I64, ctypes.c_uint32, ctypes.c_uint32, ctypes.c_double, ctypes.c_int,
                           ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double), _VP], ctypes.c_int),
}


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError("libnlome.so is not built (run paper_2503_07439_amd.build or __graft_entry__.build())")
        L = ctypes.CDLL(LIB_PATH)
        for name, (args, res) in SIGNATURES.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = res
        _lib = L
    return _lib


def check(status):
    if status != NLO_OK:
        raise NloError(status, lib().nlo_last_error().decode())
    return status


# thin same-name wrappers ----------------------------------------------------
def nlo_abi_version():
    return lib().nlo_abi_version()


def nlo_create(alpha=1.0 / 132.507, alpha_s=0.118, m_top=173.0, device=0):
    ctx = _VP()
    p = nlo_params(alpha, alpha_s, m_top, device)
    check(lib().nlo_create(ctypes.byref(ctx), ctypes.byref(p)))
    return ctx


def nlo_destroy(ctx):
    return check(lib().nlo_destroy(ctx))


def nlo_last_error():
    return lib().nlo_last_error().decode()


def nlo_num_processes():
    return lib().nlo_num_processes()


def nlo_process_info(ctx, proc_id):
    info = nlo_proc_info()
    check(lib().nlo_process_info(ctx, proc_id, ctypes.byref(info)))
    return info


def nlo_set_kernel_config(ctx, proc_id, prec, block, colour_mode=0, schedule=0):
    cfg = nlo_kernel_config(block, colour_mode, schedule)
    return check(lib().nlo_set_kernel_config(ctx, proc_id, prec, ctypes.byref(cfg)))


def nlo_get_kernel_config(ctx, proc_id, prec):
    cfg = nlo_kernel_config()
    check(lib().nlo_get_kernel_config(ctx, proc_id, prec, ctypes.byref(cfg)))
    return cfg.block, cfg.colour_mode, cfg.schedule


def nlo_me2(ctx, proc_id, n, ld, mom_ptr, me2_ptr, prec, stream_ptr):
    return check(lib().nlo_me2(ctx, proc_id, n, ld, mom_ptr, me2_ptr, prec, stream_ptr))


def nlo_me2_checked(ctx, proc_id, n, ld, mom_ptr, me2_ptr, status_ptr, prec, stream_ptr):
    return check(lib().nlo_me2_checked(ctx, proc_id, n, ld, mom_ptr, me2_ptr, status_ptr, prec, stream_ptr))


def nlo_reserve(ctx, n):
    return check(lib().nlo_reserve(ctx, n))


def nlo_integrate_subtracted(ctx, real_proc, sqrt_s_born, n, niter, nadapt, seed, stream, prec, stream_ptr):
    """(sigma_pb, error_pb, chi2_dof, per-iteration [(mean, error)])"""
    sig, err, chi = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
    it = (ctypes.c_double * (2 * niter))()
    check(lib().nlo_integrate_subtracted(ctx, real_proc, sqrt_s_born, n, niter, nadapt, seed, stream, prec,
                                         ctypes.byref(sig), ctypes.byref(err), ctypes.byref(chi), it, stream_ptr))
    return sig.value, err.value, chi.value, [(it[2 * k], it[2 * k + 1]) for k in range(niter)]


def nlo_colour_unit(ctx, proc_id, prec):
    u = ctypes.c_int()
    check(lib().nlo_colour_unit(ctx, proc_id, prec, ctypes.byref(u)))
    return u.value


def nlo_subtracted(ctx, real_proc, fks_i, fks_j, n, ld, born_ptr, xit_ptr, y_ptr, phi_ptr, mask_ptr, prec, out,
                   stream_ptr):
    return check(lib().nlo_subtracted(ctx, real_proc, fks_i, fks_j, n, ld, born_ptr, xit_ptr, y_ptr, phi_ptr,
                                      mask_ptr, prec, ctypes.byref(out), stream_ptr))


def nlo_subtracted_static(ctx, real_proc, fks_i, fks_j, n, ld, born_ptr, xit_ptr, y_ptr, phi_ptr, mask_ptr, prec,
                          out, stream_ptr):
    return check(lib().nlo_subtracted_static(ctx, real_proc, fks_i, fks_j, n, ld, born_ptr, xit_ptr, y_ptr, phi_ptr,
                                             mask_ptr, prec, ctypes.byref(out), stream_ptr))


def nlo_set_fks_threshold(ctx, threshold):
    return check(lib().nlo_set_fks_threshold(ctx, threshold))


def nlo_batch_plan(ctx, items, nbranches=0):
    arr = (nlo_work_item * len(items))(*items)
    plan = _VP()
    check(lib().nlo_batch_plan(ctx, arr, len(items), nbranches, ctypes.byref(plan)))
    return plan


def nlo_batch_run(plan, stream_ptr):
    return check(lib().nlo_batch_run(plan, stream_ptr))


def nlo_plan_destroy(plan):
    return check(lib().nlo_plan_destroy(plan))


def nlo_autotune(ctx, proc_id, prec, n, ld, mom_ptr, me2_ptr, stream_ptr):
    best = nlo_kernel_config()
    ns = ctypes.c_double()
    check(lib().nlo_autotune(ctx, proc_id, prec, n, ld, mom_ptr, me2_ptr, stream_ptr, ctypes.byref(best),
                             ctypes.byref(ns)))
    return (best.block, best.colour_mode, best.schedule), ns.value


def nlo_set_fks_config(ctx, real_proc, fks_i, fks_j, prec, real_block, colour_mode, ct_block):
    return check(lib().nlo_set_fks_config(ctx, real_proc, fks_i, fks_j, prec,
                                          ctypes.byref(nlo_fks_config(real_block, colour_mode, ct_block))))


def nlo_get_fks_config(ctx, real_proc, fks_i, fks_j, prec):
    cfg = nlo_fks_config()
    check(lib().nlo_get_fks_config(ctx, real_proc, fks_i, fks_j, prec, ctypes.byref(cfg)))
    return cfg.real_block, cfg.colour_mode, cfg.ct_block


def nlo_autotune_subtracted(ctx, real_proc, fks_i, fks_j, n, ld, born_ptr, xit_ptr, y_ptr, phi_ptr, prec, w_ptr,
                            stream_ptr):
    """((real_block, colour_mode, ct_block), ns per event)"""
    best = nlo_fks_config()
    ns = ctypes.c_double()
    check(lib().nlo_autotune_subtracted(ctx, real_proc, fks_i, fks_j, n, ld, born_ptr, xit_ptr, y_ptr, phi_ptr, prec,
                                        w_ptr, stream_ptr, ctypes.byref(best), ctypes.byref(ns)))
    return (best.real_block, best.colour_mode, best.ct_block), ns.value


def nlo_tuning_cache(ctx, path):
    """Number of entries applied from the cache file at path (None: stop merging)."""
    n = ctypes.c_int()
    check(lib().nlo_tuning_cache(ctx, path.encode() if path else None, ctypes.byref(n)))
    return n.value


def nlo_fks_buffer_create(ctx, real_proc, fks_i, fks_j, prec, threshold, w_ptr):
    b = _VP()
    check(lib().nlo_fks_buffer_create(ctx, real_proc, fks_i, fks_j, prec, threshold, w_ptr, ctypes.byref(b)))
    return b


def nlo_fks_buffer_push(buf, n, ld, born_ptr, xit_ptr, y_ptr, phi_ptr, mask_ptr, slot_ptr, stream_ptr):
    return check(lib().nlo_fks_buffer_push(buf, n, ld, born_ptr, xit_ptr, y_ptr, phi_ptr, mask_ptr, slot_ptr,
                                           stream_ptr))


def nlo_fks_buffer_flush(buf, stream_ptr):
    return check(lib().nlo_fks_buffer_flush(buf, stream_ptr))


def nlo_fks_buffer_destroy(buf):
    return check(lib().nlo_fks_buffer_destroy(buf))


def nlo_virtual_integrated(ctx, born_proc, n, ld, mom_ptr, prec, born_ptr, vi_ptr, stream_ptr):
    return check(lib().nlo_virtual_integrated(ctx, born_proc, n, ld, mom_ptr, prec, born_ptr, vi_ptr, stream_ptr))


def nlo_cut_mask(ctx, proc_id, n, ld, mom_ptr, cuts, pass_ptr, stream_ptr):
    return check(lib().nlo_cut_mask(ctx, proc_id, n, ld, mom_ptr, ctypes.byref(cuts), pass_ptr, stream_ptr))


def nlo_fks_cut_masks(ctx, real_proc, fks_i, fks_j, n, ld, born_ptr, xit_ptr, y_ptr, phi_ptr, cuts, mask_ptr,
                      stream_ptr):
    return check(lib().nlo_fks_cut_masks(ctx, real_proc, fks_i, fks_j, n, ld, born_ptr, xit_ptr, y_ptr, phi_ptr,
                                         ctypes.byref(cuts), mask_ptr, stream_ptr))


def nlo_generate_passing(ctx, proc_id, n, ld, seed, stream, first, rs_lo, rs_hi, cuts, mom_ptr, w_ptr, stream_ptr):
    """number of candidates used"""
    t = ctypes.c_uint64()
    check(lib().nlo_generate_passing(ctx, proc_id, n, ld, seed, stream, first, rs_lo, rs_hi, ctypes.byref(cuts),
                                     mom_ptr, w_ptr, ctypes.byref(t), stream_ptr))
    return t.value


def nlo_uniforms(ctx, n, seed, stream, first, slot, out_ptr, stream_ptr):
    return check(lib().nlo_uniforms(ctx, n, seed, stream, first, slot, out_ptr, stream_ptr))


def nlo_phase_space(ctx, proc_id, n, ld, seed, stream, first, sqrt_s_lo, sqrt_s_hi, mom_ptr, weight_ptr, stream_ptr):
    return check(lib().nlo_phase_space(ctx, proc_id, n, ld, seed, stream, first, sqrt_s_lo, sqrt_s_hi, mom_ptr,
                                       weight_ptr, stream_ptr))


def nlo_fks_variables(ctx, n, seed, stream, first, initial_state, xit_ptr, y_ptr, phi_ptr, stream_ptr):
    return check(lib().nlo_fks_variables(ctx, n, seed, stream, first, initial_state, xit_ptr, y_ptr, phi_ptr,
                                         stream_ptr))


def nlo_cross_section(ctx, proc_id, n, seed, stream, sqrt_s, prec, stream_ptr):
    sig, err = ctypes.c_double(), ctypes.c_double()
    check(lib().nlo_cross_section(ctx, proc_id, n, seed, stream, sqrt_s, prec, ctypes.byref(sig), ctypes.byref(err),
                                  stream_ptr))
    return sig.value, err.value


def nlo_set_fks_mask_mode(ctx, mode):
    return check(lib().nlo_set_fks_mask_mode(ctx, mode))
