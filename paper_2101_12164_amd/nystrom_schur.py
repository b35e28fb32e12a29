"""ctypes binding of libnystrom_schur.so (the C ABI in include/nystrom_schur.h).

Argument marshalling only: every numerical step runs in the library's HIP
kernels.  Functions carry the C names; device arrays are torch CUDA tensors
(their data_ptr() is passed), work is ordered on torch's current stream.
There is no CPU fallback: a missing library raises at load time.
"""

from __future__ import annotations

import ctypes
import os
from ctypes import POINTER, c_char_p, c_double, c_int32, c_int64, c_void_p

import torch

_LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libnystrom_schur.so")
_lib = None

NS_OK, NS_ERR_INVALID_ARG, NS_ERR_NOT_SPD, NS_ERR_OOM, NS_ERR_HIP, NS_ERR_NOT_CONVERGED, NS_ERR_BREAKDOWN = range(7)
NS_FP64, NS_FP32, NS_BF16 = 0, 1, 2
NS_APPLY_M2, NS_APPLY_ADEF2 = 0, 1
NS_SCHUR_AUTO, NS_SCHUR_TRIANGULAR, NS_SCHUR_LOCAL = 0, 1, 2
NS_VARIANT_M2, NS_VARIANT_M1, NS_VARIANT_M3 = 0, 1, 2
NS_OUTER_SCHUR, NS_OUTER_FULL = 0, 1
NS_LEVEL2_EXACT, NS_LEVEL2_NYSTROM = 0, 1
NS_INNER_SHIFTED, NS_INNER_FORM_A = 0, 1

STATUS_NAMES = {
    0: "NS_OK",
    1: "NS_ERR_INVALID_ARG",
    2: "NS_ERR_NOT_SPD",
    3: "NS_ERR_OOM",
    4: "NS_ERR_HIP",
    5: "NS_ERR_NOT_CONVERGED",
    6: "NS_ERR_BREAKDOWN",
}

EXPORTED = [
    "nystrom_schur_setup",
    "nystrom_schur_apply",
    "nystrom_schur_apply_noalloc",
    "nystrom_schur_pcg_solve",
    "nystrom_schur_setup_batched",
    "nystrom_schur_pcg_solve_batched",
    "nystrom_schur_schur_apply",
    "nystrom_schur_interface_solve",
    "nystrom_schur_interior_solve",
    "nystrom_schur_export_factor",
    "nystrom_schur_get_sizes",
    "nystrom_schur_get_lowrank",
    "nystrom_schur_get_basis",
    "nystrom_schur_features",
    "nystrom_schur_mlp_create",
    "nystrom_schur_mlp_get_params",
    "nystrom_schur_mlp_forward",
    "nystrom_schur_mlp_loss_grad",
    "nystrom_schur_mlp_adam_step",
    "nystrom_schur_mlp_destroy",
    "nystrom_schur_mlp_last_error",
    "nystrom_schur_kernel_timing",
    "nystrom_schur_kernel_timing_families",
    "nystrom_schur_kernel_stats",
    "nystrom_schur_get_tuning",
    "nystrom_schur_tuning_info",
    "nystrom_schur_tuning_override",
    "nystrom_schur_destroy",
    "nystrom_schur_last_error",
]

KERNEL_FAMILIES = ["chol_update", "chol_panel", "trsm_interior_f64", "trsm_interior_f32", "trsm_interface_f64",
                   "trsm_interface_f32", "schur_epi", "spmm", "local_schur_form", "local_schur_apply_f64",
                   "local_schur_apply_f32", "interface_inverse_f64", "interface_inverse_f32", "mlp_forward_bf16",
                   "mlp_backward_f32", "local_schur_apply_bf16", "interface_inverse_bf16", "gram", "block_update",
                   "small_dense", "gram_narrow", "block_update_narrow", "local_schur_apply_narrow_f64",
                   "interface_inverse_narrow_f64"]


class NsOptions(ctypes.Structure):
    _fields_ = [
        ("k", c_int32),
        ("p", c_int32),
        ("tol_inner", c_double),
        ("eig_thresh_rel", c_double),
        ("orth_drop_rel", c_double),
        ("max_inner_iters", c_int32),
        ("prec_inner", c_int32),
        ("apply_mode", c_int32),
        ("trsm_cols", c_int32),
        ("schur_mode", c_int32),
        ("omega", c_void_p),
        ("proposal", c_void_p),
        ("accept_tol", c_double),
        ("stream", c_void_p),
        ("pcg_graph_iters", c_int32),
        ("variant", c_int32),
        ("power_iters", c_int32),
        ("outer", c_int32),
        ("bcg_graph_iters", c_int32),
        ("level2", c_int32),
        ("level2_k", c_int32),
        ("level2_p", c_int32),
        ("level2_tol_inner", c_double),
        ("level2_omega", c_void_p),
        ("inner_form", c_int32),
    ]


class NsSetupInfo(ctypes.Structure):
    _fields_ = [
        ("n", c_int64),
        ("n_interior", c_int64),
        ("n_gamma", c_int64),
        ("n_junction", c_int64),
        ("n_sub", c_int32),
        ("n_level2_blocks", c_int32),
        ("k_eff", c_int32),
        ("it_inner", c_int32),
        ("inner_converged", c_int32),
        ("proposal_accepted", c_int32),
        ("bad_block", c_int32),
        ("bad_col", c_int32),
        ("inner_relres", c_double),
        ("t_extract", c_double),
        ("t_factor", c_double),
        ("t_inner", c_double),
        ("t_nystrom", c_double),
        ("t_total", c_double),
        ("inner_bf16_schur", c_int32),
        ("level2_it_inner", c_int32),
        ("level2_k_eff", c_int32),
    ]


class NsSolveInfo(ctypes.Structure):
    _fields_ = [
        ("it_pcg", c_int32),
        ("converged", c_int32),
        ("relres_schur", c_double),
        ("relres_true", c_double),
        ("t_solve", c_double),
        ("res_hist", POINTER(c_double)),
        ("res_hist_cap", c_int32),
    ]


class NsError(RuntimeError):
    def __init__(self, status, message, info=None):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {message}")
        self.status = status
        self.info = info


def library_path() -> str:
    return _LIB_PATH


def load_library() -> ctypes.CDLL:
    """Load the in-tree HIP library (build it with paper_2101_12164_amd.build)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        raise RuntimeError(f"HIP library not built: {_LIB_PATH} is missing (run paper_2101_12164_amd.build)")
    lib = ctypes.CDLL(_LIB_PATH)
    H = c_void_p
    lib.nystrom_schur_setup.argtypes = [c_int64, c_int64, c_void_p, c_void_p, c_void_p, c_void_p, POINTER(NsOptions),
                                        POINTER(H), POINTER(NsSetupInfo)]
    lib.nystrom_schur_setup.restype = c_int32
    lib.nystrom_schur_setup_batched.argtypes = [c_int32, POINTER(c_int64), POINTER(c_int64), POINTER(c_void_p),
                                                POINTER(c_void_p), POINTER(c_void_p), POINTER(c_void_p),
                                                POINTER(c_void_p), POINTER(NsOptions), POINTER(c_void_p),
                                                POINTER(NsSetupInfo)]
    lib.nystrom_schur_setup_batched.restype = c_int32
    lib.nystrom_schur_pcg_solve_batched.argtypes = [H, POINTER(c_void_p), POINTER(c_void_p), c_double, c_int32,
                                                    POINTER(NsSolveInfo)]
    lib.nystrom_schur_pcg_solve_batched.restype = c_int32
    lib.nystrom_schur_get_basis.argtypes = [H, c_void_p, POINTER(c_double)]
    lib.nystrom_schur_get_basis.restype = c_int32
    lib.nystrom_schur_features.argtypes = [c_int64, c_int64, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p,
                                           c_void_p, POINTER(c_int64), c_void_p]
    lib.nystrom_schur_features.restype = c_int32
    lib.nystrom_schur_mlp_create.argtypes = [c_int32, c_int32, c_int32, c_void_p, POINTER(c_void_p)]
    lib.nystrom_schur_mlp_create.restype = c_int32
    lib.nystrom_schur_mlp_get_params.argtypes = [c_void_p, c_void_p, c_void_p]
    lib.nystrom_schur_mlp_get_params.restype = c_int32
    lib.nystrom_schur_mlp_forward.argtypes = [c_void_p, c_void_p, c_int64, c_void_p, c_void_p]
    lib.nystrom_schur_mlp_forward.restype = c_int32
    lib.nystrom_schur_mlp_loss_grad.argtypes = [c_void_p, c_void_p, c_void_p, c_int64, POINTER(c_double), c_void_p]
    lib.nystrom_schur_mlp_loss_grad.restype = c_int32
    lib.nystrom_schur_mlp_adam_step.argtypes = [c_void_p, c_double, c_void_p]
    lib.nystrom_schur_mlp_adam_step.restype = c_int32
    lib.nystrom_schur_mlp_destroy.argtypes = [c_void_p]
    lib.nystrom_schur_mlp_destroy.restype = None
    lib.nystrom_schur_mlp_last_error.argtypes = [c_void_p]
    lib.nystrom_schur_mlp_last_error.restype = c_char_p
    lib.nystrom_schur_apply.argtypes = [H, c_void_p, c_void_p, c_int32]
    lib.nystrom_schur_apply.restype = c_int32
    lib.nystrom_schur_apply_noalloc.argtypes = [H, c_void_p, c_void_p, c_int32]
    lib.nystrom_schur_apply_noalloc.restype = c_int32
    lib.nystrom_schur_get_tuning.argtypes = [H, POINTER(c_int32)]
    lib.nystrom_schur_get_tuning.restype = c_int32
    lib.nystrom_schur_tuning_info.argtypes = [c_char_p, c_int32]
    lib.nystrom_schur_tuning_info.restype = c_int32
    lib.nystrom_schur_tuning_override.argtypes = [c_char_p, c_int32]
    lib.nystrom_schur_tuning_override.restype = c_int32
    lib.nystrom_schur_pcg_solve.argtypes = [H, c_void_p, c_void_p, c_double, c_int32, POINTER(NsSolveInfo)]
    lib.nystrom_schur_pcg_solve.restype = c_int32
    for name in ("nystrom_schur_schur_apply", "nystrom_schur_interface_solve", "nystrom_schur_interior_solve"):
        f = getattr(lib, name)
        f.argtypes = [H, c_void_p, c_void_p, c_int32, c_int32]
        f.restype = c_int32
    lib.nystrom_schur_export_factor.argtypes = [H, c_int32, c_void_p]
    lib.nystrom_schur_export_factor.restype = c_int32
    lib.nystrom_schur_get_sizes.argtypes = [H, POINTER(c_int64)]
    lib.nystrom_schur_get_sizes.restype = c_int32
    lib.nystrom_schur_get_lowrank.argtypes = [H, c_void_p, c_void_p]
    lib.nystrom_schur_get_lowrank.restype = c_int32
    lib.nystrom_schur_kernel_timing.argtypes = [c_int32]
    lib.nystrom_schur_kernel_timing.restype = None
    lib.nystrom_schur_kernel_timing_families.argtypes = [ctypes.c_uint32]
    lib.nystrom_schur_kernel_timing_families.restype = None
    lib.nystrom_schur_kernel_stats.argtypes = [c_char_p, POINTER(c_double), POINTER(c_int64), POINTER(c_double),
                                               POINTER(c_double)]
    lib.nystrom_schur_kernel_stats.restype = c_int32
    lib.nystrom_schur_destroy.argtypes = [H]
    lib.nystrom_schur_destroy.restype = None
    lib.nystrom_schur_last_error.argtypes = [H]
    lib.nystrom_schur_last_error.restype = c_char_p
    _lib = lib
    return lib


def _dev(t: torch.Tensor, dtype, name):
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a CUDA (HIP) tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} must have dtype {dtype}")
    if not t.is_contiguous():
        raise TypeError(f"{name} must be contiguous")
    return ctypes.c_void_p(t.data_ptr())


def _check(status, handle, info=None):
    if status != NS_OK:
        msg = load_library().nystrom_schur_last_error(handle).decode()
        raise NsError(status, msg, info)


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _setup_info_dict(si: NsSetupInfo) -> dict:
    return {f: getattr(si, f) for f, _ in NsSetupInfo._fields_}


def nystrom_schur_setup(row_ptr, col_idx, val, part, *, k, p, omega=None, tol_inner=0.1, eig_thresh_rel=1e-10,
                        orth_drop_rel=0.0, max_inner_iters=500, prec_inner=NS_FP64, apply_mode=NS_APPLY_M2,
                        trsm_cols=0, schur_mode=0, proposal=None, accept_tol=0.2, pcg_graph_iters=0,
                        variant=NS_VARIANT_M2, power_iters=0, outer=NS_OUTER_SCHUR, bcg_graph_iters=0,
                        level2=NS_LEVEL2_EXACT, level2_k=0, level2_p=0, level2_tol_inner=0.0, level2_omega=None,
                        inner_form=NS_INNER_SHIFTED):
    """Returns (handle, info dict).  row_ptr int64, col_idx int32, val float64, part int32, omega float64
    (n_gamma x (k+p), row-major; n_interior x (k+p) for NS_VARIANT_M3), level2_omega float64 (n_junction x
    (level2_k + level2_p), junction nodes in interface order), all CUDA tensors."""
    lib = load_library()
    n = row_ptr.numel() - 1
    nnz = val.numel()
    opt = _options(k, p, tol_inner, eig_thresh_rel, orth_drop_rel, max_inner_iters, prec_inner, apply_mode,
                   trsm_cols, schur_mode, accept_tol, pcg_graph_iters, variant, power_iters, outer, bcg_graph_iters)
    opt.omega = _dev(omega, torch.float64, "omega") if omega is not None else None
    opt.proposal = _dev(proposal, torch.float64, "proposal") if proposal is not None else None
    opt.level2 = int(level2)
    opt.level2_k, opt.level2_p = int(level2_k), int(level2_p)
    opt.level2_tol_inner = float(level2_tol_inner)
    opt.level2_omega = _dev(level2_omega, torch.float64, "level2_omega") if level2_omega is not None else None
    opt.inner_form = int(inner_form)
    h = c_void_p()
    info = NsSetupInfo()
    st = lib.nystrom_schur_setup(n, nnz, _dev(row_ptr, torch.int64, "row_ptr"), _dev(col_idx, torch.int32, "col_idx"),
                                 _dev(val, torch.float64, "val"), _dev(part, torch.int32, "part"), ctypes.byref(opt),
                                 ctypes.byref(h), ctypes.byref(info))
    _check(st, None, _setup_info_dict(info))
    return h, _setup_info_dict(info)


def _options(k, p, tol_inner, eig_thresh_rel, orth_drop_rel, max_inner_iters, prec_inner, apply_mode, trsm_cols,
             schur_mode, accept_tol, pcg_graph_iters=0, variant=NS_VARIANT_M2, power_iters=0, outer=NS_OUTER_SCHUR,
             bcg_graph_iters=0):
    opt = NsOptions()
    opt.k, opt.p = int(k), int(p)
    opt.tol_inner = tol_inner
    opt.eig_thresh_rel = eig_thresh_rel
    opt.orth_drop_rel = orth_drop_rel
    opt.max_inner_iters = max_inner_iters
    opt.prec_inner = prec_inner
    opt.apply_mode = apply_mode
    opt.trsm_cols = trsm_cols
    opt.schur_mode = schur_mode
    opt.accept_tol = accept_tol
    opt.stream = _stream()
    opt.pcg_graph_iters = pcg_graph_iters
    opt.variant = variant
    opt.power_iters = power_iters
    opt.outer = outer
    opt.bcg_graph_iters = bcg_graph_iters
    return opt


def nystrom_schur_setup_batched(problems, *, k, p, omegas=None, tol_inner=0.1, eig_thresh_rel=1e-10,
                                orth_drop_rel=0.0, max_inner_iters=500, prec_inner=NS_FP64, apply_mode=NS_APPLY_M2,
                                trsm_cols=0, schur_mode=0, pcg_graph_iters=0, variant=NS_VARIANT_M2,
                                power_iters=0, outer=NS_OUTER_SCHUR, bcg_graph_iters=0):
    """problems: list of (row_ptr, col_idx, val, part) CUDA tensors; omegas: list of n_gamma(q) x (k+p) float64
    CUDA tensors.  Returns (handle, list of info dicts)."""
    lib = load_library()
    m = len(problems)
    opt = _options(k, p, tol_inner, eig_thresh_rel, orth_drop_rel, max_inner_iters, prec_inner, apply_mode,
                   trsm_cols, schur_mode, 0.2, pcg_graph_iters, variant, power_iters, outer, bcg_graph_iters)
    n = (c_int64 * m)(*[pr[0].numel() - 1 for pr in problems])
    nnz = (c_int64 * m)(*[pr[2].numel() for pr in problems])
    ptrs = [(c_void_p * m)(*[_dev(pr[i], dt, nm) for pr in problems])
            for i, (dt, nm) in enumerate([(torch.int64, "row_ptr"), (torch.int32, "col_idx"),
                                          (torch.float64, "val"), (torch.int32, "part")])]
    om = (c_void_p * m)(*[_dev(o, torch.float64, "omega") for o in omegas]) if omegas is not None else None
    h = c_void_p()
    infos = (NsSetupInfo * m)()
    st = lib.nystrom_schur_setup_batched(m, n, nnz, ptrs[0], ptrs[1], ptrs[2], ptrs[3], om, ctypes.byref(opt),
                                         ctypes.byref(h), infos)
    out = [_setup_info_dict(infos[q]) for q in range(m)]
    _check(st, None, out)
    return h, out


def nystrom_schur_pcg_solve_batched(handle, bs, xs=None, rtol=1e-8, maxit=1000, hist_cap=0,
                                    raise_on_not_converged=True):
    """bs: list of float64 CUDA tensors (each problem's right-hand side, its own node order)."""
    lib = load_library()
    m = len(bs)
    if xs is None:
        xs = [torch.empty_like(b) for b in bs]
    infos = (NsSolveInfo * m)()
    hists = [(c_double * max(hist_cap, 1))() for _ in range(m)]
    for q in range(m):
        infos[q].res_hist = ctypes.cast(hists[q], POINTER(c_double))
        infos[q].res_hist_cap = hist_cap
    bp = (c_void_p * m)(*[_dev(b, torch.float64, "b") for b in bs])
    xp = (c_void_p * m)(*[_dev(x, torch.float64, "x") for x in xs])
    st = lib.nystrom_schur_pcg_solve_batched(handle, bp, xp, rtol, maxit, infos)
    out = []
    for q in range(m):
        i = infos[q]
        d = dict(it_pcg=i.it_pcg, converged=i.converged, relres_schur=i.relres_schur, relres_true=i.relres_true,
                 t_solve=i.t_solve, status=st)
        if hist_cap:
            d["res_hist"] = [hists[q][j] for j in range(min(hist_cap, i.it_pcg + 1))]
        out.append(d)
    if st == NS_ERR_NOT_CONVERGED and not raise_on_not_converged:
        return xs, out
    _check(st, handle, out)
    return xs, out


def nystrom_schur_apply_noalloc(handle, r: torch.Tensor, z: torch.Tensor):
    """z = M r through the allocation-free entry point (z must be given: nothing is allocated)."""
    lib = load_library()
    ncols = 1 if r.dim() == 1 else r.shape[1]
    st = lib.nystrom_schur_apply_noalloc(handle, _dev(r, torch.float64, "r"), _dev(z, torch.float64, "z"), ncols)
    _check(st, handle)
    return z


def nystrom_schur_apply(handle, r: torch.Tensor, z: torch.Tensor = None):
    lib = load_library()
    ncols = 1 if r.dim() == 1 else r.shape[1]
    if z is None:
        z = torch.empty_like(r)
    _check(lib.nystrom_schur_apply(handle, _dev(r, torch.float64, "r"), _dev(z, torch.float64, "z"), ncols), handle)
    return z


def nystrom_schur_pcg_solve(handle, b: torch.Tensor, x: torch.Tensor = None, rtol=1e-8, maxit=1000,
                            hist_cap=0, raise_on_not_converged=True):
    lib = load_library()
    if x is None:
        x = torch.empty_like(b)
    info = NsSolveInfo()
    hist = (c_double * max(hist_cap, 1))()
    info.res_hist = ctypes.cast(hist, POINTER(c_double))
    info.res_hist_cap = hist_cap
    st = lib.nystrom_schur_pcg_solve(handle, _dev(b, torch.float64, "b"), _dev(x, torch.float64, "x"), rtol, maxit,
                                     ctypes.byref(info))
    out = dict(it_pcg=info.it_pcg, converged=info.converged, relres_schur=info.relres_schur,
               relres_true=info.relres_true, t_solve=info.t_solve, status=st)
    if hist_cap:
        out["res_hist"] = [hist[i] for i in range(min(hist_cap, info.it_pcg + 1))]
    if st == NS_ERR_NOT_CONVERGED and not raise_on_not_converged:
        return x, out
    _check(st, handle, out)
    return x, out


def _op(name, handle, X, prec, out_rows=None):
    lib = load_library()
    ncols = 1 if X.dim() == 1 else X.shape[1]
    Y = torch.empty_like(X)
    _check(getattr(lib, name)(handle, _dev(X, torch.float64, "X"), _dev(Y, torch.float64, "Y"), ncols, prec), handle)
    return Y


def nystrom_schur_schur_apply(handle, X, prec=NS_FP64):
    return _op("nystrom_schur_schur_apply", handle, X, prec)


def nystrom_schur_interface_solve(handle, X, prec=NS_FP64):
    return _op("nystrom_schur_interface_solve", handle, X, prec)


def nystrom_schur_interior_solve(handle, X, prec=NS_FP64):
    return _op("nystrom_schur_interior_solve", handle, X, prec)


def nystrom_schur_get_sizes(handle) -> dict:
    lib = load_library()
    out = (c_int64 * 8)()
    _check(lib.nystrom_schur_get_sizes(handle, out), handle)
    keys = ["n", "n_interior", "n_gamma", "n_sub", "n_junction", "n_level2_blocks", "k_eff", "nprob"]
    return dict(zip(keys, list(out)))


def nystrom_schur_export_factor(handle, block: int, nb: int, device="cuda"):
    lib = load_library()
    L = torch.empty((nb, nb), dtype=torch.float64, device=device)
    _check(lib.nystrom_schur_export_factor(handle, block, _dev(L, torch.float64, "L")), handle)
    return L.t()  # stored column-major


def nystrom_schur_get_tuning(handle):
    """The automatic settings that apply to a handle's sizes (see the header)."""
    lib = load_library()
    out = (c_int32 * 4)()
    _check(lib.nystrom_schur_get_tuning(handle, out), handle)
    return {"trsm_cols": out[0], "pcg_graph_iters": out[1], "bcg_graph_iters": out[2], "ls_gemm_cols": out[3]}


def nystrom_schur_tuning_info():
    """(number of table entries loaded for the current device, the table's path)."""
    lib = load_library()
    buf = ctypes.create_string_buffer(4096)
    n = lib.nystrom_schur_tuning_info(buf, 4096)
    return n, buf.value.decode()


def nystrom_schur_tuning_override(kernel, value):
    """Process-wide value of an automatic setting (0 removes it), over the table."""
    return load_library().nystrom_schur_tuning_override(kernel.encode(), int(value))


def nystrom_schur_get_lowrank(handle, device="cuda"):
    lib = load_library()
    sz = nystrom_schur_get_sizes(handle)
    ke, ng = sz["k_eff"], sz["n_gamma"]
    Z = torch.empty((ng, max(ke, 1)), dtype=torch.float64, device=device)
    S = torch.empty(max(ke, 1), dtype=torch.float64, device=device)
    _check(lib.nystrom_schur_get_lowrank(handle, _dev(Z, torch.float64, "Z"), _dev(S, torch.float64, "Sigma")),
           handle)
    return Z[:, :ke], S[:ke]


def nystrom_schur_get_basis(handle, device="cuda"):
    """(U, rho): the Nystrom basis (n_gamma x k_eff, or None when an accepted proposal replaced it) and the
    eigen-residual of the judged proposal (0 when none was given)."""
    lib = load_library()
    sz = nystrom_schur_get_sizes(handle)
    ke, ng = sz["k_eff"], sz["n_gamma"]
    rho = c_double()
    U = torch.empty((ng, max(ke, 1)), dtype=torch.float64, device=device)
    st = lib.nystrom_schur_get_basis(handle, _dev(U, torch.float64, "U"), ctypes.byref(rho))
    if st == NS_ERR_INVALID_ARG:
        _check(lib.nystrom_schur_get_basis(handle, None, ctypes.byref(rho)), handle)
        return None, rho.value
    _check(st, handle)
    return U[:, :ke], rho.value


def nystrom_schur_features(row_ptr, col_idx, val, part, coords=None):
    """Interface-node features (n_gamma x 16 float32 CUDA tensor)."""
    lib = load_library()
    n = row_ptr.numel() - 1
    X = torch.empty((n, 16), dtype=torch.float32, device=row_ptr.device)
    ng = c_int64()
    cp = _dev(coords, torch.float64, "coords") if coords is not None else None
    st = lib.nystrom_schur_features(n, val.numel(), _dev(row_ptr, torch.int64, "row_ptr"),
                                    _dev(col_idx, torch.int32, "col_idx"), _dev(val, torch.float64, "val"),
                                    _dev(part, torch.int32, "part"), cp, _dev(X, torch.float32, "X"),
                                    ctypes.byref(ng), _stream())
    _check(st, None)
    return X[:ng.value]


def _mlp_check(status, m):
    if status != NS_OK:
        raise NsError(status, load_library().nystrom_schur_mlp_last_error(m).decode())


def nystrom_schur_mlp_create(d_in, hidden, d_out, params):
    """params: flat float32 array (W1, b1, W2, b2, W3, b3; weights row-major in x out)."""
    import numpy as np

    lib = load_library()
    p = np.ascontiguousarray(params, dtype=np.float32)
    m = c_void_p()
    st = lib.nystrom_schur_mlp_create(d_in, hidden, d_out, p.ctypes.data_as(c_void_p), ctypes.byref(m))
    _mlp_check(st, None)
    return m


def nystrom_schur_mlp_get_params(m, n_params):
    import numpy as np

    p = np.empty(n_params, dtype=np.float32)
    g = np.empty(n_params, dtype=np.float32)
    _mlp_check(load_library().nystrom_schur_mlp_get_params(m, p.ctypes.data_as(c_void_p),
                                                           g.ctypes.data_as(c_void_p)), m)
    return p, g


def nystrom_schur_mlp_forward(m, X, d_out):
    Z0 = torch.empty((X.shape[0], d_out), dtype=torch.float64, device=X.device)
    _mlp_check(load_library().nystrom_schur_mlp_forward(m, _dev(X, torch.float32, "X"), X.shape[0],
                                                        _dev(Z0, torch.float64, "Z0"), _stream()), m)
    return Z0


def nystrom_schur_mlp_loss_grad(m, X, U):
    loss = c_double()
    _mlp_check(load_library().nystrom_schur_mlp_loss_grad(m, _dev(X, torch.float32, "X"), _dev(U, torch.float64, "U"),
                                                          X.shape[0], ctypes.byref(loss), _stream()), m)
    return loss.value


def nystrom_schur_mlp_adam_step(m, lr):
    _mlp_check(load_library().nystrom_schur_mlp_adam_step(m, lr, _stream()), m)


def nystrom_schur_mlp_destroy(m):
    load_library().nystrom_schur_mlp_destroy(m)


def nystrom_schur_mlp_last_error(m=None) -> str:
    return load_library().nystrom_schur_mlp_last_error(m).decode()


def nystrom_schur_kernel_timing(enable: bool):
    """Turn per-kernel HIP-event timing on/off (and reset the totals)."""
    load_library().nystrom_schur_kernel_timing(1 if enable else 0)


def nystrom_schur_kernel_timing_families(families):
    """Time only the named kernel families (and reset the totals); an empty list turns timing off."""
    mask = 0
    for f in families:
        mask |= 1 << KERNEL_FAMILIES.index(f)
    load_library().nystrom_schur_kernel_timing_families(mask)


def nystrom_schur_kernel_stats(family: str):
    """dict(ms, launches, bytes, flops) of one kernel family since timing was enabled."""
    ms, cnt, by, fl = c_double(), c_int64(), c_double(), c_double()
    st = load_library().nystrom_schur_kernel_stats(family.encode(), ctypes.byref(ms), ctypes.byref(cnt),
                                                   ctypes.byref(by), ctypes.byref(fl))
    if st != NS_OK:
        raise NsError(st, f"unknown kernel family {family}")
    return dict(ms=ms.value, launches=cnt.value, bytes=by.value, flops=fl.value)


def nystrom_schur_destroy(handle):
    load_library().nystrom_schur_destroy(handle)


def nystrom_schur_last_error(handle=None) -> str:
    return load_library().nystrom_schur_last_error(handle).decode()


class NystromSchur:
    """Owning wrapper: builds the preconditioner on construction, frees it on close()."""

    def __init__(self, row_ptr, col_idx, val, part, **kw):
        self.handle, self.setup_info = nystrom_schur_setup(row_ptr, col_idx, val, part, **kw)

    def apply(self, r):
        return nystrom_schur_apply(self.handle, r)

    def solve(self, b, rtol=1e-8, maxit=1000, hist_cap=0, raise_on_not_converged=True):
        return nystrom_schur_pcg_solve(self.handle, b, rtol=rtol, maxit=maxit, hist_cap=hist_cap,
                                       raise_on_not_converged=raise_on_not_converged)

    def sizes(self):
        return nystrom_schur_get_sizes(self.handle)

    def close(self):
        if self.handle is not None and self.handle.value:
            nystrom_schur_destroy(self.handle)
        self.handle = None

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
