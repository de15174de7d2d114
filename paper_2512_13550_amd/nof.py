"""ctypes binding of libnof.so (the C ABI declared in include/nof.h).

Argument marshalling only: every step of the path runs in the library's HIP
kernels.  Tensors must be contiguous and live on the GPU; workspaces are
allocated here as caller-owned device buffers and passed in.  The import fails
loudly if the library has not been built; there is no fallback.
"""
from __future__ import annotations

import ctypes
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libnof.so")
if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_2512_13550_amd.build`")
lib = ctypes.CDLL(LIB_PATH)

# status codes and enums (mirror include/nof.h)
OK, E_NULL, E_DIM, E_DTYPE, E_PREC, E_WORKSPACE, E_HIP, E_NOT_CONVERGED, E_ARG = 0, -1, -2, -3, -4, -5, -6, -7, -8
F64, F32, BF16, BF16X4, I8X4 = 0, 1, 2, 3, 4
P_F64, P_F32, P_BF16X1, P_BF16X3, P_BF16X6, P_BF16X10, P_I8X10 = 0, 1, 2, 3, 4, 5, 6

_vp, _i, _sz, _d = ctypes.c_void_p, ctypes.c_int, ctypes.c_size_t, ctypes.c_double


def _sig(name, res, *args):
    f = getattr(lib, name)
    f.restype = res
    f.argtypes = list(args)
    return f


_sig("nof_status_str", ctypes.c_char_p, _i)
_sig("nof_mo_transform_ws", _sz, _i, _i, _i, _i, _i, _i)
_sig("nof_mo_transform", _i, _i, _i, _i, _vp, _i, _vp, _vp, _i, _vp, _i, _vp, _sz, _vp)
_sig("nof_mo_transform_stage_ws", _sz, _i, _i, _i, _i)
_sig("nof_split_B_i8_bytes", _sz, _i, _i)
_sig("nof_split_B_i8", _i, _i, _i, _vp, _i, _vp, _sz, _vp)
_sig("nof_split_B_bytes", _sz, _i, _i)
_sig("nof_split_B", _i, _i, _i, _vp, _i, _vp, _sz, _vp)
_sig("nof_mo_transform_stage1", _i, _i, _i, _i, _vp, _i, _vp, _vp, _i, _i, _vp, _sz, _vp)
_sig("nof_mo_transform_stage2", _i, _i, _i, _i, _vp, _i, _vp, _vp, _i, _vp, _i, _vp, _sz, _vp)
_sig("nof_jk_diag_ws", _sz, _i, _i, _i)
_sig("nof_jk_diag", _i, _i, _i, _vp, _i, _vp, _vp, _vp, _vp, _sz, _vp)
_sig("nof_gen_fock_ws", _sz, _i, _i, _i, _i)
_sig("nof_exchange_fock_ws", _sz, _i, _i, _i, _i)
_sig("nof_exchange_fock", _i, _i, _i, _vp, _i, _vp, _vp, _i, _vp, _sz, _vp)
_sig("nof_fock_terms_ws", _sz, _i, _i, _i, _i)
_sig("nof_fock_terms", _i, _i, _i, _vp, _i, _vp, _vp, _vp, _vp, _i, _vp, _sz, _vp)
_sig("nof_coulomb_fock_ws", _sz, _i, _i, _i)
_sig("nof_coulomb_fock", _i, _i, _i, _vp, _i, _vp, _vp, _vp, _vp, _vp, _sz, _vp)
_sig("nof_lambda_grad", _i, _i, _vp, _vp, _vp, _vp, _vp, _vp, _vp)
_sig("nof_gen_fock", _i, _i, _i, _vp, _i, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _i, _vp, _sz, _vp)
_sig("nof_energy_ws", _sz, _i)
_sig("nof_energy", _i, _i, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _sz, _vp)
_sig("nof_coeffs_from_cumulant", _i, _i, _vp, _vp, _vp, _vp, _vp, _vp)
_sig("nof_expm_antisym_ws", _sz, _i)
_sig("nof_expm_antisym", _i, _i, _vp, _vp, _vp, _sz, _vp)
_sig("nof_rotate_orbitals_ws", _sz, _i, _i)
_sig("nof_rotate_orbitals", _i, _i, _i, _vp, _vp, _vp, _vp, _sz, _vp)
_sig("nof_adam_step", _i, _i, _vp, _vp, _vp, _i, _d, _d, _d, _d, _vp, _vp)
_sig("nof_occ_ws", _sz, _i, _i, _i)
_sig("nof_occ_energy_grad", _i, _i, _i, _i, _vp, _i, _i, _vp, _vp, _i, _vp, _vp, _vp, _vp, _vp, _vp, _vp,
     _sz, _vp)
_sig("nof_occ_optimize", _i, _i, _i, _i, _vp, _i, _i, _vp, _i, _vp, _vp, _vp, _vp, _vp, _vp, _i, _d, _vp,
     _sz, _vp)
_sig("nof_occ_optimize_noalloc", _i, _i, _i, _i, _vp, _i, _i, _vp, _i, _vp, _vp, _vp, _vp, _vp, _vp, _i, _d,
     _vp)
_sig("nof_functional_coeffs", _i, _i, _i, _i, _vp, _i, _vp, _vp, _vp, _vp, _vp, _sz, _vp)
_PLAN_ARGS = [_vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _sz, _vp]
_sig("nof_plan_create", _i, ctypes.POINTER(_vp), _i, _i, _i, _i, _i)
_sig("nof_plan_ws", _sz, _vp)
_sig("nof_plan_layout", _i, _vp, ctypes.POINTER(_sz), ctypes.POINTER(_sz), _i)
_sig("nof_plan_get_config", _i, _vp, ctypes.POINTER(_i))
_sig("nof_plan_set_config", _i, _vp, ctypes.POINTER(_i))
_sig("nof_plan_iteration", _i, *_PLAN_ARGS)
_sig("nof_plan_autotune", _i, *_PLAN_ARGS)
_sig("nof_plan_capture", _i, *_PLAN_ARGS)
_sig("nof_plan_launch", _i, _vp, _vp)
_sig("nof_plan_destroy", _i, _vp)
_sig("nof_mlp_nparams", _i)
_sig("nof_mlp_ws", _sz, _i)
_sig("nof_mlp_features_ws", _sz, _i)
_sig("nof_mlp_features", _i, _i, _vp, _i, _vp, _vp, _vp, _vp, _sz, _vp)
_sig("nof_mlp_forward", _i, _i, _vp, _vp, _vp, _vp)
_sig("nof_mlp_targets", _i, _i, _vp, _vp, _vp)
_sig("nof_mlp_loss_grad", _i, _i, _vp, _vp, _vp, _vp, _vp, _vp, _sz, _vp)
_sig("nof_mlp_adam", _i, _i, _vp, _vp, _vp, _vp, _i, ctypes.c_float, ctypes.c_float, ctypes.c_float,
     ctypes.c_float, _vp)
_sig("nof_mlp_warm_gamma", _i, _i, _i, _i, _vp, _i, _vp, _d, _vp, _vp, _vp)

class SolveParams(ctypes.Structure):
    _fields_ = [("max_outer", _i), ("no_steps", _i), ("lr", _d), ("beta1", _d), ("beta2", _d),
                ("eps", _d), ("tol_lambda", _d), ("tol_energy", _d), ("on_maxit", _i), ("on_tol", _d),
                ("tol_orth", _d), ("orbopt", _i), ("maxoff", _d)]


class SolveResult(ctypes.Structure):
    _fields_ = [("E", _d), ("asym", _d), ("outer", _i), ("no_steps", _i), ("on_iters", _i),
                ("converged", _i), ("status", _i), ("orth", _d), ("on_unconverged", _i)]


_sig("nof_solve_ws", _sz, _i, _i, _i, _i, _i, _i, _i)
_sig("nof_pseudo_fock_diag_ws", _sz, _i)
_sig("nof_pseudo_fock_diag", _i, _i, _vp, _vp, _d, _vp, _vp, _vp, _vp, _sz, _vp)
_sig("nof_orthonormalize_ws", _sz, _i, _i)
_sig("nof_orthonormalize", _i, _i, _i, _vp, _vp, _d, _vp, _vp, _sz, _vp)
_sig("nof_dipole_ws", _sz, _i, _i)
_sig("nof_dipole", _i, _i, _i, _vp, _vp, _vp, _vp, _vp, _sz, _vp)
_sig("nof_nlop_romberg", _i, _i, _d, _vp, _vp, _vp, _vp, _vp, _vp)
_sig("nof_nlop_isotropic", _i, _vp, _vp, _vp)
_sig("nof_solve", _i, _i, _i, _i, _vp, _i, _vp, _vp, _i, _i, _vp, _i, _i, _vp, _vp, _i,
     ctypes.POINTER(SolveParams), ctypes.POINTER(SolveResult), _vp, _sz, _vp)
_sig("nof_plan_solve_ws", _sz, _vp, _i, _i)
_sig("nof_plan_solve", _i, _vp, _vp, _vp, _vp, _i, _i, _vp, _i, _i, _vp, _vp,
     ctypes.POINTER(SolveParams), ctypes.POINTER(SolveResult), _vp, _sz, _vp)
MAP_TRIG, MAP_SOFTMAX = 0, 1
FUNC_HF, FUNC_PNOF5, FUNC_PNOF7 = 0, 1, 2

DECLARED = [
    "nof_status_str", "nof_mo_transform_ws", "nof_mo_transform", "nof_mo_transform_stage1",
    "nof_mo_transform_stage2", "nof_mo_transform_stage_ws", "nof_split_B_bytes", "nof_split_B",
    "nof_split_B_i8_bytes", "nof_split_B_i8",
    "nof_jk_diag_ws", "nof_jk_diag",
    "nof_gen_fock_ws", "nof_gen_fock", "nof_exchange_fock_ws", "nof_exchange_fock",
    "nof_fock_terms_ws", "nof_fock_terms", "nof_coulomb_fock_ws", "nof_coulomb_fock", "nof_lambda_grad", "nof_energy_ws", "nof_energy", "nof_coeffs_from_cumulant",
    "nof_expm_antisym_ws", "nof_expm_antisym", "nof_rotate_orbitals_ws", "nof_rotate_orbitals",
    "nof_orthonormalize_ws", "nof_orthonormalize",
    "nof_adam_step", "nof_occ_ws", "nof_occ_energy_grad", "nof_occ_optimize", "nof_occ_optimize_noalloc",
    "nof_functional_coeffs", "nof_plan_create", "nof_plan_ws", "nof_plan_layout", "nof_plan_get_config",
    "nof_plan_set_config", "nof_plan_iteration", "nof_plan_autotune", "nof_plan_capture",
    "nof_plan_launch", "nof_plan_destroy", "nof_mlp_nparams", "nof_mlp_ws", "nof_mlp_features_ws",
    "nof_solve_ws", "nof_solve", "nof_pseudo_fock_diag_ws", "nof_pseudo_fock_diag", "nof_plan_solve_ws", "nof_plan_solve", "nof_dipole_ws", "nof_dipole", "nof_nlop_romberg",
    "nof_nlop_isotropic", "nof_mlp_features", "nof_mlp_forward", "nof_mlp_targets", "nof_mlp_loss_grad", "nof_mlp_adam", "nof_mlp_warm_gamma",
]


class NofError(RuntimeError):
    def __init__(self, code: int, where: str):
        self.code = code
        super().__init__(f"{where}: {lib.nof_status_str(code).decode()} (status {code})")


def check(rc: int, where: str) -> None:
    if rc != OK:
        raise NofError(rc, where)


_TDT = {torch.float64: F64, torch.float32: F32, torch.bfloat16: BF16}
_PREC_OF = {F64: P_F64, F32: P_F32}


def _p(t):
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError("tensor must be on the GPU")
    if not t.is_contiguous():
        raise ValueError("tensor must be contiguous")
    return t.data_ptr()


def _f64(t, name):
    if t.dtype != torch.float64:
        raise TypeError(f"{name} must be float64")
    return _p(t)


def stream_handle(stream=None):
    s = torch.cuda.current_stream() if stream is None else stream
    return s.cuda_stream


def workspace(nbytes: int, device) -> torch.Tensor:
    return torch.empty(max(int(nbytes), 1), dtype=torch.uint8, device=device)


# ---------------------------------------------------------------------------
class SplitB:
    """B as the four fixed-point BF16 planes written by nof_split_B, the input
    of the P_BF16X10 transform (split once, reused by every iteration)."""

    def __init__(self, B, stream=None):
        naux, nbf, _ = B.shape
        self.shape = tuple(B.shape)
        self.device = B.device
        nbytes = lib.nof_split_B_bytes(naux, nbf)
        self.planes = workspace(nbytes, B.device)
        check(lib.nof_split_B(naux, nbf, _p(B), _TDT[B.dtype], _p(self.planes), nbytes,
                              stream_handle(stream)), "nof_split_B")


class SplitBI8:
    """B as the four fixed-point INT8 planes and row exponents written by
    nof_split_B_i8, the input of the P_I8X10 transform (split once)."""

    def __init__(self, B, stream=None):
        naux, nbf, _ = B.shape
        self.shape = tuple(B.shape)
        self.device = B.device
        nbytes = lib.nof_split_B_i8_bytes(naux, nbf)
        self.planes = workspace(nbytes, B.device)
        check(lib.nof_split_B_i8(naux, nbf, _p(B), _TDT[B.dtype], _p(self.planes), nbytes,
                                 stream_handle(stream)), "nof_split_B_i8")


def _b_arg(B):
    """(storage code, device pointer) of a B argument: a tensor, a SplitB or a
    SplitBI8."""
    if isinstance(B, SplitB):
        return BF16X4, _p(B.planes)
    if isinstance(B, SplitBI8):
        return I8X4, _p(B.planes)
    return _TDT[B.dtype], _p(B)


def _default_prec(Bt):
    return {F64: P_F64, F32: P_F32, BF16X4: P_BF16X10, I8X4: P_I8X10}.get(Bt, P_F64)


def mo_transform(B, C, prec=None, b=None, D=None, ws=None, stream=None):
    """b^P = C^T B^P C and D[P][p] = b^P_pp (nof_mo_transform).

    prec defaults to the arithmetic of B's storage (FP64 or FP32); the BF16
    split forms (P_BF16X1/X3/X6) take B in FP32 (or BF16 for X3/X6) and
    produce b in FP32."""
    naux, nbf, _ = B.shape
    norb = C.shape[1]
    Bt, Bp = _b_arg(B)
    prec = _default_prec(Bt) if prec is None else prec
    bdtype = torch.float64 if prec == P_F64 else torch.float32
    if b is None:
        b = torch.empty((naux, norb, norb), dtype=bdtype, device=B.device)
    bt = _TDT[b.dtype]
    if D is None:
        D = torch.empty((naux, norb), dtype=torch.float64, device=B.device)
    need = lib.nof_mo_transform_ws(naux, nbf, norb, Bt, bt, prec)
    if need == 0:
        raise NofError(E_DTYPE, "nof_mo_transform_ws")
    if ws is None or ws.numel() < need:
        ws = workspace(need, B.device)
    check(lib.nof_mo_transform(naux, nbf, norb, Bp, Bt, _f64(C, "C"), _p(b), bt, _p(D), prec,
                               _p(ws), ws.numel(), stream_handle(stream)), "nof_mo_transform")
    return b, D


def _stage_ws(naux, nbf, norb, prec, device, ws):
    need = lib.nof_mo_transform_stage_ws(naux, nbf, norb, prec)
    if ws is None or ws.numel() < need:
        ws = workspace(need, device)
    return ws


def transform_stage1(B, C, T, prec=None, ws=None, stream=None):
    """T^P = B^P C (first half of nof_mo_transform) into caller-owned T."""
    naux, nbf, _ = B.shape
    norb = C.shape[1]
    bt, Bp = _b_arg(B)
    prec = _default_prec(bt) if prec is None else prec
    ws = _stage_ws(naux, nbf, norb, prec, B.device, ws)
    check(lib.nof_mo_transform_stage1(naux, nbf, norb, Bp, bt, _f64(C, "C"), _p(T), _TDT[T.dtype],
                                      prec, _p(ws), ws.numel(), stream_handle(stream)),
          "nof_mo_transform_stage1")
    return T


def transform_stage2(T, C, b, D, prec=None, ws=None, stream=None):
    """b^P = C^T T^P and D (second half of nof_mo_transform)."""
    naux, nbf, norb = T.shape
    bt = _TDT[b.dtype]
    prec = _PREC_OF.get(bt, P_F64) if prec is None else prec
    ws = _stage_ws(naux, nbf, norb, prec, T.device, ws)
    check(lib.nof_mo_transform_stage2(naux, nbf, norb, _p(T), _TDT[T.dtype], _f64(C, "C"), _p(b), bt,
                                      _p(D), prec, _p(ws), ws.numel(), stream_handle(stream)),
          "nof_mo_transform_stage2")
    return b, D


def one_electron(H, C, stream=None):
    """h = C^T H C through the same transform with naux = 1."""
    b, _ = mo_transform(H.reshape(1, *H.shape), C, prec=P_F64, stream=stream)
    return b[0]


def jk_diag(b, D, want_J=True, want_K=True, J=None, K=None, ws=None, stream=None):
    naux, norb, _ = b.shape
    bt = _TDT[b.dtype]
    dev = b.device
    if want_J and J is None:
        J = torch.empty((norb, norb), dtype=torch.float64, device=dev)
    if want_K and K is None:
        K = torch.empty((norb, norb), dtype=torch.float64, device=dev)
    need = lib.nof_jk_diag_ws(naux, norb, bt)
    if ws is None or ws.numel() < need:
        ws = workspace(need, dev)
    check(lib.nof_jk_diag(naux, norb, _p(b), bt, _f64(D, "D"), _p(J) if want_J else None,
                          _p(K) if want_K else None, _p(ws), ws.numel(), stream_handle(stream)),
          "nof_jk_diag")
    return (J if want_J else None), (K if want_K else None)


def gen_fock(b, D, n, h, cJ, cK, want_grad=True, want_K=False, prec=None, out=None, ws=None,
             stream=None):
    """lambda, grad (and optionally K) of the generalized-Fock build (nof_gen_fock)."""
    naux, norb, _ = b.shape
    bt = _TDT[b.dtype]
    prec = _PREC_OF.get(bt, P_F64) if prec is None else prec
    dev = b.device
    if out is None:
        out = {}
    lam = out.get("lam")
    if lam is None:
        lam = torch.empty((norb, norb), dtype=torch.float64, device=dev)
    g = out.get("g") if want_grad else None
    if want_grad and g is None:
        g = torch.empty((norb, norb), dtype=torch.float64, device=dev)
    K = out.get("K") if want_K else None
    if want_K and K is None:
        K = torch.empty((norb, norb), dtype=torch.float64, device=dev)
    need = lib.nof_gen_fock_ws(naux, norb, bt, prec)
    if ws is None or ws.numel() < need:
        ws = workspace(need, dev)
    check(lib.nof_gen_fock(naux, norb, _p(b), bt, _f64(D, "D"), _f64(n, "n"), _f64(h, "h"),
                           _f64(cJ, "cJ"), _f64(cK, "cK"), _p(lam), _p(g), _p(K), prec, _p(ws),
                           ws.numel(), stream_handle(stream)), "nof_gen_fock")
    return lam, g, K


def exchange_fock(b, cK, prec=None, F2=None, ws=None, stream=None):
    """F2_rs = sum_P sum_q b^P_rq cK_sq b^P_qs alone (nof_exchange_fock)."""
    naux, norb, _ = b.shape
    bt = _TDT[b.dtype]
    prec = _PREC_OF.get(bt, P_F64) if prec is None else prec
    if F2 is None:
        F2 = torch.empty((norb, norb), dtype=torch.float64, device=b.device)
    need = lib.nof_exchange_fock_ws(naux, norb, bt, prec)
    if ws is None or ws.numel() < need:
        ws = workspace(need, b.device)
    check(lib.nof_exchange_fock(naux, norb, _p(b), bt, _f64(cK, "cK"), _p(F2), prec, _p(ws), ws.numel(),
                                stream_handle(stream)), "nof_exchange_fock")
    return F2


def fock_terms(b, D, cJ, cK, prec=None, F=None, ws=None, stream=None):
    """F = F2 - F1 in one contraction, the Coulomb-type term folded into the
    exchange-type product's right operand (nof_fock_terms)."""
    naux, norb, _ = b.shape
    bt = _TDT[b.dtype]
    prec = _PREC_OF.get(bt, P_F64) if prec is None else prec
    if F is None:
        F = torch.empty((norb, norb), dtype=torch.float64, device=b.device)
    need = lib.nof_fock_terms_ws(naux, norb, bt, prec)
    if ws is None or ws.numel() < need:
        ws = workspace(need, b.device)
    check(lib.nof_fock_terms(naux, norb, _p(b), bt, _f64(D, "D"), _f64(cJ, "cJ"), _f64(cK, "cK"), _p(F),
                             prec, _p(ws), ws.numel(), stream_handle(stream)), "nof_fock_terms")
    return F


def coulomb_fock(b, D, cJ, F1=None, K=None, want_K=True, ws=None, stream=None):
    """F1_rs = sum_P b^P_rs (D cJ)[P][s] and K from the same pass (nof_coulomb_fock)."""
    naux, norb, _ = b.shape
    bt = _TDT[b.dtype]
    dev = b.device
    if F1 is None:
        F1 = torch.empty((norb, norb), dtype=torch.float64, device=dev)
    if want_K and K is None:
        K = torch.empty((norb, norb), dtype=torch.float64, device=dev)
    need = lib.nof_coulomb_fock_ws(naux, norb, bt)
    if ws is None or ws.numel() < need:
        ws = workspace(need, dev)
    check(lib.nof_coulomb_fock(naux, norb, _p(b), bt, _f64(D, "D"), _f64(cJ, "cJ"), _p(F1),
                               _p(K) if want_K else None, _p(ws), ws.numel(), stream_handle(stream)),
          "nof_coulomb_fock")
    return F1, (K if want_K else None)


def lambda_grad(n, h, F1, F2, lam=None, g=None, want_grad=True, stream=None):
    """lambda = n_s h_rs + F1 - F2 and grad = 4(lambda - lambda^T) (nof_lambda_grad);
    F1 = None: F2 is the combined F2 - F1 of fock_terms."""
    norb = n.shape[0]
    if lam is None:
        lam = torch.empty((norb, norb), dtype=torch.float64, device=n.device)
    if want_grad and g is None:
        g = torch.empty_like(lam)
    f1 = None if F1 is None else _f64(F1, "F1")
    check(lib.nof_lambda_grad(norb, _f64(n, "n"), _f64(h, "h"), f1, _f64(F2, "F2"), _p(lam),
                              _p(g) if want_grad else None, stream_handle(stream)), "nof_lambda_grad")
    return lam, (g if want_grad else None)


def energy(n, h, J, K, cJ, cK, E=None, ws=None, stream=None):
    norb = n.shape[0]
    if E is None:
        E = torch.empty((), dtype=torch.float64, device=n.device)
    need = lib.nof_energy_ws(norb)
    if ws is None or ws.numel() < need:
        ws = workspace(need, n.device)
    check(lib.nof_energy(norb, _f64(n, "n"), _f64(h, "h"), _f64(J, "J"), _f64(K, "K"),
                         _f64(cJ, "cJ"), _f64(cK, "cK"), _p(E), _p(ws), ws.numel(), stream_handle(stream)),
          "nof_energy")
    return E


def coeffs_from_cumulant(n, Delta, Pi, stream=None):
    norb = n.shape[0]
    cJ = torch.empty((norb, norb), dtype=torch.float64, device=n.device)
    cK = torch.empty_like(cJ)
    check(lib.nof_coeffs_from_cumulant(norb, _f64(n, "n"), _f64(Delta, "Delta"), _f64(Pi, "Pi"),
                                       _p(cJ), _p(cK), stream_handle(stream)), "nof_coeffs_from_cumulant")
    return cJ, cK


def expm_antisym(y, U=None, ws=None, stream=None):
    """U = exp(y) for antisymmetric y (nof_expm_antisym)."""
    norb = y.shape[0]
    if U is None:
        U = torch.empty_like(y)
    need = lib.nof_expm_antisym_ws(norb)
    if ws is None or ws.numel() < need:
        ws = workspace(need, y.device)
    check(lib.nof_expm_antisym(norb, _f64(y, "y"), _p(U), _p(ws), ws.numel(), stream_handle(stream)),
          "nof_expm_antisym")
    return U


def rotate_orbitals(C, U, Cout=None, ws=None, stream=None):
    """Cout = C U (nof_rotate_orbitals)."""
    nbf, norb = C.shape
    if Cout is None:
        Cout = torch.empty_like(C)
    need = lib.nof_rotate_orbitals_ws(nbf, norb)
    if ws is None or ws.numel() < need:
        ws = workspace(need, C.device)
    check(lib.nof_rotate_orbitals(nbf, norb, _f64(C, "C"), _f64(U, "U"), _p(Cout), _p(ws), ws.numel(),
                                  stream_handle(stream)), "nof_rotate_orbitals")
    return Cout


def orthonormalize(C, S=None, tol=1e-10, err=None, ws=None, stream=None):
    """Check max|C^T S C - I| and repair C in place past tol (nof_orthonormalize);
    returns the device scalar err."""
    nbf, norb = C.shape
    if err is None:
        err = torch.empty((), dtype=torch.float64, device=C.device)
    need = lib.nof_orthonormalize_ws(nbf, norb)
    if ws is None or ws.numel() < need:
        ws = workspace(need, C.device)
    check(lib.nof_orthonormalize(nbf, norb, _f64(C, "C"), _f64(S, "S") if S is not None else None,
                                 float(tol), _p(err), _p(ws), ws.numel(), stream_handle(stream)),
          "nof_orthonormalize")
    return err


def adam_step(g, m, v, t, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8, y=None, stream=None):
    """One ADAM step on the orbital gradient; returns the rotation generator y."""
    norb = g.shape[0]
    if y is None:
        y = torch.empty_like(g)
    check(lib.nof_adam_step(norb, _f64(g, "g"), _f64(m, "m"), _f64(v, "v"), int(t), lr, beta1, beta2,
                            eps, _p(y), stream_handle(stream)), "nof_adam_step")
    return y


class Rotation:
    """Preallocated FP64 rotation step C <- C exp(y) (workspace reused)."""

    def __init__(self, norb, nbf, device):
        self.U = torch.empty((norb, norb), dtype=torch.float64, device=device)
        self.ws = workspace(lib.nof_expm_antisym_ws(norb), device)
        self.ws_rot = workspace(lib.nof_rotate_orbitals_ws(nbf, norb), device)

    def apply(self, C, y, Cout, stream=None):
        expm_antisym(y, self.U, self.ws, stream)
        return rotate_orbitals(C, self.U, Cout, self.ws_rot, stream)


def _i32(t, name):
    if t.dtype != torch.int32:
        raise TypeError(f"{name} must be int32")
    return _p(t)


class Occupations:
    """Occupation-number update at fixed orbitals for one pairing structure."""

    def __init__(self, norb, members, mapping=MAP_TRIG, functional=FUNC_PNOF5):
        self.norb = int(norb)
        self.members = members.to(torch.int32).contiguous()
        self.ns, ng1 = self.members.shape
        self.ng = ng1 - 1
        self.map, self.func = int(mapping), int(functional)
        dev = self.members.device
        self.ws = workspace(lib.nof_occ_ws(self.norb, self.ns, self.ng), dev)
        self.info = torch.zeros(4, dtype=torch.int32, device=dev)

    def _h(self, h):
        # a full [norb][norb] h is read along its diagonal, a [norb] vector directly
        return (_f64(h, "h"), self.norb + 1) if h.dim() == 2 else (_f64(h, "h"), 1)

    def energy_grad(self, gamma, h, J, K, stream=None):
        dev = gamma.device
        n = torch.empty(self.norb, dtype=torch.float64, device=dev)
        E = torch.empty((), dtype=torch.float64, device=dev)
        g = torch.empty_like(gamma)
        hp, hs = self._h(h)
        check(lib.nof_occ_energy_grad(self.norb, self.ns, self.ng, _p(self.members), self.map, self.func,
                                      _f64(gamma, "gamma"), hp, hs, _f64(J, "J"), _f64(K, "K"), _p(n),
                                      _p(E), _p(g), _p(self.info), _p(self.ws), self.ws.numel(),
                                      stream_handle(stream)), "nof_occ_energy_grad")
        return E, g, n

    def optimize(self, gamma, h, J, K, maxit=2000, tol=1e-8, stream=None):
        """L-BFGS in place on gamma; returns (E, n, info) with info = [iters, converged, status]."""
        dev = gamma.device
        n = torch.empty(self.norb, dtype=torch.float64, device=dev)
        E = torch.empty((), dtype=torch.float64, device=dev)
        hp, hs = self._h(h)
        check(lib.nof_occ_optimize(self.norb, self.ns, self.ng, _p(self.members), self.map, self.func,
                                   hp, hs, _f64(J, "J"), _f64(K, "K"), _f64(gamma, "gamma"), _p(n), _p(E),
                                   _p(self.info), int(maxit), float(tol), _p(self.ws), self.ws.numel(),
                                   stream_handle(stream)), "nof_occ_optimize")
        return E, n, self.info

    def coefficients(self, n, stream=None):
        cJ = torch.empty((self.norb, self.norb), dtype=torch.float64, device=n.device)
        cK = torch.empty_like(cJ)
        check(lib.nof_functional_coeffs(self.norb, self.ns, self.ng, _p(self.members), self.func,
                                        _f64(n, "n"), _p(cJ), _p(cK), _p(self.info), _p(self.ws),
                                        self.ws.numel(), stream_handle(stream)), "nof_functional_coeffs")
        return cJ, cK


class BatchPlan:
    """Batched iteration for ninst instances sharing B (nof_plan_*).

    Inputs are bound at construction (their device buffers are read on every
    call, so update them in place between iterations)."""

    def __init__(self, B, C, H, n, cJ, cK, prec=None):
        """B: FP64 (P_F64), FP32 (P_F32), a SplitB (P_BF16X10) or a SplitBI8 (P_I8X10)."""
        self.ninst, nbf, norb = C.shape
        naux = B.shape[0]
        bt = _b_arg(B)[0]
        self.prec = _default_prec(bt) if prec is None else prec
        self.handle = _vp()
        check(lib.nof_plan_create(ctypes.byref(self.handle), self.ninst, naux, nbf, norb, self.prec),
              "nof_plan_create")
        dev = B.device
        self.ws = workspace(lib.nof_plan_ws(self.handle), dev)
        self.inputs = (B, C, H, n, cJ, cK)
        for t, name in zip(self.inputs[1:], ("C", "H", "n", "cJ", "cK")):
            _f64(t, name)
        self.E = torch.empty(self.ninst, dtype=torch.float64, device=dev)
        self.solve_ws = None
        self.lam = torch.empty((self.ninst, norb, norb), dtype=torch.float64, device=dev)
        self.g = torch.empty_like(self.lam)

    def _args(self):
        B, C, H, n, cJ, cK = self.inputs
        return (self.handle, _b_arg(B)[1], _p(C), _p(H), _p(n), _p(cJ), _p(cK), _p(self.E), _p(self.lam),
                _p(self.g), _p(self.ws), self.ws.numel())

    def iteration(self, stream=None):
        check(lib.nof_plan_iteration(*self._args(), stream_handle(stream)), "nof_plan_iteration")
        return self.E, self.lam, self.g

    def autotune(self, stream=None):
        check(lib.nof_plan_autotune(*self._args(), stream_handle(stream)), "nof_plan_autotune")
        return self.config

    def capture(self, stream):
        check(lib.nof_plan_capture(*self._args(), stream_handle(stream)), "nof_plan_capture")

    def launch(self, stream):
        check(lib.nof_plan_launch(self.handle, stream_handle(stream)), "nof_plan_launch")
        return self.E, self.lam, self.g

    def solve(self, members, mapping, functional, gamma, n_out=None, stream=None, max_outer=100,
              no_steps=30, lr=0.01, beta1=0.9, beta2=0.999, eps=1e-8, tol_lambda=1e-5,
              tol_energy=1e-9, on_maxit=2000, on_tol=1e-8, tol_orth=1e-10):
        """Alternating NO + ON optimisation of every instance (nof_plan_solve).
        The bound C [ninst][nbf][norb] and gamma [ninst][ns][ng] are updated in
        place; returns one result dict per instance."""
        B, C, H = self.inputs[:3]
        _, ns, ng = gamma.shape
        if members.dtype != torch.int32:
            raise TypeError("members must be int32")
        need = lib.nof_plan_solve_ws(self.handle, ns, ng)
        if need == 0:
            raise NofError(E_DIM, "nof_plan_solve_ws")
        if self.solve_ws is None or self.solve_ws.numel() < need:
            self.solve_ws = workspace(need, C.device)
        prm = SolveParams(max_outer, no_steps, lr, beta1, beta2, eps, tol_lambda, tol_energy, on_maxit,
                          on_tol, tol_orth, 2, 1.0)
        res = (SolveResult * self.ninst)()
        rc = lib.nof_plan_solve(self.handle, _b_arg(B)[1], _f64(H, "H"), _f64(C, "C"), ns, ng, _p(members),
                                int(mapping), int(functional), _f64(gamma, "gamma"), _p(n_out),
                                ctypes.byref(prm), res, _p(self.solve_ws), self.solve_ws.numel(),
                                stream_handle(stream))
        out = [{f: getattr(r, f) for f, _ in SolveResult._fields_} for r in res]
        if rc != E_NOT_CONVERGED:
            check(rc, "nof_plan_solve")
        return out

    @property
    def config(self):
        cfg = (ctypes.c_int * 4)()
        check(lib.nof_plan_get_config(self.handle, cfg), "nof_plan_get_config")
        return list(cfg)

    @config.setter
    def config(self, cfg):
        arr = (ctypes.c_int * 4)(*[int(x) for x in cfg])
        check(lib.nof_plan_set_config(self.handle, arr), "nof_plan_set_config")

    def __del__(self):
        h = getattr(self, "handle", None)
        if h is not None and h.value and lib is not None:     # lib is None at interpreter exit
            lib.nof_plan_destroy(h)
            self.handle = None


def _f32(t, name):
    if t.dtype != torch.float32:
        raise TypeError(f"{name} must be float32")
    return _p(t)


def mlp_features(h, J, K, stream=None):
    """[norb][5] standardised FP32 features (nof_mlp_features); h full or its diagonal."""
    norb = J.shape[0]
    X = torch.empty((norb, 5), dtype=torch.float32, device=J.device)
    ws = workspace(lib.nof_mlp_features_ws(norb), J.device)
    hs = norb + 1 if h.dim() == 2 else 1
    check(lib.nof_mlp_features(norb, _f64(h, "h"), hs, _f64(J, "J"), _f64(K, "K"), _p(X), _p(ws),
                               ws.numel(), stream_handle(stream)), "nof_mlp_features")
    return X


def mlp_targets(n, stream=None):
    theta = torch.empty(n.numel(), dtype=torch.float32, device=n.device)
    check(lib.nof_mlp_targets(n.numel(), _f64(n, "n"), _p(theta), stream_handle(stream)), "nof_mlp_targets")
    return theta


def mlp_forward(X, params, theta=None, stream=None):
    rows = X.shape[0]
    if theta is None:
        theta = torch.empty(rows, dtype=torch.float32, device=X.device)
    check(lib.nof_mlp_forward(rows, _f32(X, "X"), _f32(params, "params"), _p(theta),
                              stream_handle(stream)), "nof_mlp_forward")
    return theta


def mlp_loss_grad(X, target, params, grad=None, loss=None, ws=None, stream=None):
    rows = X.shape[0]
    if grad is None:
        grad = torch.empty_like(params)
    if loss is None:
        loss = torch.empty((), dtype=torch.float32, device=X.device)
    need = lib.nof_mlp_ws(rows)
    if ws is None or ws.numel() < need:
        ws = workspace(need, X.device)
    check(lib.nof_mlp_loss_grad(rows, _f32(X, "X"), _f32(target, "target"), _f32(params, "params"),
                                _p(grad), _p(loss), _p(ws), ws.numel(), stream_handle(stream)),
          "nof_mlp_loss_grad")
    return loss, grad


def mlp_adam(params, grad, m, v, t, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8, stream=None):
    check(lib.nof_mlp_adam(params.numel(), _f32(params, "params"), _f32(grad, "grad"), _f32(m, "m"),
                           _f32(v, "v"), int(t), lr, beta1, beta2, eps, stream_handle(stream)),
          "nof_mlp_adam")


def mlp_warm_gamma(theta, members, mapping, norb, nfloor=1e-12, info=None, stream=None):
    ns, ng1 = members.shape
    gamma = torch.empty((ns, ng1 - 1), dtype=torch.float64, device=theta.device)
    check(lib.nof_mlp_warm_gamma(norb, ns, ng1 - 1, _i32(members, "members"), int(mapping),
                                 _f32(theta, "theta"), float(nfloor), _p(gamma), _p(info),
                                 stream_handle(stream)),
          "nof_mlp_warm_gamma")
    return gamma


def solve(B, C, H, members, mapping, functional, gamma, prec=None, n=None, ws=None, stream=None,
          max_outer=100, no_steps=30, lr=0.01, beta1=0.9, beta2=0.999, eps=1e-8, tol_lambda=1e-5,
          tol_energy=1e-9, on_maxit=2000, on_tol=1e-8, tol_orth=1e-10, orbopt=2, maxoff=1.0):
    """Alternating NO + ON optimisation to convergence (nof_solve).  C and gamma
    are updated in place; returns the result as a dict."""
    naux, nbf, _ = B.shape
    norb = C.shape[1]
    ns, ng = gamma.shape
    Bt, Bp = _b_arg(B)
    prec = _default_prec(Bt) if prec is None else prec
    if members.dtype != torch.int32:
        raise TypeError("members must be int32")
    need = lib.nof_solve_ws(naux, nbf, norb, ns, ng, Bt, prec)
    if need == 0:
        raise NofError(E_DIM, "nof_solve_ws")
    if ws is None or ws.numel() < need:
        ws = workspace(need, C.device)
    prm = SolveParams(max_outer, no_steps, lr, beta1, beta2, eps, tol_lambda, tol_energy, on_maxit, on_tol,
                      tol_orth, orbopt, maxoff)
    res = SolveResult()
    check(lib.nof_solve(naux, nbf, norb, Bp, Bt, _f64(H, "H"), _f64(C, "C"), ns, ng, _p(members),
                        mapping, functional, _f64(gamma, "gamma"), _p(n), prec, ctypes.byref(prm),
                        ctypes.byref(res), _p(ws), ws.numel(), stream_handle(stream)), "nof_solve")
    return {f: getattr(res, f) for f, _ in SolveResult._fields_}


def pseudo_fock_diag(lam, diag=None, maxoff=1.0, V=None, eig=None, ws=None, stream=None):
    """One iterative-diagonalization step (nof_pseudo_fock_diag): returns
    (V, eig, info) with info = [sweeps, assignment ok] (device)."""
    norb = lam.shape[0]
    dev = lam.device
    if V is None:
        V = torch.empty((norb, norb), dtype=torch.float64, device=dev)
    if eig is None:
        eig = torch.empty(norb, dtype=torch.float64, device=dev)
    info = torch.zeros(2, dtype=torch.int32, device=dev)
    need = lib.nof_pseudo_fock_diag_ws(norb)
    if need == 0:
        raise NofError(E_DIM, "nof_pseudo_fock_diag_ws")
    if ws is None or ws.numel() < need:
        ws = workspace(need, dev)
    check(lib.nof_pseudo_fock_diag(norb, _f64(lam, "lambda"), _p(diag) if diag is not None else None,
                                   float(maxoff), _p(V), _p(eig), _p(info), _p(ws), ws.numel(),
                                   stream_handle(stream)), "nof_pseudo_fock_diag")
    return V, eig, info


def dipole(C, n, d, mu=None, ws=None, stream=None):
    """mu = -2 sum_p n_p (C^T d C)_pp (nof_dipole), a device scalar."""
    nbf, norb = C.shape
    if mu is None:
        mu = torch.empty((), dtype=torch.float64, device=C.device)
    need = lib.nof_dipole_ws(nbf, norb)
    if ws is None or ws.numel() < need:
        ws = workspace(need, C.device)
    check(lib.nof_dipole(nbf, norb, _f64(C, "C"), _f64(n, "n"), _f64(d, "d"), _p(mu), _p(ws), ws.numel(),
                         stream_handle(stream)), "nof_dipole")
    return mu


def nlop_romberg(mu0, mu_p, mu_m, step, stream=None):
    """alpha, beta, gamma tables and selections (nof_nlop_romberg); mu_p, mu_m
    hold mu(+-h_k) for k = 1 .. npoint+1."""
    npoint = mu_p.shape[0] - 1
    table = torch.empty((3, npoint, npoint), dtype=torch.float64, device=mu_p.device)
    result = torch.empty((3, 4), dtype=torch.float64, device=mu_p.device)
    check(lib.nof_nlop_romberg(npoint, step, _f64(mu0, "mu0"), _f64(mu_p, "mu_p"), _f64(mu_m, "mu_m"),
                               _p(table), _p(result), stream_handle(stream)), "nof_nlop_romberg")
    return table, result


def nlop_isotropic(alpha, stream=None):
    """(mean, anisotropy) of the diagonal polarizabilities alpha[3] (nof_nlop_isotropic)."""
    out = torch.empty(2, dtype=torch.float64, device=alpha.device)
    check(lib.nof_nlop_isotropic(_f64(alpha, "alpha"), _p(out), stream_handle(stream)), "nof_nlop_isotropic")
    return out
