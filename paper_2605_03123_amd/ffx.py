"""Python binding of libffx (include/ffx.h): argument marshalling only.

Every operation runs in the HIP kernels of libffx.so; torch is used for device
memory and the current HIP stream.  Importing this module loads the library
and raises ImportError if it has not been built (python -m
paper_2605_03123_amd.build) -- there is no fallback path.

State vectors are torch tensors of dtype complex128 or complex64 on a ROCm
device, shaped (dim_a, dim_b) (or flat), contiguous, alpha-major as in the
paper's representation (Sec. 3.1).  Functions return a new tensor unless
``out`` is given (``out=vec`` evolves in place), following the functional style
of Sec. 4.1.
"""
from __future__ import annotations

import ctypes
import os
from functools import lru_cache

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "libffx.so")
if not os.path.exists(_LIB_PATH):
    raise ImportError(f"libffx.so not found at {_LIB_PATH}; build it with `python -m paper_2605_03123_amd.build`")
_lib = ctypes.CDLL(_LIB_PATH)

_c_double_p = ctypes.POINTER(ctypes.c_double)
_c_int_p = ctypes.POINTER(ctypes.c_int)
_c_u64_p = ctypes.POINTER(ctypes.c_uint64)

FFX_C128, FFX_C64 = 0, 1
ERRORS = {-1: "FFX_EINVAL", -2: "FFX_ENOTUNITARY", -3: "FFX_ENOMEM", -4: "FFX_EDEVICE", -5: "FFX_EUNSUPPORTED"}


class FFXError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{ERRORS.get(code, code)}: {msg}")
        self.code = code


class _DFHam(ctypes.Structure):
    _fields_ = [("norb", ctypes.c_int), ("n_terms", ctypes.c_int), ("h", _c_double_p),
                ("J", _c_double_p), ("U", _c_double_p)]


class _LUCJ(ctypes.Structure):
    _fields_ = [("norb", ctypes.c_int), ("n_reps", ctypes.c_int), ("params", _c_double_p)]


def _sig(name, res, args):
    f = getattr(_lib, name)
    f.restype = res
    f.argtypes = args
    return f


_vp = ctypes.c_void_p
_last_error = _sig("ffx_last_error", ctypes.c_char_p, [])
_dim = _sig("ffx_dim", ctypes.c_int64, [ctypes.c_int, ctypes.c_int])
_strings = _sig("ffx_strings", ctypes.c_int, [ctypes.c_int, ctypes.c_int, _c_u64_p])
_givens = _sig("ffx_givens_decomposition", ctypes.c_int,
               [ctypes.c_int, _c_double_p, _c_int_p, _c_double_p, _c_double_p, _c_double_p])
_plan_create = _sig("ffx_plan_create", ctypes.c_int,
                    [ctypes.POINTER(_vp), ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int])
_plan_destroy = _sig("ffx_plan_destroy", ctypes.c_int, [_vp])
_plan_info = _sig("ffx_plan_info", ctypes.c_int,
                  [_vp, ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int64)])
_plan_strings = _sig("ffx_plan_strings", ctypes.c_int, [_vp, ctypes.c_int, _c_u64_p])
_rot = _sig("ffx_apply_orbital_rotation", ctypes.c_int, [_vp, _vp, _c_double_p, _c_double_p, _vp])
_rot_dense = _sig("ffx_apply_orbital_rotation_dense", ctypes.c_int, [_vp, _vp, _c_double_p, _c_double_p, _vp, _vp])
_numop = _sig("ffx_apply_num_op_sum_evolution", ctypes.c_int,
              [_vp, _vp, _c_double_p, _c_double_p, ctypes.c_double, _c_double_p, _vp])
_dc = _sig("ffx_apply_diag_coulomb_evolution", ctypes.c_int,
           [_vp, _vp, _c_double_p, _c_double_p, _c_double_p, ctypes.c_double, _c_double_p, _vp])
_trotter = _sig("ffx_apply_df_trotter_step", ctypes.c_int,
                [_vp, _vp, ctypes.POINTER(_DFHam), ctypes.c_double, ctypes.c_int, ctypes.c_int, _vp])
_trotter_dc = _sig("ffx_simulate_trotter_diag_coulomb", ctypes.c_int,
                   [_vp, _vp, _c_double_p, _c_double_p, _c_double_p, _c_double_p, ctypes.c_double, ctypes.c_int,
                    ctypes.c_int, _vp])
_lucj_np = _sig("ffx_lucj_n_params", ctypes.c_int, [ctypes.c_int, ctypes.c_int])
_lucj = _sig("ffx_apply_lucj", ctypes.c_int, [_vp, _vp, ctypes.POINTER(_LUCJ), _vp])
_ws = _sig("ffx_workspace_bytes", ctypes.c_int64, [_vp, ctypes.c_int])
_energy = _sig("ffx_df_energy", ctypes.c_int, [_vp, _vp, ctypes.POINTER(_DFHam), _c_double_p, _vp, _vp])
_hact = _sig("ffx_apply_df_hamiltonian", ctypes.c_int, [_vp, _vp, _vp, ctypes.POINTER(_DFHam), _vp, _vp])
_exact = _sig("ffx_df_evolve_exact", ctypes.c_int,
              [_vp, _vp, ctypes.POINTER(_DFHam), ctypes.c_double, ctypes.c_double, _vp,
               ctypes.POINTER(ctypes.c_int), _vp])
_dist = _sig("ffx_state_distance", ctypes.c_int, [_vp, _vp, _vp, _c_double_p, _vp])
_ci = ctypes.c_int
_numint = _sig("ffx_apply_num_interaction", _ci, [_vp, _vp, ctypes.c_double, _ci, _ci, _vp])
_numnum = _sig("ffx_apply_num_num_interaction", _ci, [_vp, _vp, ctypes.c_double, _ci, _ci, _ci, _ci, _vp])
_givensg = _sig("ffx_apply_givens_rotation", _ci, [_vp, _vp, ctypes.c_double, _ci, _ci, _ci, _vp])
_tunnel = _sig("ffx_apply_tunneling_interaction", _ci, [_vp, _vp, ctypes.c_double, _ci, _ci, _ci, _vp])
_quad = _sig("ffx_apply_quad_ham_evolution", _ci, [_vp, _vp, _c_double_p, _c_double_p, ctypes.c_double, _vp])
_slater = _sig("ffx_slater_determinant", _ci, [_vp, _vp, _c_int_p, _c_int_p, _c_double_p, _c_double_p, _vp])
_ucj = _sig("ffx_apply_ucj", _ci, [_vp, _vp, _ci, _c_double_p, _c_double_p, _c_double_p, _c_double_p,
                                   _c_double_p, _c_double_p, _c_double_p, _vp])
_sstate = _sig("ffx_sample_state", _ci, [_vp, _vp, _c_double_p, ctypes.c_int64, ctypes.POINTER(ctypes.c_int64), _vp])
_sstate_na = _sig("ffx_sample_state_noalloc", _ci, [_vp, _vp, _vp, ctypes.c_int64, _vp, _vp])
_sslater = _sig("ffx_sample_slater", _ci, [_vp, _c_int_p, _c_int_p, _c_double_p, _c_double_p, _c_double_p, _c_double_p,
                                           ctypes.c_int64, _c_u64_p, _c_u64_p, _vp])
_tenable = _sig("ffx_timing_enable", ctypes.c_int, [_vp, ctypes.c_int])
_tread = _sig("ffx_timing_read", ctypes.c_int,
              [_vp, ctypes.c_int, _c_double_p, ctypes.POINTER(ctypes.c_int64), _c_double_p, _c_double_p])
_egrad = _sig("ffx_lucj_energy_grad", ctypes.c_int,
              [_vp, ctypes.POINTER(_LUCJ), ctypes.POINTER(_DFHam), _c_double_p, _c_double_p, _vp, _vp, _vp])


def _check(code: int):
    if code != 0:
        raise FFXError(code, _last_error().decode())


def _dptr(a: np.ndarray):
    return a.ctypes.data_as(_c_double_p)


def _real(m, shape=None) -> np.ndarray:
    a = np.ascontiguousarray(np.asarray(m, dtype=np.float64))
    if shape is not None and a.shape != shape:
        raise ValueError(f"expected shape {shape}, got {a.shape}")
    return a


def _cplx(m, shape=None) -> np.ndarray:
    a = np.ascontiguousarray(np.asarray(m, dtype=np.complex128))
    if shape is not None and a.shape != shape:
        raise ValueError(f"expected shape {shape}, got {a.shape}")
    return a.view(np.float64)


def _stream(device) -> ctypes.c_void_p:
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


# ---------------------------------------------------------------------------
# host-only helpers
# ---------------------------------------------------------------------------

def dim(norb: int, n: int) -> int:
    d = _dim(norb, n)
    if d < 0:
        raise ValueError("bad norb / n")
    return int(d)


def strings(norb: int, n: int) -> np.ndarray:
    out = np.zeros(dim(norb, n), dtype=np.uint64)
    _check(_strings(norb, n, out.ctypes.data_as(_c_u64_p)))
    return out


def givens_decomposition(U):
    """-> (p, c, s, phase) with U = diag(exp(i phase)) G_K ... G_1 (host, FP64)."""
    U = np.asarray(U)
    norb = U.shape[0]
    Uc = _cplx(U, (norb, norb))
    K = norb * (norb - 1) // 2
    p = np.zeros(K, dtype=np.int32)
    c = np.zeros(K)
    s = np.zeros(K, dtype=np.complex128)
    ph = np.zeros(norb)
    _check(_givens(norb, _dptr(Uc), p.ctypes.data_as(_c_int_p), _dptr(c), _dptr(s.view(np.float64)), _dptr(ph)))
    return p, c, s, ph


# ---------------------------------------------------------------------------
# plans
# ---------------------------------------------------------------------------

class Plan:
    """Device tables for one (norb, nelec, dtype, device); see ffx_plan_create."""

    def __init__(self, norb: int, nelec, dtype=torch.complex128, device=0):
        if isinstance(device, torch.device):
            device = device.index or 0
        self.norb = int(norb)
        self.nelec = (int(nelec[0]), int(nelec[1]))
        self.dtype = dtype
        self.device = int(device)
        code = {torch.complex128: FFX_C128, torch.complex64: FFX_C64}.get(dtype)
        if code is None:
            raise ValueError("dtype must be torch.complex128 or torch.complex64")
        h = _vp()
        _check(_plan_create(ctypes.byref(h), self.norb, self.nelec[0], self.nelec[1], code, self.device))
        self._h = h
        da, db, nb = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
        _check(_plan_info(h, ctypes.byref(da), ctypes.byref(db), ctypes.byref(nb)))
        self.dim_a, self.dim_b, self.state_bytes = da.value, db.value, nb.value
        self._ws = {}

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            try:
                _plan_destroy(h)
            except Exception:
                pass
            self._h = None

    @property
    def handle(self):
        return self._h

    def strings(self, spin: int) -> np.ndarray:
        out = np.zeros(self.dim_b if spin else self.dim_a, dtype=np.uint64)
        _check(_plan_strings(self._h, spin, out.ctypes.data_as(_c_u64_p)))
        return out

    def workspace(self, what: int) -> torch.Tensor:
        n = int(_ws(self._h, what))
        ws = self._ws.get(what)
        if ws is None or ws.numel() < n:
            ws = torch.empty(n, dtype=torch.uint8, device=f"cuda:{self.device}")
            self._ws[what] = ws
        return ws

    def timing(self, enable: bool):
        """Start (reset) or stop per-launch event timing of the Givens window passes."""
        _check(_tenable(self._h, int(bool(enable))))

    def timing_read(self, kind: int, spin: int):
        """-> (kernel ms, launches, algorithmic bytes, algorithmic VALU slots) of the recorded
        launches of one kind (0 = window passes, 1 = segment passes, 2 = segment passes on row planes)
        rotating one spin."""
        ms, n, b, v = ctypes.c_double(), ctypes.c_int64(), ctypes.c_double(), ctypes.c_double()
        _check(_tread(self._h, 2 * kind + spin, ctypes.byref(ms), ctypes.byref(n), ctypes.byref(b), ctypes.byref(v)))
        return ms.value, n.value, b.value, v.value

    def check_vec(self, vec: torch.Tensor):
        if vec.dtype != self.dtype:
            raise TypeError(f"state dtype {vec.dtype} does not match the plan ({self.dtype})")
        if not vec.is_cuda or (vec.device.index or 0) != self.device:
            raise ValueError("state must live on the plan's device")
        if not vec.is_contiguous():
            raise ValueError("state must be contiguous")
        if vec.numel() != self.dim_a * self.dim_b:
            raise ValueError(f"state has {vec.numel()} entries, expected {self.dim_a} x {self.dim_b}")


@lru_cache(maxsize=64)
def _plan_cached(norb, nelec, dtype, device) -> Plan:
    return Plan(norb, nelec, dtype, device)


def get_plan(norb: int, nelec, dtype=torch.complex128, device=0) -> Plan:
    return _plan_cached(int(norb), (int(nelec[0]), int(nelec[1])), dtype, int(device))


def _prepare(vec: torch.Tensor, norb, nelec, out, plan=None):
    if plan is None:
        plan = get_plan(norb, nelec, vec.dtype, vec.device.index or 0)
    plan.check_vec(vec)
    if out is None:
        out = vec.clone()
    elif out is not vec:
        plan.check_vec(out)
        out.copy_(vec)
    return plan, out


def _df_struct(ham, norb):
    h = _real(ham.h, (norb, norb))
    L = int(np.asarray(ham.J).shape[0])
    J = _real(ham.J, (L, norb, norb)) if L else np.zeros((0, norb, norb))
    U = _cplx(ham.U, (L, norb, norb)) if L else np.zeros((0, norb, norb, 2))
    keep = (h, J, U)
    s = _DFHam(norb, L, _dptr(h), _dptr(J), _dptr(U))
    return s, keep


def _lucj_struct(params, norb, n_reps):
    p = _real(params)
    if p.size != _lucj_np(norb, n_reps):
        raise ValueError(f"expected {_lucj_np(norb, n_reps)} LUCJ parameters, got {p.size}")
    return _LUCJ(norb, n_reps, _dptr(p)), p


# ---------------------------------------------------------------------------
# gates (Table 1)
# ---------------------------------------------------------------------------

def apply_orbital_rotation(vec: torch.Tensor, U, norb: int, nelec, *, U_b=None, out=None, plan=None) -> torch.Tensor:
    plan, out = _prepare(vec, norb, nelec, out, plan)
    Ua = _cplx(U, (norb, norb))
    Ub = _cplx(U_b, (norb, norb)) if U_b is not None else None
    _check(_rot(plan.handle, _vp(out.data_ptr()), _dptr(Ua), _dptr(Ub) if Ub is not None else None,
                _stream(out.device)))
    return out


def apply_orbital_rotation_dense(vec: torch.Tensor, U, norb: int, nelec, *, U_b=None, out=None,
                                 plan=None) -> torch.Tensor:
    """The orbital rotation in its dense compound-matrix form on the matrix cores (complex128, small sectors)."""
    plan, out = _prepare(vec, norb, nelec, out, plan)
    Ua = _cplx(U, (norb, norb))
    Ub = _cplx(U_b, (norb, norb)) if U_b is not None else None
    ws = plan.workspace(3)
    _check(_rot_dense(plan.handle, _vp(out.data_ptr()), _dptr(Ua), _dptr(Ub) if Ub is not None else None,
                      _vp(ws.data_ptr()), _stream(out.device)))
    return out


def apply_num_op_sum_evolution(vec: torch.Tensor, lam, time: float, norb: int, nelec, *, lam_b=None,
                               orbital_rotation=None, out=None, plan=None) -> torch.Tensor:
    """exp(-i t sum lam_p n_p) (Table 1); with orbital_rotation B, in the rotated basis."""
    plan, out = _prepare(vec, norb, nelec, out, plan)
    la = _real(lam, (norb,))
    lb = _real(lam_b, (norb,)) if lam_b is not None else None
    B = _cplx(orbital_rotation, (norb, norb)) if orbital_rotation is not None else None
    _check(_numop(plan.handle, _vp(out.data_ptr()), _dptr(la), _dptr(lb) if lb is not None else None,
                  float(time), _dptr(B) if B is not None else None, _stream(out.device)))
    return out


def apply_diag_coulomb_evolution(vec: torch.Tensor, J, time: float, norb: int, nelec, *, J_ab=None, J_bb=None,
                                 orbital_rotation=None, out=None, plan=None) -> torch.Tensor:
    """exp(-1/2 i t sum J n n) (Table 1); with orbital_rotation B, in the rotated basis."""
    plan, out = _prepare(vec, norb, nelec, out, plan)
    Jaa = _real(J, (norb, norb))
    Jab = _real(J_ab, (norb, norb)) if J_ab is not None else None
    Jbb = _real(J_bb, (norb, norb)) if J_bb is not None else None
    B = _cplx(orbital_rotation, (norb, norb)) if orbital_rotation is not None else None
    _check(_dc(plan.handle, _vp(out.data_ptr()), _dptr(Jaa), _dptr(Jab) if Jab is not None else None,
               _dptr(Jbb) if Jbb is not None else None, float(time), _dptr(B) if B is not None else None,
               _stream(out.device)))
    return out


def apply_num_interaction(vec: torch.Tensor, theta: float, p: int, spin: int, norb: int, nelec, *, out=None,
                          plan=None) -> torch.Tensor:
    """exp(i theta n_{p,spin}) (Table 1); spin 0 = alpha, 1 = beta."""
    plan, out = _prepare(vec, norb, nelec, out, plan)
    _check(_numint(plan.handle, _vp(out.data_ptr()), float(theta), int(p), int(spin), _stream(out.device)))
    return out


def apply_num_num_interaction(vec: torch.Tensor, theta: float, p: int, sigma: int, q: int, tau: int, norb: int,
                              nelec, *, out=None, plan=None) -> torch.Tensor:
    """exp(i theta n_{p,sigma} n_{q,tau}) (Table 1)."""
    plan, out = _prepare(vec, norb, nelec, out, plan)
    _check(_numnum(plan.handle, _vp(out.data_ptr()), float(theta), int(p), int(sigma), int(q), int(tau),
                   _stream(out.device)))
    return out


def apply_givens_rotation(vec: torch.Tensor, theta: float, p: int, q: int, spin: int, norb: int, nelec, *,
                          out=None, plan=None) -> torch.Tensor:
    """exp(theta (a+_{p,spin} a_{q,spin} - a+_{q,spin} a_{p,spin})) (Table 1)."""
    plan, out = _prepare(vec, norb, nelec, out, plan)
    _check(_givensg(plan.handle, _vp(out.data_ptr()), float(theta), int(p), int(q), int(spin), _stream(out.device)))
    return out


def apply_tunneling_interaction(vec: torch.Tensor, theta: float, p: int, q: int, spin: int, norb: int, nelec, *,
                                out=None, plan=None) -> torch.Tensor:
    """exp(i theta (a+_{p,spin} a_{q,spin} + h.c.)) (Table 1)."""
    plan, out = _prepare(vec, norb, nelec, out, plan)
    _check(_tunnel(plan.handle, _vp(out.data_ptr()), float(theta), int(p), int(q), int(spin), _stream(out.device)))
    return out


def apply_quad_ham_evolution(vec: torch.Tensor, M, time: float, norb: int, nelec, *, M_b=None, out=None,
                             plan=None) -> torch.Tensor:
    """exp(-i t sum M^sigma_pq a+_{p sigma} a_{q sigma}) for Hermitian M (Table 1)."""
    plan, out = _prepare(vec, norb, nelec, out, plan)
    Ma = _cplx(M, (norb, norb))
    Mb = _cplx(M_b, (norb, norb)) if M_b is not None else None
    _check(_quad(plan.handle, _vp(out.data_ptr()), _dptr(Ma), _dptr(Mb) if Mb is not None else None, float(time),
                 _stream(out.device)))
    return out


def _occ(o, n):
    if o is None:
        return None, None
    a = np.ascontiguousarray(np.asarray(o, dtype=np.int32))
    if a.shape != (n,):
        raise ValueError(f"expected {n} occupied orbitals, got shape {a.shape}")
    return a.ctypes.data_as(_c_int_p), a


def slater_determinant(norb: int, nelec, *, occ_a=None, occ_b=None, U=None, U_b=None, dtype=torch.complex128,
                       device=0, out=None, plan=None) -> torch.Tensor:
    """script-U(U)|occ> (Sec. 2.4); occ default: the lowest orbitals; U default: the identity."""
    plan = plan or get_plan(norb, nelec, dtype, device)
    if out is None:
        out = torch.empty((plan.dim_a, plan.dim_b), dtype=dtype, device=f"cuda:{device}")
    plan.check_vec(out)
    pa, ka = _occ(occ_a, int(nelec[0]))
    pb, kb = _occ(occ_b, int(nelec[1]))
    Ua = _cplx(U, (norb, norb)) if U is not None else None
    Ub = _cplx(U_b, (norb, norb)) if U_b is not None else None
    _check(_slater(plan.handle, _vp(out.data_ptr()), pa, pb, _dptr(Ua) if Ua is not None else None,
                   _dptr(Ub) if Ub is not None else None, _stream(out.device)))
    return out


def apply_ucj(norb: int, nelec, U, J, *, U_b=None, J_ab=None, J_bb=None, final=None, final_b=None,
              dtype=torch.complex128, device=0, out=None, plan=None) -> torch.Tensor:
    """[script-U(F)] prod_k script-U(U_k) D_k script-U(U_k)^dag |HF> with per-spin U and full J (Sec. 4.5.1).
    U, U_b: (n_reps, norb, norb) unitaries; J, J_ab, J_bb: (n_reps, norb, norb) real."""
    plan = plan or get_plan(norb, nelec, dtype, device)
    if out is None:
        out = torch.empty((plan.dim_a, plan.dim_b), dtype=dtype, device=f"cuda:{device}")
    plan.check_vec(out)
    R = int(np.asarray(U).shape[0])
    Ua = _cplx(U, (R, norb, norb))
    Ub = _cplx(U_b, (R, norb, norb)) if U_b is not None else None
    Ja = _real(J, (R, norb, norb))
    Jab = _real(J_ab, (R, norb, norb)) if J_ab is not None else None
    Jbb = _real(J_bb, (R, norb, norb)) if J_bb is not None else None
    Fa = _cplx(final, (norb, norb)) if final is not None else None
    Fb = _cplx(final_b, (norb, norb)) if final_b is not None else None
    opt = lambda a: _dptr(a) if a is not None else None
    _check(_ucj(plan.handle, _vp(out.data_ptr()), R, _dptr(Ua), opt(Ub), _dptr(Ja), opt(Jab), opt(Jbb), opt(Fa),
                opt(Fb), _stream(out.device)))
    return out


def sample_state(vec: torch.Tensor, u, norb: int, nelec, *, plan=None) -> np.ndarray:
    """Addresses i_a * dim_b + i_b sampled from |vec|^2 by the uniforms u in [0, 1) (Sec. 6.1)."""
    plan = plan or get_plan(norb, nelec, vec.dtype, vec.device.index or 0)
    plan.check_vec(vec)
    uu = _real(u).reshape(-1)
    out = np.zeros(uu.size, dtype=np.int64)
    _check(_sstate(plan.handle, _vp(vec.data_ptr()), _dptr(uu), uu.size,
                   out.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), _stream(vec.device)))
    return out


def sample_state_noalloc(vec: torch.Tensor, u: torch.Tensor, out: torch.Tensor, norb: int, nelec, *,
                         plan=None) -> torch.Tensor:
    """sample_state with device uniforms u (float64) and a device result tensor out (int64), through the
    library's allocation-free entry point (enqueues only; -1 marks an invalid uniform or norm)."""
    plan = plan or get_plan(norb, nelec, vec.dtype, vec.device.index or 0)
    plan.check_vec(vec)
    if u.dtype != torch.float64 or out.dtype != torch.int64 or not u.is_contiguous() or not out.is_contiguous():
        raise ValueError("u must be contiguous float64 and out contiguous int64")
    if u.device != vec.device or out.device != vec.device or out.numel() < u.numel():
        raise ValueError("u and out must be on the state's device, out at least as long as u")
    _check(_sstate_na(plan.handle, _vp(vec.data_ptr()), _vp(u.data_ptr()), u.numel(), _vp(out.data_ptr()),
                      _stream(vec.device)))
    return out


def sample_slater(norb: int, nelec, u_a, u_b, *, U=None, U_b=None, occ_a=None, occ_b=None,
                  dtype=torch.complex128, device=0, plan=None):
    """(masks_a, masks_b) sampled from the Slater determinant script-U(U)|occ> (Sec. 4.5.4); u_a: (n_samples,
    n_alpha) and u_b: (n_samples, n_beta) uniforms in [0, 1)."""
    plan = plan or get_plan(norb, nelec, dtype, device)
    na, nb = int(nelec[0]), int(nelec[1])
    ua = _real(u_a).reshape(-1)
    ub = _real(u_b).reshape(-1)
    n = ua.size // na if na else ub.size // max(nb, 1)
    if ua.size != n * na or ub.size != n * nb:
        raise ValueError("u_a and u_b must hold n_samples x n_alpha and n_samples x n_beta uniforms")
    pa, ka = _occ(occ_a, na)
    pb, kb = _occ(occ_b, nb)
    Ua = _cplx(U, (norb, norb)) if U is not None else None
    Ub = _cplx(U_b, (norb, norb)) if U_b is not None else None
    ma = np.zeros(n, dtype=np.uint64)
    mb = np.zeros(n, dtype=np.uint64)
    _check(_sslater(plan.handle, pa, pb, _dptr(Ua) if Ua is not None else None, _dptr(Ub) if Ub is not None else None,
                    _dptr(ua), _dptr(ub), n, ma.ctypes.data_as(_c_u64_p), mb.ctypes.data_as(_c_u64_p),
                    _stream(torch.device(f"cuda:{plan.device}"))))
    return ma, mb


def simulate_trotter_double_factorized(vec: torch.Tensor, ham, time: float, norb: int, nelec, *,
                                       n_steps: int = 1, order: int = 0, out=None, plan=None) -> torch.Tensor:
    """exp(-i H time) vec by n_steps steps of the order-`order` product formula (Sec. 4.5.3)."""
    plan, out = _prepare(vec, norb, nelec, out, plan)
    s, keep = _df_struct(ham, norb)
    dt = float(time) / max(n_steps, 1)
    _check(_trotter(plan.handle, _vp(out.data_ptr()), ctypes.byref(s), dt, int(n_steps), int(order),
                    _stream(out.device)))
    return out


def simulate_trotter_diag_coulomb(vec: torch.Tensor, h, J, time: float, norb: int, nelec, *, J_ab=None, J_bb=None,
                                  n_steps: int = 1, order: int = 0, out=None, plan=None) -> torch.Tensor:
    """exp(-i H time) vec for the diagonal Coulomb Hamiltonian (one-body h, two-body J^{aa} = J, J^{ab}, J^{bb};
    Eq. diagonal-coulomb-hamiltonian) by n_steps steps of the order-`order` product formula (Sec. 4.5.3)."""
    plan, out = _prepare(vec, norb, nelec, out, plan)
    hh = _real(h, (norb, norb))
    Ja = _real(J, (norb, norb))
    Jab = _real(J_ab, (norb, norb)) if J_ab is not None else None
    Jbb = _real(J_bb, (norb, norb)) if J_bb is not None else None
    dt = float(time) / max(n_steps, 1)
    _check(_trotter_dc(plan.handle, _vp(out.data_ptr()), _dptr(hh), _dptr(Ja),
                       _dptr(Jab) if Jab is not None else None, _dptr(Jbb) if Jbb is not None else None, dt,
                       int(n_steps), int(order), _stream(out.device)))
    return out


def apply_lucj(params, norb: int, nelec, n_reps: int, *, dtype=torch.complex128, device=0,
               out=None, plan=None) -> torch.Tensor:
    plan = plan or get_plan(norb, nelec, dtype, device)
    if out is None:
        out = torch.empty((plan.dim_a, plan.dim_b), dtype=dtype, device=f"cuda:{device}")
    plan.check_vec(out)
    s, keep = _lucj_struct(params, norb, n_reps)
    _check(_lucj(plan.handle, _vp(out.data_ptr()), ctypes.byref(s), _stream(out.device)))
    return out


def df_energy(vec: torch.Tensor, ham, norb: int, nelec, *, plan=None) -> float:
    plan = plan or get_plan(norb, nelec, vec.dtype, vec.device.index or 0)
    plan.check_vec(vec)
    s, keep = _df_struct(ham, norb)
    ws = plan.workspace(0)
    e = ctypes.c_double()
    _check(_energy(plan.handle, _vp(vec.data_ptr()), ctypes.byref(s), ctypes.byref(e), _vp(ws.data_ptr()),
                   _stream(vec.device)))
    return e.value


def apply_df_hamiltonian(vec: torch.Tensor, ham, norb: int, nelec, *, out=None, plan=None) -> torch.Tensor:
    """H vec for the DF Hamiltonian (Sec. 4.2); out must not be vec."""
    plan = plan or get_plan(norb, nelec, vec.dtype, vec.device.index or 0)
    plan.check_vec(vec)
    if out is None:
        out = torch.empty_like(vec)
    plan.check_vec(out)
    s, keep = _df_struct(ham, norb)
    ws = plan.workspace(0)
    _check(_hact(plan.handle, _vp(vec.data_ptr()), _vp(out.data_ptr()), ctypes.byref(s), _vp(ws.data_ptr()),
                 _stream(vec.device)))
    return out


def evolve_exact(vec: torch.Tensor, ham, time: float, norb: int, nelec, *, tol: float = 1e-12, out=None,
                 plan=None):
    """(exp(-i H time) vec, number of Hamiltonian actions) by a Chebyshev expansion (Sec. 6.2)."""
    plan, out = _prepare(vec, norb, nelec, out, plan)
    s, keep = _df_struct(ham, norb)
    ws = plan.workspace(2)
    k = ctypes.c_int()
    _check(_exact(plan.handle, _vp(out.data_ptr()), ctypes.byref(s), float(time), float(tol), _vp(ws.data_ptr()),
                  ctypes.byref(k), _stream(out.device)))
    return out, k.value


def state_distance(x: torch.Tensor, y: torch.Tensor, norb: int, nelec, *, plan=None) -> float:
    """||x - y||_2 accumulated in FP64 (the Trotter error measure of Sec. 6.2)."""
    plan = plan or get_plan(norb, nelec, x.dtype, x.device.index or 0)
    plan.check_vec(x)
    plan.check_vec(y)
    d = ctypes.c_double()
    _check(_dist(plan.handle, _vp(x.data_ptr()), _vp(y.data_ptr()), ctypes.byref(d), _stream(x.device)))
    return d.value


def lucj_energy_grad(params, ham, norb: int, nelec, n_reps: int, *, dtype=torch.complex128, device=0,
                     psi_out: torch.Tensor | None = None, plan=None):
    """(E, dE/dtheta) of the LUCJ state under the DF Hamiltonian, by the adjoint method."""
    plan = plan or get_plan(norb, nelec, dtype, device)
    s, keep = _lucj_struct(params, norb, n_reps)
    hs, hkeep = _df_struct(ham, norb)
    grad = np.zeros(keep.size)
    e = ctypes.c_double()
    ws = plan.workspace(1)
    if psi_out is not None:
        plan.check_vec(psi_out)
    _check(_egrad(plan.handle, ctypes.byref(s), ctypes.byref(hs), ctypes.byref(e), _dptr(grad),
                  _vp(psi_out.data_ptr()) if psi_out is not None else None, _vp(ws.data_ptr()),
                  _stream(torch.device(f"cuda:{device}"))))
    return e.value, grad


_chain = _sig("ffx_df_chain_energy_grad", ctypes.c_int,
               [_vp, _vp, ctypes.POINTER(_DFHam), ctypes.POINTER(_DFHam), ctypes.c_double, ctypes.c_int,
                ctypes.POINTER(ctypes.c_double), _c_double_p, _c_double_p, _c_double_p, _vp, _vp, _vp])


def df_chain_energy_grad(vec0: torch.Tensor, ham, obs, dt: float, n_steps: int, norb: int, nelec, *,
                         psi_out: torch.Tensor | None = None, plan=None):
    """(E, {'h', 'J', 'U'}) for E = Re <psi_T|H_obs|psi_T>, psi_T = S_0(dt)^n_steps vec0, by the adjoint method.

    'h' (N, N) and 'J' (L, N, N): derivatives for moving the symmetric pair (p, q), (q, p) together;
    'U' (L, 2, N, N): U_t -> U_t expm(A - A^dag), [t, 0] = d/d Re A, [t, 1] = d/d Im A.
    """
    plan = plan or get_plan(norb, nelec, vec0.dtype, vec0.device.index or 0)
    plan.check_vec(vec0)
    hs, hk = _df_struct(ham, norb)
    os_, ok = _df_struct(obs, norb)
    L = hs.n_terms
    gh = np.zeros((norb, norb))
    gJ = np.zeros((max(L, 1), norb, norb))
    gU = np.zeros((max(L, 1), 2, norb, norb))
    e = ctypes.c_double()
    ws = plan.workspace(1)
    if psi_out is not None:
        plan.check_vec(psi_out)
    _check(_chain(plan.handle, _vp(vec0.data_ptr()), ctypes.byref(hs), ctypes.byref(os_), float(dt), int(n_steps),
                  ctypes.byref(e), _dptr(gh), _dptr(gJ), _dptr(gU),
                  _vp(psi_out.data_ptr()) if psi_out is not None else None, _vp(ws.data_ptr()),
                  _stream(vec0.device)))
    return e.value, {"h": gh, "J": gJ[:L], "U": gU[:L]}


class LUCJEnergy(torch.autograd.Function):
    """E(theta) for a LUCJ ansatz under a DF Hamiltonian, differentiable in theta.

    forward(params (float64 CPU tensor), ham, norb, nelec, n_reps, dtype) -> 0-dim float64 tensor.
    When params needs a gradient, forward runs the adjoint (ffx_lucj_energy_grad) and the backward
    multiplies the gradient it returned; otherwise forward only prepares the ansatz state and takes its
    energy (ffx_apply_lucj, ffx_df_energy).
    """

    @staticmethod
    def forward(ctx, params, ham, norb, nelec, n_reps, dtype=torch.complex128, device=0):
        p = params.detach().cpu().numpy()
        if ctx.needs_input_grad[0]:
            e, g = lucj_energy_grad(p, ham, norb, nelec, n_reps, dtype=dtype, device=device)
            ctx.save_for_backward(torch.from_numpy(g).to(params.dtype))
        else:
            psi = apply_lucj(p, norb, nelec, n_reps, dtype=dtype, device=device)
            e = df_energy(psi, ham, norb, nelec)
        return params.new_tensor(e)

    @staticmethod
    def backward(ctx, g_out):
        (g,) = ctx.saved_tensors
        return g_out * g, None, None, None, None, None, None


class _DFTerms:
    """(h, J, U) of a DF Hamiltonian as host arrays."""

    def __init__(self, h, J, U):
        self.h, self.J, self.U = h, J, U


class DFChainEnergy(torch.autograd.Function):
    """E = Re <psi_T|H_obs|psi_T>, psi_T = S_0(dt)^n_steps vec0 under the DF Hamiltonian (h, J, U)
    (Sec. 4.5.3), differentiable in h, J and U by the library's adjoint method (ffx_df_chain_energy_grad:
    the costate is pulled back through every gate while psi is uncomputed; no state is stored).

    forward(h (N x N float64), J (L x N x N float64), U (L x N x N complex128 unitaries), vec0 (device
    state), obs (the fixed observable, any object with h, J, U), dt, n_steps, norb, nelec) -> 0-dim
    float64 tensor.

    Gradients, in PyTorch's conventions:
      * h and J_t enter through their symmetric parts, so the entry (p, q) off the diagonal receives half
        of the library's derivative for moving h_pq and h_qp together, a diagonal entry all of it;
      * for U the library differentiates along U_t -> U_t expm(A - A^dag) at A = 0; for the skew-Hermitian
        direction Y = U_t^dag dU_t that is dE = Re sum conj(G) Y with G = (dE/dRe A + i dE/dIm A) / 2, and
        the gradient returned is U_t G (dE = Re sum conj(grad) dU for every dU that keeps U_t unitary).
    When none of h, J, U needs a gradient, forward runs the product formula and the energy only.
    """

    @staticmethod
    def forward(ctx, h, J, U, vec0, obs, dt, n_steps, norb, nelec):
        ham = _DFTerms(h.detach().cpu().numpy(), J.detach().cpu().numpy(), U.detach().cpu().numpy())
        if any(ctx.needs_input_grad[:3]):
            e, g = df_chain_energy_grad(vec0, ham, obs, dt, n_steps, norb, nelec)
            gh = torch.from_numpy(0.5 * (g["h"] + np.diag(np.diag(g["h"]))))
            gJ = torch.from_numpy(0.5 * (g["J"] + g["J"] * np.eye(norb)))
            G = torch.from_numpy(0.5 * (g["U"][:, 0] + 1j * g["U"][:, 1]))
            gU = U.detach().cpu().to(torch.complex128) @ G
            ctx.save_for_backward(gh.to(h.dtype), gJ.to(J.dtype), gU.to(U.dtype))
        else:
            psi = simulate_trotter_double_factorized(vec0, ham, dt * n_steps, norb, nelec, n_steps=n_steps, order=0)
            e = df_energy(psi, obs, norb, nelec)
        return h.new_tensor(e)

    @staticmethod
    def backward(ctx, g_out):
        gh, gJ, gU = ctx.saved_tensors
        return g_out * gh, g_out * gJ, g_out * gU, None, None, None, None, None, None


# ---------------------------------------------------------------------------
# batched LUCJ energy + adjoint gradient (one cooperative launch by default)
# ---------------------------------------------------------------------------
_batch_create = _sig("ffx_batch_create", ctypes.c_int,
                     [ctypes.POINTER(_vp), ctypes.c_int, _c_int_p, _c_int_p, _c_int_p, ctypes.c_int, ctypes.c_int])
_batch_destroy = _sig("ffx_batch_destroy", ctypes.c_int, [_vp])
_batch_ws = _sig("ffx_batch_workspace_bytes", ctypes.c_int64, [_vp])
_batch_eg = _sig("ffx_batch_lucj_energy_grad", ctypes.c_int,
                 [_vp, ctypes.POINTER(_LUCJ), ctypes.POINTER(_DFHam), _c_double_p, _c_double_p, _vp, _vp])
_batch_tune = _sig("ffx_batch_tune", ctypes.c_int,
                   [_vp, ctypes.POINTER(_LUCJ), ctypes.POINTER(_DFHam), _vp, _vp, _c_int_p, _c_int_p])
_batch_timing = _sig("ffx_batch_timing", ctypes.c_int,
                     [_vp, _c_double_p, _c_double_p, _c_int_p])
_batch_single = _sig("ffx_batch_single_launch", ctypes.c_int, [_vp, ctypes.c_int])
_batch_queue = _sig("ffx_batch_queue", ctypes.c_int,
                    [_vp, ctypes.POINTER(_LUCJ), ctypes.POINTER(_DFHam), _vp, _vp, ctypes.c_void_p,
                     ctypes.c_int64, ctypes.POINTER(ctypes.c_int64)])
_batch_persistent = _sig("ffx_batch_persistent", ctypes.c_int, [_vp, ctypes.c_int])
_batch_info = _sig("ffx_batch_info", ctypes.c_int,
                   [_vp, _c_int_p, _c_int_p, _c_int_p, ctypes.POINTER(ctypes.c_int64)])


class Batch:
    """Many independent sectors [(norb, (n_alpha, n_beta)), ...] run together.

    lucj_energy_grad(params_list, hams, n_reps) returns (energies, grads):
    every instance's LUCJ forward pass, costate, energy and reverse sweep run
    together, one kernel launch per pass level shared by all instances.
    """

    def __init__(self, sectors, dtype=torch.complex64, device=0):
        self.sectors = [(int(n), (int(a), int(b))) for n, (a, b) in sectors]
        self.dtype = dtype
        self.device = device
        k = len(self.sectors)
        norb = (ctypes.c_int * k)(*[s[0] for s in self.sectors])
        na = (ctypes.c_int * k)(*[s[1][0] for s in self.sectors])
        nb = (ctypes.c_int * k)(*[s[1][1] for s in self.sectors])
        code = FFX_C128 if dtype == torch.complex128 else FFX_C64
        h = _vp()
        torch.cuda.init()
        _check(_batch_create(ctypes.byref(h), k, norb, na, nb, code, device))
        self._h = h
        self._ws = None

    def __del__(self):
        h = getattr(self, "_h", None)
        if h and _batch_destroy is not None:  # module globals may be gone at interpreter exit
            _batch_destroy(h)

    def workspace(self) -> torch.Tensor:
        n = int(_batch_ws(self._h))
        if self._ws is None or self._ws.numel() < n:
            self._ws = torch.empty(n, dtype=torch.uint8, device=f"cuda:{self.device}")
        return self._ws

    def _args(self, params_list, hams, n_reps):
        k = len(self.sectors)
        if len(params_list) != k or len(hams) != k:
            raise ValueError("one parameter vector and one Hamiltonian per instance")
        ops = (_LUCJ * k)()
        hs = (_DFHam * k)()
        keep = []
        for i, ((norb, _), p, ham) in enumerate(zip(self.sectors, params_list, hams)):
            s, kp = _lucj_struct(p, norb, n_reps)
            d, kh = _df_struct(ham, norb)
            ops[i] = s
            hs[i] = d
            keep += [kp, kh]
        return ops, hs, keep

    def lucj_energy_grad(self, params_list, hams, n_reps: int):
        ops, hs, keep = self._args(params_list, hams, n_reps)
        k = len(self.sectors)
        sizes = [int(_lucj_np(n, n_reps)) for n, _ in self.sectors]
        energies = np.zeros(k)
        grads = np.zeros(sum(sizes))
        ws = self.workspace()
        _check(_batch_eg(self._h, ops, hs, _dptr(energies), _dptr(grads), _vp(ws.data_ptr()),
                         _stream(ws.device)))
        out, off = [], 0
        for n in sizes:
            out.append(grads[off:off + n].copy())
            off += n
        return energies, out

    def tune(self, params_list, hams, n_reps: int):
        ops, hs, keep = self._args(params_list, hams, n_reps)
        t, r = ctypes.c_int(), ctypes.c_int()
        ws = self.workspace()
        _check(_batch_tune(self._h, ops, hs, _vp(ws.data_ptr()), _stream(ws.device), ctypes.byref(t),
                           ctypes.byref(r)))
        return t.value, r.value

    def timing(self) -> dict:
        """Device ms of the last call's launches, wall ms of the whole call, number of launches."""
        d, c, n = ctypes.c_double(), ctypes.c_double(), ctypes.c_int()
        _check(_batch_timing(self._h, ctypes.byref(d), ctypes.byref(c), ctypes.byref(n)))
        return {"device_ms": d.value, "call_ms": c.value, "launches": n.value}

    def single_launch(self, enable: bool = True):
        """Run later calls as one cooperative launch over all pass levels, or with enable=False as one
        launch per pass kind of each level (the default)."""
        _check(_batch_single(self._h, int(bool(enable))))

    def persistent(self, enable: bool = True):
        """The task-queue persistent launch (switched off: enable=True raises)."""
        _check(_batch_persistent(self._h, int(bool(enable))))

    def queue(self, params_list, hams, n_reps: int) -> np.ndarray:
        """The task queue of a call with these arguments, nothing launched: one row per pass, in task order,
        columns (level, instance, kind, tasks, dependency count, first task)."""
        ops, hs, keep = self._args(params_list, hams, n_reps)
        ws = self.workspace()
        n = ctypes.c_int64()
        _check(_batch_queue(self._h, ops, hs, _vp(ws.data_ptr()), _stream(ws.device), None, 0, ctypes.byref(n)))
        out = np.zeros((n.value, 6), dtype=np.int64)
        _check(_batch_queue(self._h, ops, hs, _vp(ws.data_ptr()), _stream(ws.device),
                            out.ctypes.data_as(ctypes.c_void_p), n.value, ctypes.byref(n)))
        return out

    def info(self) -> dict:
        t, r, b, lds = ctypes.c_int(), ctypes.c_int(), ctypes.c_int(), ctypes.c_int64()
        _check(_batch_info(self._h, ctypes.byref(t), ctypes.byref(r), ctypes.byref(b), ctypes.byref(lds)))
        return {"target_elems": t.value, "stage_rots": r.value, "blocks": b.value, "lds_bytes": lds.value}
