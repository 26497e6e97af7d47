"""ctypes binding of the trap C ABI (include/trap.h).

Argument marshalling only: every step of the computation runs in the HIP
library.  Device vectors are torch tensors on a ROCm device (contiguous,
layout [z][o][n][s]); torch supplies the memory and the stream.  Loading fails
loudly when the library has not been built.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libtrap.so")

TRAP_FP64 = 0
TRAP_FP32 = 1
TRAP_PATH_AUTO, TRAP_PATH_FUSED, TRAP_PATH_CHUNKED = 0, 1, 2
TRAP_PRD_AD, TRAP_PRD_AA = 0, 1
TRAP_FORMAL_DELO_LINEAR, TRAP_FORMAL_DELOPAR, TRAP_FORMAL_BESSER = 0, 1, 2
TRAP_INTERP_SPLINE, TRAP_INTERP_WENO4 = 0, 1
STATUS = {0: "TRAP_OK", -1: "TRAP_EINVAL", -2: "TRAP_ENOMEM", -3: "TRAP_EDEVICE",
          -4: "TRAP_ENOCONV", -5: "TRAP_ESTATE", -6: "TRAP_ENAN"}

EXPORTED = ["trap_create", "trap_destroy", "trap_set_problem", "trap_precompute",
            "trap_apply_sigma", "trap_formal_solve", "trap_apply_operator", "trap_rhs",
            "trap_gmres_solve", "trap_emergent", "trap_get_info", "trap_footprint",
            "trap_profile", "trap_stage_times", "trap_set_path", "trap_set_prd_mode", "trap_gmres_begin",
            "trap_gmres_step_batch", "trap_gmres_end", "trap_precompute_preconditioner",
            "trap_apply_preconditioner", "trap_apply_preconditioner_noalloc", "trap_preconditioner_tables", "trap_set_formal_scheme",
            "trap_set_interpolation",
            "trap_formal_from_field", "trap_emergent_los", "trap_aar_solve", "trap_kernel_rows",
            "trap_faddeeva", "trap_hip_notes", "trap_last_error"]
STAGES = ["comoving", "contract_fp32", "r3", "angular", "backinterp", "formal", "kernel_rows",
          "contract_fp64"]

_dp = ctypes.POINTER(ctypes.c_double)


class AtomDesc(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int), ("lambda0_A", ctypes.c_double), ("mass_amu", ctypes.c_double),
                ("J_l", ctypes.c_double), ("J_u", ctypes.c_double), ("g_l", ctypes.c_double),
                ("g_u", ctypes.c_double), ("L_l", ctypes.c_int), ("L_u", ctypes.c_int),
                ("S", ctypes.c_double), ("fs_split_x", ctypes.c_double), ("r_E", ctypes.c_double)]


class ProblemDesc(ctypes.Structure):
    _fields_ = [("n_z", ctypes.c_int), ("n_nu", ctypes.c_int), ("n_mu", ctypes.c_int),
                ("n_chi", ctypes.c_int), ("x", _dp), ("tau_line", _dp), ("T", _dp), ("xi", _dp),
                ("a", _dp), ("eps", _dp), ("W_T", _dp), ("v", _dp), ("B", _dp),
                ("T_ref", ctypes.c_double), ("kappa_c", _dp), ("sigma_c", _dp),
                ("n_los", ctypes.c_int), ("los_mu", _dp)]


class Info(ctypes.Structure):
    _fields_ = [("n_z", ctypes.c_int), ("n_nu", ctypes.c_int), ("n_dir", ctypes.c_int),
                ("n_theta", ctypes.c_int), ("n_slots", ctypes.c_int), ("n_up", ctypes.c_int),
                ("n_lo", ctypes.c_int), ("n_trans", ctypes.c_int), ("n_unknowns", ctypes.c_size_t),
                ("bytes_kernel_fp64", ctypes.c_size_t), ("bytes_kernel_fp32", ctypes.c_size_t),
                ("bytes_device_total", ctypes.c_size_t), ("flops_contraction", ctypes.c_double),
                ("bytes_contraction_fp64", ctypes.c_double), ("bytes_contraction_fp32", ctypes.c_double),
                ("kernel_rows_mirrored", ctypes.c_longlong), ("kernel_entries", ctypes.c_longlong),
                ("band_reach", ctypes.c_int), ("flops_contraction_fp32", ctypes.c_double),
                ("kernel_entries_fp32", ctypes.c_longlong), ("band_reach_fp32", ctypes.c_int)]


class SolveOpts(ctypes.Structure):
    _fields_ = [("tol", ctypes.c_double), ("restart", ctypes.c_int), ("max_iters", ctypes.c_int),
                ("max_outer", ctypes.c_int), ("inner", ctypes.c_int), ("inner_tol", ctypes.c_double),
                ("zero_guess", ctypes.c_int), ("precond_sweeps", ctypes.c_int)]


class AarOpts(ctypes.Structure):
    _fields_ = [("tol", ctypes.c_double), ("max_iters", ctypes.c_int), ("depth", ctypes.c_int),
                ("period", ctypes.c_int), ("omega", ctypes.c_double), ("beta", ctypes.c_double),
                ("zero_guess", ctypes.c_int), ("precond_sweeps", ctypes.c_int), ("inner", ctypes.c_int),
                ("inner_tol", ctypes.c_double), ("max_outer", ctypes.c_int)]


class SolveStats(ctypes.Structure):
    _fields_ = [("outer_steps", ctypes.c_int), ("inner_iters", ctypes.c_int),
                ("applies_fp64", ctypes.c_int), ("applies_fp32", ctypes.c_int),
                ("applies_grouped", ctypes.c_int), ("applies_precond", ctypes.c_int),
                ("final_rel_res", ctypes.c_double), ("ms_total", ctypes.c_double)]


class StageStats(ctypes.Structure):
    _fields_ = [("ms", ctypes.c_double * 8), ("launches", ctypes.c_int * 8),
                ("flops_contraction", ctypes.c_double * 2), ("bytes_contraction", ctypes.c_double * 2)]


_lib = None


def load_library(path: str = LIB_PATH):
    """Load libtrap.so (built by paper_2505_20968_amd.build); raise if absent."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"HIP library not built: {path} is missing "
                           "(run `python -m paper_2505_20968_amd.build`)")
    # torch first: the HIP runtime it brings is then the one the library binds
    # to (loaded the other way round, the two runtimes see no device)
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    lib = ctypes.CDLL(path)
    vp = ctypes.c_void_p
    lib.trap_create.argtypes = [ctypes.POINTER(vp), ctypes.c_int, vp]
    lib.trap_destroy.argtypes = [vp]
    lib.trap_set_problem.argtypes = [vp, ctypes.POINTER(AtomDesc), ctypes.POINTER(ProblemDesc)]
    lib.trap_precompute.argtypes = [vp, ctypes.c_int]
    lib.trap_apply_sigma.argtypes = [vp, vp, vp, ctypes.c_int, ctypes.c_int]
    lib.trap_formal_solve.argtypes = [vp, vp, vp, ctypes.c_int, ctypes.c_int]
    lib.trap_apply_operator.argtypes = [vp, vp, vp, ctypes.c_int]
    lib.trap_rhs.argtypes = [vp, vp]
    lib.trap_gmres_solve.argtypes = [vp, ctypes.POINTER(SolveOpts), vp, ctypes.POINTER(SolveStats)]
    lib.trap_emergent.argtypes = [vp, vp, _dp]
    lib.trap_get_info.argtypes = [vp, ctypes.POINTER(Info)]
    lib.trap_footprint.argtypes = [ctypes.POINTER(AtomDesc), ctypes.POINTER(ProblemDesc), ctypes.c_int,
                                   ctypes.POINTER(ctypes.c_size_t)]
    lib.trap_profile.argtypes = [vp, ctypes.c_int]
    lib.trap_set_path.argtypes = [vp, ctypes.c_int]
    lib.trap_set_prd_mode.argtypes = [vp, ctypes.c_int]
    lib.trap_gmres_begin.argtypes = [vp, ctypes.POINTER(SolveOpts), vp]
    lib.trap_gmres_step_batch.argtypes = [ctypes.POINTER(vp), ctypes.c_int, ctypes.POINTER(ctypes.c_int)]
    lib.trap_gmres_end.argtypes = [vp, ctypes.POINTER(SolveStats)]
    lib.trap_stage_times.argtypes = [vp, ctypes.POINTER(StageStats)]
    lib.trap_precompute_preconditioner.argtypes = [vp]
    lib.trap_set_formal_scheme.argtypes = [vp, ctypes.c_int]
    lib.trap_set_interpolation.argtypes = [vp, ctypes.c_int]
    lib.trap_apply_preconditioner.argtypes = [vp, vp, vp, ctypes.c_int, ctypes.c_int]
    lib.trap_apply_preconditioner_noalloc.argtypes = [vp, vp, vp, ctypes.c_int, ctypes.c_int]
    lib.trap_preconditioner_tables.argtypes = [vp, _dp, _dp, _dp]
    lib.trap_formal_from_field.argtypes = [vp, vp, ctypes.c_int, vp]
    lib.trap_aar_solve.argtypes = [vp, ctypes.POINTER(AarOpts), vp, ctypes.POINTER(SolveStats)]
    lib.trap_emergent_los.argtypes = [vp, vp, _dp]
    lib.trap_kernel_rows.argtypes = [vp, ctypes.c_int, ctypes.c_int, ctypes.c_int, _dp, _dp, _dp]
    lib.trap_faddeeva.argtypes = [ctypes.c_int, _dp, _dp, ctypes.c_int, _dp]
    lib.trap_hip_notes.argtypes = [ctypes.POINTER(ctypes.c_longlong), ctypes.c_char_p, ctypes.c_size_t]
    lib.trap_last_error.restype = ctypes.c_char_p
    for name in EXPORTED:
        if name != "trap_last_error":
            getattr(lib, name).restype = ctypes.c_int
    _lib = lib
    return lib


class TrapError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{STATUS.get(code, code)}: {msg}")
        self.code = code


def _check(code: int):
    if code != 0:
        raise TrapError(code, _lib.trap_last_error().decode(errors="replace"))


def _atom_desc(atom) -> AtomDesc:
    return AtomDesc(kind=0 if atom.kind == "two_level" else 1, lambda0_A=atom.lambda0_A,
                    mass_amu=atom.mass_amu, J_l=atom.J_l, J_u=atom.J_u, g_l=atom.g_l, g_u=atom.g_u,
                    L_l=int(atom.L_l), L_u=int(atom.L_u), S=float(atom.S),
                    fs_split_x=float(atom.fs_split_x), r_E=float(atom.r_E))


def _problem_desc(prob):
    keep = {k: np.ascontiguousarray(getattr(prob, k), dtype=np.float64)
            for k in ("x", "tau_line", "T", "xi", "a", "eps", "W_T", "v", "B")}
    for k in ("kappa_c", "sigma_c"):
        v = getattr(prob, k, None)
        if v is not None:
            v = np.ascontiguousarray(v, dtype=np.float64)
            if v.shape != (prob.n_z, prob.n_nu):
                raise ValueError(f"{k} must have shape (n_z, n_nu)")
            keep[k] = v
    los = getattr(prob, "los_mu", None)
    if los is not None:
        keep["los_mu"] = np.ascontiguousarray(np.ravel(los), dtype=np.float64)
    ptr = {k: v.ctypes.data_as(_dp) for k, v in keep.items()}
    d = ProblemDesc(n_z=prob.n_z, n_nu=prob.n_nu, n_mu=prob.n_mu, n_chi=prob.n_chi,
                    T_ref=float(prob.T_ref), n_los=0 if los is None else int(keep["los_mu"].size), **ptr)
    return d, keep


def footprint(prob, store_mask: int = 3) -> int:
    lib = load_library()
    d, keep = _problem_desc(prob)
    out = ctypes.c_size_t(0)
    _check(lib.trap_footprint(ctypes.byref(_atom_desc(prob.atom)), ctypes.byref(d), store_mask,
                              ctypes.byref(out)))
    return int(out.value)


def hip_notes():
    """(count, latest record) of the HIP failures the library recorded outside
    a call's own return (teardown calls, errors pending at an entry point)."""
    lib = load_library()
    n = ctypes.c_longlong()
    buf = ctypes.create_string_buffer(512)
    _check(lib.trap_hip_notes(ctypes.byref(n), buf, 512))
    return n.value, buf.value.decode(errors="replace")


def faddeeva(v, a, device: int = 0) -> np.ndarray:
    """The library's device Faddeeva function W(a, v) = w(v + i a) at the points (v, a)."""
    lib = load_library()
    v = np.ascontiguousarray(np.broadcast_arrays(np.asarray(v, float), np.asarray(a, float))[0], dtype=float)
    a = np.ascontiguousarray(np.broadcast_to(np.asarray(a, float), v.shape), dtype=float)
    out = np.zeros(v.shape + (2,))
    _check(lib.trap_faddeeva(int(device), v.ravel().ctypes.data_as(_dp), a.ravel().ctypes.data_as(_dp),
                             int(v.size), out.ctypes.data_as(_dp)))
    return out[..., 0] + 1j * out[..., 1]


def gmres_step_batch(contexts) -> list:
    """Advance every context's solve by one step (trap_gmres_step_batch);
    returns per context 1 while running, else its final status."""
    lib = load_library()
    n = len(contexts)
    arr = (ctypes.c_void_p * n)(*[c.h.value for c in contexts])
    st = (ctypes.c_int * n)()
    _check(lib.trap_gmres_step_batch(arr, n, st))
    return list(st)


def _prec_of(t) -> int:
    import torch
    if t.dtype == torch.float64:
        return TRAP_FP64
    if t.dtype == torch.float32:
        return TRAP_FP32
    raise TypeError(f"unsupported dtype {t.dtype}")


class Context:
    """One problem on one device; wraps trap_ctx."""

    def __init__(self, device: int = 0, stream=None):
        import torch
        self.lib = load_library()
        self.device = device
        if stream is None:
            stream = torch.cuda.current_stream(device)
        self.stream = stream
        h = ctypes.c_void_p()
        _check(self.lib.trap_create(ctypes.byref(h), device, ctypes.c_void_p(stream.cuda_stream)))
        self.h = h
        self.prob = None
        self.shape = None

    def close(self):
        if self.h is not None and self.h.value:
            self.lib.trap_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _vec(self, t, prec=None):
        if not t.is_cuda or not t.is_contiguous():
            raise ValueError("vectors must be contiguous device tensors")
        if tuple(t.shape) != self.shape:
            raise ValueError(f"vector shape {tuple(t.shape)} != {self.shape}")
        if prec is not None and _prec_of(t) != prec:
            raise TypeError("precision mismatch")
        return ctypes.c_void_p(t.data_ptr())

    def set_problem(self, prob):
        d, keep = _problem_desc(prob)
        _check(self.lib.trap_set_problem(self.h, ctypes.byref(_atom_desc(prob.atom)), ctypes.byref(d)))
        self.prob = prob
        n_los = 0 if getattr(prob, "los_mu", None) is None else int(np.size(prob.los_mu))
        self.n_dir_grid = prob.n_mu * prob.n_chi
        self.n_los = n_los
        self.shape = (prob.n_z, (prob.n_mu + n_los) * prob.n_chi, prob.n_nu, 4)

    def precompute(self, store_mask: int = 3):
        _check(self.lib.trap_precompute(self.h, store_mask))

    def set_formal_scheme(self, scheme: int):
        """TRAP_FORMAL_DELO_LINEAR (0), TRAP_FORMAL_DELOPAR (1) or TRAP_FORMAL_BESSER (2),
        before precompute."""
        _check(self.lib.trap_set_formal_scheme(self.h, int(scheme)))

    def set_interpolation(self, mode: int):
        """TRAP_INTERP_SPLINE (0) or TRAP_INTERP_WENO4 (1) for the observer/comoving
        frequency transforms, before precompute."""
        _check(self.lib.trap_set_interpolation(self.h, int(mode)))

    def precompute_preconditioner(self):
        _check(self.lib.trap_precompute_preconditioner(self.h))

    def apply_preconditioner(self, r, out, sweeps: int, prec: int = TRAP_FP64):
        _check(self.lib.trap_apply_preconditioner(self.h, self._vec(r, TRAP_FP64), self._vec(out, TRAP_FP64),
                                                  int(sweeps), int(prec)))

    def apply_preconditioner_noalloc(self, r, out, sweeps: int, prec: int = TRAP_FP64):
        """apply_preconditioner with the library's fixed device scratch (no allocation)."""
        _check(self.lib.trap_apply_preconditioner_noalloc(self.h, self._vec(r, TRAP_FP64),
                                                          self._vec(out, TRAP_FP64), int(sweeps), int(prec)))

    def preconditioner_tables(self) -> dict:
        nz, nd, nn = self.shape[0], self.shape[1], self.shape[2]
        phi = np.zeros((nz, nn, nn))
        c = np.zeros((nz, nn, nn))
        lloc = np.zeros((nz, nd, nn))
        _check(self.lib.trap_preconditioner_tables(self.h, phi.ctypes.data_as(_dp), c.ctypes.data_as(_dp),
                                                   lloc.ctypes.data_as(_dp)))
        return {"Phi": phi, "C": c, "L": lloc}

    def apply_sigma(self, I, eps, add_thermal: bool = False):
        p = _prec_of(I)
        _check(self.lib.trap_apply_sigma(self.h, self._vec(I, p), self._vec(eps, p), p, int(add_thermal)))

    def formal_solve(self, eps, I, with_boundary: bool = True):
        p = _prec_of(I)
        _check(self.lib.trap_formal_solve(self.h, self._vec(eps, p), self._vec(I, p), int(with_boundary), p))

    def apply_operator(self, x, y):
        p = _prec_of(x)
        _check(self.lib.trap_apply_operator(self.h, self._vec(x, p), self._vec(y, p), p))

    def rhs(self, b):
        _check(self.lib.trap_rhs(self.h, self._vec(b, TRAP_FP64)))

    def gmres_solve(self, I, tol: float = 1e-8, restart: int = 40, max_iters: int = 2000,
                    inner: int = TRAP_FP64, max_outer: int = 8, inner_tol: float = 1e-7,
                    raise_on_noconv: bool = True, zero_guess: bool = False, precond_sweeps: int = 0):
        o = SolveOpts(tol=tol, restart=restart, max_iters=max_iters, max_outer=max_outer, inner=inner,
                      inner_tol=inner_tol, zero_guess=int(zero_guess), precond_sweeps=int(precond_sweeps))
        st = SolveStats()
        code = self.lib.trap_gmres_solve(self.h, ctypes.byref(o), self._vec(I, TRAP_FP64), ctypes.byref(st))
        if code != 0 and (raise_on_noconv or code != -4):
            _check(code)
        return {"outer_steps": st.outer_steps, "inner_iters": st.inner_iters,
                "applies_fp64": st.applies_fp64, "applies_fp32": st.applies_fp32, "applies_grouped": st.applies_grouped,
                "applies_precond": st.applies_precond,
                "final_rel_res": st.final_rel_res, "ms_total": st.ms_total, "status": code}

    def aar_solve(self, I, tol: float = 1e-8, max_iters: int = 2000, depth: int = 7, period: int = 6,
                  omega: float = 1.0, beta: float = 1.0, zero_guess: bool = False, precond_sweeps: int = 0,
                  inner: int = TRAP_FP64, inner_tol: float = 1e-4, max_outer: int = 10,
                  raise_on_noconv: bool = True):
        """Alternating Anderson-Richardson solve (trap_aar_solve): FP64, or with
        inner=TRAP_FP32 FP64 defect correction around FP32 inner iterations."""
        o = AarOpts(tol=tol, max_iters=max_iters, depth=depth, period=period, omega=omega, beta=beta,
                    zero_guess=int(zero_guess), precond_sweeps=int(precond_sweeps), inner=int(inner),
                    inner_tol=float(inner_tol), max_outer=int(max_outer))
        st = SolveStats()
        code = self.lib.trap_aar_solve(self.h, ctypes.byref(o), self._vec(I, TRAP_FP64), ctypes.byref(st))
        if code != 0 and (raise_on_noconv or code != -4):
            _check(code)
        return {"anderson_steps": st.outer_steps, "residuals": st.inner_iters, "applies_fp64": st.applies_fp64,
                "applies_fp32": st.applies_fp32, "applies_precond": st.applies_precond, "final_rel_res": st.final_rel_res, "ms_total": st.ms_total,
                "status": code}

    def gmres_begin(self, I, tol: float = 1e-8, restart: int = 40, max_iters: int = 2000,
                    inner: int = TRAP_FP64, max_outer: int = 8, inner_tol: float = 1e-7,
                    zero_guess: bool = False, precond_sweeps: int = 0):
        """Start a solve that trap_gmres_step_batch advances (see gmres_step_batch)."""
        o = SolveOpts(tol=tol, restart=restart, max_iters=max_iters, max_outer=max_outer, inner=inner,
                      inner_tol=inner_tol, zero_guess=int(zero_guess), precond_sweeps=int(precond_sweeps))
        self._solution = I           # the library writes into I until the solve ends
        _check(self.lib.trap_gmres_begin(self.h, ctypes.byref(o), self._vec(I, TRAP_FP64)))

    def gmres_end(self, raise_on_noconv: bool = True) -> dict:
        st = SolveStats()
        code = self.lib.trap_gmres_end(self.h, ctypes.byref(st))
        if code != 0 and (raise_on_noconv or code != -4):
            _check(code)
        self._solution = None
        return {"outer_steps": st.outer_steps, "inner_iters": st.inner_iters,
                "applies_fp64": st.applies_fp64, "applies_fp32": st.applies_fp32, "applies_grouped": st.applies_grouped,
                "applies_precond": st.applies_precond,
                "final_rel_res": st.final_rel_res, "ms_total": st.ms_total, "status": code}

    def emergent(self, I) -> np.ndarray:
        n_up = self.n_dir_grid // 2
        out = np.zeros((n_up, self.shape[2], 4))
        _check(self.lib.trap_emergent(self.h, self._vec(I, TRAP_FP64), out.ctypes.data_as(_dp)))
        return out

    def formal_from_field(self, I, out):
        """out = Lambda (Sigma I + eps_th) + t (FP64, trap_formal_from_field).  I has
        either every direction of this context or only its quadrature directions."""
        if _prec_of(I) != TRAP_FP64 or not I.is_contiguous() or I.dim() != 4:
            raise TypeError("I must be a contiguous FP64 [z][dir][n][4] tensor")
        if I.shape[1] not in (self.shape[1], self.n_dir_grid) or (I.shape[0], I.shape[2]) != (
                self.shape[0], self.shape[2]):
            raise ValueError(f"I shape {tuple(I.shape)} does not fit {self.shape}")
        _check(self.lib.trap_formal_from_field(self.h, ctypes.c_void_p(I.data_ptr()), int(I.shape[1]),
                                               self._vec(out, TRAP_FP64)))

    def emergent_los(self, I) -> np.ndarray:
        """Emergent Stokes vectors along the lines of sight, [los][chi][n][4]."""
        out = np.zeros((self.n_los, self.prob.n_chi, self.shape[2], 4))
        _check(self.lib.trap_emergent_los(self.h, self._vec(I, TRAP_FP64), out.ctypes.data_as(_dp)))
        return out

    def set_prd_mode(self, mode: int):
        """TRAP_PRD_AD or TRAP_PRD_AA; takes effect at the next set_problem."""
        _check(self.lib.trap_set_prd_mode(self.h, int(mode)))

    def set_path(self, path: int):
        """Sigma implementation: TRAP_PATH_AUTO, TRAP_PATH_FUSED or TRAP_PATH_CHUNKED."""
        _check(self.lib.trap_set_path(self.h, int(path)))

    def profile(self, enable: bool = True):
        _check(self.lib.trap_profile(self.h, int(enable)))

    def stage_times(self) -> dict:
        st = StageStats()
        _check(self.lib.trap_stage_times(self.h, ctypes.byref(st)))
        out = {name: {"ms": st.ms[i], "launches": st.launches[i]} for i, name in enumerate(STAGES)}
        out["flops_contraction"] = {"fp32": st.flops_contraction[0], "fp64": st.flops_contraction[1]}
        out["bytes_contraction"] = {"fp32": st.bytes_contraction[0], "fp64": st.bytes_contraction[1]}
        return out

    def kernel_rows(self, z: int, theta: int, t: int):
        """FP64 kernel M[z][theta][t] as a dense complex [n_nu][n_nu] array, with
        its scattering angle and the transition's reduced shift."""
        nn = self.shape[2]
        out = np.zeros((2, nn, nn))
        th = ctypes.c_double()
        sh = ctypes.c_double()
        _check(self.lib.trap_kernel_rows(self.h, int(z), int(theta), int(t), ctypes.byref(th), ctypes.byref(sh),
                                         out.ctypes.data_as(_dp)))
        return out[0] + 1j * out[1], th.value, sh.value

    def info(self) -> dict:
        i = Info()
        _check(self.lib.trap_get_info(self.h, ctypes.byref(i)))
        return {f: getattr(i, f) for f, _ in Info._fields_}
