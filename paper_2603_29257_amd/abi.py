"""ctypes binding of librisp (argument marshalling only; every step runs in the HIP library).

The names follow the C ABI in include/risp.h. Device buffers are PyTorch tensors on the context's
device; the library orders its work on a dedicated stream that is joined with PyTorch's current
stream around each call. Importing this module fails loudly if librisp.so has not been built.
"""
from __future__ import annotations

import ctypes as C
import os
import weakref
from dataclasses import dataclass

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIBPATH = os.path.join(HERE, "librisp.so")

RISP_OK, RISP_PENDING = 0, 1
RISP_E_ARG, RISP_E_SHAPE, RISP_E_NOMEM, RISP_E_HIP, RISP_E_NOTCONV, RISP_E_STATE, RISP_E_NOTFOUND = (
    -1, -2, -3, -4, -5, -6, -7)
FP64, FP32, BF16 = 0, 1, 2
RSH_COMBINED, RSH_SPLIT = 0, 1
J_MO, J_AO_DIRECT = 0, 1
WIN_ABSOLUTE, WIN_FRONTIER = 0, 1
PRECISIONS = {"fp64": FP64, "fp32": FP32, "bf16": BF16}

EXPORTS = ("risp_last_error", "risp_ctx_create", "risp_ctx_destroy", "risp_ctx_profile", "risp_select_aux", "risp_window",
           "risp_screen", "risp_int2c", "risp_int3c", "risp_build_factors", "risp_factors_query",
           "risp_factors_free", "risp_sigma", "risp_sigma_noalloc", "risp_davidson_full", "risp_properties", "risp_spectrum", "risp_davidson", "risp_serve_config", "risp_job_footprint",
           "risp_submit", "risp_poll", "risp_serve_stats_get", "risp_device_usage")


class RispError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"librisp status {code}: {msg}")
        self.code = code


class Shell(C.Structure):
    _fields_ = [("atom", C.c_int32), ("l", C.c_int32), ("exponent", C.c_double), ("coef", C.c_double)]


class SystemC(C.Structure):
    _fields_ = [("natm", C.c_int32), ("coords", C.POINTER(C.c_double)), ("Z", C.POINTER(C.c_int32)),
                ("aux_radius", C.POINTER(C.c_double)), ("nshell", C.c_int32), ("shells", C.POINTER(Shell)),
                ("nao", C.c_int32), ("nmo", C.c_int32), ("nocc", C.c_int32),
                ("mo_coeff", C.POINTER(C.c_double)), ("mo_energy", C.POINTER(C.c_double))]


class ParamsC(C.Structure):
    _fields_ = [("c_x", C.c_double), ("beta", C.c_double), ("omega", C.c_double), ("window_ev", C.c_double),
                ("theta", C.c_double), ("schwarz_tau", C.c_double), ("rsh_mode", C.c_int32),
                ("window_mode", C.c_int32), ("precision", C.c_int32), ("h_in_aux", C.c_int32),
                ("bf16_scale", C.c_int32), ("build_chunk_kib", C.c_int32), ("j_mode", C.c_int32),
                ("full_tddft", C.c_int32), ("dense_transform", C.c_int32),
                ("bf16_coulomb_fp32", C.c_int32)]


class DavOptsC(C.Structure):
    _fields_ = [("nstates", C.c_int32), ("block", C.c_int32), ("max_space", C.c_int32), ("max_iter", C.c_int32),
                ("tol", C.c_double), ("correction_pass", C.c_int32), ("correction_steps", C.c_int32),
                ("bf16_tol", C.c_double), ("nx0", C.c_int32), ("flags", C.c_int32),
                ("x0", C.POINTER(C.c_float)), ("ncorr", C.c_int32), ("correction_ncorr", C.c_int32)]


class DavInfoC(C.Structure):
    _fields_ = [("iters", C.c_int32), ("restarts", C.c_int32), ("sigma_vectors", C.c_int32),
                ("converged", C.c_int32), ("correction_iters", C.c_int32), ("correction_vectors", C.c_int32),
                ("t_build", C.c_double), ("t_sigma", C.c_double), ("t_subspace", C.c_double),
                ("t_correct", C.c_double), ("t_sigma_correct", C.c_double), ("sigma_flops", C.c_double),
                ("sigma_flops_correct", C.c_double), ("hbm_bytes", C.c_int64), ("resid_hist", C.c_double * 256)]


class PhaseStatC(C.Structure):
    _fields_ = [("launches", C.c_int64), ("ms", C.c_double), ("flops", C.c_double), ("bytes", C.c_double)]


DAV_VERBOSE = 1  # risp_dav_opts.flags: one stderr line per Davidson iteration
DAV_SPILL = 2  # risp_dav_opts.flags: subspace vectors and products in pinned host memory
DAV_OLSEN = 4  # risp_dav_opts.flags: Olsen's correction vectors
DAV_FP32_BASIS = 8  # risp_dav_opts.flags: FP32 basis vectors in the BF16 correction pass

PHASES = ("coulomb_y", "coulomb_j", "exchange_m", "exchange_k", "other")


class FactorsDescC(C.Structure):
    _fields_ = [("nao", C.c_int32), ("nmo", C.c_int32), ("nocc", C.c_int32), ("nvir", C.c_int32),
                ("naux_j", C.c_int32), ("naux_k", C.c_int32), ("nocc_k", C.c_int32), ("nvir_k", C.c_int32),
                ("npair", C.c_int32), ("precision", C.c_int32), ("bytes", C.c_int64),
                ("t_ia", C.c_void_p), ("t_ij", C.c_void_p), ("t_ab", C.c_void_p), ("scale_ia", C.c_void_p),
                ("scale_k", C.c_void_p), ("occ_k", C.c_void_p), ("vir_k", C.c_void_p),
                ("ld_ia", C.c_int64), ("ld_ij", C.c_int32), ("ld_ab", C.c_int32), ("diag_a", C.c_void_p),
                ("t_ij_lo", C.c_void_p), ("t_ab_lo", C.c_void_p)]


class ServeOptsC(C.Structure):
    _fields_ = [("hbm_budget_bytes", C.c_int64), ("max_active", C.c_int32), ("use_graphs", C.c_int32)]


class ResultC(C.Structure):
    _fields_ = [("status", C.c_int32), ("nstates", C.c_int32), ("energies", C.POINTER(C.c_double)),
                ("vectors", C.POINTER(C.c_float)), ("info", DavInfoC), ("t_submit", C.c_double),
                ("t_admit", C.c_double), ("t_first_sigma", C.c_double), ("t_done", C.c_double),
                ("message", C.c_char * 256)]


class ServeStatsC(C.Structure):
    _fields_ = [("queued", C.c_int32), ("active", C.c_int32), ("done", C.c_int32), ("reserved", C.c_int32),
                ("budget_bytes", C.c_int64), ("used_bytes", C.c_int64), ("ticks", C.c_int64),
                ("graph_ticks", C.c_int64)]


def load_library(path: str = LIBPATH):
    if not os.path.exists(path):
        raise ImportError(f"librisp.so not built at {path}: run paper_2603_29257_amd.build.build()")
    lib = C.CDLL(path)
    vp, i32, dbl = C.c_void_p, C.c_int32, C.c_double
    P = C.POINTER
    lib.risp_last_error.restype = C.c_char_p
    sigs = {
        "risp_ctx_create": [i32, vp, P(vp)],
        "risp_ctx_destroy": [vp],
        "risp_ctx_profile": [vp, i32, i32, P(PhaseStatC)],
        "risp_select_aux": [P(SystemC), P(ParamsC), i32, P(Shell), P(i32), P(Shell), P(i32)],
        "risp_window": [vp, i32, i32, P(dbl), dbl, i32, P(i32), P(i32), P(i32), P(i32)],
        "risp_screen": [vp, P(SystemC), i32, P(Shell), dbl, i32, P(i32), P(i32)],
        "risp_int2c": [vp, P(SystemC), i32, P(Shell), dbl, P(dbl)],
        "risp_int3c": [vp, P(SystemC), i32, P(Shell), i32, i32, dbl, dbl, P(dbl)],
        "risp_build_factors": [vp, P(SystemC), P(ParamsC), P(vp)],
        "risp_factors_query": [vp, P(FactorsDescC)],
        "risp_factors_free": [vp],
        "risp_sigma": [vp, vp, i32, vp, vp, i32],
        "risp_sigma_noalloc": [vp, vp, i32, vp, vp, i32],
        "risp_davidson_full": [vp, vp, P(DavOptsC), P(dbl), P(C.c_float), P(C.c_float), P(DavInfoC)],
        "risp_sigma_full": [vp, vp, i32, vp, vp, vp, i32],
        "risp_properties": [vp, P(SystemC), P(dbl), i32, P(dbl), vp, P(dbl), P(dbl), P(dbl), P(dbl)],
        "risp_spectrum": [vp, i32, P(dbl), P(dbl), dbl, dbl, dbl, i32, P(dbl)],
        "risp_davidson": [vp, vp, P(DavOptsC), P(dbl), P(C.c_float), P(DavInfoC)],
        "risp_serve_config": [vp, P(ServeOptsC)],
        "risp_job_footprint": [P(SystemC), P(ParamsC), P(DavOptsC), P(C.c_int64)],
        "risp_submit": [vp, P(SystemC), P(ParamsC), P(DavOptsC), P(C.c_uint64)],
        "risp_poll": [vp, C.c_uint64, P(ResultC)],
        "risp_serve_stats_get": [vp, P(ServeStatsC)],
        "risp_device_usage": [P(C.c_int64), P(C.c_int64), i32],
    }
    for name, args in sigs.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = i32
    return lib


_LIB = load_library()


def _check(code):
    if code < 0:
        raise RispError(code, _LIB.risp_last_error().decode())
    return code


def _ptr(a, ctype):
    return a.ctypes.data_as(C.POINTER(ctype))


@dataclass
class Params:
    """Method parameters (risp_params)."""
    c_x: float = 0.22
    beta: float = 0.78
    omega: float = 0.2
    window_ev: float = 40.0
    theta: float = 0.2
    schwarz_tau: float = 1e-10
    rsh_mode: int = RSH_COMBINED
    window_mode: int = WIN_ABSOLUTE
    precision: int = FP32
    h_in_aux: bool = False
    bf16_scale: bool = True
    build_chunk_kib: int = 0
    j_mode: int = 0  # J_MO or J_AO_DIRECT
    full_tddft: bool = False  # also build the exchange factor over (i, a) for full TDDFT-risp
    dense_transform: bool = False  # first MO transform over dense integral slabs (validation)
    bf16_coulomb_fp32: bool = False  # BF16: Coulomb term from the FP32 copy of T_ia

    def c(self):
        return ParamsC(self.c_x, self.beta, self.omega, self.window_ev, self.theta, self.schwarz_tau,
                       self.rsh_mode, self.window_mode, self.precision, int(self.h_in_aux),
                       int(self.bf16_scale), int(self.build_chunk_kib), int(self.j_mode), int(self.full_tddft),
                       int(self.dense_transform), int(self.bf16_coulomb_fp32))


def device_usage(reset_peak=False):
    """(live, peak) device bytes held by the library's own allocations in this process; reset_peak
    first sets the high-water mark to the live value."""
    live, peak = C.c_int64(), C.c_int64()
    _check(_LIB.risp_device_usage(C.byref(live), C.byref(peak), int(bool(reset_peak))))
    return live.value, peak.value


class System:
    """risp_system marshalled from a molecule-like object (coords, Z, aux_radius, shells, nao, nocc,
    mo_coeff, mo_energy). The numpy arrays stay referenced for the lifetime of this object."""

    def __init__(self, mol):
        self.coords = np.ascontiguousarray(mol.coords, dtype=np.float64)
        self.Z = np.ascontiguousarray(mol.Z, dtype=np.int32)
        self.radius = np.ascontiguousarray(mol.aux_radius, dtype=np.float64)
        self.shells = shells_array(mol.shells)
        self.C = np.ascontiguousarray(mol.mo_coeff, dtype=np.float64)
        self.e = np.ascontiguousarray(mol.mo_energy, dtype=np.float64)
        self.nao = int(mol.nao)
        self.nmo = int(self.C.shape[1])
        self.nocc = int(mol.nocc)
        self.c = SystemC(len(self.Z), _ptr(self.coords, C.c_double), _ptr(self.Z, C.c_int32),
                         _ptr(self.radius, C.c_double), len(self.shells), self.shells, self.nao, self.nmo,
                         self.nocc, _ptr(self.C, C.c_double), _ptr(self.e, C.c_double))


def shells_array(shells):
    arr = (Shell * len(shells))()
    for k, (a, l, e, cf) in enumerate(shells):
        arr[k] = Shell(int(a), int(l), float(e), float(cf))
    return arr


def shells_list(arr, n):
    return [(arr[k].atom, arr[k].l, arr[k].exponent, arr[k].coef) for k in range(n)]


@dataclass
class DavInfo:
    iters: int
    restarts: int
    sigma_vectors: int
    converged: bool
    correction_iters: int
    correction_vectors: int
    t_build: float
    t_sigma: float
    t_subspace: float
    t_correct: float
    t_sigma_correct: float
    sigma_flops: float
    sigma_flops_correct: float
    hbm_bytes: int
    resid_hist: list


class Factors:
    def __init__(self, ctx, handle):
        self.ctx = ctx
        self.handle = handle
        ctx._factors.add(self)
        d = FactorsDescC()
        _check(_LIB.risp_factors_query(handle, C.byref(d)))
        self.desc = d
        for k, _ in FactorsDescC._fields_:
            if not k.startswith("t_") and not k.startswith("scale") and k not in ("occ_k", "vir_k"):
                setattr(self, k, getattr(d, k))

    def free(self):
        if self.handle:
            _check(_LIB.risp_factors_free(self.handle))
            self.handle = None
            self.ctx._factors.discard(self)

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass

    def tensor(self, which, padded=False):
        """Copy of a stored factor or index set as a torch tensor on the device.

        Factors are stored with rows padded to a multiple of 8 elements; the copy is returned with
        the padding removed unless `padded` is set (then the last axis has the stored length)."""
        import torch
        d = self.desc
        dt = {FP64: torch.float64, FP32: torch.float32, BF16: torch.bfloat16}[d.precision]
        shapes = {"t_ia": ((d.naux_j, d.ld_ia), dt), "t_ij": ((d.nocc_k, d.naux_k, d.ld_ij), dt),
                  "t_ab": ((d.naux_k, d.nvir_k, d.ld_ab), dt), "scale_ia": ((d.naux_j,), torch.float32),
                  "t_ij_lo": ((d.nocc_k, d.naux_k, d.ld_ij), torch.bfloat16),
                  "t_ab_lo": ((d.naux_k, d.nvir_k, d.ld_ab), torch.bfloat16),
                  "scale_k": ((d.naux_k,), torch.float32), "occ_k": ((d.nocc_k,), torch.int32),
                  "vir_k": ((d.nvir_k,), torch.int32), "diag_a": ((d.nocc, d.nvir), torch.float64)}
        shape, dtype = shapes[which]
        ptr = getattr(d, which)
        if which == "t_ia" and not ptr and d.naux_j > 0:
            raise ValueError("t_ia is not stored by factors built with the AO Coulomb route")
        out = torch.zeros(shape, dtype=dtype, device=self.ctx.device)
        if ptr and out.numel():
            nbytes = out.numel() * out.element_size()
            self.ctx.synchronize()
            _memcpy_d2d(out.data_ptr(), ptr, nbytes)
        if padded:
            return out
        if which == "t_ia":
            return out[:, :d.nocc * d.nvir].reshape(d.naux_j, d.nocc, d.nvir)
        if which in ("t_ij", "t_ij_lo"):
            return out[:, :, :d.nocc_k]
        if which in ("t_ab", "t_ab_lo"):
            return out[:, :, :d.nvir_k]
        return out


def job_footprint(sys: System, prm: Params, nstates=15, block=0, max_space=0):
    """Device bytes the admission rule reserves for a job (host-side estimate)."""
    o = DavOptsC(nstates, block, max_space, 0, 1e-5, 1, 0, 0.0, 0, 0, None)
    p = prm.c()
    out = C.c_int64()
    _check(_LIB.risp_job_footprint(C.byref(sys.c), C.byref(p), C.byref(o), C.byref(out)))
    return out.value


def _memcpy_d2d(dst, src, nbytes):
    import torch
    # a raw device-to-device copy through a tensor view of the source
    src_t = torch.cuda.ByteTensor  # noqa: F841  (keeps torch initialised)
    hip = C.CDLL("libamdhip64.so")
    hip.hipMemcpy.argtypes = [C.c_void_p, C.c_void_p, C.c_size_t, C.c_int]
    hip.hipMemcpy.restype = C.c_int
    rc = hip.hipMemcpy(C.c_void_p(dst), C.c_void_p(src), C.c_size_t(nbytes), 3)
    if rc != 0:
        raise RispError(RISP_E_HIP, f"hipMemcpy failed ({rc})")


class Context:
    """risp_ctx on one device, with its own (default-priority) stream."""

    def __init__(self, device: int = 0):
        import torch
        self.device = torch.device("cuda", device)
        self.stream = torch.cuda.Stream(device=self.device)
        h = C.c_void_p()
        self._factors = weakref.WeakSet()
        _check(_LIB.risp_ctx_create(device, C.c_void_p(self.stream.cuda_stream), C.byref(h)))
        self.handle = h

    def close(self):
        if self.handle:
            for F in list(self._factors):
                F.free()
            _check(_LIB.risp_ctx_destroy(self.handle))
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def synchronize(self):
        self.stream.synchronize()

    def profile(self, enable=True, reset=False):
        """Switch sigma phase timing; returns the counters accumulated so far as
        {arithmetic: {phase: counters}} with arithmetic "fp64", "fp32" or "bf16"."""
        arr = (PhaseStatC * (len(PHASES) * 3))()
        _check(_LIB.risp_ctx_profile(self.handle, int(enable), int(reset), arr))
        out = {}
        for prec, name_p in ((FP64, "fp64"), (FP32, "fp32"), (BF16, "bf16")):
            base = prec * len(PHASES)
            out[name_p] = {name: dict(launches=arr[base + k].launches, ms=arr[base + k].ms,
                                      flops=arr[base + k].flops, bytes=arr[base + k].bytes)
                           for k, name in enumerate(PHASES)}
        return out

    # ---- stages ----
    def select_aux(self, sys: System, prm: Params):
        cap = max(1, len(sys.Z))
        J, K = (Shell * (2 * cap))(), (Shell * (2 * cap))()
        nj, nk = C.c_int32(), C.c_int32()
        p = prm.c()
        _check(_LIB.risp_select_aux(C.byref(sys.c), C.byref(p), 2 * cap, J, C.byref(nj), K, C.byref(nk)))
        return shells_list(J, nj.value), shells_list(K, nk.value)

    def window(self, mo_energy, nocc, window_ev=40.0, mode=WIN_ABSOLUTE):
        e = np.ascontiguousarray(mo_energy, dtype=np.float64)
        nmo = len(e)
        o = np.zeros(nocc, np.int32)
        v = np.zeros(nmo - nocc, np.int32)
        no, nv = C.c_int32(), C.c_int32()
        _check(_LIB.risp_window(self.handle, nmo, nocc, _ptr(e, C.c_double), window_ev, mode,
                                _ptr(o, C.c_int32), C.byref(no), _ptr(v, C.c_int32), C.byref(nv)))
        return o[:no.value].copy(), v[:nv.value].copy()

    def screen(self, sys: System, aux, tau):
        aa = shells_array(aux)
        nsh = len(sys.shells)
        cap = nsh * (nsh + 1) // 2
        pairs = np.zeros((cap, 2), np.int32)
        n = C.c_int32()
        _check(_LIB.risp_screen(self.handle, C.byref(sys.c), len(aux), aa, tau, cap, _ptr(pairs, C.c_int32),
                                C.byref(n)))
        return pairs[:n.value].copy()

    def int2c(self, sys: System, aux, omega=0.0):
        aa = shells_array(aux)
        nf = sum(1 if s[1] == 0 else 3 for s in aux)
        out = np.zeros((nf, nf))
        _check(_LIB.risp_int2c(self.handle, C.byref(sys.c), len(aux), aa, omega, _ptr(out, C.c_double)))
        return out

    def int3c(self, sys: System, aux, begin=0, end=None, omega=0.0, tau=0.0):
        end = len(aux) if end is None else end
        aa = shells_array(aux)
        nf = sum(1 if s[1] == 0 else 3 for s in aux[begin:end])
        out = np.zeros((nf, sys.nao, sys.nao))
        _check(_LIB.risp_int3c(self.handle, C.byref(sys.c), len(aux), aa, begin, end, omega, tau,
                               _ptr(out, C.c_double)))
        return out

    # ---- the method ----
    def build_factors(self, sys: System, prm: Params) -> Factors:
        h = C.c_void_p()
        p = prm.c()
        _check(_LIB.risp_build_factors(self.handle, C.byref(sys.c), C.byref(p), C.byref(h)))
        return Factors(self, h)

    def sigma(self, F: Factors, X, out=None, noalloc=False):
        """sigma = A X for a device tensor X [m][nocc][nvir] (float64 for FP64 factors, else float32).

        noalloc: call risp_sigma_noalloc (workspaces in the library's fixed scratch array; `out`
        should then be given, so that nothing is allocated on this path either)."""
        import torch
        want = torch.float64 if F.desc.precision == FP64 else torch.float32
        if X.dtype != want or X.device != self.device or not X.is_contiguous():
            raise ValueError(f"X must be a contiguous {want} tensor on {self.device}")
        if X.dim() != 3 or X.shape[1] != F.nocc or X.shape[2] != F.nvir:
            raise ValueError("X must have shape [m, nocc, nvir]")
        if out is None:
            out = torch.empty_like(X)
        elif out.shape != X.shape or out.dtype != want or out.device != self.device or not out.is_contiguous():
            raise ValueError("out must be a contiguous tensor shaped and typed like X")
        cur = torch.cuda.current_stream(self.device)
        self.stream.wait_stream(cur)
        fn = _LIB.risp_sigma_noalloc if noalloc else _LIB.risp_sigma
        _check(fn(self.handle, F.handle, X.shape[0], C.c_void_p(X.data_ptr()),
                  C.c_void_p(out.data_ptr()), FP64 if want == torch.float64 else FP32))
        cur.wait_stream(self.stream)
        X.record_stream(self.stream)
        out.record_stream(self.stream)
        return out

    def properties(self, sys: System, energies, X, origin=(0.0, 0.0, 0.0)):
        """Transition dipoles mu, magnetic terms m [n][3], oscillator strengths f and rotatory strengths R [n]
        of states with energies [n] (Hartree) and amplitudes X: a contiguous float32 device tensor
        [n][nocc][nvir]."""
        import torch
        e = np.ascontiguousarray(energies, dtype=np.float64)
        n = len(e)
        if X.dtype != torch.float32 or X.device != self.device or not X.is_contiguous():
            raise ValueError(f"X must be a contiguous float32 tensor on {self.device}")
        if X.dim() != 3 or X.shape[0] != n:
            raise ValueError("X must have shape [n, nocc, nvir] with n = len(energies)")
        o = np.ascontiguousarray(origin, dtype=np.float64)
        mu, md, f, R = np.zeros((n, 3)), np.zeros((n, 3)), np.zeros(n), np.zeros(n)
        cur = torch.cuda.current_stream(self.device)
        self.stream.wait_stream(cur)
        _check(_LIB.risp_properties(self.handle, C.byref(sys.c), _ptr(o, C.c_double), n, _ptr(e, C.c_double),
                                    C.c_void_p(X.data_ptr()), _ptr(mu, C.c_double), _ptr(md, C.c_double),
                                    _ptr(f, C.c_double), _ptr(R, C.c_double)))
        return mu, md, f, R

    def spectrum(self, energies, strengths, hwhm, e0, de, npts):
        """Lorentzian-broadened spectrum on the grid e0 + q de, q < npts (host array)."""
        e = np.ascontiguousarray(energies, dtype=np.float64)
        st = np.ascontiguousarray(strengths, dtype=np.float64)
        if e.shape != st.shape:
            raise ValueError("energies and strengths differ in length")
        out = np.zeros(int(npts))
        _check(_LIB.risp_spectrum(self.handle, len(e), _ptr(e, C.c_double), _ptr(st, C.c_double), float(hwhm),
                                  float(e0), float(de), int(npts), _ptr(out, C.c_double)))
        return out

    # ---- serving ----
    def serve_config(self, budget_bytes=0, max_active=0, use_graphs=True):
        o = ServeOptsC(int(budget_bytes), int(max_active), int(use_graphs))
        _check(_LIB.risp_serve_config(self.handle, C.byref(o)))

    def submit(self, sys: System, prm: Params, nstates, tol=1e-5, block=0, max_space=0, max_iter=0,
               correction_pass=True, correction_steps=0, bf16_tol=0.0, ncorr=0, correction_ncorr=0, spill=False):
        o = DavOptsC(nstates, block, max_space, max_iter, tol, int(correction_pass), correction_steps, bf16_tol,
                     0, DAV_SPILL if spill else 0, None, ncorr, correction_ncorr)
        p = prm.c()
        jid = C.c_uint64()
        _check(_LIB.risp_submit(self.handle, C.byref(sys.c), C.byref(p), C.byref(o), C.byref(jid)))
        return jid.value

    def poll(self, job_id, nstates, ov=None):
        """None while pending; else a dict with the job's status, energies, vectors and timestamps."""
        e = np.zeros(nstates)
        vec = np.zeros((nstates, ov), np.float32) if ov else None
        r = ResultC()
        r.energies = _ptr(e, C.c_double)
        r.vectors = _ptr(vec, C.c_float) if vec is not None else None
        rc = _LIB.risp_poll(self.handle, C.c_uint64(job_id), C.byref(r))
        if rc == RISP_PENDING:
            return None
        _check(rc)
        info = r.info
        n = min(256, info.iters + info.correction_iters)
        return dict(status=r.status, energies=e[:r.nstates], vectors=None if vec is None else vec[:r.nstates],
                    t_submit=r.t_submit, t_admit=r.t_admit, t_first_sigma=r.t_first_sigma, t_done=r.t_done,
                    message=r.message.decode(), iters=info.iters, correction_iters=info.correction_iters,
                    converged=bool(info.converged), sigma_flops=info.sigma_flops + info.sigma_flops_correct,
                    t_build=info.t_build, resid_hist=list(info.resid_hist[:n]))

    def serve_stats(self):
        st = ServeStatsC()
        _check(_LIB.risp_serve_stats_get(self.handle, C.byref(st)))
        return {k: getattr(st, k) for k, _ in ServeStatsC._fields_ if k != "reserved"}

    def sigma_full(self, F: Factors, V):
        """(A + B) V and (A - B) V (full TDDFT-risp) for a device tensor V [m][nocc][nvir] in the factor
        precision; the factors must have been built with Params(full_tddft=True)."""
        import torch
        want = torch.float64 if F.desc.precision == FP64 else torch.float32
        if V.dtype != want or V.device != self.device or not V.is_contiguous():
            raise ValueError(f"V must be a contiguous {want} tensor on {self.device}")
        if V.dim() != 3 or V.shape[1] != F.nocc or V.shape[2] != F.nvir:
            raise ValueError("V must have shape [m, nocc, nvir]")
        P, M = torch.empty_like(V), torch.empty_like(V)
        cur = torch.cuda.current_stream(self.device)
        self.stream.wait_stream(cur)
        _check(_LIB.risp_sigma_full(self.handle, F.handle, V.shape[0], C.c_void_p(V.data_ptr()),
                                    C.c_void_p(P.data_ptr()), C.c_void_p(M.data_ptr()),
                                    FP64 if want == torch.float64 else FP32))
        cur.wait_stream(self.stream)
        return P, M

    def davidson_full(self, F: Factors, nstates, tol=1e-5, block=0, max_space=0, max_iter=0, verbose=False,
                      want_vectors=True, allow_notconv=False):
        """Full TDDFT-risp: lowest excitation energies and X + Y, X - Y [nstates][nocc*nvir] (host)."""
        ov = F.nocc * F.nvir
        e = np.zeros(nstates)
        xp = np.zeros((nstates, ov), np.float32) if want_vectors else None
        xm = np.zeros((nstates, ov), np.float32) if want_vectors else None
        o = DavOptsC(nstates, block, max_space, max_iter, tol, 0, 0, 0.0, 0, DAV_VERBOSE if verbose else 0, None, 0, 0)
        info = DavInfoC()
        import torch
        torch.cuda.current_stream(self.device).synchronize()
        rc = _LIB.risp_davidson_full(self.handle, F.handle, C.byref(o), _ptr(e, C.c_double),
                                     None if xp is None else _ptr(xp, C.c_float),
                                     None if xm is None else _ptr(xm, C.c_float), C.byref(info))
        if rc < 0 and not (allow_notconv and rc == RISP_E_NOTCONV):
            _check(rc)
        n = min(256, info.iters)
        di = DavInfo(info.iters, info.restarts, info.sigma_vectors, bool(info.converged), 0, 0, info.t_build,
                     info.t_sigma, info.t_subspace, 0.0, 0.0, info.sigma_flops, 0.0, info.hbm_bytes,
                     list(info.resid_hist[:n]))
        return e, xp, xm, di

    def davidson(self, F: Factors, nstates, tol=1e-5, block=0, max_space=0, max_iter=0, correction_pass=True,
                 x0=None, want_vectors=True, allow_notconv=False, correction_steps=0, bf16_tol=0.0, verbose=False,
                 ncorr=0, correction_ncorr=0, spill=False, olsen=False, fp32_basis=False):
        ov = F.nocc * F.nvir
        e = np.zeros(nstates)
        vec = np.zeros((nstates, ov), np.float32) if want_vectors else None
        x0a = None
        if x0 is not None:
            x0a = np.ascontiguousarray(x0, dtype=np.float32).reshape(-1, ov)
        o = DavOptsC(nstates, block, max_space, max_iter, tol, int(correction_pass), correction_steps, bf16_tol,
                     0 if x0a is None else x0a.shape[0],
                     (DAV_VERBOSE if verbose else 0) | (DAV_SPILL if spill else 0) | (DAV_OLSEN if olsen else 0)
                     | (DAV_FP32_BASIS if fp32_basis else 0),
                     None if x0a is None else _ptr(x0a, C.c_float), ncorr, correction_ncorr)
        info = DavInfoC()
        import torch
        torch.cuda.current_stream(self.device).synchronize()
        rc = _LIB.risp_davidson(self.handle, F.handle, C.byref(o), _ptr(e, C.c_double),
                                None if vec is None else _ptr(vec, C.c_float), C.byref(info))
        if rc < 0 and not (allow_notconv and rc == RISP_E_NOTCONV):
            _check(rc)
        n = min(256, info.iters + info.correction_iters)
        di = DavInfo(info.iters, info.restarts, info.sigma_vectors, bool(info.converged), info.correction_iters,
                     info.correction_vectors, info.t_build, info.t_sigma, info.t_subspace, info.t_correct,
                     info.t_sigma_correct, info.sigma_flops, info.sigma_flops_correct, info.hbm_bytes,
                     list(info.resid_hist[:n]))
        return e, vec, di
