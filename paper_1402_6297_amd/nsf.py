"""Python binding of libnsf (include/nsf.h): argument marshalling only.

Each ``nsf_*`` function here calls the C function of the same name.  Device
buffers are torch tensors on a HIP device (complex128 / float64, contiguous);
host buffers are numpy arrays.  A nonzero error status raises ``NsfError``
(``NSF_NOT_CONVERGED`` is returned, not raised, by the solvers).  Nothing here
computes any part of the method: if libnsf.so is missing the first call
raises.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# NSF_LIB names another build of the same library (for A/B timing of builds)
LIB_PATH = os.environ.get("NSF_LIB") or os.path.join(_HERE, "libnsf.so")

NSF_OK = 0
NSF_NOT_CONVERGED = 1
NSF_E_ARG = -1
NSF_E_KPOINT = -2
NSF_E_BASIS = -3
NSF_E_NOT_HHPD = -4
NSF_E_BREAKDOWN = -5
NSF_E_NOMEM = -6
NSF_E_HIP = -7
NSF_E_STATE = -8

NSF_MEDIUM_NONE, NSF_MEDIUM_CHIRAL, NSF_MEDIUM_PSEUDOCHIRAL, NSF_MEDIUM_GENERAL = 0, 1, 2, 3
NSF_MEDIUM_NFSEP = 4

NSF_OPT_FFT_PATH = 1
NSF_OPT_MID_COLS = 2
NSF_OPT_CG_GRAPH = 3
NSF_OPT_X_ROWS = 4
NSF_OPT_YZ_COLS = 5
NSF_OPT_MID_PAIRS = 6
NSF_OPT_CG_START = 7
NSF_OPT_VERIFY = 8
NSF_OPT_ORTHO_GATE = 9
NSF_OPT_GMRES_RESTART = 10
NSF_OPT_MEDIUM_PALETTE = 11
NSF_OPT_CG_RELAX = 12
NSF_OPT_WARM_CHAIN = 13
NSF_OPT_CG_RING = 14
NSF_OPT_VACUUM = 15

EXPORTED = [
    "nsf_plan_create", "nsf_plan_destroy", "nsf_plan_query", "nsf_plan_set_option",
    "nsf_set_medium_chiral", "nsf_set_medium_pseudochiral", "nsf_set_medium_tensor",
    "nsf_apply_Pr", "nsf_apply_Qr", "nsf_apply_PrH", "nsf_apply_QrH",
    "nsf_apply_Ar", "nsf_apply_Br", "nsf_profile_Ar", "nsf_cg_solve", "nsf_eigs", "nsf_eig_grad",
    "nsf_hermitian_eig", "nsf_device_info", "nsf_status_string", "nsf_last_error",
    "nsf_batch_create", "nsf_batch_plan", "nsf_batch_eigs", "nsf_batch_destroy",
    "nsf_plan_autotune", "nsf_batch_autotune", "nsf_plan_workspace_size", "nsf_plan_set_workspace",
    "nsf_fields", "nsf_eigs_set_start", "nsf_schur_sorted", "nsf_set_medium_nfsep", "nsf_apply_nfsep",
    "nsf_nfsep_solve", "nsf_eigs_nfsep", "nsf_plan_medium_info", "nsf_cg_solve_noalloc",
]


class nsf_stats(C.Structure):
    _fields_ = [("matvecs", C.c_longlong), ("cg_iters_total", C.c_longlong),
                ("cg_solves", C.c_int), ("lanczos_steps", C.c_int), ("restarts", C.c_int),
                ("converged", C.c_int), ("ortho_passes", C.c_int), ("cg_iters_avg", C.c_double),
                ("ms_total", C.c_double),
                ("bytes_alg", C.c_double), ("ms_cg", C.c_double), ("ms_orth", C.c_double),
                ("ms_restart", C.c_double)]

    def as_dict(self):
        return {name: getattr(self, name) for name, _ in self._fields_}


class nsf_tune(C.Structure):
    _fields_ = [("fft_path", C.c_int), ("mid_cols", C.c_int), ("x_rows", C.c_int), ("yz_cols", C.c_int),
                ("mid_pairs", C.c_int), ("us_best", C.c_double), ("us_default", C.c_double), ("tried", C.c_int)]

    def as_dict(self):
        return {name: getattr(self, name) for name, _ in self._fields_}


class nsf_device(C.Structure):
    _fields_ = [("name", C.c_char * 64), ("compute_units", C.c_int), ("clock_khz", C.c_int),
                ("memory_clock_khz", C.c_int), ("memory_bus_bits", C.c_int),
                ("total_memory", C.c_longlong), ("l2_bytes", C.c_longlong),
                ("lds_per_block", C.c_int), ("lds_per_cu", C.c_int), ("warp_size", C.c_int)]

    def as_dict(self):
        d = {name: getattr(self, name) for name, _ in self._fields_}
        d["name"] = d["name"].decode()
        return d


class NsfError(RuntimeError):
    def __init__(self, status, message):
        super().__init__(f"[{status}] {message}")
        self.status = status


_lib = None


def lib():
    """Load libnsf.so (built in-tree); raise if it is missing."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is not built: run `python -m paper_1402_6297_amd.build`")
    L = C.CDLL(LIB_PATH)
    P, I, D, VP = C.c_void_p, C.c_int, C.c_double, C.c_void_p
    DP = C.POINTER(C.c_double)
    sig = {
        "nsf_plan_create": (I, [C.POINTER(P), I, I, I, D, DP, D, D, VP]),
        "nsf_plan_destroy": (None, [P]),
        "nsf_plan_set_option": (I, [P, I, I]),
        "nsf_plan_query": (I, [P, C.POINTER(C.c_longlong), C.POINTER(I), DP, DP]),
        "nsf_set_medium_chiral": (I, [P, VP, VP, I]),
        "nsf_set_medium_pseudochiral": (I, [P, I, I, VP, VP, I]),
        "nsf_set_medium_tensor": (I, [P, VP, VP, VP, VP, I]),
        "nsf_apply_Pr": (I, [P, VP, VP]),
        "nsf_apply_Qr": (I, [P, VP, VP]),
        "nsf_apply_PrH": (I, [P, VP, VP]),
        "nsf_apply_QrH": (I, [P, VP, VP]),
        "nsf_apply_Ar": (I, [P, VP, VP]),
        "nsf_apply_Br": (I, [P, VP, VP]),
        "nsf_profile_Ar": (I, [P, VP, VP, I, DP, I, C.POINTER(I), DP]),
        "nsf_cg_solve": (I, [P, VP, VP, D, I, C.POINTER(I), DP]),
        "nsf_cg_solve_noalloc": (I, [P, VP, VP, D, I, C.POINTER(I), DP]),
        "nsf_eigs": (I, [P, I, D, D, I, I, C.c_ulonglong, DP, VP, DP, C.POINTER(nsf_stats)]),
        "nsf_eig_grad": (I, [P, I, DP, VP, DP, VP, VP]),
        "nsf_hermitian_eig": (I, [I, VP, DP, VP]),
        "nsf_schur_sorted": (I, [I, VP, VP, VP]),
        "nsf_plan_medium_info": (I, [P, C.POINTER(I), C.POINTER(C.c_longlong)]),
        "nsf_set_medium_nfsep": (I, [P, VP, VP, VP, VP, I]),
        "nsf_apply_nfsep": (I, [P, VP, VP]),
        "nsf_nfsep_solve": (I, [P, VP, VP, D, I, I, C.POINTER(I), DP]),
        "nsf_eigs_nfsep": (I, [P, I, D, D, I, I, C.c_ulonglong, VP, VP, DP, C.POINTER(nsf_stats)]),
        "nsf_device_info": (I, [I, C.POINTER(nsf_device)]),
        "nsf_batch_create": (I, [C.POINTER(P), I, VP, VP, D, D, D, VP]),
        "nsf_batch_plan": (I, [P, I, C.POINTER(P)]),
        "nsf_batch_eigs": (I, [P, I, D, D, I, I, C.c_ulonglong, DP, DP, C.POINTER(nsf_stats),
                               C.POINTER(C.c_void_p), C.POINTER(I)]),
        "nsf_batch_destroy": (None, [P]),
        "nsf_plan_autotune": (I, [P, I, C.POINTER(nsf_tune)]),
        "nsf_plan_workspace_size": (I, [P, I, I, C.POINTER(C.c_size_t)]),
        "nsf_fields": (I, [P, VP, VP]),
        "nsf_eigs_set_start": (I, [P, VP, I]),
        "nsf_plan_set_workspace": (I, [P, VP, C.c_size_t]),
        "nsf_batch_autotune": (I, [P, I, C.POINTER(I)]),
        "nsf_status_string": (C.c_char_p, [I]),
        "nsf_last_error": (C.c_char_p, [P]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(L, name)
        fn.restype = res
        fn.argtypes = args
    _lib = L
    return L


def _check(status, plan=None):
    if status < 0:
        msg = lib().nsf_last_error(plan)
        raise NsfError(status, (msg or b"").decode() or lib().nsf_status_string(status).decode())
    return status


def _dptr(t, dtype_name, need=None):
    """Device pointer of a contiguous torch tensor of the given dtype holding at
    least ``need`` elements (the library reads or writes that many)."""
    import torch

    want = {"c128": torch.complex128, "f64": torch.float64}[dtype_name]
    if not isinstance(t, torch.Tensor) or t.dtype != want or not t.is_cuda or not t.is_contiguous():
        raise TypeError(f"expected a contiguous {want} tensor on a HIP device")
    if need is not None and t.numel() < need:
        raise ValueError(f"tensor holds {t.numel()} elements, the call needs {need}")
    return C.c_void_p(t.data_ptr())


def _plan_n(plan):
    """Voxel count n of a plan (host query)."""
    n = C.c_longlong()
    _check(lib().nsf_plan_query(plan, C.byref(n), None, None, None), plan)
    return n.value


def _host_exact(a, count, what):
    if a.size != count:
        raise ValueError(f"{what}: {a.size} values, the plan's grid needs {count}")


def _hptr(a, dtype=np.float64):
    a = np.ascontiguousarray(a, dtype=dtype)
    return a, C.c_void_p(a.ctypes.data)


def current_stream():
    """hipStream_t of torch's current stream (0 if no device is visible)."""
    import torch

    if not torch.cuda.is_available():
        return 0
    return torch.cuda.current_stream().cuda_stream


# --------------------------------------------------------------------- calls

def nsf_plan_create(n1, n2, n3, a, k, alpha=-1.0, beta=2.0, stream=None):
    plan = C.c_void_p()
    kk = (C.c_double * 3)(*[float(x) for x in k])
    s = current_stream() if stream is None else stream
    _check(lib().nsf_plan_create(C.byref(plan), int(n1), int(n2), int(n3), float(a), kk,
                                 float(alpha), float(beta), C.c_void_p(s)))
    return plan


def nsf_plan_destroy(plan):
    lib().nsf_plan_destroy(plan)


def nsf_plan_set_option(plan, option, value):
    return _check(lib().nsf_plan_set_option(plan, int(option), int(value)), plan)


def nsf_plan_query(plan):
    n, kind = C.c_longlong(), C.c_int()
    smin, smax = C.c_double(), C.c_double()
    _check(lib().nsf_plan_query(plan, C.byref(n), C.byref(kind), C.byref(smin), C.byref(smax)), plan)
    return dict(n=n.value, medium_kind=kind.value, sigma_min=smin.value, sigma_max=smax.value)


def _medium_ptrs(plan, eps, gamma):
    n = _plan_n(plan)
    try:
        import torch
        if isinstance(eps, torch.Tensor):
            for t, what in ((eps, "eps"), (gamma, "gamma")):
                if isinstance(t, torch.Tensor) and t.numel() != n:
                    raise ValueError(f"{what}: {t.numel()} values, the plan's grid needs {n}")
            return (eps, gamma), _dptr(eps, "f64", n), _dptr(gamma, "f64", n), 1
    except ImportError:  # pragma: no cover
        pass
    e, pe = _hptr(np.ravel(eps))
    g, pg = _hptr(np.ravel(gamma))
    _host_exact(e, n, "eps")
    _host_exact(g, n, "gamma")
    return (e, g), pe, pg, 0


def nsf_set_medium_chiral(plan, eps, gamma):
    keep, pe, pg, on_dev = _medium_ptrs(plan, eps, gamma)
    return _check(lib().nsf_set_medium_chiral(plan, pe, pg, on_dev), plan)


def nsf_set_medium_pseudochiral(plan, axis_a, axis_b, eps, gamma):
    keep, pe, pg, on_dev = _medium_ptrs(plan, eps, gamma)
    return _check(lib().nsf_set_medium_pseudochiral(plan, int(axis_a), int(axis_b), pe, pg, on_dev), plan)


def _set_tensors(name, plan, eps, mu, xi, zeta):
    fields = [eps, mu, xi, zeta]
    n = _plan_n(plan)
    try:
        import torch
        if isinstance(eps, torch.Tensor):
            for t, what in zip(fields, ("eps", "mu", "xi", "zeta")):
                if isinstance(t, torch.Tensor) and t.numel() != 9 * n:
                    raise ValueError(f"{what}: {t.numel()} values, the plan's grid needs 9 x {n}")
            ptrs = [_dptr(t, "c128", 9 * n) for t in fields]
            return _check(getattr(lib(), name)(plan, *ptrs, 1), plan)
    except ImportError:  # pragma: no cover
        pass
    keep = [np.ascontiguousarray(np.reshape(f, (-1, 3, 3)), dtype=np.complex128) for f in fields]
    for k, what in zip(keep, ("eps", "mu", "xi", "zeta")):
        _host_exact(k, 9 * n, what)
    return _check(getattr(lib(), name)(plan, *[C.c_void_p(k.ctypes.data) for k in keep], 0), plan)


def nsf_set_medium_tensor(plan, eps, mu, xi, zeta):
    """General medium: four (n, 3, 3) complex128 tensor fields (numpy on the host, or
    contiguous torch tensors on the device), voxel order g = i1 + n1 i2 + n1 n2 i3."""
    return _set_tensors("nsf_set_medium_tensor", plan, eps, mu, xi, zeta)


def nsf_set_medium_nfsep(plan, eps, mu, xi, zeta):
    """NFSEP medium (any nonsingular B): tensors laid out as for nsf_set_medium_tensor."""
    return _set_tensors("nsf_set_medium_nfsep", plan, eps, mu, xi, zeta)


def _apply(name, plan, src, dst, src_per_n=4, dst_per_n=4):
    n = _plan_n(plan)
    return _check(getattr(lib(), name)(plan, _dptr(src, "c128", src_per_n * n),
                                       _dptr(dst, "c128", dst_per_n * n)), plan)


def nsf_fields(plan, y4n, eh6n):
    return _apply("nsf_fields", plan, y4n, eh6n, 4, 6)


def nsf_apply_Pr(plan, y2n, x3n):
    return _apply("nsf_apply_Pr", plan, y2n, x3n, 2, 3)


def nsf_apply_Qr(plan, y2n, x3n):
    return _apply("nsf_apply_Qr", plan, y2n, x3n, 2, 3)


def nsf_apply_PrH(plan, x3n, y2n):
    return _apply("nsf_apply_PrH", plan, x3n, y2n, 3, 2)


def nsf_apply_QrH(plan, x3n, y2n):
    return _apply("nsf_apply_QrH", plan, x3n, y2n, 3, 2)


def nsf_apply_Ar(plan, u4n, out4n):
    return _apply("nsf_apply_Ar", plan, u4n, out4n)


def nsf_apply_Br(plan, u4n, out4n):
    return _apply("nsf_apply_Br", plan, u4n, out4n)


def nsf_profile_Ar(plan, u4n, out4n, reps=20):
    """Returns (per-kernel average ms list, whole-apply average ms)."""
    ms = (C.c_double * 16)()
    npass = C.c_int()
    whole = C.c_double()
    n = _plan_n(plan)
    _check(lib().nsf_profile_Ar(plan, _dptr(u4n, "c128", 4 * n), _dptr(out4n, "c128", 4 * n), int(reps),
                                ms, 16, C.byref(npass), C.byref(whole)), plan)
    return [ms[i] for i in range(npass.value)], whole.value


def nsf_cg_solve(plan, b, x, rtol=1e-10, maxit=10000):
    it, rel = C.c_int(), C.c_double()
    n = _plan_n(plan)
    st = _check(lib().nsf_cg_solve(plan, _dptr(b, "c128", 4 * n), _dptr(x, "c128", 4 * n), float(rtol),
                                   int(maxit), C.byref(it), C.byref(rel)), plan)
    return st, it.value, rel.value


def nsf_cg_solve_noalloc(plan, b, x, rtol=1e-10, maxit=10000):
    it, rel = C.c_int(), C.c_double()
    n = _plan_n(plan)
    st = _check(lib().nsf_cg_solve_noalloc(plan, _dptr(b, "c128", 4 * n), _dptr(x, "c128", 4 * n),
                                           float(rtol), int(maxit), C.byref(it), C.byref(rel)), plan)
    return st, it.value, rel.value


def nsf_plan_medium_info(plan):
    pal, vb = C.c_int(), C.c_longlong()
    _check(lib().nsf_plan_medium_info(plan, C.byref(pal), C.byref(vb)), plan)
    return {"palette": pal.value, "voxel_bytes": vb.value}


def nsf_apply_nfsep(plan, y4n, out4n):
    return _apply("nsf_apply_nfsep", plan, y4n, out4n)


def nsf_nfsep_solve(plan, b, x, rtol=1e-10, maxit=0, restart=0):
    it, rel = C.c_int(), C.c_double()
    n = _plan_n(plan)
    st = _check(lib().nsf_nfsep_solve(plan, _dptr(b, "c128", 4 * n), _dptr(x, "c128", 4 * n), float(rtol),
                                      int(maxit), int(restart), C.byref(it), C.byref(rel)), plan)
    return st, it.value, rel.value


def nsf_eigs_nfsep(plan, nev, res_tol=1e-8, inner_rtol=1e-10, max_basis=0, max_restarts=0, seed=0, Y=None):
    """Returns (status, omega[nev] complex, resid[nev], stats dict); Y (4n x nev device) filled if given."""
    omega = np.zeros(nev, dtype=np.complex128)
    resid = np.zeros(nev)
    st = nsf_stats()
    yp = _dptr(Y, "c128", int(nev) * 4 * _plan_n(plan)) if Y is not None else None
    status = _check(lib().nsf_eigs_nfsep(plan, int(nev), float(res_tol), float(inner_rtol), int(max_basis),
                                         int(max_restarts), C.c_ulonglong(seed), C.c_void_p(omega.ctypes.data),
                                         yp, resid.ctypes.data_as(C.POINTER(C.c_double)), C.byref(st)), plan)
    return status, omega, resid, st.as_dict()


def nsf_eigs(plan, nev, res_tol=1e-8, cg_rtol=1e-10, max_basis=0, max_restarts=0, seed=0, Y=None):
    """Returns (status, omega[nev], resid[nev], stats dict); Y (4n x nev device) is filled if given."""
    omega = np.zeros(nev)
    resid = np.zeros(nev)
    st = nsf_stats()
    yp = _dptr(Y, "c128", int(nev) * 4 * _plan_n(plan)) if Y is not None else None
    status = _check(lib().nsf_eigs(plan, int(nev), float(res_tol), float(cg_rtol), int(max_basis),
                                   int(max_restarts), C.c_ulonglong(seed),
                                   omega.ctypes.data_as(C.POINTER(C.c_double)), yp,
                                   resid.ctypes.data_as(C.POINTER(C.c_double)), C.byref(st)), plan)
    return status, omega, resid, st.as_dict()


def nsf_eig_grad(plan, omega, Y, weights, d_eps, d_gamma):
    om, _ = _hptr(np.ravel(omega))
    w, _ = _hptr(np.ravel(weights))
    if w.size != om.size:
        raise ValueError(f"{w.size} weights for {om.size} eigenvalues")
    n = _plan_n(plan)
    return _check(lib().nsf_eig_grad(plan, len(om), om.ctypes.data_as(C.POINTER(C.c_double)),
                                     _dptr(Y, "c128", om.size * 4 * n), w.ctypes.data_as(C.POINTER(C.c_double)),
                                     _dptr(d_eps, "f64", n), _dptr(d_gamma, "f64", n)), plan)


def nsf_hermitian_eig(H):
    H = np.ascontiguousarray(H, dtype=np.complex128)
    m = H.shape[0]
    w = np.zeros(m)
    V = np.zeros((m, m), dtype=np.complex128)
    _check(lib().nsf_hermitian_eig(m, C.c_void_p(H.ctypes.data), w.ctypes.data_as(C.POINTER(C.c_double)),
                                   C.c_void_p(V.ctypes.data)))
    return w, V


def nsf_schur_sorted(A):
    """Complex Schur form A = Z T Z^* with the NFSEP Ritz order (host)."""
    A = np.asfortranarray(A, dtype=np.complex128)
    m = A.shape[0]
    T = np.zeros((m, m), dtype=np.complex128, order="F")
    Z = np.zeros((m, m), dtype=np.complex128, order="F")
    _check(lib().nsf_schur_sorted(m, C.c_void_p(A.ctypes.data), C.c_void_p(T.ctypes.data),
                                  C.c_void_p(Z.ctypes.data)))
    return T, Z


def nsf_device_info(device=0):
    d = nsf_device()
    _check(lib().nsf_device_info(int(device), C.byref(d)))
    return d.as_dict()


def nsf_batch_create(grids, ks, a=1.0, alpha=-1.0, beta=2.0, stream=None):
    g = np.ascontiguousarray(np.asarray(grids, dtype=np.int32).reshape(-1, 3))
    k = np.ascontiguousarray(np.asarray(ks, dtype=np.float64).reshape(-1, 3))
    if len(g) != len(k):
        raise ValueError("grids and ks differ in length")
    b = C.c_void_p()
    s = current_stream() if stream is None else stream
    _check(lib().nsf_batch_create(C.byref(b), len(g), C.c_void_p(g.ctypes.data), C.c_void_p(k.ctypes.data),
                                  float(a), float(alpha), float(beta), C.c_void_p(s)))
    return b


def nsf_batch_plan(batch, i):
    p = C.c_void_p()
    _check(lib().nsf_batch_plan(batch, int(i), C.byref(p)))
    return p


def nsf_batch_eigs(batch, count, nev, res_tol=1e-8, cg_rtol=1e-10, max_basis=0, max_restarts=0, seed=0,
                   Y=None):
    """Returns (status, omega[count, nev], resid[count, nev], list of stats dicts, wave size).
    Y: optional list of count device tensors (or None entries) of nev x 4n complex128."""
    omega = np.zeros((count, nev))
    resid = np.zeros((count, nev))
    st = (nsf_stats * count)()
    wave = C.c_int()
    yp = None
    if Y is not None:
        if len(Y) != count:
            raise ValueError(f"{len(Y)} vector buffers for {count} instances")
        yp = (C.c_void_p * count)(*[(_dptr(t, "c128", int(nev) * 4 * _plan_n(nsf_batch_plan(batch, i))).value
                                     if t is not None else None) for i, t in enumerate(Y)])
    status = _check(lib().nsf_batch_eigs(batch, int(nev), float(res_tol), float(cg_rtol), int(max_basis),
                                         int(max_restarts), C.c_ulonglong(seed),
                                         omega.ctypes.data_as(C.POINTER(C.c_double)),
                                         resid.ctypes.data_as(C.POINTER(C.c_double)), st, yp, C.byref(wave)))
    return status, omega, resid, [x.as_dict() for x in st], wave.value


def nsf_eigs_set_start(plan, Y0):
    """Y0: device tensor of count x 4n complex128 (kept alive by the caller until the
    next eigensolve returns), or None to clear."""
    if Y0 is None:
        return _check(lib().nsf_eigs_set_start(plan, None, 0), plan)
    count = Y0.shape[0] if Y0.dim() == 2 else 1
    return _check(lib().nsf_eigs_set_start(plan, _dptr(Y0, "c128", count * 4 * _plan_n(plan)), int(count)),
                  plan)


def nsf_plan_autotune(plan, reps=10):
    """Returns the chosen tiling and timings as a dict (see nsf_tune)."""
    t = nsf_tune()
    _check(lib().nsf_plan_autotune(plan, int(reps), C.byref(t)), plan)
    return t.as_dict()


def nsf_plan_workspace_size(plan, nev, max_basis=0):
    b = C.c_size_t()
    _check(lib().nsf_plan_workspace_size(plan, int(nev), int(max_basis), C.byref(b)), plan)
    return b.value


def nsf_plan_set_workspace(plan, buf):
    """buf: a contiguous torch tensor on the device (kept alive by the caller), or None."""
    if buf is None:
        return _check(lib().nsf_plan_set_workspace(plan, None, 0), plan)
    nbytes = buf.numel() * buf.element_size()
    return _check(lib().nsf_plan_set_workspace(plan, C.c_void_p(buf.data_ptr()), nbytes), plan)


def nsf_batch_autotune(batch, reps=10):
    shapes = C.c_int()
    _check(lib().nsf_batch_autotune(batch, int(reps), C.byref(shapes)))
    return shapes.value


def nsf_batch_destroy(batch):
    lib().nsf_batch_destroy(batch)


def nsf_status_string(status):
    return lib().nsf_status_string(int(status)).decode()


def nsf_last_error(plan=None):
    return (lib().nsf_last_error(plan) or b"").decode()


# ------------------------------------------------------------ convenience

class Batch:
    """Owns an ``nsf_batch`` of instances given as (grid, k) pairs."""

    def __init__(self, grids, ks, a=1.0, alpha=-1.0, beta=2.0, stream=None):
        self.count = len(grids)
        self.grids = [tuple(int(x) for x in g) for g in grids]
        self.handle = nsf_batch_create(grids, ks, a, alpha, beta, stream)

    def plan(self, i):
        return nsf_batch_plan(self.handle, i)

    def set_chiral(self, i, eps, gamma):
        return nsf_set_medium_chiral(self.plan(i), eps, gamma)

    def set_pseudochiral(self, i, axis_a, axis_b, eps, gamma):
        return nsf_set_medium_pseudochiral(self.plan(i), axis_a, axis_b, eps, gamma)

    def set_tensor(self, i, eps, mu, xi, zeta):
        return nsf_set_medium_tensor(self.plan(i), eps, mu, xi, zeta)

    def set_start(self, i, Y0):
        self._starts = getattr(self, "_starts", {})
        self._starts[i] = Y0
        return nsf_eigs_set_start(self.plan(i), Y0)

    def eigs(self, nev, **kw):
        return nsf_batch_eigs(self.handle, self.count, nev, **kw)

    def autotune(self, reps=10):
        return nsf_batch_autotune(self.handle, reps)

    def close(self):
        if getattr(self, "handle", None) is not None and _lib is not None:
            nsf_batch_destroy(self.handle)
        self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


class Plan:
    """Owns an ``nsf_plan``; frees it on ``close()`` / garbage collection."""

    def __init__(self, grid, k, a=1.0, alpha=-1.0, beta=2.0, stream=None):
        self.grid = tuple(int(x) for x in grid)
        self.k = tuple(float(x) for x in k)
        self.a, self.alpha, self.beta = float(a), float(alpha), float(beta)
        self.n = self.grid[0] * self.grid[1] * self.grid[2]
        self.handle = nsf_plan_create(*self.grid, self.a, self.k, self.alpha, self.beta, stream)

    def close(self):
        if getattr(self, "handle", None) is not None and _lib is not None:
            nsf_plan_destroy(self.handle)
        self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def set_option(self, option, value):
        return nsf_plan_set_option(self.handle, option, value)

    def query(self):
        return nsf_plan_query(self.handle)

    def set_chiral(self, eps, gamma):
        return nsf_set_medium_chiral(self.handle, eps, gamma)

    def set_pseudochiral(self, axis_a, axis_b, eps, gamma):
        return nsf_set_medium_pseudochiral(self.handle, axis_a, axis_b, eps, gamma)

    def set_tensor(self, eps, mu, xi, zeta):
        return nsf_set_medium_tensor(self.handle, eps, mu, xi, zeta)

    def medium_info(self):
        return nsf_plan_medium_info(self.handle)

    def set_nfsep(self, eps, mu, xi, zeta):
        return nsf_set_medium_nfsep(self.handle, eps, mu, xi, zeta)

    def K(self, y, out):
        return nsf_apply_nfsep(self.handle, y, out)

    def nfsep_solve(self, b, x, **kw):
        return nsf_nfsep_solve(self.handle, b, x, **kw)

    def eigs_nfsep(self, nev, **kw):
        return nsf_eigs_nfsep(self.handle, nev, **kw)

    def Ar(self, u, out):
        return nsf_apply_Ar(self.handle, u, out)

    def profile_Ar(self, u, out, reps=20):
        return nsf_profile_Ar(self.handle, u, out, reps)

    def fields(self, y, eh):
        return nsf_fields(self.handle, y, eh)

    def set_start(self, Y0):
        self._start = Y0  # alive until the next eigensolve
        return nsf_eigs_set_start(self.handle, Y0)

    def Br(self, u, out):
        return nsf_apply_Br(self.handle, u, out)

    def Pr(self, y, x):
        return nsf_apply_Pr(self.handle, y, x)

    def Qr(self, y, x):
        return nsf_apply_Qr(self.handle, y, x)

    def PrH(self, x, y):
        return nsf_apply_PrH(self.handle, x, y)

    def QrH(self, x, y):
        return nsf_apply_QrH(self.handle, x, y)

    def cg(self, b, x, rtol=1e-10, maxit=10000):
        return nsf_cg_solve(self.handle, b, x, rtol, maxit)

    def cg_noalloc(self, b, x, rtol=1e-10, maxit=10000):
        return nsf_cg_solve_noalloc(self.handle, b, x, rtol, maxit)

    def eigs(self, nev, **kw):
        return nsf_eigs(self.handle, nev, **kw)

    def eig_grad(self, omega, Y, weights, d_eps, d_gamma):
        return nsf_eig_grad(self.handle, omega, Y, weights, d_eps, d_gamma)

    def autotune(self, reps=10):
        return nsf_plan_autotune(self.handle, reps)

    def workspace_size(self, nev, max_basis=0):
        return nsf_plan_workspace_size(self.handle, nev, max_basis)

    def set_workspace(self, buf):
        self._workspace = buf  # keep the caller's tensor alive with the plan
        return nsf_plan_set_workspace(self.handle, buf)
