"""Thin ctypes binding of the C ABI in include/jam.h.

Argument marshalling only: every numerical step runs in the library's HIP
kernels.  The functions keep the C names (``jam_create``, ``jam_eval``,
``jam_eval_batch``, ``jam_eval_maps``, ``jam_vjp``, ``jam_destroy``, ...);
``Context`` wraps them for torch tensors, which serve only as device memory
and streams.  Loading fails loudly when the built library is missing.
"""
from __future__ import annotations

import ctypes
import os
from typing import List, Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libjam.so")

c_int32 = ctypes.c_int32
c_int64 = ctypes.c_int64
c_double = ctypes.c_double
c_void_p = ctypes.c_void_p
c_size_t = ctypes.c_size_t
P_double = ctypes.POINTER(c_double)
P_int32 = ctypes.POINTER(c_int32)

JAM_OK = 0
STATUS_NAMES = {0: "JAM_OK", 1: "JAM_E_INVALID_ARG", 2: "JAM_E_DEPROJECTION",
                3: "JAM_E_NONPHYSICAL", 4: "JAM_E_WORKSPACE", 5: "JAM_E_DEVICE",
                6: "JAM_E_UNSUPPORTED"}

EXPORTED = ("jam_create", "jam_destroy", "jam_batch_sizes", "jam_workspace_size",
            "jam_prepare", "jam_eval_batch", "jam_eval", "jam_eval_maps", "jam_vjp",
            "jam_gauss_legendre", "jam_timing", "jam_plan_info", "jam_last_error",
            "jam_set_kinematics", "jam_chi2", "jam_eval_chi2", "jam_vjp_chi2", "jam_mge1d",
            "jam_mge1d_vjp", "jam_beta_logistic", "jam_beta_logistic_vjp",
            "jam_eval_batch_noalloc")


class JamGeometry(ctypes.Structure):
    _fields_ = [("n_lum", c_int32), ("lum_sigma", P_double), ("lum_q", P_double),
                ("lum_I0", P_double), ("n_mass", c_int32), ("mass_sigma", P_double),
                ("mass_q", P_double), ("mass_S0", P_double), ("bh_sigma", c_double),
                ("distance_mpc", c_double), ("nx", c_int32), ("ny", c_int32),
                ("pixsize", c_double), ("xc", c_double), ("yc", c_double),
                ("supersample", c_int32), ("psf_n", c_int32), ("psf", P_double),
                ("n_bins", c_int32), ("bin_index", P_int32), ("n_u", c_int32)]


class JamOptions(ctypes.Structure):
    _fields_ = [("form", c_int32), ("autotune", c_int32), ("tune_cache", ctypes.c_char_p),
                ("launch", c_int32), ("graph", c_int32), ("alignment", c_int32)]


class JamBatch(ctypes.Structure):
    _fields_ = [("n", c_int32), ("geom_idx", P_int32), ("inc", c_void_p),
                ("mass_scale", c_void_p), ("m_bh", c_void_p), ("beta", c_void_p),
                ("lum_I0", c_void_p), ("mass_S0", c_void_p)]


class JamGrads(ctypes.Structure):
    _fields_ = [("inc", c_void_p), ("mass_scale", c_void_p), ("m_bh", c_void_p),
                ("beta", c_void_p), ("lum_I0", c_void_p), ("mass_S0", c_void_p)]


class JamError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


_lib = None


def load(path: str = LIB_PATH):
    """Load the built library (raises if it is missing) and declare its ABI."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"JAM HIP library not built: {path} is missing "
                           "(build it with python paper_2504_01302_amd/build.py)")
    lib = ctypes.CDLL(path)
    lib.jam_create.argtypes = [c_int32, ctypes.POINTER(JamGeometry), ctypes.POINTER(JamOptions),
                               ctypes.POINTER(c_void_p)]
    lib.jam_destroy.argtypes = [c_void_p]
    lib.jam_destroy.restype = None
    lib.jam_batch_sizes.argtypes = [c_void_p, c_int32, P_int32, ctypes.POINTER(c_int64),
                                    ctypes.POINTER(c_int64), ctypes.POINTER(c_int64)]
    lib.jam_workspace_size.argtypes = [c_void_p, c_int32, P_int32, c_int32,
                                       ctypes.POINTER(c_size_t)]
    lib.jam_prepare.argtypes = [c_void_p, c_int32, P_int32]
    for fn in (lib.jam_eval_batch, lib.jam_eval):
        fn.argtypes = [c_void_p, ctypes.POINTER(JamBatch), c_void_p, c_void_p, c_void_p,
                       c_size_t, c_void_p]
    lib.jam_eval_batch_noalloc.argtypes = [c_void_p, ctypes.POINTER(JamBatch), c_void_p,
                                           c_void_p, c_void_p]
    lib.jam_eval_maps.argtypes = [c_void_p, ctypes.POINTER(JamBatch), c_void_p, c_void_p,
                                  c_void_p, c_void_p, c_size_t, c_void_p]
    lib.jam_vjp.argtypes = [c_void_p, ctypes.POINTER(JamBatch), c_void_p, c_void_p,
                            ctypes.POINTER(JamGrads), c_void_p, c_size_t, c_void_p]
    lib.jam_gauss_legendre.argtypes = [c_int32, P_double, P_double]
    lib.jam_timing.argtypes = [c_void_p, c_int32, ctypes.POINTER(c_double), ctypes.POINTER(c_int64),
                               ctypes.POINTER(c_double), ctypes.POINTER(c_int64)]
    lib.jam_plan_info.argtypes = [c_void_p, c_int32, P_int32, P_int32]
    lib.jam_set_kinematics.argtypes = [c_void_p, c_int32, P_double, P_double]
    lib.jam_mge1d.argtypes = [c_int32, c_int32, c_void_p, c_int32, P_double, c_int32, c_void_p,
                              c_void_p]
    lib.jam_mge1d_vjp.argtypes = [c_int32, c_int32, c_void_p, c_int32, P_double, c_int32,
                                  c_void_p, c_void_p, c_void_p]
    lib.jam_chi2.argtypes = [c_void_p, ctypes.POINTER(JamBatch), c_void_p, c_void_p, c_void_p,
                             c_void_p]
    lib.jam_beta_logistic.argtypes = [c_void_p, ctypes.POINTER(JamBatch), c_void_p, c_void_p,
                                      c_void_p]
    lib.jam_beta_logistic_vjp.argtypes = [c_void_p, ctypes.POINTER(JamBatch), c_void_p, c_void_p,
                                          c_void_p, c_void_p]
    lib.jam_eval_chi2.argtypes = [c_void_p, ctypes.POINTER(JamBatch), c_void_p, c_void_p,
                                  c_void_p, c_void_p, c_size_t, c_void_p]
    lib.jam_vjp_chi2.argtypes = [c_void_p, ctypes.POINTER(JamBatch), c_void_p, c_void_p,
                                 ctypes.POINTER(JamGrads), c_void_p, c_size_t, c_void_p]
    lib.jam_last_error.restype = ctypes.c_char_p
    for name in EXPORTED:
        f = getattr(lib, name)
        if name not in ("jam_destroy", "jam_last_error"):
            f.restype = c_int32
    _lib = lib
    return lib


def _check(status: int):
    if status != JAM_OK:
        raise JamError(status, load().jam_last_error().decode())


# ---------------------------------------------------------------------------
# The C functions, under their own names.
# ---------------------------------------------------------------------------

def jam_gauss_legendre(n: int):
    x = np.zeros(n)
    w = np.zeros(n)
    _check(load().jam_gauss_legendre(n, x.ctypes.data_as(P_double), w.ctypes.data_as(P_double)))
    return x, w


def _geometry_struct(g, keep: list) -> JamGeometry:
    def arr(a, dt=np.float64):
        a = np.ascontiguousarray(np.asarray(a, dtype=dt))
        keep.append(a)
        return a.ctypes.data_as(P_double if dt == np.float64 else P_int32)
    return JamGeometry(
        g.n_lum, arr(g.lum_sigma), arr(g.lum_q), arr(g.lum_I0),
        g.n_mass, arr(g.mass_sigma), arr(g.mass_q), arr(g.mass_S0),
        float(g.bh_sigma), float(g.distance_mpc), int(g.nx), int(g.ny),
        float(g.pixsize), float(g.xc), float(g.yc), int(g.supersample),
        int(g.psf_n), arr(g.psf), int(g.n_bins), arr(g.bin_index, np.int32), int(g.n_u))


def jam_create(geometries: Sequence, form: int = 0, autotune: int = 0,
               tune_cache: Optional[str] = None, launch: int = 0, graph: int = 0,
               alignment: int = 0) -> int:
    keep: list = []
    arr = (JamGeometry * len(geometries))(*[_geometry_struct(g, keep) for g in geometries])
    opt = JamOptions(form, autotune, tune_cache.encode() if tune_cache else None, launch, graph,
                     alignment)
    out = c_void_p()
    _check(load().jam_create(len(geometries), arr, ctypes.byref(opt), ctypes.byref(out)))
    return out.value


def jam_destroy(ctx: int):
    if ctx:
        load().jam_destroy(c_void_p(ctx))


def _idx(geom_idx) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(geom_idx, dtype=np.int32))


def jam_batch_sizes(ctx: int, geom_idx):
    gi = _idx(geom_idx)
    b, l, m = c_int64(), c_int64(), c_int64()
    _check(load().jam_batch_sizes(c_void_p(ctx), len(gi), gi.ctypes.data_as(P_int32),
                                  ctypes.byref(b), ctypes.byref(l), ctypes.byref(m)))
    return b.value, l.value, m.value


def jam_workspace_size(ctx: int, geom_idx, with_vjp: bool) -> int:
    gi = _idx(geom_idx)
    out = c_size_t()
    _check(load().jam_workspace_size(c_void_p(ctx), len(gi), gi.ctypes.data_as(P_int32),
                                     int(with_vjp), ctypes.byref(out)))
    return out.value


def jam_plan_info(ctx: int, geom_idx) -> dict:
    gi = _idx(geom_idx)
    info = np.zeros(9, np.int32)
    _check(load().jam_plan_info(c_void_p(ctx), len(gi), gi.ctypes.data_as(P_int32),
                                info.ctypes.data_as(P_int32)))
    keys = ("rule", "tau", "gran", "launch", "num_items", "num_grid", "sens_items", "sens_grid",
            "num_kernel")
    return dict(zip(keys, (int(v) for v in info)))


def jam_prepare(ctx: int, geom_idx):
    gi = _idx(geom_idx)
    _check(load().jam_prepare(c_void_p(ctx), len(gi), gi.ctypes.data_as(P_int32)))


def jam_timing(ctx: int, enable: bool):
    """Start (enable) or stop kernel timing; stopping returns
    (numerator_ms, numerator_launches, sens_ms, sens_launches)."""
    a, b, c, d = c_double(), c_int64(), c_double(), c_int64()
    _check(load().jam_timing(c_void_p(ctx), int(enable), ctypes.byref(a), ctypes.byref(b),
                             ctypes.byref(c), ctypes.byref(d)))
    return a.value, b.value, c.value, d.value


def _ptr(t) -> Optional[int]:
    return None if t is None else t.data_ptr()


def _batch(geom_idx: np.ndarray, inc, mass_scale, m_bh, beta, lum_I0, mass_S0) -> JamBatch:
    return JamBatch(len(geom_idx), geom_idx.ctypes.data_as(P_int32), _ptr(inc),
                    _ptr(mass_scale), _ptr(m_bh), _ptr(beta), _ptr(lum_I0), _ptr(mass_S0))


def jam_eval_batch(ctx, geom_idx, inc, mass_scale, m_bh, beta, lum_I0, mass_S0,
                   vrms2, status, ws, stream: int):
    gi = _idx(geom_idx)
    b = _batch(gi, inc, mass_scale, m_bh, beta, lum_I0, mass_S0)
    _check(load().jam_eval_batch(c_void_p(ctx), ctypes.byref(b), _ptr(vrms2), _ptr(status),
                                 _ptr(ws), ws.numel() * ws.element_size(), c_void_p(stream)))


def jam_eval(ctx, geom_idx, inc, mass_scale, m_bh, beta, lum_I0, mass_S0,
             vrms2, status, ws, stream: int):
    gi = _idx(geom_idx)
    b = _batch(gi, inc, mass_scale, m_bh, beta, lum_I0, mass_S0)
    _check(load().jam_eval(c_void_p(ctx), ctypes.byref(b), _ptr(vrms2), _ptr(status),
                           _ptr(ws), ws.numel() * ws.element_size(), c_void_p(stream)))


def jam_eval_batch_noalloc(ctx, geom_idx, inc, mass_scale, m_bh, beta, lum_I0, mass_S0,
                           vrms2, status, stream: int):
    gi = _idx(geom_idx)
    b = _batch(gi, inc, mass_scale, m_bh, beta, lum_I0, mass_S0)
    _check(load().jam_eval_batch_noalloc(c_void_p(ctx), ctypes.byref(b), _ptr(vrms2),
                                         _ptr(status), c_void_p(stream)))


def jam_eval_maps(ctx, geom_idx, inc, mass_scale, m_bh, beta, lum_I0, mass_S0,
                  N_map, I_map, status, ws, stream: int):
    gi = _idx(geom_idx)
    b = _batch(gi, inc, mass_scale, m_bh, beta, lum_I0, mass_S0)
    _check(load().jam_eval_maps(c_void_p(ctx), ctypes.byref(b), _ptr(N_map), _ptr(I_map),
                                _ptr(status), _ptr(ws), ws.numel() * ws.element_size(),
                                c_void_p(stream)))


def jam_vjp(ctx, geom_idx, inc, mass_scale, m_bh, beta, lum_I0, mass_S0, vrms2, cot,
            g_inc, g_mass_scale, g_m_bh, g_beta, g_lum_I0, g_mass_S0, ws, stream: int):
    gi = _idx(geom_idx)
    b = _batch(gi, inc, mass_scale, m_bh, beta, lum_I0, mass_S0)
    gr = JamGrads(_ptr(g_inc), _ptr(g_mass_scale), _ptr(g_m_bh), _ptr(g_beta),
                  _ptr(g_lum_I0), _ptr(g_mass_S0))
    _check(load().jam_vjp(c_void_p(ctx), ctypes.byref(b), _ptr(vrms2), _ptr(cot),
                          ctypes.byref(gr), _ptr(ws), ws.numel() * ws.element_size(),
                          c_void_p(stream)))


def jam_set_kinematics(ctx: int, geom: int, vrms_obs, cov):
    v = np.ascontiguousarray(vrms_obs, dtype=np.float64)
    c = np.ascontiguousarray(cov, dtype=np.float64)
    if c.size != v.size * v.size:
        raise ValueError("cov must be n_bins x n_bins")
    _check(load().jam_set_kinematics(c_void_p(ctx), int(geom), v.ctypes.data_as(P_double),
                                      c.ctypes.data_as(P_double)))


def jam_chi2(ctx, geom_idx, vrms2, chi2, dchi2, stream: int):
    gi = _idx(geom_idx)
    b = _batch(gi, None, None, None, None, None, None)
    _check(load().jam_chi2(c_void_p(ctx), ctypes.byref(b), _ptr(vrms2), _ptr(chi2), _ptr(dchi2),
                           c_void_p(stream)))


def jam_eval_chi2(ctx, geom_idx, inc, mass_scale, m_bh, beta, lum_I0, mass_S0,
                  chi2, vrms2, status, ws, stream: int):
    gi = _idx(geom_idx)
    b = _batch(gi, inc, mass_scale, m_bh, beta, lum_I0, mass_S0)
    _check(load().jam_eval_chi2(c_void_p(ctx), ctypes.byref(b), _ptr(chi2), _ptr(vrms2),
                                _ptr(status), _ptr(ws), ws.numel() * ws.element_size(),
                                c_void_p(stream)))


def jam_vjp_chi2(ctx, geom_idx, inc, mass_scale, m_bh, beta, lum_I0, mass_S0, vrms2, cot,
                 g_inc, g_mass_scale, g_m_bh, g_beta, g_lum_I0, g_mass_S0, ws, stream: int):
    gi = _idx(geom_idx)
    b = _batch(gi, inc, mass_scale, m_bh, beta, lum_I0, mass_S0)
    gr = JamGrads(_ptr(g_inc), _ptr(g_mass_scale), _ptr(g_m_bh), _ptr(g_beta),
                  _ptr(g_lum_I0), _ptr(g_mass_S0))
    _check(load().jam_vjp_chi2(c_void_p(ctx), ctypes.byref(b), _ptr(vrms2), _ptr(cot),
                               ctypes.byref(gr), _ptr(ws), ws.numel() * ws.element_size(),
                               c_void_p(stream)))


def jam_beta_logistic(ctx, geom_idx, prof, beta, stream: int):
    gi = _idx(geom_idx)
    b = _batch(gi, None, None, None, None, None, None)
    _check(load().jam_beta_logistic(c_void_p(ctx), ctypes.byref(b), _ptr(prof), _ptr(beta),
                                    c_void_p(stream)))


def jam_beta_logistic_vjp(ctx, geom_idx, prof, cot, grad, stream: int):
    gi = _idx(geom_idx)
    b = _batch(gi, None, None, None, None, None, None)
    _check(load().jam_beta_logistic_vjp(c_void_p(ctx), ctypes.byref(b), _ptr(prof), _ptr(cot),
                                        _ptr(grad), c_void_p(stream)))


def jam_mge1d(comp, sigma, euler_p: int = 10, out=None, stream=None):
    """Peak amplitudes [n_prof, n_sigma] of the 1-D MGE of cored power-law
    profiles; comp is a float64 device tensor [n_prof, n_comp, 3]."""
    import torch
    comp = comp.contiguous()
    sig = np.ascontiguousarray(sigma, dtype=np.float64)
    amp = out if out is not None else torch.empty(comp.shape[0], len(sig), dtype=torch.float64,
                                                  device=comp.device)
    s = stream if stream is not None else torch.cuda.current_stream(comp.device).cuda_stream
    _check(load().jam_mge1d(comp.shape[0], comp.shape[1], _ptr(comp), len(sig),
                            sig.ctypes.data_as(P_double), int(euler_p), _ptr(amp), c_void_p(s)))
    return amp


def jam_mge1d_vjp(comp, sigma, cot, euler_p: int = 10, stream=None):
    """Gradient [n_prof, n_comp, 3] of sum(cot * amp) with respect to comp."""
    import torch
    comp = comp.contiguous()
    cot = cot.contiguous()
    sig = np.ascontiguousarray(sigma, dtype=np.float64)
    grad = torch.empty_like(comp)
    s = stream if stream is not None else torch.cuda.current_stream(comp.device).cuda_stream
    _check(load().jam_mge1d_vjp(comp.shape[0], comp.shape[1], _ptr(comp), len(sig),
                                sig.ctypes.data_as(P_double), int(euler_p), _ptr(cot),
                                _ptr(grad), c_void_p(s)))
    return grad


# ---------------------------------------------------------------------------
# Convenience wrapper for torch device tensors.
# ---------------------------------------------------------------------------

class Context:
    """Owns a library context for a list of geometries.

    Parameter tensors are float64 on the GPU, packed model after model as
    the C ABI describes; ``geom_idx`` is a host integer array.
    """

    def __init__(self, geometries: Sequence, form: int = 0, autotune: int = 0,
                 tune_cache: Optional[str] = None, launch: int = 0, graph: int = 0,
                 alignment: int = 0):
        self.geometries = list(geometries)
        self.handle = jam_create(self.geometries, form, autotune, tune_cache, launch, graph,
                                 alignment)
        self._ws = {}

    def close(self):
        if self.handle:
            jam_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def workspace(self, geom_idx, with_vjp: bool, device=None):
        import torch
        n = jam_workspace_size(self.handle, geom_idx, with_vjp)
        key = (bool(with_vjp), str(device))
        ws = self._ws.get(key)
        if ws is None or ws.numel() < n:
            # 256-byte aligned (the caching allocator aligns to at least 512)
            ws = torch.empty(max(n, 256), dtype=torch.uint8, device=device or "cuda")
            self._ws[key] = ws
        return ws

    def sizes(self, geom_idx):
        return jam_batch_sizes(self.handle, geom_idx)

    def plan_info(self, geom_idx) -> dict:
        return jam_plan_info(self.handle, geom_idx)

    def eval_batch(self, geom_idx, inc, mass_scale, m_bh, beta, lum_I0=None, mass_S0=None,
                   stream=None, out=None, status=None):
        import torch
        dev = inc.device
        nb, _, _ = self.sizes(geom_idx)
        vr = out if out is not None else torch.empty(nb, dtype=torch.float64, device=dev)
        st = status if status is not None else torch.empty(len(geom_idx), dtype=torch.int32, device=dev)
        ws = self.workspace(geom_idx, False, dev)
        s = stream if stream is not None else torch.cuda.current_stream(dev).cuda_stream
        jam_eval_batch(self.handle, geom_idx, inc, mass_scale, m_bh, beta, lum_I0, mass_S0,
                       vr, st, ws, s)
        return vr, st

    def eval_maps(self, geom_idx, inc, mass_scale, m_bh, beta, lum_I0=None, mass_S0=None,
                  stream=None):
        import torch
        dev = inc.device
        total = 0
        for g in (self.geometries[i] for i in np.asarray(geom_idx)):
            nxp = g.nx * g.supersample + g.psf_n - 1
            nyp = g.ny * g.supersample + g.psf_n - 1
            total += nxp * nyp
        N = torch.empty(total, dtype=torch.float64, device=dev)
        I = torch.empty(total, dtype=torch.float64, device=dev)
        st = torch.empty(len(geom_idx), dtype=torch.int32, device=dev)
        ws = self.workspace(geom_idx, False, dev)
        s = stream if stream is not None else torch.cuda.current_stream(dev).cuda_stream
        jam_eval_maps(self.handle, geom_idx, inc, mass_scale, m_bh, beta, lum_I0, mass_S0,
                      N, I, st, ws, s)
        return N, I, st

    def vjp(self, geom_idx, inc, mass_scale, m_bh, beta, lum_I0, mass_S0, vrms2, cot,
            stream=None):
        import torch
        dev = inc.device
        n = len(geom_idx)
        _, nl, nm = self.sizes(geom_idx)
        z = lambda k: torch.empty(k, dtype=torch.float64, device=dev)
        g = dict(inc=z(n), mass_scale=z(n), m_bh=z(n), beta=z(nl), lum_I0=z(nl), mass_S0=z(nm))
        ws = self.workspace(geom_idx, True, dev)
        s = stream if stream is not None else torch.cuda.current_stream(dev).cuda_stream
        jam_vjp(self.handle, geom_idx, inc, mass_scale, m_bh, beta, lum_I0, mass_S0, vrms2, cot,
                g["inc"], g["mass_scale"], g["m_bh"], g["beta"], g["lum_I0"], g["mass_S0"], ws, s)
        return g


    def beta_logistic(self, geom_idx, prof, out=None, stream=None):
        """Packed beta_k from logistic anisotropy profiles prof [n, 4] =
        (beta_0, beta_inf, r_a, alpha), sampled at each tracer sigma."""
        import torch
        prof = prof.contiguous()
        _, nl, _ = self.sizes(geom_idx)
        beta = out if out is not None else torch.empty(nl, dtype=torch.float64, device=prof.device)
        s = stream if stream is not None else torch.cuda.current_stream(prof.device).cuda_stream
        jam_beta_logistic(self.handle, geom_idx, prof, beta, s)
        return beta

    def beta_logistic_vjp(self, geom_idx, prof, cot, stream=None):
        """Gradient [n, 4] of sum(cot * beta) with respect to the profiles."""
        import torch
        prof = prof.contiguous()
        grad = torch.empty_like(prof)
        s = stream if stream is not None else torch.cuda.current_stream(prof.device).cuda_stream
        jam_beta_logistic_vjp(self.handle, geom_idx, prof, cot.contiguous(), grad, s)
        return grad

    def set_kinematics(self, geom: int, vrms_obs, cov):
        jam_set_kinematics(self.handle, geom, vrms_obs, cov)

    def chi2(self, geom_idx, vrms2, want_grad: bool = False, stream=None):
        """chi^2 per model from packed v_rms^2 (and d chi^2 / d v_rms^2)."""
        import torch
        dev = vrms2.device
        c = torch.empty(len(geom_idx), dtype=torch.float64, device=dev)
        d = torch.empty_like(vrms2) if want_grad else None
        s = stream if stream is not None else torch.cuda.current_stream(dev).cuda_stream
        jam_chi2(self.handle, geom_idx, vrms2, c, d, s)
        return c, d

    def eval_chi2(self, geom_idx, inc, mass_scale, m_bh, beta, lum_I0=None, mass_S0=None,
                  stream=None, keep_vrms2: bool = False):
        import torch
        dev = inc.device
        nb, _, _ = self.sizes(geom_idx)
        c = torch.empty(len(geom_idx), dtype=torch.float64, device=dev)
        vr = torch.empty(nb, dtype=torch.float64, device=dev) if keep_vrms2 else None
        st = torch.empty(len(geom_idx), dtype=torch.int32, device=dev)
        ws = self.workspace(geom_idx, False, dev)
        s = stream if stream is not None else torch.cuda.current_stream(dev).cuda_stream
        jam_eval_chi2(self.handle, geom_idx, inc, mass_scale, m_bh, beta, lum_I0, mass_S0,
                      c, vr, st, ws, s)
        return c, vr, st

    def vjp_chi2(self, geom_idx, inc, mass_scale, m_bh, beta, lum_I0, mass_S0, cot,
                 vrms2=None, stream=None):
        import torch
        dev = inc.device
        n = len(geom_idx)
        _, nl, nm = self.sizes(geom_idx)
        z = lambda k: torch.empty(k, dtype=torch.float64, device=dev)
        g = dict(inc=z(n), mass_scale=z(n), m_bh=z(n), beta=z(nl), lum_I0=z(nl), mass_S0=z(nm))
        ws = self.workspace(geom_idx, True, dev)
        s = stream if stream is not None else torch.cuda.current_stream(dev).cuda_stream
        jam_vjp_chi2(self.handle, geom_idx, inc, mass_scale, m_bh, beta, lum_I0, mass_S0,
                     vrms2, cot, g["inc"], g["mass_scale"], g["m_bh"], g["beta"], g["lum_I0"],
                     g["mass_S0"], ws, s)
        return g


def pack_params(workload, device="cuda", amplitudes: bool = False):
    """Device tensors of a workload's per-model parameters, packed as the
    C ABI expects.  Returns a dict with inc, mass_scale, m_bh, beta and, if
    ``amplitudes``, lum_I0 and mass_S0 (geometry defaults unless overridden)."""
    import torch
    ps = workload.params
    gs = workload.geometries
    gi = workload.geom_idx
    t = lambda a: torch.as_tensor(np.asarray(a, dtype=np.float64), device=device)
    out = dict(inc=t([p.inc for p in ps]), mass_scale=t([p.mass_scale for p in ps]),
               m_bh=t([p.m_bh for p in ps]),
               beta=t(np.concatenate([np.asarray(p.beta, np.float64) for p in ps])))
    if amplitudes:
        out["lum_I0"] = t(np.concatenate([
            p.lum_I0 if p.lum_I0 is not None else gs[i].lum_I0 for p, i in zip(ps, gi)]))
        out["mass_S0"] = t(np.concatenate([
            p.mass_S0 if p.mass_S0 is not None else gs[i].mass_S0 for p, i in zip(ps, gi)]))
    else:
        out["lum_I0"] = None
        out["mass_S0"] = None
    return out
