"""Thin ctypes binding of liblisatd (include/lisatd.h).

Argument marshalling only: every step of the likelihood runs in the HIP
kernels of liblisatd.so.  Device buffers are torch tensors on a ROCm device;
the binding passes their data pointers and the current torch stream.  If the
library has not been built this module raises at import: there is no CPU
fallback.
"""
import ctypes
import math
import os

import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liblisatd.so")

LT_FP64, LT_MIXED = 0, 1
LT_ORBIT_STATIC_EQUAL, LT_ORBIT_KEPLER, LT_ORBIT_TABLE = 0, 1, 2
LT_CH_A, LT_CH_E, LT_CH_T = 1, 2, 4
MODE_BITS = {(2, 2): 1, (2, 1): 2, (3, 3): 4, (3, 2): 8, (4, 4): 16}
MODE_ORDER = ((2, 2), (2, 1), (3, 3), (3, 2), (4, 4))
ARM_M = 2.5e9
AU_M = 1.495978707e11

if not os.path.exists(LIB_PATH):
    raise ImportError("liblisatd.so is not built (run `python -m paper_2501_08261_amd.build`)")
_lib = ctypes.CDLL(LIB_PATH)


class Grid(ctypes.Structure):
    _fields_ = [("t0", ctypes.c_double), ("dt", ctypes.c_double), ("n", ctypes.c_int64)]


class WfCfg(ctypes.Structure):
    _fields_ = [("mode_mask", ctypes.c_int), ("precessing", ctypes.c_int), ("f_low", ctypes.c_double),
                ("f_ref", ctypes.c_double), ("precision", ctypes.c_int), ("coarse", ctypes.c_int)]


class Orbit(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int), ("arm_m", ctypes.c_double), ("au_m", ctypes.c_double),
                ("phase0", ctypes.c_double), ("t_ref", ctypes.c_double), ("n_tab", ctypes.c_int64),
                ("tab_t0", ctypes.c_double), ("tab_dt", ctypes.c_double), ("pos", ctypes.c_void_p),
                ("ltt", ctypes.c_void_p)]


class TdiCfg(ctypes.Structure):
    _fields_ = [("generation", ctypes.c_int), ("channels", ctypes.c_int), ("taps", ctypes.c_int),
                ("out_xyz", ctypes.c_int)]


class Psd(ctypes.Structure):
    _fields_ = [("S", ctypes.c_void_p * 3), ("f_lo", ctypes.c_double), ("f_hi", ctypes.c_double)]


class Data(ctypes.Structure):
    _fields_ = [("aet", ctypes.c_void_p), ("dd", ctypes.c_double)]


class Tuning(ctypes.Structure):
    _fields_ = [("chunk", ctypes.c_int), ("rotate", ctypes.c_int), ("persistent", ctypes.c_int),
                ("wg_per_cu", ctypes.c_int)]

    def as_dict(self):
        return {"chunk": self.chunk, "rotate": self.rotate, "persistent": self.persistent, "wg_per_cu": self.wg_per_cu}


class SamplerCfg(ctypes.Structure):
    _fields_ = [("n_walkers", ctypes.c_int), ("n_temps", ctypes.c_int), ("dim", ctypes.c_int),
                ("param_kind", ctypes.c_int), ("target", ctypes.c_int), ("stretch_a", ctypes.c_double),
                ("t_max", ctypes.c_double), ("seed", ctypes.c_uint64), ("t_c", ctypes.c_double),
                ("lo", ctypes.c_void_p), ("hi", ctypes.c_void_p), ("n_gauss", ctypes.c_int),
                ("gauss_mean", ctypes.c_void_p), ("gauss_icov", ctypes.c_void_p)]


LT_PARAMS_ALIGNED10, LT_PARAMS_PRECESSING14, LT_PARAMS_RAW = 0, 1, 2
LT_TARGET_TDI, LT_TARGET_GAUSS = 0, 1

_P = ctypes.c_void_p
_I64 = ctypes.c_int64
_sig = {
    "lt_last_error": ([], ctypes.c_char_p),
    "lt_ctx_create": ([ctypes.c_int, ctypes.POINTER(_P)], ctypes.c_int),
    "lt_ctx_destroy": ([_P], ctypes.c_int),
    "lt_phenomt_modes": ([_P, _P, _I64, ctypes.POINTER(WfCfg), ctypes.POINTER(Grid), _P, _P], ctypes.c_int),
    "lt_phenomt_polarizations": ([_P, _P, _I64, ctypes.POINTER(WfCfg), ctypes.POINTER(Grid), _P, _P], ctypes.c_int),
    "lt_lisa_tdi_response": ([_P, _P, _I64, ctypes.POINTER(WfCfg), ctypes.POINTER(Grid), ctypes.POINTER(Orbit),
                              ctypes.POINTER(TdiCfg), _P, _P, _P], ctypes.c_int),
    "lt_tdi_loglike": ([_P, _P, _I64, ctypes.POINTER(WfCfg), ctypes.POINTER(Grid), ctypes.POINTER(Orbit),
                        ctypes.POINTER(TdiCfg), ctypes.POINTER(Psd), ctypes.POINTER(Data), _P, _P, _P, _P,
                        ctypes.c_size_t, _P], ctypes.c_int),
    "lt_tdi_loglike_noalloc": ([_P, _P, _I64, ctypes.POINTER(WfCfg), ctypes.POINTER(Grid), ctypes.POINTER(Orbit),
                                ctypes.POINTER(TdiCfg), ctypes.POINTER(Psd), ctypes.POINTER(Data), _P, _P, _P, _P],
                               ctypes.c_int),
    "lt_ctx_set_tuning": ([_P, ctypes.POINTER(Tuning)], ctypes.c_int),
    "lt_ctx_get_tuning": ([_P, ctypes.POINTER(Tuning)], ctypes.c_int),
    "lt_autotune": ([_P, _P, _I64, ctypes.POINTER(WfCfg), ctypes.POINTER(Grid), ctypes.POINTER(Orbit),
                     ctypes.POINTER(TdiCfg), ctypes.POINTER(Psd), ctypes.POINTER(Data), ctypes.c_char_p, ctypes.c_int,
                     ctypes.POINTER(Tuning), ctypes.POINTER(ctypes.c_double), _P], ctypes.c_int),
    "lt_workspace_size": ([_P, _I64, ctypes.POINTER(WfCfg), ctypes.POINTER(Grid), ctypes.POINTER(TdiCfg),
                           ctypes.POINTER(ctypes.c_size_t), ctypes.POINTER(ctypes.c_size_t)], ctypes.c_int),
    "lt_noise_inner": ([_P, _P, _I64, ctypes.POINTER(Grid), ctypes.POINTER(Psd), ctypes.c_int, ctypes.c_int, _P, _P],
                       ctypes.c_int),
    "lt_rfft": ([_P, _P, _I64, _I64, ctypes.c_double, ctypes.c_int, _P, _P], ctypes.c_int),
    "lt_psd_sangria": ([ctypes.POINTER(Grid), ctypes.c_int, ctypes.c_double, _P, _P], ctypes.c_int),
    "lt_sampler_create": ([ctypes.c_int, ctypes.POINTER(SamplerCfg), ctypes.POINTER(WfCfg), ctypes.POINTER(Grid),
                           ctypes.POINTER(Orbit), ctypes.POINTER(TdiCfg), ctypes.POINTER(Psd), ctypes.POINTER(Data),
                           ctypes.POINTER(_P)], ctypes.c_int),
    "lt_sampler_destroy": ([_P], ctypes.c_int),
    "lt_sampler_set_state": ([_P, _P], ctypes.c_int),
    "lt_sampler_step": ([_P, ctypes.c_int, _P], ctypes.c_int),
    "lt_sampler_get_state": ([_P, _P, _P, _P, _P, _P], ctypes.c_int),
    "lt_sampler_set_flow": ([_P, _P], ctypes.c_int),
    "lt_sampler_set_flow_fold": ([_P, ctypes.c_int, ctypes.c_double, ctypes.c_double], ctypes.c_int),
    "lt_sampler_set_flow_walk": ([_P, ctypes.c_double], ctypes.c_int),
    "lt_sampler_flow_counts": ([_P, _P], ctypes.c_int),
    "lt_flow_set_mix": ([_P, ctypes.c_double], ctypes.c_int),
    "lt_sampler_set_flow_exclusive": ([_P, ctypes.c_int], ctypes.c_int),
    "lt_sampler_set_flow_mixture": ([_P, _P, ctypes.c_double], ctypes.c_int),
    "lt_fisher": ([_P, _P, ctypes.c_int, ctypes.c_double, _P, ctypes.POINTER(WfCfg), ctypes.POINTER(Grid),
                   ctypes.POINTER(Orbit), ctypes.POINTER(TdiCfg), ctypes.POINTER(Psd), _P], ctypes.c_int),
    "lt_fisher_draw": ([_P, _P, ctypes.c_int, _P, _P, _I64, ctypes.c_uint64, ctypes.c_double, _P], ctypes.c_int),
    "lt_flow_create": ([ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.POINTER(_P)],
                       ctypes.c_int),
    "lt_flow_destroy": ([_P], ctypes.c_int),
    "lt_flow_num_params": ([_P], _I64),
    "lt_flow_set_params": ([_P, _P, _P, _P], ctypes.c_int),
    "lt_flow_get_params": ([_P, _P], ctypes.c_int),
    "lt_flow_set_whitening": ([_P, _P, _P], ctypes.c_int),
    "lt_flow_log_prob": ([_P, _P, _I64, _P, _P], ctypes.c_int),
    "lt_flow_sample": ([_P, _P, _I64, _P, _P, _P], ctypes.c_int),
    "lt_flow_loss_grad": ([_P, _P, _I64, _P, _P], ctypes.c_int),
    "lt_flow_train": ([_P, _P, _I64, ctypes.c_int, ctypes.c_int, ctypes.c_double, _P], ctypes.c_int),
    "lt_profile_enable": ([_P, ctypes.c_int], ctypes.c_int),
    "lt_profile_read": ([_P, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int64), ctypes.c_int],
                        ctypes.c_int),
}
for _name, (_args, _res) in _sig.items():
    _f = getattr(_lib, _name)
    _f.argtypes = _args
    _f.restype = _res

EXPORTED = tuple(_sig)


class LisaTDError(RuntimeError):
    pass


def _check(status):
    if status != 0:
        raise LisaTDError("liblisatd error %d: %s" % (status, _lib.lt_last_error().decode()))


def _ptr(t, name="tensor", dtype=None, numel=None, shape=None, device=None):
    """Data pointer of a device tensor after the checks that keep a kernel inside its buffers:
    a contiguous tensor on a ROCm device (on `device` when given), of `dtype`, with exactly
    `numel` elements or the given shape (None entries match any size).  Raises ValueError
    before anything reaches the library."""
    if t is None:
        return None
    if not isinstance(t, torch.Tensor):
        raise ValueError("%s: torch tensor required" % name)
    if dtype is not None and t.dtype != dtype:
        raise ValueError("%s: dtype %s, expected %s" % (name, t.dtype, dtype))
    if shape is not None and (t.dim() != len(shape) or
                              any(w is not None and int(w) != int(a) for a, w in zip(t.shape, shape))):
        raise ValueError("%s: shape %s, expected %s" % (name, tuple(t.shape), tuple(shape)))
    if numel is not None and t.numel() != int(numel):
        raise ValueError("%s: %d elements, expected %d" % (name, t.numel(), int(numel)))
    if not t.is_contiguous():
        raise ValueError("%s: contiguous tensor required" % name)
    if not t.is_cuda:
        raise ValueError("%s: device tensor required" % name)
    if device is not None and t.device.index != device:
        raise ValueError("%s: on device %s, the context is on device %d" % (name, t.device, device))
    return ctypes.c_void_p(t.data_ptr())


def _psd_struct(psd, n, f_lo, f_hi, device=None):
    """lt_psd for a device FP64 tensor [3][n/2+1] (one row per channel A, E, T)."""
    _ptr(psd, "psd", torch.float64, shape=(3, n // 2 + 1), device=device)
    return Psd((ctypes.c_void_p * 3)(*[psd[i].data_ptr() for i in range(3)]), f_lo, f_hi)


def _params_ptr(params, device=None):
    return _ptr(params, "params", torch.float64, shape=(None, 16), device=device)


def _stream(stream=None):
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def mode_mask(modes):
    m = 0
    for lm in modes:
        m |= MODE_BITS[tuple(lm)]
    return m


def real_dtype(precision):
    return torch.float64 if precision == LT_FP64 else torch.float32


class Context:
    """Owns one lt_ctx (plans, orbit tables, scratch) on one HIP device."""

    def __init__(self, device=0):
        self.device = device
        h = ctypes.c_void_p()
        _check(_lib.lt_ctx_create(device, ctypes.byref(h)))
        self.h = h

    def close(self):
        if self.h:
            _check(_lib.lt_ctx_destroy(self.h))
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- configuration helpers --------------------------------------------
    @staticmethod
    def grid(g):
        return Grid(g["t0"], g["dt"], g["n"])

    @staticmethod
    def wf_cfg(modes=((2, 2),), precessing=False, f_low=1e-4, f_ref=1e-4, precision=LT_FP64, coarse=1):
        """coarse=2: waveform on every second sample, linear in between (see lt_wf_cfg)."""
        return WfCfg(mode_mask(modes), int(precessing), f_low, f_ref, precision, int(coarse))

    @staticmethod
    def orbit(kind="static", arm=ARM_M, au=AU_M, phase0=0.0, t_ref=0.0, table=None):
        """kind "static", "kepler" or "table"; table = (t0, dt, pos [n][3][3] m, ltt [n][6] s)."""
        if kind == "table":
            import numpy as np
            t0, dt, pos, ltt = table
            pos = np.ascontiguousarray(pos, dtype=np.float64)
            ltt = np.ascontiguousarray(ltt, dtype=np.float64)
            if pos.ndim != 3 or pos.shape[1:] != (3, 3) or ltt.shape != (pos.shape[0], 6):
                raise ValueError("table: pos [n][3][3], ltt [n][6]")
            o = Orbit(LT_ORBIT_TABLE, arm, au, phase0, t_ref, pos.shape[0], t0, dt, pos.ctypes.data, ltt.ctypes.data)
            o._keep = (pos, ltt)          # the arrays live as long as the struct
            return o
        k = LT_ORBIT_STATIC_EQUAL if kind == "static" else LT_ORBIT_KEPLER
        return Orbit(k, arm, au, phase0, t_ref)

    @staticmethod
    def tdi_cfg(generation=15, channels=7, taps=2, out_xyz=False):
        return TdiCfg(generation, channels, taps, int(out_xyz))

    # -- entry points ---------------------------------------------------------
    def phenomt_modes(self, params, g, cfg, out, stream=None):
        """out: device FP64 [B][n_modes][n] complex, e.g. a float64 tensor [B, n_modes, n, 2]."""
        B, n = params.shape[0], int(g["n"])
        nm = bin(int(cfg.mode_mask) & 31).count("1")
        pp = _params_ptr(params, self.device)
        po = _ptr(out, "modes", torch.float64, numel=B * nm * n * 2, device=self.device)
        _check(_lib.lt_phenomt_modes(self.h, pp, B, ctypes.byref(cfg), ctypes.byref(self.grid(g)), po,
                                     _stream(stream)))
        return out

    def phenomt_polarizations(self, params, g, cfg, out, stream=None):
        """out: device FP64 [B][2][n] (h+, hx)."""
        B, n = params.shape[0], int(g["n"])
        pp = _params_ptr(params, self.device)
        po = _ptr(out, "hpc", torch.float64, numel=B * 2 * n, device=self.device)
        _check(_lib.lt_phenomt_polarizations(self.h, pp, B, ctypes.byref(cfg), ctypes.byref(self.grid(g)), po,
                                             _stream(stream)))
        return out

    def lisa_tdi_response(self, params, g, cfg, orbit, tdi, out, status=None, stream=None):
        """out: device [B][3][n] in real_dtype(cfg.precision); status: device int32 [B] or None."""
        B, n = params.shape[0], int(g["n"])
        pp = _params_ptr(params, self.device)
        po = _ptr(out, "out", real_dtype(cfg.precision), numel=B * 3 * n, device=self.device)
        ps = _ptr(status, "status", torch.int32, numel=B, device=self.device)
        _check(_lib.lt_lisa_tdi_response(self.h, pp, B, ctypes.byref(cfg), ctypes.byref(self.grid(g)),
                                         ctypes.byref(orbit), ctypes.byref(tdi), po, ps, _stream(stream)))
        return out

    def tdi_loglike(self, params, g, cfg, orbit, tdi, psd, data_aet, dd, logl, logl_full=None, status=None,
                    f_lo=3e-4, f_hi=0.02, stream=None, workspace=None):
        """psd: device FP64 [3][n/2+1]; data_aet: device [3][n] in real_dtype(cfg.precision); logl,
        logl_full: device FP64 [B] (logl may be None when logl_full is given); status: int32 [B];
        workspace: None (the context's scratch) or a device uint8 tensor (see workspace_size)."""
        B, n = params.shape[0], int(g["n"])
        pp = _params_ptr(params, self.device)
        P = _psd_struct(psd, n, f_lo, f_hi, self.device)
        D = Data(_ptr(data_aet, "data", real_dtype(cfg.precision), numel=3 * n, device=self.device), float(dd))
        pl = _ptr(logl, "logl", torch.float64, numel=B, device=self.device)
        pf = _ptr(logl_full, "logl_full", torch.float64, numel=B, device=self.device)
        ps = _ptr(status, "status", torch.int32, numel=B, device=self.device)
        pw = _ptr(workspace, "workspace", torch.uint8, shape=(None,), device=self.device)
        wb = workspace.numel() if workspace is not None else 0
        _check(_lib.lt_tdi_loglike(self.h, pp, B, ctypes.byref(cfg), ctypes.byref(self.grid(g)),
                                   ctypes.byref(orbit), ctypes.byref(tdi), ctypes.byref(P), ctypes.byref(D),
                                   pl, pf, ps, pw, wb, _stream(stream)))
        return logl

    def tdi_loglike_noalloc(self, params, g, cfg, orbit, tdi, psd, data_aet, dd, logl, logl_full=None, status=None,
                            f_lo=3e-4, f_hi=0.02, stream=None):
        """tdi_loglike with the library's fixed scratch: allocates nothing (the grid's FFT plan and
        the orbit's node table must already be in the context)."""
        B, n = params.shape[0], int(g["n"])
        pp = _params_ptr(params, self.device)
        P = _psd_struct(psd, n, f_lo, f_hi, self.device)
        D = Data(_ptr(data_aet, "data", real_dtype(cfg.precision), numel=3 * n, device=self.device), float(dd))
        pl = _ptr(logl, "logl", torch.float64, numel=B, device=self.device)
        pf = _ptr(logl_full, "logl_full", torch.float64, numel=B, device=self.device)
        ps = _ptr(status, "status", torch.int32, numel=B, device=self.device)
        _check(_lib.lt_tdi_loglike_noalloc(self.h, pp, B, ctypes.byref(cfg), ctypes.byref(self.grid(g)),
                                           ctypes.byref(orbit), ctypes.byref(tdi), ctypes.byref(P), ctypes.byref(D),
                                           pl, pf, ps, _stream(stream)))
        return logl

    def set_tuning(self, chunk=256, rotate=1, persistent=0, wg_per_cu=4):
        """Launch shape of the likelihood (lt_tuning); results do not depend on it."""
        t = Tuning(int(chunk), int(rotate), int(persistent), int(wg_per_cu))
        _check(_lib.lt_ctx_set_tuning(self.h, ctypes.byref(t)))

    def get_tuning(self):
        t = Tuning()
        _check(_lib.lt_ctx_get_tuning(self.h, ctypes.byref(t)))
        return t.as_dict()

    def autotune(self, params, g, cfg, orbit, tdi, psd, data_aet, dd, cache_path=None, reps=3, f_lo=3e-4, f_hi=0.02,
                 stream=None):
        """lt_autotune: the fastest launch shape for this workload (cached in cache_path); returns
        (tuning dict, ms per call or -1 when read from the cache)."""
        B, n = params.shape[0], int(g["n"])
        pp = _params_ptr(params, self.device)
        P = _psd_struct(psd, n, f_lo, f_hi, self.device)
        D = Data(_ptr(data_aet, "data", real_dtype(cfg.precision), numel=3 * n, device=self.device), float(dd))
        t, ms = Tuning(), ctypes.c_double()
        path = cache_path.encode() if cache_path else None
        _check(_lib.lt_autotune(self.h, pp, B, ctypes.byref(cfg), ctypes.byref(self.grid(g)), ctypes.byref(orbit),
                                ctypes.byref(tdi), ctypes.byref(P), ctypes.byref(D), path, int(reps), ctypes.byref(t),
                                ctypes.byref(ms), _stream(stream)))
        return t.as_dict(), ms.value

    def workspace_size(self, batch, g, cfg, tdi):
        """(bytes for full chunks, bytes for chunks of one template) of tdi_loglike's workspace."""
        full, one = ctypes.c_size_t(), ctypes.c_size_t()
        _check(_lib.lt_workspace_size(self.h, int(batch), ctypes.byref(cfg), ctypes.byref(self.grid(g)),
                                      ctypes.byref(tdi), ctypes.byref(full), ctypes.byref(one)))
        return int(full.value), int(one.value)

    def noise_inner(self, x, g, psd, out, channels=7, precision=LT_FP64, f_lo=3e-4, f_hi=0.02, stream=None):
        """x: device [B][3][n] in real_dtype(precision); out: device FP64 [B]."""
        B, n = x.shape[0], int(g["n"])
        px = _ptr(x, "x", real_dtype(precision), numel=B * 3 * n, device=self.device)
        P = _psd_struct(psd, n, f_lo, f_hi, self.device)
        po = _ptr(out, "out", torch.float64, numel=B, device=self.device)
        _check(_lib.lt_noise_inner(self.h, px, B, ctypes.byref(self.grid(g)), ctypes.byref(P), channels, precision,
                                   po, _stream(stream)))
        return out

    def rfft(self, x, dt, out, precision=LT_FP64, stream=None):
        """x: device [rows][n] in real_dtype(precision); out: [rows][n/2+1] complex of the same real type
        (e.g. a tensor [rows, n/2+1, 2])."""
        rdt = real_dtype(precision)
        px = _ptr(x, "x", rdt, shape=(None, None), device=self.device)
        rows, n = x.shape
        po = _ptr(out, "spec", rdt, numel=rows * (n // 2 + 1) * 2, device=self.device)
        _check(_lib.lt_rfft(self.h, px, rows, n, dt, precision, po, _stream(stream)))
        return out

    def profile_enable(self, on=True):
        _check(_lib.lt_profile_enable(self.h, int(on)))

    def profile_read(self, n=5):
        ms = (ctypes.c_double * n)()
        cnt = (ctypes.c_int64 * n)()
        _check(_lib.lt_profile_read(self.h, ms, cnt, n))
        return list(ms), list(cnt)


def psd_sangria(g, generation, out, arm=ARM_M, stream=None):
    """Fills out [3][n/2+1] (device FP64) with the PSD of Eqs. (2.14)-(2.15)."""
    po = _ptr(out, "S", torch.float64, numel=3 * (int(g["n"]) // 2 + 1))
    _check(_lib.lt_psd_sangria(ctypes.byref(Grid(g["t0"], g["dt"], g["n"])), generation, arm, po, _stream(stream)))
    return out


def _host(a, dtype=None):
    import numpy as np
    arr = np.ascontiguousarray(a, dtype=dtype or np.float64)
    return arr, ctypes.c_void_p(arr.ctypes.data)


class Sampler:
    """On-device parallel-tempered ensemble sampler (lt_sampler_*).

    target "tdi": likelihood = lt_tdi_loglike with (g, cfg, orbit, tdi, psd,
    data_aet, dd); target "gauss": means [n][dim], icov [dim][dim]."""

    def __init__(self, n_walkers, n_temps, dim, lo, hi, seed, target="tdi", param_kind="aligned10",
                 stretch_a=2.0, t_max=10.0, t_c=0.0, means=None, icov=None, g=None, cfg=None, orbit=None,
                 tdi=None, psd=None, data_aet=None, dd=0.0, f_lo=3e-4, f_hi=0.02, device=0):
        import numpy as np
        self.T, self.W, self.d = n_temps, n_walkers, dim
        kinds = {"aligned10": LT_PARAMS_ALIGNED10, "precessing14": LT_PARAMS_PRECESSING14, "raw": LT_PARAMS_RAW}
        self._lo, plo = _host(lo)
        self._hi, phi = _host(hi)
        c = SamplerCfg(n_walkers, n_temps, dim, kinds[param_kind],
                       LT_TARGET_TDI if target == "tdi" else LT_TARGET_GAUSS, stretch_a, t_max, seed, t_c, plo, phi,
                       0, None, None)
        args = [None] * 6
        if target == "gauss":
            self._m, pm = _host(np.atleast_2d(means))
            self._ic, pic = _host(icov)
            c.n_gauss, c.gauss_mean, c.gauss_icov = self._m.shape[0], pm, pic
        else:
            self._psd = _psd_struct(psd, int(g["n"]), f_lo, f_hi, device)
            self._data = Data(_ptr(data_aet, "data", real_dtype(cfg.precision), numel=3 * int(g["n"]),
                                   device=device), float(dd))
            self._keep = (psd, data_aet)
            args = [ctypes.byref(cfg), ctypes.byref(Grid(g["t0"], g["dt"], g["n"])), ctypes.byref(orbit),
                    ctypes.byref(tdi), ctypes.byref(self._psd), ctypes.byref(self._data)]
        h = ctypes.c_void_p()
        _check(_lib.lt_sampler_create(device, ctypes.byref(c), *args, ctypes.byref(h)))
        self.h = h

    def set_state(self, pos):
        import numpy as np
        arr, p = _host(np.reshape(pos, (self.T, self.W, self.d)))
        _check(_lib.lt_sampler_set_state(self.h, p))

    def step(self, n=1, stream=None):
        _check(_lib.lt_sampler_step(self.h, int(n), _stream(stream)))

    def state(self):
        import numpy as np
        pos = np.zeros((self.T, self.W, self.d))
        logl = np.zeros((self.T, self.W))
        logp = np.zeros((self.T, self.W))
        step = np.zeros(1, dtype=np.uint64)
        cnt = np.zeros(4, dtype=np.int64)
        _check(_lib.lt_sampler_get_state(self.h, pos.ctypes.data, logl.ctypes.data, logp.ctypes.data,
                                         step.ctypes.data, cnt.ctypes.data))
        return pos, logl, logp, int(step[0]), cnt

    def set_flow(self, flow):
        """Attach a Flow (None: detach) for independence moves on the cold rung."""
        _check(_lib.lt_sampler_set_flow(self.h, flow.h if flow is not None else None))
        self._flow = flow

    def set_flow_fold(self, index, period=math.pi, start=0.0):
        """Fold coordinate `index` (-1: none) into [start, start + period) for the flow move."""
        _check(_lib.lt_sampler_set_flow_fold(self.h, int(index), float(period), float(start)))

    def set_flow_walk(self, step):
        """Latent-space random walk of this step as the flow move (0: independence proposals)."""
        _check(_lib.lt_sampler_set_flow_walk(self.h, float(step)))

    def set_flow_mix(self, p_flow):
        """Probability that a step runs the flow move (1: every step; 0: the plain sampler)."""
        _check(_lib.lt_flow_set_mix(self.h, float(p_flow)))

    def set_flow_mixture(self, flow2, w_first):
        """Second flow of a two-component proposal w_first q1 + (1 - w_first) q2 (None: one flow)."""
        _check(_lib.lt_sampler_set_flow_mixture(self.h, flow2.h if flow2 is not None else None, float(w_first)))
        self._flow2 = flow2

    def set_flow_exclusive(self, on):
        """On steps that run the flow move, skip the cold rung's stretch moves (lt_sampler_set_flow_exclusive)."""
        _check(_lib.lt_sampler_set_flow_exclusive(self.h, int(bool(on))))

    def flow_counts(self):
        import numpy as np
        c = np.zeros(2, dtype=np.int64)
        _check(_lib.lt_sampler_flow_counts(self.h, c.ctypes.data))
        return int(c[0]), int(c[1])

    def close(self):
        if self.h:
            _check(_lib.lt_sampler_destroy(self.h))
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def fisher(ctx, x0, param_kind, t_c, steps, g, cfg, orbit, tdi, psd, f_lo=3e-4, f_hi=0.02):
    """Fisher matrix in the sampling coordinates (lt_fisher); psd: device [3][n/2+1]."""
    import numpy as np
    kinds = {"aligned10": LT_PARAMS_ALIGNED10, "precessing14": LT_PARAMS_PRECESSING14}
    x, px = _host(x0)
    st, ps = _host(steps)
    d = x.size
    G = np.zeros((d, d))
    P = _psd_struct(psd, int(g["n"]), f_lo, f_hi, ctx.device)
    _check(_lib.lt_fisher(ctx.h, px, kinds[param_kind], float(t_c), ps, ctypes.byref(cfg),
                          ctypes.byref(Grid(g["t0"], g["dt"], g["n"])), ctypes.byref(orbit), ctypes.byref(tdi),
                          ctypes.byref(P), G.ctypes.data))
    return G


def fisher_draw(x0, gamma, lo, hi, count, seed, reg=1e-10):
    """count draws from N(x0, gamma^-1) inside [lo, hi] (lt_fisher_draw), host [count][d]."""
    import numpy as np
    x, px = _host(x0)
    G, pg = _host(gamma)
    l, pl = _host(lo)
    h, ph = _host(hi)
    out = np.zeros((int(count), x.size))
    _check(_lib.lt_fisher_draw(px, pg, x.size, pl, ph, int(count), int(seed), float(reg), out.ctypes.data))
    return out


class Flow:
    """RealNVP-style flow proposal (lt_flow_*); parameter vector layout as in include/lisatd.h."""

    def __init__(self, dim, n_layers=8, hidden=256, max_batch=4096, device=0):
        h = ctypes.c_void_p()
        _check(_lib.lt_flow_create(device, dim, n_layers, hidden, max_batch, ctypes.byref(h)))
        self.h, self.d, self.L, self.H, self.max_batch = h, dim, n_layers, hidden, max_batch
        self.device = device

    @property
    def num_params(self):
        return int(_lib.lt_flow_num_params(self.h))

    def set_params(self, params, mu, sigma):
        import numpy as np
        w, pw = _host(params, np.float32)
        if w.size != self.num_params:
            raise ValueError("expected %d parameters" % self.num_params)
        m, pm = _host(mu)
        s, ps = _host(sigma)
        _check(_lib.lt_flow_set_params(self.h, pw, pm, ps))

    def set_whitening(self, mu, L):
        """x = L u + mu with L lower triangular (e.g. the Cholesky factor of a sample covariance)."""
        import numpy as np
        m, pm = _host(mu)
        Lh, pl = _host(np.reshape(L, (self.d, self.d)))
        _check(_lib.lt_flow_set_whitening(self.h, pm, pl))

    def get_params(self):
        import numpy as np
        w = np.zeros(self.num_params, dtype=np.float32)
        _check(_lib.lt_flow_get_params(self.h, w.ctypes.data))
        return w

    def _rows(self, x, name="x"):
        """Pointer of device FP64 rows [n][dim] on the flow's device."""
        return _ptr(x, name, torch.float64, shape=(None, self.d), device=self.device)

    def log_prob(self, x, out=None, stream=None):
        px = self._rows(x)
        out = out if out is not None else torch.empty(x.shape[0], dtype=torch.float64, device=x.device)
        po = _ptr(out, "logq", torch.float64, numel=x.shape[0], device=self.device)
        _check(_lib.lt_flow_log_prob(self.h, px, x.shape[0], po, _stream(stream)))
        return out

    def sample(self, z, stream=None):
        pz = self._rows(z, "z")
        x = torch.empty_like(z)
        logq = torch.empty(z.shape[0], dtype=torch.float64, device=z.device)
        _check(_lib.lt_flow_sample(self.h, pz, z.shape[0], _ptr(x), _ptr(logq), _stream(stream)))
        return x, logq

    def loss_grad(self, x):
        import numpy as np
        px = self._rows(x)
        logq = np.zeros(x.shape[0])
        g = np.zeros(self.num_params, dtype=np.float32)
        _check(_lib.lt_flow_loss_grad(self.h, px, x.shape[0], logq.ctypes.data, g.ctypes.data))
        return logq, g

    def train(self, x, steps, batch, lr, stream=None):
        px = self._rows(x)
        _check(_lib.lt_flow_train(self.h, px, x.shape[0], int(steps), int(batch), float(lr), _stream(stream)))

    def close(self):
        if self.h:
            _check(_lib.lt_flow_destroy(self.h))
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def flow_init_params(d, n_layers, hidden, seed):
    """Starting weights: hidden layers' weights and biases uniform in +-0.5 / sqrt(fan-in), zero
    output layer (the identity flow).  Smaller than He-normal on purpose: trained on a window of
    a sampler's chain, a flow started from He-normal weights generalises worse to the next window
    (independence-move acceptance about 13 % against 30 % on the precessing posterior)."""
    import numpy as np
    rng = np.random.default_rng(seed)
    da, db = d // 2, d - d // 2
    ua, uh = 0.5 / math.sqrt(da), 0.5 / math.sqrt(hidden)
    parts = []
    for _ in range(n_layers):
        parts += [rng.uniform(-ua, ua, hidden * da), rng.uniform(-ua, ua, hidden),
                  rng.uniform(-uh, uh, hidden * hidden), rng.uniform(-uh, uh, hidden),
                  np.zeros(2 * db * hidden), np.zeros(2 * db)]
    return np.concatenate(parts).astype(np.float32)


def flow_pack(P):
    """Oracle-style parameter list (dicts W1, b1, W2, b2, W3, b3 per layer) -> FP32 vector."""
    import numpy as np
    parts = []
    for p in P:
        for k in ("W1", "b1", "W2", "b2", "W3", "b3"):
            parts.append(np.asarray(p[k], dtype=np.float32).ravel())
    return np.concatenate(parts)


def flow_unpack(w, d, n_layers, hidden):
    """FP32 vector -> list of per-layer dicts (float64 arrays)."""
    import numpy as np
    da, db = d // 2, d - d // 2
    shapes = (("W1", (hidden, da)), ("b1", (hidden,)), ("W2", (hidden, hidden)), ("b2", (hidden,)),
              ("W3", (2 * db, hidden)), ("b3", (2 * db,)))
    out, off = [], 0
    for _ in range(n_layers):
        p = {}
        for k, shp in shapes:
            n = int(np.prod(shp))
            p[k] = np.asarray(w[off:off + n], dtype=np.float64).reshape(shp)
            off += n
        out.append(p)
    if off != len(w):
        raise ValueError("parameter vector length does not match the flow shape")
    return out
