"""Thin ctypes binding of libme.so (include/me.h): argument marshalling only.

Every step of the matrix-element path runs in the HIP kernels of libme.so; torch is used
for device memory and streams.  Loading fails loudly if the library was not built -- there
is no fallback.
"""
import ctypes
import os

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libme.so")

ME_FP64, ME_MIXED_FP16, ME_MIXED_BF16 = 0, 1, 2
ME_OPT_FUSED_COLOUR = 1
PRECISIONS = {"fp64": ME_FP64, "mixed_fp16": ME_MIXED_FP16, "mixed_bf16": ME_MIXED_BF16}
ME_OK = 0
PROCESSES = ["ee_mumu", "gg_tt", "gg_ttg", "gg_ttgg", "gg_ttggg", "gg_gg", "ee_mumu_z"]


class MeError(RuntimeError):
    pass


class MeInfo(ctypes.Structure):
    _fields_ = [("n_par", ctypes.c_int), ("n_diagrams", ctypes.c_int), ("n_amplitudes", ctypes.c_int),
                ("n_colors", ctypes.c_int), ("n_hel", ctypes.c_int), ("n_good_hel", ctypes.c_int),
                ("precision", ctypes.c_int), ("avg_factor", ctypes.c_double), ("sym_factor", ctypes.c_double),
                ("flops_amp_lane", ctypes.c_double), ("flops_amp_exec_lane", ctypes.c_double),
                ("n_partial_slots", ctypes.c_int), ("flops_colour_lane", ctypes.c_double),
                ("bytes_resident", ctypes.c_int64), ("bytes_per_event_scratch", ctypes.c_int64),
                ("chunk_events", ctypes.c_int64), ("n_order", ctypes.c_int), ("helicity_groups", ctypes.c_int),
                ("lines_per_diagram", ctypes.c_int), ("fused_colour", ctypes.c_int)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


EXPORTS = ["me_create", "me_destroy", "me_info", "me_last_error", "rambo_momenta", "me_sigma",
           "me_sigma_noalloc", "me_reserve_scratch", "me_release_scratch", "me_scratch_bytes", "me_sigma_hel", "me_sigma_select", "me_sigma_alphas", "me_sigma_channel", "me_diagrams", "me_colour_flows", "me_good_helicities", "me_helicity_ratios",
           "me_profile", "me_set_option"]

_lib = None


def load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise MeError(f"{LIB_PATH} is not built: run __graft_entry__.build() (hipcc for gfx950)")
    L = ctypes.CDLL(LIB_PATH)
    vp, D = ctypes.c_void_p, ctypes.POINTER(ctypes.c_double)
    L.me_create.restype = vp
    L.me_create.argtypes = [ctypes.c_char_p, D, ctypes.c_int, D, ctypes.c_int, ctypes.c_int, vp]
    L.me_destroy.argtypes = [vp]
    L.me_destroy.restype = None
    L.me_info.argtypes = [vp, ctypes.POINTER(MeInfo)]
    L.me_last_error.restype = ctypes.c_char_p
    L.rambo_momenta.argtypes = [vp, ctypes.c_uint64, ctypes.c_double, ctypes.c_int64, ctypes.c_int64, vp, vp]
    L.me_sigma.argtypes = [vp, vp, ctypes.c_int64, vp, vp]
    L.me_sigma_noalloc.argtypes = [vp, vp, ctypes.c_int64, vp, vp]
    L.me_reserve_scratch.argtypes = [vp, ctypes.c_int64, vp]
    L.me_release_scratch.argtypes = [vp, vp]
    L.me_scratch_bytes.argtypes = [vp]
    L.me_scratch_bytes.restype = ctypes.c_int64
    L.me_sigma_hel.argtypes = [vp, vp, ctypes.c_int64, vp, vp, vp]
    L.me_sigma_select.argtypes = [vp, vp, ctypes.c_int64, vp, vp, vp, vp, vp, vp]
    L.me_colour_flows.argtypes = [vp, ctypes.POINTER(ctypes.c_int)]
    L.me_sigma_alphas.argtypes = [vp, vp, ctypes.c_int64, vp, vp, vp]
    L.me_sigma_channel.argtypes = [vp, vp, ctypes.c_int64, vp, vp, vp]
    L.me_diagrams.argtypes = [vp, ctypes.POINTER(ctypes.c_int)]
    L.me_good_helicities.argtypes = [vp, ctypes.POINTER(ctypes.c_byte)]
    L.me_helicity_ratios.argtypes = [vp, D]
    L.me_profile.argtypes = [vp, ctypes.c_int, D, D, ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int64)]
    L.me_set_option.argtypes = [vp, ctypes.c_int, ctypes.c_int]
    _lib = L
    return L


def last_error():
    return load().me_last_error().decode()


def _check(rc, what):
    if rc != ME_OK:
        raise MeError(f"{what} failed ({rc}): {last_error()}")


def _stream_ptr(stream):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


class Process:
    """One process handle: ``rambo`` makes device momenta, ``sigma`` the averaged |M|^2."""

    def __init__(self, name, m_top=173.0, alpha_em=1.0 / 132.507, alpha_s=0.118, precision="fp64",
                 stream=None):
        L = load()
        self.name = name
        masses = (ctypes.c_double * 1)(m_top)
        coup = (ctypes.c_double * 2)(alpha_em, alpha_s)
        prec = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
        h = L.me_create(name.encode(), masses, 1, coup, 2, prec, _stream_ptr(stream))
        if not h:
            raise MeError(f"me_create({name}) failed: {last_error()}")
        self._h = ctypes.c_void_p(h)
        self.info = self._info()
        self.n_par = self.info["n_par"]

    def _info(self):
        i = MeInfo()
        _check(load().me_info(self._h, ctypes.byref(i)), "me_info")
        return i.as_dict()

    def close(self):
        if getattr(self, "_h", None):
            load().me_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def rambo(self, seed, sqrt_s, n_evt, evt0=0, out=None, stream=None):
        import torch
        if out is None:
            out = torch.empty((n_evt, self.n_par, 4), dtype=torch.float64, device="cuda")
        _check(load().rambo_momenta(self._h, seed, sqrt_s, evt0, n_evt, ctypes.c_void_p(out.data_ptr()),
                                    _stream_ptr(stream)), "rambo_momenta")
        return out

    def sigma(self, momenta, out=None, per_helicity=False, stream=None):
        import torch
        assert momenta.is_cuda and momenta.dtype == torch.float64 and momenta.is_contiguous()
        n = momenta.shape[0]
        assert momenta.shape[1:] == (self.n_par, 4)
        if out is None:
            out = torch.empty(n, dtype=torch.float64, device=momenta.device)
        if per_helicity:
            hel = torch.empty((n, self.info["n_good_hel"]), dtype=torch.float64, device=momenta.device)
            _check(load().me_sigma_hel(self._h, ctypes.c_void_p(momenta.data_ptr()), n,
                                       ctypes.c_void_p(out.data_ptr()), ctypes.c_void_p(hel.data_ptr()),
                                       _stream_ptr(stream)), "me_sigma_hel")
            return out, hel
        _check(load().me_sigma(self._h, ctypes.c_void_p(momenta.data_ptr()), n, ctypes.c_void_p(out.data_ptr()),
                               _stream_ptr(stream)), "me_sigma")
        return out

    def sigma_noalloc(self, momenta, out, stream=None):
        """me_sigma_noalloc: as sigma, with the library's static scratch (allocates nothing;
        out must be given)"""
        import torch
        assert momenta.is_cuda and momenta.dtype == torch.float64 and momenta.is_contiguous()
        n = momenta.shape[0]
        assert momenta.shape[1:] == (self.n_par, 4)
        assert out.is_cuda and out.dtype == torch.float64 and out.is_contiguous() and out.shape == (n,)
        _check(load().me_sigma_noalloc(self._h, ctypes.c_void_p(momenta.data_ptr()), n,
                                       ctypes.c_void_p(out.data_ptr()), _stream_ptr(stream)), "me_sigma_noalloc")
        return out

    def reserve_scratch(self, n_evt, stream=None):
        """allocate now the scratch of every me_sigma call of at most n_evt events on `stream`"""
        _check(load().me_reserve_scratch(self._h, int(n_evt), _stream_ptr(stream)), "me_reserve_scratch")

    def release_scratch(self, stream=None):
        _check(load().me_release_scratch(self._h, _stream_ptr(stream)), "me_release_scratch")

    def scratch_bytes(self):
        n = load().me_scratch_bytes(self._h)
        if n < 0:
            raise MeError(f"me_scratch_bytes failed: {last_error()}")
        return n

    def select(self, momenta, r_hel, r_col, stream=None):
        """(|M|^2, helicity-combination index, colour-flow index) per event, the two choices
        drawn with the caller's uniforms r_hel, r_col (device float64 [n_evt])"""
        import torch
        assert momenta.is_cuda and momenta.dtype == torch.float64 and momenta.is_contiguous()
        n = momenta.shape[0]
        assert momenta.shape[1:] == (self.n_par, 4)
        for r in (r_hel, r_col):
            assert r.is_cuda and r.dtype == torch.float64 and r.is_contiguous() and r.shape == (n,)
        out = torch.empty(n, dtype=torch.float64, device=momenta.device)
        hel = torch.empty(n, dtype=torch.int32, device=momenta.device)
        col = torch.empty(n, dtype=torch.int32, device=momenta.device)
        _check(load().me_sigma_select(self._h, ctypes.c_void_p(momenta.data_ptr()), n,
                                      ctypes.c_void_p(r_hel.data_ptr()), ctypes.c_void_p(r_col.data_ptr()),
                                      ctypes.c_void_p(out.data_ptr()), ctypes.c_void_p(hel.data_ptr()),
                                      ctypes.c_void_p(col.data_ptr()), _stream_ptr(stream)), "me_sigma_select")
        return out, hel, col

    def sigma_alphas(self, momenta, alpha_s, out=None, stream=None):
        """averaged |M|^2 with the strong coupling alpha_s[e] (device float64 [n_evt]) per event"""
        import torch
        assert momenta.is_cuda and momenta.dtype == torch.float64 and momenta.is_contiguous()
        n = momenta.shape[0]
        assert momenta.shape[1:] == (self.n_par, 4)
        assert alpha_s.is_cuda and alpha_s.dtype == torch.float64 and alpha_s.is_contiguous() and alpha_s.shape == (n,)
        if out is None:
            out = torch.empty(n, dtype=torch.float64, device=momenta.device)
        _check(load().me_sigma_alphas(self._h, ctypes.c_void_p(momenta.data_ptr()), n,
                                      ctypes.c_void_p(alpha_s.data_ptr()), ctypes.c_void_p(out.data_ptr()),
                                      _stream_ptr(stream)), "me_sigma_alphas")
        return out

    def sigma_channel(self, momenta, channel, out=None, stream=None):
        """averaged |M|^2 times the single-diagram weight of channel[e] (device int32 [n_evt],
        -1: none)"""
        import torch
        assert momenta.is_cuda and momenta.dtype == torch.float64 and momenta.is_contiguous()
        n = momenta.shape[0]
        assert momenta.shape[1:] == (self.n_par, 4)
        assert channel.is_cuda and channel.dtype == torch.int32 and channel.is_contiguous() and channel.shape == (n,)
        if out is None:
            out = torch.empty(n, dtype=torch.float64, device=momenta.device)
        _check(load().me_sigma_channel(self._h, ctypes.c_void_p(momenta.data_ptr()), n,
                                       ctypes.c_void_p(channel.data_ptr()), ctypes.c_void_p(out.data_ptr()),
                                       _stream_ptr(stream)), "me_sigma_channel")
        return out

    def diagrams(self):
        """internal lines of every Feynman diagram (tuples of particle masks, side without particle 0)"""
        k = self.info["lines_per_diagram"]
        nd = self.info["n_diagrams"]
        buf = (ctypes.c_int * (nd * k))()
        n = load().me_diagrams(self._h, buf)
        if n < 0:
            raise MeError(f"me_diagrams failed: {last_error()}")
        return [tuple(x for x in buf[d * k:(d + 1) * k] if x) for d in range(n)]

    def colour_flows(self):
        """gluon ordering of every colour flow (list of tuples, flow order of the jamps)"""
        nc = self.info["n_colors"]
        buf = (ctypes.c_int * (nc * 8))()
        n = load().me_colour_flows(self._h, buf)
        if n < 0:
            raise MeError(f"me_colour_flows failed: {last_error()}")
        k = self.info["n_order"]
        return [tuple(buf[f * k:(f + 1) * k]) for f in range(n)]

    def profile(self, enable):
        """switch launch timing on/off; returns what was recorded since the last call:
        (ms amplitude kernel, ms colour sum, launches of each)"""
        a, c = ctypes.c_double(), ctypes.c_double()
        na, nc = ctypes.c_int64(), ctypes.c_int64()
        _check(load().me_profile(self._h, int(enable), ctypes.byref(a), ctypes.byref(c), ctypes.byref(na),
                                 ctypes.byref(nc)), "me_profile")
        return a.value, c.value, na.value, nc.value

    def set_fused_colour(self, enable):
        """colour sum inside the FP64 amplitude kernel where the process has one (default on)"""
        _check(load().me_set_option(self._h, ME_OPT_FUSED_COLOUR, int(bool(enable))), "me_set_option")
        self.info = self._info()

    def good_helicities(self):
        n = self.info["n_good_hel"]
        buf = (ctypes.c_byte * (n * self.n_par))()
        load().me_good_helicities(self._h, buf)
        return [tuple(buf[k * self.n_par:(k + 1) * self.n_par]) for k in range(n)]

    def good_helicities_index(self):
        """helicity-combination index of every good helicity (particle i's bit at 2^(n_par-1-i))"""
        return [sum(((l + 1) // 2) << (self.n_par - 1 - i) for i, l in enumerate(c)) for c in self.good_helicities()]

    def helicity_ratios(self):
        n = self.info["n_hel"]
        buf = (ctypes.c_double * n)()
        load().me_helicity_ratios(self._h, buf)
        return list(buf)
