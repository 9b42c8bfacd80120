"""Torch-tensor wrappers over the C ABI (include/smartap.h).

Tensors only carry device memory; every step runs in libsmartap.so. Work is
queued on torch's current stream of the context's device.
"""
from __future__ import annotations

import ctypes as C

import numpy as np
import torch

from . import lib as L

L.load()  # fail loudly at import when the library is missing


def _stream(device):
    return C.c_void_p(torch.cuda.current_stream(device).cuda_stream)


def _ptr(t):
    return C.c_void_p(0 if t is None else t.data_ptr())


def _buf(t, device, dtype, numel, what):
    """Pointer of a caller buffer that a kernel reads or writes whole: it
    must be a contiguous tensor on the context's device with the element
    type and at least the element count the call uses."""
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{what} must be a torch tensor")
    if t.device != device:
        raise ValueError(f"{what} is on {t.device}, the context is on {device}")
    if t.dtype != dtype:
        raise ValueError(f"{what} has dtype {t.dtype}, expected {dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{what} must be contiguous")
    if t.numel() < numel:
        raise ValueError(f"{what} holds {t.numel()} elements, the call uses {numel}")
    return _ptr(t)


def _dev(t, device, dtype):
    t = torch.as_tensor(t)
    return t.to(device=device, dtype=dtype).contiguous()


class Context:
    def __init__(self, device: int = 0):
        self.lib = L.load()
        self.device = torch.device("cuda", device)
        h = C.c_void_p()
        L.check(self.lib.smart_init(device, C.byref(h)))
        self.h = h
        self._filters = {}

    def close(self):
        if self.h:
            self.lib.smart_finalize(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- filters -------------------------------------------------------------
    def filter(self, kind: int, params=None) -> int:
        key = (kind, None if params is None else tuple(float(p) for p in params))
        if key in self._filters:
            return self._filters[key]
        fid = C.c_int()
        if params is None:
            L.check(self.lib.smart_filter_define(self.h, kind, None, 0, C.byref(fid)))
        else:
            arr = (C.c_double * len(params))(*params)
            L.check(self.lib.smart_filter_define(self.h, kind, arr, len(params), C.byref(fid)))
        self._filters[key] = fid.value
        return fid.value

    def filter_table(self, fid: int) -> np.ndarray:
        n = C.c_int()
        L.check(self.lib.smart_filter_table(self.h, fid, None, C.byref(n)))
        buf = (C.c_float * (4 * n.value))()
        L.check(self.lib.smart_filter_table(self.h, fid, buf, C.byref(n)))
        return np.frombuffer(buf, dtype=np.float32).reshape(n.value, 4).copy()

    def filter_pieces(self, fid: int, theta_ap: float = 0.0) -> np.ndarray:
        """The filter's cubic pieces as the kernels read them ([n, 4] float64;
        see smart_filter_pieces): the table in x for theta_ap = 0, else the
        general walk's table in sin(theta) for that aperture."""
        n = C.c_int()
        L.check(self.lib.smart_filter_pieces(self.h, fid, float(theta_ap), None, C.byref(n)))
        buf = (C.c_double * (4 * n.value))()
        L.check(self.lib.smart_filter_pieces(self.h, fid, float(theta_ap), buf, C.byref(n)))
        return np.frombuffer(buf, dtype=np.float64).reshape(n.value, 4).copy()

    # -- data ----------------------------------------------------------------
    def bin_galaxies(self, ra, dec, g1, g2, w=None, nside_bin=4096, pixel_sums=False) -> "Data":
        d = self.device
        ra = _dev(ra, d, torch.float64)
        dec = _dev(dec, d, torch.float64)
        g1 = _dev(g1, d, torch.float32)
        g2 = _dev(g2, d, torch.float32)
        w = None if w is None else _dev(w, d, torch.float32)
        h = C.c_void_p()
        L.check(self.lib.smart_bin_galaxies(self.h, ra.numel(), _ptr(ra), _ptr(dec), _ptr(g1), _ptr(g2), _ptr(w),
                                            nside_bin, 1 if pixel_sums else 0, _stream(d), C.byref(h)))
        return Data(self, h)

    def pixel_map(self, nside, pix, W, G1, G2, E2) -> "Data":
        d = self.device
        pix = _dev(pix, d, torch.int64)
        cols = [_dev(x, d, torch.float32) for x in (W, G1, G2, E2)]
        h = C.c_void_p()
        L.check(self.lib.smart_pixel_map(self.h, nside, pix.numel(), _ptr(pix), *[_ptr(c) for c in cols],
                                         _stream(d), C.byref(h)))
        return Data(self, h)

    def plan(self, data: "Data", variant: int, nside_out: int, out_pix, thetas, filters,
             precision: int = L.PREC_FP32_GEO64) -> "Plan":
        d = self.device
        out_pix = _dev(out_pix, d, torch.int64)
        thetas = list(thetas)
        filters = list(filters)
        th = (C.c_double * len(thetas))(*thetas)
        fi = (C.c_int * len(filters))(*filters)
        h = C.c_void_p()
        L.check(self.lib.smart_plan_create(self.h, data.h, variant, nside_out, out_pix.numel(), _ptr(out_pix),
                                           len(thetas), th, fi, precision, _stream(d), C.byref(h)))
        return Plan(self, h, data, out_pix.numel(), len(thetas), precision)

    def noise_angles(self, seed: int, r_first: int, n_real: int, n_src: int, out=None):
        """Counter-based realisation angles (see smart_noise_angles): [n_real][n_src] float32."""
        if out is None:
            out = torch.empty(n_real, n_src, dtype=torch.float32, device=self.device)
        p = _buf(out, self.device, torch.float32, n_real * n_src, "out")
        L.check(self.lib.smart_noise_angles(self.h, seed, r_first, n_real, n_src, p, _stream(self.device)))
        return out

    def noise_galaxy_angles(self, seed: int, r_first: int, n_real: int, n_gal: int, out=None):
        """Galaxy-level angles (see smart_noise_galaxy_angles): [n_real][n_gal] float32."""
        if out is None:
            out = torch.empty(n_real, n_gal, dtype=torch.float32, device=self.device)
        p = _buf(out, self.device, torch.float32, n_real * n_gal, "out")
        L.check(self.lib.smart_noise_galaxy_angles(self.h, seed, r_first, n_real, n_gal, p, _stream(self.device)))
        return out

    def detect_peaks(self, nside: int, pix, values, threshold: float = float("-inf"), noise_sd=None):
        """Detections of a map (see smart_detect_peaks): increasing int64 pixels."""
        d = self.device
        pix = _dev(pix, d, torch.int64)
        val = _dev(values, d, torch.float64)
        sd = None if noise_sd is None else _dev(noise_sd, d, torch.float64)
        n = pix.numel()
        if val.numel() != n or (sd is not None and sd.numel() != n):
            raise ValueError("pixels, values and noise must have the same length")
        out = torch.empty(max(n, 1), dtype=torch.int64, device=d)
        cnt = C.c_int64()
        L.check(self.lib.smart_detect_peaks(self.h, nside, n, _ptr(pix), _ptr(val), _ptr(sd), float(threshold),
                                            _ptr(out), C.byref(cnt), _stream(d)))
        return out[: cnt.value]

    def mixed_batch(self, plans, norms, outs, noalloc=False):
        """All plans in one persistent launch (smart_mixed_batch, or with
        noalloc=True smart_mixed_batch_noalloc: no device allocation)."""
        n = len(plans)
        if len(norms) != n or len(outs) != n:
            raise ValueError("plans, norms and outs must have the same length")
        ph = (C.c_void_p * n)(*[p.h.value for p in plans])
        nh = (C.c_int * n)(*norms)
        oh = (C.c_void_p * n)(*[_buf(o, self.device, p.out_dtype, p.n_scales * 5 * p.n_out, "out").value or 0
                                for p, o in zip(plans, outs)])
        fn = self.lib.smart_mixed_batch_noalloc if noalloc else self.lib.smart_mixed_batch
        L.check(fn(self.h, n, ph, nh, oh, _stream(self.device)))


class Data:
    def __init__(self, ctx: Context, h):
        self.ctx = ctx
        self.h = h

    def info(self):
        n = C.c_int64()
        ns = C.c_int()
        pf = C.c_int64()
        nd = C.c_int64()
        rb = C.c_double()
        L.check(self.ctx.lib.smart_data_info(self.h, C.byref(n), C.byref(ns), C.byref(pf), C.byref(nd), C.byref(rb)))
        return {"n_gal": n.value, "nside": ns.value, "pix_first": pf.value, "n_dense": nd.value, "r_bin": rb.value}

    def barycentre(self) -> "Data":
        """sphS_pixB data: the occupied pixels at their galaxies' barycentres (see smart_barycentre_map)."""
        h = C.c_void_p()
        L.check(self.ctx.lib.smart_barycentre_map(self.h, _stream(self.ctx.device), C.byref(h)))
        return Data(self.ctx, h)

    def n_sources(self) -> int:
        """Number of occupied source pixels (columns of the realisation angles)."""
        n = C.c_int64()
        L.check(self.ctx.lib.smart_data_sources(self.h, C.byref(n), None, None))
        return n.value

    def sources(self):
        """Occupied source pixels of the pixel variant (device int64 tensor)."""
        n = C.c_int64()
        L.check(self.ctx.lib.smart_data_sources(self.h, C.byref(n), None, None))
        t = torch.empty(n.value, dtype=torch.int64, device=self.ctx.device)
        L.check(self.ctx.lib.smart_data_sources(self.h, C.byref(n), _ptr(t), _stream(self.ctx.device)))
        return t

    def export(self, order=False, offsets=False, sums=False):
        inf = self.info()
        d = self.ctx.device
        o = torch.empty(inf["n_gal"], dtype=torch.int64, device=d) if order else None
        f = torch.empty(12 * inf["nside"] ** 2 + 1, dtype=torch.int64, device=d) if offsets else None
        s = torch.empty(inf["n_dense"], 4, dtype=torch.float32, device=d) if sums else None
        L.check(self.ctx.lib.smart_data_export(self.h, _ptr(o), _ptr(f), _ptr(s), _stream(d)))
        return o, f, s

    def free(self):
        if self.h:
            self.ctx.lib.smart_data_free(self.h)
            self.h = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


class Plan:
    def __init__(self, ctx, h, data, n_out, n_scales, precision):
        self.ctx = ctx
        self.h = h
        self.data = data  # keep alive
        self.n_out = n_out
        self.n_scales = n_scales
        self.precision = precision

    @property
    def out_dtype(self):
        """Element type of the maps of run() and mixed batches."""
        return torch.float64 if self.precision in (L.PREC_FP64, L.PREC_FP32_OUT64) else torch.float32

    def empty_out(self):
        return torch.empty(self.n_scales, 5, self.n_out, dtype=self.out_dtype, device=self.ctx.device)

    def run(self, norm: int, out=None):
        if out is None:
            out = self.empty_out()
        p = _buf(out, self.ctx.device, self.out_dtype, self.n_scales * 5 * self.n_out, "out")
        L.check(self.ctx.lib.smart_run(self.h, norm, p, _stream(self.ctx.device)))
        return out

    def last_pairs(self) -> float:
        v = C.c_double()
        L.check(self.ctx.lib.smart_last_pairs(self.h, _stream(self.ctx.device), C.byref(v)))
        return v.value

    def tiles(self, scale: int = 0):
        """(belt items as an [n, 2] int32 tensor of (list position, length), general tile indices)."""
        nb, ng = C.c_int(), C.c_int()
        L.check(self.ctx.lib.smart_plan_tiles(self.h, scale, C.byref(nb), C.byref(ng), None, None, None))
        b = torch.empty(max(nb.value, 1), 2, dtype=torch.int32, device=self.ctx.device)
        g = torch.empty(max(ng.value, 1), dtype=torch.int32, device=self.ctx.device)
        L.check(self.ctx.lib.smart_plan_tiles(self.h, scale, C.byref(nb), C.byref(ng), _ptr(b), _ptr(g),
                                              _stream(self.ctx.device)))
        return b[: nb.value], g[: ng.value]

    def autotune(self, budget_ms: int = 2000, cache_path=None):
        """Measure and keep the fastest launch choices of every scale (see smart_autotune)."""
        path = None if cache_path is None else str(cache_path).encode()
        L.check(self.ctx.lib.smart_autotune(self.h, int(budget_ms), path, _stream(self.ctx.device)))

    def galaxy_form(self, scale: int = 0) -> int:
        """Galaxy kernel form of a scale (GAL_LANE or GAL_WAVE; galaxy-variant FP32 plans)."""
        f = C.c_int()
        L.check(self.ctx.lib.smart_plan_galaxy_form(self.h, scale, C.byref(f)))
        return f.value

    def set_galaxy_form(self, scale: int, form: int):
        L.check(self.ctx.lib.smart_plan_set_galaxy_form(self.h, scale, form))

    def set_timing(self, enable: bool = True):
        L.check(self.ctx.lib.smart_plan_set_timing(self.h, 1 if enable else 0))

    def kernel_ms(self, scale: int = 0):
        """(belt kernel ms, general kernel ms) of the last timed run."""
        b, g = C.c_double(), C.c_double()
        L.check(self.ctx.lib.smart_plan_kernel_ms(self.h, scale, C.byref(b), C.byref(g)))
        return b.value, g.value

    def noise_batch(self, u, n_real: int, norm: int, precision: int, out=None):
        """Pixel-level realisations: u is [n_real][n_src] (see Data.sources)."""
        dev = self.ctx.device
        if out is None:
            out = torch.empty(self.n_scales, n_real, 2, self.n_out, dtype=torch.float32, device=dev)
        pu = _buf(u, dev, torch.float32, n_real * self.data.n_sources(), "u")
        po = _buf(out, dev, torch.float32, self.n_scales * n_real * 2 * self.n_out, "out")
        L.check(self.ctx.lib.smart_noise_batch(self.h, pu, n_real, norm, precision, po, _stream(dev)))
        return out

    def noise_seeded(self, seed: int, r_first: int, n_real: int, norm: int, precision: int, moments=False,
                     out=None):
        """Realisations with device-drawn angles (see smart_noise_seeded). Maps:
        [n_scales][n_real][2][n_out] float32; moments: [n_scales][4][n_out]
        float64 sums of E, E^2, B, B^2, added to `out` (zeros when None)."""
        dev = self.ctx.device
        if moments:
            if out is None:
                out = torch.zeros(self.n_scales, 4, self.n_out, dtype=torch.float64, device=dev)
            po = _buf(out, dev, torch.float64, self.n_scales * 4 * self.n_out, "out")
        else:
            if out is None:
                out = torch.empty(self.n_scales, n_real, 2, self.n_out, dtype=torch.float32, device=dev)
            po = _buf(out, dev, torch.float32, self.n_scales * n_real * 2 * self.n_out, "out")
        L.check(self.ctx.lib.smart_noise_seeded(self.h, seed, r_first, n_real, norm, precision, 1 if moments else 0,
                                                po, _stream(dev)))
        return out

    def noise_galaxy_batch(self, u, n_real: int, norm: int, out=None):
        """Galaxy-level realisations: u is [n_real][n_gal] in catalogue order."""
        dev = self.ctx.device
        if out is None:
            out = torch.empty(self.n_scales, n_real, 2, self.n_out, dtype=torch.float32, device=dev)
        pu = _buf(u, dev, torch.float32, n_real * self.data.info()["n_gal"], "u")
        po = _buf(out, dev, torch.float32, self.n_scales * n_real * 2 * self.n_out, "out")
        L.check(self.ctx.lib.smart_noise_galaxy_batch(self.h, pu, n_real, norm, po, _stream(dev)))
        return out

    def noise_galaxy_seeded(self, seed: int, r_first: int, n_real: int, norm: int, moments=False, out=None):
        """Galaxy-level realisations with device-drawn angles on the matrix cores
        (see smart_noise_galaxy_seeded); outputs as for noise_seeded."""
        dev = self.ctx.device
        if moments:
            if out is None:
                out = torch.zeros(self.n_scales, 4, self.n_out, dtype=torch.float64, device=dev)
            po = _buf(out, dev, torch.float64, self.n_scales * 4 * self.n_out, "out")
        else:
            if out is None:
                out = torch.empty(self.n_scales, n_real, 2, self.n_out, dtype=torch.float32, device=dev)
            po = _buf(out, dev, torch.float32, self.n_scales * n_real * 2 * self.n_out, "out")
        L.check(self.ctx.lib.smart_noise_galaxy_seeded(self.h, seed, r_first, n_real, norm, 1 if moments else 0, po,
                                                       _stream(dev)))
        return out

    def free(self):
        if self.h:
            self.ctx.lib.smart_plan_free(self.h)
            self.h = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass
