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

    def mixed_batch(self, plans, norms, outs):
        n = len(plans)
        ph = (C.c_void_p * n)(*[p.h.value for p in plans])
        nh = (C.c_int * n)(*norms)
        oh = (C.c_void_p * n)(*[o.data_ptr() for o in outs])
        L.check(self.lib.smart_mixed_batch(self.h, n, ph, nh, oh, _stream(self.device)))


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

    def empty_out(self):
        dt = torch.float64 if self.precision == L.PREC_FP64 else torch.float32
        return torch.empty(self.n_scales, 5, self.n_out, dtype=dt, device=self.ctx.device)

    def run(self, norm: int, out=None):
        if out is None:
            out = self.empty_out()
        L.check(self.ctx.lib.smart_run(self.h, norm, _ptr(out), _stream(self.ctx.device)))
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

    def set_timing(self, enable: bool = True):
        L.check(self.ctx.lib.smart_plan_set_timing(self.h, 1 if enable else 0))

    def kernel_ms(self, scale: int = 0):
        """(belt kernel ms, general kernel ms) of the last timed run."""
        b, g = C.c_double(), C.c_double()
        L.check(self.ctx.lib.smart_plan_kernel_ms(self.h, scale, C.byref(b), C.byref(g)))
        return b.value, g.value

    def noise_batch(self, u, n_real: int, norm: int, precision: int, out=None):
        if out is None:
            out = torch.empty(self.n_scales, n_real, 2, self.n_out, dtype=torch.float32, device=self.ctx.device)
        L.check(self.ctx.lib.smart_noise_batch(self.h, _ptr(u), n_real, norm, precision, _ptr(out),
                                               _stream(self.ctx.device)))
        return out

    def noise_galaxy_batch(self, u, n_real: int, norm: int, out=None):
        """Galaxy-level realisations: u is [n_real][n_gal] in catalogue order."""
        if out is None:
            out = torch.empty(self.n_scales, n_real, 2, self.n_out, dtype=torch.float32, device=self.ctx.device)
        L.check(self.ctx.lib.smart_noise_galaxy_batch(self.h, _ptr(u), n_real, norm, _ptr(out),
                                                      _stream(self.ctx.device)))
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
