"""Python face of the C ABI: one Plan per scanner geometry and spectrum pair.

Every method marshals torch device tensors into the matching ``deam_*`` call
of libdeam.so on torch's current stream; all arithmetic runs in the HIP
kernels.  Tensors follow the layouts of include/deam.h: images [n_ch, V]
and sinograms [n_ch, R], channel-major, C-contiguous, on the plan's device.
"""
from __future__ import annotations

import ctypes as C

import numpy as np
import torch

from . import _lib as L


def _ptr(t):
    return None if t is None else C.c_void_p(t.data_ptr())


def _stream():
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


class Plan:
    """A DEAM plan (geometry tables and energy table on the device).

    geom: any object with the fields of ``deam_geometry`` (e.g.
    ``workloads.Geometry``); I0, mu: (2, n_energy) float64 arrays;
    precision: "mixed" (FP32 projections, FP64 reductions and update) or "fp64".
    """

    def __init__(self, geom, I0, mu, precision="mixed"):
        self.lib = L.load()
        if precision not in ("mixed", "fp64"):
            raise ValueError("precision must be 'mixed' or 'fp64'")
        self.precision = precision
        self.dtype = torch.float32 if precision == "mixed" else torch.float64
        self.geom = geom
        g = L.DeamGeometry(int(geom.kind), geom.nx, geom.ny, geom.nz, geom.dx, geom.dy, geom.dz,
                           geom.n_views, geom.n_rows, geom.n_cols, geom.sid, geom.sdd,
                           geom.dgamma, geom.col_offset, geom.drow_iso, geom.beta0,
                           geom.views_per_rot, geom.feed_per_rot)
        I0 = np.ascontiguousarray(I0, dtype=np.float64)
        mu = np.ascontiguousarray(mu, dtype=np.float64)
        if I0.shape != mu.shape or I0.ndim != 2 or I0.shape[0] != 2:
            raise ValueError("I0 and mu must both have shape (2, n_energy)")
        self.device = torch.device("cuda", torch.cuda.current_device())
        self._p = C.c_void_p()
        L.check(self.lib.deam_plan_create(C.byref(g), I0.shape[1], I0.ctypes.data_as(C.c_void_p),
                                          mu.ctypes.data_as(C.c_void_p),
                                          L.PREC_MIXED if precision == "mixed" else L.PREC_FP64,
                                          C.byref(self._p)))
        R, V = C.c_int64(), C.c_int64()
        L.check(self.lib.deam_plan_sizes(self._p, C.byref(R), C.byref(V)))
        self.R, self.V = R.value, V.value
        self._ws = {}

    def __del__(self):
        p = getattr(self, "_p", None)
        if p is not None and p.value:
            try:
                self.lib.deam_plan_destroy(p)
            except Exception:
                pass
            self._p = None

    # -- workspace -------------------------------------------------------------
    def workspace_bytes(self, op):
        n = C.c_size_t()
        L.check(self.lib.deam_workspace_size(self._p, op, C.byref(n)))
        return n.value

    def workspace(self, op):
        """Cached 256-byte aligned device workspace for an operation."""
        need = self.workspace_bytes(op)
        buf = self._ws.get(op)
        if buf is None or buf[2] < need:
            raw = torch.empty(need + 256, dtype=torch.uint8, device=self.device)
            off = (-raw.data_ptr()) % 256
            self._ws[op] = (raw, off, need)
            buf = self._ws[op]
        raw, off, n = buf
        return C.c_void_p(raw.data_ptr() + off), C.c_size_t(n)

    def _check(self, t, shape, dtype, name):
        if t is None:
            return
        if not isinstance(t, torch.Tensor) or t.device != self.device:
            raise ValueError(f"{name} must be a tensor on {self.device}")
        if t.dtype != dtype or tuple(t.shape) != tuple(shape) or not t.is_contiguous():
            raise ValueError(f"{name}: expected contiguous {dtype} {tuple(shape)}, "
                             f"got {t.dtype} {tuple(t.shape)}")

    # -- operations ----------------------------------------------------------------
    def metal_trace(self, M, t, want_T=False):
        """mask[y] = (sum_x h(x,y) M(x) >= t); optionally the FP64 trace T."""
        self._check(M, (self.V,), torch.uint8, "M")
        mask = torch.empty(self.R, dtype=torch.uint8, device=self.device)
        T = torch.empty(self.R, dtype=torch.float64, device=self.device) if want_T else None
        ws, n = self.workspace(L.OP_METAL_TRACE)
        L.check(self.lib.deam_metal_trace(self._p, _ptr(M), float(t), _ptr(mask), _ptr(T), ws, n,
                                          _stream()))
        return (mask, T) if want_T else mask

    def forward(self, c):
        """l[c] = H c[c] for c of shape (n_ch, V), n_ch in {1, 2}."""
        n_ch = c.shape[0]
        self._check(c, (n_ch, self.V), self.dtype, "c")
        l = torch.empty((n_ch, self.R), dtype=self.dtype, device=self.device)
        ws, n = self.workspace(L.OP_FORWARD)
        L.check(self.lib.deam_forward(self._p, _ptr(c), n_ch, _ptr(l), ws, n, _stream()))
        return l

    def poly_mean(self, l, d, mask=None, mode=L.W_AM, v=None, want_g=False, want_obj=False):
        self._check(l, (2, self.R), self.dtype, "l")
        if mode != L.W_VJP:
            self._check(d, (2, self.R), torch.float32, "d")
        self._check(mask, (self.R,), torch.uint8, "mask")
        self._check(v, (4 if mode == L.W_STEP_VJP else 2, self.R), self.dtype, "v")
        nw = 4 if mode == L.W_AM else 2
        w = torch.empty((nw, self.R), dtype=self.dtype, device=self.device)
        g = torch.empty((2, self.R), dtype=self.dtype, device=self.device) if want_g else None
        obj = torch.empty(1, dtype=torch.float64, device=self.device) if want_obj else None
        ws, n = self.workspace(L.OP_POLY_MEAN)
        L.check(self.lib.deam_poly_mean(self._p, _ptr(l), _ptr(d), _ptr(mask), mode, _ptr(v),
                                        _ptr(w), _ptr(g), _ptr(obj), ws, n, _stream()))
        return w, g, obj

    def backproject(self, w, nonneg=False):
        """b[c] = H^T w[c] for w of shape (n_ch, R), n_ch in {1, 2, 4}.
        nonneg=True promises w >= 0 everywhere (the AM weights): the
        accumulation deam_iterate uses (packed for 4 channels of a mixed plan)."""
        n_ch = w.shape[0]
        self._check(w, (n_ch, self.R), self.dtype, "w")
        b = torch.empty((n_ch, self.V), dtype=self.dtype, device=self.device)
        ws, n = self.workspace(L.OP_BACKPROJECT)
        L.check(self.lib.deam_backproject(self._p, _ptr(w), n_ch, L.BP_NONNEG if nonneg else 0,
                                          _ptr(b), ws, n, _stream()))
        return b

    def update(self, c64, b, Z, want_proj=False):
        """In-place c_i <- c_i - ln(b~_i / b^_i) / Z_i; returns the projection copy if asked."""
        self._check(c64, (2, self.V), torch.float64, "c64")
        self._check(b, (4, self.V), self.dtype, "b")
        Zh = np.ascontiguousarray(Z, dtype=np.float64)
        cp = torch.empty((2, self.V), dtype=self.dtype, device=self.device) if want_proj else None
        L.check(self.lib.deam_update(self._p, _ptr(c64), _ptr(cp), _ptr(b),
                                     Zh.ctypes.data_as(C.c_void_p), _stream()))
        return cp

    def iterate(self, c64, d, mask, Z, n_iter, obj_hist=None, c_proj=None):
        """n_iter DEAM iterations in place on c64; obj_hist (device float64 [n_iter])
        receives the masked I-divergence at each iterate, c_proj ([2, V] in the
        plan precision) the final iterate's copy."""
        self._check(c64, (2, self.V), torch.float64, "c64")
        self._check(c_proj, (2, self.V), self.dtype, "c_proj")
        self._check(d, (2, self.R), torch.float32, "d")
        self._check(mask, (self.R,), torch.uint8, "mask")
        self._check(obj_hist, (n_iter,), torch.float64, "obj_hist")
        Zh = np.ascontiguousarray(Z, dtype=np.float64)
        ws, n = self.workspace(L.OP_ITERATE)
        L.check(self.lib.deam_iterate(self._p, _ptr(c64), _ptr(c_proj), _ptr(d), _ptr(mask),
                                      Zh.ctypes.data_as(C.c_void_p), int(n_iter), _ptr(obj_hist),
                                      ws, n, _stream()))
        return c64

    def iterate_sync(self, c64, d, mask, Z, n_iter, c_proj=None):
        """iterate() that waits for the device and returns the objective history
        as a host float64 array (deam_iterate_sync: a device fault raises)."""
        self._check(c64, (2, self.V), torch.float64, "c64")
        self._check(c_proj, (2, self.V), self.dtype, "c_proj")
        self._check(d, (2, self.R), torch.float32, "d")
        self._check(mask, (self.R,), torch.uint8, "mask")
        Zh = np.ascontiguousarray(Z, dtype=np.float64)
        hist = np.zeros(max(int(n_iter), 0))
        ws, n = self.workspace(L.OP_ITERATE)
        L.check(self.lib.deam_iterate_sync(self._p, _ptr(c64), _ptr(c_proj), _ptr(d), _ptr(mask),
                                           Zh.ctypes.data_as(C.c_void_p), int(n_iter),
                                           hist.ctypes.data_as(C.c_void_p), ws, n, _stream()))
        return hist

    def validate_inputs(self, c64=None, d=None):
        """Debug check (synchronous): c64 finite, d finite and >= 0.  Returns
        the numbers of offending entries; raises DeamError when any is found."""
        self._check(c64, (2, self.V), torch.float64, "c64")
        self._check(d, (2, self.R), torch.float32, "d")
        ws, n = self.workspace(L.OP_BACKPROJECT)
        bad = (C.c_int64 * 2)()
        rc = self.lib.deam_validate_inputs(self._p, _ptr(c64), _ptr(d), bad, ws, n, _stream())
        if rc not in (0, -7):
            L.check(rc)
        counts = (bad[0], bad[1])
        if rc == -7:
            L.check(rc)
        return counts

    def penalty(self, c64, lam, delta):
        """R(c) of Eq. 6 (fair potential, 1/distance neighbourhood) as a
        0-d float64 device tensor."""
        self._check(c64, (2, self.V), torch.float64, "c64")
        out = torch.empty((), dtype=torch.float64, device=self.device)
        ws, n = self.workspace(L.OP_PENALTY)
        L.check(self.lib.deam_penalty(self._p, _ptr(c64), float(lam), float(delta), _ptr(out),
                                      ws, n, _stream()))
        return out

    def update_penalized(self, c_prev, b, Z, lam, delta, want_proj=False):
        """Penalised c-step from c_prev (float64 (2, V)) with the
        backprojections b: returns the new iterate (and its projection copy)."""
        self._check(c_prev, (2, self.V), torch.float64, "c_prev")
        self._check(b, (4, self.V), self.dtype, "b")
        Zh = np.ascontiguousarray(Z, dtype=np.float64)
        out = torch.empty((2, self.V), dtype=torch.float64, device=self.device)
        cp = torch.empty((2, self.V), dtype=self.dtype, device=self.device) if want_proj else None
        L.check(self.lib.deam_update_penalized(self._p, _ptr(c_prev), _ptr(out), _ptr(cp), _ptr(b),
                                               Zh.ctypes.data_as(C.c_void_p), float(lam),
                                               float(delta), _stream()))
        return (out, cp) if want_proj else out

    def iterate_penalized(self, c64, d, mask, Z, lam, delta, n_iter, obj_hist=None):
        """n_iter penalised DEAM iterations in place on c64; obj_hist receives
        the masked I-divergence + R at each iterate."""
        self._check(c64, (2, self.V), torch.float64, "c64")
        self._check(d, (2, self.R), torch.float32, "d")
        self._check(mask, (self.R,), torch.uint8, "mask")
        self._check(obj_hist, (n_iter,), torch.float64, "obj_hist")
        Zh = np.ascontiguousarray(Z, dtype=np.float64)
        ws, n = self.workspace(L.OP_ITERATE_PENALIZED)
        L.check(self.lib.deam_iterate_penalized(self._p, _ptr(c64), _ptr(d), _ptr(mask),
                                                Zh.ctypes.data_as(C.c_void_p), float(lam),
                                                float(delta), int(n_iter), _ptr(obj_hist), ws, n,
                                                _stream()))
        return c64

    def pack_mask(self, mask):
        """Bit-packed trace: int32 tensor of ceil(R / 32) words."""
        self._check(mask, (self.R,), torch.uint8, "mask")
        bits = torch.empty((self.R + 31) // 32, dtype=torch.int32, device=self.device)
        L.check(self.lib.deam_pack_mask(self._p, _ptr(mask), _ptr(bits), _stream()))
        return bits

    def iterate_packed(self, c64, d, bits, Z, n_iter, obj_hist=None):
        """iterate() with the bit-packed trace of pack_mask()."""
        self._check(c64, (2, self.V), torch.float64, "c64")
        self._check(d, (2, self.R), torch.float32, "d")
        self._check(bits, ((self.R + 31) // 32,), torch.int32, "bits")
        self._check(obj_hist, (n_iter,), torch.float64, "obj_hist")
        Zh = np.ascontiguousarray(Z, dtype=np.float64)
        ws, n = self.workspace(L.OP_ITERATE)
        L.check(self.lib.deam_iterate_packed(self._p, _ptr(c64), _ptr(d), _ptr(bits),
                                             Zh.ctypes.data_as(C.c_void_p), int(n_iter),
                                             _ptr(obj_hist), ws, n, _stream()))
        return c64

    def set_bowtie(self, bt):
        """Bowtie filter: bt (2, n_cols) path lengths (mm) in the basis per
        channel, or None to remove it."""
        if bt is None:
            L.check(self.lib.deam_plan_set_bowtie(self._p, None))
            return
        b = np.ascontiguousarray(bt, dtype=np.float64)
        if b.shape != (2, self.geom.n_cols):
            raise ValueError(f"bowtie must have shape (2, {self.geom.n_cols})")
        L.check(self.lib.deam_plan_set_bowtie(self._p, b.ctypes.data_as(C.c_void_p)))

    def dilate_mask(self, mask, radius):
        """Trace dilated by `radius` channels (same view and row)."""
        self._check(mask, (self.R,), torch.uint8, "mask")
        out = torch.empty_like(mask)
        L.check(self.lib.deam_dilate_mask(self._p, _ptr(mask), int(radius), _ptr(out), _stream()))
        return out

    def fbp(self, p):
        """Fan-beam FBP of line integrals p (n_ch, R), n_ch in {1, 2}: (n_ch, V)."""
        n_ch = p.shape[0]
        self._check(p, (n_ch, self.R), self.dtype, "p")
        img = torch.empty((n_ch, self.V), dtype=self.dtype, device=self.device)
        ws, n = self.workspace(L.OP_FBP)
        L.check(self.lib.deam_fbp(self._p, _ptr(p), n_ch, _ptr(img), ws, n, _stream()))
        return img

    def nmar(self, p, mask, p_prior, eps):
        """NMAR of both sinograms p (2, R) across the trace mask with the prior's
        projections p_prior (2, R)."""
        self._check(p, (2, self.R), self.dtype, "p")
        self._check(p_prior, (2, self.R), self.dtype, "p_prior")
        self._check(mask, (self.R,), torch.uint8, "mask")
        out = torch.empty_like(p)
        L.check(self.lib.deam_nmar(self._p, _ptr(p), _ptr(mask), _ptr(p_prior), float(eps),
                                   _ptr(out), _stream()))
        return out

    def mar_init(self, d, prm):
        """MAR initialisation from the counts d (2, R) float32 with the
        parameters prm (dict: t, water (2,), air_frac, bone_frac, metal_frac,
        eps): returns (c64 (2, V) float64, M (V,) uint8, mask (R,) uint8)."""
        self._check(d, (2, self.R), torch.float32, "d")
        P = L.DeamMarParams(float(prm["t"]), (C.c_double * 2)(*[float(x) for x in prm["water"]]),
                            float(prm["air_frac"]), float(prm["bone_frac"]),
                            float(prm["metal_frac"]), float(prm["eps"]))
        c = torch.empty((2, self.V), dtype=torch.float64, device=self.device)
        M = torch.empty(self.V, dtype=torch.uint8, device=self.device)
        mask = torch.empty(self.R, dtype=torch.uint8, device=self.device)
        ws, n = self.workspace(L.OP_MAR_INIT)
        L.check(self.lib.deam_mar_init(self._p, _ptr(d), C.byref(P), _ptr(c), _ptr(M), _ptr(mask),
                                       ws, n, _stream()))
        return c, M, mask

    def iterate_os(self, c64, d, mask, Z, n_sub, n_iter, obj_hist=None):
        """n_iter epochs of ordered-subset DEAM (n_sub interleaved view subsets)
        in place on c64; obj_hist receives the masked I-divergence at the start
        of each epoch."""
        self._check(c64, (2, self.V), torch.float64, "c64")
        self._check(d, (2, self.R), torch.float32, "d")
        self._check(mask, (self.R,), torch.uint8, "mask")
        self._check(obj_hist, (n_iter,), torch.float64, "obj_hist")
        Zh = np.ascontiguousarray(Z, dtype=np.float64)
        ws, n = self.workspace(L.OP_ITERATE)
        L.check(self.lib.deam_iterate_os(self._p, _ptr(c64), _ptr(d), _ptr(mask),
                                         Zh.ctypes.data_as(C.c_void_p), int(n_sub), int(n_iter),
                                         _ptr(obj_hist), ws, n, _stream()))
        return c64

    def iterate_vjp(self, c64, d, mask, Z, G):
        """Vector-Jacobian product of one DEAM iteration at c64 for the upstream
        gradient G (both float64 (2, V)): returns (dPhi/dc)^T G."""
        self._check(c64, (2, self.V), torch.float64, "c64")
        self._check(d, (2, self.R), torch.float32, "d")
        self._check(mask, (self.R,), torch.uint8, "mask")
        self._check(G, (2, self.V), torch.float64, "G")
        Zh = np.ascontiguousarray(Z, dtype=np.float64)
        out = torch.empty((2, self.V), dtype=torch.float64, device=self.device)
        ws, n = self.workspace(L.OP_ITERATE_VJP)
        L.check(self.lib.deam_iterate_vjp(self._p, _ptr(c64), _ptr(d), _ptr(mask),
                                          Zh.ctypes.data_as(C.c_void_p), _ptr(G), _ptr(out),
                                          ws, n, _stream()))
        return out

    def iterate_timed(self, c64, d, mask, Z, n_iter, obj_hist=None):
        """iterate() plus per-kernel device times (ms summed over the iterations):
        dict(fp_poly, backproject, update, loop).  Synchronises the stream."""
        self._check(c64, (2, self.V), torch.float64, "c64")
        self._check(d, (2, self.R), torch.float32, "d")
        self._check(mask, (self.R,), torch.uint8, "mask")
        self._check(obj_hist, (n_iter,), torch.float64, "obj_hist")
        Zh = np.ascontiguousarray(Z, dtype=np.float64)
        ws, n = self.workspace(L.OP_ITERATE)
        ms = (C.c_float * 4)()
        L.check(self.lib.deam_iterate_timed(self._p, _ptr(c64), None, _ptr(d), _ptr(mask),
                                            Zh.ctypes.data_as(C.c_void_p), int(n_iter),
                                            _ptr(obj_hist), ws, n, _stream(), ms))
        return dict(fp_poly=ms[0], backproject=ms[1], update=ms[2], loop=ms[3])


def iterate_dual(plan_lo, plan_hi, c64, d_lo, mask_lo, d_hi, mask_hi, Z, n_iter, obj_hist=None):
    """DEAM with a system operator and a trace per scan (deam_iterate_dual).
    plan_lo / plan_hi carry only their own spectrum; d_lo, d_hi are (2, R_j)
    float32 with the scan's counts in its own channel."""
    lib = plan_lo.lib
    plan_lo._check(c64, (2, plan_lo.V), torch.float64, "c64")
    plan_lo._check(d_lo, (2, plan_lo.R), torch.float32, "d_lo")
    plan_hi._check(d_hi, (2, plan_hi.R), torch.float32, "d_hi")
    plan_lo._check(mask_lo, (plan_lo.R,), torch.uint8, "mask_lo")
    plan_hi._check(mask_hi, (plan_hi.R,), torch.uint8, "mask_hi")
    plan_lo._check(obj_hist, (n_iter,), torch.float64, "obj_hist")
    n = C.c_size_t(0)
    L.check(lib.deam_dual_workspace_size(plan_lo._p, plan_hi._p, C.byref(n)))
    key = ("dual", id(plan_hi))
    buf = plan_lo._ws.get(key)
    if buf is None or buf[2] < n.value:      # cached on plan_lo, like its own workspaces
        raw = torch.empty(int(n.value) + 256, dtype=torch.uint8, device=plan_lo.device)
        plan_lo._ws[key] = (raw, (-raw.data_ptr()) % 256, int(n.value))
        buf = plan_lo._ws[key]
    raw, off, _ = buf
    base = raw.data_ptr()
    Zh = np.ascontiguousarray(Z, dtype=np.float64)
    L.check(lib.deam_iterate_dual(plan_lo._p, plan_hi._p, _ptr(c64), _ptr(d_lo), _ptr(mask_lo),
                                  _ptr(d_hi), _ptr(mask_hi), Zh.ctypes.data_as(C.c_void_p),
                                  int(n_iter), _ptr(obj_hist), C.c_void_p(base + off),
                                  int(n.value), _stream()))
    return c64
