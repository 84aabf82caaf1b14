"""ctypes front end of the FP64 CPU oracle (deam_oracle.c).

TEST INFRASTRUCTURE ONLY: imported by the tests, the smoke check and the
CPU-baseline leg of the benchmark.  The GPU library never calls it.

Each function mirrors one step of the DEAM hot path:
    forward      l = H c                      (Eq. 8, the inner sum over voxels)
    backproject  b = H^T w                    (transpose of the same h)
    poly_mean    per-ray energy sums, weights and objective terms
                 (Eq. 8; Eqs. 9-10; Eq. 11 substitution p = q on the trace)
    update       c_i <- c_i - ln(b~_i / b^_i) / Z_i
    iterate      the DEAM loop with the masked I-divergence history (Eq. 5)
    step_vjp     vector-Jacobian product of one iteration (chain rule through
                 the update, the backprojection, the weights and Eq. 8)
    metal_trace  T = H M, mask = [T >= t]     (Eqs. 2-3)
    poly_mean_bt, iterate_bt
                 a bowtie filter: per-channel spectra I0_j(y,E)
    iterate_dual separate system operators and traces for the two scans
    dilate_mask  trace dilation along the channels
    iterate_os   ordered subsets of views: per epoch one DEAM step per
                 interleaved view subset, backprojecting only that subset
    fair, penalty, update_pen, iterate_pen
                 the penalised iteration: potential of Eq. 7 (the convex
                 "fair" reading), penalty of Eq. 6, and the decoupled
                 per-voxel c-step solved by bisection
"""
from __future__ import annotations

import contextlib
import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liboracle.so")

W_AM, W_GRAD, W_VJP, W_STEP_VJP = 0, 1, 2, 3


class OrcGeom(C.Structure):
    _fields_ = [("kind", C.c_int), ("nx", C.c_int), ("ny", C.c_int), ("nz", C.c_int),
                ("dx", C.c_double), ("dy", C.c_double), ("dz", C.c_double),
                ("n_views", C.c_int), ("n_rows", C.c_int), ("n_cols", C.c_int),
                ("sid", C.c_double), ("sdd", C.c_double), ("dgamma", C.c_double),
                ("col_offset", C.c_double), ("drow_iso", C.c_double),
                ("beta0", C.c_double), ("views_per_rot", C.c_double),
                ("feed_per_rot", C.c_double)]


def compile_library(src, out):
    """gcc build of an oracle source file into a shared library."""
    subprocess.check_call(["gcc", "-O2", "-std=c99", "-D_GNU_SOURCE", "-fopenmp", "-fPIC",
                           "-shared", "-fno-fast-math", "-ffp-contract=off",
                           "-I", _HERE, "-o", out, src, "-lm"])
    return out


def build(force=False):
    """Compile liboracle.so with gcc (FP64, OpenMP, no fast-math)."""
    src = os.path.join(_HERE, "deam_oracle.c")
    if not force and os.path.exists(LIB_PATH) and os.path.getmtime(LIB_PATH) >= os.path.getmtime(src):
        return LIB_PATH
    tmp = LIB_PATH + ".tmp"
    compile_library(src, tmp)
    os.replace(tmp, LIB_PATH)
    return LIB_PATH


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            build()
        _lib = _setup(C.CDLL(LIB_PATH))
    return _lib


@contextlib.contextmanager
def use_library(path):
    """Temporarily route every oracle call to another build of deam_oracle.c
    (used by the tests that plant mistakes in a copy of the oracle)."""
    global _lib
    saved = lib()
    _lib = _setup(C.CDLL(path))
    try:
        yield
    finally:
        _lib = saved


def _setup(L):
    """Declare the argument types of the oracle entry points."""
    P = np.ctypeslib.ndpointer
    d1 = P(dtype=np.float64, flags="C_CONTIGUOUS")
    u1 = P(dtype=np.uint8, flags="C_CONTIGUOUS")
    i1 = P(dtype=np.int64, flags="C_CONTIGUOUS")
    G = C.POINTER(OrcGeom)
    L.orc_num_threads.restype = C.c_int
    L.orc_set_num_threads.argtypes = [C.c_int]
    L.orc_ray.argtypes = [G, C.c_long, d1, d1]
    L.orc_siddon_ray.argtypes = [G, d1, d1, i1, d1, C.c_int]
    L.orc_siddon_ray.restype = C.c_int
    L.orc_forward.argtypes = [G, C.c_int, d1, d1]
    L.orc_forward_rays.argtypes = [G, C.c_int, d1, C.c_long, i1, d1]
    L.orc_backproject.argtypes = [G, C.c_int, d1, d1]
    L.orc_poly_mean.argtypes = [C.c_long, C.c_int, d1, d1, d1, d1, C.c_void_p, C.c_int,
                                C.c_void_p, d1, C.c_void_p, C.c_void_p]
    L.orc_poly_mean_bt.argtypes = [C.c_long, C.c_int, d1, d1, d1, C.c_int, d1, d1, C.c_void_p,
                                   C.c_int, C.c_void_p, d1, C.c_void_p, C.c_void_p]
    L.orc_iterate_bt.argtypes = [G, C.c_int, d1, d1, d1, d1, C.c_void_p, d1, C.c_int, d1, C.c_void_p]
    L.orc_iterate_bt.restype = C.c_int
    L.orc_sum.argtypes = [C.c_long, d1]
    L.orc_sum.restype = C.c_double
    L.orc_update.argtypes = [C.c_long, d1, d1, d1]
    L.orc_metal_trace.argtypes = [G, u1, C.c_double, u1, C.c_void_p]
    L.orc_iterate.argtypes = [G, C.c_int, d1, d1, d1, C.c_void_p, d1, C.c_int, d1, C.c_void_p]
    L.orc_iterate.restype = C.c_int
    L.orc_iterate_b.argtypes = [G, C.c_int, d1, d1, d1, C.c_void_p, d1, C.c_int, d1, C.c_void_p,
                                C.c_void_p]
    L.orc_iterate_b.restype = C.c_int
    L.orc_objective.argtypes = [G, C.c_int, d1, d1, d1, C.c_void_p, d1, C.c_int]
    L.orc_objective.restype = C.c_double
    L.orc_nll_grad.argtypes = [G, C.c_int, d1, d1, d1, C.c_void_p, d1, C.c_void_p]
    L.orc_nll_grad.restype = C.c_double
    L.orc_step_vjp.argtypes = [G, C.c_int, d1, d1, d1, C.c_void_p, d1, d1, d1, C.c_void_p]
    L.orc_step_vjp.restype = C.c_int
    L.orc_fair.argtypes = [C.c_double, C.c_double]
    L.orc_fair.restype = C.c_double
    L.orc_fair_d1.argtypes = [C.c_double, C.c_double]
    L.orc_fair_d1.restype = C.c_double
    L.orc_penalty.argtypes = [G, d1, C.c_double, C.c_double]
    L.orc_penalty.restype = C.c_double
    L.orc_update_pen.argtypes = [G, d1, d1, C.c_double, C.c_double, d1, d1]
    L.orc_update_pen_voxels.argtypes = [G, d1, d1, C.c_double, C.c_double, d1, C.c_long, i1, d1]
    L.orc_iterate_pen.argtypes = [G, C.c_int, d1, d1, d1, C.c_void_p, d1, C.c_double,
                                  C.c_double, C.c_int, d1, C.c_void_p]
    L.orc_iterate_pen.restype = C.c_int
    L.orc_iterate_os.argtypes = [G, C.c_int, d1, d1, d1, C.c_void_p, d1, C.c_int, C.c_int, d1,
                                 C.c_void_p]
    L.orc_iterate_os.restype = C.c_int
    L.orc_iterate_dual.argtypes = [C.c_void_p, C.c_int, d1, d1,
                                   C.c_void_p, C.c_void_p, d1, C.c_int, d1, C.c_void_p]
    L.orc_iterate_dual.restype = C.c_int
    L.orc_dilate_mask.argtypes = [G, u1, C.c_int, u1]
    return L


def num_threads():
    return lib().orc_num_threads()


def set_num_threads(n):
    """Threads of the oracle's parallel loops from now on (timing only)."""
    lib().orc_set_num_threads(int(n))


def geom_struct(g):
    return OrcGeom(g.kind, g.nx, g.ny, g.nz, g.dx, g.dy, g.dz, g.n_views, g.n_rows,
                   g.n_cols, g.sid, g.sdd, g.dgamma, g.col_offset, g.drow_iso, g.beta0,
                   g.views_per_rot, g.feed_per_rot)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _ptr(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def ray(g, index):
    S, P = np.zeros(3), np.zeros(3)
    lib().orc_ray(C.byref(geom_struct(g)), index, S, P)
    return S, P


def siddon(g, S, P):
    """(voxel indices, lengths) of one ray S->P through the grid of g."""
    cap = g.nx + g.ny + g.nz + 16
    idx = np.zeros(cap, dtype=np.int64)
    ln = np.zeros(cap)
    n = lib().orc_siddon_ray(C.byref(geom_struct(g)), _f64(S), _f64(P), idx, ln, cap)
    if n < 0:
        raise RuntimeError("siddon capacity exceeded")
    return idx[:n].copy(), ln[:n].copy()


def forward(g, img):
    img = _f64(img)
    nch = img.size // g.n_voxels
    out = np.zeros(nch * g.n_rays)
    lib().orc_forward(C.byref(geom_struct(g)), nch, img.reshape(-1), out)
    return out.reshape(nch, g.n_rays)


def forward_rays(g, img, rays):
    img = _f64(img)
    rays = np.ascontiguousarray(rays, dtype=np.int64)
    nch = img.size // g.n_voxels
    out = np.zeros(nch * len(rays))
    lib().orc_forward_rays(C.byref(geom_struct(g)), nch, img.reshape(-1), len(rays), rays, out)
    return out.reshape(nch, len(rays))


def backproject(g, sino):
    sino = _f64(sino)
    nch = sino.size // g.n_rays
    out = np.zeros(nch * g.n_voxels)
    lib().orc_backproject(C.byref(geom_struct(g)), nch, sino.reshape(-1), out)
    return out.reshape(nch, g.n_voxels)


def poly_mean(I0, mu, l, d, mask=None, mode=W_AM, v=None):
    """Per-ray weights, expected counts g and objective terms.

    mode W_AM  : w (4, R) = (w~1, w~2, w^1, w^2); obj = masked I-divergence terms
    mode W_GRAD: w (2, R) = u_i = sum_j (r_j - 1) a_ij; obj = NLL terms g - d ln g
    mode W_VJP : w (2, R) = -sum_j v_j a_ij
    mode W_STEP_VJP: v (4, R) = (dloss/dw~_1, dloss/dw~_2, dloss/dw^_1, dloss/dw^_2);
                 w (2, R) = dloss/dl_k (chain rule through g, a and the
                 second moments sum_E mu_i mu_k q_j)
    """
    I0, mu, l, d = _f64(I0), _f64(mu), _f64(l), _f64(d)
    R = l.shape[-1]
    nE = I0.shape[-1]
    nw = 4 if mode == W_AM else 2
    w = np.zeros(nw * R)
    g = np.zeros(2 * R)
    obj = np.zeros(R)
    m = None if mask is None else np.ascontiguousarray(mask, dtype=np.uint8)
    vv = None if v is None else _f64(v)
    lib().orc_poly_mean(R, nE, I0.reshape(-1), mu.reshape(-1), l.reshape(-1), d.reshape(-1),
                        _ptr(m), mode, _ptr(vv), w, g.ctypes.data_as(C.c_void_p),
                        obj.ctypes.data_as(C.c_void_p))
    return w.reshape(nw, R), g.reshape(2, R), obj


def total(x):
    x = _f64(x).reshape(-1)
    return lib().orc_sum(x.size, x)


def update(b, Z, c):
    b, c = _f64(b), _f64(c).copy()
    V = c.shape[-1]
    lib().orc_update(V, b.reshape(-1), _f64(Z), c.reshape(-1))
    return c


def metal_trace(g, M, t):
    M = np.ascontiguousarray(M, dtype=np.uint8).reshape(-1)
    mask = np.zeros(g.n_rays, dtype=np.uint8)
    T = np.zeros(g.n_rays)
    lib().orc_metal_trace(C.byref(geom_struct(g)), M, float(t), mask, T.ctypes.data_as(C.c_void_p))
    return mask, T


def iterate(g, I0, mu, d, mask, Z, c0, n_iter, want_b=False):
    """Run n_iter DEAM iterations from c0; returns (c, objective history), and
    with want_b also the last iteration's backprojections b (4, V)
    (b~_1, b~_2, b^_1, b^_2)."""
    c = _f64(c0).copy()
    hist = np.zeros(max(n_iter, 1))
    b = np.zeros((4, g.n_voxels)) if want_b else None
    m = None if mask is None else np.ascontiguousarray(mask, dtype=np.uint8)
    rc = lib().orc_iterate_b(C.byref(geom_struct(g)), I0.shape[-1], _f64(I0).reshape(-1),
                             _f64(mu).reshape(-1), _f64(d).reshape(-1), _ptr(m), _f64(Z),
                             n_iter, c.reshape(-1), hist.ctypes.data_as(C.c_void_p), _ptr(b))
    if rc != 0:
        raise MemoryError("oracle iterate allocation failed")
    return (c, hist[:n_iter], b) if want_b else (c, hist[:n_iter])


def step_vjp(g, I0, mu, d, mask, Z, c, G):
    """Vector-Jacobian product of one DEAM iteration c -> c - ln(b~/b^)/Z at c
    for the upstream gradient G (both (2, V)): G + H^T lambda."""
    m = None if mask is None else np.ascontiguousarray(mask, dtype=np.uint8)
    out = np.zeros(2 * g.n_voxels)
    rc = lib().orc_step_vjp(C.byref(geom_struct(g)), I0.shape[-1], _f64(I0).reshape(-1),
                            _f64(mu).reshape(-1), _f64(d).reshape(-1), _ptr(m), _f64(Z),
                            _f64(c).reshape(-1), _f64(G).reshape(-1),
                            out.ctypes.data_as(C.c_void_p))
    if rc != 0:
        raise MemoryError("oracle step_vjp allocation failed")
    return out.reshape(2, g.n_voxels)


def objective(g, I0, mu, d, mask, c, mode=W_AM):
    m = None if mask is None else np.ascontiguousarray(mask, dtype=np.uint8)
    return lib().orc_objective(C.byref(geom_struct(g)), I0.shape[-1], _f64(I0).reshape(-1),
                               _f64(mu).reshape(-1), _f64(d).reshape(-1), _ptr(m),
                               _f64(c).reshape(-1), mode)


def nll_grad(g, I0, mu, d, mask, c):
    m = None if mask is None else np.ascontiguousarray(mask, dtype=np.uint8)
    grad = np.zeros(2 * g.n_voxels)
    L = lib().orc_nll_grad(C.byref(geom_struct(g)), I0.shape[-1], _f64(I0).reshape(-1),
                           _f64(mu).reshape(-1), _f64(d).reshape(-1), _ptr(m),
                           _f64(c).reshape(-1), grad.ctypes.data_as(C.c_void_p))
    return L, grad.reshape(2, g.n_voxels)


def fair(t, delta):
    """phi(t) of Eq. 7 (fair reading), elementwise."""
    f = lib().orc_fair
    return np.vectorize(lambda x: f(float(x), float(delta)), otypes=[float])(t)


def fair_d1(t, delta):
    f = lib().orc_fair_d1
    return np.vectorize(lambda x: f(float(x), float(delta)), otypes=[float])(t)


def penalty(g, c, lam, delta):
    """R(c) of Eq. 6 for c (2, V)."""
    return lib().orc_penalty(C.byref(geom_struct(g)), _f64(c).reshape(-1), float(lam), float(delta))


def update_pen(g, b, Z, lam, delta, c_prev):
    """Penalised c-step from c_prev (2, V) with the backprojections b (4, V)."""
    out = np.zeros(2 * g.n_voxels)
    lib().orc_update_pen(C.byref(geom_struct(g)), _f64(b).reshape(-1), _f64(Z), float(lam),
                         float(delta), _f64(c_prev).reshape(-1), out)
    return out.reshape(2, g.n_voxels)


def update_pen_voxels(g, b, Z, lam, delta, c_prev, voxels):
    """The penalised c-step at the chosen voxels only: (2, len(voxels))."""
    vox = np.ascontiguousarray(voxels, dtype=np.int64)
    out = np.zeros(2 * len(vox))
    lib().orc_update_pen_voxels(C.byref(geom_struct(g)), _f64(b).reshape(-1), _f64(Z), float(lam),
                                float(delta), _f64(c_prev).reshape(-1), len(vox), vox, out)
    return out.reshape(2, len(vox))


def iterate_pen(g, I0, mu, d, mask, Z, lam, delta, c0, n_iter):
    """n_iter penalised DEAM iterations from c0; returns (c, history of the
    masked I-divergence + R(c))."""
    c = _f64(c0).copy()
    hist = np.zeros(max(n_iter, 1))
    m = None if mask is None else np.ascontiguousarray(mask, dtype=np.uint8)
    rc = lib().orc_iterate_pen(C.byref(geom_struct(g)), I0.shape[-1], _f64(I0).reshape(-1),
                               _f64(mu).reshape(-1), _f64(d).reshape(-1), _ptr(m), _f64(Z),
                               float(lam), float(delta), n_iter, c.reshape(-1),
                               hist.ctypes.data_as(C.c_void_p))
    if rc != 0:
        raise MemoryError("oracle iterate_pen allocation failed")
    return c, hist[:n_iter]


def iterate_os(g, I0, mu, d, mask, Z, c0, n_sub, n_iter):
    """n_iter epochs of ordered-subset DEAM with n_sub interleaved view
    subsets; returns (c, masked I-divergence at the start of each epoch)."""
    c = _f64(c0).copy()
    hist = np.zeros(max(n_iter, 1))
    m = None if mask is None else np.ascontiguousarray(mask, dtype=np.uint8)
    rc = lib().orc_iterate_os(C.byref(geom_struct(g)), I0.shape[-1], _f64(I0).reshape(-1),
                              _f64(mu).reshape(-1), _f64(d).reshape(-1), _ptr(m), _f64(Z),
                              int(n_sub), n_iter, c.reshape(-1), hist.ctypes.data_as(C.c_void_p))
    if rc != 0:
        raise MemoryError("oracle iterate_os failed")
    return c, hist[:n_iter]


def iterate_dual(geoms, I0, mu, ds, masks, Z, c0, n_iter):
    """DEAM with one geometry, counts and trace per scan: geoms, ds, masks are
    pairs (low, high); ds[j] has shape (R_j,).  Returns (c, history of the sum
    of the two masked I-divergences)."""
    c = _f64(c0).copy()
    hist = np.zeros(max(n_iter, 1))
    gs = [geom_struct(g) for g in geoms]
    gp = (C.c_void_p * 2)(*[C.cast(C.pointer(x), C.c_void_p) for x in gs])
    dk = [_f64(x).reshape(-1) for x in ds]
    dp = (C.c_void_p * 2)(*[x.ctypes.data_as(C.c_void_p) for x in dk])
    mk = [None if m is None else np.ascontiguousarray(m, dtype=np.uint8).reshape(-1) for m in masks]
    mp = (C.c_void_p * 2)(*[None if m is None else m.ctypes.data_as(C.c_void_p) for m in mk])
    rc = lib().orc_iterate_dual(C.cast(gp, C.c_void_p), I0.shape[-1], _f64(I0).reshape(-1),
                                _f64(mu).reshape(-1), C.cast(dp, C.c_void_p), C.cast(mp, C.c_void_p),
                                _f64(Z), n_iter, c.reshape(-1), hist.ctypes.data_as(C.c_void_p))
    if rc != 0:
        raise MemoryError("oracle iterate_dual failed")
    return c, hist[:n_iter]


def dilate_mask(g, mask, radius):
    m = np.ascontiguousarray(mask, dtype=np.uint8).reshape(-1)
    out = np.zeros_like(m)
    lib().orc_dilate_mask(C.byref(geom_struct(g)), m, int(radius), out)
    return out


def poly_mean_bt(I0, mu, bt, l, d, mask=None, mode=W_AM, v=None):
    """poly_mean with a bowtie: bt (2, n_cols) basis path lengths (mm) of the
    filter per channel; ray y belongs to channel y mod n_cols."""
    I0, mu, l, d, bt = _f64(I0), _f64(mu), _f64(l), _f64(d), _f64(bt)
    R = l.shape[-1]
    nE = I0.shape[-1]
    nw = 4 if mode == W_AM else 2
    w = np.zeros(nw * R)
    g = np.zeros(2 * R)
    obj = np.zeros(R)
    m = None if mask is None else np.ascontiguousarray(mask, dtype=np.uint8)
    vv = None if v is None else _f64(v)
    lib().orc_poly_mean_bt(R, nE, I0.reshape(-1), mu.reshape(-1), bt.reshape(-1), bt.shape[-1],
                           l.reshape(-1), d.reshape(-1), _ptr(m), mode, _ptr(vv), w,
                           g.ctypes.data_as(C.c_void_p), obj.ctypes.data_as(C.c_void_p))
    return w.reshape(nw, R), g.reshape(2, R), obj


def iterate_bt(g, I0, mu, bt, d, mask, Z, c0, n_iter):
    """DEAM with a bowtie filter bt (2, n_cols)."""
    c = _f64(c0).copy()
    hist = np.zeros(max(n_iter, 1))
    m = None if mask is None else np.ascontiguousarray(mask, dtype=np.uint8)
    rc = lib().orc_iterate_bt(C.byref(geom_struct(g)), I0.shape[-1], _f64(I0).reshape(-1),
                              _f64(mu).reshape(-1), _f64(bt).reshape(-1), _f64(d).reshape(-1),
                              _ptr(m), _f64(Z), n_iter, c.reshape(-1),
                              hist.ctypes.data_as(C.c_void_p))
    if rc != 0:
        raise MemoryError("oracle iterate_bt failed")
    return c, hist[:n_iter]
