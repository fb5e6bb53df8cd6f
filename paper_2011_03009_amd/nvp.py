"""Python binding of the nvp C ABI.

Every function here only marshals arguments: torch tensors provide device
memory (their data pointers) and the current HIP stream; all computation runs
in the library's HIP kernels.  There is no CPU fallback: without the built
library every call raises.
"""

import ctypes
import weakref

import torch

from . import _native
from ._native import Grid, Medium, Problem

NVP_C64, NVP_C128 = 0, 1
NVP_QUAD_BALL, NVP_QUAD_CORRECTED = 0, 1
TIMING_KINDS = ("ktab", "kfft", "xfwd", "yfwd", "zconv", "yinv", "xinv", "src")
_DT = {NVP_C64: torch.complex64, NVP_C128: torch.complex128}


class NvpError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__("nvp status %d (%s): %s" % (status, _native.lib().nvp_status_str(status).decode(), msg))
        self.status = status


def _check(st, ctx=None):
    if st != 0:
        L = _native.lib()
        raise NvpError(st, (L.nvp_last_error(ctx) or b"").decode())


def prec_of(dtype):
    if dtype == torch.complex64:
        return NVP_C64
    if dtype == torch.complex128:
        return NVP_C128
    raise ValueError("fields must be complex64 or complex128")


def medium(m):
    """Medium from a mapping with c0, rho0, beta, alpha0_db, eta."""
    if isinstance(m, Medium):
        return m
    return Medium(m["c0"], m["rho0"], m["beta"], m["alpha0_db"], m["eta"])


def grid(g):
    """Grid from an nvp Grid, or any object/mapping with origin, h, n."""
    if isinstance(g, Grid):
        return g
    if isinstance(g, dict):
        o, h, n = g["origin"], g["h"], g["n"]
    else:
        o, h, n = g.origin, g.h, g.n
    return Grid((ctypes.c_double * 3)(*[float(v) for v in o]), float(h), (ctypes.c_int64 * 3)(*[int(v) for v in n]))


def grid_tuple(g):
    return tuple(g.origin), g.h, tuple(g.n)


# ------------------------------------------------------------- host constants and grids

def wavenumber(med, f0, n):
    kr, ki = ctypes.c_double(), ctypes.c_double()
    _check(_native.lib().nvp_wavenumber(ctypes.byref(medium(med)), f0, n, ctypes.byref(kr), ctypes.byref(ki)))
    return complex(kr.value, ki.value)


def cascade_constant(med, f0, n):
    c = ctypes.c_double()
    _check(_native.lib().nvp_cascade_constant(ctypes.byref(medium(med)), f0, n, ctypes.byref(c)))
    return c.value


def spacing(med, f0, n, n_w=6):
    h = ctypes.c_double()
    _check(_native.lib().nvp_spacing(ctypes.byref(medium(med)), f0, n, n_w, ctypes.byref(h)))
    return h.value


def _d3(v):
    return (ctypes.c_double * 3)(*[float(x) for x in v])


def _i3(v):
    return (ctypes.c_int64 * 3)(*[int(x) for x in v])


def grid_from_counts(focus, h, n, i_f):
    g = Grid()
    _check(_native.lib().nvp_grid_from_counts(_d3(focus), h, _i3(n), _i3(i_f), ctypes.byref(g)))
    return g


def grid_from_box(focus, lo, hi, h):
    g = Grid()
    i_f = (ctypes.c_int64 * 3)()
    _check(_native.lib().nvp_grid_from_box(_d3(focus), _d3(lo), _d3(hi), h, ctypes.byref(g), i_f))
    return g, tuple(i_f)


def rule_of_thumb_box(n, l, R, d, eps=1e-4):
    lo, hi = (ctypes.c_double * 3)(), (ctypes.c_double * 3)()
    _check(_native.lib().nvp_rule_of_thumb_box(n, l, R, d, eps, lo, hi))
    return tuple(lo), tuple(hi)


def transfer_axis(dst_origin, dst_h, dst_n, src_origin, src_h, src_n, order):
    """(base int32[dst_n], weights float64[dst_n, order + 1]) of one axis, computed by the library."""
    import numpy as np
    base = np.empty(dst_n, dtype=np.int32)
    w = np.empty((dst_n, order + 1), dtype=np.float64)
    _check(_native.lib().nvp_transfer_axis(dst_origin, dst_h, dst_n, src_origin, src_h, src_n, order,
                                           base.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                                           w.ctypes.data_as(ctypes.POINTER(ctypes.c_double))))
    return base, w


def circulant_size(n):
    m = ctypes.c_int64()
    _check(_native.lib().nvp_circulant_size(n, ctypes.byref(m)))
    return m.value


def transform_lengths():
    """The compiled transform lengths (circulant sizes per axis), increasing."""
    L = _native.lib()
    n = ctypes.c_int()
    _check(L.nvp_transform_lengths(None, 0, ctypes.byref(n)))
    buf = (ctypes.c_int32 * n.value)()
    _check(L.nvp_transform_lengths(buf, n.value, ctypes.byref(n)))
    return [int(v) for v in buf]


# ------------------------------------------------------------- context

def _ptr(t):
    return ctypes.c_void_p(t.data_ptr())


def _need(t, dtype, numel, what):
    if not isinstance(t, torch.Tensor) or t.device.type != "cuda":
        raise ValueError("%s must be a CUDA (HIP) tensor" % what)
    if t.dtype != dtype or not t.is_contiguous() or t.numel() != numel:
        raise ValueError("%s must be contiguous %s with %d elements" % (what, dtype, numel))


class Context:
    """nvp_ctx bound to a device and a HIP stream (default: torch's current stream)."""

    def __init__(self, device=0, stream=None):
        dev = torch.device("cuda", device) if isinstance(device, int) else torch.device(device)
        self.device = dev
        if stream is None:
            stream = torch.cuda.current_stream(dev)
        self.stream = stream
        h = ctypes.c_void_p()
        _check(_native.lib().nvp_ctx_create(dev.index or 0, ctypes.c_void_p(stream.cuda_stream), ctypes.byref(h)))
        self.handle = h
        self._users = weakref.WeakSet()  # plans, batches and networks made with this context

    def sync(self):
        _check(_native.lib().nvp_ctx_sync(self.handle), self.handle)

    def close(self):
        """Destroys the context after every plan, batch and network still made with it."""
        if self.handle:
            for u in list(self._users):
                u.close()
            _native.lib().nvp_ctx_destroy(self.handle)
            self.handle = None

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def incident_field(ctx, k, scale, points, g, prec=NVP_C64, out=None):
    """scale * sum_j exp(i k r) / (4 pi r) over the points (float64 CUDA tensor [n, 3]) at the centres of g."""
    g = grid(g)
    n = tuple(g.n)
    _points(points)
    dtype = torch.complex128 if prec == NVP_C128 else torch.complex64
    if out is None:
        out = torch.empty(n, dtype=dtype, device=points.device)
    _need(out, dtype, n[0] * n[1] * n[2], "out")
    k, scale = complex(k), complex(scale)
    _check(_native.lib().nvp_incident_field(ctx.handle, k.real, k.imag, scale.real, scale.imag, _ptr(points),
                                            points.shape[0], ctypes.byref(g), _ptr(out), prec), ctx.handle)
    return out


def _points(points, what="points"):
    if not isinstance(points, torch.Tensor) or points.device.type != "cuda" or points.dtype != torch.float64 \
            or not points.is_contiguous() or points.dim() != 2 or points.shape[1] != 3:
        raise ValueError("%s must be a contiguous float64 CUDA tensor of shape (n, 3)" % what)
    return points


def incident_at(ctx, k, scale, points, targets, prec=NVP_C64, out=None):
    """The incident_field sum at arbitrary targets (float64 CUDA tensor [m, 3])."""
    _points(points)
    _points(targets, "targets")
    dtype = torch.complex128 if prec == NVP_C128 else torch.complex64
    if out is None:
        out = torch.empty(targets.shape[0], dtype=dtype, device=points.device)
    _need(out, dtype, targets.shape[0], "out")
    k, scale = complex(k), complex(scale)
    _check(_native.lib().nvp_incident_at(ctx.handle, k.real, k.imag, scale.real, scale.imag, _ptr(points),
                                         points.shape[0], _ptr(targets), targets.shape[0], _ptr(out), prec),
           ctx.handle)
    return out


def radiated_power(ctx, k, scale, points, centre, radius, rho0, c0, n_r=512, n_theta=512):
    """Power through the disc x = centre[0] of the given radius (midpoint rule, n_r x n_theta nodes)."""
    _points(points)
    k, scale = complex(k), complex(scale)
    c = (ctypes.c_double * 3)(*[float(v) for v in centre])
    out = ctypes.c_double()
    _check(_native.lib().nvp_radiated_power(ctx.handle, k.real, k.imag, scale.real, scale.imag, _ptr(points),
                                            points.shape[0], c, float(radius), float(rho0), float(c0), int(n_r),
                                            int(n_theta), ctypes.byref(out)), ctx.handle)
    return out.value


def vie_solve(ctx, kb, g, q, rhs, p=None, tol=1e-10, max_iter=500):
    """Solve p - sum_j K_kb(x_i - x_j) q_j p_j = rhs on grid g (BiCGStab); p: initial guess (zeros if None).
    Returns (p, iterations, true relative residual)."""
    g = grid(g)
    n = tuple(g.n)
    numel = n[0] * n[1] * n[2]
    _need(q, q.dtype, numel, "q")
    _need(rhs, q.dtype, numel, "rhs")
    if p is None:
        p = torch.zeros(n, dtype=q.dtype, device=q.device)
    _need(p, q.dtype, numel, "p")
    kb = complex(kb)
    it, rr = ctypes.c_int(), ctypes.c_double()
    _check(_native.lib().nvp_vie_solve(ctx.handle, kb.real, kb.imag, ctypes.byref(g), _ptr(q), _ptr(rhs), _ptr(p),
                                       prec_of(q.dtype), float(tol), int(max_iter), ctypes.byref(it),
                                       ctypes.byref(rr)), ctx.handle)
    return p, it.value, rr.value


def set_quadrature(ctx, rule):
    """Quadrature rule of the context's later potentials, solves and plans (NVP_QUAD_BALL: the
    paper's; NVP_QUAD_CORRECTED: the corrected lattice rule)."""
    _check(_native.lib().nvp_ctx_set_quadrature(ctx.handle, int(rule)), ctx.handle)


def quadrature_weights(rule, k, h):
    """(K(0), face addition) of a quadrature rule, complex."""
    w = (ctypes.c_double * 4)()
    k = complex(k)
    _check(_native.lib().nvp_quadrature_weights(int(rule), k.real, k.imag, float(h), w))
    return complex(w[0], w[1]), complex(w[2], w[3])


def difference_term(ctx, gt, out, ga, a, zero_a, gb, b, zero_b, order, scale):
    """out += scale * T(a) * conj(T(b)) on grid gt (in place; out, a, b of one complex dtype)."""
    gt, ga, gb = grid(gt), grid(ga), grid(gb)
    prec = prec_of(out.dtype)
    for t, g, what in ((out, gt, "out"), (a, ga, "a"), (b, gb, "b")):
        _need(t, out.dtype, int(g.n[0] * g.n[1] * g.n[2]), what)
    _check(_native.lib().nvp_difference_term(ctx.handle, ctypes.byref(gt), _ptr(out), ctypes.byref(ga), _ptr(a),
                                             int(bool(zero_a)), ctypes.byref(gb), _ptr(b), int(bool(zero_b)),
                                             int(order), float(scale), prec), ctx.handle)
    return out


def volume_potential(ctx, k, g, f, out=None):
    """u = -sum_j K(x_i - x_j) f_j on grid g (complex64 or complex128 f of shape g.n)."""
    g = grid(g)
    n = tuple(g.n)
    prec = prec_of(f.dtype)
    _need(f, f.dtype, n[0] * n[1] * n[2], "f")
    if out is None:
        out = torch.empty(n, dtype=f.dtype, device=f.device)
    _need(out, f.dtype, n[0] * n[1] * n[2], "out")
    k = complex(k)
    _check(_native.lib().nvp_volume_potential(ctx.handle, k.real, k.imag, ctypes.byref(g), _ptr(f), _ptr(out), prec),
           ctx.handle)
    return out


def volume_potential_box(ctx, k, g, f, box, scale, out=None):
    """u = scale * sum_{j in box} K(x_i - x_j) f_j on all of grid g; box: 6 inclusive voxel indices
    (lo_x, lo_y, lo_z, hi_x, hi_y, hi_z) or None for the whole grid.  scale = C_n gives p_n."""
    g = grid(g)
    n = tuple(g.n)
    prec = prec_of(f.dtype)
    _need(f, f.dtype, n[0] * n[1] * n[2], "f")
    if out is None:
        out = torch.empty(n, dtype=f.dtype, device=f.device)
    _need(out, f.dtype, n[0] * n[1] * n[2], "out")
    k = complex(k)
    b = None if box is None else (ctypes.c_int64 * 6)(*[int(v) for v in box])
    _check(_native.lib().nvp_volume_potential_box(ctx.handle, k.real, k.imag, ctypes.byref(g), _ptr(f), b,
                                                  float(scale), _ptr(out), prec), ctx.handle)
    return out


def field_lin3(ctx, out, a=None, b=None, c=None, al=0.0, be=0.0):
    """out = a + al b + be c on device tensors of one complex dtype (None operands count as zero)."""
    prec = prec_of(out.dtype)
    n = out.numel()
    for t, w in ((a, "a"), (b, "b"), (c, "c")):
        if t is not None:
            _need(t, out.dtype, n, w)
    al, be = complex(al), complex(be)
    A = (ctypes.c_double * 2)(al.real, al.imag)
    B = (ctypes.c_double * 2)(be.real, be.imag)
    p = lambda t: None if t is None else _ptr(t)  # noqa: E731
    _check(_native.lib().nvp_field_lin3(ctx.handle, n, _ptr(out), p(a), p(b), p(c), A, B, prec), ctx.handle)
    return out


def field_diff_norms(ctx, a, b):
    """(sum |a - b|^2, sum |a|^2) in FP64 for device tensors of one complex dtype."""
    prec = prec_of(a.dtype)
    _need(b, a.dtype, a.numel(), "b")
    out = (ctypes.c_double * 2)()
    _check(_native.lib().nvp_field_diff_norms(ctx.handle, a.numel(), _ptr(a), _ptr(b), prec, out), ctx.handle)
    return float(out[0]), float(out[1])


def volume_potential_noalloc(ctx, k, g, f, out):
    """nvp_volume_potential_noalloc: the operator of volume_potential with the library's fixed device
    scratch (no device allocation in the call); `out` is the caller's output tensor."""
    g = grid(g)
    n = tuple(g.n)
    prec = prec_of(f.dtype)
    _need(f, f.dtype, n[0] * n[1] * n[2], "f")
    _need(out, f.dtype, n[0] * n[1] * n[2], "out")
    k = complex(k)
    _check(_native.lib().nvp_volume_potential_noalloc(ctx.handle, k.real, k.imag, ctypes.byref(g), _ptr(f),
                                                      _ptr(out), prec), ctx.handle)
    return out


class CascadePlan:
    """nvp_plan of harmonics 2..n_harm on their own grids."""

    def __init__(self, ctx, med, f0, g1, grids, prec=NVP_C64, order=1):
        self.ctx = ctx
        self.g1 = grid(g1)
        self.grids = [grid(g) for g in grids]
        self.n_harm = len(self.grids) + 1
        self.prec = prec
        self.dtype = _DT[prec]
        arr = (Grid * len(self.grids))(*self.grids)
        h = ctypes.c_void_p()
        _check(_native.lib().nvp_plan_cascade(ctx.handle, ctypes.byref(medium(med)), f0, self.n_harm,
                                              ctypes.byref(self.g1), arr, prec, order, ctypes.byref(h)), ctx.handle)
        self.handle = h
        ctx._users.add(self)

    def shape(self, n):
        g = self.g1 if n == 1 else self.grids[n - 2]
        return tuple(g.n)

    def regrid(self, n, g):
        """Replace harmonic n's grid (nvp_plan_regrid): tables laid out again, the other
        harmonics' kernel spectra kept."""
        g = grid(g)
        _check(_native.lib().nvp_plan_regrid(self.handle, int(n), ctypes.byref(g)), self.ctx.handle)
        self.grids[n - 2] = g

    def workspace_bytes(self):
        b = ctypes.c_size_t()
        _check(_native.lib().nvp_plan_workspace_bytes(self.handle, ctypes.byref(b)))
        return b.value

    def work_bytes(self):
        """Least size of a caller workspace (the plan's transient work buffers)."""
        b = ctypes.c_size_t()
        _check(_native.lib().nvp_plan_work_bytes(self.handle, ctypes.byref(b)))
        return b.value

    def set_workspace(self, ws):
        """Run in the caller's device memory `ws` (a tensor of at least work_bytes() bytes, kept alive
        here), or in work buffers of the plan's own again (ws None)."""
        if ws is None:
            _check(_native.lib().nvp_plan_set_workspace(self.handle, None, 0), self.ctx.handle)
        else:
            nbytes = ws.numel() * ws.element_size()
            _check(_native.lib().nvp_plan_set_workspace(self.handle, ctypes.c_void_p(ws.data_ptr()), nbytes),
                   self.ctx.handle)
        self._ws = ws

    def set_kernel_cache(self, enable):
        _check(_native.lib().nvp_plan_set_kernel_cache(self.handle, int(bool(enable))))

    def set_overlap(self, enable):
        """Kernel spectra on a second stream, concurrently with the convolutions (default on)."""
        _check(_native.lib().nvp_plan_set_overlap(self.handle, int(bool(enable))))

    def set_timing(self, enable):
        _check(_native.lib().nvp_plan_set_timing(self.handle, int(bool(enable))))

    def get_timing(self):
        k = len(TIMING_KINDS)
        ms = (ctypes.c_double * k)()
        cnt = (ctypes.c_int64 * k)()
        _check(_native.lib().nvp_plan_get_timing(self.handle, ms, cnt, k), self.ctx.handle)
        return {name: (ms[i], cnt[i]) for i, name in enumerate(TIMING_KINDS)}

    def _sz(self, n):
        s = self.shape(n)
        return s[0] * s[1] * s[2]

    def execute_harmonic(self, n, fields, out=None):
        """fields[m-1] = p_m on its grid, m = 1..n-1; returns p_n."""
        if len(fields) != n - 1:
            raise ValueError("harmonic %d needs %d fields" % (n, n - 1))
        for m, f in enumerate(fields, start=1):
            _need(f, self.dtype, self._sz(m), "p_%d" % m)
        if out is None:
            out = torch.empty(self.shape(n), dtype=self.dtype, device=fields[0].device)
        _need(out, self.dtype, self._sz(n), "out")
        arr = (ctypes.c_void_p * len(fields))(*[f.data_ptr() for f in fields])
        _check(_native.lib().nvp_execute_harmonic(self.handle, n, arr, _ptr(out)), self.ctx.handle)
        return out

    def source_term(self, n, fields, out=None):
        """f_n on the grid of harmonic n from fields[m-1] = p_m, m = 1..n-1."""
        if len(fields) != n - 1:
            raise ValueError("harmonic %d needs %d fields" % (n, n - 1))
        for m, f in enumerate(fields, start=1):
            _need(f, self.dtype, self._sz(m), "p_%d" % m)
        if out is None:
            out = torch.empty(self.shape(n), dtype=self.dtype, device=fields[0].device)
        _need(out, self.dtype, self._sz(n), "out")
        arr = (ctypes.c_void_p * len(fields))(*[f.data_ptr() for f in fields])
        _check(_native.lib().nvp_source_term(self.handle, n, arr, _ptr(out)), self.ctx.handle)
        return out

    def autotune(self, cache_path=None, reps=3):
        """Time the launch choices of each harmonic and keep the fastest (optionally through a cache file)."""
        _check(_native.lib().nvp_plan_autotune(self.handle, cache_path.encode() if cache_path else None, reps),
               self.ctx.handle)

    def tuning(self, n):
        c = (ctypes.c_int * 5)()
        _check(_native.lib().nvp_plan_get_tuning(self.handle, n, c))
        return dict(x_tile=c[0], y_tile=c[1], quads=c[2], src=c[3], src_cx=c[4])

    def set_tuning(self, n, x_tile=0, y_tile=0, quads=0, src=-1, src_cx=0):
        """Launch choices of harmonic n (see tuning())."""
        c = (ctypes.c_int * 5)(x_tile, y_tile, quads, src, src_cx)
        _check(_native.lib().nvp_plan_set_tuning(self.handle, n, c), self.ctx.handle)

    def execute(self, p1, outs=None):
        """p1 on g1 -> [p_2, ..., p_n_harm]."""
        _need(p1, self.dtype, self._sz(1), "p1")
        if outs is None:
            outs = [torch.empty(self.shape(n), dtype=self.dtype, device=p1.device)
                    for n in range(2, self.n_harm + 1)]
        for n, o in zip(range(2, self.n_harm + 1), outs):
            _need(o, self.dtype, self._sz(n), "p_%d" % n)
        arr = (ctypes.c_void_p * len(outs))(*[o.data_ptr() for o in outs])
        _check(_native.lib().nvp_execute_cascade(self.handle, _ptr(p1), arr), self.ctx.handle)
        return outs

    def close(self):
        if self.handle:
            _native.lib().nvp_plan_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Batch:
    """nvp_batch: many cascades executed together (as one HIP graph from the second execution on)."""

    def __init__(self, ctx, problems, prec=NVP_C64, order=1):
        """problems: list of dicts with med, f0, g1, grids (the grids of p_2..p_n)."""
        self.ctx = ctx
        self.prec = prec
        self.dtype = _DT[prec]
        self._gn = []
        arr = (Problem * len(problems))()
        self.shapes = []
        for i, pr in enumerate(problems):
            gn = (Grid * len(pr["grids"]))(*[grid(g) for g in pr["grids"]])
            self._gn.append(gn)
            g1 = grid(pr["g1"])
            arr[i] = Problem(medium(pr["med"]), float(pr["f0"]), len(pr["grids"]) + 1, g1,
                             ctypes.cast(gn, ctypes.POINTER(Grid)))
            self.shapes.append([tuple(g1.n)] + [tuple(g.n) for g in gn])
        h = ctypes.c_void_p()
        _check(_native.lib().nvp_batch_create(ctx.handle, len(problems), arr, prec, order, ctypes.byref(h)),
               ctx.handle)
        self.handle = h
        ctx._users.add(self)

    def set_graph(self, enable, branches=4):
        _check(_native.lib().nvp_batch_set_graph(self.handle, int(bool(enable)), branches), self.ctx.handle)

    def set_grouped(self, enable):
        """Multi-task launches per pass and transform length (level by level over the problems)."""
        _check(_native.lib().nvp_batch_set_grouped(self.handle, int(bool(enable))), self.ctx.handle)

    def autotune(self, cache_path=None, reps=3):
        _check(_native.lib().nvp_batch_autotune(self.handle, cache_path.encode() if cache_path else None, reps),
               self.ctx.handle)

    def outputs(self, device="cuda"):
        """Freshly allocated outputs: per problem, [p_2, ..., p_n]."""
        return [[torch.empty(s, dtype=self.dtype, device=device) for s in sh[1:]] for sh in self.shapes]

    def execute(self, p1s, outs):
        """p1s[i]: p_1 of problem i; outs[i]: its [p_2, ..., p_n] (written)."""
        ins, flat = [], []
        for i, sh in enumerate(self.shapes):
            _need(p1s[i], self.dtype, sh[0][0] * sh[0][1] * sh[0][2], "p1 of problem %d" % i)
            ins.append(p1s[i].data_ptr())
            for j, s in enumerate(sh[1:]):
                _need(outs[i][j], self.dtype, s[0] * s[1] * s[2], "output %d of problem %d" % (j, i))
                flat.append(outs[i][j].data_ptr())
        a = (ctypes.c_void_p * len(ins))(*ins)
        b = (ctypes.c_void_p * len(flat))(*flat)
        _check(_native.lib().nvp_batch_execute(self.handle, a, b), self.ctx.handle)
        return outs

    def close(self):
        if self.handle:
            _native.lib().nvp_batch_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ------------------------------------------------------------- truncation boxes

def qbox(ctx, f, q0):
    """Localisation boxes of f (3-D complex tensor) for thresholds q0: int64 array [len(q0)][6]."""
    import numpy as np
    n = tuple(f.shape)
    if len(n) != 3:
        raise ValueError("f must be 3-D")
    _need(f, f.dtype, n[0] * n[1] * n[2], "f")
    q = np.ascontiguousarray(np.asarray(q0, dtype=np.float64).reshape(-1))
    box = np.zeros((len(q), 6), dtype=np.int64)
    _check(_native.lib().nvp_qbox(ctx.handle, _i3(n), _ptr(f), prec_of(f.dtype), len(q),
                                  q.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                  box.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))), ctx.handle)
    return box


def box_potential(ctx, k, g, f, target, boxes):
    """-sum over each box of K(x_target - x_j) f_j; complex128 numpy array, one value per box."""
    import numpy as np
    g = grid(g)
    n = tuple(g.n)
    _need(f, f.dtype, n[0] * n[1] * n[2], "f")
    b = np.ascontiguousarray(np.asarray(boxes, dtype=np.int64).reshape(-1, 6))
    out = np.zeros(2 * len(b), dtype=np.float64)
    k = complex(k)
    _check(_native.lib().nvp_box_potential(ctx.handle, k.real, k.imag, ctypes.byref(g), _ptr(f), prec_of(f.dtype),
                                           _i3(target), len(b), b.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                                           out.ctypes.data_as(ctypes.POINTER(ctypes.c_double))), ctx.handle)
    return out[0::2] + 1j * out[1::2]


# ------------------------------------------------------------- box predictor

BOXNET_PARAMS = 8899
BOXNET_IN, BOXNET_OUT = 5, 3


class BoxNet:
    """nvp_boxnet: the box-predictor MLP; inputs and targets are float32 CUDA tensors."""

    def __init__(self, ctx, max_batch):
        self.ctx = ctx
        self.max_batch = int(max_batch)
        h = ctypes.c_void_p()
        _check(_native.lib().nvp_boxnet_create(ctx.handle, self.max_batch, ctypes.byref(h)), ctx.handle)
        self.handle = h
        ctx._users.add(self)

    def set_params(self, params):
        import numpy as np
        p = np.ascontiguousarray(np.asarray(params, dtype=np.float32).reshape(-1))
        _check(_native.lib().nvp_boxnet_set_params(self.handle, p.ctypes.data_as(ctypes.POINTER(ctypes.c_float)),
                                                   p.size), self.ctx.handle)

    def get_params(self):
        import numpy as np
        p = np.zeros(BOXNET_PARAMS, dtype=np.float32)
        _check(_native.lib().nvp_boxnet_get_params(self.handle, p.ctypes.data_as(ctypes.POINTER(ctypes.c_float)),
                                                   p.size), self.ctx.handle)
        return p

    def set_norm(self, mean, std):
        import numpy as np
        m = np.ascontiguousarray(np.asarray(mean, dtype=np.float32))
        s = np.ascontiguousarray(np.asarray(std, dtype=np.float32))
        _check(_native.lib().nvp_boxnet_set_norm(self.handle, m.ctypes.data_as(ctypes.POINTER(ctypes.c_float)),
                                                 s.ctypes.data_as(ctypes.POINTER(ctypes.c_float))), self.ctx.handle)

    def _io(self, x, t=None):
        B = x.shape[0]
        if not 1 <= B <= self.max_batch:
            raise ValueError("batch of %d outside 1..%d" % (B, self.max_batch))
        _need(x, torch.float32, B * BOXNET_IN, "x")
        if t is not None:
            _need(t, torch.float32, B * BOXNET_OUT, "t")
        return B

    def predict(self, x, out=None):
        B = self._io(x)
        if out is None:
            out = torch.empty((B, BOXNET_OUT), dtype=torch.float32, device=x.device)
        _need(out, torch.float32, B * BOXNET_OUT, "out")
        _check(_native.lib().nvp_boxnet_predict(self.handle, B, _ptr(x), _ptr(out)), self.ctx.handle)
        return out

    def grads(self, x, t, tau):
        """(gradient tensor [8899], loss) without updating the parameters."""
        B = self._io(x, t)
        g = torch.empty(BOXNET_PARAMS, dtype=torch.float32, device=x.device)
        loss = ctypes.c_float()
        _check(_native.lib().nvp_boxnet_grads(self.handle, B, _ptr(x), _ptr(t), float(tau), _ptr(g),
                                              ctypes.byref(loss)), self.ctx.handle)
        return g, loss.value

    def train_step(self, x, t, tau, lr, want_loss=True):
        B = self._io(x, t)
        loss = ctypes.c_float()
        _check(_native.lib().nvp_boxnet_train_step(self.handle, B, _ptr(x), _ptr(t), float(tau), float(lr),
                                                   ctypes.byref(loss) if want_loss else None), self.ctx.handle)
        return loss.value if want_loss else None

    def close(self):
        if self.handle:
            _native.lib().nvp_boxnet_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
