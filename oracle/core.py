"""ORACLE — test infrastructure only (see the package docstring).

Plain FP64 statement of the nested-mesh volume-potential cascade of Groth et
al. (arXiv 2011.03009), in the paper's order and notation:

  Section 2, equation "power_law" and the line after "cascade_1":
      k_n = n w / c0 + i alpha(n w)
  Section 2, equation "cascade_2", solved by the volume potential of
  Section 3, equations "vol_pot"/"vol_pot_approx"/"harm2"-"harm5":
      p_n = -(beta w^2 n^2 / (2 rho0 c0^4)) int_{D_n} G_{k_n} f_n,
      f_n = sum_{m=1}^{n-1} p_m p_{n-m}
  Section 3.1, equation "quad": midpoint rule off the diagonal, equal-volume
      sphere on the self voxel; the discrete operator is Toeplitz and the
      paper evaluates it by circulant embedding and the FFT.
  Section 6 (the nested-mesh algorithm): harmonic i on its own box D_i with
      spacing lambda_i / 6; lower harmonics interpolated onto the new mesh
      (linear in the paper; higher order recommended there for accuracy).

Readings of passages that the paper leaves open are stated where they are
used (attenuation units, grid alignment, transfer boundary handling).
"""

import ctypes
import math
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_DIR = os.path.join(_HERE, "_build")
_LIB_PATH = os.path.join(_LIB_DIR, "liboracle_vp.so")
_lib = None


# --------------------------------------------------------------------------
# native direct sum (vp_direct.c)
# --------------------------------------------------------------------------

def build(force=True):
    """Compile vp_direct.c with gcc (plain FP64, no fast-math)."""
    if not force and os.path.exists(_LIB_PATH):
        return _LIB_PATH
    os.makedirs(_LIB_DIR, exist_ok=True)
    tmp = _LIB_PATH + ".tmp%d" % os.getpid()
    cmd = ["gcc", "-O2", "-fopenmp", "-ffp-contract=off", "-fPIC", "-shared",
           os.path.join(_HERE, "vp_direct.c"), "-o", tmp, "-lm"]
    subprocess.check_call(cmd)
    os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build()
        lib = ctypes.CDLL(_LIB_PATH)
        i64p = ctypes.POINTER(ctypes.c_int64)
        dp = ctypes.POINTER(ctypes.c_double)
        lib.oracle_conv_direct.argtypes = [i64p, ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                           dp, ctypes.c_int64, i64p, dp]
        lib.oracle_conv_direct.restype = ctypes.c_int
        lib.oracle_kernel_table.argtypes = [i64p, ctypes.c_double, ctypes.c_double, ctypes.c_double, dp]
        lib.oracle_kernel_table.restype = ctypes.c_int
        _lib = lib
    return _lib


def _i64arr(v):
    return (ctypes.c_int64 * len(v))(*[int(x) for x in v])


# --------------------------------------------------------------------------
# constants (Section 2)
# --------------------------------------------------------------------------

def angular_frequency(f0):
    return 2.0 * math.pi * f0


def attenuation(alpha0_db, eta, f_hz):
    """Power-law attenuation in Np/m at frequency f_hz.

    Reading: the medium table gives alpha0 in dB/m at 1 MHz with eta the
    frequency exponent (its header is garbled), so
    alpha(f) = alpha0 (f / 1 MHz)^eta / (20 log10 e).
    """
    return alpha0_db * (f_hz / 1.0e6) ** eta / (20.0 * math.log10(math.e))


def wavenumber(n, f0, medium):
    """k_n = n w / c0 + i alpha(n f0) (equation "power_law" with n w)."""
    return complex(2.0 * math.pi * n * f0 / medium["c0"],
                   attenuation(medium["alpha0_db"], medium["eta"], n * f0))


def cascade_constant(n, f0, medium):
    """C_n with p_n = C_n int G f_n: -(beta w^2 n^2) / (2 rho0 c0^4) (eqs. cascade_2, vol_pot)."""
    w = angular_frequency(f0)
    return -medium["beta"] * w * w * n * n / (2.0 * medium["rho0"] * medium["c0"] ** 4)


def wavelength(n, f0, c0):
    return c0 / (n * f0)


def spacing(n, f0, c0, n_w=6):
    """delta x = lambda_n / n_w (Section 3.3: n_w = 6 voxels per own wavelength)."""
    return wavelength(n, f0, c0) / n_w


# --------------------------------------------------------------------------
# grids (Section 3.1 voxel meshes; Section 5 domains; Section 6 step 1)
# --------------------------------------------------------------------------

class Grid:
    """Voxel centres origin + i h, i in [0, n) per axis; arrays are C order, z fastest."""

    def __init__(self, origin, h, n):
        self.origin = tuple(float(o) for o in origin)
        self.h = float(h)
        self.n = tuple(int(v) for v in n)

    def coords(self, axis):
        return self.origin[axis] + np.arange(self.n[axis], dtype=np.float64) * self.h

    def size(self):
        return self.n[0] * self.n[1] * self.n[2]

    def same_as(self, other):
        return self.origin == other.origin and self.h == other.h and self.n == other.n

    def __repr__(self):
        return "Grid(origin=%r, h=%r, n=%r)" % (self.origin, self.h, self.n)


def _nint(x):
    """Round half up (the same rule on every side that builds grids)."""
    return int(math.floor(x + 0.5))


def grid_from_counts(focus, h, n, i_f):
    """Reading: the focus is the centre of voxel i_f on every axis."""
    return Grid([focus[a] - i_f[a] * h for a in range(3)], h, n)


def grid_from_box(focus, lo, hi, h):
    """Voxel grid of a cuboid [lo, hi] at spacing h whose voxel i_f sits on the focus.

    n_a = max(1, nint((hi_a - lo_a) / h)), i_f,a = nint((focus_a - lo_a) / h).
    """
    n = [max(1, _nint((hi[a] - lo[a]) / h)) for a in range(3)]
    i_f = [_nint((focus[a] - lo[a]) / h) for a in range(3)]
    return grid_from_counts(focus, h, n, i_f), tuple(i_f)


def reference_box(l, R, d, eps=1.0e-4):
    """D_2 = [l - L, l + d] x [-R, R]^2, L = sqrt(l^2 - R^2) - eps (equation "domain")."""
    L = math.sqrt(l * l - R * R) - eps
    return (l - L, -R, -R), (l + d, R, R)


def rule_of_thumb_box(n, l, R, d, eps=1.0e-4):
    """D_n: pre-focal length and width of D_2 scaled by lambda_n / lambda_2 = 2 / n; post-focal d fixed.

    Reading: the rule of thumb's formula (Section 5) rather than its table row.
    """
    L = math.sqrt(l * l - R * R) - eps
    s = 2.0 / n
    return (l - s * L, -s * R, -s * R), (l + d, s * R, s * R)


# --------------------------------------------------------------------------
# kernel of the quadrature (Section 3.1, equation "quad")
# --------------------------------------------------------------------------

def self_cell(k, h):
    """Integral of G_k over the ball of the voxel's volume about its centre."""
    a = (3.0 / (4.0 * math.pi)) ** (1.0 / 3.0) * h
    k = complex(k)
    return (np.exp(1j * k * a) * (1.0 - 1j * k * a) - 1.0) / (k * k)


def kernel_offsets(k, h, n):
    """K at voxel offsets [0,n0) x [0,n1) x [0,n2): h^3 G_k(|d| h), self voxel from self_cell."""
    k = complex(k)
    a = np.arange(n[0], dtype=np.float64)[:, None, None]
    b = np.arange(n[1], dtype=np.float64)[None, :, None]
    c = np.arange(n[2], dtype=np.float64)[None, None, :]
    r = h * np.sqrt(a * a + b * b + c * c)
    r[0, 0, 0] = 1.0
    K = h ** 3 * np.exp(1j * k * r) / (4.0 * math.pi * r)
    K[0, 0, 0] = self_cell(k, h)
    return K


# --------------------------------------------------------------------------
# the discrete operator  out_i = sum_j K(x_i - x_j) f_j
# --------------------------------------------------------------------------

def conv_direct(f, h, k, targets=None):
    """Direct O(N^2) sum (the definition).  targets: flat C-order indices, or None for all."""
    lib = _load()
    f = np.ascontiguousarray(f, dtype=np.complex128)
    n = f.shape
    k = complex(k)
    if targets is None:
        out = np.empty(n, dtype=np.complex128)
        nt, tp = 0, None
    else:
        targets = np.ascontiguousarray(targets, dtype=np.int64)
        out = np.empty(targets.shape[0], dtype=np.complex128)
        nt = targets.shape[0]
        tp = targets.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))
    rc = lib.oracle_conv_direct(_i64arr(n), h, k.real, k.imag,
                                f.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), nt, tp,
                                out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
    if rc != 0:
        raise MemoryError("oracle_conv_direct failed (%d)" % rc)
    return out


def embedded_kernel(k, h, n, M):
    """Circulant embedding: K(d) at d mod M for |d| <= n - 1 per axis, zero elsewhere.

    The paper embeds the Toeplitz operator in a circulant of twice the size
    (Section 3.1); any M >= 2n - 1 is exact.
    """
    Kt = kernel_offsets(k, h, n)
    Kc = np.zeros(M, dtype=np.complex128)
    idx = []
    src = []
    for a in range(3):
        d = np.arange(-(n[a] - 1), n[a])
        idx.append(np.mod(d, M[a]))
        src.append(np.abs(d))
    Kc[np.ix_(*idx)] = Kt[np.ix_(*src)]
    return Kc


def conv_circulant(f, h, k, M=None, workers=None):
    """The same sum by the circulant FFT (library FFT, FP64); M defaults to 2n."""
    import scipy.fft as sfft
    f = np.asarray(f, dtype=np.complex128)
    n = f.shape
    if M is None:
        M = tuple(2 * v for v in n)
    if workers is None:
        workers = os.cpu_count() or 1
    Kc = embedded_kernel(k, h, n, M)
    F = np.zeros(M, dtype=np.complex128)
    F[:n[0], :n[1], :n[2]] = f
    U = sfft.ifftn(sfft.fftn(Kc, workers=workers) * sfft.fftn(F, workers=workers), workers=workers)
    return np.ascontiguousarray(U[:n[0], :n[1], :n[2]])


def volume_potential(f, h, k, method="direct", M=None):
    """u = -int_D G_k f, discretised by equation "quad" (equation "vol_pot_approx")."""
    if method == "direct":
        return -conv_direct(f, h, k)
    return -conv_circulant(f, h, k, M=M)


# --------------------------------------------------------------------------
# transfer between meshes (Section 6, step 2(a))
# --------------------------------------------------------------------------

def transfer_axis(dst_origin, dst_h, dst_n, src_origin, src_h, src_n, order):
    """Base index and weights of 1-D interpolation from a source axis onto target centres.

    Reading: target coordinates are clamped into the source hull (constant
    extension); order 1 is the paper's linear interpolation, order 3 the
    four-point Lagrange interpolant with its stencil shifted inward at edges.
    Returns (base: int64[dst_n], w: float64[dst_n, order + 1]).
    """
    if order not in (1, 3):
        raise ValueError("order must be 1 or 3")
    if src_n < order + 1:
        raise ValueError("source axis too short for this order")
    x = dst_origin + np.arange(dst_n, dtype=np.float64) * dst_h
    s = (x - src_origin) / src_h
    s = np.minimum(np.maximum(s, 0.0), float(src_n - 1))
    i0 = np.minimum(np.floor(s), float(src_n - 2))
    if order == 1:
        t = s - i0
        return i0.astype(np.int64), np.stack([1.0 - t, t], axis=1)
    base = np.minimum(np.maximum(i0 - 1.0, 0.0), float(src_n - 4))
    u = s - base
    w = np.stack([-(u - 1.0) * (u - 2.0) * (u - 3.0) / 6.0,
                  u * (u - 2.0) * (u - 3.0) / 2.0,
                  -u * (u - 1.0) * (u - 3.0) / 2.0,
                  u * (u - 1.0) * (u - 2.0) / 6.0], axis=1)
    return base.astype(np.int64), w


def transfer(field, src, dst, order):
    """Tensor-product interpolation of `field` (on grid src) at the centres of grid dst.

    A tensor-product interpolant applies the 1-D rule along each axis in
    turn; that is how it is evaluated here.  Reading: a field on the very
    grid it is wanted on is passed through unchanged.
    """
    field = np.asarray(field, dtype=np.complex128)
    if src.same_as(dst):
        return field.copy()
    out = field
    for a in range(3):
        base, w = transfer_axis(dst.origin[a], dst.h, dst.n[a], src.origin[a], src.h, src.n[a], order)
        acc = None
        for j in range(w.shape[1]):
            taken = np.take(out, base + j, axis=a)
            sh = [1, 1, 1]
            sh[a] = dst.n[a]
            term = taken * w[:, j].reshape(sh)
            acc = term if acc is None else acc + term
        out = acc
    return out


# --------------------------------------------------------------------------
# source term, one harmonic, the cascade (equations cascade_2, harm2-harm5;
# the nested-mesh algorithm of Section 6)
# --------------------------------------------------------------------------

def source_term(n, v):
    """f_n = sum_{m=1}^{n-1} v_m v_{n-m} (no conjugates; the terms with i + j > n dropped)."""
    f = None
    for m in range(1, n):
        t = v[m] * v[n - m]
        f = t if f is None else f + t
    return f


def harmonic(n, fields, grid, f0, medium, order, method="direct", targets=None, M=None, rule="ball"):
    """p_n on `grid` from lower harmonics fields = {m: (array, Grid)} for m = 1..n-1.

    method "direct": the definition; "fft": the circulant cross-check;
    targets (direct only): flat indices of the voxels to evaluate;
    rule "ball": equation "quad" of the paper, "corrected": the corrected
    quadrature of oracle/quadrature.py (every voxel).
    """
    v = {m: transfer(fields[m][0], fields[m][1], grid, order) for m in range(1, n)}
    f = source_term(n, v)
    k = wavenumber(n, f0, medium)
    C = cascade_constant(n, f0, medium)
    if rule == "corrected":
        from . import quadrature
        if targets is not None:
            raise ValueError("the corrected rule evaluates every voxel")
        if method == "direct":
            return C * quadrature.conv_direct_corrected(f, grid.h, k)
        return C * quadrature.conv_circulant_corrected(f, grid.h, k, M=M)
    if rule != "ball":
        raise ValueError("rule must be 'ball' or 'corrected'")
    if method == "direct":
        return C * conv_direct(f, grid.h, k, targets=targets)
    if targets is not None:
        raise ValueError("targets need method='direct'")
    return C * conv_circulant(f, grid.h, k, M=M)


def cascade(p1, g1, grids, f0, medium, order, method="fft", rule="ball"):
    """Harmonics 2..max(grids) in order; grids = {n: Grid}.  Returns {n: array}."""
    fields = {1: (np.asarray(p1, dtype=np.complex128), g1)}
    out = {}
    for n in sorted(grids):
        p = harmonic(n, fields, grids[n], f0, medium, order, method=method, rule=rule)
        fields[n] = (p, grids[n])
        out[n] = p
    return out


# --------------------------------------------------------------------------
# measurement helpers (Sections 3.3 and 5)
# --------------------------------------------------------------------------

def focal_index(grid, focus):
    return tuple(_nint((focus[a] - grid.origin[a]) / grid.h) for a in range(3))


def rel_l2(a, b):
    a = np.asarray(a)
    b = np.asarray(b)
    return float(np.linalg.norm((a - b).ravel()) / np.linalg.norm(b.ravel()))
