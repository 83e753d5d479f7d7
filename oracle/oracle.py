"""Plain FP64 CPU oracle of the MSM -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this module.  It shares no code with the HIP library
``paper_2510_05961_amd``; the heavy loops live in ``msm_oracle.c`` (plain C,
FP64, OpenMP over independent outer loops), the orchestration and the exact
constants live here.

What it computes is the MSM approximation in its level-wise form
(Sec. "Fundamentals of the multilevel summation method"):

    U      = U^0 + U^{1+}
    U^0    = 1/2 sum_i sum_{j != i, r_ij < a} q_i q_j k_0(r_ij)
             - 1/2 sum_i q_i^2 sum_{l >= 1} k_l(0)                (eq. U_zero)
    U^{1+} = 1/2 sum_l (q~^l)^T K^l q~^l                 (eq. U_oneplus_grid_approx)
    q~^l_m = sum_i q_i phi^l_m(r_i)                           (eq. grid_charge)

with the grid charge of EVERY level obtained by direct anterpolation.  The
nested scheme of eq. (u_oneplus_nested_eval) reaches exactly this value
because B-splines nest (restriction reproduces the coarser anterpolation)
and prolongation is the transpose of restriction.  dE/dq_i = phi_i and
F_i = -grad_i U follow from eqs. (analytic_uoneplus_position_grad) and
(analytic_uoneplus_charge_grad) level by level.

Readings where the paper is silent:
  * L counts grid levels l = 1..L; kernels k_0..k_L.
  * periodic axis: N_top = max(1, floor(box/(h 2^(L-1)) + 1/2)),
    N_1 = N_top 2^(L-1), h_l = box/N_l;
    free axis: h_l = h 2^(l-1), grid indices -p/2+1 .. ceil(box/h_l)+p/2-1.
  * the top level keeps every top-grid pair; on periodic axes the partial
    kernel k_L is summed over all images with the Ewald method
    (tin-foil boundary, neutralising background):
        G_L(x) = psi(x) - sum_images s(|x + j|),
        s(r)   = (1/r - gamma(r/R)/R) [r < R],  R = 2^(L-1) a.
  * two periodic axes: 2-D Ewald with alpha = 3/min of their lengths;
    only non-neutral slabs depend on that convention.
  * one periodic axis: 1-D Ewald (Fourier part through the incomplete
    Bessel function); the divergent constant of a non-neutral line is fixed
    so that psi -> -(2/L) ln(rho/L) far from the axis.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess

import numpy as np

from . import constants as C

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
MAXL = 16


def build(force: bool = True) -> str:
    """Compile msm_oracle.c into liboracle.so (gcc, -O2, OpenMP)."""
    src = os.path.join(_HERE, "msm_oracle.c")
    if force or not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(src):
        tmp = _LIB_PATH + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c99",
                               "-D_DEFAULT_SOURCE", "-o", tmp, src, "-lm"])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


class _Geom(ctypes.Structure):
    _fields_ = [("p", ctypes.c_int), ("L", ctypes.c_int), ("M", ctypes.c_int),
                ("a", ctypes.c_double), ("box", ctypes.c_double * 3),
                ("periodic", ctypes.c_int * 3),
                ("n", (ctypes.c_int * 3) * MAXL), ("lo", (ctypes.c_int * 3) * MAXL),
                ("h", (ctypes.c_double * 3) * MAXL), ("omega", ctypes.c_double * 32),
                ("tri", ctypes.c_int), ("H", ctypes.c_double * 9), ("Hinv", ctypes.c_double * 9),
                ("nu", ctypes.c_int)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build(force=False)
        L = ctypes.CDLL(_LIB_PATH)
        d, i, P = ctypes.c_double, ctypes.c_int, ctypes.c_void_p
        G = ctypes.POINTER(_Geom)
        for name in ("orc_gamma", "orc_gamma_d1", "orc_gamma_d2"):
            getattr(L, name).argtypes = [i, d]
            getattr(L, name).restype = d
        L.orc_num_threads.restype = i
        L.orc_set_num_threads.argtypes = [i]
        L.orc_set_num_threads.restype = None
        L.orc_kernel.argtypes = [i, i, d, i, d]
        L.orc_kernel.restype = d
        L.orc_gamma_nu.argtypes = [i, i, d, i]
        L.orc_gamma_nu.restype = d
        L.orc_kernel_nu.argtypes = [i, i, i, d, i, d]
        L.orc_kernel_nu.restype = d
        L.orc_k0_nu.argtypes = [i, d, i, d, i]
        L.orc_k0_nu.restype = d
        L.orc_direct_nu.argtypes = [i, i, P, P, P, P]
        L.orc_direct_nu.restype = None
        for name in ("orc_k0_d1", "orc_k0_d2"):
            getattr(L, name).argtypes = [d, i, d]
            getattr(L, name).restype = d
        for name in ("orc_bspline", "orc_bspline_d1", "orc_bspline_d2"):
            getattr(L, name).argtypes = [i, d]
            getattr(L, name).restype = d
        L.orc_anterpolate.argtypes = [G, i, i, P, P, P]
        L.orc_anterpolate.restype = i
        L.orc_anterpolate_dipole.argtypes = [G, i, i, P, P, P, P]
        L.orc_anterpolate_dipole.restype = i
        L.orc_stencil.argtypes = [G, i, P, P]
        L.orc_stencil.restype = None
        L.orc_conv.argtypes = [G, i, P, P, P, P, i, P]
        L.orc_conv.restype = None
        L.orc_interpolate.argtypes = [G, i, i, P, P, P, P, P]
        L.orc_interpolate.restype = i
        L.orc_interpolate_vjp.argtypes = [G, i, i, P, P, P, P, P, P, P]
        L.orc_interpolate_vjp.restype = i
        L.orc_short_range.argtypes = [G, i, P, P, i, P, P, P]
        L.orc_short_range.restype = None
        L.orc_short_range_cells.argtypes = [G, i, P, P, i, P, P, P]
        L.orc_short_range_cells.restype = None
        L.orc_short_range_vjp.argtypes = [G, i, P, P, P, i, P, P, P]
        L.orc_short_range_vjp.restype = None
        L.orc_short_range_vjp_cells.argtypes = [G, i, P, P, P, P, P]
        L.orc_short_range_vjp_cells.restype = None
        L.orc_direct_coulomb.argtypes = [i, P, P, P, P]
        L.orc_direct_coulomb.restype = None
        for name in ("orc_ewald3d", "orc_ewald2d", "orc_ewald3d_cell"):
            getattr(L, name).argtypes = [P, d, P, i]
            getattr(L, name).restype = d
        L.orc_ewald3d_r6.argtypes = [P, d, P, i]
        L.orc_ewald3d_r6.restype = d
        L.orc_ewald_r6.argtypes = [P, ctypes.c_uint, d, P, i]
        L.orc_ewald_r6.restype = d
        L.orc_ewald3d_cell_r6.argtypes = [P, d, P, i]
        L.orc_ewald3d_cell_r6.restype = d
        L.orc_ewald1d.argtypes = [P, i, d, P, i]
        L.orc_ewald1d.restype = d
        L.orc_ewald_psi.argtypes = [P, ctypes.c_uint, d, P, i]
        L.orc_ewald_psi.restype = d
        L.orc_ewald_potentials_mask.argtypes = [P, ctypes.c_uint, d, i, P, P, P]
        L.orc_ewald_potentials_mask.restype = None
        L.orc_ewald_potentials.argtypes = [P, i, d, i, P, P, P]
        L.orc_ewald_potentials.restype = None
        L.orc_ewald_potentials_cell.argtypes = [P, d, i, P, P, P]
        L.orc_ewald_potentials_cell.restype = None
        L.orc_ewald3d_system.argtypes = [P, d, i, P, P, P, P]
        L.orc_ewald3d_system.restype = None
        _lib = L
    return _lib


def _ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p) if a is not None else None


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


# --------------------------------------------------------------------------
# scalar functions (thin wrappers, used by the pins)
# --------------------------------------------------------------------------
def num_threads():
    return int(lib().orc_num_threads())


def set_num_threads(n):
    """Threads of the oracle's OpenMP loops from now on (n >= 1)."""
    lib().orc_set_num_threads(int(n))


def gamma(p, rho):
    return lib().orc_gamma(p, float(rho))


def kernel(l, L, a, p, r, nu=1):
    """Partial kernel k_l(r) of r^-nu (nu = 1: Coulomb)."""
    if nu == 1:
        return lib().orc_kernel(l, L, float(a), p, float(r))
    return lib().orc_kernel_nu(int(nu), l, L, float(a), p, float(r))


def gamma_nu(nu, p, rho, deriv=0):
    return lib().orc_gamma_nu(int(nu), int(p), float(rho), int(deriv))


def direct_sum(pos, q, nu):
    """Exact all-pairs non-periodic sums of q_j r^-nu: potentials and forces."""
    pos, q = _f64(pos), _f64(q)
    phi = np.zeros(len(q))
    F = np.zeros((len(q), 3))
    lib().orc_direct_nu(int(nu), len(q), _ptr(pos), _ptr(q), _ptr(phi), _ptr(F))
    return phi, F


def bspline(p, t, deriv=0):
    f = (lib().orc_bspline, lib().orc_bspline_d1, lib().orc_bspline_d2)[deriv]
    return f(p, float(t))


def ewald_alpha_3d(box):
    """Balances the real- and reciprocal-space work; the 3-D result does not
    depend on alpha."""
    return math.sqrt(math.pi) / (box[0] * box[1] * box[2]) ** (1.0 / 3.0)


def ewald_alpha_slab(box):
    """Convention fixing the constant of non-neutral slabs."""
    return 3.0 / min(box[0], box[1])


def ewald_alpha_line(L):
    """1-D sum: any alpha gives the same result; alpha L = 1 keeps both the
    image sum (about 14 images) and the Fourier sum (2 terms) short."""
    return 1.0 / L


def _mask(periodic, slab):
    if periodic is None:
        return 3 if slab else 7
    return sum(1 << k for k in range(3) if periodic[k])


def _default_alpha(box, mask):
    per = [k for k in range(3) if (mask >> k) & 1]
    if len(per) == 3:
        return ewald_alpha_3d(box)
    if len(per) == 2:
        return 3.0 / min(box[per[0]], box[per[1]])
    return ewald_alpha_line(box[per[0]])


def ewald_psi(box, x, slab=False, alpha=None, reg=False, periodic=None):
    """Potential of a unit charge and its images along the periodic axes
    (periodic: 3 bools; default all, or x and y with slab=True)."""
    box = _f64(box)
    x = _f64(x)
    mask = _mask(periodic, slab)
    if alpha is None:
        alpha = _default_alpha(box, mask)
    return lib().orc_ewald_psi(_ptr(box), mask, float(alpha), _ptr(x), int(reg))


def ewald_potentials(box, pos, q, slab=False, alpha=None, periodic=None):
    """phi_i = sum_j q_j psi(r_i - r_j) (j = i uses the regular part)."""
    box, pos, q = _f64(box), _f64(pos), _f64(q)
    mask = _mask(periodic, slab)
    if alpha is None:
        alpha = _default_alpha(box, mask)
    phi = np.zeros(len(q))
    lib().orc_ewald_potentials_mask(_ptr(box), mask, float(alpha), len(q), _ptr(pos), _ptr(q),
                                    _ptr(phi))
    return phi


def _default_alpha_r6(box, mask):
    """Any alpha gives the same r^-6 lattice sum; these keep both parts short."""
    per = [box[k] for k in range(3) if (mask >> k) & 1]
    if len(per) == 3:
        return ewald_alpha_3d(box)
    return (3.0 if len(per) == 2 else 2.0) / min(per)


def ewald_psi_r6(box, x, alpha=None, reg=False, periodic=(True, True, True)):
    """sum_n |x + n|^-6 over the lattice of the periodic axes (Ewald method;
    reg=True at x = 0 leaves out n = 0)."""
    box = _f64(box)
    mask = _mask(periodic, False)
    if alpha is None:
        alpha = _default_alpha_r6(box, mask)
    return lib().orc_ewald_r6(_ptr(box), mask, float(alpha), _ptr(_f64(x)), int(reg))


def ewald_potentials_r6(box, pos, q, alpha=None, periodic=(True, True, True)):
    """phi_i = sum_j q_j sum_n' |r_i - r_j + n|^-6 (n = 0 left out for j = i)."""
    pos, q = _f64(pos), _f64(q)
    phi = np.zeros(len(q))
    for i in range(len(q)):
        for j in range(len(q)):
            phi[i] += q[j] * ewald_psi_r6(box, pos[i] - pos[j], alpha, reg=(i == j),
                                          periodic=periodic)
    return phi


def ewald3d_system(box, pos, q, alpha=None):
    """Potentials and forces of a 3-D periodic box by the structure-factor
    Ewald sum; the potentials are those of ewald_potentials(box, pos, q).
    alpha=None puts the real-space cutoff at half the shortest edge."""
    box, pos, q = _f64(box), _f64(pos), _f64(q)
    if alpha is None:
        alpha = 0.0
    phi = np.zeros(len(q))
    F = np.zeros((len(q), 3))
    lib().orc_ewald3d_system(_ptr(box), float(alpha), len(q), _ptr(pos), _ptr(q), _ptr(phi),
                             _ptr(F))
    return phi, F


def cell_matrix(cell):
    """H with the lattice vectors as columns, from cell = rows a, b, c."""
    return np.ascontiguousarray(np.asarray(cell, dtype=np.float64).T)


def ewald_alpha_cell(cell):
    return math.sqrt(math.pi) / abs(np.linalg.det(np.asarray(cell, dtype=np.float64))) ** (1 / 3)


def ewald_psi_cell(cell, x, alpha=None, reg=False):
    """3-D Ewald potential of a unit charge and its images on the lattice
    spanned by the rows of cell (tin-foil, neutralising background)."""
    H = cell_matrix(cell)
    if alpha is None:
        alpha = ewald_alpha_cell(cell)
    return lib().orc_ewald3d_cell(_ptr(H), float(alpha), _ptr(_f64(x)), int(reg))


def ewald_psi_cell_r6(cell, x, alpha=None, reg=False):
    """sum_n |x + H n|^-6 over the lattice spanned by the rows of cell."""
    H = cell_matrix(cell)
    if alpha is None:
        alpha = ewald_alpha_cell(cell)
    return lib().orc_ewald3d_cell_r6(_ptr(H), float(alpha), _ptr(_f64(x)), int(reg))


def ewald_potentials_cell_r6(cell, pos, q, alpha=None):
    """phi_i = sum_j q_j sum_n' |r_i - r_j + H n|^-6 (n = 0 left out for j = i)."""
    pos, q = _f64(pos), _f64(q)
    phi = np.zeros(len(q))
    for i in range(len(q)):
        for j in range(len(q)):
            phi[i] += q[j] * ewald_psi_cell_r6(cell, pos[i] - pos[j], alpha, reg=(i == j))
    return phi


def ewald_potentials_cell(cell, pos, q, alpha=None):
    H = cell_matrix(cell)
    pos, q = _f64(pos), _f64(q)
    if alpha is None:
        alpha = ewald_alpha_cell(cell)
    phi = np.zeros(len(q))
    lib().orc_ewald_potentials_cell(_ptr(H), float(alpha), len(q), _ptr(pos), _ptr(q), _ptr(phi))
    return phi


def direct_coulomb(pos, q):
    """Exact all-pairs non-periodic Coulomb potentials and forces."""
    pos, q = _f64(pos), _f64(q)
    phi = np.zeros(len(q))
    F = np.zeros((len(q), 3))
    lib().orc_direct_coulomb(len(q), _ptr(pos), _ptr(q), _ptr(phi), _ptr(F))
    return phi, F


# --------------------------------------------------------------------------
# the MSM oracle
# --------------------------------------------------------------------------
class OracleMSM:
    """Level-wise FP64 MSM for one orthorhombic box or triclinic cell.

    box: 3 lengths; periodic: 3 bools (any combination); p: even B-spline
    order; h: requested level-1 spacing; a: level-zero cutoff; L: number of grid levels; M: half-width of omega'
    (default p).

    cell: rows a, b, c of a triclinic cell (all axes periodic; box is then
    ignored).  Positions are mapped to the unit cube, s = [a b c]^{-1} r, and
    every grid lives there (Sec. MSM core algorithm, long-range part): N_l
    points along each lattice vector by the periodic rule above with the
    vector's length, basis functions of s, gradients taken back to r through
    H^{-T}, stencil samples k_l(|H (n / N_l)|), the top level summed over the
    lattice with the triclinic Ewald sum.  The cutoff must not exceed half
    the cell's smallest width V / |face| (minimum image).

    nu: the kernel k(r) = r^-nu split the same way (gamma_nu: the Taylor
    polynomial of s^(-nu/2)); 1 is Coulomb, 6 the dispersion kernel, in free
    space (the top level is the plain dense sum), in an orthorhombic box with
    any periodic axes or in a triclinic cell (the top level sums k_L over the
    lattice of the periodic axes with the Ewald method for r^-6).
    """

    def __init__(self, box, periodic, p, h, a, L, M=None, cell=None, ntop=None, nu=1):
        self.cell = None if cell is None else np.asarray(cell, dtype=np.float64).reshape(3, 3)
        if self.cell is not None:
            self.H = cell_matrix(self.cell)
            self.Hinv = np.linalg.inv(self.H)
            lengths = [float(np.linalg.norm(self.cell[k])) for k in range(3)]
            widths = [1.0 / float(np.linalg.norm(self.Hinv[k])) for k in range(3)]
            periodic = (True, True, True)
            box = (1.0, 1.0, 1.0)
        self.box = [float(b) for b in box]
        self.periodic = [bool(x) for x in periodic]
        self.p, self.h, self.a, self.L = int(p), float(h), float(a), int(L)
        self.M = self.p if M is None else int(M)
        self.nu = int(nu)  # kernel r^-nu: 1 (Coulomb) or 6 (dispersion), any geometry
        assert self.nu in (1, 6)
        assert self.p % 2 == 0 and self.p >= 2 and 1 <= self.L <= MAXL
        for k in range(3):
            if self.periodic[k]:
                w = widths[k] if self.cell is not None else self.box[k]
                assert self.a <= w / 2 + 1e-12, "cutoff exceeds half the box"
        self.omega_exact = C.omega_prime(self.p, self.M)
        self.omega = [float(w) for w in self.omega_exact]
        self.levels = []  # per level: (n[3], lo[3], h[3]) (h: fractional in a cell)
        for l in range(1, self.L + 1):
            n, lo, hl = [], [], []
            for k in range(3):
                if self.periodic[k]:
                    edge = lengths[k] if self.cell is not None else self.box[k]
                    nt = max(1, int(math.floor(edge / (self.h * 2 ** (self.L - 1)) + 0.5)))
                    if ntop is not None:  # grid counts held fixed (cell derivatives)
                        nt = int(ntop[k])
                    nk = nt * 2 ** (self.L - 1) // 2 ** (l - 1)
                    n.append(nk)
                    lo.append(0)
                    hl.append(self.box[k] / nk)
                else:
                    hk = self.h * 2 ** (l - 1)
                    lo_k = -self.p // 2 + 1
                    hi_k = int(math.ceil(self.box[k] / hk - 1e-9)) + self.p // 2 - 1
                    n.append(hi_k - lo_k + 1)
                    lo.append(lo_k)
                    hl.append(hk)
            self.levels.append((n, lo, hl))
        g = _Geom()
        g.p, g.L, g.M, g.a = self.p, self.L, self.M, self.a
        g.nu = self.nu
        for k in range(3):
            g.box[k] = self.box[k]
            g.periodic[k] = int(self.periodic[k])
        for l, (n, lo, hl) in enumerate(self.levels):
            for k in range(3):
                g.n[l][k], g.lo[l][k], g.h[l][k] = n[k], lo[k], hl[k]
        for j, w in enumerate(self.omega):
            g.omega[j] = w
        g.tri = int(self.cell is not None)
        if self.cell is not None:
            for k in range(9):
                g.H[k] = float(self.H.flat[k])
                g.Hinv[k] = float(self.Hinv.flat[k])
        self._g = g
        self._gp = ctypes.pointer(g)
        self._stencils = {}

    # ---------------------------------------------------------------- grids
    def grid_shape(self, level):
        n = self.levels[level - 1][0]
        return (n[2], n[1], n[0])

    def spacing(self, level):
        return tuple(self.levels[level - 1][2])

    def check_domain(self, pos):
        for k in range(3):
            if not self.periodic[k]:
                x = pos[:, k]
                if np.any(x < 0) or np.any(x > self.box[k]):
                    raise ValueError("position outside the non-periodic domain")

    def grid_charge(self, level, pos, q):
        """q~^l by direct anterpolation (eq. grid_charge, Alg. anterpolation)."""
        pos, q = _f64(pos), _f64(q)
        out = np.zeros(self.grid_shape(level))
        rc = lib().orc_anterpolate(self._gp, level, len(q), _ptr(pos), _ptr(q), _ptr(out))
        if rc:
            raise ValueError("particle outside the grid")
        return out

    def dipole_charge(self, level, pos, q, v):
        pos, q, v = _f64(pos), _f64(q), _f64(v)
        out = np.zeros(self.grid_shape(level))
        rc = lib().orc_anterpolate_dipole(self._gp, level, len(q), _ptr(pos), _ptr(q), _ptr(v),
                                          _ptr(out))
        if rc:
            raise ValueError("particle outside the grid")
        return out

    # ------------------------------------------------------------- stencils
    def stencil(self, level):
        """(W, K): K^l over |d_k| <= W_k, K[dz+Wz, dy+Wy, dx+Wx]."""
        if level in self._stencils:
            return self._stencils[level]
        n, lo, hl = self.levels[level - 1]
        if level < self.L:
            W = []
            for k in range(3):
                # |n_k| reach of the support |x| < 2^l a along grid axis k
                reach = (2 ** level * self.a * n[k] * float(np.linalg.norm(self.Hinv[k]))
                         if self.cell is not None else 2 ** level * self.a / hl[k])
                w = int(math.floor(reach)) + self.M
                if not self.periodic[k]:
                    w = min(w, n[k] - 1)
                W.append(w)
            Wc = (ctypes.c_int * 3)(*W)
            K = np.zeros((2 * W[2] + 1, 2 * W[1] + 1, 2 * W[0] + 1))
            lib().orc_stencil(self._gp, level, Wc, _ptr(K))
        else:
            W, K = self._top_stencil()
        self._stencils[level] = (W, K)
        return W, K

    def _G_top(self, x):
        """Top-level kernel summed over the periodic images (see module doc)."""
        L, a, p = self.L, self.a, self.p
        npd = sum(self.periodic)
        if npd == 0:
            r = math.sqrt(x[0] ** 2 + x[1] ** 2 + x[2] ** 2)
            return kernel(L, L, a, p, r, self.nu)
        R = 2 ** (L - 1) * a
        if self.cell is not None:
            # x is Cartesian; images x + H j over the lattice
            nu = self.nu
            val = (ewald_psi_cell(self.cell, x, reg=True) if nu == 1
                   else ewald_psi_cell_r6(self.cell, x, reg=True))
            s = self.Hinv @ np.asarray(x, dtype=np.float64)
            nimg = [int(math.ceil(R * float(np.linalg.norm(self.Hinv[k])) + abs(s[k]))) + 1
                    for k in range(3)]
            for jz in range(-nimg[2], nimg[2] + 1):
                for jy in range(-nimg[1], nimg[1] + 1):
                    for jx in range(-nimg[0], nimg[0] + 1):
                        d = np.asarray(x) + self.H @ np.array([jx, jy, jz], dtype=np.float64)
                        r = float(np.sqrt(d @ d))
                        if r == 0.0:
                            val += gamma_nu(nu, p, 0.0) / R ** nu
                        elif r < R:
                            val -= r ** -nu - gamma_nu(nu, p, r / R) / R ** nu
            return val
        nu = self.nu
        if nu == 1:
            val = ewald_psi(self.box, x, periodic=self.periodic, reg=True)
        else:
            val = ewald_psi_r6(self.box, x, reg=True, periodic=self.periodic)
        # k_L = gamma_nu(r/R)/R^nu = r^-nu - (r^-nu - gamma_nu(r/R)/R^nu) for r < R
        nimg = [int(math.ceil((R + abs(x[k])) / self.box[k])) + 1 if self.periodic[k] else 0
                for k in range(3)]
        for jz in range(-nimg[2], nimg[2] + 1):
            for jy in range(-nimg[1], nimg[1] + 1):
                for jx in range(-nimg[0], nimg[0] + 1):
                    d = (x[0] + jx * self.box[0], x[1] + jy * self.box[1], x[2] + jz * self.box[2])
                    r = math.sqrt(d[0] ** 2 + d[1] ** 2 + d[2] ** 2)
                    if r == 0.0:
                        val += gamma_nu(nu, p, 0.0) / R ** nu
                    elif r < R:
                        val -= r ** -nu - gamma_nu(nu, p, r / R) / R ** nu
        return val

    def _top_stencil(self):
        """K^L over all top-grid offsets: sum_k omega'omega'omega' G(h_L o (d-k)).

        Periodic axis with N points: offsets -N//2..N//2, where for even N the
        two ends are the same residue and each carries half of its value (the
        wrapped convolution adds them back together)."""
        n, lo, hl = self.levels[self.L - 1]
        M = self.M
        W = []
        for k in range(3):
            W.append(n[k] // 2 if self.periodic[k] else n[k] - 1)
        # table of G over the integer offsets that can occur
        rng = [range(-W[k] - M, W[k] + M + 1) for k in range(3)]
        cache = {}

        def G(ix, iy, iz):
            key = [ix, iy, iz]
            for k in range(3):
                if self.periodic[k]:
                    key[k] %= n[k]
            key = tuple(key)
            if key not in cache:
                u = (key[0] * hl[0], key[1] * hl[1], key[2] * hl[2])
                if self.cell is not None:
                    u = tuple(self.H @ np.asarray(u))
                cache[key] = self._G_top(u)
            return cache[key]

        # table T over every offset d - k that occurs, then the plain sum
        # K(d) = sum_k omega'(kx) omega'(ky) omega'(kz) T(d - k), vectorised over d
        T = np.empty((len(rng[2]), len(rng[1]), len(rng[0])))
        for a_, iz in enumerate(rng[2]):
            for b_, iy in enumerate(rng[1]):
                for c_, ix in enumerate(rng[0]):
                    T[a_, b_, c_] = G(ix, iy, iz)
        om = self.omega
        K = np.zeros((2 * W[2] + 1, 2 * W[1] + 1, 2 * W[0] + 1))
        for kz in range(-M, M + 1):
            for ky in range(-M, M + 1):
                for kx in range(-M, M + 1):
                    # T index of offset (d - k) is d - k + W + M; d runs over -W..W
                    K += om[abs(kx)] * om[abs(ky)] * om[abs(kz)] * T[
                        M - kz:M - kz + 2 * W[2] + 1, M - ky:M - ky + 2 * W[1] + 1,
                        M - kx:M - kx + 2 * W[0] + 1]
        for k in range(3):
            if self.periodic[k] and n[k] % 2 == 0 and n[k] > 1:
                sl = [slice(None)] * 3
                for end_ in (0, 2 * W[k]):
                    sl[2 - k] = end_
                    K[tuple(sl)] *= 0.5

        return W, K

    def level_potential(self, level, qgrid, points=None):
        """e^l = K^l q~^l at all grid points (or the listed flat indices)."""
        W, K = self.stencil(level)
        qgrid = _f64(qgrid)
        out = np.zeros(self.grid_shape(level))
        Wc = (ctypes.c_int * 3)(*W)
        if points is None:
            lib().orc_conv(self._gp, level, Wc, _ptr(K), _ptr(qgrid), _ptr(out), -1, None)
        else:
            pts = np.ascontiguousarray(points, dtype=np.int32)
            lib().orc_conv(self._gp, level, Wc, _ptr(K), _ptr(qgrid), _ptr(out), len(pts),
                           _ptr(pts))
        return out

    def self_constant(self):
        """sum_{l=1..L} k_l(0) (eq. U_zero, second term)."""
        return sum(kernel(l, self.L, self.a, self.p, 0.0, self.nu) for l in range(1, self.L + 1))

    def support_points(self, level, pos):
        """Flat indices of the grid points whose basis is non-zero at pos."""
        n, lo, hl = self.levels[level - 1]
        p = self.p
        pts = set()
        for r in np.atleast_2d(pos):
            if self.cell is not None:
                r = self.Hinv @ np.asarray(r, dtype=np.float64)
            idx = []
            for k in range(3):
                x = r[k]
                if self.periodic[k]:
                    x = x - self.box[k] * math.floor(x / self.box[k])
                base = math.floor(x / hl[k])
                ax = []
                for j in range(p):
                    m = base - p // 2 + 1 + j
                    ai = m % n[k] if self.periodic[k] else m - lo[k]
                    if 0 <= ai < n[k]:
                        ax.append(ai)
                idx.append(ax)
            for iz in idx[2]:
                for iy in idx[1]:
                    for ix in idx[0]:
                        pts.add((iz * n[1] + iy) * n[0] + ix)
        return np.array(sorted(pts), dtype=np.int32)

    # --------------------------------------------------------------- energy
    def short_range(self, pos, q, sel=None, cells=None):
        pos, q = _f64(pos), _f64(q)
        n = len(q)
        if sel is None:
            phi = np.zeros(n)
            F = np.zeros((n, 3))
            if cells is None:
                cells = n > 4000
            if cells:
                lib().orc_short_range_cells(self._gp, n, _ptr(pos), _ptr(q), -1, None, _ptr(phi),
                                            _ptr(F))
            else:
                lib().orc_short_range(self._gp, n, _ptr(pos), _ptr(q), -1, None, _ptr(phi),
                                      _ptr(F))
        else:
            sel = np.ascontiguousarray(sel, dtype=np.int32)
            phi = np.zeros(len(sel))
            F = np.zeros((len(sel), 3))
            if cells is None:
                cells = n > 4000
            fn = lib().orc_short_range_cells if cells else lib().orc_short_range
            fn(self._gp, n, _ptr(pos), _ptr(q), len(sel), _ptr(sel), _ptr(phi), _ptr(F))
        return phi, F

    def compute(self, pos, q):
        """Energy, per-particle potential phi_i = dE/dq_i and forces."""
        pos, q = _f64(pos), _f64(q)
        self.check_domain(pos)
        n = len(q)
        phi0, F0 = self.short_range(pos, q)
        phi1 = np.zeros(n)
        F1 = np.zeros((n, 3))
        grids = []
        for l in range(1, self.L + 1):
            qg = self.grid_charge(l, pos, q)
            eg = self.level_potential(l, qg)
            lib().orc_interpolate(self._gp, l, n, _ptr(pos), _ptr(q), _ptr(eg), _ptr(phi1),
                                  _ptr(F1))
            grids.append((qg, eg))
        phi = phi0 + phi1 - q * self.self_constant()
        F = F0 + F1
        E = 0.5 * float(np.dot(q, phi))
        return {"E": E, "phi": phi, "F": F, "phi0": phi0, "F0": F0, "phi1": phi1, "F1": F1,
                "grids": grids}

    def sampled(self, pos, q, sel):
        """phi_i and F_i for the listed particles only (full-size parity)."""
        pos, q = _f64(pos), _f64(q)
        self.check_domain(pos)
        sel = np.asarray(sel, dtype=np.int64)
        phi0, F0 = self.short_range(pos, q, sel=sel)
        ps, qs = _f64(pos[sel]), _f64(q[sel])
        phi1 = np.zeros(len(sel))
        F1 = np.zeros((len(sel), 3))
        for l in range(1, self.L + 1):
            qg = self.grid_charge(l, pos, q)
            pts = self.support_points(l, ps)
            eg = self.level_potential(l, qg, points=pts)
            lib().orc_interpolate(self._gp, l, len(sel), _ptr(ps), _ptr(qs), _ptr(eg), _ptr(phi1),
                                  _ptr(F1))
        phi = phi0 + phi1 - qs * self.self_constant()
        return phi, F0 + F1

    def short_range_vjp(self, pos, q, v, sel=None, cells=None):
        """Cotangents of sum_i v_i . F0_i (short-range forces): (dq, dr), for
        all particles or the listed ones (brute force over all partners)."""
        pos, q, v = _f64(pos), _f64(q), _f64(v)
        n = len(q)
        if sel is None:
            sq = np.zeros(n)
            sr = np.zeros((n, 3))
            if cells is None:
                cells = n > 4000
            if cells:
                lib().orc_short_range_vjp_cells(self._gp, n, _ptr(pos), _ptr(q), _ptr(v),
                                                _ptr(sq), _ptr(sr))
            else:
                lib().orc_short_range_vjp(self._gp, n, _ptr(pos), _ptr(q), _ptr(v), -1, None,
                                          _ptr(sq), _ptr(sr))
        else:
            sel = np.ascontiguousarray(sel, dtype=np.int32)
            sq = np.zeros(len(sel))
            sr = np.zeros((len(sel), 3))
            lib().orc_short_range_vjp(self._gp, n, _ptr(pos), _ptr(q), _ptr(v), len(sel),
                                      _ptr(sel), _ptr(sq), _ptr(sr))
        return sq, sr

    def backward(self, pos, q, gE, v, cells=None, w=None):
        """Cotangents (dL/dq, dL/dr) of L = gE * E + sum_i v_i . F_i
        (+ sum_i w_i phi_i when w, the cotangent of phi = dE/dq, is given:
        see _phi_cotangent)."""
        pos, q, v = _f64(pos), _f64(q), _f64(v)
        if w is not None:
            dq, dr = self._phi_cotangent(pos, q, _f64(w), lambda c: self.compute(pos, c))
            gq, gr = self.backward(pos, q, gE, v, cells=cells)
            return gq + dq, gr + dr
        res = self.compute(pos, q)
        n = len(q)
        gq = gE * res["phi"].copy()
        gr = -gE * res["F"].copy()
        sq, sr = self.short_range_vjp(pos, q, v, cells=cells)
        for l in range(1, self.L + 1):
            psi = res["grids"][l - 1][1]
            D = self.dipole_charge(l, pos, q, v)
            psiD = self.level_potential(l, D)
            lib().orc_interpolate_vjp(self._gp, l, n, _ptr(pos), _ptr(q), _ptr(v), _ptr(psi),
                                      _ptr(psiD), _ptr(sq), _ptr(sr))
        return gq + sq, gr + sr

    def cell_gradient(self, pos, q, eps=1e-5):
        """dE/dH at fixed Cartesian positions (H: lattice vectors as columns),
        by central differences of the energy with the grid counts held fixed:
        the plain definition of the derivative, in FP64."""
        assert self.cell is not None, "a triclinic oracle (cell=...) is needed"
        ntop = [self.levels[self.L - 1][0][k] for k in range(3)]
        scale = float(np.abs(self.H).max())
        out = np.zeros((3, 3))
        for r in range(3):
            for c in range(3):
                E = []
                for sgn in (1.0, -1.0):
                    Hp = self.H.copy()
                    Hp[r, c] += sgn * eps * scale
                    o = OracleMSM(None, None, self.p, self.h, self.a, self.L, self.M,
                                  cell=Hp.T, ntop=ntop, nu=self.nu)
                    E.append(o.compute(pos, q)["E"])
                out[r, c] = (E[0] - E[1]) / (2 * eps * scale)
        return out

    @staticmethod
    def _phi_cotangent(pos, q, w, run):
        """Cotangents of sum_i w_i phi_i.  The MSM energy is a quadratic form,
        E(q) = q^T G q / 2 with G symmetric (the interpolated level kernels,
        the short-range pairs and the constant self term), so phi = G q and
        sum_i w_i phi_i = w^T G q is bilinear: its q-gradient is G w, the
        potentials computed with charges w, and its r-gradient follows from
        polarising E, w^T G q = E(q + w) - E(q) - E(w), as
        F(q) + F(w) - F(q + w).  run(c) evaluates phi and F for charges c."""
        a, b, c = run(q), run(w), run(q + w)
        return b["phi"], a["F"] + b["F"] - c["F"]

    def sampled_backward(self, pos, q, gE, v, sel, w=None):
        """backward() for the listed particles only: the grid charges and
        dipole grids of every level come from all particles, the level
        potentials are evaluated only at the grid points the listed
        particles touch (full-size parity)."""
        pos, q, v = _f64(pos), _f64(q), _f64(v)
        self.check_domain(pos)
        sel = np.asarray(sel, dtype=np.int64)
        if w is not None:
            def run(c):
                phi, F = self.sampled(pos, c, sel)
                return {"phi": phi, "F": F}
            dq, dr = self._phi_cotangent(pos, q, _f64(w), run)
            gq, gr = self.sampled_backward(pos, q, gE, v, sel)
            return gq + dq, gr + dr
        phi, F = self.sampled(pos, q, sel)
        sq, sr = self.short_range_vjp(pos, q, v, sel=sel)
        ps, qs, vs = _f64(pos[sel]), _f64(q[sel]), _f64(v[sel])
        for l in range(1, self.L + 1):
            pts = self.support_points(l, ps)
            psi = self.level_potential(l, self.grid_charge(l, pos, q), points=pts)
            psiD = self.level_potential(l, self.dipole_charge(l, pos, q, v), points=pts)
            lib().orc_interpolate_vjp(self._gp, l, len(sel), _ptr(ps), _ptr(qs), _ptr(vs),
                                      _ptr(psi), _ptr(psiD), _ptr(sq), _ptr(sr))
        return gE * phi + sq, -gE * F + sr


# --------------------------------------------------------------------------
# molecular dynamics of charged Lennard-Jones particles (Sec. MD simulation
# of charged Lennard-Jonesium): the short-range partner of the MSM energy
# and the velocity-Verlet integrator, written out plainly
# --------------------------------------------------------------------------
def lj_switch(r, rc, ron):
    """S(r): 1 up to ron, 1 - 10 x^3 + 15 x^4 - 6 x^5 with x = (r - ron)/(rc -
    ron) between, 0 from rc on (S, S', S'' continuous), and dS/dr."""
    r = np.asarray(r, dtype=np.float64)
    x = np.clip((r - ron) / (rc - ron), 0.0, 1.0)
    S = 1.0 - 10.0 * x ** 3 + 15.0 * x ** 4 - 6.0 * x ** 5
    dS = (-30.0 * x ** 2 + 60.0 * x ** 3 - 30.0 * x ** 4) / (rc - ron)
    return S, dS


def lj_energy_forces(box, periodic, pos, eps, sigma, rc, ron):
    """E = sum over pairs i < j of 4 eps [(sigma/r)^12 - (sigma/r)^6] S(r),
    minimum image on periodic axes (rc at most half a periodic edge), and
    F_i = -dE/dr_i; all pairs, FP64."""
    pos = _f64(pos)
    box = np.asarray(box, dtype=np.float64)
    per = np.asarray(periodic, dtype=bool)
    d = pos[:, None, :] - pos[None, :, :]
    d[..., per] -= box[per] * np.round(d[..., per] / box[per])
    r = np.sqrt(np.sum(d * d, axis=-1))
    np.fill_diagonal(r, np.inf)
    inside = r < rc
    rr = np.where(inside, r, 1.0)
    sr6 = (sigma / rr) ** 6
    u = 4.0 * eps * (sr6 * sr6 - sr6)
    du = 4.0 * eps * (-12.0 * sr6 * sr6 + 6.0 * sr6) / rr
    S, dS = lj_switch(rr, rc, ron)
    E = 0.5 * float(np.sum(np.where(inside, u * S, 0.0)))
    c = np.where(inside, -(du * S + u * dS) / rr, 0.0)
    F = np.sum(c[..., None] * d, axis=1)
    return E, F


def velocity_verlet(x, v, m, forces, dt, nsteps):
    """nsteps of v += dt/2 F/m, x += dt v, F = forces(x), v += dt/2 F/m from
    (x, v) with forces F = forces(x)[0]; forces returns (F, energies).
    Returns x, v and the list of (kinetic energy, energies) after each step."""
    x, v = _f64(x).copy(), _f64(v).copy()
    m = _f64(m)[:, None]
    F, _ = forces(x)
    log = []
    for _ in range(nsteps):
        v += 0.5 * dt * F / m
        x += dt * v
        F, e = forces(x)
        v += 0.5 * dt * F / m
        log.append((0.5 * float(np.sum(m * v * v)), e))
    return x, v, log
