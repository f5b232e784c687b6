"""ctypes binding of the FP64 CPU oracle (``m2m_oracle.c``).

TEST INFRASTRUCTURE: imported only by the test-suite, the package smoke check
and the CPU-baseline leg of the benchmark. The product path never loads it.
"""

from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "m2m_oracle.c")
LIB = os.path.join(HERE, "liboracle.so")

KIN = {"none": 0, "v2": 1, "gh": 2, "losvd": 3}
SCF_KEYS = ("scf_lmax", "scf_nr", "scf_rmin", "scf_rmax", "scf_every")
DENS = {"bins": 0, "alm": 1}
ENTROPY = {"mpr": 0, "gwr": 1}


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (-O2, IEEE double, OpenMP)."""
    if force or not os.path.exists(LIB):
        cmd = ["gcc", "-O2", "-std=gnu11", "-fopenmp", "-fPIC", "-shared", "-o", LIB, SRC, "-lm"]
        subprocess.run(cmd, check=True)
    return LIB


class Potential(C.Structure):
    _fields_ = [(k, C.c_double) for k in ("G", "M_star", "a", "upsilon", "M200", "c", "r_s",
                                          "v0", "r0", "q", "scf_rmin", "scf_rmax")] + [
        ("scf_lmax", C.c_int32), ("scf_nr", C.c_int32), ("scf_every", C.c_int32)]


class Layout(C.Structure):
    _fields_ = [("n_r", C.c_int32), ("r_min", C.c_double), ("r_max", C.c_double),
                ("n_R", C.c_int32), ("R_min", C.c_double), ("R_max", C.c_double),
                ("kin", C.c_int32), ("gh_nmax", C.c_int32), ("n_v", C.c_int32),
                ("v_min", C.c_double), ("v_max", C.c_double), ("dens", C.c_int32),
                ("l_max", C.c_int32)]


class Params(C.Structure):
    _fields_ = [("dt", C.c_double), ("eps", C.c_double), ("mu", C.c_double),
                ("alpha", C.c_double), ("mass", C.c_double), ("entropy", C.c_int32),
                ("n_E", C.c_int32), ("n_x", C.c_int32), ("prior_every", C.c_int32),
                ("E_lo", C.c_double), ("E_hi", C.c_double), ("smooth", C.c_int32),
                ("cells", C.c_int32)]


_dp = C.POINTER(C.c_double)


class Model(C.Structure):
    _fields_ = [("n", C.c_int64)] + [(k, _dp) for k in
                                     ("x", "y", "z", "vx", "vy", "vz", "u", "uhat")] + [
        ("pot", Potential), ("lay", Layout), ("par", Params), ("J", C.c_int32),
        ("Y", _dp), ("sigma", _dp), ("Vp", _dp), ("sp", _dp),
        ("ytilde", _dp), ("yraw", _dp), ("delta", _dp), ("chi2", C.c_double),
        ("kstep", C.c_int64), ("flag", C.POINTER(C.c_uint8)), ("band", C.c_double),
        ("nthreads", C.c_int32), ("ucell", _dp), ("scf", _dp), ("tstep", C.c_int64)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            build()
        L = C.CDLL(LIB)
        L.orc_phi.restype = C.c_double
        L.orc_phi.argtypes = [C.POINTER(Potential), C.c_double]
        L.orc_phi3.restype = C.c_double
        L.orc_phi3.argtypes = [C.POINTER(Potential), C.c_double, C.c_double, C.c_double]
        L.orc_mass.restype = C.c_double
        L.orc_mass.argtypes = [C.POINTER(Potential), C.c_double]
        L.orc_lc.restype = C.c_double
        L.orc_lc.argtypes = [C.POINTER(Potential), C.c_double]
        L.orc_accel.argtypes = [C.POINTER(Potential), C.c_double, C.c_double, C.c_double, _dp]
        L.orc_J.restype = C.c_int32
        L.orc_J.argtypes = [C.POINTER(Layout)]
        L.orc_hermite.restype = C.c_double
        L.orc_hermite.argtypes = [C.c_int, C.c_double]
        L.orc_gh_u.restype = C.c_double
        L.orc_gh_u.argtypes = [C.c_int, C.c_double]
        L.orc_plm.restype = C.c_double
        L.orc_plm.argtypes = [C.c_int, C.c_int, C.c_double]
        L.orc_ylm.restype = C.c_double
        L.orc_ylm.argtypes = [C.c_int, C.c_int, C.c_double, C.c_double]
        L.orc_kernels.restype = C.c_int
        L.orc_kernels.argtypes = [C.POINTER(Layout), _dp, _dp] + [C.c_double] * 4 + [
            C.POINTER(C.c_int32), _dp]
        L.orc_deposit.argtypes = [C.c_int64] + [_dp] * 7 + [C.c_int64, C.c_double,
                                                             C.POINTER(Layout), _dp, _dp, _dp,
                                                             _dp, _dp, C.c_double, C.c_int32]
        L.orc_cell.restype = C.c_int32
        L.orc_cell.argtypes = [C.POINTER(Potential), C.POINTER(Params)] + [C.c_double] * 6 + [
            _dp, _dp]
        L.orc_cells.argtypes = [C.POINTER(Potential), C.POINTER(Params), C.c_int64] + [_dp] * 6 + [
            C.POINTER(C.c_int32), _dp, _dp]
        L.orc_init.argtypes = [C.POINTER(Model)]
        L.orc_refresh_priors.argtypes = [C.POINTER(Model)]
        L.orc_smooth_grid.restype = C.c_int
        L.orc_smooth_grid.argtypes = [C.POINTER(Params), _dp, _dp]
        L.orc_smooth_grid_at.restype = C.c_int
        L.orc_smooth_grid_at.argtypes = [C.POINTER(Params), _dp, C.c_double]
        L.orc_steps.argtypes = [C.POINTER(Model), C.c_int32, C.c_int32, _dp]
        L.orc_cell_mass.argtypes = [C.POINTER(Potential), C.POINTER(Params), C.c_int64] + [
            _dp] * 7 + [C.c_double, _dp]
        L.orc_push.argtypes = [C.POINTER(Potential), C.c_double, C.c_int64] + [_dp] * 6 + [
            C.c_int32]
        L.orc_scf_table.argtypes = [C.POINTER(Potential), C.c_int64] + [_dp] * 4 + [
            C.c_double, _dp, C.c_int32]
        L.orc_scf_phi.restype = C.c_double
        L.orc_scf_phi.argtypes = [C.POINTER(Potential), _dp] + [C.c_double] * 3
        L.orc_scf_accel.argtypes = [C.POINTER(Potential), _dp] + [C.c_double] * 3 + [_dp]
        _lib = L
    return _lib


def _p(a):
    return a.ctypes.data_as(_dp)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def potential(d) -> Potential:
    d = d.as_dict() if hasattr(d, "as_dict") else d
    return Potential(**{k: float(d[k]) for k in ("G", "M_star", "a", "upsilon", "M200", "c", "r_s")},
                     v0=float(d.get("v0", 0.0)), r0=float(d.get("r0", 1.0)), q=float(d.get("q", 1.0)),
                     scf_rmin=float(d.get("scf_rmin", 0.0)), scf_rmax=float(d.get("scf_rmax", 0.0)),
                     scf_lmax=int(d.get("scf_lmax", 0)), scf_nr=int(d.get("scf_nr", 0)),
                     scf_every=int(d.get("scf_every", 1)))


def scf_size(pot) -> int:
    """Entries of the self-consistent potential's node table (0 without it)."""
    P = potential(pot)
    return P.scf_nr * (P.scf_lmax + 1) ** 2 * 2


def scf_table(pot, parts: dict, u=None, mass=1.0, nthreads=1):
    """Node table of the particles' multipole potential: array (scf_nr,
    (scf_lmax+1)^2, 2) of Phi_lm(rho_k) and r dPhi_lm/dr there."""
    P = potential(pot)
    x, y, z = (_f64(parts[k]) for k in ("x", "y", "z"))
    u = _f64(np.ones(x.size) if u is None else u)
    tab = np.zeros(scf_size(pot))
    lib().orc_scf_table(C.byref(P), x.size, _p(x), _p(y), _p(z), _p(u), float(mass), _p(tab),
                        int(nthreads))
    return tab.reshape(P.scf_nr, (P.scf_lmax + 1) ** 2, 2)


def scf_phi(pot, tab, x, y, z) -> float:
    t = _f64(tab).reshape(-1)
    return lib().orc_scf_phi(C.byref(potential(pot)), _p(t), float(x), float(y), float(z))


def scf_accel(pot, tab, x, y, z):
    t = _f64(tab).reshape(-1)
    g = np.zeros(3)
    lib().orc_scf_accel(C.byref(potential(pot)), _p(t), float(x), float(y), float(z), _p(g))
    return g


def layout(d: dict) -> Layout:
    dens = d.get("dens", "bins")
    return Layout(n_r=d["n_r"], r_min=d["r_min"], r_max=d["r_max"], n_R=d["n_R"],
                  R_min=d["R_min"], R_max=d["R_max"], kin=KIN[d["kin"]], gh_nmax=d["gh_nmax"],
                  n_v=d["n_v"], v_min=d["v_min"], v_max=d["v_max"],
                  dens=DENS[dens] if isinstance(dens, str) else int(dens),
                  l_max=int(d.get("l_max", 0)))


def params(d: dict) -> Params:
    return Params(dt=d["dt"], eps=d["eps"], mu=d["mu"], alpha=d["alpha"], mass=d["mass"],
                  entropy=ENTROPY[d["entropy"]], n_E=d["n_E"], n_x=d["n_x"],
                  prior_every=d["prior_every"], E_lo=d["E_lo"], E_hi=d["E_hi"],
                  smooth=int(d.get("smooth", 0)), cells=int(d.get("cells", 0)))


def n_cells(par: dict) -> int:
    """Cells of the prior grid: n_E n_x, twice that with the L_z split (cells bit 0)."""
    return int(par["n_E"]) * int(par["n_x"]) * (2 if int(par.get("cells", 0)) & 1 else 1)


def smooth_grid(par: dict, grid):
    """Thin-plate smoothing of an n_E x n_x prior grid with the GCV-chosen
    lambda (Sec. 2.3.2); returns (smoothed grid, lambda)."""
    w = _f64(grid).copy().reshape(-1)
    if w.size != int(par["n_E"]) * int(par["n_x"]):
        raise ValueError("grid size does not match n_E * n_x")
    lam = C.c_double()
    if lib().orc_smooth_grid(C.byref(params(dict(par, smooth=1))), _p(w), C.byref(lam)) != 0:
        raise RuntimeError("orc_smooth_grid failed")
    return w, lam.value


def smooth_grid_at(par: dict, grid, lam: float):
    """The same smoothing with a given lambda (no search)."""
    w = _f64(grid).copy().reshape(-1)
    if w.size != int(par["n_E"]) * int(par["n_x"]):
        raise ValueError("grid size does not match n_E * n_x")
    if lib().orc_smooth_grid_at(C.byref(params(dict(par, smooth=1))), _p(w), float(lam)) != 0:
        raise RuntimeError("orc_smooth_grid_at failed")
    return w


def J_of(lay: dict) -> int:
    return int(lib().orc_J(C.byref(layout(lay))))


def phi(pot, r: float) -> float:
    return lib().orc_phi(C.byref(potential(pot)), float(r))


def phi3(pot, x: float, y: float, z: float) -> float:
    return lib().orc_phi3(C.byref(potential(pot)), float(x), float(y), float(z))


def lc(pot, E: float) -> float:
    return lib().orc_lc(C.byref(potential(pot)), float(E))


def accel(pot, x, y, z):
    g = np.zeros(3)
    lib().orc_accel(C.byref(potential(pot)), float(x), float(y), float(z), _p(g))
    return g


def hermite(n: int, x: float) -> float:
    return lib().orc_hermite(int(n), float(x))


def gh_u(n: int, nu: float) -> float:
    return lib().orc_gh_u(int(n), float(nu))


def plm(l: int, m: int, x: float) -> float:
    """Associated Legendre function P_l^m(x) with the Condon-Shortley phase."""
    return lib().orc_plm(int(l), int(m), float(x))


def ylm(l: int, m: int, ct: float, phi: float) -> float:
    """Real orthonormal spherical harmonic at cos(theta) = ct and azimuth phi."""
    return lib().orc_ylm(int(l), int(m), float(ct), float(phi))


def kernels(lay: dict, x, y, z, vz, V_p=None, sigma_p=None):
    """Non-zero kernels of one point: dict {j: K_j} (entries of a point on a
    mesh radius with zero weight included)."""
    nR = max(lay["n_R"], 1)
    V = _f64(np.zeros(nR) if V_p is None else V_p)
    S = _f64(np.ones(nR) if sigma_p is None else sigma_p)
    idx = np.zeros(512, dtype=np.int32)
    val = np.zeros(512)
    n = lib().orc_kernels(C.byref(layout(lay)), _p(V), _p(S), float(x), float(y), float(z),
                          float(vz), idx.ctypes.data_as(C.POINTER(C.c_int32)), _p(val))
    return {int(idx[k]): float(val[k]) for k in range(n)}


def deposit(parts: dict, u, lay: dict, mass=1.0, n_norm=None, V_p=None, sigma_p=None,
            band=0.0, nthreads=1, with_abs=False):
    """y_j = (mass / n_norm) sum_i u_i K_j(z_i). With ``with_abs`` also returns
    the absolute sums and the sums over particles within ``band`` of an edge."""
    x, y, z, vx, vy, vz = (_f64(parts[k]) for k in ("x", "y", "z", "vx", "vy", "vz"))
    u = _f64(u)
    n = x.size
    J = J_of(lay)
    nR = max(lay["n_R"], 1)
    V = _f64(np.zeros(nR) if V_p is None else V_p)
    S = _f64(np.ones(nR) if sigma_p is None else sigma_p)
    out = np.zeros(J)
    ya = np.zeros(J)
    yb = np.zeros(J)
    lib().orc_deposit(n, _p(x), _p(y), _p(z), _p(vx), _p(vy), _p(vz), _p(u),
                      n if n_norm is None else int(n_norm), float(mass), C.byref(layout(lay)),
                      _p(V), _p(S), _p(out), _p(ya) if with_abs else None,
                      _p(yb) if with_abs else None, float(band), int(nthreads))
    return (out, ya, yb) if with_abs else out


def cells(pot, par: dict, parts: dict):
    x, y, z, vx, vy, vz = (_f64(parts[k]) for k in ("x", "y", "z", "vx", "vy", "vz"))
    n = x.size
    c = np.zeros(n, dtype=np.int32)
    E = np.zeros(n)
    xc = np.zeros(n)
    lib().orc_cells(C.byref(potential(pot)), C.byref(params(par)), n, _p(x), _p(y), _p(z),
                    _p(vx), _p(vy), _p(vz), c.ctypes.data_as(C.POINTER(C.c_int32)), _p(E), _p(xc))
    return c, E, xc


def cell_mass(pot, par: dict, parts: dict, u, mass=1.0):
    x, y, z, vx, vy, vz = (_f64(parts[k]) for k in ("x", "y", "z", "vx", "vy", "vz"))
    out = np.zeros(n_cells(par))
    lib().orc_cell_mass(C.byref(potential(pot)), C.byref(params(par)), x.size, _p(x), _p(y),
                        _p(z), _p(vx), _p(vy), _p(vz), _p(_f64(u)), float(mass), _p(out))
    return out


def push(pot, dt, parts: dict, nsteps: int):
    """Advance copies of the particles nsteps DKD steps; returns the new dict."""
    arr = {k: _f64(parts[k]).copy() for k in ("x", "y", "z", "vx", "vy", "vz")}
    lib().orc_push(C.byref(potential(pot)), float(dt), arr["x"].size,
                   *[_p(arr[k]) for k in ("x", "y", "z", "vx", "vy", "vz")], int(nsteps))
    return arr


class OracleFit:
    """One M2M fit on the CPU in FP64 (owns copies of all arrays)."""

    def __init__(self, pot, lay: dict, par: dict, parts: dict, Y, sigma, V_p=None,
                 sigma_p=None, u=None, uhat=None, track_flags=False, band=3e-5, nthreads=1):
        self.arr = {k: _f64(parts[k]).copy() for k in ("x", "y", "z", "vx", "vy", "vz")}
        n = self.arr["x"].size
        self.n = n
        self.arr["u"] = _f64(np.ones(n) if u is None else u).copy()
        self.arr["uhat"] = _f64(np.ones(n) if uhat is None else uhat).copy()
        self.J = J_of(lay)
        nR = max(lay["n_R"], 1)
        self.Y = _f64(Y).copy()
        self.sigma = _f64(sigma).copy()
        self.Vp = _f64(np.zeros(nR) if V_p is None else V_p).copy()
        self.sp = _f64(np.ones(nR) if sigma_p is None else sigma_p).copy()
        self.ytilde = np.zeros(self.J)
        self.yraw = np.zeros(self.J)
        self.delta = np.zeros(self.J)
        self.flag = np.zeros(n, dtype=np.uint8) if track_flags else None
        m = Model()
        m.n = n
        for k in ("x", "y", "z", "vx", "vy", "vz", "u", "uhat"):
            setattr(m, k, _p(self.arr[k]))
        pot = pot.as_dict() if hasattr(pot, "as_dict") else dict(pot)
        pot.update({k: par[k] for k in SCF_KEYS if k in par})  # the expansion may come with par
        m.pot = potential(pot)
        m.lay = layout(lay)
        m.par = params(par)
        m.J = self.J
        m.Y, m.sigma, m.Vp, m.sp = _p(self.Y), _p(self.sigma), _p(self.Vp), _p(self.sp)
        m.ytilde, m.yraw, m.delta = _p(self.ytilde), _p(self.yraw), _p(self.delta)
        m.kstep = 0
        m.flag = self.flag.ctypes.data_as(C.POINTER(C.c_uint8)) if track_flags else None
        m.band = band
        m.nthreads = nthreads
        self.ucell = np.ones(n_cells(par))
        m.ucell = _p(self.ucell)
        self.scf = np.zeros(max(scf_size(pot), 1))
        m.scf = _p(self.scf)
        m.tstep = 0
        self.m = m
        if self.Y.size != self.J or self.sigma.size != self.J:
            raise ValueError("target length does not match the layout")
        if lib().orc_init(C.byref(m)) != 0:
            raise RuntimeError("orc_init failed")

    @property
    def chi2(self) -> float:
        return float(self.m.chi2)

    @property
    def kstep(self) -> int:
        return int(self.m.kstep)

    def step(self, n: int, correct: bool = True):
        hist = np.zeros(max(n, 1))
        lib().orc_steps(C.byref(self.m), int(n), int(bool(correct)), _p(hist))
        return hist[:n]

    def refresh_priors(self):
        lib().orc_refresh_priors(C.byref(self.m))

    def weights(self, mass=1.0):
        return self.arr["u"] * mass / self.n

    def state(self) -> dict:
        return {k: v.copy() for k, v in self.arr.items()}
