"""ctypes binding of ``libm2m.so`` (declared in ``include/m2m.h``).

Argument marshalling only: every step of the M2M path runs in the HIP
library. The functions keep the C names; failures raise ``M2MError`` with the
library's status and message. Loading fails loudly when the library has not
been built.
"""

from __future__ import annotations

import ctypes as C
import os

import numpy as np

from .build import LIB

M2M_OK, M2M_EINVAL, M2M_ENOMEM, M2M_EDEVICE, M2M_ESTATE, M2M_ENONFINITE, M2M_EUNSUPPORTED = range(7)
STATUS_NAMES = {0: "M2M_OK", 1: "M2M_EINVAL", 2: "M2M_ENOMEM", 3: "M2M_EDEVICE",
                4: "M2M_ESTATE", 5: "M2M_ENONFINITE", 6: "M2M_EUNSUPPORTED"}
M2M_F32, M2M_F64 = 0, 1
M2M_S_MPR, M2M_S_GWR = 0, 1
M2M_KIN_NONE, M2M_KIN_V2, M2M_KIN_GH, M2M_KIN_LOSVD = 0, 1, 2, 3
KIN = {"none": M2M_KIN_NONE, "v2": M2M_KIN_V2, "gh": M2M_KIN_GH, "losvd": M2M_KIN_LOSVD}
ENTROPY = {"mpr": M2M_S_MPR, "gwr": M2M_S_GWR}
M2M_DENS_BINS, M2M_DENS_ALM = 0, 1
DENS = {"bins": M2M_DENS_BINS, "alm": M2M_DENS_ALM}
DTYPE = {"f32": M2M_F32, "f64": M2M_F64}


class M2MError(RuntimeError):
    def __init__(self, status: int, where: str, msg: str = ""):
        self.status = status
        super().__init__(f"{where}: {STATUS_NAMES.get(status, status)}" + (f" ({msg})" if msg else ""))


class m2m_potential(C.Structure):
    _fields_ = [(k, C.c_double) for k in ("G", "M_star", "a", "upsilon", "M200", "c", "r_s",
                                          "v0", "r0", "q")]


class m2m_obs_layout(C.Structure):
    _fields_ = [("n_r", C.c_int32), ("r_min", C.c_double), ("r_max", C.c_double),
                ("n_R", C.c_int32), ("R_min", C.c_double), ("R_max", C.c_double),
                ("kin", C.c_int32), ("gh_nmax", C.c_int32), ("n_v", C.c_int32),
                ("v_min", C.c_double), ("v_max", C.c_double), ("dens", C.c_int32),
                ("l_max", C.c_int32)]


class m2m_params(C.Structure):
    _fields_ = [("dt", C.c_double), ("eps", C.c_double), ("mu", C.c_double),
                ("alpha", C.c_double), ("mass", C.c_double), ("entropy", C.c_int32),
                ("n_E", C.c_int32), ("n_x", C.c_int32), ("prior_every", C.c_int32),
                ("E_lo", C.c_double), ("E_hi", C.c_double), ("smooth", C.c_int32),
                ("cells", C.c_int32), ("scf_lmax", C.c_int32), ("scf_nr", C.c_int32),
                ("scf_rmin", C.c_double), ("scf_rmax", C.c_double), ("scf_every", C.c_int32)]


_vp = C.c_void_p
_dp = C.POINTER(C.c_double)
_i32 = C.c_int32
_st = C.c_int  # m2m_status

# name -> (restype, argtypes)
SIGNATURES = {
    "m2m_num_observables": (_i32, [C.POINTER(m2m_obs_layout)]),
    "m2m_workspace_bytes": (C.c_size_t, [C.POINTER(m2m_obs_layout), C.POINTER(m2m_params),
                                         C.c_int64, _i32]),
    "m2m_create": (_st, [C.POINTER(m2m_potential), C.POINTER(m2m_obs_layout),
                         C.POINTER(m2m_params), C.c_int64, _i32] + [_vp] * 8 +
                   [_vp, C.c_size_t, _vp, C.POINTER(_vp)]),
    "m2m_set_targets": (_st, [_vp, _i32, _dp, _dp, _dp, _dp]),
    "m2m_step": (_st, [_vp, _i32, _i32]),
    "m2m_update_priors": (_st, [_vp]),
    "m2m_refresh_potential": (_st, [_vp]),
    "m2m_get_potential": (_st, [_vp, _dp, _i32]),
    "m2m_get_weights": (_st, [_vp, _vp, _i32]),
    "m2m_get_observables": (_st, [_vp, _dp, _dp, _dp, _dp]),
    "m2m_get_chi2_history": (_st, [_vp, _dp, _i32, C.POINTER(_i32)]),
    "m2m_observe": (_st, [_vp, _dp, _dp, _dp]),
    "m2m_observe_noalloc": (_st, [C.POINTER(m2m_obs_layout), C.c_double, C.c_int64, _i32] +
                            [_vp] * 7 + [_dp, _dp, _dp, _vp]),
    "m2m_get_state": (_st, [_vp, _vp, C.POINTER(C.c_size_t)]),
    "m2m_set_state": (_st, [_vp, _vp, C.c_size_t]),
    "m2m_profile_step": (_st, [_vp, _i32, _i32, _dp, _dp]),
    "m2m_destroy": (_st, [_vp]),
    "m2m_smoothing_basis": (_st, [_i32, _i32, C.c_double, C.c_double, _dp,
                                  C.POINTER(C.c_size_t)]),
    "m2m_last_error": (C.c_char_p, [_vp]),
    "m2m_set_launch": (_st, [_i32, _i32]),
    "m2m_get_launch": (_st, [C.POINTER(_i32)] * 2),
    "m2m_set_deposit_mode": (_st, [_i32]),
    "m2m_set_batch_groups": (_st, [_i32]),
    "m2m_set_private_copies": (_st, [_i32]),
    "m2m_set_batch_graphs": (_st, [_i32]),
    "m2m_get_batch_graphs": (_i32, []),
    "m2m_get_private_copies": (_i32, []),
    "m2m_get_batch_groups": (_i32, []),
    "m2m_get_deposit_mode": (_i32, []),
    "m2m_set_interleave": (_st, [_i32]),
    "m2m_get_interleave": (_i32, []),
    "m2m_batch_create": (_st, [_i32, C.c_size_t, _vp, C.POINTER(_vp)]),
    "m2m_batch_admit": (_st, [_vp, _vp, _i32]),
    "m2m_batch_run": (_st, [_vp, _i32]),
    "m2m_batch_poll": (_st, [_vp, C.POINTER(_vp), _i32, C.POINTER(_i32), C.POINTER(_i32)]),
    "m2m_batch_poll_lagged": (_st, [_vp, C.POINTER(_vp), _i32, C.POINTER(_i32), C.POINTER(_i32)]),
    "m2m_batch_footprint": (C.c_size_t, [_vp]),
    "m2m_batch_profile": (_st, [_vp, _i32, _dp, _dp]),
    "m2m_batch_particles": (C.c_int64, [_vp]),
    "m2m_batch_cancel": (_st, [_vp, _vp]),
    "m2m_batch_destroy": (_st, [_vp]),
}

_lib = None


def lib():
    """The loaded HIP library (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            raise ImportError(f"{LIB} is missing: build it with paper_1202_2355_amd.build.build()")
        L = C.CDLL(LIB)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def last_error(ctx) -> str:
    if not ctx:
        return ""
    s = lib().m2m_last_error(ctx)
    return s.decode() if s else ""


def check(status: int, where: str, ctx=None):
    if status != M2M_OK:
        raise M2MError(status, where, last_error(ctx))


def potential(d) -> m2m_potential:
    d = d.as_dict() if hasattr(d, "as_dict") else d
    return m2m_potential(**{k: float(d[k]) for k in ("G", "M_star", "a", "upsilon", "M200", "c", "r_s")},
                         v0=float(d.get("v0", 0.0)), r0=float(d.get("r0", 1.0)),
                         q=float(d.get("q", 1.0)))


def obs_layout(d: dict) -> m2m_obs_layout:
    kin = KIN[d["kin"]] if isinstance(d["kin"], str) else int(d["kin"])
    dens = d.get("dens", "bins")
    return m2m_obs_layout(n_r=d["n_r"], r_min=d["r_min"], r_max=d["r_max"], n_R=d["n_R"],
                          R_min=d["R_min"], R_max=d["R_max"], kin=kin,
                          gh_nmax=d.get("gh_nmax", 0), n_v=d.get("n_v", 0),
                          v_min=d.get("v_min", 0.0), v_max=d.get("v_max", 0.0),
                          dens=DENS[dens] if isinstance(dens, str) else int(dens),
                          l_max=int(d.get("l_max", 0)))


def params(d: dict) -> m2m_params:
    ent = ENTROPY[d["entropy"]] if isinstance(d["entropy"], str) else int(d["entropy"])
    return m2m_params(dt=d["dt"], eps=d["eps"], mu=d["mu"], alpha=d["alpha"], mass=d["mass"],
                      entropy=ent, n_E=d["n_E"], n_x=d["n_x"], prior_every=d["prior_every"],
                      E_lo=d["E_lo"], E_hi=d["E_hi"], smooth=int(d.get("smooth", 0)),
                      cells=int(d.get("cells", 0)), scf_lmax=int(d.get("scf_lmax", 0)),
                      scf_nr=int(d.get("scf_nr", 0)), scf_rmin=float(d.get("scf_rmin", 0.0)),
                      scf_rmax=float(d.get("scf_rmax", 0.0)),
                      scf_every=int(d.get("scf_every", 1)))


# ---- thin wrappers with the C names ------------------------------------------
def m2m_num_observables(layout: dict) -> int:
    return int(lib().m2m_num_observables(C.byref(obs_layout(layout))))


def m2m_workspace_bytes(layout: dict, par: dict, n: int, dtype: str = "f32") -> int:
    return int(lib().m2m_workspace_bytes(C.byref(obs_layout(layout)), C.byref(params(par)),
                                         int(n), DTYPE[dtype]))


def m2m_set_launch(block: int, tiles_per_cu: int):
    check(lib().m2m_set_launch(int(block), int(tiles_per_cu)), "m2m_set_launch")


M2M_DEPOSIT_F64, M2M_DEPOSIT_F32_COMPENSATED = 0, 1
DEPOSIT = {"f64": M2M_DEPOSIT_F64, "f32c": M2M_DEPOSIT_F32_COMPENSATED}


def m2m_set_deposit_mode(mode):
    mode = DEPOSIT[mode] if isinstance(mode, str) else int(mode)
    check(lib().m2m_set_deposit_mode(mode), "m2m_set_deposit_mode")


def m2m_set_batch_graphs(on: int):
    """Batches rebuilt from now on replay captured graphs (1) or launch every
    step directly (0)."""
    check(lib().m2m_set_batch_graphs(int(on)), "m2m_set_batch_graphs")


def m2m_get_batch_graphs() -> int:
    return int(lib().m2m_get_batch_graphs())


def m2m_set_private_copies(copies: int):
    """Most private copies of the in-tile bins (1, 2, 4, 8; 0: automatic) for
    contexts created from now on."""
    check(lib().m2m_set_private_copies(int(copies)), "m2m_set_private_copies")


def m2m_get_private_copies() -> int:
    return int(lib().m2m_get_private_copies())


def m2m_set_batch_groups(groups: int):
    """Groups a batch of two or more fits steps as (1 or 2, overlapping on
    their own streams) from its next rebuild on."""
    check(lib().m2m_set_batch_groups(int(groups)), "m2m_set_batch_groups")


def m2m_get_batch_groups() -> int:
    return int(lib().m2m_get_batch_groups())


def m2m_get_deposit_mode() -> int:
    return int(lib().m2m_get_deposit_mode())


def m2m_set_interleave(mode: int):
    """Particles of a tile for single fits created from now on: contiguous
    (0), interleaved chunks (1), or by state size (-1, the default)."""
    check(lib().m2m_set_interleave(int(mode)), "m2m_set_interleave")


def m2m_get_interleave() -> int:
    return int(lib().m2m_get_interleave())


def m2m_get_launch():
    b, t = _i32(), _i32()
    lib().m2m_get_launch(C.byref(b), C.byref(t))
    return b.value, t.value


def m2m_smoothing_basis(n_E: int, n_x: int, hE: float, hx: float) -> np.ndarray:
    """The prior-smoothing penalty's eigendecomposition as the library holds
    it: the n_E n_x eigenvalues of the four parity blocks, then their
    eigenvector matrices (host only)."""
    n = C.c_size_t(0)
    check(lib().m2m_smoothing_basis(int(n_E), int(n_x), float(hE), float(hx), None, C.byref(n)),
          "m2m_smoothing_basis")
    out = np.zeros(n.value)
    check(lib().m2m_smoothing_basis(int(n_E), int(n_x), float(hE), float(hx),
                                    out.ctypes.data_as(_dp), C.byref(n)), "m2m_smoothing_basis")
    return out


def m2m_observe_noalloc(layout: dict, mass: float, n: int, dtype: str, ptrs, V_p=None,
                        sigma_p=None, stream=None) -> np.ndarray:
    """y_j (J values) of n particles at the device addresses ``ptrs`` (x, y,
    z, vx, vy, vz, u) with total mass ``mass``, computed in the library's
    static device scratch (no device allocation). ``stream``: a HIP stream
    handle (int) or None for the null stream."""
    L = obs_layout(layout)
    J = m2m_num_observables(layout)
    y = np.zeros(max(J, 1))
    keep = [None if a is None else np.ascontiguousarray(a, dtype=np.float64) for a in (V_p, sigma_p)]
    args = [None if a is None else a.ctypes.data_as(_dp) for a in keep]
    if len(ptrs) != 7:
        raise ValueError("ptrs: the seven addresses x, y, z, vx, vy, vz, u")
    st = lib().m2m_observe_noalloc(C.byref(L), float(mass), int(n), DTYPE[dtype],
                                   *[_vp(int(p)) if p else None for p in ptrs], args[0], args[1],
                                   y.ctypes.data_as(_dp), _vp(int(stream)) if stream else None)
    if st != M2M_OK:
        msg = lib().m2m_last_error(None)
        raise M2MError(st, "m2m_observe_noalloc", msg.decode() if msg else "")
    return y[:J]
