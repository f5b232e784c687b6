"""One M2M fit on the GPU: device-resident particles behind an ``m2m_ctx``.

PyTorch provides the device memory (the particle arrays are torch tensors the
fit keeps alive) and the stream; every computation runs in ``libm2m.so``.
"""

from __future__ import annotations

import ctypes as C

import numpy as np
import torch

from . import _abi as A

FIELDS = ("x", "y", "z", "vx", "vy", "vz")


def _torch_dtype(dtype: str):
    return {"f32": torch.float32, "f64": torch.float64}[dtype]


def _dp(a: np.ndarray | None):
    if a is None:
        return None
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _f64(a):
    return None if a is None else np.ascontiguousarray(np.asarray(a, dtype=np.float64))


class Fit:
    """Particles (dict of arrays x, y, z, vx, vy, vz), a potential, an
    observable layout and step parameters (dicts as built by ``workloads``).

    ``u`` and ``u_prior`` default to 1 (equal weights, flat priors)."""

    def __init__(self, potential, layout: dict, params: dict, particles: dict, dtype: str = "f32",
                 u=None, u_prior=None, device: str = "cuda", stream=None):
        A.lib()
        self.dtype = dtype
        self.layout = dict(layout)
        self.params = dict(params)
        tdt = _torch_dtype(dtype)
        self.n = int(particles["x"].shape[0]) if hasattr(particles["x"], "shape") else len(particles["x"])
        # every device operation of this fit (the state copies below, the
        # library's work) is ordered on one stream
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        self.J = A.m2m_num_observables(self.layout)
        self.n_R = self.layout["n_R"] if self.layout["kin"] != "none" else 0
        ws_bytes = A.m2m_workspace_bytes(self.layout, self.params, self.n, dtype)
        with torch.cuda.stream(self.stream):
            # the eight state arrays back to back in one allocation (each start
            # 256-byte aligned): a state about the size of the 256 MB Infinity
            # Cache streams up to 1.2x faster packed than spread over separate
            # allocations, whose placement leaves cache sets unevenly used
            esz = 8 if dtype == "f64" else 4
            stride = (self.n * esz + 255) // 256 * 256 // esz
            self._buf = torch.empty(8 * stride, dtype=tdt, device=device)
            self.t = {}
            for f, k in enumerate((*FIELDS, "u", "uh")):
                self.t[k] = self._buf[f * stride:f * stride + self.n]
            for k in FIELDS:
                v = particles[k]
                src = (v if torch.is_tensor(v) else torch.as_tensor(np.asarray(v)))
                self.t[k].copy_(src.reshape(-1))
            for k, v in (("u", u), ("uh", u_prior)):
                if v is None:
                    self.t[k].fill_(1.0)
                else:
                    self.t[k].copy_((v if torch.is_tensor(v) else torch.as_tensor(np.asarray(v))).reshape(-1))
            # the library's workspace comes from torch's caching allocator, so
            # that creating and closing fits allocates no device memory directly
            # (no device-wide synchronization while other fits run)
            self._ws = torch.empty(max(ws_bytes, 1), dtype=torch.uint8, device=device)
        ctx = C.c_void_p()
        ptrs = [C.c_void_p(self.t[k].data_ptr()) for k in (*FIELDS, "u", "uh")]
        st = A.lib().m2m_create(C.byref(A.potential(potential)), C.byref(A.obs_layout(self.layout)),
                                C.byref(A.params(self.params)), self.n, A.DTYPE[dtype], *ptrs,
                                C.c_void_p(self._ws.data_ptr()), C.c_size_t(ws_bytes),
                                C.c_void_p(self.stream.cuda_stream), C.byref(ctx))
        A.check(st, "m2m_create")
        self.ctx = ctx

    # ------------------------------------------------------------- calls --
    def _chk(self, st, where):
        A.check(st, where, self.ctx)

    def set_targets(self, Y, sigma, V_p=None, sigma_p=None):
        Y, sigma, V_p, sigma_p = _f64(Y), _f64(sigma), _f64(V_p), _f64(sigma_p)
        self._chk(A.lib().m2m_set_targets(self.ctx, int(Y.size), _dp(Y), _dp(sigma), _dp(V_p),
                                          _dp(sigma_p)), "m2m_set_targets")

    def step(self, n_steps: int, correct: bool = True):
        self._chk(A.lib().m2m_step(self.ctx, int(n_steps), int(bool(correct))), "m2m_step")

    def update_priors(self):
        self._chk(A.lib().m2m_update_priors(self.ctx), "m2m_update_priors")

    def refresh_potential(self):
        """Rebuild the self-consistent stellar potential from the current
        particles and weights (params scf_nr > 0)."""
        self._chk(A.lib().m2m_refresh_potential(self.ctx), "m2m_refresh_potential")

    def potential_table(self) -> np.ndarray:
        """Node table of the self-consistent potential: array (scf_nr,
        (scf_lmax+1)^2, 2) of Phi_lm(rho_k) and r dPhi_lm/dr there."""
        K, L = int(self.params.get("scf_nr", 0)), int(self.params.get("scf_lmax", 0))
        out = np.zeros(max(K * (L + 1) ** 2 * 2, 1))
        self._chk(A.lib().m2m_get_potential(self.ctx, _dp(out), int(out.size)),
                  "m2m_get_potential")
        return out.reshape(K, (L + 1) ** 2, 2)

    def weights(self) -> np.ndarray:
        out = np.empty(self.n, dtype=np.float64 if self.dtype == "f64" else np.float32)
        self._chk(A.lib().m2m_get_weights(self.ctx, out.ctypes.data_as(C.c_void_p), 0),
                  "m2m_get_weights")
        return out

    def weights_device(self) -> torch.Tensor:
        out = torch.empty_like(self.t["u"])
        self._chk(A.lib().m2m_get_weights(self.ctx, C.c_void_p(out.data_ptr()), 1),
                  "m2m_get_weights")
        return out

    def observables(self) -> dict:
        y, yt, d = np.zeros(self.J), np.zeros(self.J), np.zeros(self.J)
        c2 = C.c_double()
        self._chk(A.lib().m2m_get_observables(self.ctx, _dp(y), _dp(yt), _dp(d), C.byref(c2)),
                  "m2m_get_observables")
        return dict(y=y, ytilde=yt, delta=d, chi2=c2.value)

    def chi2_history(self, max_n: int = 8192) -> np.ndarray:
        out = np.zeros(max_n)
        n = C.c_int32()
        self._chk(A.lib().m2m_get_chi2_history(self.ctx, _dp(out), int(max_n), C.byref(n)),
                  "m2m_get_chi2_history")
        return out[: n.value]

    def observe(self, V_p=None, sigma_p=None) -> np.ndarray:
        y = np.zeros(self.J)
        self._chk(A.lib().m2m_observe(self.ctx, _dp(_f64(V_p)), _dp(_f64(sigma_p)), _dp(y)),
                  "m2m_observe")
        return y

    def profile_step(self, n_steps: int, correct: bool = True):
        """(step kernel, reduction) times in ms per step from HIP events around
        graph replays with and without one extra measuring reduction per step;
        runs 2 * 32 * ceil(n / 32) steps (batch: 2 * 8 * ceil(n / 8))."""
        a, b = C.c_double(), C.c_double()
        self._chk(A.lib().m2m_profile_step(self.ctx, int(n_steps), int(bool(correct)), C.byref(a),
                                           C.byref(b)), "m2m_profile_step")
        return a.value, b.value

    def get_state(self) -> bytes:
        n = C.c_size_t()
        self._chk(A.lib().m2m_get_state(self.ctx, None, C.byref(n)), "m2m_get_state")
        buf = C.create_string_buffer(n.value)
        self._chk(A.lib().m2m_get_state(self.ctx, buf, C.byref(n)), "m2m_get_state")
        return buf.raw[: n.value]

    def set_state(self, blob: bytes):
        buf = C.create_string_buffer(blob, len(blob))
        self._chk(A.lib().m2m_set_state(self.ctx, buf, len(blob)), "m2m_set_state")

    def particles(self) -> dict:
        """Host copies (float64) of the particle state, u and u_prior.
        Pending prior assignments are applied first."""
        self.weights()  # synchronizes and flushes pending priors
        return {k: v.detach().cpu().numpy().astype(np.float64) for k, v in self.t.items()}

    def close(self):
        if getattr(self, "ctx", None):
            A.check(A.lib().m2m_destroy(self.ctx), "m2m_destroy")
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()
