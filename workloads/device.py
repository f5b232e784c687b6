"""Seeded draws made on the GPU with torch (input plumbing for the serving
workload, where thousands of initial models are needed at request rate).

Same models as ``dynamics.sample_plummer_jeans``: Plummer radii and
isotropic Gaussian velocities with the Jeans dispersion of the tracer in the
request's potential, redrawn until bound. Random numbers come from torch's
device Philox generator keyed by the request seed.
"""

from __future__ import annotations

import math

import numpy as np

from .dynamics import PlummerTracer, Potential, _jeans_sigma2_table


def _psi_torch(pot: Potential, r):
    import torch
    out = pot.G * pot.M_star * pot.upsilon / (r + pot.a)
    if pot.has_nfw:
        q = r / pot.r_s
        l = torch.where(q > 1e-6, torch.log1p(q) / torch.clamp(q, min=1e-300), 1.0 - 0.5 * q)
        out = out + pot.G * pot.M200 / pot._fc() / pot.r_s * l
    return out


def plummer_jeans_device(n: int, pot: Potential, seed: int, device="cuda", b: float = 1.0,
                         dtype=None):
    """Dict of device tensors x, y, z, vx, vy, vz (``dtype``, default float32)."""
    import torch
    dtype = torch.float32 if dtype is None else dtype
    g = torch.Generator(device=device)
    g.manual_seed(int(seed))
    f64 = torch.float64
    u = torch.rand(n, generator=g, device=device, dtype=f64).clamp_(1e-12, 1.0 - 1e-12)
    r = b / torch.sqrt(u.pow(-2.0 / 3.0) - 1.0)
    ct = 2.0 * torch.rand(n, generator=g, device=device, dtype=f64) - 1.0
    st = torch.sqrt(torch.clamp(1.0 - ct * ct, min=0.0))
    ph = 2.0 * math.pi * torch.rand(n, generator=g, device=device, dtype=f64)
    rt, s2 = _jeans_sigma2_table(pot, PlummerTracer(1.0, b))
    lrt = torch.as_tensor(np.log(rt), device=device)
    s2t = torch.as_tensor(s2, device=device)
    lr = torch.log(r).clamp(lrt[0], lrt[-1])
    i = torch.clamp(torch.searchsorted(lrt, lr) - 1, 0, lrt.numel() - 2)
    f = (lr - lrt[i]) / (lrt[i + 1] - lrt[i])
    sig = torch.sqrt(s2t[i] + f * (s2t[i + 1] - s2t[i]))
    psi = _psi_torch(pot, r)
    v = torch.randn(3, n, generator=g, device=device, dtype=f64) * sig
    for _ in range(64):
        bad = 0.5 * (v * v).sum(0) >= psi
        nb = int(bad.sum())
        if nb == 0:
            break
        v[:, bad] = torch.randn(3, nb, generator=g, device=device, dtype=f64) * sig[bad]
    x = r * st * torch.cos(ph)
    y = r * st * torch.sin(ph)
    z = r * ct
    return {k: t.to(dtype).contiguous() for k, t in
            (("x", x), ("y", y), ("z", z), ("vx", v[0]), ("vy", v[1]), ("vz", v[2]))}


def om_model_device(n: int, pot: Potential, r_a: float, seed: int, device="cuda", dtype=None,
                    df=None):
    """Hernquist(1, 1) tracer with Osipkov-Merritt anisotropy radius ``r_a``
    (inf: isotropic) in ``pot``: the model of ``dynamics.sample_om_model``,
    drawn on the device. The DF table f(Q) comes from ``EddingtonDF``."""
    import torch
    from .dynamics import EddingtonDF, HernquistTracer, R_CLIP, _envelope
    dtype = torch.float32 if dtype is None else dtype
    tracer = HernquistTracer(1.0, 1.0)
    if df is None:
        df = EddingtonDF(pot, tracer, r_a)
    g = torch.Generator(device=device)
    g.manual_seed(int(seed))
    f64 = torch.float64
    u = torch.rand(n, generator=g, device=device, dtype=f64).clamp_(1e-300, 1.0 - 1e-16)
    q = torch.sqrt(u)
    r = torch.clamp(q / (1.0 - q), max=R_CLIP)
    ct = 2.0 * torch.rand(n, generator=g, device=device, dtype=f64) - 1.0
    st = torch.sqrt(torch.clamp(1.0 - ct * ct, min=0.0))
    ph = 2.0 * math.pi * torch.rand(n, generator=g, device=device, dtype=f64)
    psi = _psi_torch(pot, r)
    Qt = torch.as_tensor(df.Q, device=device)
    lft = torch.as_tensor(df.lnf, device=device)

    def fQ(Q):
        Qc = Q.clamp(Qt[0], Qt[-1])
        i = torch.clamp(torch.searchsorted(Qt, Qc) - 1, 0, Qt.numel() - 2)
        w = (Qc - Qt[i]) / (Qt[i + 1] - Qt[i])
        val = torch.exp(lft[i] + w * (lft[i + 1] - lft[i]))
        return torch.where(Q > Qt[0], val, torch.zeros_like(val))

    r_grid = np.logspace(-7, 9, 400)
    env_g = torch.as_tensor(_envelope(pot, df, r_grid) * 1.6, device=device)
    pos = (torch.log10(r).clamp(-7.0, 9.0) + 7.0) / 16.0 * (r_grid.size - 1)
    i0 = torch.clamp(pos.floor().long(), 0, r_grid.size - 2)
    env = torch.maximum(env_g[i0], env_g[i0 + 1]) * 1.25
    s_out = torch.empty(n, device=device, dtype=f64)
    todo = torch.arange(n, device=device)
    for _ in range(10_000):
        if todo.numel() == 0:
            break
        s = torch.rand(todo.numel(), generator=g, device=device, dtype=f64)
        a = torch.rand(todo.numel(), generator=g, device=device, dtype=f64)
        p = s * s * fQ(psi[todo] * (1.0 - s * s))
        acc = a * env[todo] < p
        s_out[todo[acc]] = s[acc]
        todo = todo[~acc]
    if todo.numel():
        raise RuntimeError("velocity rejection did not converge")
    vp = s_out * torch.sqrt(2.0 * psi)
    cv = 2.0 * torch.rand(n, generator=g, device=device, dtype=f64) - 1.0
    sv = torch.sqrt(torch.clamp(1.0 - cv * cv, min=0.0))
    pv = 2.0 * math.pi * torch.rand(n, generator=g, device=device, dtype=f64)
    scale = 1.0 if math.isinf(r_a) else 1.0 / torch.sqrt(1.0 + (r / r_a) ** 2)
    vr = vp * cv
    vth = vp * sv * torch.cos(pv) * scale
    vph = vp * sv * torch.sin(pv) * scale
    cp, sp = torch.cos(ph), torch.sin(ph)
    out = {"x": r * st * cp, "y": r * st * sp, "z": r * ct,
           "vx": vr * st * cp + vth * ct * cp - vph * sp,
           "vy": vr * st * sp + vth * ct * sp + vph * cp,
           "vz": vr * ct - vth * st}
    return {k: t.to(dtype).contiguous() for k, t in out.items()}
