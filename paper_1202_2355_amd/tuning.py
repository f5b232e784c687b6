"""Launch parameters of the step kernel per workload class, as the autotuner
(``autotune.py``) picked them on an MI355X, and their application.

A class is the kind of run (one fit, or a batch of fits), the particle-state
type, the kind of kinematic observables and, for one fit, the order of
magnitude of its particle count. Its parameters are the step kernel's block
size and tiles per compute unit, the in-tile deposit mode, the most private
bin copies per block, and for batches the number of overlapping groups and
whether their steps are replayed from captured graphs.
They are library settings for contexts and batches created afterwards, so
``use`` is called before a fit or batch is made; tests call it to run at the
benchmarked shapes.
"""

from __future__ import annotations

import json
import math
import os

from . import _abi as A

TUNED_FILE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tuned.json")

DEFAULT = {"block": 1024, "tiles_per_cu": 1, "deposit": "f64", "private_copies": 0, "groups": 2,
           "graphs": 0}
DEFAULT_F64 = dict(DEFAULT, block=256)


def class_key(mode: str, dtype: str, layout: dict, n: int | None = None) -> str:
    """'single:<dtype>:<kin>:<log10 N>' or 'batch:<dtype>:<kin>'; kin carries
    '+alm' for spherical-harmonic density observables."""
    kin = layout["kin"] + ("+alm" if layout.get("dens") == "alm" else "")
    if mode == "batch":
        return f"batch:{dtype}:{kin}"
    if mode != "single":
        raise ValueError(mode)
    return f"single:{dtype}:{kin}:{int(round(math.log10(max(int(n), 1))))}"


def load(path: str = TUNED_FILE) -> dict:
    try:
        with open(path) as fh:
            return json.load(fh).get("classes", {})
    except (OSError, ValueError):
        return {}


def lookup(mode: str, dtype: str, layout: dict, n: int | None = None, table=None) -> dict:
    """The tuned parameters of the class, else those of the nearest tuned
    size of the same run kind, state type and kinematics, else defaults."""
    table = load() if table is None else table
    base = DEFAULT_F64 if dtype == "f64" else DEFAULT
    key = class_key(mode, dtype, layout, n)
    if key in table:
        return dict(base, **table[key]["params"])
    if mode == "single":
        stem, mag = key.rsplit(":", 1)
        near = [(abs(int(k.rsplit(":", 1)[1]) - int(mag)), k) for k in table
                if k.rsplit(":", 1)[0] == stem]
        if near:
            return dict(base, **table[min(near)[1]]["params"])
    return dict(base)


def apply(params: dict) -> None:
    """Make ``params`` the library's settings for contexts and batches made
    from now on."""
    A.m2m_set_launch(int(params["block"]), int(params["tiles_per_cu"]))
    A.m2m_set_deposit_mode(params["deposit"])
    A.m2m_set_private_copies(int(params["private_copies"]))
    A.m2m_set_batch_groups(int(params["groups"]))
    A.m2m_set_batch_graphs(int(params["graphs"]))


def current() -> dict:
    b, t = A.m2m_get_launch()
    dep = {v: k for k, v in A.DEPOSIT.items()}[A.m2m_get_deposit_mode()]
    return {"block": b, "tiles_per_cu": t, "deposit": dep,
            "private_copies": A.m2m_get_private_copies(), "groups": A.m2m_get_batch_groups(),
            "graphs": A.m2m_get_batch_graphs()}


def use(mode: str, dtype: str, layout: dict, n: int | None = None) -> dict:
    """Apply the tuned parameters of a class; returns them."""
    p = lookup(mode, dtype, layout, n)
    apply(p)
    return p


class tuned:
    """Context manager: the tuned parameters of a class inside, the previous
    settings restored on exit."""

    def __init__(self, mode: str, dtype: str, layout: dict, n: int | None = None):
        self.args = (mode, dtype, layout, n)

    def __enter__(self):
        self.before = current()
        self.params = use(*self.args)
        return self.params

    def __exit__(self, *exc):
        apply(self.before)


def record(key: str, params: dict, us_per_step: float, source: str, path: str = TUNED_FILE):
    """Store the autotuner's pick for a class in the table."""
    try:
        with open(path) as fh:
            d = json.load(fh)
    except (OSError, ValueError):
        d = {}
    d.setdefault("classes", {})[key] = {"params": params, "us_per_step": us_per_step,
                                         "source": source}
    with open(path, "w") as fh:
        json.dump(d, fh, indent=1, sort_keys=True)
        fh.write("\n")
