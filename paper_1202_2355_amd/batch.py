"""Many fits stepping together (``m2m_batch_*``): per step one fused step
kernel over the tiles of the admitted fits and one finalize kernel, in two
overlapping groups of fits on streams of their own."""

from __future__ import annotations

import ctypes as C

import torch

from . import _abi as A


class Batch:
    def __init__(self, max_fits: int = 64, hbm_budget: int = 0, stream=None):
        A.lib()
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        h = C.c_void_p()
        A.check(A.lib().m2m_batch_create(int(max_fits), int(hbm_budget),
                                         C.c_void_p(self.stream.cuda_stream), C.byref(h)),
                "m2m_batch_create")
        self.h = h
        self.max_fits = max_fits
        self.by_ctx = {}

    def admit(self, fit, n_steps: int) -> bool:
        """Admit ``fit`` for ``n_steps`` steps; False if the budget or the
        slot count does not allow it now."""
        st = A.lib().m2m_batch_admit(self.h, fit.ctx, int(n_steps))
        if st == A.M2M_ENOMEM:
            return False
        A.check(st, "m2m_batch_admit", fit.ctx)
        self.by_ctx[fit.ctx.value] = fit
        return True

    def run(self, steps_per_launch: int):
        A.check(A.lib().m2m_batch_run(self.h, int(steps_per_launch)), "m2m_batch_run")

    def _poll(self, fn, where):
        cap = max(1, len(self.by_ctx))
        arr = (C.c_void_p * cap)()
        nd, na = C.c_int32(), C.c_int32()
        st = fn(self.h, arr, cap, C.byref(nd), C.byref(na))
        done = [self.by_ctx.pop(arr[i]) for i in range(nd.value)]
        if st != A.M2M_OK:
            raise A.M2MError(st, where)
        return done, na.value

    def poll(self):
        """(finished fits, number still active); synchronizes."""
        return self._poll(A.lib().m2m_batch_poll, "m2m_batch_poll")

    def poll_lagged(self):
        """(fits finished by the end of the run before the latest, number
        still in the batch); waits only for that earlier run, so the latest
        run keeps the GPU busy while the caller retires fits and admits new
        ones."""
        return self._poll(A.lib().m2m_batch_poll_lagged, "m2m_batch_poll_lagged")

    def cancel(self, fit):
        A.check(A.lib().m2m_batch_cancel(self.h, fit.ctx), "m2m_batch_cancel")
        self.by_ctx.pop(fit.ctx.value, None)

    def profile(self, n_steps: int):
        """(step kernel, rest of the step) in ms per step from HIP events
        around each step kernel of n_steps batched steps launched one kernel
        at a time."""
        a, b = C.c_double(), C.c_double()
        A.check(A.lib().m2m_batch_profile(self.h, int(n_steps), C.byref(a), C.byref(b)),
                "m2m_batch_profile")
        return a.value, b.value

    def particles(self) -> int:
        """Particles of the fits that still have steps left."""
        return int(A.lib().m2m_batch_particles(self.h))

    @property
    def footprint(self) -> int:
        return int(A.lib().m2m_batch_footprint(self.h))

    @property
    def active(self) -> int:
        return len(self.by_ctx)

    def run_to_completion(self, steps_per_launch: int = 64, max_steps: int = 10_000_000):
        done = []
        ran = 0
        while self.by_ctx:
            if ran > max_steps:
                raise RuntimeError("batch did not finish within max_steps")
            self.run(steps_per_launch)
            ran += steps_per_launch
            d, _ = self.poll()
            done += d
        return done

    def close(self):
        if getattr(self, "h", None):
            A.check(A.lib().m2m_batch_destroy(self.h), "m2m_batch_destroy")
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
