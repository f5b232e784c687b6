"""The batch without draining (m2m_batch_poll_lagged): fits are handed back
exactly one run after the run in which they finished, fits admitted while
earlier runs are still in flight join the next run (its tables are copied on
the batch stream without waiting), and every fit ends with the result of the
same fit run alone. Fits handed back are closed at once or stepped on alone
while the latest run may still execute (their own work waits for it)."""

import sys

import numpy as np
import pytest

from m2m_testlib import cast, oracle_targets
from workloads import workload

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _say(*a):
    print("[gpu-test]", *a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def Fit():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1202_2355_amd import _abi
    _abi.lib()
    from paper_1202_2355_amd.fit import Fit
    return Fit


SPL = 16


def test_lagged_poll_hands_back_one_run_late_with_results_of_the_fit_alone(oracle, Fit):
    from paper_1202_2355_amd.batch import Batch
    wl = workload(2)
    T = oracle_targets(oracle, wl)
    # (particles, steps, run before which the fit is admitted)
    plan = [(9_001, 16, 0), (20_011, 48, 0), (33_333, 32, 0), (5_003, 80, 0), (12_007, 32, 2)]
    extra = 8   # steps the first fit runs alone after it was handed back
    _say("lagged batch", plan)
    parts = [cast(wl.initial_particles(n=n, seed=40 + k), "f32") for k, (n, _, _) in enumerate(plan)]

    def make(k):
        f = Fit(wl.potential, wl.layout, wl.params, parts[k], dtype="f32")
        f.set_targets(T["Y"], T["sigma"], T["V_p"], T["sigma_p"])
        return f

    alone = []
    for k, (n, steps, _) in enumerate(plan):
        f = make(k)
        f.step(steps)
        ref = (f.particles()["u"], f.observables()["ytilde"])
        if k == 0:
            f.step(extra)
            ref = ref + (f.particles()["u"],)
        alone.append(ref)
        f.close()

    # the batch on a stream of its own: the fits' own work (creation, the
    # steps after hand-back) runs on the current stream
    b = Batch(max_fits=8, stream=torch.cuda.Stream())
    fits = {}
    back = {}
    turn = 0
    first = None
    while len(back) < len(plan):
        for k, (n, steps, at) in enumerate(plan):
            if at == turn:
                fits[k] = make(k)
                assert b.admit(fits[k], steps)
        b.run(SPL)
        turn += 1
        done, _ = b.poll_lagged()
        if turn == 1:
            assert done == []   # no run before the latest yet
        for f in done:
            k = next(k for k, g in fits.items() if g is f)
            back[k] = turn
            u, yt = f.particles()["u"], f.observables()["ytilde"]
            np.testing.assert_allclose(u, alone[k][0], rtol=1e-5)
            assert np.abs(yt - alone[k][1]).max() <= 1e-6 * np.abs(alone[k][1]).max()
            if k == 0:
                first = f      # stepped on alone below, while runs continue
            else:
                f.close()      # closed at once: destroy waits for the runs that read it
        if first is not None and turn == back[0]:
            first.step(extra)
        assert turn <= 12, back
    # a fit of s steps admitted before run a finishes in run a + ceil(s / SPL)
    # and is handed back by the poll after the next run
    for k, (n, steps, at) in enumerate(plan):
        assert back[k] == at + -(-steps // SPL) + 1, (k, back)
    np.testing.assert_allclose(first.particles()["u"], alone[0][2], rtol=1e-5)
    first.close()
    b.close()
