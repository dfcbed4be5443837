"""GPU tests of the concurrent race (Algorithm 1).  This file sorts first among
the GPU tests so the CPU leg's child process starts before the test process
has touched the GPU."""

import pytest

from oracle.kkt import kkt
from paper_2607_03627_amd import uclp
from paper_2607_03627_amd.instances import make_instance
from paper_2607_03627_amd.race import race

pytestmark = pytest.mark.gpu


def test_gpu_leg_wins_on_the_6049_bus_grid():
    # HiGHS needs minutes for this LP; the FP32 PDHG reaches 1e-4 well inside
    # the first 0.5 s poll interval
    lp = make_instance("large_kc0", 0)
    r = race(lp, uclp.uc_lp_opts_default(precision=uclp.UC_LP_FP32_MIXED), poll_s=0.5, timeout_s=600)
    print("race", r.winner, r.seconds, [(x.name, x.status, x.seconds) for x in r.results], flush=True)
    assert r.winner == "gpu-pdhg" and r.polls == 1
    gpu, cpu = r.results
    assert cpu.status == "TERMINATED"
    assert kkt(lp, gpu.x, gpu.y).rel_kkt <= 1e-4 * 1.001


def test_cpu_leg_wins_when_the_gpu_leg_cannot_finish():
    lp = make_instance("tiny", 0, n_periods=6)
    slow = uclp.uc_lp_opts_default(precision=uclp.UC_LP_FP64, eps_rel=1e-30, iter_limit=10 ** 9, time_limit_s=120)
    r = race(lp, slow, poll_s=0.5, timeout_s=120)
    print("race", r.winner, r.seconds, [(x.name, x.status, x.seconds) for x in r.results], flush=True)
    assert r.winner == "cpu-highs-ipm"
    gpu, cpu = r.results
    assert gpu.status == "TERMINATED"
    assert kkt(lp, cpu.x, cpu.y).rel_kkt <= 1e-7
