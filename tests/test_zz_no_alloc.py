"""GPU test of mcx_run_static, the entry point that allocates nothing (its
event queues and tally table sit in the library's fixed device array).

It must transport the same histories into the same tallies as mcx_run:
histories are independent and their random streams depend only on (seed,
history id) (Sec. 4.3), so the smaller bank and tally table of the static
array change the schedule, not the events, and Sum q / Sum q^2 agree up to
the order of FP64 summation (1e-11 relative).  Two calls in a row share the
array, the second with fewer histories and another seed: the second must not
see the first's contents."""
import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu


def _mcx():
    import paper_2003_00796_amd as mcx
    return mcx


def _same(a, b, rtol=1e-11):
    scale = max(np.abs(b).max(), 1e-300)
    bad = np.abs(a - b) > rtol * np.abs(b) + 1e-13 * scale
    assert not bad.any(), (int(bad.sum()), float(np.abs(a - b).max()), scale)


CASES = [("hetero_broad_64", 1, 60000, 20000), ("electron_200", 0, 3000, 1000), ("water_pencil_32", 0, 50000, 7000)]


@pytest.mark.parametrize("name,precision,n1,n2", CASES)
def test_static_run_equals_run_on_two_calls(name, precision, n1, n2):
    mcx = _mcx()
    wl = W.workload(name, n1)
    ref = mcx.Simulator(precision, 0).setup(wl)
    sta = mcx.Simulator(precision, 0).setup(wl)
    try:
        for seed, first, n in ((wl["seed"], 0, n1), (wl["seed"] + 7, 1000, n2)):
            print(f"case {name} precision {precision} seed {seed} histories [{first}, {first + n})", flush=True)
            ref.reset()
            sta.reset()
            ref.run(seed, first, n)
            sta.run_static(seed, first, n)
            q_r, q2_r = ref.tally()
            q_s, q2_s = sta.tally()
            assert q_r.sum() > 0.0
            _same(q_s, q_r)
            _same(q2_s, q2_r)
            st_r, st_s = ref.stats(), sta.stats()
            assert st_s["histories"] == st_r["histories"] == n
            for k in ("flights", "esteps", "deposits", "secondaries", "escaped", "absorbed"):
                assert st_s[k] == st_r[k], k
            d_r, s_r = ref.dose()
            d_s, s_s = sta.dose()
            _same(d_s, d_r)
    finally:
        ref.close()
        sta.close()


def test_static_run_refuses_test_mode_and_keeps_working():
    mcx = _mcx()
    wl = W.workload("water_pencil_32", 4000)
    sim = mcx.Simulator(0, 0).setup(wl)
    try:
        sim.set_test_mode(True)
        with pytest.raises(mcx.MCXError) as ei:
            sim.run_static(wl["seed"], 0, 4000)
        assert "MCX_E_UNSUPPORTED" in str(ei.value)
        sim.set_test_mode(False)
        sim.reset()
        sim.run_static(wl["seed"], 0, 4000)
        assert sim.stats()["histories"] == 4000
    finally:
        sim.close()
