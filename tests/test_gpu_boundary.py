"""GPU tests of the run-control part of the C ABI: cancellation with resume,
checkpoint and restore in a new context, and runs in caller-owned device
memory.  Each compares with an uninterrupted run in library-owned memory on
the same seeded inputs: histories are independent and their random streams
depend only on (seed, history id) (Sec. 4.3), so every split of [0, N) must
give the same per-history event hashes, and Sum q / Sum q^2 equal up to the
order of FP64 summation (1e-11 relative)."""
import threading

import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu


def _mcx():
    import paper_2003_00796_amd as mcx
    return mcx


def _base(wl, n, precision, launch, test=True):
    mcx = _mcx()
    sim = mcx.Simulator(precision, 0).setup(wl)
    sim.set_launch(*launch)
    sim.set_test_mode(test)
    sim.run(wl["seed"], 0, n)
    h = sim.history_results(n)[0] if test else None
    q, q2 = sim.tally()
    st = sim.stats()
    sim.close()
    return dict(hash=h, q=q, q2=q2, stats=st)


def _same_tally(q, q2, base, rtol=1e-11):
    assert np.allclose(q, base["q"], rtol=rtol, atol=1e-14)
    assert np.allclose(q2, base["q2"], rtol=rtol, atol=1e-14)


@pytest.mark.parametrize("precision", [0, 1])
def test_cancel_then_resume_equals_the_uninterrupted_run(precision):
    """A cancel requested before the run is honoured at the first completion
    check: admission closes, the histories already started finish and are
    tallied, and the run reports the watermark.  Running the rest gives the
    uninterrupted run.  A small bank (population target 4096) and 8 steps per
    visit keep the first batch of iterations from admitting every history."""
    mcx = _mcx()
    wl = W.workload("hetero_broad_64", 20000)
    n = 20000
    launch = (16384, 256, 8)
    base = _base(wl, n, precision, launch)
    sim = mcx.Simulator(precision, 0).setup(wl)
    sim.set_launch(*launch)
    sim.set_test_mode(True)
    sim.cancel()
    with pytest.raises(mcx.MCXCancelled) as ei:
        sim.run(wl["seed"], 0, n)
    w = ei.value.next_history
    print("cancelled at", w, "of", n)
    assert 0 < w < n
    st = sim.stats()
    assert st["histories"] == w and st["next_history"] == w
    h1 = sim.history_results(n)[0]
    assert not h1[w:].any()  # no history after the watermark started
    assert np.array_equal(h1[:w], base["hash"][:w])
    sim.run(wl["seed"], w, n - w)  # the request was consumed: this run completes
    h2 = sim.history_results(n - w)[0]
    assert np.array_equal(np.concatenate([h1[:w], h2]), base["hash"])
    q, q2 = sim.tally()
    _same_tally(q, q2, base)
    st = sim.stats()
    assert st["histories"] == n and st["next_history"] == n
    for k in ("flights", "esteps", "crossings", "deposits", "secondaries"):
        assert st[k] == base["stats"][k], k
    sim.close()


def test_cancel_from_another_thread_then_resume():
    """mcx_cancel called from a second host thread while mcx_run transports
    1e7 histories (mixed precision; a bank of 2^20 records admits them over
    some 40 iterations): the run stops early, and the tallies of the stopped
    run plus the rest equal one uninterrupted run."""
    mcx = _mcx()
    wl = W.workload("hetero_broad_64", 10_000_000)
    n = 10_000_000
    launch = (1 << 20, 256, 128)
    sim = mcx.Simulator(mcx.MIXED, 0).setup(wl)
    sim.set_launch(*launch)
    sim.run(wl["seed"], 0, 1000)  # allocate the run memory outside the race
    sim.reset()
    t = threading.Timer(0.02, sim.cancel)
    t.start()
    try:
        sim.run(wl["seed"], 0, n)
        w = n
    except mcx.MCXCancelled as e:
        w = e.next_history
    t.join()
    print("cancelled at", w, "of", n)
    if w == n:
        sim.close()
        pytest.skip("the run ended before the cancel request")
    assert 0 < w < n
    assert sim.stats()["histories"] == w
    sim.run(wl["seed"], w, n - w)
    q, q2 = sim.tally()
    sim.close()
    base = _base(wl, n, mcx.MIXED, launch, test=False)
    _same_tally(q, q2, base, rtol=1e-10)


def test_checkpoint_restore_resumes_in_a_new_context():
    """Half the histories in one context, checkpoint, the other half in a new
    context restored from it: the same tallies, history count and event
    counters as one run.  A damaged, truncated or mismatched checkpoint is
    refused; the gradient needs a run of its own context."""
    mcx = _mcx()
    wl = W.workload("hetero_broad_64", 6000)
    n, half = 6000, 2500
    launch = (1 << 20, 256, 128)
    base = _base(wl, n, 0, launch, test=False)
    s1 = mcx.Simulator(0, 0).setup(wl)
    s1.set_launch(*launch)
    s1.run(wl["seed"], 0, half)
    ck = s1.checkpoint()
    st1 = s1.stats()
    d1, _ = s1.dose()
    s1.close()
    nv = 64 ** 3
    assert len(ck) > 16 * nv

    s2 = mcx.Simulator(0, 0).setup(wl)
    s2.set_launch(*launch)
    s2.restore(ck)
    st2 = s2.stats()
    for k in ("histories", "next_history", "flights", "esteps", "deposits", "e_dep"):
        assert st2[k] == st1[k], k
    d2, _ = s2.dose()
    assert np.array_equal(d1, d2)
    s2.run(wl["seed"], half, n - half)
    q, q2 = s2.tally()
    _same_tally(q, q2, base)
    st = s2.stats()
    assert st["histories"] == n
    for k in ("flights", "esteps", "crossings", "deposits"):
        assert st[k] == base["stats"][k], k
    with pytest.raises(mcx.MCXError):
        s2.dose_backward(np.zeros((64, 64, 64)))
    bad = bytearray(ck)
    bad[len(bad) // 2] ^= 1
    with pytest.raises(mcx.MCXError):
        s2.restore(bytes(bad))
    with pytest.raises(mcx.MCXError):
        s2.restore(ck[:-8])
    s2.close()
    s3 = mcx.Simulator(mcx.MIXED, 0).setup(wl)
    with pytest.raises(mcx.MCXError):
        s3.restore(ck)  # another precision
    s3.close()


def test_run_in_caller_owned_workspace():
    """Queues, counters and a 2^22-slot tally table carved from a torch
    tensor give the histories and tallies of library-owned memory; a
    workspace too small for the bank is refused, and the context returns to
    its own memory."""
    import torch
    mcx = _mcx()
    wl = W.workload("hetero_broad_64", 4000)
    n = 4000
    launch = (1 << 20, 256, 128)
    base = _base(wl, n, 0, launch)
    sim = mcx.Simulator(0, 0).setup(wl)
    sim.set_launch(*launch)
    sim.set_test_mode(True)
    full = sim.workspace_size()
    fixed = full - (1 << 29) * 16
    assert fixed > 8 * (1 << 20) * 80  # eight queues of 2^20 records
    ws = torch.empty(fixed + (1 << 22) * 16 + 4096, dtype=torch.uint8, device="cuda:0")
    sim.set_workspace(ws)
    sim.run(wl["seed"], 0, n)
    h = sim.history_results(n)[0]
    assert np.array_equal(h, base["hash"])
    q, q2 = sim.tally()
    _same_tally(q, q2, base)
    small = torch.empty(fixed // 2, dtype=torch.uint8, device="cuda:0")
    with pytest.raises(mcx.MCXError):
        sim.set_workspace(small)
    assert sim.stats()["esteps"] == base["stats"]["esteps"]  # kept across the change
    sim.reset()
    sim.run(wl["seed"], 0, n)
    q, q2 = sim.tally()
    _same_tally(q, q2, base)
    sim.set_workspace(ws)
    sim.set_launch(1 << 21, 0, 0)  # the queues no longer fit with a table of 2^20 slots
    with pytest.raises(mcx.MCXError):
        sim.run(wl["seed"], 0, n)
    sim.set_workspace(None)
    sim.close()
    del ws, small


def test_setup_changes_after_a_run_invalidate_the_gradient_replays():
    """The gradient replays the last run's histories with the context's
    physics: once the transport parameters, a material or the sources change
    after the run, the replays would run other physics or other histories,
    so mcx_dose_backward refuses with MCX_E_STATE until a new run."""
    mcx = _mcx()
    wl = W.workload("water_pencil_32", 2000)
    g = np.zeros((32, 32, 32))
    for change in ("transport", "material", "sources"):
        sim = mcx.Simulator(0, 0).setup(wl)
        sim.run(wl["seed"], 0, 2000)
        sim.dose_backward(g)  # valid right after the run
        if change == "transport":
            sim.set_transport(dict(wl["transport"], flags=mcx.ANNIH_FLIGHT))
            sim.load_material(wl["material"], 0)
        elif change == "material":
            sim.load_material(wl["material"], 0)
        else:
            sim.set_sources(wl["sources"])
        with pytest.raises(mcx.MCXError, match="STATE"):
            sim.dose_backward(g)
        sim.reset()
        sim.run(wl["seed"], 0, 2000)
        sim.dose_backward(g)
        sim.close()


def test_rejected_phantom_load_leaves_no_phantom():
    """A phantom with a material index >= 4 or a non-positive density is
    rejected by the host checks, which all run before any device state
    changes: the previous phantom, its tallies and its run (for the gradient)
    stay intact and usable."""
    mcx = _mcx()
    wl = W.workload("water_pencil_32", 2000)
    sim = mcx.Simulator(0, 0).setup(wl)
    sim.run(wl["seed"], 0, 2000)
    q0, _ = sim.tally()
    bad = dict(wl["phantom"], mat=np.full((32, 32, 32), 7, dtype=np.uint8))
    with pytest.raises(mcx.MCXError, match="INVALID"):
        sim.load_phantom(bad)
    # validated on the host first: the old phantom, tallies and run are intact
    q1, _ = sim.tally()
    assert np.array_equal(q0, q1)
    sim.dose_backward(np.zeros((32, 32, 32)))
    neg = dict(wl["phantom"], rho=-np.ones((32, 32, 32)))
    with pytest.raises(mcx.MCXError, match="INVALID"):
        sim.load_phantom(neg)
    sim.reset()
    sim.run(wl["seed"], 0, 2000)
    q2, _ = sim.tally()
    assert np.array_equal(q0 > 0, q2 > 0) and np.allclose(q0, q2, rtol=1e-11, atol=1e-14)
    sim.close()
