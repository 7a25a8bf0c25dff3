"""Benchmark of the particle-history loop on one MI355X.

Workload: 6 MeV photons, 10 x 10 cm parallel field on a 128^3 heterogeneous
phantom of 2 mm voxels (water, lung slab, 8 bone spheres), 1e7 histories per
step; FP32 physics with FP64 positions/tallies ("mixed") is the headline, the
FP64 path is timed on the same steps and the same random streams beside it.

A step is one whole transport of the step's histories (source, photon
flights and interactions, Class II electron/positron steps, tally flush);
inputs are resident in HBM before the timed region starts.

Prints one JSON line with the metric, the mixed-vs-FP64 comparison (speed-up
and high-dose deviation), the roofline of the dominant kernel, the Class II
step, for the mixed path, the FP64 path and the gradient's replays (each
measured live with HIP events recorded around each launch on the run's
stream), and the oracle timed on a bounded sample on the host CPU.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# VALU issue ceiling: 256 CUs x 4 SIMDs, a wave64 VALU instruction occupies a
# 16-lane SIMD for 4 cycles, 2.4 GHz -> 256 * 2.4e9 wave-instructions/s
VALU_ISSUE_PEAK = 256 * 4 / 4 * 2.4  # G wave-instructions/s
COUNTERS = os.path.join(ROOT, "profiles", "k_estep_counters_hetero_broad_128.json")


def kernel_source_digest() -> str:
    h = hashlib.sha256()
    for f in ("transport_kernels.h", "transport_device.h", "mcx_internal.h"):
        with open(os.path.join(ROOT, "paper_2003_00796_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def estep_algorithmic_bytes(st: dict, fp64: bool) -> float:
    """Bytes the Class II step kernel must move by its algorithm: each e+-
    record read and written (positions 3 x f64, direction and energy 4 x T,
    uid u64, history/counter/voxel/flags 4 x u32), one density per step, and
    per tally insertion the key (load + compare-and-swap) and the score
    (atomic read-modify-write)."""
    t = 8 if fp64 else 4
    rec = 3 * 8 + 4 * t + 8 + 4 * 4
    return st["evisits"] * rec + st["ewrites"] * rec + st["esteps"] * t + st["inserts"] * 32


def high_dose_deviation(d_mix: np.ndarray, d_64: np.ndarray) -> dict:
    hi = d_64 >= 0.5 * d_64.max()
    rel = (d_mix[hi] - d_64[hi]) / d_64[hi]
    return dict(voxels=int(hi.sum()), rms=float(np.sqrt(np.mean(rel ** 2))), max=float(np.max(np.abs(rel))),
                sum_ratio=float(d_mix.sum() / d_64.sum()))


def depth_dose(d: np.ndarray) -> np.ndarray:
    """Dose summed over each depth plane (z is the first axis)."""
    return d.reshape(d.shape[0], -1).sum(axis=1)


def paired_deviation(d_mix: list, d_64: list, frac: float = 0.5) -> dict:
    """Mixed against FP64 on the same streams, K batches (one per seed):
    the deviation Delta_b = D_mix,b - D_64,b of each batch splits into a
    systematic part, the mean over batches, and a statistical part (the few
    histories whose FP32 rounding took another branch), whose size the
    batch-to-batch spread measures.  Over the voxels with D_64 >= frac of the
    maximum: the mean relative shift with its standard error; the RMS of the
    per-voxel mean shift and the RMS its noise alone would give; the
    systematic RMS that remains, sqrt(max(0, rms^2 - noise^2)); the same
    for the depth-dose curve (dose summed over each plane, planes above half
    its maximum)."""
    k = len(d_mix)
    dm = np.array([a - b for a, b in zip(d_mix, d_64)])
    d64 = np.mean(d_64, axis=0)
    hi = d64 >= frac * d64.max()
    rel = dm[:, hi] / d64[hi]
    out = dict(batches=k, voxel_threshold=frac, voxels=int(hi.sum()), per_batch_rms=float(np.sqrt(np.mean(rel ** 2))))
    if k < 2:
        return out
    mean_v = rel.mean(axis=0)
    se_v = rel.std(axis=0, ddof=1) / np.sqrt(k)
    shift_b = rel.mean(axis=1)  # each batch's mean relative shift over the set
    rms = float(np.sqrt(np.mean(mean_v ** 2)))
    noise = float(np.sqrt(np.mean(se_v ** 2)))
    pdd = np.array([depth_dose(a) - depth_dose(b) for a, b in zip(d_mix, d_64)])
    p64 = depth_dose(d64)
    ph = p64 >= 0.5 * p64.max()
    prel = pdd[:, ph] / p64[ph]
    pm, pse = prel.mean(axis=0), prel.std(axis=0, ddof=1) / np.sqrt(k)
    prms, pnoise = float(np.sqrt(np.mean(pm ** 2))), float(np.sqrt(np.mean(pse ** 2)))
    out.update(mean_shift=float(shift_b.mean()), mean_shift_se=float(shift_b.std(ddof=1) / np.sqrt(k)),
               rms_of_mean=rms, rms_noise=noise, systematic_rms=float(np.sqrt(max(0.0, rms ** 2 - noise ** 2))),
               z_mean=float(np.mean(mean_v / np.where(se_v > 0, se_v, np.inf))),
               depth_planes=int(ph.sum()), depth_rms_of_mean=prms, depth_rms_noise=pnoise,
               depth_systematic_rms=float(np.sqrt(max(0.0, prms ** 2 - pnoise ** 2))),
               depth_max=float(np.max(np.abs(pm))))
    return out


def load_counters():
    """The counters file, if it was taken on the current kernel source."""
    if not os.path.exists(COUNTERS):
        return None
    with open(COUNTERS) as fh:
        prof = json.load(fh)
    return prof if prof.get("kernel_source_digest") == kernel_source_digest() else None


def roofline(st: dict, fp64: bool = False) -> dict:
    """Roofline of the Class II step kernel k_estep (the dominant kernel) over
    the timed launches, mixed (FP32 physics) or FP64.  The step is bound by
    VALU issue: `achieved` is the VALU wave-instructions per e+- step counted
    by the hardware counters for this kernel source, times the steps of a
    launch (counted live), over the launch time measured with HIP events.
    The HBM view beside it uses the algorithmic bytes and the counted
    traffic."""
    launches = st["timed_iterations"]
    if not launches:
        return None
    avg_s = st["ms_estep"] / launches * 1e-3
    esteps = st["esteps"] / launches
    alg = estep_algorithmic_bytes(st, fp64=fp64) / launches
    hbm = {"algorithmic_bytes_per_launch": alg, "achieved": alg / avg_s / 1e9, "peak": HBM_PEAK_GBS, "unit": "GB/s",
           "frac": alg / avg_s / 1e9 / HBM_PEAK_GBS}
    prof = load_counters()
    out = {"kernel": "k_estep<double>" if fp64 else "k_estep<float>", "avg_launch_ms": avg_s * 1e3,
           "launches": launches, "esteps_per_launch": esteps}
    if prof is None:  # counters taken on another kernel source: the HBM view alone
        out.update(bound="hbm", achieved=hbm["achieved"], peak=HBM_PEAK_GBS, unit="GB/s", frac=hbm["frac"],
                   traffic=None)
        return out
    kp = prof["fp64_k_estep"] if fp64 else prof
    wi = kp["valu_wave_instr_per_estep"] * esteps
    traffic = kp["hbm_bytes_per_estep"] * esteps
    hbm["traffic_GBs"] = traffic / avg_s / 1e9
    out.update(bound="alu", achieved=wi / avg_s / 1e9, peak=VALU_ISSUE_PEAK, unit="G VALU wave-instr/s",
               frac=wi / avg_s / 1e9 / VALU_ISSUE_PEAK, traffic=traffic,
               valu_wave_instr_per_estep=kp["valu_wave_instr_per_estep"],
               valu_lane_utilisation=kp["valu_lane_utilisation"], hbm=hbm)
    if not fp64:
        out["valu_lane_utilisation_per_kernel"] = {k: v["lane_utilisation"] for k, v in
                                                   prof.get("valu_lane_utilisation_per_kernel", {}).items()}
    return out


def replay_roofline(ms_estep: float, launches: int, esteps_forward: int) -> dict:
    """Roofline of the gradient's two replays of k_estep (FP64): the VALU
    wave-instructions the counters give per forward e+- step for replay A and
    for replay B (look-ahead and pass), times the forward steps, over the
    replays' k_estep time measured with HIP events."""
    prof = load_counters()
    if prof is None or not launches or not ms_estep > 0.0:
        return None
    rp = prof["gradient_replays"]
    per_step = sum(v["valu_wave_instr_per_forward_step"] for k, v in rp.items() if k.startswith("replay"))
    achieved = per_step * esteps_forward / (ms_estep * 1e-3) / 1e9
    return {"kernel": "k_estep<double> replays A + B", "bound": "alu", "k_estep_ms": ms_estep,
            "launches": launches, "valu_wave_instr_per_forward_step": per_step, "achieved": achieved,
            "peak": VALU_ISSUE_PEAK, "unit": "G VALU wave-instr/s", "frac": achieved / VALU_ISSUE_PEAK,
            "valu_lane_utilisation": {k: v["valu_lane_utilisation"] for k, v in rp.items()}}


def target_detector_efficiency(mcx, W, sync, args, n: int = 1_000_000) -> dict:
    """Efficiency 1/(sigma^2 T) of the energy deposited in the first 0.5 cm
    detector layer behind the target (reached by bremsstrahlung photons
    only), forced over analog, mixed precision, one run of n histories each."""
    wl = W.workload("target_detector", n)
    res = {}
    for key, t in (("analog", wl["transport"]),
                   ("forced", dict(wl["transport"], force_in=args.forcing[0], force_br=args.forcing[1],
                                   split_br=args.split_br))):
        sim = mcx.Simulator(mcx.MIXED, 0).setup(dict(wl, transport=t))
        sim.set_launch(args.bank, 256, 128)  # forced emissions: tens of photons per history
        run_steps(sim, n, [91], sync)
        tt = run_steps(sim, n, [92], sync)[0]
        q, q2 = sim.tally()
        sim.close()
        det_q, det_q2 = q[23], q2[23]
        # variance of the mean energy per history in the first detector
        # layer (Eq. (2) of the paper: histories are independent)
        var = (det_q2 / n - (det_q / n) ** 2) / n
        res[key] = dict(seconds=tt, mean_mev=det_q / n, var=var)
    eff = (res["analog"]["var"] * res["analog"]["seconds"]) / (res["forced"]["var"] * res["forced"]["seconds"])
    return dict(workload="target_detector: 2 MeV e- pencil, 1.5 cm water target, 10 cm air, 2 cm water detector",
                histories=n, analog=res["analog"], forced=res["forced"], efficiency_gain=float(eff))


def progress(msg: str) -> None:
    """One line per finished leg on stderr (the JSON line stays on stdout)."""
    print(f"[bench {time.strftime('%H:%M:%S')}] {msg}", file=sys.stderr, flush=True)


def run_steps(sim, n, seeds, sync, doses=None, time_last=False):
    """One timed run per seed (tallies reset before each); with `doses`, each
    step's dose is appended to it after the timed region.  With `time_last`
    the last run records HIP events around its kernel launches, which the
    roofline reads (the statistics cover the last run alone); the other runs
    replay their batches of iterations as graphs, as untimed runs do (a run
    with events launches its kernels one by one)."""
    times = []
    for i, s in enumerate(seeds):
        sim.reset()
        if time_last and i == len(seeds) - 1:
            sim.set_timing(True)
        sync()
        t0 = time.perf_counter()
        sim.run(s, 0, n)
        sync()
        times.append(time.perf_counter() - t0)
        if doses is not None:
            doses.append(sim.dose()[0])
    return times


def smooth_target(d: np.ndarray) -> np.ndarray:
    """T_v = Dbar (0.5 + s_v): s is Gaussian-smoothed (sigma = 3 voxels) white
    noise (PCG64 seed 5) scaled to [0, 1]; Dbar the mean dose over the
    voxels with D >= 10% of the maximum."""
    from scipy.ndimage import gaussian_filter
    rng = np.random.Generator(np.random.PCG64(5))
    s = gaussian_filter(rng.standard_normal(d.shape), 3.0)
    s = (s - s.min()) / (s.max() - s.min())
    dbar = d[d >= 0.1 * d.max()].mean()
    return dbar * (0.5 + s)


def gradient_timing(mcx, W, sync, n: int = 10_000_000) -> dict:
    """Forward + backward (two replays) on the 64^3 heterogeneous phantom,
    6 MeV field, loss sum_v (D_v - T_v)^2 with a seeded smooth target.  The
    reported times are those of the graph-replayed launches; the backward is
    then repeated with per-kernel HIP events for the replays' roofline."""
    wl = W.workload("hetero_broad_64", n)
    sim = mcx.Simulator(mcx.FP64, 0).setup(wl)
    sim.run(777, 0, min(n, 200_000))  # warm-up
    sim.dose_backward(np.zeros(wl["phantom"]["shape"]))
    sim.reset()
    sync()
    t0 = time.perf_counter()
    sim.run(1, 0, n)
    d, _ = sim.dose()
    sync()
    t1 = time.perf_counter()
    esteps = sim.stats()["esteps"]
    target = smooth_target(d)  # built outside the timed intervals
    dl = 2.0 * (d - target)
    sync()
    t2 = time.perf_counter()
    g = sim.dose_backward(dl)
    sync()
    t3 = time.perf_counter()
    # the same replays with events around every launch (not graph-replayed);
    # the kernel times add up over them
    sim.set_timing(True)
    st0 = sim.stats()
    sim.dose_backward(dl)
    sync()
    st1 = sim.stats()
    sim.close()
    ms = st1["ms_estep"] - st0["ms_estep"]
    return dict(workload="hetero_broad_64: 6 MeV 10x10 field, 64^3 x 4 mm, FP64", histories=n,
                forward_s=t1 - t0, backward_s=t3 - t2, fwd_bwd_s=(t1 - t0) + (t3 - t2),
                grad_abs_max=float(np.abs(g).max()), esteps_forward=esteps, replay_k_estep_ms=ms,
                roofline=replay_roofline(ms, st1["timed_iterations"] - st0["timed_iterations"], esteps),
                target=target)


def gradient_fd_check(mcx, W, sync, target, n_batch: int = 1_000_000, batches: int = 10, n_vox: int = 16,
                      h: float = 0.01, transport: dict | None = None) -> dict:
    """The replay gradient against common-random-number central differences
    on the same workload: 16 voxels drawn (PCG64 seed 6) among those inside
    the field with D >= 10% of the maximum; each batch b (seed 100 + b,
    histories [0, n_batch)) gives one replay gradient and, for each voxel,
    (L(rho + h rho_j) - L(rho - h rho_j)) / (2 h rho_j) with the same seed
    and histories; L = sum_v (D_v - T_v)^2 with the target frozen.  Means and
    standard errors over the batches.  Both estimators of the replay are
    taken from the same runs: the default one and the one with the soft
    deflection's energy term (term E)."""
    wl = W.workload("hetero_broad_64", n_batch)
    if transport is not None:
        wl["transport"] = transport
    ph = wl["phantom"]
    sim = mcx.Simulator(mcx.FP64, 0).setup(wl)
    sim.run(99, 0, n_batch)
    d0, _ = sim.dose()
    sim.reset()
    nz, ny, nx = ph["shape"]
    dx = ph["voxel"][0]
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    xc = (x + 0.5) * dx + ph["origin"][0]
    yc = (y + 0.5) * dx + ph["origin"][1]
    src = wl["sources"][0]
    inside = (np.abs(xc - src["pos"][0]) < 0.5 * src["width"][0] - dx) & \
             (np.abs(yc - src["pos"][1]) < 0.5 * src["width"][1] - dx)
    elig = np.argwhere(inside & (d0 >= 0.1 * d0.max()))
    pick = elig[np.random.Generator(np.random.PCG64(6)).choice(len(elig), size=n_vox, replace=False)]
    vox = [tuple(int(c) for c in v) for v in pick]
    est = np.zeros((batches, n_vox))
    est_e = np.zeros((batches, n_vox))
    t0 = time.perf_counter()
    t_e = 0.0
    for b in range(batches):
        sim.reset()
        sim.run(100 + b, 0, n_batch)
        d, _ = sim.dose()
        sim.set_gradient(0)
        g = sim.dose_backward(2.0 * (d - target))
        est[b] = [g[v] for v in vox]
        sync()
        t1 = time.perf_counter()
        sim.set_gradient(mcx.GRAD_DEFLECTION_ENERGY)
        g = sim.dose_backward(2.0 * (d - target))
        est_e[b] = [g[v] for v in vox]
        sync()
        t_e += time.perf_counter() - t1
    t_grad = time.perf_counter() - t0 - t_e
    fd = np.zeros((batches, n_vox))
    t0 = time.perf_counter()
    for k, v in enumerate(vox):
        sims = {}
        for sg in (1, -1):
            rho = ph["rho"].copy()
            rho[v] *= 1.0 + sg * h
            sims[sg] = mcx.Simulator(mcx.FP64, 0).setup(dict(wl, phantom=dict(ph, rho=rho)))
        for b in range(batches):
            vals = {}
            for sg, sm in sims.items():
                sm.reset()
                sm.run(100 + b, 0, n_batch)
                d, _ = sm.dose()
                vals[sg] = float(((d - target) ** 2).sum())
            fd[b, k] = (vals[1] - vals[-1]) / (2.0 * h * ph["rho"][v])
        for sm in sims.values():
            sm.close()
        progress(f"finite differences: voxel {k + 1} of {n_vox}")
    t_fd = time.perf_counter() - t0
    sim.close()
    sync()
    f, fse = fd.mean(0), fd.std(0, ddof=1) / np.sqrt(batches)

    def versus_fd(e):
        m, se = e.mean(0), e.std(0, ddof=1) / np.sqrt(batches)
        zz = (m - f) / np.sqrt(se ** 2 + fse ** 2)
        return dict(replay=m.tolist(), replay_se=se.tolist(), replay_batches=e.tolist(), z=zz.tolist(),
                    z_mean=float(zz.mean()), z_rms=float(np.sqrt((zz ** 2).mean())), z_max=float(np.abs(zz).max()),
                    chi2=float((zz ** 2).sum()), median_rel_se=float(np.median(se / np.abs(m))))

    out = dict(voxels=vox, fd=f.tolist(), fd_se=fse.tolist(), fd_batches=fd.tolist(), dof=n_vox,
               h=h, batches=batches, histories_per_batch=n_batch, replay_s=t_grad, replay_term_e_s=t_e, fd_s=t_fd)
    out.update(versus_fd(est))
    out["with_deflection_energy_term"] = versus_fd(est_e)
    return out


def beamlet_comparison(mcx, W, sync, total: int, cache: str) -> dict:
    """512 beamlets with lognormal history counts in one autotuned run (a
    batch of iterations is one HIP graph launch) against one run per beamlet."""
    wl = W.workload("beamlets_256", total)
    sim = mcx.Simulator(mcx.MIXED, 0).setup(wl)
    t0 = time.perf_counter()
    chosen = sim.autotune(200_000, cache)
    t_tune = time.perf_counter() - t0
    sim.run(999, 0, 200_000)
    sim.reset()
    sync()
    t0 = time.perf_counter()
    sim.run(1, 0, sim.n_hist_total)
    sync()
    t_batched = time.perf_counter() - t0
    d_all, _ = sim.dose()
    # the same run with the per-beamlet dose-influence output
    sim.set_influence(True, 30)
    sim.reset()
    sync()
    t0 = time.perf_counter()
    sim.run(1, 0, sim.n_hist_total)
    sync()
    t_infl = time.perf_counter() - t0
    n_entries = sim.influence_count()
    sim.set_influence(False)
    sim.reset()
    sync()
    t0 = time.perf_counter()
    first = 0
    for src in wl["sources"]:
        sim.run(1, first, src["n_hist"])
        first += src["n_hist"]
    sync()
    t_each = time.perf_counter() - t0
    d_each, _ = sim.dose()
    sim.close()
    hi = d_all >= 0.5 * d_all.max()
    return dict(workload="beamlets_256: 512 beamlets 4-15 MeV, lognormal counts, 256^3 x 2 mm noise phantom, mixed",
                histories=int(sum(x["n_hist"] for x in wl["sources"])), autotuned=dict(zip(("bank", "block", "steps"), chosen)),
                autotune_s=t_tune, batched_s=t_batched, per_beamlet_s=t_each,
                batched_with_influence_s=t_infl, influence_entries=n_entries,
                batched_hist_per_s=sum(x["n_hist"] for x in wl["sources"]) / t_batched,
                speedup=t_each / t_batched,
                same_dose_rel_max=float(np.max(np.abs(d_all[hi] - d_each[hi]) / d_all[hi])))


def _oracle_shard(args):
    """One history range of the workload through the oracle (own process)."""
    name, first, n = args
    import oracle as O
    import workloads as W
    wl = W.workload(name)
    tb = O.Tables(wl["material"], wl["transport"])
    t0 = time.perf_counter()
    O.run(tb, wl["phantom"], wl["sources"], wl["seed"], first, n)
    return time.perf_counter() - t0


def host_cpu() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(name: str, n_per_proc: int, procs: int, repeats: int = 3, stride: int | None = None) -> dict:
    """The oracle on the host cores, sharded by history range over `procs`
    processes (independent histories, as the paper's multi-process runs): the
    rate is the histories over the slowest shard's time (setup excluded),
    the median of `repeats` repetitions.  Shard k starts at history
    k * stride (default: contiguous shards)."""
    import concurrent.futures as cf
    import multiprocessing as mp
    step = stride or n_per_proc
    jobs = [(name, k * step, n_per_proc) for k in range(procs)]
    rates, singles, slow, work = [], [], [], []
    with cf.ProcessPoolExecutor(max_workers=procs, mp_context=mp.get_context("spawn")) as ex:
        for _ in range(repeats):
            times = list(ex.map(_oracle_shard, jobs))
            rates.append(procs * n_per_proc / max(times))
            singles.append(n_per_proc / (sum(times) / len(times)))
            slow.append(max(times))
            work.append(sum(times))
    i = int(np.argsort(rates)[len(rates) // 2])
    return dict(value=rates[i], unit="histories/s", cores=procs, kind="oracle", host_cpu=host_cpu(),
                host_logical_cpus=os.cpu_count(), single_core=float(np.median(singles)), repeats=repeats,
                sample=(f"histories [0, {procs * n_per_proc})" if step == n_per_proc else
                        f"{procs} ranges of {n_per_proc} histories spaced {step} apart") +
                       f" of the same workload in {procs} single-thread FP64 "
                       f"oracle processes of {n_per_proc} histories each, median of {repeats} repetitions "
                       f"({slow[i]:.1f} s the slowest shard, {work[i]:.0f} s of CPU work)")


def cpu_baseline_configs(procs: int) -> dict:
    """The oracle on the other workloads, the same way: the 1 MeV photon
    pencil in full (1e5 histories), and bounded samples of the 20 MeV
    electron pencil, the 512 beamlets (ranges spread over all 5e7 history
    ids, so beamlets enter by their history counts) and the 64^3 gradient
    field."""
    import workloads as W
    out = {}
    n_beam = sum(s["n_hist"] for s in W.beamlet_sources())
    for name, n, stride in (("water_pencil_32", 100_000 // procs, None), ("electron_200", 600, None),
                            ("beamlets_256", 3000, n_beam // procs), ("hetero_broad_64", 6000, None)):
        r = cpu_baseline(name, n, procs, stride=stride)
        out[name] = {k: r[k] for k in ("value", "single_core", "sample")}
        progress(f"oracle on {name}: {r['value']:.4g} histories/s on {procs} processes")
    return out


def small_config_rates(mcx, W, sync, steps: int = 5) -> dict:
    """GPU rates of the 1 MeV photon pencil (1e5 histories, 32^3): FP64 and
    mixed, `steps` timed runs after one warm-up."""
    wl = W.workload("water_pencil_32")
    n = wl["sources"][0]["n_hist"]
    out = {}
    for key, prec in (("fp64", mcx.FP64), ("mixed", mcx.MIXED)):
        sim = mcx.Simulator(prec, 0).setup(wl)
        run_steps(sim, n, [500], sync)
        t = run_steps(sim, n, list(range(1, steps + 1)), sync)
        sim.close()
        out[key] = dict(value=n * len(t) / sum(t), ms=1e3 * sum(t) / len(t))
    out["workload"] = "water_pencil_32: 1 MeV photon pencil, 32^3 x 6.25 mm water, 1e5 histories"
    return out


def electron_comparison(mcx, W, sync, n: int = 1_000_000, batches: int = 4) -> dict:
    """20 MeV electron pencil on a 200^3 x 1 mm water cube: mixed and FP64 on
    the same streams, `batches` runs of n histories each.  A pencil's dose
    has few voxels near its maximum, so the high-dose sets are the voxels
    with D >= 10% of the maximum and the depth-dose planes above half the
    depth-dose maximum."""
    wl = W.workload("electron_200", n)
    out = {}
    doses = {}
    seeds = [1 + i for i in range(batches)]
    for name, prec in (("mixed", mcx.MIXED), ("fp64", mcx.FP64)):
        sim = mcx.Simulator(prec, 0).setup(wl)
        sim.run(777, 0, min(n, 100_000))
        doses[name] = []
        t = run_steps(sim, n, seeds, sync, doses[name])
        sim.close()
        out[name] = dict(value=n * len(t) / sum(t), ms=1e3 * sum(t) / len(t))
    out["mixed_over_fp64"] = out["mixed"]["value"] / out["fp64"]["value"]
    pd = paired_deviation(doses["mixed"], doses["fp64"], frac=0.1)
    dm, d6 = np.mean(doses["mixed"], axis=0), np.mean(doses["fp64"], axis=0)
    hi = d6 >= 0.1 * d6.max()
    rel = (dm[hi] - d6[hi]) / d6[hi]
    out["deviation"] = dict(paired=pd, voxels_above_10pct=int(hi.sum()),
                            voxel_rms_above_10pct=float(np.sqrt(np.mean(rel ** 2))),
                            sum_ratio=float(dm.sum() / d6.sum()))
    out["workload"] = f"electron_200: 20 MeV e- pencil, 200^3 x 1 mm water, {batches} x {n} histories"
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--hist", type=int, default=10_000_000, help="histories per step")
    ap.add_argument("--cpu-sample", type=int, default=6_000, help="oracle histories per host process")
    # the host share of a one-GPU benchmark node is 16 cores, whatever os.cpu_count() reports
    ap.add_argument("--cpu-procs", type=int, default=16, help="oracle processes (host cores used)")
    ap.add_argument("--no-cpu-configs", action="store_true", help="time the oracle on the benchmark workload only")
    ap.add_argument("--no-electron", action="store_true", help="skip the 20 MeV electron workload")
    ap.add_argument("--straggling", action="store_true",
                    help="also time the mixed step with soft energy-loss straggling on")
    ap.add_argument("--materials", action="store_true",
                    help="also time the mixed step on the same phantom with bone spheres of a second material")
    ap.add_argument("--annih-flight", action="store_true",
                    help="also time the mixed step with positron annihilation in flight on")
    ap.add_argument("--forcing", type=float, nargs=2, metavar=("F_IN", "F_BR"), default=None,
                    help="also time the workload with interaction forcing of hard collisions and bremsstrahlung")
    ap.add_argument("--split-br", type=int, default=0, choices=(0, 1, 2),
                    help="with --forcing: bremsstrahlung photons per emission")
    ap.add_argument("--no-fp64", action="store_true")
    # records per event queue: 2^26 puts a quarter of it, 16.8 M particles,
    # in flight at once (all histories of a 1e7 step are admitted together)
    ap.add_argument("--bank", type=int, default=1 << 26)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-gradient", action="store_true")
    ap.add_argument("--no-fd-check", action="store_true", help="skip the finite-difference check of the gradient")
    ap.add_argument("--beamlets", type=int, default=50_000_000, metavar="TOTAL",
                    help="512 beamlets with TOTAL histories batched vs one run each (0: skip)")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="BYTES",
                    help="only copy BYTES between two device buffers (calibrates the HBM byte counters)")
    args = ap.parse_args()
    if args.copy_calibration:
        import torch
        n = args.copy_calibration // 4
        x = torch.ones(n, dtype=torch.float32, device="cuda")
        y = torch.empty_like(x)
        for _ in range(3):
            y.copy_(x)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes": n * 4, "launches": 3}))
        return
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); the transport shards by history range "
              "and would need one all-reduce of the tallies, which the single-GPU benchmark does not perform.", file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_2003_00796_amd as mcx
    import workloads as W

    def sync():
        torch.cuda.synchronize()

    torch.cuda.init()
    wl = W.workload("hetero_broad_128", args.hist)
    n = args.hist
    warm_seeds = [1000 + i for i in range(args.warmup)]
    seeds = [1 + i for i in range(args.steps)]

    mix = mcx.Simulator(mcx.MIXED, 0).setup(wl)
    mix.set_launch(args.bank, 256, 128)
    run_steps(mix, n, warm_seeds, sync)
    doses_mix = []
    t_mix = run_steps(mix, n, seeds, sync, doses_mix, time_last=True)
    st = mix.stats()
    d_mix, s_mix = mix.dose()
    mix.close()
    progress(f"mixed: {len(t_mix)} steps, {n * len(t_mix) / sum(t_mix):.4g} histories/s")

    result_64 = None
    if not args.no_fp64:
        f64 = mcx.Simulator(mcx.FP64, 0).setup(wl)
        f64.set_launch(args.bank, 256, 128)
        run_steps(f64, n, warm_seeds, sync)
        doses_64 = []
        t_64 = run_steps(f64, n, seeds, sync, doses_64, time_last=True)
        d_64, _ = f64.dose()
        st_64 = f64.stats()
        f64.close()
        result_64 = dict(value=n * len(t_64) / sum(t_64), ms_per_step=1e3 * sum(t_64) / len(t_64),
                         esteps_per_history=st_64["esteps"] / n, roofline=roofline(st_64, fp64=True))
        dev = high_dose_deviation(d_mix, d_64)
        # the timed steps as paired batches: systematic part and noise floor
        dev["paired_batches"] = paired_deviation(doses_mix, doses_64)
        del doses_mix, doses_64
        progress(f"fp64: {len(t_64)} steps, {result_64['value']:.4g} histories/s")

    value = n * len(t_mix) / sum(t_mix)
    ms = {"k_source": st["ms_source"], "k_flight": st["ms_flight"], "k_knock": st["ms_knock"],
          "k_estep": st["ms_estep"]}
    out = {
        "metric": "histories/s, mixed vs FP64 at matched dose; fwd+bwd density-gradient time",
        "value": value,
        "unit": "histories/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * sum(t_mix) / len(t_mix),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "hetero_broad_128: 6 MeV photon 10x10 cm field, 128^3 x 2 mm phantom "
                               "(water, lung slab 0.26, 8 bone spheres 1.85), mixed precision (FP32 physics, "
                               "FP64 positions and tallies)", "histories_per_step": n, "parallelism": "single GPU",
                   "launch": {"bank": args.bank, "block": 256, "steps": 128}},
        "fp64": result_64,
        "mixed_over_fp64": (value / result_64["value"]) if result_64 else None,
        "high_dose_deviation": dev if result_64 else None,
        # the statistics are those of the last timed step (each step starts
        # from a reset of the tallies and statistics)
        "kernel_ms_per_step": ms,
        "events_per_history": {k: st[k] / n for k in ("flights", "esteps", "crossings", "deposits", "inserts",
                                                      "evisits")},
        "roofline": roofline(st),
    }
    if args.straggling or args.annih_flight:
        extra = (mcx.STRAGGLING if args.straggling else 0) | (mcx.ANNIH_FLIGHT if args.annih_flight else 0)
        t = dict(wl["transport"], flags=wl["transport"].get("flags", 0) | extra)
        sg = mcx.Simulator(mcx.MIXED, 0).setup(dict(wl, transport=t))
        sg.set_launch(args.bank, 256, 128)
        run_steps(sg, n, warm_seeds, sync)
        t_sg = run_steps(sg, n, seeds, sync)
        d_sg, s_sg = sg.dose()
        st_sg = sg.stats()  # the last step's (each step starts from a reset)
        sg.close()
        hi = d_mix >= 0.5 * d_mix.max()
        z = (d_sg[hi] - d_mix[hi]) / np.sqrt(s_sg[hi] ** 2 + s_mix[hi] ** 2)
        out["extended_physics"] = dict(straggling=bool(args.straggling), annih_flight=bool(args.annih_flight),
                                 value=n * len(t_sg) / sum(t_sg), ms_per_step=1e3 * sum(t_sg) / len(t_sg),
                                 esteps_per_history=st_sg["esteps"] / n, annihilations_per_history=st_sg["annih"] / n,
                                 dose_vs_main=dict(high_dose_deviation(d_sg, d_mix), z_rms=float(np.sqrt(np.mean(z ** 2))),
                                                   z_mean=float(np.mean(z))))
    if args.forcing:
        f_in, f_br = args.forcing
        t = dict(wl["transport"], force_in=f_in, force_br=f_br, split_br=args.split_br)
        sf = mcx.Simulator(mcx.MIXED, 0).setup(dict(wl, transport=t))
        sf.set_launch(args.bank, 256, 128)
        run_steps(sf, n, warm_seeds, sync)
        t_f = run_steps(sf, n, seeds, sync)
        d_f, s_f = sf.dose()
        st_f = sf.stats()
        sf.close()
        hi = d_mix >= 0.5 * d_mix.max()
        z = (d_f[hi] - d_mix[hi]) / np.sqrt(s_f[hi] ** 2 + s_mix[hi] ** 2)
        # efficiency 1 / (sigma^2 T) of the high-dose voxels, forced over analog
        eff = (np.mean(s_mix[hi] ** 2) * sum(t_mix)) / (np.mean(s_f[hi] ** 2) * sum(t_f))
        out["interaction_forcing"] = dict(force_in=f_in, force_br=f_br, split_br=args.split_br, value=n * len(t_f) / sum(t_f),
                                          ms_per_step=1e3 * sum(t_f) / len(t_f),
                                          esteps_per_history=st_f["esteps"] / n,
                                          hard_br_per_history=st_f["hard_br"] / n,
                                          high_dose_efficiency_vs_analog=float(eff),
                                          dose_vs_main=dict(z_rms=float(np.sqrt(np.mean(z ** 2))),
                                                            z_mean=float(np.mean(z))))
    if args.forcing:
        out["interaction_forcing"]["target_detector"] = target_detector_efficiency(mcx, W, sync, args)
    if args.materials:
        wm = W.workload("hetero_mm_128", n)
        sm = mcx.Simulator(mcx.MIXED, 0).setup(wm)
        sm.set_launch(args.bank, 256, 128)
        run_steps(sm, n, warm_seeds, sync)
        t_mm = run_steps(sm, n, seeds, sync)
        d_mm, _ = sm.dose()
        st_mm = sm.stats()
        sm.close()
        out["several_materials"] = dict(workload="hetero_mm_128: the same field and phantom, bone spheres of a second "
                                                 "material (synthetic cortical bone)",
                                        value=n * len(t_mm) / sum(t_mm), ms_per_step=1e3 * sum(t_mm) / len(t_mm),
                                        esteps_per_history=st_mm["esteps"] / n,
                                        summed_dose_ratio_to_one_material=float(d_mm.sum() / d_mix.sum()))
    if not args.no_gradient:
        out["gradient"] = gradient_timing(mcx, W, sync)
        target = out["gradient"].pop("target")
        progress(f"gradient: forward + backward {out['gradient']['fwd_bwd_s']:.3f} s")
        if not args.no_fd_check:
            out["gradient"]["fd_check"] = gradient_fd_check(mcx, W, sync, target)
            progress(f"gradient finite-difference check: z_rms {out['gradient']['fd_check']['z_rms']:.3f}")
    if args.beamlets:
        import tempfile
        with tempfile.TemporaryDirectory() as td:
            out["beamlets"] = beamlet_comparison(mcx, W, sync, args.beamlets, os.path.join(td, "autotune.jsonl"))
        progress(f"beamlets: batched {out['beamlets']['batched_s']:.3f} s, one run each {out['beamlets']['per_beamlet_s']:.3f} s")
    if not args.no_electron:
        out["electron"] = electron_comparison(mcx, W, sync)
        progress(f"electrons: mixed {out['electron']['mixed']['value']:.4g}, fp64 {out['electron']['fp64']['value']:.4g} histories/s")
    out["water_pencil"] = small_config_rates(mcx, W, sync)
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline("hetero_broad_128", args.cpu_sample, args.cpu_procs)
        progress(f"oracle on hetero_broad_128: {out['cpu_baseline']['value']:.4g} histories/s")
        if not args.no_cpu_configs:
            out["cpu_baseline"]["other_workloads"] = cpu_baseline_configs(args.cpu_procs)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
