"""Benchmark of the Monte Carlo KBC lattice Boltzmann hot path on one MI355X.

A step is one tick of the whole ensemble: one fused collide-and-stream
launch over every sample (with the double-precision per-sample reductions
fused in on the saved ticks), inputs resident in HBM. The default workload is
the randomized Taylor-Green ensemble of 64 samples at 64^3 in FP32 shifted
populations (Re 1600, projected perturbation, reductions every 50 steps).

Prints one JSON line: aggregate MLUPS, the roofline of the collide-and-stream
kernel (HBM bytes of the algorithm / measured launch time), the measured
bandwidth of a plain copy kernel, the single-sample FP64 step on the same GPU,
and the oracle timed on the host cores.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0     # MI355X HBM3E
# q loads + q stores per node update
BYTES_PER_LUP = {("f32s", 27): 216, ("f64", 27): 432, ("f32s", 19): 152, ("f64", 19): 304}

# sources the collide-and-stream kernel is compiled from (the counter summary
# is valid only for the exact sources it was taken with)
STEP_SOURCES = ["lattice.h", "lbm_device.h", "step_kernel.h", "step_d3q27_f32.hip", "step_d3q27_f64.hip",
                "step_d3q19_f32.hip", "step_d3q19_f64.hip"]


def step_source_hash():
    import hashlib
    h = hashlib.sha256()
    for name in STEP_SOURCES:
        h.update(open(os.path.join(ROOT, "paper_2608_23786_amd", "csrc", name), "rb").read())
    return h.hexdigest()


def counter_traffic(workload):
    """HBM bytes per collide-and-stream launch from the committed counter
    summary, or None when the kernel source changed since it was taken."""
    path = os.path.join(ROOT, "profiles", f"kbc_step_{workload}.traffic.txt")
    if not os.path.exists(path):
        return None
    vals = dict(line.strip().split("=", 1) for line in open(path) if "=" in line and not line.startswith("#"))
    if step_source_hash() != vals.get("kernel_source_sha256"):
        return None
    return int(vals["traffic_bytes_per_launch"])


def build_ensemble(wl, mc, torch):
    samples = []
    for g in wl.groups:
        samples += [mc.Sample(g.n, g.u0, g.re, g.amp, g.project, g.stride)] * g.count
    ens = mc.Ensemble(samples, wl.precision, lattice=wl.lattice)
    ens.init(wl.seed)
    return ens


def cells_per_tick(ens, tick):
    return sum(s.n ** 3 for s in ens.samples if tick % s.stride == 0)


def timed_ticks(ens, torch, ticks, record_every):
    """Run `ticks` ticks from the current state; return (seconds, lattice updates)."""
    t0 = ens.ticks
    lups = sum(cells_per_tick(ens, t0 + k) for k in range(ticks))
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    ens.synchronize()
    ev0.record(ens.stream)
    ens.step(ticks, record_every=record_every)
    ev1.record(ens.stream)
    ens.synchronize()
    return ev0.elapsed_time(ev1) / 1e3, lups


def stream_bandwidth(mc, torch, nbytes=4 << 30, reps=5):
    src = torch.empty(nbytes // 4, dtype=torch.float32, device="cuda").fill_(1.0)
    dst = torch.empty_like(src)
    s = torch.cuda.current_stream()
    mc.stream_copy(dst, src, s)
    torch.cuda.synchronize()
    best = 0.0
    for _ in range(reps):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(s)
        mc.stream_copy(dst, src, s)
        e1.record(s)
        torch.cuda.synchronize()
        best = max(best, 2 * nbytes / (e0.elapsed_time(e1) / 1e3) / 1e9)
    del src, dst
    torch.cuda.empty_cache()
    return best


def kernel_roofline(ens, wl, torch, ticks):
    """Average duration of the collide-and-stream launches (HIP events on the
    ensemble's stream, one pair per launch) and the algorithmic bandwidth."""
    ens.use_graphs(False)
    ens.time_launches(True)
    t0 = ens.ticks
    lups = sum(cells_per_tick(ens, t0 + k) for k in range(ticks))
    ens.step(ticks)
    avg_ms, launches = ens.launch_time()
    ens.time_launches(False)
    ens.use_graphs(True)
    bytes_per_launch = BYTES_PER_LUP[wl.precision, wl.lattice] * lups / launches
    achieved = bytes_per_launch / (avg_ms / 1e3) / 1e9
    return avg_ms, launches, bytes_per_launch, achieved


def launch_sweep(ens, wl, torch, ticks=20):
    """Algorithmic GB/s of the collide-and-stream kernel for every launch shape
    (state is checkpointed and restored around the sweep)."""
    ck = ens.checkpoint()
    keep = ens.get_launch()
    rows = []
    for block in (128, 256, 512, 1024):
        if wl.precision == "f64" and block == 1024:
            continue
        for xcd in (0, 1):
            for buf in (0, 1):
                for nt in (0, 1):
                    ens.set_launch(block, xcd, buf, nt)
                    ens.step(2)
                    avg_ms, _, _, gbs = kernel_roofline(ens, wl, torch, ticks)
                    rows.append({"block": block, "xcd_remap": xcd, "buffer_addressing": buf, "nontemporal": nt,
                                 "avg_ms": round(avg_ms, 5), "GBps": round(gbs, 1)})
                    print(f"[sweep] block {block:4d} xcd {xcd} buf {buf} nt {nt}: {avg_ms:.4f} ms {gbs:.0f} GB/s",
                          file=sys.stderr, flush=True)
    ens.set_launch(*keep)
    ens.restore(ck)
    return rows


def fp64_single(mc, torch, n, u0, re, ticks=200):
    ens = mc.Ensemble([mc.Sample(n, u0, re)], "f64")
    ens.init(0)
    ens.step(20)
    sec, lups = timed_ticks(ens, torch, ticks, 0)
    return lups / sec / 1e6


def fp64_batched(mc, torch, ticks=100):
    """The 64 x 64^3 RTGV ensemble of the default workload in FP64 populations
    (same physics and seed): aggregate MLUPS and the kernel's algorithmic
    bandwidth at 432 B per node update, for comparison with the FP32 path."""
    import dataclasses
    import mc_inputs
    wl = dataclasses.replace(mc_inputs.WORKLOADS["rtgv64x64_f32"], precision="f64")
    ens = build_ensemble(wl, mc, torch)
    tuned = ens.autotune(reps=1)
    ens.step(20)
    sec, lups = timed_ticks(ens, torch, ticks, 0)
    avg_ms, _, _, gbs = kernel_roofline(ens, wl, torch, 20)
    out = {"samples": wl.m, "n": wl.groups[0].n, "ticks": ticks, "MLUPS": round(lups / sec / 1e6, 1),
           "launch": dict(zip(("block", "xcd_remap", "buffer_addressing", "nontemporal"), tuned)),
           "kernel_avg_ms": round(avg_ms, 5), "bytes_per_lup": BYTES_PER_LUP[wl.precision, wl.lattice],
           "kernel_GBps_algorithmic": round(gbs, 1), "kernel_frac_of_peak": round(gbs / HBM_PEAK_GBS, 4)}
    del ens
    torch.cuda.empty_cache()
    return out


def bench_mixed(mc, torch, with_sf=True):
    """Uneven batch 32 x 64^3 + 12 x 128^3 + 4 x 256^3 (strides 16:4:1), 1000
    ticks, FP64 reductions fused every 16 ticks (all samples at equal physical
    time) and, when with_sf, the FP64 structure function of every sample per
    saved tick (one batch of launches per resolution) with the ensemble mean
    and standard deviation of KE and S2 per resolution, both of the state the
    save's record tick reads (the record tick captures its velocity for the
    structure functions). Returns a dict of throughput figures and the last
    save's statistics."""
    import mc_inputs
    wl = mc_inputs.WORKLOADS["mixed48_f32"]
    ens = build_ensemble(wl, mc, torch)
    tuned = ens.autotune(reps=1)
    ens.step(32)
    ticks, every = wl.ticks, wl.save_every
    groups, first = [], 0
    for g in wl.groups:
        groups.append((first, g.count))
        first += g.count
    work = ens._dev_empty((max(int(mc.lib().mclbm_observables_range_work_bytes(ens._ctx, a, c)) for a, c in groups),),
                          torch.uint8)
    if with_sf:
        ens.capture_velocity()   # each save's record tick writes the velocity the observables read
    t0 = ens.ticks
    lups = sum(cells_per_tick(ens, t0 + k) for k in range(ticks))
    ens.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    sf_sec = 0.0
    e0.record(ens.stream)
    saves = 0
    stats = []
    for k in range(0, ticks, every):
        rec = ens.step(min(every, ticks - k), record_every=every)
        saves += 1
        if with_sf:
            # per resolution group: the structure functions, then the ensemble
            # mean and standard deviation of KE and of S2
            stats = []
            for a, c in groups:
                s2, _ = ens.observables_velocity_range(a, c, work=work, structure=True, spectrum=False)
                stats.append((mc.ensemble_moments(rec[0, a:a + c, 4:5], stream=ens.stream),
                               mc.ensemble_moments(s2, stream=ens.stream)))
    e1.record(ens.stream)
    ens.synchronize()
    sec = e0.elapsed_time(e1) / 1e3
    if stats:
        last = {}
        for g, ((ke_m, ke_s), (s2_m, s2_s)) in zip(wl.groups, stats):
            u2 = g.u0 ** 2
            last[f"{g.count}x{g.n}^3"] = {"E_KE": round(float(ke_m[0]) / u2, 8), "sigma_KE": round(float(ke_s[0]) / u2, 8),
                                          "E_S2_r1": round(float(s2_m[0]) / u2, 8),
                                          "sigma_S2_r1": round(float(s2_s[0]) / u2, 8)}
    out = {"workload": wl.name, "ticks": ticks, "saves": saves, "lattice_updates": lups,
           "seconds": round(sec, 4), "MLUPS_including_observables": round(lups / sec / 1e6, 1),
           "launch": dict(zip(("block", "xcd_remap", "buffer_addressing", "nontemporal"), tuned))}
    if stats:
        out["last_save_statistics_u_over_U0"] = last
    # the same ticks without the structure functions and the capture (first
    # realign to a tick where every sample steps)
    ens.capture_velocity(False)
    ens.step((-ens.ticks) % every)
    ens.synchronize()
    e0.record(ens.stream)
    for k in range(0, ticks, every):
        ens.step(min(every, ticks - k), record_every=every)
    e1.record(ens.stream)
    ens.synchronize()
    sec2 = e0.elapsed_time(e1) / 1e3
    out["MLUPS_lbm_and_reductions"] = round(lups / sec2 / 1e6, 1)
    out["structure_function_share"] = round(max(0.0, 1 - sec2 / sec), 4) if with_sf else 0.0
    if ens.check() >= 0:
        raise SystemExit("mixed workload became unstable")
    del ens, work
    torch.cuda.empty_cache()
    return out


def bench_adjoint(mc, torch):
    """8 x 128^3 FP32: forward 1000 steps with checkpoints every 50, then the
    discrete adjoint (recompute per segment + reverse collide-and-stream) to
    d(mean KE)/dY."""
    import mc_inputs
    wl = mc_inputs.WORKLOADS["adjoint128x8_f32"]
    ens = build_ensemble(wl, mc, torch)
    cells = sum(s.n ** 3 for s in ens.samples)
    ticks, every = wl.ticks, wl.save_every
    e = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
    ens.synchronize()
    e[0].record(ens.stream)
    ck = ens.forward_ckpt(ticks, every)
    e[1].record(ens.stream)
    dj, ke = ens.backward(ticks, every, ck)
    e[2].record(ens.stream)
    ens.synchronize()
    fwd = e[0].elapsed_time(e[1]) / 1e3
    bwd = e[1].elapsed_time(e[2]) / 1e3
    out = {"workload": wl.name, "steps": ticks, "ckpt_every": every,
           "forward_seconds": round(fwd, 4), "backward_seconds": round(bwd, 4),
           "total_seconds": round(fwd + bwd, 4),
           "forward_MLUPS": round(cells * ticks / fwd / 1e6, 1),
           "backward_MLUPS": round(cells * ticks / bwd / 1e6, 1),
           "backward_bytes_per_lup": 324 + 216 * (ticks - (ticks + every - 1) // every) / ticks,
           "dJdY_norm": float(dj.norm()), "J": float(ke.mean())}
    out["backward_GBps_algorithmic"] = round(out["backward_bytes_per_lup"] * cells * ticks / bwd / 1e9, 1)
    del ens, ck
    torch.cuda.empty_cache()
    return out


def bench_lattice(mc, torch, name, ticks=500):
    """Another lattice on the 64-sample ensemble: autotuned launch, timed
    ticks with the reductions fused every 50, kernel roofline."""
    import mc_inputs
    wl = mc_inputs.WORKLOADS[name]
    ens = build_ensemble(wl, mc, torch)
    tuned = ens.autotune(reps=3)
    ens.step(20)
    sec, lups = timed_ticks(ens, torch, ticks, wl.save_every)
    avg_ms, launches, bpl, achieved = kernel_roofline(ens, wl, torch, 40)
    if ens.check() >= 0:
        raise SystemExit(f"{name} became unstable")
    out = {"workload": wl.name, "lattice": f"D3Q{wl.lattice}", "ticks": ticks, "MLUPS": round(lups / sec / 1e6, 1),
           "launch": dict(zip(("block", "xcd_remap", "buffer_addressing", "nontemporal"), tuned)),
           "kernel_avg_ms": round(avg_ms, 5), "bytes_per_lup": BYTES_PER_LUP[wl.precision, wl.lattice],
           "kernel_GBps_algorithmic": round(achieved, 1), "kernel_frac_of_peak": round(achieved / HBM_PEAK_GBS, 4)}
    del ens
    torch.cuda.empty_cache()
    return out


def bench_exact(mc, torch, ticks=200):
    """The default 64 x 64^3 ensemble with the exact entropic stabiliser (the
    minimiser of the discrete H-function by safeguarded Newton steps in every
    node, 256-thread blocks): MLUPS, the kernel's algorithmic bandwidth, and
    the mean gamma of both stabilisers after the timed ticks."""
    import mc_inputs
    wl = mc_inputs.WORKLOADS["rtgv64x64_f32"]
    ens = build_ensemble(wl, mc, torch)
    ens.set_stabiliser("exact")
    ens.step(20)
    sec, lups = timed_ticks(ens, torch, ticks, 0)
    avg_ms, _, _, achieved = kernel_roofline(ens, wl, torch, 20)
    gamma_exact = float(ens.reduce()[:, 7].mean())
    ens.set_stabiliser("closed_form")
    gamma_closed = float(ens.reduce()[:, 7].mean())
    if ens.check() >= 0:
        raise SystemExit("exact-stabiliser run became unstable")
    out = {"workload": wl.name, "stabiliser": "exact", "ticks": ticks, "MLUPS": round(lups / sec / 1e6, 1),
           "kernel_avg_ms": round(avg_ms, 5), "kernel_GBps_algorithmic": round(achieved, 1),
           "kernel_frac_of_peak": round(achieved / HBM_PEAK_GBS, 4),
           "mean_gamma_exact": round(gamma_exact, 5), "mean_gamma_closed_form_same_state": round(gamma_closed, 5)}
    del ens
    torch.cuda.empty_cache()
    return out


def bench_sequence(mc, torch):
    """Capacity run of the vanishing-viscosity sequence: 8 samples at each of
    128^3, 256^3 and 512^3 in one ensemble (132 GB of FP32 populations), the
    same Y at every resolution, strides 16:4:1, FP64 records every 16 ticks.
    After the timed ticks: the FP64 energy spectrum and structure function
    of every sample; the 1-point Wasserstein distance and the relative L1
    sample error of the 128^3 and 256^3 ensembles against the 512^3 one, on
    the velocities at the 8^3 nodes common to all resolutions (physical
    units u / U0), and their orders of convergence in N."""
    import mc_inputs
    import numpy as np
    wl = mc_inputs.WORKLOADS["sequence512x8_f32"]
    samples = []
    for g in wl.groups:
        samples += [mc.Sample(g.n, g.u0, g.re, g.amp, g.project, g.stride)] * g.count
    # launch shape: autotuned on the group of the finest resolution alone,
    # which steps on every tick and carries 95 % of the updates (tuning the
    # whole ensemble would time 64 ticks per candidate: its largest stride is
    # 16); the group and the tuner's copy of it take 232 GB
    finest = wl.groups[-1]
    proxy = mc.Ensemble([mc.Sample(finest.n, finest.u0, finest.re, finest.amp, finest.project)] * finest.count,
                        wl.precision, lattice=wl.lattice)
    proxy.init(wl.seed)
    tuned = proxy.autotune(reps=1)
    del proxy
    torch.cuda.empty_cache()
    ens = mc.Ensemble(samples, wl.precision, lattice=wl.lattice)
    per = wl.groups[0].count
    y = np.tile(mc_inputs.draw_y(wl.seed, per), (len(wl.groups), 1))
    ens.init(0, torch.from_numpy(y))
    ens.set_launch(*tuned)
    ticks, every = wl.ticks, wl.save_every
    sec, lups = timed_ticks(ens, torch, ticks, every)
    if ens.check() >= 0:
        raise SystemExit("sequence workload became unstable")
    # FP64 energy spectrum and structure function of every sample (one batch
    # of launches per resolution), ensemble means in units of U0^2
    obs = {}
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ens.synchronize()
    e0.record(ens.stream)
    first = 0
    for g in wl.groups:
        s2, ek = ens.observables_range(first, g.count)
        obs[g.n] = (s2, ek, g.u0)
        first += g.count
    e1.record(ens.stream)
    ens.synchronize()
    obs_sec = e0.elapsed_time(e1) / 1e3
    spectra = {f"{n}^3": {"S2_r1_r2_r4": [round(float(s2[:, r - 1].mean()) / u0 ** 2, 10) for r in (1, 2, 4)],
                          "E_peak_kappa": int(ek.mean(dim=0).argmax())}
               for n, (s2, ek, u0) in obs.items()}
    del obs
    # distances of the coarser ensembles to the finest one (the reference)
    # and the least-squares orders of convergence over log N: Wasserstein
    # (EOWC, from W_{1,1}) and sample-wise (EOSC, from the vector L1 error)
    pv = ens.point_values(8, physical=True)       # [m][3][8^3], u / U0
    nref, ref = wl.groups[-1].n, pv[(len(wl.groups) - 1) * per:].contiguous()
    ns, w1, err = [], [], []
    for k, g in enumerate(wl.groups[:-1]):
        cur = pv[k * per:(k + 1) * per].contiguous()
        w1.append(float(mc.w1_1pt(cur, ref, 8).sum()))          # on the current stream, like pv
        err.append(mc.sample_error(cur, ref, 8).cpu().tolist())
        ns.append(g.n)
    # and between consecutive resolutions
    w1c = {}
    for k in range(len(wl.groups) - 1):
        lo, hi = pv[k * per:(k + 1) * per].contiguous(), pv[(k + 1) * per:(k + 2) * per].contiguous()
        w1c[f"{wl.groups[k].n}^3-{wl.groups[k + 1].n}^3"] = round(float(mc.w1_1pt(lo, hi, 8).sum()), 8)
    conv = {"reference_n": nref,
            "W1_1pt_u_over_U0": {f"{n}^3": round(v, 8) for n, v in zip(ns, w1)},
            "W1_1pt_consecutive_u_over_U0": w1c,
            "sample_error_L1_xyz_vec": {f"{n}^3": [round(v, 6) for v in e] for n, e in zip(ns, err)},
            "EOWC_W1_1pt": round(mc.eoc_slope(ns, w1), 4),
            "EOSC_vec": round(mc.eoc_slope(ns, [e[3] for e in err]), 4)}
    gb = sum(s.n ** 3 for s in samples) * BYTES_PER_LUP[wl.precision, wl.lattice] / 2 / 1e9
    out = {"workload": wl.name, "ticks": ticks, "steps": [ticks // g.stride for g in wl.groups],
           "population_GB": round(gb, 1), "lattice_updates": lups, "seconds": round(sec, 4),
           "MLUPS": round(lups / sec / 1e6, 1),
           "launch": dict(zip(("block", "xcd_remap", "buffer_addressing", "nontemporal"), tuned)),
           "observables_seconds": round(obs_sec, 4), "ensemble_mean_observables": spectra,
           "convergence": conv}
    del ens, pv
    torch.cuda.empty_cache()
    return out


def bench_sequence_to_onset(mc, torch, name, launch=None, rec_every=16):
    """The vanishing-viscosity sequence in acoustic scaling run to t = 9 (the
    onset of turbulence of the Taylor-Green vortex): 8 samples per resolution
    with the same Y at every N, U0 = 0.05 at every N (time step proportional
    to dx, strides 4:2:1), Re = 12.5 N, FP64 kinetic-energy records every
    `rec_every` ticks. At every save (t = 1, 2, ..., 9): per resolution the
    ensemble mean and standard deviation of KE, both dissipation-rate forms
    (the decay of the records' kinetic energy, and the paper's decay of the
    summed shell spectrum over the last `rec_every` ticks) with the
    Kolmogorov length, the mean structure function at common physical lags,
    the mean spectrum and the mean compensated spectrum; between
    resolutions, on the 8^3 common nodes in units of U0, W_{1,1} and the
    relative L1 sample error of each coarser ensemble against the finest, and
    their orders of convergence (EOWC, EOSC). Prints one line per save."""
    import mc_inputs
    import numpy as np
    wl = mc_inputs.WORKLOADS[name]
    samples = []
    for g in wl.groups:
        samples += [mc.Sample(g.n, g.u0, g.re, g.amp, g.project, g.stride)] * g.count
    ens = mc.Ensemble(samples, wl.precision, lattice=wl.lattice)
    per = wl.groups[0].count
    y = np.tile(mc_inputs.draw_y(wl.seed, per), (len(wl.groups), 1))
    ens.init(0, torch.from_numpy(y))
    tuned = launch if launch is not None else ens.autotune(reps=1)
    ens.set_launch(*tuned)
    finest = wl.groups[-1]
    dt = 2 * np.pi / finest.n * finest.u0              # physical time of one tick
    firsts, first = [], 0
    for g in wl.groups:
        firsts.append(first)
        first += g.count
    work = ens._dev_empty((max(int(mc.lib().mclbm_observables_range_work_bytes(ens._ctx, a, g.count))
                               for a, g in zip(firsts, wl.groups)),), torch.uint8)
    coarse = wl.groups[0].n
    records, saves = [], []
    lups, sec = 0, 0.0
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    nsave = wl.ticks // wl.save_every
    for k in range(1, nsave + 1):
        t0 = ens.ticks
        lups += sum(cells_per_tick(ens, t0 + j) for j in range(wl.save_every))
        ens.synchronize()
        e0.record(ens.stream)
        records.append(ens.step(wl.save_every - rec_every, record_every=rec_every))
        e1.record(ens.stream)
        ens.synchronize()
        sec += e0.elapsed_time(e1) / 1e3
        ek_a = [ens.observables_range(a, g.count, work, structure=False)[1].clone() for a, g in zip(firsts, wl.groups)]
        e0.record(ens.stream)
        records.append(ens.step(rec_every, record_every=rec_every))
        e1.record(ens.stream)
        ens.synchronize()
        sec += e0.elapsed_time(e1) / 1e3
        bad = ens.check()
        tick = ens.ticks
        t = tick * dt
        row = {"tick": tick, "t": round(t, 4), "unstable_sample": bad, "groups": {}}
        pv = ens.point_values(8, physical=True)
        ref = pv[firsts[-1]:].contiguous()
        ns, w1, err = [], [], []
        for gi, (a, g) in enumerate(zip(firsts, wl.groups)):
            s2, ek_b = ens.observables_range(a, g.count, work)
            series = torch.stack([ek_a[gi], ek_b])
            d_sp, eta_sp = ens.dissipation_spectra(a, series, tick - rec_every, rec_every)
            ekc = ens.compensate(a, d_sp[1].contiguous(), ek=ek_b)[1]
            red = ens.reduce()[a:a + g.count]
            ke_m, ke_s = mc.ensemble_moments(red[:, 4:5].contiguous())
            u2 = g.u0 ** 2
            lag = [r * g.n // coarse for r in (1, 2, 4, 8)]
            s2m = s2.mean(dim=0).cpu().numpy() / u2
            ekm = ek_b.mean(dim=0).cpu().numpy() / u2
            ekcm = ekc.mean(dim=0).cpu().numpy()
            row["groups"][f"{g.count}x{g.n}^3"] = {
                "E_KE": float(ke_m[0]) / u2, "sigma_KE": float(ke_s[0]) / u2,
                "E_d_spectral": float(d_sp[1].mean()), "eta_spectral": float(eta_sp[1]),
                "E_S2_at_lag_dx128_x1_2_4_8": [float(s2m[r - 1]) for r in lag],
                "E_spectrum_kappa_2_8_32": [float(ekm[kk]) for kk in (2, 8, 32) if kk < len(ekm)],
                "E_compensated_spectrum_kappa_4_8_16": [float(ekcm[kk]) for kk in (4, 8, 16) if kk < len(ekcm)],
                "E_kappa_peak": int(np.argmax(ekm))}
            if gi < len(wl.groups) - 1:
                cur = pv[a:a + g.count].contiguous()
                w1.append(float(mc.w1_1pt(cur, ref, 8).sum()))
                err.append(mc.sample_error(cur, ref, 8).cpu().tolist())
                ns.append(g.n)
        row["reference_n"] = finest.n
        row["W1_1pt_u_over_U0"] = {f"{n}^3": w for n, w in zip(ns, w1)}
        row["W1_1pt_consecutive_u_over_U0"] = {
            f"{lo.n}^3-{hi.n}^3": float(mc.w1_1pt(pv[a:a + lo.count].contiguous(), pv[b:b + hi.count].contiguous(),
                                                  8).sum())
            for (a, lo), (b, hi) in zip(zip(firsts, wl.groups), zip(firsts[1:], wl.groups[1:]))}
        row["sample_error_L1_vec"] = {f"{n}^3": e[3] for n, e in zip(ns, err)}
        if all(v > 0 for v in w1) and all(e[3] > 0 for e in err):
            row["EOWC"] = mc.eoc_slope(ns, w1)
            row["EOSC"] = mc.eoc_slope(ns, [e[3] for e in err])
        saves.append(row)
        print(f"[onset] t = {t:.3f} (tick {tick}): " + "; ".join(
            f"{key} E[KE] {v['E_KE']:.5f} E[d] {v['E_d_spectral']:.5f}" for key, v in row["groups"].items()) +
            f"; W1 {[round(v, 5) for v in w1]} EOWC {row.get('EOWC', float('nan')):.3f} "
            f"EOSC {row.get('EOSC', float('nan')):.3f} ({lups / sec / 1e6:.0f} MLUPS)", flush=True)
        if bad >= 0:
            break
    rec = torch.cat(records)
    # the kinetic-energy form of the dissipation rate from all records, at
    # the record nearest each save
    d_ke, _ = ens.dissipation(rec, 0, rec_every, eta=False)
    d_ke = d_ke.cpu().numpy()
    for row in saves:
        j = min(row["tick"] // rec_every, d_ke.shape[0] - 1)
        for a, g in zip(firsts, wl.groups):
            row["groups"][f"{g.count}x{g.n}^3"]["E_d_kinetic_energy"] = float(d_ke[j, a:a + g.count].mean())
    out = {"workload": wl.name, "ticks": ens.ticks, "t_end": round(ens.ticks * dt, 4),
           "steps": [ens.steps(a) for a in firsts], "lattice_updates": lups, "seconds": round(sec, 3),
           "MLUPS": round(lups / sec / 1e6, 1),
           "launch": dict(zip(("block", "xcd_remap", "buffer_addressing", "nontemporal"), tuned)),
           "groups": [f"{g.count}x{g.n}^3 U0 {g.u0} Re {g.re} stride {g.stride}" for g in wl.groups],
           "saves": saves}
    del ens, work
    torch.cuda.empty_cache()
    return out


# ensembles for the counter runs of the collide-and-stream kernel beyond the
# default workload: (lattice, samples, n, block, buffer addressing)
TRAFFIC_PROBES = ((27, 8, 128, 512, 1), (27, 4, 256, 512, 1), (27, 1, 512, 512, 0), (19, 64, 64, 256, 1))


def traffic_probe(mc, torch, ticks=4):
    """A few plain ticks of each TRAFFIC_PROBES ensemble (FP32, graphs off), for
    hardware-counter passes; prints one line per ensemble."""
    for q, m, n, block, buf in TRAFFIC_PROBES:
        ens = mc.Ensemble([mc.Sample(n, 0.05 * 32 / n, 25.0 * n, 0.05, True)] * m, "f32s", lattice=q)
        ens.init(3)
        ens.set_launch(block, 0, buf, 1)
        ens.use_graphs(False)
        ens.step(ticks)
        ens.synchronize()
        print(f"[traffic-probe] D3Q{q} {m} x {n}^3 block {block} buffer {buf}: {ticks} ticks", flush=True)
        del ens
        torch.cuda.empty_cache()


# resolution groups of the observables probe: (samples, n)
OBSERVABLES_PROBES = ((32, 64), (12, 128), (4, 256), (1, 512))


def observables_probe(mc, torch, reps=3):
    """The FP64 spectrum and structure function of each OBSERVABLES_PROBES
    group (FP32 D3Q27 ensembles a few ticks after initialisation, one set of
    launches per group), `reps` times, timed with HIP events, from the
    populations and from the velocity a record tick captured, with the
    record tick timed with and without the capture; for kernel-trace and
    counter passes. Prints two lines per group."""
    def timed(ens, fn):
        fn()
        ens.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(ens.stream)
        for _ in range(reps):
            fn()
        e1.record(ens.stream)
        ens.synchronize()
        return e0.elapsed_time(e1) / reps

    for m, n in OBSERVABLES_PROBES:
        ens = mc.Ensemble([mc.Sample(n, 0.05 * 32 / n, 25.0 * n, 0.05, True)] * m, "f32s")
        ens.init(5)
        ens.step(3)
        ms = timed(ens, lambda: ens.observables_range(0, m))
        print(f"[observables-probe] {m} x {n}^3: {ms:.3f} ms per set of launches, "
              f"{ms * 1e6 / (m * n ** 3):.4f} ns per node", flush=True)
        rec = timed(ens, lambda: ens.step(1, record_every=1))
        ens.capture_velocity()
        rec_u = timed(ens, lambda: ens.step(1, record_every=1))
        ms_u = timed(ens, lambda: ens.observables_velocity_range(0, m))
        print(f"[observables-probe] {m} x {n}^3 from the captured velocity: {ms_u:.3f} ms per set of launches; "
              f"record tick {rec:.3f} ms, {rec_u:.3f} ms with the capture", flush=True)
        del ens
        torch.cuda.empty_cache()


def adjoint_probe(mc, torch, steps=20, every=10):
    """A short forward with checkpoints and the backward sweep of the adjoint
    workload's ensemble (8 x 128^3 FP32, graphs as in the benchmark), timed
    with HIP events; for kernel-trace and counter passes."""
    import mc_inputs
    wl = mc_inputs.WORKLOADS["adjoint128x8_f32"]
    ens = build_ensemble(wl, mc, torch)
    ck = ens.forward_ckpt(steps, every)
    ens.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(ens.stream)
    dj, _ = ens.backward(steps, every, ck)
    e1.record(ens.stream)
    ens.synchronize()
    sec = e0.elapsed_time(e1) / 1e3
    lups = sum(s.n ** 3 for s in ens.samples) * steps
    print(f"[adjoint-probe] {wl.name}: {steps} reverse steps (checkpoints every {every}) in {sec * 1e3:.1f} ms, "
          f"{lups / sec / 1e6:.0f} MLUPS, |dJ/dY| {float(dj.norm()):.4e}", flush=True)


def stabiliser_probe(mc, torch, ticks=8):
    """A few plain ticks (graphs off, 256-thread blocks) of the default
    64 x 64^3 ensemble with the closed-form and then the exact stabiliser,
    timed per launch; for kernel-trace and counter passes."""
    import mc_inputs
    ens = build_ensemble(mc_inputs.WORKLOADS["rtgv64x64_f32"], mc, torch)
    ens.set_launch(256, 0, 1, 1)
    ens.use_graphs(False)
    ens.step(2)
    for mode in ("closed_form", "exact"):
        ens.set_stabiliser(mode)
        ens.time_launches(True)
        ens.step(ticks)
        avg, n = ens.launch_time()
        ens.time_launches(False)
        print(f"[stabiliser-probe] {mode}: {n} launches, {avg:.4f} ms average, "
              f"{216 * 64 * 64 ** 3 / avg / 1e6:.0f} GB/s algorithmic", flush=True)


def cpu_baseline(seconds_target=15.0, large=True):
    """The oracle on one 64^3 RTGV sample of the workload, on all host cores
    (and two steps on one core); for context also the 32^3 FP64 TGV
    configuration in full and, with `large`, one step of one 256^3 sample of
    the mixed-resolution workload (its initialisation untimed, ~15 s)."""
    import numpy as np
    import mc_inputs
    import oracle
    wl = mc_inputs.WORKLOADS["rtgv64x64_f32"]
    g = wl.groups[0]
    y = mc_inputs.draw_y(wl.seed, 1)[0]
    om = oracle.omega_shear(oracle.lattice_viscosity(g.n, g.u0, g.re))
    f = oracle.init_populations(g.n, g.u0, g.amp, y, g.project)
    threads = len(os.sched_getaffinity(0))
    t = time.perf_counter()
    oracle.run(f, g.n, 2, om, threads=threads)
    probe = time.perf_counter() - t
    steps = max(2, min(2000, int(seconds_target / max(probe / 2, 1e-6))))
    t = time.perf_counter()
    oracle.run(f, g.n, steps, om, threads=threads)
    sec = time.perf_counter() - t
    _, u_ref = oracle.moments(f, g.n)       # sample 0 after 2 + steps steps
    t = time.perf_counter()
    oracle.run(f, g.n, 2, om, threads=1)
    one = time.perf_counter() - t
    # the single-sample FP64 configuration in full (32^3 TGV, Re 100, 100
    # steps), on all cores
    tgv = mc_inputs.WORKLOADS["tgv32_f64"].groups[0]
    f32 = oracle.init_populations(tgv.n, tgv.u0, 0.0, np.zeros(24), False)
    t = time.perf_counter()
    oracle.run(f32, tgv.n, 100, oracle.omega_shear(oracle.lattice_viscosity(tgv.n, tgv.u0, tgv.re)), threads=threads)
    sec32 = time.perf_counter() - t
    mlups256 = None
    if large:
        mixed = mc_inputs.WORKLOADS["mixed48_f32"]
        g256 = mixed.groups[-1]
        y256 = mc_inputs.draw_y(mixed.seed, mixed.m)[mixed.m - 1]
        f256 = oracle.init_populations(g256.n, g256.u0, g256.amp, y256, g256.project)
        t = time.perf_counter()
        oracle.run(f256, g256.n, 1, oracle.omega_shear(oracle.lattice_viscosity(g256.n, g256.u0, g256.re)),
                   threads=threads)
        mlups256 = round(g256.n ** 3 / (time.perf_counter() - t) / 1e6, 3)
        del f256
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as fh:
            model = next((ln.split(":", 1)[1].strip() for ln in fh if ln.startswith("model name")), model)
    except OSError:
        pass
    return {"value": g.n ** 3 * steps / sec / 1e6, "unit": "MLUPS", "cores": threads, "kind": "oracle",
            "sample": f"1 RTGV sample at {g.n}^3 of the 64x64^3 workload, {steps} steps, FP64 moment-space "
                      f"KBC collision, two-lattice pull streaming ({sec:.1f} s)",
            "single_core_MLUPS": round(g.n ** 3 * 2 / one / 1e6, 3),
            "tgv32_f64_100_steps_MLUPS": round(tgv.n ** 3 * 100 / sec32 / 1e6, 3),
            "rtgv256_one_sample_one_step_MLUPS": mlups256, "cpu_model": model}, (2 + steps, u_ref)


def measured_error(mc, torch, wl, launch, steps, u_ref):
    """Relative L2 and maximum error of the velocity of sample 0 of the
    workload after `steps` steps in the benchmark's launch shape
    (graph-captured ticks, reductions fused as in the timed run) against the
    oracle's field of the same sample (the CPU baseline's run)."""
    import numpy as np
    ens = build_ensemble(wl, mc, torch)
    if launch is not None:
        ens.set_launch(*launch)
    ens.step(steps, record_every=wl.save_every if steps >= wl.save_every else 0)
    _, u = ens.moments(0)
    u = u.cpu().numpy().reshape(u_ref.shape)
    del ens
    torch.cuda.empty_cache()
    return {"rel_l2_u_vs_oracle": float(np.linalg.norm(u - u_ref) / np.linalg.norm(u_ref)),
            "max_abs_u_error_over_max_abs_u": float(np.max(np.abs(u - u_ref)) / np.max(np.abs(u_ref))),
            "steps": steps, "sample": 0, "target_rel_l2": 1e-5 if wl.precision == "f32s" else 1e-12}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=500)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--workload", default="rtgv64x64_f32")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-autotune", action="store_true")
    ap.add_argument("--roofline-ticks", type=int, default=40)
    ap.add_argument("--skip-fp64", action="store_true", help="skip the single-sample FP64 reference runs")
    ap.add_argument("--copy-gib", type=float, default=4.0, help="size of the copy-kernel bandwidth probe")
    ap.add_argument("--sweep", action="store_true", help="time every launch shape and report the table")
    ap.add_argument("--no-extra", action="store_true", help="skip the mixed-resolution and adjoint workloads")
    ap.add_argument("--no-capacity", action="store_true", help="skip the 132 GB vanishing-viscosity sequence")
    ap.add_argument("--traffic-probe", action="store_true",
                    help="only run a few ticks of the larger-lattice and D3Q19 ensembles (for counter passes)")
    ap.add_argument("--stabiliser-probe", action="store_true",
                    help="only run a few ticks with each stabiliser (for counter passes)")
    ap.add_argument("--adjoint-probe", action="store_true",
                    help="only run a short forward and backward of the adjoint workload (for counter passes)")
    ap.add_argument("--observables-probe", action="store_true",
                    help="only time the FP64 observables of one group per resolution (for counter passes)")
    ap.add_argument("--onset", default=None, choices=["sequence512x8_acoustic_f32", "sequence256x8_acoustic_f32"],
                    help="only run this acoustic vanishing-viscosity sequence to t = 9 and print its statistics")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (the library has no multi-GPU path); got --gpus {args.gpus}",
              file=sys.stderr)
        sys.exit(2)

    import torch
    import mc_inputs
    import paper_2608_23786_amd as mc

    if args.traffic_probe:
        traffic_probe(mc, torch)
        return
    if args.adjoint_probe:
        adjoint_probe(mc, torch)
        return
    if args.stabiliser_probe:
        stabiliser_probe(mc, torch)
        return
    if args.observables_probe:
        observables_probe(mc, torch)
        return
    if args.onset:
        # the finest group of the 512^3 sequence holds 8 samples of 14.5 GB:
        # plain pointers, block 512, XCD-contiguous blocks (the tuned shape of
        # the diffusive sequence's 512^3 group)
        launch = (512, 1, 0, 1) if args.onset.startswith("sequence512") else None
        print(json.dumps(bench_sequence_to_onset(mc, torch, args.onset, launch)), flush=True)
        return
    wl = mc_inputs.WORKLOADS[args.workload]
    print(f"[bench] workload {wl.name}: {wl.m} samples, precision {wl.precision}", file=sys.stderr, flush=True)
    b_meas = stream_bandwidth(mc, torch, nbytes=int(args.copy_gib * (1 << 30)) // 16 * 16)
    print(f"[bench] copy kernel: {b_meas:.0f} GB/s", file=sys.stderr, flush=True)
    ens = build_ensemble(wl, mc, torch)
    tuned = None
    if not args.no_autotune:
        tuned = ens.autotune(reps=5)
        print(f"[bench] autotuned launch: block {tuned[0]}, xcd remap {tuned[1]}, buffer addressing {tuned[2]}, "
              f"non-temporal {tuned[3]}", file=sys.stderr, flush=True)
    sweep = launch_sweep(ens, wl, torch) if args.sweep else None
    ens.step(args.warmup)
    rec_every = wl.save_every if wl.save_every and args.steps >= wl.save_every else 0
    sec, lups = timed_ticks(ens, torch, args.steps, rec_every)
    mlups = lups / sec / 1e6
    bad = ens.check()
    if bad >= 0:
        raise SystemExit(f"sample {bad} became unstable")
    print(f"[bench] {args.steps} ticks in {sec:.3f} s: {mlups:.0f} MLUPS", file=sys.stderr, flush=True)
    avg_ms, launches, bpl, achieved = kernel_roofline(ens, wl, torch, args.roofline_ticks)
    print(f"[bench] collide-stream: {launches} launches, {avg_ms:.4f} ms avg, {achieved:.0f} GB/s algorithmic",
          file=sys.stderr, flush=True)
    f64 = f64_batch = None
    if not args.skip_fp64:
        f64 = {"32^3 TGV Re 100 MLUPS": round(fp64_single(mc, torch, 32, 0.05, 100.0), 1),
               "64^3 Re 1600 MLUPS": round(fp64_single(mc, torch, 64, 0.025, 1600.0), 1)}
        if wl.name == "rtgv64x64_f32":
            f64_batch = fp64_batched(mc, torch)
            print(f"[bench] fp64 batched: {f64_batch}", file=sys.stderr, flush=True)
    extra = {}
    if not args.no_extra:
        del ens
        torch.cuda.empty_cache()
        extra["mixed48"] = bench_mixed(mc, torch)
        print(f"[bench] mixed48: {extra['mixed48']}", file=sys.stderr, flush=True)
        extra["adjoint128x8"] = bench_adjoint(mc, torch)
        print(f"[bench] adjoint128x8: {extra['adjoint128x8']}", file=sys.stderr, flush=True)
        if wl.lattice == 27:
            extra["d3q19"] = bench_lattice(mc, torch, "rtgv64x64_f32_d3q19")
            print(f"[bench] d3q19: {extra['d3q19']}", file=sys.stderr, flush=True)
        if wl.name == "rtgv64x64_f32":
            extra["exact_stabiliser"] = bench_exact(mc, torch)
            print(f"[bench] exact stabiliser: {extra['exact_stabiliser']}", file=sys.stderr, flush=True)
        if not args.no_capacity:
            extra["sequence512x8"] = bench_sequence(mc, torch)
            print(f"[bench] sequence512x8: {extra['sequence512x8']}", file=sys.stderr, flush=True)
    out = {
        "metric": "aggregate MLUPS & % HBM roofline, batched FP32 vs plain FP64, at stated rel. error",
        "value": round(mlups, 1),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(sec / args.steps * 1e3, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if wl.precision == "f32s" else "f64",
        "data": "synthetic",
        "config": {"workload": wl.name, "samples": wl.m, "lattice": f"D3Q{wl.lattice}",
                   "lattices": [f"{g.count}x{g.n}^3 stride {g.stride}" for g in wl.groups],
                   "precision": "FP32 shifted populations (f - w), FP64 reductions" if wl.precision == "f32s"
                   else "FP64", "reduce_every": rec_every, "launch": dict(zip(("block", "xcd_remap", "buffer_addressing", "nontemporal"),
                                                                          tuned or (256, 0, 1, 1))),
                   "error_vs_oracle": None},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": counter_traffic(wl.name),
                     "traffic_unit": "bytes per launch", "algorithmic_bytes_per_launch": int(round(bpl)),
                     "kernel": "kbc_step_kernel", "bytes_per_lup": BYTES_PER_LUP[wl.precision, wl.lattice],
                     "avg_launch_ms": round(avg_ms, 5), "launches_timed": launches,
                     "measured_copy_GBps": round(b_meas, 1), "frac_of_measured_copy": round(achieved / b_meas, 4)},
        "fp64_single_sample": f64,
        **({"fp64_batched_64x64": f64_batch} if f64_batch else {}),
        **({"launch_sweep": sweep} if sweep else {}),
        **extra,
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"], (err_steps, u_ref) = cpu_baseline()
        out["config"]["error_vs_oracle"] = measured_error(mc, torch, wl, tuned, err_steps, u_ref)
        print(f"[bench] velocity error vs oracle: {out['config']['error_vs_oracle']}", file=sys.stderr, flush=True)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
