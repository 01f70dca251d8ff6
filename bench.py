"""Benchmark: FP64 RK2 finite-volume Euler steps per second on one MI355X,
with the other per-GPU cases and the forms built on the step beside it.

    python bench.py [--gpus 1] [--steps 100] [--warmup 5] [--size 512]
                    [--case sine|plane] [--no-cpu-baseline] [--no-forms]
                    [--no-cases] [--case-sizes 512,256]
                    [--forms f32,batch,learned] [--learned-iters N] [--copy-probe MIB]

A step is one RK2 step of the whole hot path on the periodic cube: the two
fused substep kernels, with the CFL max-reduction fused into the second one
(the time step stays on the device; one extra reduction pass starts the timed
sequence).  Inputs are synthetic and already resident in HBM when timing
starts: the smooth case rho = 1 + 0.2 sin(2 pi (x+y+z)), v = (1,1,1), p = 1
(exact cell averages), or the seeded random-plane Riemann case (seed 0).

Prints one JSON line with the cell-update rate of the timed block (no
per-kernel events inside it), the roofline of the dominant kernel
(per-launch algorithmic HBM bytes over its average event-timed duration,
from a second block of the same length with HIP events around every launch,
against the 8 TB/s HBM3E peak and against the ceiling the library's
streaming probe measures for the kernel's read:write mix), the step-level
fraction of the HBM peak, and the CPU oracle timed on a bounded sample on
the host cores (all threads; then one eighth of them and one, on a smaller
sample).  After the reported block of steps, four more blocks of the same
length give the spread of the rate (reported with their median), and 20
steps of the host-synchronised path (gs_fluid_dt, then gs_fluid_step) and
20 of the host-synchronised path on the step's fused max (gs_fluid_step_dt)
give their rates.  Under "cases" the random-plane Riemann case and the smooth case
at 512^3 and 256^3 are timed the same way, FP64 and FP32 (with the FP32
error per field on the 512^3 Riemann case).  Under "forms" the FP32 form is
timed the same way on the headline input, with its speedup over FP64 and
its L1 and L-infinity error per field against the FP64 solution of the same
input after the same steps (the FP32 run is driven with the FP64 run's time
steps; the FP64 path itself matches the CPU oracle to 1e-12); then the
batched and learned-correction forms.
"""
import argparse
import hashlib
import json
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E, published
# FP64 vector peak 78.6 TFLOP/s counts an FMA as 2 flops: 256 CUs x 64 FP64
# lanes per clock x 2.4 GHz = 39.3 T lane operations per second, the issue
# rate of one wave64 VALU instruction per SIMD per 4 clocks
VALU_LANE_OPS_PEAK_T = 39.3
# algorithmic HBM bytes per cell and launch
BYTES_PER_CELL = {
    "f64": {0: 80.0,     # substep 1: read U(n), write U(1)
            1: 120.0,    # substep 2: read U(1) and U(n), write U(n+1)
            2: 40.0},    # dt reduction: read U
    "f32": {0: 60.0,     # substep 1: read U(n), write U(1) and dU(U(n))
            1: 120.0,    # substep 2: read U(1), dU(U(n)), U(n) and its
                         # compensation; write U(n+1) and its compensation
            2: 20.0},    # dt reduction: read the head
}
KERNEL_NAMES = {0: "stage_kernel<1> (substep 1)", 1: "stage_kernel<2> (substep 2 + dt max)",
                2: "rate reduction"}
METRIC = "cell-updates/s per RK2 step & HBM GB/s; plain FP64 vs chosen forms @ L1 err"
# the stage kernels' source and the build script that sets their flags
KERNEL_SOURCES = ["paper_1812_07977_amd/csrc/gs_fluid.hip", "paper_1812_07977_amd/csrc/stage.hpp",
                  "paper_1812_07977_amd/csrc/euler_math.hpp", "paper_1812_07977_amd/build.py"]


def source_hash():
    h = hashlib.sha256()
    for rel in KERNEL_SOURCES:
        with open(os.path.join(ROOT, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def profile_figure(key, size, case, dtype="f64"):
    """A per-launch figure from the committed rocprofv3 counter summary of
    the stage kernels, if it was taken on the current kernel source; else
    None (the counters no longer describe the code)."""
    tag = "" if dtype == "f64" else "_" + dtype
    path = os.path.join(ROOT, "profiles", f"counters_stage_kernels_{size}cubed_{case}{tag}.md")
    if not os.path.exists(path):
        return None
    text = open(path).read()
    m = re.search(r"^source_sha256_16:\s*(\w+)", text, re.M)
    if not m or m.group(1) != source_hash():
        return None
    m = re.search(rf"^{key}:\s*([0-9.eE+]+)", text, re.M)
    return float(m.group(1)) if m else None


def make_input(size, case):
    import workloads as wl
    if case == "sine":
        return wl.sine_wave(size, size, size)
    return wl.random_plane(size, size, size, seed=0)


def cpu_baseline(case, size=256, steps=10):
    """The oracle as it stands, on a bounded sample: the same case on a
    size^3 mesh for `steps` RK2 steps, using every host core OpenMP gives it;
    then, on a 128^3 sample of 2 steps, with one eighth of those threads (the
    host share of one GPU of eight) and with one thread."""
    import oracle
    oracle.lib()
    every = oracle.threads()

    def rate(n, nsteps):
        U = make_input(n, case)
        h = 1.0 / n
        t0 = time.perf_counter()
        taken = len(oracle.run(U, (h, h, h), 1.4, 0.5, oracle.PERIODIC, nsteps))
        return n ** 3 * taken / (time.perf_counter() - t0), taken, time.perf_counter() - t0

    value, taken, el = rate(size, steps)
    by_threads = {str(every): round(value)}
    for nt in sorted({max(every // 8, 1), 1}, reverse=True):
        oracle.set_threads(nt)
        by_threads[str(nt)] = round(rate(128, 2)[0])
    oracle.set_threads(every)
    return {"value": value, "unit": "cell-updates/s", "cores": every,
            "kind": "oracle",
            "sample": f"{case} case on a {size}^3 periodic mesh, {taken} RK2 step(s) incl. dt, "
                      f"{el:.1f} s wall",
            "by_threads": by_threads,
            "by_threads_sample": f"{case} case on a 128^3 periodic mesh, 2 RK2 steps"}


def timed_run(U0, n, dtype, steps, warmup, tile_y, chunk_z, repeats=1, host_steps=0,
              case="sine"):
    """Warm-up and timed gs_fluid_advance runs of one form from U0; returns
    the figures and the dt of every step (warm-up first).  The reported
    block of `steps` steps runs without per-kernel events; repeats > 1 times
    that many blocks in all (the first is the reported one).  Then one more
    block of `steps` steps with HIP events around every launch gives the
    per-kernel durations, and host_steps > 0 times that many host-dt steps."""
    import torch
    from paper_1812_07977_amd import Fluid
    F = Fluid((n, n, n), gamma=1.4, cfl=0.5, bc="periodic", dtype=dtype)
    F.set_launch(tile_y, chunk_z)
    S = F.state_from(U0)
    log_w = torch.zeros(max(warmup, 1), dtype=torch.float64, device="cuda")
    log_t = torch.zeros(max(steps, 1), dtype=torch.float64, device="cuda")
    if warmup:
        F.advance(S, warmup, 0.0, log_w)
    F.sync()

    stream = torch.cuda.current_stream()
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0.record(stream)
    F.advance(S, steps, 0.0, log_t)
    t1.record(stream)
    F.sync()
    torch.cuda.synchronize()
    total_ms = t0.elapsed_time(t1)
    t_sim = F.time
    # a copy: for FP64 the state itself is returned, and the blocks below
    # advance it further
    result = F.to_f64(S).clone() if dtype == "f64" else None
    dts = torch.cat([log_w[:warmup], log_t[:steps]]).cpu().numpy()
    extra = {}
    if repeats > 1:
        # further timed blocks of the same length, continuing the run
        reps = [total_ms]
        for _ in range(repeats - 1):
            torch.cuda.synchronize()
            t0.record(stream)
            F.advance(S, steps)
            t1.record(stream)
            F.sync()
            reps.append(t0.elapsed_time(t1))
        extra["repeat_ms"] = reps
    # per-kernel durations: HIP events the library records on its stream
    # around every launch, in a block of its own
    F.profile(True)
    for k in range(3):
        F.kernel_ms(k)
    torch.cuda.synchronize()
    t0.record(stream)
    F.advance(S, steps)
    t1.record(stream)
    F.sync()
    per_kernel = {k: F.kernel_ms(k) for k in range(3)}
    extra["profiled_block_ms"] = t0.elapsed_time(t1)
    F.profile(False)
    if host_steps:
        # the host-synchronised path: a reduction and a read-back of dt
        # before every step
        torch.cuda.synchronize()
        t0.record(stream)
        for _ in range(host_steps):
            F.step(S, F.dt(S))
        t1.record(stream)
        F.sync()
        extra["host_dt_ms"] = t0.elapsed_time(t1)
        extra["host_steps"] = host_steps
        # the same loop on the max each step fuses into its second substep
        # (gs_fluid_step_dt): one 8-byte read-back per step, no reduction
        dt = F.dt(S)
        torch.cuda.synchronize()
        t0.record(stream)
        for _ in range(host_steps):
            dt = F.step_dt(S, dt)
        t1.record(stream)
        F.sync()
        extra["host_dt_last_ms"] = t0.elapsed_time(t1)
    F.close()
    return {"total_ms": total_ms, "per_kernel": per_kernel, "t_sim": t_sim, **extra}, dts, result


def hbm_ceilings(mib=2048, reps=3):
    """Measured HBM ceilings from the library's streaming probe
    (gs_fluid_stream_probe): the best of `reps` event-timed runs over arrays
    of mib MiB for each read:write mix (copy 1:1 and add 2:1, the mixes of
    the two substeps) with and without non-temporal stores, in GB/s of bytes
    read plus written; and torch's device-to-device copy for comparison."""
    import torch
    from paper_1812_07977_amd import stream_probe
    nel = mib * 1024 * 1024 // 8
    a = torch.rand(nel, dtype=torch.float64, device="cuda")
    b = torch.rand(nel, dtype=torch.float64, device="cuda")
    c = torch.empty_like(a)
    stream = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    out = {}

    def best(fn, nbytes):
        top = 0.0
        for _ in range(reps + 1):      # the first run is a warm-up
            torch.cuda.synchronize()
            e0.record(stream)
            fn()
            e1.record(stream)
            torch.cuda.synchronize()
            top = max(top, nbytes / (e0.elapsed_time(e1) / 1e3) / 1e9)
        return round(top, 1)

    for nt in (False, True):
        tag = "_nt" if nt else ""
        out["copy_1to1" + tag] = best(lambda: stream_probe(a, c, nontemporal=nt), 2 * nel * 8)
        out["add_2to1" + tag] = best(lambda: stream_probe(a, c, b=b, nontemporal=nt), 3 * nel * 8)
    out["torch_copy"] = best(lambda: c.copy_(a), 2 * nel * 8)
    del a, b, c
    return out


def roofline(dtype, n, case, per_kernel):
    cells = n ** 3
    dom = max((0, 1), key=lambda k: per_kernel[k][0])
    ms_sum, launches = per_kernel[dom]
    avg_s = ms_sum / launches / 1e3
    bpc = BYTES_PER_CELL[dtype][dom]
    achieved = bpc * cells / avg_s / 1e9
    traffic = profile_figure(f"hbm_bytes_per_launch_kernel{dom}", n, case, dtype)
    roof = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
            "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": traffic, "kernel": KERNEL_NAMES[dom],
            "avg_launch_ms": round(avg_s * 1e3, 4),
            "bytes_per_launch": bpc * cells}
    # the same kernel against the vector ALU: VALU lane operations per launch
    # (wave64 VALU instructions counted by rocprofv3, x64) over the same
    # duration, against the issue peak of one wave64 instruction per SIMD per
    # 4 clocks
    valu = profile_figure(f"valu_lane_ops_per_launch_kernel{dom}", n, case, dtype)
    alu = None
    if valu is not None:
        a_t = valu / avg_s / 1e12
        alu = {"bound": "alu", "achieved": round(a_t, 2), "peak": VALU_LANE_OPS_PEAK_T,
               "unit": "T VALU lane-ops/s", "frac": round(a_t / VALU_LANE_OPS_PEAK_T, 4),
               "ops_per_launch": valu}
    return roof, alu


def f32_error(U0, n, dts, U64):
    """The FP32 form driven with the FP64 run's time steps from the same
    input: relative L1 and L-infinity error per field against the FP64
    result U64 (device)."""
    import torch
    from paper_1812_07977_amd import Fluid
    F = Fluid((n, n, n), gamma=1.4, cfl=0.5, bc="periodic", dtype="f32")
    S = F.state_from(U0)
    for dt in dts:
        F.step(S, float(dt))
    F.sync()
    U32 = F.to_f64(S)
    F.close()
    del S
    l1, linf = [], []
    for f in range(5):
        d = (U32[f] - U64[f]).abs()
        ref = U64[f].abs()
        s1, sinf = float(ref.sum()), float(ref.max())
        if sinf == 0.0:
            s1, sinf = float(U64.abs().sum()) / 5, float(U64.abs().max())
        l1.append(float(f"{float(d.sum()) / s1:.3e}"))
        linf.append(float(f"{float(d.max()) / sinf:.3e}"))
    return l1, linf


def equal_cost_plain(net, alpha, seed, eval_steps, n):
    """The corrected n^3 solve against a plain FP32 solve on a finer mesh of
    about the same cost, both measured against one finer reference: the
    held-out problem `seed` is sampled on a (3n)^3 mesh, solved there in
    FP64, and its conservative averages over 3^3 and 2^3 cells give the
    n^3 and (3n/2)^3 references (and the initial states of the coarse
    solves).  The n^3 solves take the plain n^3 run's own CFL steps; the
    (3n/2)^3 solve takes its own CFL steps to the same end time."""
    import numpy as np
    import torch
    import torch.nn.functional as tf
    import workloads as wl
    from paper_1812_07977_amd import Fluid
    r, m = 3 * n, 3 * n // 2
    U0 = torch.from_numpy(wl.random_plane(r, r, r, seed=seed)).cuda()

    def avg(U, k):
        return tf.avg_pool3d(U.unsqueeze(0), k).squeeze(0).contiguous()

    def l1(ref, S, F):
        d = (F.to_f64(S) - ref).abs().sum(dim=(1, 2, 3))
        a = ref.abs().sum(dim=(1, 2, 3))
        return [round(float(d[list(g)].sum() / a[list(g)].sum()), 5) for g in ((0,), (1, 2, 3), (4,))]

    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)

    def timed(fn):
        torch.cuda.synchronize()
        ev0.record()
        fn()
        ev1.record()
        torch.cuda.synchronize()
        return ev0.elapsed_time(ev1)

    Cn = Fluid((n,) * 3, bc="periodic", dtype="f32")
    plain = Cn.state_from(avg(U0, 3))
    dts = []
    for _ in range(eval_steps):
        dt = Cn.dt(plain)
        dts.append(dt)
        Cn.step(plain, dt)
    T = float(sum(dts))
    corr = Cn.state_from(avg(U0, 3))

    def corrected():
        for dt in dts:
            Cn.step(corr, dt)
            if alpha > 0:
                net.correct(corr)
    ms_corr = timed(corrected)
    Cm = Fluid((m,) * 3, bc="periodic", dtype="f32")
    fine_m = Cm.state_from(avg(U0, 2))
    # count the finer solve's own CFL steps to T, then time exactly those
    log = torch.zeros(4 * eval_steps, dtype=torch.float64, device="cuda")
    Cm.time = 0.0
    Cm.advance(fine_m, 4 * eval_steps, T, log)
    Cm.sync()
    steps_m = int((log > 0).sum())
    fine_m = Cm.state_from(avg(U0, 2))
    Cm.time = 0.0
    ms_m = timed(lambda: Cm.advance(fine_m, steps_m, T))
    Fr = Fluid((r,) * 3, bc="periodic", dtype="f64")
    Ur = U0.clone()
    del U0
    Fr.time = 0.0
    Fr.advance(Ur, 8 * eval_steps, T)
    Fr.sync()
    out = {
        "reference": f"{r}^3 FP64 solve of seed {seed} to t = {T:.5f}, averaged over 3^3 and 2^3 cells",
        f"corrected_{n}": {"ms": round(ms_corr, 2), "l1": l1(avg(Ur, 3), corr, Cn)},
        f"plain_{n}": {"l1": l1(avg(Ur, 3), plain, Cn)},
        f"plain_{m}": {"ms": round(ms_m, 2), "steps": steps_m, "l1": l1(avg(Ur, 2), fine_m, Cm)},
        "l1_fields": ["rho", "momentum (all components)", "E"],
    }
    for F in (Cn, Cm, Fr):
        F.close()
    return out


def learned_form(n=128, iters=8000, eval_steps=200, stride=10,
                 eval_seeds=(99, 98, 97, 96, 95, 94, 93, 92)):
    """The learned-correction form on the coarse/fine pair n^3 / (2n)^3
    (periodic unit cubes): train the network on fine FP64 runs restricted
    2:1 (seeded random-plane Riemann problems and sine waves), then time, to
    the same end time on a held-out Riemann problem, the fine FP64 solve, the
    plain coarse FP32 solve and the corrected coarse FP32 solve, and measure
    both coarse solves' L1 errors against the restricted fine solve on each
    held-out problem (timings from the first)."""
    import numpy as np
    import torch
    import workloads as wl
    from paper_1812_07977_amd import Fluid
    from paper_1812_07977_amd import learned as L
    f = 2 * n
    t0 = time.perf_counter()
    net = L.CorrectionNet((n, n, n))
    net.set_params(L.init_params(0))
    net.set_norm(np.zeros(5), np.ones(5), np.ones(5))

    def sine(seed):
        rng = np.random.default_rng(seed)
        k = tuple(int(v) for v in rng.integers(-2, 3, 3))
        k = (1, 1, 1) if k == (0, 0, 0) else k
        v = tuple(float(x) for x in rng.uniform(-1, 1, 3))
        return wl.sine_wave(f, f, f, k=k, v=v, amp=0.2)

    states = [torch.from_numpy(wl.random_plane(f, f, f, seed=s)).cuda() for s in range(12)]
    states += [torch.from_numpy(sine(s)).cuda() for s in (100, 101, 102, 103)]
    # training states spread over the whole evaluated time window
    inputs, raw = L.generate_samples(net, states, eval_steps, stride=stride)
    mu, sigma, tau = L.normalisation(inputs, raw)
    net.set_norm(mu, sigma, tau)
    tt = torch.tensor(tau, dtype=torch.float32, device="cuda")[:, None, None, None]
    targets = [r / tt for r in raw]
    del raw
    L.train(net, inputs, targets, iters, lr=3e-4)
    del inputs, targets
    del states
    # blend factor fitted on validation problems (neither trained on nor
    # evaluated), so that a correction that does not generalise is damped
    val = [torch.from_numpy(wl.random_plane(f, f, f, seed=s)).cuda() for s in (50, 51, 52)]
    alpha, blend_errs = L.fit_blend(net, val, eval_steps, alphas=(0.0, 0.25, 0.5, 0.75, 1.0))
    del val
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0

    Cp = Fluid((n,) * 3, bc="periodic", dtype="f32")
    Ff = Fluid((f,) * 3, bc="periodic", dtype="f64")
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)

    def timed(fn):
        torch.cuda.synchronize()
        ev0.record()
        fn()
        ev1.record()
        torch.cuda.synchronize()
        return ev0.elapsed_time(ev1)

    per_seed = []
    for seed in eval_seeds:
        U0 = torch.from_numpy(wl.random_plane(f, f, f, seed=seed)).cuda()
        # the time grid: the plain coarse run's own CFL steps
        plain = net.restrict(U0)
        dts = []
        for _ in range(eval_steps):
            dt = Cp.dt(plain)
            dts.append(dt)
            Cp.step(plain, dt)
        T = float(sum(dts))
        plain = net.restrict(U0)
        ms_plain = timed(lambda: [Cp.step(plain, dt) for dt in dts])
        corr = net.restrict(U0)
        a0, f0 = net.counts()

        def corrected():
            for dt in dts:
                Cp.step(corr, dt)
                if alpha > 0:
                    net.correct(corr)
        ms_corr = timed(corrected)
        a1, f1 = net.counts()
        # the fine FP64 solve to the same time: count its steps once, then time
        Uf = U0.clone()
        log = torch.zeros(8 * eval_steps, dtype=torch.float64, device="cuda")
        Ff.time = 0.0
        Ff.advance(Uf, 8 * eval_steps, T, log)
        Ff.sync()
        nfine = int((log > 0).sum())
        Uf = U0.clone()
        Ff.time = 0.0
        ms_fine = timed(lambda: Ff.advance(Uf, nfine, T))
        errs = L._errors(net, Uf, plain, corr)
        per_seed.append(dict(seed=seed, T=T, ms_plain=ms_plain, ms_corr=ms_corr, ms_fine=ms_fine,
                             nfine=nfine, applied=a1 - a0, fallbacks=f1 - f0,
                             corr=[round(x, 5) for x in errs["l1_corrected"]],
                             plain=[round(x, 5) for x in errs["l1_plain"]]))
        del U0, Uf, plain, corr
    Ff.close()
    Cp.close()
    equal_cost = equal_cost_plain(net, alpha, eval_seeds[0], eval_steps, n)
    net.close()
    first = per_seed[0]
    ratios = [float(np.mean(r["corr"]) / np.mean(r["plain"])) for r in per_seed]
    return {
        "workload": f"held-out random-plane Riemann problems (seeds {list(eval_seeds)}), {n}^3 coarse "
                    f"FP32 + network vs {f}^3 FP64, {eval_steps} coarse steps each (timings: seed "
                    f"{first['seed']}, to t = {first['T']:.5f})",
        "value": n ** 3 * eval_steps / (first["ms_corr"] / 1e3), "unit": "coarse cell-updates/s",
        "ms_corrected": round(first["ms_corr"], 2), "ms_plain_coarse": round(first["ms_plain"], 2),
        "ms_fine_f64": round(first["ms_fine"], 2), "fine_steps": first["nfine"],
        "speedup_vs_f64": round(first["ms_fine"] / first["ms_corr"], 3),
        "l1_rel_err_corrected": first["corr"],
        "l1_rel_err_plain_coarse": first["plain"],
        "l1_fields": ["rho", "momentum (all components)", "E"],
        "error_vs": f"the {f}^3 FP64 solve restricted 2:1 at the same time",
        "per_seed": [{k: r[k] for k in ("seed", "corr", "plain", "applied", "fallbacks")}
                     for r in per_seed],
        "mean_l1_ratio_corrected_over_plain": round(float(np.mean(ratios)), 4),
        "worst_l1_ratio_corrected_over_plain": round(float(np.max(ratios)), 4),
        "best_l1_ratio_corrected_over_plain": round(float(np.min(ratios)), 4),
        "fraction_improved": round(float(np.mean([r < 1.0 for r in ratios])), 4),
        "l1_ratio_per_seed": {str(r["seed"]): round(q, 4) for r, q in zip(per_seed, ratios)},
        "corrections_applied": first["applied"], "fallbacks": first["fallbacks"], "blend": alpha,
        "blend_fit_l1": {str(k): round(v, 5) for k, v in blend_errs.items()},
        "blend_fit_on": "random-plane Riemann problems, seeds 50-52 (validation)",
        "equal_cost": equal_cost,
        "training": f"{iters} Adam steps on 16 trajectories x {eval_steps // stride} states "
                    f"(every {stride}th of {eval_steps} steps; {f}^3 FP64 restricted), "
                    f"{t_train:.1f} s incl. data",
    }


def batched_form(dtype, steps=20, count=64, seed=1):
    """The batched form: count seeded random-plane Riemann problems with
    meshes drawn from 32..160 per axis (periodic), each with its own device
    time step, advanced as one autotuned batch (one captured graph replay per
    step) and, from the same inputs, one problem at a time through the
    single-problem path; whole-batch cell-updates/s of both."""
    import torch
    import workloads as wl
    from paper_1812_07977_amd import Fluid
    from paper_1812_07977_amd.batch import Batch
    dims, probs = wl.random_batch(count, seed)
    cells = sum(nx * ny * nz for nx, ny, nz in dims)
    handles = [Fluid((nx, ny, nz), bc="periodic", dtype=dtype) for nx, ny, nz in dims]
    init = [F.state_from(U0) for F, U0 in zip(handles, probs)]
    del probs
    states = [S.clone() for S in init]
    B = Batch(dims, states, bc="periodic", dtype=dtype)
    t0 = time.perf_counter()
    ty, kz, _ = B.autotune()
    t_tune = time.perf_counter() - t0
    B.advance(2)                                   # warm-up (captures the graphs)
    B.sync()
    for S, S0 in zip(states, init):
        S.copy_(S0)
    B.close()
    B = Batch(dims, states, bc="periodic", dtype=dtype)
    B.set_launch(ty, kz)
    B.advance(1)
    B.sync()
    for S, S0 in zip(states, init):
        S.copy_(S0)
    B.close()
    B = Batch(dims, states, bc="periodic", dtype=dtype)
    B.set_launch(ty, kz)
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    ev0.record()
    B.advance(steps)
    ev1.record()
    B.sync()
    torch.cuda.synchronize()
    ms_batch = ev0.elapsed_time(ev1)
    B.close()
    # one problem at a time, default launch shape of the single-problem path
    seq = [S.clone() for S in init]
    for F, S in zip(handles, seq):
        F.advance(S, 1)
    torch.cuda.synchronize()
    seq = [S.clone() for S in init]
    torch.cuda.synchronize()
    ev0.record()
    for F, S in zip(handles, seq):
        F.advance(S, steps)
    ev1.record()
    torch.cuda.synchronize()
    ms_seq = ev0.elapsed_time(ev1)
    for F in handles:
        F.close()
    return {
        "workload": f"{count} random-plane Riemann problems, meshes 32..160 per axis "
                    f"(seed {seed}), {cells / 1e6:.1f} M cells, periodic, {steps} steps, "
                    "per-problem device dt",
        "value": cells * steps / (ms_batch / 1e3), "unit": "cell-updates/s",
        "ms_per_step": ms_batch / steps,
        "sequential_value": cells * steps / (ms_seq / 1e3),
        "speedup_vs_one_at_a_time": round(ms_seq / ms_batch, 3),
        "launch": {"tile_y": ty, "chunk_z": kz, "autotune_s": round(t_tune, 2)},
    }


def add_ceiling(roof, ceil):
    """The dominant kernel's rate against the probe's ceiling for its
    read:write mix (the second substep reads two arrays per array written:
    the add mix; the first reads one: the copy mix), the better of the
    plain and non-temporal stores."""
    mix = "add_2to1" if "substep 2" in roof["kernel"] else "copy_1to1"
    c = max(ceil[mix], ceil[mix + "_nt"])
    roof["ceiling_gbs"] = c
    roof["ceiling_mix"] = mix
    roof["frac_of_ceiling"] = round(roof["achieved"] / c, 4)


def case_entry(case, n, dtype, steps, warmup, ceil, U0=None):
    """One more timed configuration: the same measurement as the headline
    (device dt, `steps` steps after `warmup`) for another case, size or
    form; returns (entry, dts, FP64 result or None, U0)."""
    if U0 is None:
        U0 = make_input(n, case)
    r, dts, res = timed_run(U0, n, dtype, steps, warmup, 0, 0, case=case)
    cells = n ** 3
    ms = r["total_ms"] / steps
    roof, _ = roofline(dtype, n, case, r["per_kernel"])
    add_ceiling(roof, ceil)
    bpc = 200.0 if dtype == "f64" else 180.0
    entry = {
        "workload": f"{'sine' if case == 'sine' else 'random-plane Riemann (seed 0)'} {n}^3 "
                    f"periodic, {dtype.upper()}, device dt",
        "value": cells * steps / (r["total_ms"] / 1e3), "unit": "cell-updates/s",
        "ms_per_step": round(ms, 4),
        "hbm_gbs_algorithmic": round(bpc * cells / (ms / 1e3) / 1e9, 1),
        "per_kernel_avg_ms": {KERNEL_NAMES[k]: round(v[0] / max(v[1], 1), 4)
                              for k, v in r["per_kernel"].items()},
        "roofline": {k: roof[k] for k in ("kernel", "achieved", "frac", "frac_of_ceiling",
                                          "avg_launch_ms")},
    }
    return entry, dts, res, U0


def other_cases(args, ceil, headline):
    """The rest of the per-GPU configurations beside the headline: the
    random-plane Riemann case (seed 0) and the smooth case at each of the
    sizes in --case-sizes (default 512^3 and 256^3), FP64 and the FP32 form;
    for the FP32 form of the Riemann case at the largest size also its L1 /
    L-infinity error per field against FP64."""
    out = {}
    sizes = [int(v) for v in args.case_sizes.split(",") if v]
    for n, case in [(m, c) for m in sizes for c in ("plane", "sine")]:
        if (case, n) == headline:
            continue
        print(f"bench: case {case} {n}^3", file=sys.stderr, flush=True)
        e64, dts, U64, U0 = case_entry(case, n, "f64", args.steps, args.warmup, ceil)
        e32, _, _, _ = case_entry(case, n, "f32", args.steps, args.warmup, ceil, U0=U0)
        e32["speedup_vs_f64"] = round(e64["ms_per_step"] / e32["ms_per_step"], 3)
        if n == max(sizes) and case == "plane":
            l1, linf = f32_error(U0, n, dts, U64)
            e32["l1_rel_err"], e32["linf_rel_err"] = l1, linf
            e32["error_vs"] = (f"FP64 solution of the same input after the same "
                               f"{args.warmup + args.steps} steps (same dt sequence)")
        del U64, U0
        key = f"{case}_{n}"
        out[key + "_f64"] = e64
        out[key + "_f32"] = e32
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--size", type=int, default=512)
    ap.add_argument("--case", choices=["sine", "plane"], default="sine")
    ap.add_argument("--tile-y", type=int, default=0)
    ap.add_argument("--chunk-z", type=int, default=0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-forms", action="store_true", help="time the FP64 form only")
    ap.add_argument("--no-cases", action="store_true",
                    help="skip the other per-GPU cases (512^3 Riemann, 256^3 sine and Riemann)")
    ap.add_argument("--case-sizes", default="512,256",
                    help="mesh sizes of the other per-GPU cases (comma list)")
    ap.add_argument("--forms", default="f32,batch,learned",
                    help="comma list of the forms to run beside FP64: f32, batch, learned")
    ap.add_argument("--learned-iters", type=int, default=8000,
                    help="Adam steps of the learned form's training")
    ap.add_argument("--copy-probe", type=int, default=0,
                    help="also run one plain device copy of this many MiB (counter scaling)")
    args = ap.parse_args()

    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); the library has no "
              "multi-GPU path", file=sys.stderr)
        sys.exit(2)

    import torch

    n = args.size
    print(f"bench: {args.case} {n}^3 periodic, FP64, warmup {args.warmup}, steps {args.steps}",
          file=sys.stderr, flush=True)
    U0 = make_input(n, args.case)

    if args.copy_probe:
        # a plain streaming kernel of known size for scaling HBM counters:
        # an elementwise negation reads copy_probe MiB and writes as many
        nb = args.copy_probe * 1024 * 1024 // 8
        a = torch.ones(nb, dtype=torch.float64, device="cuda")
        b = torch.empty_like(a)
        torch.neg(a, out=b)
        torch.cuda.synchronize()
        del a, b

    r64, dts64, U64 = timed_run(U0, n, "f64", args.steps, args.warmup, args.tile_y, args.chunk_z,
                                repeats=5, host_steps=20, case=args.case)
    print("bench: HBM ceilings (streaming probe)", file=sys.stderr, flush=True)
    ceil = hbm_ceilings()

    cells = n ** 3
    ms_per_step = r64["total_ms"] / args.steps
    rate = cells * args.steps / (r64["total_ms"] / 1e3)
    alg_bytes_step = 200.0 * cells + 40.0 * cells / args.steps
    roof, alu = roofline("f64", n, args.case, r64["per_kernel"])
    add_ceiling(roof, ceil)
    step_gbs = alg_bytes_step / (ms_per_step / 1e3) / 1e9

    line = {
        "metric": METRIC, "value": rate, "unit": "cell-updates/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_per_step,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"{args.case} {n}^3 periodic cube, FP64, minmod PLM + HLL + RK2, "
                               f"CFL 0.5, device dt", "grid": [n, n, n], "case": args.case,
                   "gamma": 1.4, "cfl": 0.5, "bc": "periodic"},
        "hbm_gbs_algorithmic": round(step_gbs, 1),
        "step_frac_of_hbm_peak": round(step_gbs / HBM_PEAK_GBS, 4),
        "per_kernel_avg_ms": {KERNEL_NAMES[k]: round(v[0] / max(v[1], 1), 4)
                              for k, v in r64["per_kernel"].items()},
        "per_kernel_note": "HIP events around every launch, in a separate block of the same "
                           f"{args.steps} steps right after the timed one (the timed block "
                           "records no per-kernel events)",
        "sim_time": r64["t_sim"],
        "repeats": {"blocks": len(r64["repeat_ms"]), "steps_each": args.steps,
                    "cell_updates_per_s": [round(cells * args.steps / (t / 1e3)) for t in r64["repeat_ms"]],
                    "median": round(cells * args.steps / (sorted(r64["repeat_ms"])[len(r64["repeat_ms"]) // 2] / 1e3))},
        "host_dt": {"value": cells * r64["host_steps"] / (r64["host_dt_ms"] / 1e3),
                    "unit": "cell-updates/s", "steps": r64["host_steps"],
                    "ms_per_step": r64["host_dt_ms"] / r64["host_steps"],
                    "note": "gs_fluid_dt (reduction + 8-byte read-back + sync) then gs_fluid_step, "
                            "240 B/cell-update"},
        "host_dt_last": {"value": cells * r64["host_steps"] / (r64["host_dt_last_ms"] / 1e3),
                         "unit": "cell-updates/s", "steps": r64["host_steps"],
                         "ms_per_step": r64["host_dt_last_ms"] / r64["host_steps"],
                         "note": "gs_fluid_step_dt (the step with its fused max, then an 8-byte "
                                 "read-back + sync, no reduction), 200 B/cell-update"},
        "hbm_ceiling_gbs": ceil,
        "roofline": roof,
        "alu": alu,
        "context": "paper: ~12X wall-time speedup of one V100 over 7 Power9 cores "
                   "(Summit, 256^3 per rank, incl. host transfers)",
    }

    if not args.no_cases:
        line["cases"] = other_cases(args, ceil, (args.case, n))

    forms = set() if args.no_forms else {f for f in args.forms.split(",") if f}
    line["forms"] = {}
    if "f32" in forms:
        print("bench: FP32 form", file=sys.stderr, flush=True)
        r32, _, _ = timed_run(U0, n, "f32", args.steps, args.warmup, args.tile_y, args.chunk_z)
        ms32 = r32["total_ms"] / args.steps
        roof32, alu32 = roofline("f32", n, args.case, r32["per_kernel"])
        add_ceiling(roof32, ceil)
        print("bench: FP32 form error against FP64", file=sys.stderr, flush=True)
        l1, linf = f32_error(U0, n, dts64, U64)
        line["forms"]["f32"] = {
            "value": cells * args.steps / (r32["total_ms"] / 1e3), "unit": "cell-updates/s",
            "ms_per_step": ms32, "speedup_vs_f64": round(ms_per_step / ms32, 3),
            "dtype": "f32 state and flux arithmetic; f64 primitive recovery, dt, totals",
            "hbm_gbs_algorithmic": round((180.0 * cells + 20.0 * cells / args.steps)
                                         / (ms32 / 1e3) / 1e9, 1),
            "per_kernel_avg_ms": {KERNEL_NAMES[k]: round(v[0] / max(v[1], 1), 4)
                                  for k, v in r32["per_kernel"].items()},
            "l1_rel_err": l1, "linf_rel_err": linf,
            "error_vs": f"FP64 solution of the same input after the same {args.warmup + args.steps} "
                        "steps (same dt sequence)",
            "roofline": roof32, "alu": alu32}
    del U64
    if "batch" in forms:
        print("bench: batched form", file=sys.stderr, flush=True)
        line["forms"]["batch_f64"] = batched_form("f64")
        line["forms"]["batch_f32"] = batched_form("f32")
    if "learned" in forms:
        print("bench: learned-correction form (training, then timing)", file=sys.stderr, flush=True)
        line["forms"]["learned"] = learned_form(iters=args.learned_iters)

    if not args.no_cpu_baseline:
        print("bench: timing the CPU oracle on a bounded sample", file=sys.stderr, flush=True)
        line["cpu_baseline"] = cpu_baseline(args.case)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
