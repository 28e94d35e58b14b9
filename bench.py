"""Benchmark of the e-ph collision integral on one MI355X.

Workload: the tight-binding transport system (4-band cubic model on a 100^3
k grid, 0.3 eV window, 50^3 q grid, 3 Debye + 3 Einstein modes, lognormal
|g|^2, sigma = 8 meV, ~2e8 unordered channels), synthetic and seeded.

A step is one evaluation of I[f] (Eq. 2) over every channel at B = 1 in FP64
-- the operator every other form is built from -- by the plan's default
pass (single copy over pair records).  `value` is scattering channels per
second of that step with all inputs resident in HBM.  The other forms (the
other layouts, FP32, forward + reverse, B = 64 with its ALU roofline, RK4
step, transport iteration, phonon side, coupled step, CPU oracle on all host
cores) are timed after the main loop and reported under "forms".

Prints one JSON line.  Options: --steps K --warmup W --gpus 1 [--quick]
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

HBM_PEAK_GBS = 8000.0
# Algorithmic bytes per unordered channel.  The single-copy pass over entries
# streams one entry per channel (|g|^2 + packed partner/mode word); the
# per-row pass streams both entries of each channel.  The single-copy pass
# over pair records (the default where they are built) streams one partner
# word per state pair and one |g|^2 per mode slot: pair_bytes() below.
BYTES_PER_CHANNEL_ENTRIES = {"f64": 12.0, "f32": 8.0}
BYTES_PER_CHANNEL_ROWS = {"f64": 24.0, "f32": 16.0}


LAYOUT_NAMES = {1: "duplicated rows", 2: "single copy, one entry per channel",
                3: "single copy over pair records"}
KERNEL_OF_LAYOUT = {1: "k_fwd_tiled", 2: "k_fwd_sym", 3: "k_fwd_pairs"}


# Published MI355X vector peaks (TFLOP/s) for the ALU-bound batched passes
VECTOR_PEAK_TFLOPS = {"f64": 78.6, "f32": 157.3}


def batched_alu_roofline(ms, dtype, pairs, entries, B, reverse=False):
    """ALU roofline of a B-vector pass from its algorithmic floating-point
    operations: per entry the coefficients (two Gaussians and about 20 other
    operations: 30 counted), per merged run of one partner (one pair, both
    orientations: 2 x pairs runs) and vector 5 operations forward
    (acc_a += a (1 - f), acc_b += b f) or 12 reverse (u, the two sums over
    the vectors' products, and the dL/df accumulation)."""
    flops = 30.0 * entries + (12.0 if reverse else 5.0) * 2.0 * pairs * B
    achieved = flops / (ms * 1e-3) / 1e12
    peak = VECTOR_PEAK_TFLOPS[dtype]
    return {"bound": "alu", "achieved": achieved, "peak": peak, "unit": "TFLOP/s", "frac": achieved / peak,
            "flops_per_pass": flops}


def pair_bytes(info, n_modes, dtype):
    """Bytes per channel of the pass the plan runs at B = 1: pair records
    (4 B partner + n_modes |g|^2 slots per pair) or one entry per channel."""
    if info["layout"] == 3 and info["pair_records"] > 0:
        es = 8 if dtype == "f64" else 4
        return info["pair_records"] * (4 + n_modes * es) / info["channels_kept"]
    return BYTES_PER_CHANNEL_ENTRIES[dtype]
# reverse pass: the same entry stream, the channel index of the entry that
# writes dL/d|g|^2 (4 B) and that FP64 value (8 B), per unordered channel
VJP_BYTES_PER_CHANNEL = {"f64": 24.0 + 4.0 + 8.0, "f32": 16.0 + 4.0 + 8.0}


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def kernels_source_hash():
    import hashlib
    with open(os.path.join(ROOT, "paper_2511_03683_amd", "csrc", "kernels.hpp"), "rb") as fh:
        return hashlib.sha256(fh.read()).hexdigest()[:16]


def profiled_traffic(tag):
    """HBM bytes per launch of the kernel `tag`, from the committed counter
    summary under profiles/ (FETCH_SIZE and WRITE_SIZE scaled by a copy
    kernel), or None when there is none or the kernel source has changed
    since the counters were taken."""
    import glob
    h = kernels_source_hash()
    for path in sorted(glob.glob(os.path.join(ROOT, "profiles", "*.txt"))):
        kv = {}
        with open(path) as fh:
            for line in fh:
                if ":" in line:
                    k, v = line.split(":", 1)
                    kv[k.strip()] = v.strip()
        if kv.get("kernel_tag") == tag and kv.get("kernels_hpp_sha256_16") == h:
            try:
                return float(kv["traffic_bytes_per_launch"])
            except (KeyError, ValueError):
                return None
    return None


def transport_solve(E, plan, f0, vel, nph, timed, tol=1e-8, max_iter=2000):
    """Mobility at 300 K iterated to a relative change of tol (or to the
    working precision's floor), timed as one call."""
    res = {}

    def run():
        res.update(E.iterate_transport(plan, f0, vel, 300.0, nph, tol=tol, max_iter=max_iter))

    ms, _ = timed(run, 1, 0)
    mu = res["mu"]
    out = dict(tol=tol, iterations=res["iters"], converged=res["converged"],
               stagnated=res["stagnated"], last_relative_change=res["resid"], ms_total=ms,
               mobility_xx_cm2_per_Vs=float(mu[0, 0]), mobility_yy_cm2_per_Vs=float(mu[1, 1]))
    log(f"transport solve: {res['iters']} iterations, converged={res['converged']} "
        f"stagnated={res['stagnated']} change={res['resid']:.2e}, mu_xx={mu[0, 0]:.2f} cm2/Vs, "
        f"{ms:.1f} ms")
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--quick", action="store_true", help="smaller system (for a fast check)")
    ap.add_argument("--no-forms", action="store_true")
    ap.add_argument("--batch-only", action="store_true",
                    help="after the main step run only the B = 64 forward and reverse passes "
                         "(for tracing the batched kernels)")
    ap.add_argument("--single-only", action="store_true",
                    help="after the main step run only the B = 1 reverse pass, the phonon-side "
                         "rate and the transport iterations (for tracing their kernels)")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--cpu-channels", type=int, default=20_000_000,
                    help="channels of the one-core oracle timing")
    ap.add_argument("--dtype", choices=("f64", "f32"), default="f64",
                    help="precision of the main step (f32 only with --no-forms, for profiling)")
    ap.add_argument("--copy-calib", action="store_true",
                    help="also run a plain 1 GiB read + 1 GiB write elementwise kernel "
                         "(hardware-counter calibration)")
    args = ap.parse_args()
    if args.dtype != "f64" and not (args.no_forms or args.batch_only or args.single_only):
        ap.error("--dtype f32 times the main step only; add --no-forms or --batch-only")
    if args.batch_only or args.single_only:
        args.no_forms = True
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(the destination-sharded design is described in DESIGN.md)", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_2511_03683_amd as E
    import synth

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    stream = torch.cuda.Stream(device=dev)

    if args.copy_calib:
        a = torch.ones(1 << 28, dtype=torch.float32, device=dev)
        b = torch.empty_like(a)
        for _ in range(3):
            torch.mul(a, 1.0, out=b)
        torch.cuda.synchronize()
        log("copy calibration: 3 x (1 GiB read + 1 GiB write) elementwise kernels")
        del a, b

    # a plain device copy (1 GiB read + 1 GiB write) as the practical HBM ceiling
    src = torch.ones(1 << 27, dtype=torch.float64, device=dev)
    dst = torch.empty_like(src)
    for _ in range(2):
        dst.copy_(src)
    torch.cuda.synchronize()
    c0, c1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    c0.record()
    for _ in range(10):
        dst.copy_(src)
    c1.record()
    torch.cuda.synchronize()
    copy_gbps = 2.0 * src.numel() * 8 * 10 / (c0.elapsed_time(c1) * 1e-3) / 1e9
    log(f"device copy: {copy_gbps:.0f} GB/s")
    del src, dst

    t0 = time.time()
    if args.quick:
        s = synth.tb_system(kn=60, qn=30, target_states=5000)
        wname = "tb60_q30_6modes"
    else:
        s = synth.tb_system()
        wname = "tb100_q50_6modes"
    log(f"system {wname}: S={s.n_states} channels={s.n_channels} ({time.time() - t0:.1f}s)")
    rng = np.random.default_rng(2511)
    f_np = np.clip(synth.fermi_dirac(s.eps, 0.05, 300.0) * (0.8 + 0.4 * rng.uniform(size=s.n_states)), 0, 1)
    nph_np = s.nph(300.0)
    nch = s.n_channels

    def tens(a, dt):
        return torch.as_tensor(np.ascontiguousarray(a), dtype=dt, device=dev)

    t0 = time.time()
    mdt = torch.float64 if args.dtype == "f64" else torch.float32
    plan64 = E.build_channels(s, dtype=args.dtype, device=0)
    info64 = E.plan_info(plan64)
    layout64 = info64["layout"]
    bpc = pair_bytes(info64, s.n_modes, args.dtype)
    log(f"{args.dtype} plan built ({time.time() - t0:.1f}s), info={info64}, {bpc:.3f} B per channel")
    f64, n64 = tens(f_np, mdt), tens(nph_np, mdt)
    I64 = torch.empty_like(f64)

    def timed(fn, reps, warm):
        with torch.cuda.stream(stream):
            for _ in range(warm):
                fn()
        stream.synchronize()
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        w0 = time.perf_counter()
        with torch.cuda.stream(stream):
            ev0.record(stream)
            for _ in range(reps):
                fn()
            ev1.record(stream)
        stream.synchronize()
        torch.cuda.synchronize()
        wall = time.perf_counter() - w0
        return ev0.elapsed_time(ev1) / reps, wall

    fwd64 = lambda: E.collision_integral(plan64, f64, n64, out=I64)

    def settle(fn, secs=0.25):
        # untimed passes for a quarter of a second, so that timed steps see the
        # device in its steady state (clocks, first touches of fresh pages) as
        # a serving loop would: after the plan is built, and after a tuning
        # change (which re-tiles on the host while the device idles)
        t_s, n_s = time.perf_counter(), 0
        while time.perf_counter() - t_s < secs:
            with torch.cuda.stream(stream):
                for _ in range(20):
                    fn()
            stream.synchronize()
            n_s += 20
        return n_s

    def retune(plan, fn, **kw):
        E.set_tuning(plan, **kw)
        settle(fn)

    # then the W warmup steps
    n_settle = settle(fwd64)
    with torch.cuda.stream(stream):
        for _ in range(args.warmup):
            fwd64()
    stream.synchronize()
    # the library brackets each launch of the forward kernel with HIP events on
    # its stream during the timed steps: the kernel's own mean launch duration
    E.kernel_timing(plan64, True)
    ms, wall = timed(fwd64, args.steps, 0)
    kernel_ms, kernel_launches = E.kernel_timing(plan64, False)
    if kernel_launches != args.steps:
        raise RuntimeError(f"{kernel_launches} timed kernel launches for {args.steps} steps")
    value = nch / (ms * 1e-3)
    achieved = bpc * nch / (ms * 1e-3) / 1e9
    kernel_gbps = bpc * nch / (kernel_ms * 1e-3) / 1e9
    log(f"fwd {args.dtype}: {ms:.3f} ms/eval, {value:.3e} ch/s, {achieved:.0f} GB/s algorithmic "
        f"(wall {wall:.2f}s for {args.steps}); kernel alone {kernel_ms:.3f} ms, {kernel_gbps:.0f} GB/s")

    forms = {}

    def vjp_b1(reps):
        lam = tens(rng.normal(size=s.n_states), torch.float64)
        gg = torch.zeros(nch, dtype=torch.float64, device=dev)
        ms_v, _ = timed(lambda: E.collision_vjp(plan64, f64, n64, lam, want_f=True, gg2=gg), reps, 1)
        forms["vjp_f64_b1"] = dict(ms=ms_v, channels_per_s=nch / (ms_v * 1e-3),
                                   algorithmic_GBps=VJP_BYTES_PER_CHANNEL["f64"] * nch / (ms_v * 1e-3) / 1e9)
        return ms_v

    def phonon_rate(reps):
        dN = torch.empty((s.n_q, s.n_modes), dtype=torch.float64, device=dev)
        msp, _ = timed(lambda: E.phonon_rate(plan64, f64, n64, out=dN), reps, 1)
        forms["phonon_rate_f64"] = dict(ms=msp, channels_per_s=nch / (msp * 1e-3),
                                        bins=int(s.n_q * s.n_modes),
                                        note="channels grouped by phonon pair {q, -q}; one wave per "
                                             "chunk of pair records, no atomics")
        log(f"phonon rate fp64: {msp:.3f} ms")

    def transport_iter():
        vel = tens(s.vel, torch.float64)
        f0 = tens(synth.fermi_dirac(s.eps, -0.1, 300.0), torch.float64)
        t1, _ = timed(lambda: E.iterate_transport(plan64, f0, vel, 300.0, n64, tol=0.0, max_iter=1), 1, 1)
        t6, _ = timed(lambda: E.iterate_transport(plan64, f0, vel, 300.0, n64, tol=0.0, max_iter=6), 1, 0)
        forms["transport_iter_f64"] = dict(ms_per_iteration=(t6 - t1) / 5.0, ms_setup_plus_one=t1)
        log(f"transport fp64: {(t6 - t1) / 5:.3f} ms/iteration, setup+1 {t1:.3f} ms")
        return vel, f0

    if args.single_only:
        if args.dtype != "f64":
            ap.error("--single-only times the FP64 plan")
        ms_v = vjp_b1(args.steps)
        log(f"vjp fp64: {ms_v:.3f} ms")
        phonon_rate(args.steps)
        transport_iter()
    if args.batch_only:
        B = 64
        tuned = E.autotune(plan64, B)
        F = tens(synth.batch_occupations(s), mdt)
        IB = torch.empty_like(F)
        msb, _ = timed(lambda: E.collision_integral(plan64, F, n64, out=IB), args.steps, 1)
        LB = tens(rng.normal(size=(B, s.n_states)), mdt)
        ggb = torch.zeros(nch, dtype=torch.float64, device=dev)
        msbv, _ = timed(lambda: E.collision_vjp(plan64, F, n64, LB, want_f=True, gg2=ggb), args.steps, 1)
        forms[f"fwd_{args.dtype}_b64"] = dict(ms=msb, per_vector_channels_per_s=B * nch / (msb * 1e-3),
                                              batch_partners=tuned["batch_partners"])
        forms[f"vjp_{args.dtype}_b64"] = dict(ms=msbv, per_vector_channels_per_s=B * nch / (msbv * 1e-3))
        log(f"B=64 {args.dtype}: forward {msb:.3f} ms, reverse {msbv:.3f} ms")
        del F, IB, LB, ggb

    if not args.no_forms:
        forms["fwd_f64_b1"] = dict(ms=ms, channels_per_s=value, algorithmic_GBps=achieved,
                                   layout=LAYOUT_NAMES[layout64], bytes_per_channel=bpc)
        # the other layouts of the same pass: one entry per channel (single
        # copy without pair records) and the per-row pass (each channel
        # evaluated in both of its rows)
        if layout64 == 3:
            # the pair pass with the polynomial exponential (no LDS table reads)
            retune(plan64, fwd64, fp64_exp=2)
            msp2, _ = timed(fwd64, args.steps, args.warmup)
            retune(plan64, fwd64, fp64_exp=1)
            forms["fwd_f64_b1_pairs_polyexp"] = dict(ms=msp2, channels_per_s=nch / (msp2 * 1e-3),
                                                     algorithmic_GBps=bpc * nch / (msp2 * 1e-3) / 1e9)
            log(f"fwd fp64 pair records, polynomial exponential: {msp2:.3f} ms")
            # the pair passes with the records of each tile in destination
            # order (the default sorts them by q)
            retune(plan64, fwd64, pair_order=2)
            msd, _ = timed(fwd64, args.steps, args.warmup)
            msdv = vjp_b1(max(3, args.steps // 4))
            retune(plan64, fwd64, pair_order=1)
            forms["fwd_f64_b1_pairs_destination_order"] = dict(
                ms=msd, reverse_ms=msdv, channels_per_s=nch / (msd * 1e-3),
                algorithmic_GBps=bpc * nch / (msd * 1e-3) / 1e9)
            log(f"fwd / vjp fp64 pair records in destination order: {msd:.3f} / {msdv:.3f} ms")
            # q order in groups of 64 table rows: a destination's records stay
            # together inside a group, so the reverse pass's dL/d|g|^2 writes
            # are more contiguous
            retune(plan64, fwd64, pair_rows=64)
            msg, _ = timed(fwd64, args.steps, args.warmup)
            msgv = vjp_b1(max(3, args.steps // 4))
            retune(plan64, fwd64, pair_rows=1)
            forms["fwd_f64_b1_pairs_rows64"] = dict(
                ms=msg, reverse_ms=msgv, channels_per_s=nch / (msg * 1e-3),
                algorithmic_GBps=bpc * nch / (msg * 1e-3) / 1e9)
            log(f"fwd / vjp fp64 pair records in q order by groups of 64 rows: {msg:.3f} / {msgv:.3f} ms")
            retune(plan64, fwd64, layout=2)
            mse, _ = timed(fwd64, args.steps, args.warmup)
            forms["fwd_f64_b1_entries"] = dict(ms=mse, channels_per_s=nch / (mse * 1e-3),
                                               algorithmic_GBps=BYTES_PER_CHANNEL_ENTRIES["f64"] * nch
                                               / (mse * 1e-3) / 1e9,
                                               layout="single copy, one entry per channel")
            log(f"fwd fp64 single copy over entries: {mse:.3f} ms")
        retune(plan64, fwd64, layout=1)
        msr, _ = timed(fwd64, args.steps, args.warmup)
        retune(plan64, fwd64, layout=layout64)
        forms["fwd_f64_b1_rows"] = dict(ms=msr, channels_per_s=nch / (msr * 1e-3),
                                        algorithmic_GBps=BYTES_PER_CHANNEL_ROWS["f64"] * nch / (msr * 1e-3) / 1e9,
                                        layout="duplicated rows")
        log(f"fwd fp64 per-row pass: {msr:.3f} ms")
        # reverse mode (dL/df and dL/dg2), FP64
        ms_v = vjp_b1(max(3, args.steps // 4))
        forms["fwd_plus_adjoint_f64_b1"] = dict(
            ms=ms + ms_v, channels_per_s=nch / ((ms + ms_v) * 1e-3),
            algorithmic_GBps=(bpc + VJP_BYTES_PER_CHANNEL["f64"]) * nch
            / ((ms + ms_v) * 1e-3) / 1e9)
        log(f"vjp fp64: {ms_v:.3f} ms")
        # batched B = 64: 16 temperatures x 4 fields, sub-tile size from the autotuner
        B = 64
        F_np = synth.batch_occupations(s)
        tuned = E.autotune(plan64, B)
        F = tens(F_np, torch.float64)
        IB = torch.empty_like(F)
        msb, _ = timed(lambda: E.collision_integral(plan64, F, n64, out=IB), 3, 1)
        npairs_b = max(info64["pair_records"], 1)
        forms["fwd_f64_b64"] = dict(ms=msb, per_vector_channels_per_s=B * nch / (msb * 1e-3),
                                    alu_roofline=batched_alu_roofline(msb, "f64", npairs_b, 2 * nch, B),
                                    ratio_vs_b1=(B * nch / (msb * 1e-3)) / value,
                                    batch_partners=tuned["batch_partners"],
                                    vectors="16 temperatures (100-400 K) x 4 fields (0-1e5 V/m)")
        log(f"fwd fp64 B=64: {msb:.3f} ms ({forms['fwd_f64_b64']['ratio_vs_b1']:.2f}x per vector, "
            f"sub-tile {tuned['batch_partners']})")
        # batched reverse mode: dL/df of the 64 vectors and dL/d|g|^2 summed over them
        LB = tens(rng.normal(size=(B, s.n_states)), torch.float64)
        ggb = torch.zeros(nch, dtype=torch.float64, device=dev)
        msbv, _ = timed(lambda: E.collision_vjp(plan64, F, n64, LB, want_f=True, gg2=ggb), 3, 1)
        forms["vjp_f64_b64"] = dict(ms=msbv, per_vector_channels_per_s=B * nch / (msbv * 1e-3),
                                    alu_roofline=batched_alu_roofline(msbv, "f64", npairs_b, 2 * nch, B, True),
                                    ratio_vs_b1=(B * nch / (msbv * 1e-3)) / (nch / (ms_v * 1e-3)))
        forms["fwd_plus_adjoint_f64_b64"] = dict(
            ms=msb + msbv, per_vector_channels_per_s=B * nch / ((msb + msbv) * 1e-3),
            ratio_vs_b1=(ms + ms_v) * B / (msb + msbv))
        log(f"vjp fp64 B=64: {msbv:.3f} ms ({forms['vjp_f64_b64']['ratio_vs_b1']:.2f}x per vector)")
        # the same 64 vectors, each with its own bath (Bose-Einstein at its
        # temperature): the batched pass with N per vector
        temps = np.repeat(np.linspace(100.0, 400.0, 16), 4)
        NB = tens(np.stack([s.nph(float(T)) for T in temps]), torch.float64)
        mspv, _ = timed(lambda: E.collision_integral(plan64, F, NB, out=IB), 3, 1)
        forms["fwd_f64_b64_bath_per_vector"] = dict(ms=mspv, per_vector_channels_per_s=B * nch / (mspv * 1e-3),
                                                    ratio_vs_shared_bath=mspv / msb,
                                                    baths="Bose-Einstein at each vector's temperature")
        log(f"fwd fp64 B=64, bath per vector: {mspv:.3f} ms ({mspv / msb:.2f}x the shared bath)")
        msvpv, _ = timed(lambda: E.collision_vjp(plan64, F, NB, LB, want_f=True, gg2=ggb), 3, 1)
        forms["vjp_f64_b64_bath_per_vector"] = dict(ms=msvpv, per_vector_channels_per_s=B * nch / (msvpv * 1e-3),
                                                    ratio_vs_shared_bath=msvpv / msbv)
        log(f"vjp fp64 B=64, bath per vector: {msvpv:.3f} ms ({msvpv / msbv:.2f}x the shared bath)")
        del F, IB, LB, ggb, NB
        # phonon side of the same processes (dN/dt of every (q, mode)), FP64
        phonon_rate(max(3, args.steps // 4))
        # transport iteration, FP64
        vel, f0 = transport_iter()
        forms["transport_solve_f64"] = transport_solve(E, plan64, f0, vel, n64, timed)
        del vel, f0
        # differentiation: adjoint through 200 RK4 steps (checkpoint every 20) of
        # L = sum eps f(T) / sum f(T), FP64
        eps = tens(s.eps, torch.float64)
        fp0 = tens(synth.pulse_occupations(s), torch.float64)
        fT = fp0.clone()
        n_adj = 20 if args.quick else 200
        with torch.cuda.stream(stream):
            E.rt_step(plan64, fT, n64, 1.0, n_adj, use_graph=True)
            gT = (eps * fT.sum() - (eps * fT).sum()) / fT.sum() ** 2
        stream.synchronize()
        gg2 = torch.zeros(nch, dtype=torch.float64, device=dev)
        msa, _ = timed(lambda: E.rt_adjoint(plan64, fp0, n64, 1.0, n_adj, 20, gT, gg2=gg2), 1, 0)
        forms["rt_adjoint_f64"] = dict(steps=n_adj, checkpoint_every=20, ms_total=msa,
                                       ms_per_step=msa / n_adj,
                                       collision_evaluations=8 * n_adj, vjp_calls=4 * n_adj,
                                       loss="mean carrier energy at t = steps x 1 fs")
        log(f"rt adjoint fp64 ({n_adj} steps): {msa:.1f} ms")
        # field-driven dynamics (Eq. 1 with the drift term): 1e5 V/m along x, FP64
        rates = synth.field_drift_rates([1e5, 0.0, 0.0], s.kgrid)
        n_f = 10 if args.quick else 50
        ff = fp0.clone()
        try:
            E.set_field(plan64, rates)
            msf, _ = timed(lambda: E.rt_step(plan64, ff, n64, 1.0, n_f, use_graph=True), 1, 1)
            forms["rt_step_field_f64"] = dict(steps=n_f, dt_fs=1.0, ms_per_step=msf / n_f,
                                              field_V_per_m=[1e5, 0.0, 0.0],
                                              rates_per_fs=[float(r) for r in rates])
            log(f"rt step with field fp64: {msf / n_f:.3f} ms/step")
        except E.EphbteError as e:
            forms["rt_step_field_f64"] = dict(error=str(e))
        finally:
            E.set_field(plan64, [0.0, 0.0, 0.0])
        # coupled electron-phonon dynamics: f and N stepped together, FP64
        n_c = 2 if args.quick else 5
        fc, Nc = fp0.clone(), n64.clone()
        msc, _ = timed(lambda: E.rt_step_coupled(plan64, fc, Nc, 1.0, n_c), 1, 1)
        forms["rt_step_coupled_f64"] = dict(steps=n_c, dt_fs=1.0, ms_per_step=msc / n_c,
                                            phonon_bins=int(s.n_q * s.n_modes),
                                            per_stage="pack of the stage's N, electron pass, "
                                                      "phonon pass, even-part update of N")
        log(f"coupled rt step fp64: {msc / n_c:.3f} ms/step")
        # its discrete adjoint: dL/df0, dL/dN0 and dL/d|g|^2 through n_ca
        # coupled steps, checkpoints every 2, loss = mean carrier energy
        n_ca = 2 if args.quick else 4
        gfT = tens(s.eps / s.n_states, torch.float64)
        gga = torch.zeros(nch, dtype=torch.float64, device=dev)
        msca, _ = timed(lambda: E.rt_adjoint_coupled(plan64, fp0, n64, 1.0, n_ca, 2, gfT=gfT, gg2=gga), 1, 1)
        forms["rt_adjoint_coupled_f64"] = dict(steps=n_ca, checkpoint_every=2, dt_fs=1.0,
                                               ms_per_step=msca / n_ca, gradients="f0, N0, |g|^2")
        log(f"coupled rt adjoint fp64: {msca / n_ca:.1f} ms/step")
        del ff, fc, Nc, gga
        # FP64 reference trajectory for the FP32 dynamics check below
        n_ref = 20 if args.quick else 200
        fref = fp0.clone()
        with torch.cuda.stream(stream):
            E.rt_step(plan64, fref, n64, 1.0, n_ref, use_graph=True)
        stream.synchronize()
        E64_ref = float((eps * fref).sum() / fref.sum())
        del gg2, fT, gT, fref

    plan64.close()
    del plan64, f64, I64
    torch.cuda.empty_cache()

    if not args.no_forms:
        t0 = time.time()
        plan32 = E.build_channels(s, dtype="f32", device=0)
        info32 = E.plan_info(plan32)
        bpc32 = pair_bytes(info32, s.n_modes, "f32")
        log(f"fp32 plan built ({time.time() - t0:.1f}s)")
        f32, n32 = tens(f_np, torch.float32), tens(nph_np, torch.float32)
        I32 = torch.empty_like(f32)
        fwd32 = lambda: E.collision_integral(plan32, f32, n32, out=I32)
        settle(fwd32)
        ms32, _ = timed(fwd32, args.steps, args.warmup)
        forms["fwd_f32_b1"] = dict(ms=ms32, channels_per_s=nch / (ms32 * 1e-3),
                                   algorithmic_GBps=bpc32 * nch / (ms32 * 1e-3) / 1e9,
                                   layout=LAYOUT_NAMES[info32["layout"]], bytes_per_channel=bpc32)
        log(f"fwd fp32: {ms32:.3f} ms")
        if info32["layout"] == 3:
            retune(plan32, fwd32, layout=2)
            ms32e, _ = timed(fwd32, args.steps, args.warmup)
            forms["fwd_f32_b1_entries"] = dict(ms=ms32e, channels_per_s=nch / (ms32e * 1e-3),
                                               algorithmic_GBps=BYTES_PER_CHANNEL_ENTRIES["f32"] * nch
                                               / (ms32e * 1e-3) / 1e9,
                                               layout=LAYOUT_NAMES[2])
            log(f"fwd fp32 single copy over entries: {ms32e:.3f} ms")
        retune(plan32, fwd32, layout=1)
        ms32r, _ = timed(fwd32, args.steps, args.warmup)
        retune(plan32, fwd32, layout=info32["layout"])
        forms["fwd_f32_b1_rows"] = dict(ms=ms32r, channels_per_s=nch / (ms32r * 1e-3),
                                        algorithmic_GBps=BYTES_PER_CHANNEL_ROWS["f32"] * nch / (ms32r * 1e-3) / 1e9,
                                        layout="duplicated rows")
        log(f"fwd fp32 per-row pass: {ms32r:.3f} ms")
        tuned32 = E.autotune(plan32, 64)
        F32 = tens(synth.batch_occupations(s), torch.float32)
        IB32 = torch.empty_like(F32)
        msb32, _ = timed(lambda: E.collision_integral(plan32, F32, n32, out=IB32), 3, 1)
        npairs_b32 = max(info32["pair_records"], 1)
        forms["fwd_f32_b64"] = dict(ms=msb32, per_vector_channels_per_s=64 * nch / (msb32 * 1e-3),
                                    alu_roofline=batched_alu_roofline(msb32, "f32", npairs_b32, 2 * nch, 64),
                                    ratio_vs_b1=(64 * nch / (msb32 * 1e-3)) / (nch / (ms32 * 1e-3)),
                                    batch_partners=tuned32["batch_partners"])
        log(f"fwd fp32 B=64: {msb32:.3f} ms ({forms['fwd_f32_b64']['ratio_vs_b1']:.2f}x per vector)")
        LB32 = tens(rng.normal(size=(64, s.n_states)), torch.float32)
        gg32 = torch.zeros(nch, dtype=torch.float64, device=dev)
        msbv32, _ = timed(lambda: E.collision_vjp(plan32, F32, n32, LB32, want_f=True, gg2=gg32), 3, 1)
        forms["vjp_f32_b64"] = dict(ms=msbv32, per_vector_channels_per_s=64 * nch / (msbv32 * 1e-3),
                                    alu_roofline=batched_alu_roofline(msbv32, "f32", npairs_b32, 2 * nch, 64,
                                                                      True))
        log(f"vjp fp32 B=64: {msbv32:.3f} ms")
        del F32, IB32, LB32, gg32
        forms["transport_solve_f32"] = transport_solve(
            E, plan32, tens(synth.fermi_dirac(s.eps, -0.1, 300.0), torch.float32),
            tens(s.vel, torch.float32), n32, timed)
        # dynamics: hot pulse, phonons fixed at 300 K, RK4 dt = 1 fs in HIP graphs
        n_dyn = 200 if args.quick else 2000
        eps32 = tens(s.eps, torch.float64)
        fr = tens(synth.pulse_occupations(s), torch.float32)
        N0 = float(fr.double().sum())
        with torch.cuda.stream(stream):
            E.rt_step(plan32, fr, n32, 1.0, n_ref, use_graph=True)
        stream.synchronize()
        E32_ref = float((eps32 * fr.double()).sum() / fr.double().sum())
        msr, wall_r = timed(lambda: E.rt_step(plan32, fr, n32, 1.0, n_dyn - n_ref, use_graph=True), 1, 0)
        N1 = float(fr.double().sum())
        forms["rt_bte_f32"] = dict(steps=n_dyn, dt_fs=1.0, ms_per_step=msr / (n_dyn - n_ref),
                                   evaluations_per_step=4, wall_s=wall_r,
                                   particle_drift=abs(N1 - N0) / N0,
                                   mean_energy_rel_diff_vs_f64=abs(E32_ref - E64_ref) / abs(E64_ref),
                                   compared_at_step=n_ref)
        log(f"rt-BTE fp32: {msr / (n_dyn - n_ref):.3f} ms/step over {n_dyn - n_ref} steps, "
            f"particle drift {abs(N1 - N0) / N0:.2e}, mean energy vs fp64 at step {n_ref}: "
            f"{abs(E32_ref - E64_ref) / abs(E64_ref):.2e}")
        plan32.close()

    if not args.no_forms:
        # uneven batch: 16 systems of 1e5 .. 1e7 channels in one launch
        t0 = time.time()
        gsys = synth.grouped_system(n_systems=16, ch_min=1e5, ch_max=1e6 if args.quick else 1e7)
        gf = np.clip(synth.fermi_dirac(gsys.eps, 0.05, 300.0)
                     * (0.8 + 0.4 * rng.uniform(size=gsys.n_states)), 0, 1)
        for dname, tdt in (("f64", torch.float64), ("f32", torch.float32)):
            gplan = E.build_channels(gsys, dtype=dname, device=0)
            gbpc = pair_bytes(E.plan_info(gplan), gsys.n_modes, dname)
            gft, gnt = tens(gf, tdt), tens(gsys.nph(300.0), tdt)
            gI = torch.empty_like(gft)
            msg, _ = timed(lambda: E.collision_integral(gplan, gft, gnt, out=gI), args.steps, args.warmup)
            forms[f"grouped16_{dname}"] = dict(
                ms=msg, channels_per_s=gsys.n_channels / (msg * 1e-3), systems=16,
                channels=gsys.n_channels, smallest=int(np.diff(gsys.meta["ch_offsets"]).min()),
                largest=int(np.diff(gsys.meta["ch_offsets"]).max()),
                algorithmic_GBps=gbpc * gsys.n_channels / (msg * 1e-3) / 1e9)
            log(f"grouped 16 systems {dname}: {msg:.3f} ms, {gsys.n_channels / (msg * 1e-3):.3e} ch/s "
                f"({time.time() - t0:.1f}s incl. generation)")
            gplan.close()
        # phonon-phonon scattering (a Bose plan): the modes of a 10^3 q grid,
        # every pair and third branch a channel
        t0 = time.time()
        psys = synth.ph_ph_system(n=6 if args.quick else 10)
        pplan = E.build_channels(psys, dtype="f64", device=0, statistics="bose")
        pn = tens(synth.bose_occupations(psys, 300.0, seed=5), torch.float64)
        pN = tens(synth.bose_einstein(psys.hw, 300.0), torch.float64)
        pI = torch.empty_like(pn)
        msph, _ = timed(lambda: E.collision_integral(pplan, pn, pN, out=pI), args.steps, args.warmup)
        pl = tens(rng.normal(size=psys.n_states), torch.float64)
        pgg = torch.zeros(psys.n_channels, dtype=torch.float64, device=dev)
        msphv, _ = timed(lambda: E.collision_vjp(pplan, pn, pN, pl, want_f=True, gg2=pgg), args.steps, 1)
        forms["phonon_phonon_f64"] = dict(ms=msph, reverse_ms=msphv, modes=psys.n_states,
                                          channels=psys.n_channels,
                                          channels_per_s=psys.n_channels / (msph * 1e-3),
                                          plan_layout=LAYOUT_NAMES[E.plan_info(pplan)["layout"]])
        log(f"phonon-phonon fp64 ({psys.n_states} modes, {psys.n_channels} channels): forward {msph:.3f} ms, "
            f"reverse {msphv:.3f} ms ({time.time() - t0:.1f}s incl. generation)")
        pplan.close()

    cpu = None
    if not args.no_cpu:
        # the oracle's unchanged FP64 channel loop on the host cores of this machine
        import copy
        import oracle
        model = "unknown CPU"
        try:
            with open("/proc/cpuinfo") as fh:
                model = next((ln.split(":", 1)[1].strip() for ln in fh if ln.startswith("model name")),
                             model)
        except OSError:
            pass
        ncpu = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()
        a_full = oracle._Args(s, nph_np)
        w0 = time.perf_counter()
        oracle.collision_threads(s, f_np, nph_np, threads=ncpu, args=a_full)
        t_all = time.perf_counter() - w0
        # one core on a slice of the list
        n1 = min(args.cpu_channels, nch)
        ss = copy.copy(s)
        ss.ch_i, ss.ch_j, ss.ch_nu, ss.g2 = s.ch_i[:n1], s.ch_j[:n1], s.ch_nu[:n1], s.g2[:n1]
        w0 = time.perf_counter()
        oracle.collision(ss, f_np, nph_np)
        t_one = time.perf_counter() - w0
        # one RK4 step: four evaluations on all cores plus the stage updates
        w0 = time.perf_counter()
        u = np.asarray(f_np, np.float64)
        k1 = oracle.collision_threads(s, u, nph_np, threads=ncpu, args=a_full)
        k2 = oracle.collision_threads(s, u + 0.5 * k1, nph_np, threads=ncpu, args=a_full)
        k3 = oracle.collision_threads(s, u + 0.5 * k2, nph_np, threads=ncpu, args=a_full)
        k4 = oracle.collision_threads(s, u + k3, nph_np, threads=ncpu, args=a_full)
        u = u + (k1 + 2.0 * k2 + 2.0 * k3 + k4) / 6.0
        t_rk = time.perf_counter() - w0
        del a_full, k1, k2, k3, k4, u
        # one transport iteration (numpy over the oracle's coefficients) on a slice
        nt = min(20_000_000, nch)
        st_ = copy.copy(s)
        st_.ch_i, st_.ch_j, st_.ch_nu, st_.g2 = s.ch_i[:nt], s.ch_j[:nt], s.ch_nu[:nt], s.g2[:nt]
        f0t = synth.fermi_dirac(s.eps, -0.1, 300.0)
        _, Wij, Wji = oracle.transport_coeffs(st_, f0t, nph_np)
        xt = np.asarray(s.vel) * oracle.dfde_fd(f0t, 300.0)[:, None]
        w0 = time.perf_counter()
        oracle.transport_apply_W(st_, Wij, Wji, xt)
        t_tr = (time.perf_counter() - w0) * nch / nt
        del Wij, Wji
        cpu = dict(value=nch / t_all, unit="channels/s", cores=ncpu, kind="oracle",
                   sample=f"all {nch} channels, one FP64 evaluation of I by the oracle's sequential C "
                          f"channel loop run on {ncpu} threads over disjoint slices ({t_all:.2f} s), "
                          f"{model}",
                   one_core=dict(value=n1 / t_one, unit="channels/s",
                                 sample=f"first {n1} channels, one thread ({t_one:.1f} s)"),
                   rk4_step_s=t_rk, rk4_step_note=f"four evaluations on {ncpu} threads plus numpy stage updates",
                   transport_iteration_s=t_tr,
                   transport_iteration_note=f"numpy W x of the oracle over the first {nt} channels, "
                                            "scaled to the whole list")
        log(f"cpu oracle: {nch / t_all:.3e} ch/s on {ncpu} threads ({t_all:.2f} s), "
            f"{n1 / t_one:.3e} ch/s on 1 core; RK4 step {t_rk:.2f} s, transport iteration {t_tr:.2f} s")

    out = {
        "metric": "scattering channels/sec and HBM GB/s (fwd, fwd+adjoint), B=1 vs B=64",
        "value_is": "forward, B = 1, unordered channels per second (HBM GB/s in roofline; "
                    "fwd+adjoint and B = 64 in forms)",
        "value": value,
        "unit": "channels/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "settle_passes": n_settle,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": args.dtype,
        "data": "synthetic",
        "config": {"workload": wname, "n_states": s.n_states, "n_channels": nch,
                   "entries": 2 * nch, "kgrid": list(s.kgrid), "qgrid": list(s.qgrid),
                   "modes": s.n_modes, "sigma_eV": s.sigma, "batch": 1},
        "copy_GBps": copy_gbps,
        "frac_of_copy": kernel_gbps / copy_gbps,
        "roofline": {"bound": "hbm", "achieved": kernel_gbps, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": kernel_gbps / HBM_PEAK_GBS,
                     "traffic": profiled_traffic(f"{KERNEL_OF_LAYOUT[layout64]}_{args.dtype}_{wname}"),
                     "kernel": f"{KERNEL_OF_LAYOUT[layout64]} (forward pass, {LAYOUT_NAMES[layout64]})",
                     "kernel_ms": kernel_ms,
                     "kernel_ms_from": f"HIP events around each of its {kernel_launches} launches "
                                       "in the timed steps, on the launch stream",
                     "bytes_per_channel": bpc},
        "cpu_baseline": cpu,
        "forms": forms,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
