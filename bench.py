#!/usr/bin/env python3
"""Benchmark: batched DDH-MBIR EM step on one MI355X.

Workload (default): 64 independent streams at N=256, one DDH frame per stream
per step (N_k = 1, so one EM iteration per stream per step), all streams
advanced by one batched call (eager launches; --graph replays a HIP graph).
Synthetic frozen-flow frames are generated on the host, uploaded once and
cycled, so the inputs are resident in HBM when the timed region starts.

Prints one JSON line with the throughput (EM iterations per second), the
roofline position of the dominant kernel (HIP events around each launch of an
eager step on the launch stream), the plain one-stream-at-a-time rate, frame
latency percentiles of a single stream, mean Strehl, and the FP64 oracle timed
on a bounded sample on the host.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, published
# FP32 vector issue peak without packed instructions: 256 CUs x 4 SIMDs x 16
# lanes x 2.4 GHz, one lane operation per lane per cycle (Gop/s)
ALU_PEAK_GOPS = 256 * 4 * 16 * 2.4


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=200)
    p.add_argument("--warmup", type=int, default=10)
    p.add_argument("--device-warmup-ms", type=float, default=100.0,
                   help="untimed batched steps for this long before the warm-up steps, so that the GPU runs at its "
                        "steady clock (0: none)")
    p.add_argument("--streams", type=int, default=64)
    p.add_argument("--N", type=int, default=256)
    p.add_argument("--workload", choices=["uniform", "mixed"], default="uniform")
    p.add_argument("--frames", type=int, default=8, help="distinct frames per stream (cycled)")
    p.add_argument("--timing-steps", type=int, default=20)
    p.add_argument("--latency-frames", type=int, default=200)
    p.add_argument("--plain-steps", type=int, default=5)
    p.add_argument("--no-cpu-baseline", action="store_true")
    p.add_argument("--cpu-frames", type=int, default=150, help="successive frames of one stream for the oracle "
                   "baseline and the Strehl comparison")
    p.add_argument("--cpu-frames-per-core", type=int, default=30)
    p.add_argument("--mixed-steps", type=int, default=100)
    p.add_argument("--no-extras", action="store_true", help="only the timed batched step (for profiling)")
    p.add_argument("--no-serve-grad", action="store_true", help="leave out the serving and gradient summaries")
    p.add_argument("--autotune", action="store_true", help="time every tiling first and keep the fastest")
    p.add_argument("--autotune-mix", action="store_true",
                   help="tune the tilings of all sizes together on the whole batched step")
    p.add_argument("--tiles", type=str, default=None, help="row_lines,col_width,mstep_h,mstep_w for every N")
    p.add_argument("--graph", action="store_true", help="replay the batched step as a HIP graph (eager launches "
                   "are the default: they measured faster)")
    p.add_argument("--worklist", action="store_true", help="run the batched step as the persistent work-list "
                   "launch (stats, row and column passes of all streams as one work list) plus the M-step")
    p.add_argument("--lanes", type=int, default=0, help="HIP streams of the batch: 0 = one per distinct N (default), "
                   "1-8 = that many, balanced by pixels")
    p.add_argument("--serve", action="store_true", help="instead: the continuous-batching request loop (32 streams "
                   "at N in {128,256}, Poisson arrivals) against the one-frame-at-a-time loop")
    p.add_argument("--serve-rate", type=float, default=2000.0, help="aggregate frame arrival rate (Hz)")
    p.add_argument("--serve-frames", type=int, default=40, help="frames per stream")
    p.add_argument("--serve-budget", type=float, default=0.75, help="memory budget as a fraction of all streams' bytes")
    p.add_argument("--quality", action="store_true", help="instead: Strehl over the frames for N_k in {1,2,4,8} "
                   "(10 seeds) and over an alpha/lambda grid")
    p.add_argument("--quality-frames", type=int, default=150)
    p.add_argument("--grad", action="store_true", help="instead: gradient of 8 unrolled frames for 16 streams at "
                   "N=256 (hand-written adjoint, checkpoints every 2 frames)")
    p.add_argument("--grad-rounds", type=int, default=5)
    p.add_argument("--conventional", action="store_true", help="instead: conventional single-shot DH-MBIR (hundreds "
                   "of EM iterations per frame with bootstrap resets) against DDH-MBIR (1 per frame) on one stream")
    p.add_argument("--conv-iters", type=int, default=400)
    p.add_argument("--conv-reset", type=int, default=200)
    return p.parse_args()


def make_inputs(specs, n_frames):
    import ddh_synth as synth
    sims = [synth.Stream(sp) for sp in specs]
    frames = [[sm.frame(n) for n in range(n_frames)] for sm in sims]
    return sims, frames


def gpu_params(D, N, sigma_w2):
    import ddh_synth as synth
    v = synth.DEFAULT_PARAMS
    return D.make_params(N, pupil_diameter=float(N), lam=v["lam"], alpha=v["alpha"], n_k=v["n_k"],
                         sigma_w2=sigma_w2, qg_q=v["qg_q"], qg_T=v["qg_T"], qg_sigma=v["qg_sigma"],
                         beta_phi=v["beta_phi"], r_floor=v["r_floor"])


def kernel_bytes(N, fill):
    """Algorithmic HBM bytes per launch-pixel of each kernel: the inputs its
    definition must read and the outputs it must write (arrays used only on
    the pupil counted with the pupil fill fraction)."""
    f = fill
    kb = {
        "stats": 8 + 4 * f,                     # y; phi on the pupil
        "row_ifft": 12 * f + 8,                 # y, phi on the pupil; T
        "col_fused": 8 + 4 + 8 + 4,             # T, r; U, |b|^2
        "row_fft": 8 + 12 * f + 8 * f,          # U; y, phi on the pupil; (kappa, theta~) on the pupil
        "m_step": 4 + 4 + 12 * f + 4 + 4 * f,   # r, |b|^2, phi, (kappa, theta~); r, phi (pupil)
    }
    # the work-list launch runs the first four as one kernel
    kb["frame_worklist"] = kb["stats"] + kb["row_ifft"] + kb["col_fused"] + kb["row_fft"]
    # the eager step's first row pass forms the statistics in the same launch
    # (y and phi read once)
    kb["stats_row_ifft"] = kb["row_ifft"]
    return kb


def mstep_ops(fill):
    """Algorithmic FP32 lane operations of the M-step per pixel and sweep: the
    per-pixel update formulas as written, each add/mul/fma/min/max/select
    counted once and each transcendental (log2, exp2, rcp, sqrt) twice, since
    it issues at half rate."""
    neighbour = 1 + 2 + 1 + 2 + 1 + 2 + 1 + 1 + 1 + 1   # d, log2|d|, fma, exp2, 1+v, rcp, fma, mul, A+=, B fma
    combine = 4                                         # A and B from the edge and diagonal sums
    cubic = 2 + 1 + 1 + 1 + 2 + 4 + 4 + 2 + 2 + 6 + 5 + 1 + 9 + 1  # Cardano root, one Newton step, floor
    second_moment = 3 + 4 + 3                           # Eq. (3) init, Wiener factor, E|g|^2
    phi = 14                                            # pupil pixels only
    return 8 * neighbour + combine + cubic + second_moment + phi * fill


def recorded_traffic(kernel_kind, tiles):
    """(HBM bytes per launch of the dominant kernel, note) from the committed
    counter record (profiles/m_step_traffic.json); the bytes are None when
    there is no record for the kernel or the kernel source or the tiling has
    changed since the counters were taken, and the note says which."""
    import hashlib
    rec_path = os.path.join(ROOT, "profiles", "m_step_traffic.json")
    src = os.path.join(ROOT, "paper_2305_03284_amd", "csrc", "ddh_kernels.hip")
    if kernel_kind != "m_step" or not os.path.exists(rec_path):
        return None, "no counter record for this kernel"
    rec = json.load(open(rec_path))
    sha = hashlib.sha256(open(src, "rb").read()).hexdigest()[:16]
    if rec.get("source_sha256_prefix") != sha:
        return None, "kernel source changed since the counters were taken"
    if list(rec.get("tiles", [])) != list(tiles):
        return None, "tiling differs from the one the counters were taken with"
    return int(rec["traffic_bytes"]), ("profiles/m_step_traffic.json: FETCH_SIZE x %.1f + WRITE_SIZE x %.1f per "
                                       "launch, kernel source %s" % (rec["fetch_scale"], rec["write_scale"], sha))


def oracle_params(sigma_w2):
    from oracle import ddh as O
    import ddh_synth as synth
    v = synth.DEFAULT_PARAMS
    return O.Params(sigma_w2=sigma_w2, lam=v["lam"], alpha=v["alpha"], n_k=v["n_k"], qg_q=v["qg_q"],
                    qg_T=v["qg_T"], qg_sigma=v["qg_sigma"], beta_phi=v["beta_phi"], r_floor=v["r_floor"])


def oracle_baseline(spec, ys, truths):
    """FP64 oracle on the host, one thread: the DDH frames ys (uncycled) of one
    stream of the workload from the zero state.  Only the frames are timed;
    the peak Strehl of every frame's phase is computed outside the timing."""
    from threadpoolctl import threadpool_limits
    from oracle import ddh as O
    from oracle import metrics as M
    import ddh_synth as synth
    st = synth.Stream(spec)
    prm = oracle_params(st.sigma_w2)
    a = O.aperture(spec.N)
    r = np.zeros((spec.N, spec.N))
    phi = np.zeros((spec.N, spec.N))
    dt = 0.0
    strehl = []
    with threadpool_limits(limits=1):
        for y, truth in zip(ys, truths):
            t0 = time.perf_counter()
            r, phi = O.ddh_frame(r, phi, y.astype(np.complex128), a, prm)
            dt += time.perf_counter() - t0
            strehl.append(M.strehl(phi, truth, a))
    base = {"value": len(ys) * prm.n_k / dt, "unit": "EM iters/s", "cores": 1, "kind": "oracle",
            "sample": f"{len(ys)} successive DDH frames (N_k={prm.n_k}, not cycled) of one N={spec.N} stream of the "
                      f"workload from the zero state, FP64 NumPy, 1 thread, {dt:.1f} s of frame time"}
    return base, strehl


def _oracle_worker(job):
    """One process of the all-core baseline: frames of its own stream."""
    spec, n_frames = job
    from threadpoolctl import threadpool_limits
    from oracle import ddh as O
    import ddh_synth as synth
    st = synth.Stream(spec)
    prm = oracle_params(st.sigma_w2)
    a = O.aperture(spec.N)
    ys = [st.frame(n).astype(np.complex128) for n in range(n_frames)]
    r = np.zeros((spec.N, spec.N))
    phi = np.zeros((spec.N, spec.N))
    with threadpool_limits(limits=1):
        t0 = time.perf_counter()
        for y in ys:
            r, phi = O.ddh_frame(r, phi, y, a, prm)
        t1 = time.perf_counter()
    return n_frames * prm.n_k, t0, t1


def oracle_all_cores(specs, n_frames):
    """The oracle on every host core at once: one process per core, each on
    its own stream of the workload (streams are independent), one thread per
    process.  Throughput = all timed frames / the span from the first start to
    the last end."""
    import multiprocessing as mp
    cores = min(os.cpu_count() or 1, 16, len(specs))
    ctx = mp.get_context("spawn")
    with ctx.Pool(cores) as pool:
        res = pool.map(_oracle_worker, [(specs[i], n_frames) for i in range(cores)])
    frames = sum(r[0] for r in res)
    span = max(r[2] for r in res) - min(r[1] for r in res)
    return {"value": frames / span, "unit": "EM iters/s", "cores": cores, "kind": "oracle",
            "sample": f"{cores} processes x {n_frames} DDH frames, each its own N={specs[0].N} stream of the "
                      f"workload, FP64 NumPy, 1 thread per process, {span:.1f} s span"}


def serve_main(args, only=None, emit=True):
    """Serving workload: 32 streams, N in {128, 256} (1:1, seeded), frames
    arriving by a Poisson process at --serve-rate aggregate, streams starting
    within the first 50 ms, --serve-frames frames each (8 distinct frames per
    stream, cycled, resident on the device), 1 EM iteration per frame, memory
    budget --serve-budget of all streams' bytes (so later streams wait for
    admission).  The continuous-batching loop and the one-frame-at-a-time loop
    run the same arrival trace with a budget that holds every stream, with the
    smaller budget, at ten times the rate, and with every frame arriving at
    t = 0 (saturation throughput)."""
    import torch
    import paper_2305_03284_amd as D
    import ddh_synth as synth
    from paper_2305_03284_amd.serve import ServeLoop, latency_stats, poisson_requests
    specs = synth.batch_specs(sizes_ratio=((128, 1), (256, 1)), count=32, config_id=4)
    sims, frames = make_inputs(specs, 8)
    dev_frames = [[torch.from_numpy(f).cuda() for f in fr] for fr in frames]
    truth = [[torch.from_numpy(sm.phase(n).astype(np.float32)).cuda() for n in range(8)] for sm in sims]
    keys = list(range(len(specs)))
    nbytes = {k: D.stream_bytes(specs[k].N) for k in keys}
    budget = int(args.serve_budget * sum(nbytes.values()))
    out = {"metric": "frame latency, continuous-batching request loop", "unit": "ms", "n_gpus": 1,
           "higher_is_better": False, "dtype": "f32", "data": "synthetic",
           "config": {"workload": f"32 streams, N in {{128,256}} 1:1, Poisson arrivals {args.serve_rate:.0f} Hz "
                                  f"aggregate, {args.serve_frames} frames per stream, N_k=1",
                      "small_budget_bytes": budget, "all_streams_bytes": sum(nbytes.values()), "depth": 2}}
    total_bytes = sum(nbytes.values())
    runs = [("trace", args.serve_rate, total_bytes), ("trace_budget", args.serve_rate, budget),
            ("trace_10x", 10 * args.serve_rate, total_bytes), ("saturation", None, total_bytes)]
    if only is not None:
        runs = [r for r in runs if r[0] in only]
    for label, rate, bud in runs:
        rate_reqs = poisson_requests(keys, rate or args.serve_rate, args.serve_frames, seed=4,
                                     start_spread_s=0.0 if rate is None else 0.05)
        if rate is None:  # every frame ready at t = 0
            for r in rate_reqs:
                r.t_arrival = 0.0
        res = {"arrival_hz": rate, "budget_bytes": bud}
        for plain in (False, True):
            reqs = [type(r)(r.t_arrival, r.key, r.index, r.last, dev_frames[r.key][r.index % 8]) for r in rate_reqs]
            finals = {}

            def make_stream(k):
                return D.Stream(specs[k].N, gpu_params(D, specs[k].N, sims[k].sigma_w2))

            def on_retire(k, s):  # asynchronous copies; Strehl is taken after the run
                finals[k] = (s.reflectance(), s.phase())

            loop = ServeLoop(bud, max_batch=len(keys), depth=2, plain=plain)
            done = loop.run(reqs, make_stream, nbytes.__getitem__, on_retire)
            st = latency_stats(done)
            strehl = []
            for k, (r_fin, p_fin) in finals.items():
                probe = make_stream(k)
                probe.set_state(r_fin, p_fin, args.serve_frames)
                strehl.append(probe.strehl(truth[k][(args.serve_frames - 1) % 8]))
                probe.close()
            st["mean_strehl"] = float(np.mean(strehl))
            res["plain_one_at_a_time" if plain else "continuous_batching"] = {k: round(v, 4) for k, v in st.items()}
        out[label] = res
    tr = out["trace"]["continuous_batching"]
    out.update({"p50_ms": tr["p50_ms"], "p99_ms": tr["p99_ms"], "frames_per_s": tr["frames_per_s"],
                "mean_strehl": tr["mean_strehl"]})
    if emit:
        print(json.dumps(out), flush=True)
    return out


def _quality_stream_frames(args):
    """(frames, truth phases at the checkpoints) of one seeded stream, as numpy."""
    seed, T, checkpoints = args
    import ddh_synth as synth
    sm = synth.config1_stream(N=256, stream_id=seed)
    return ([sm.frame(n) for n in range(T)], {c: sm.phase(c - 1).astype(np.float32) for c in checkpoints},
            sm.sigma_w2)


def quality_inputs(T, seeds, checkpoints):
    """Generated in worker processes before this process touches the GPU."""
    import multiprocessing as mp
    with mp.get_context("fork").Pool(min(len(seeds), 10)) as pool:
        return pool.map(_quality_stream_frames, [(sd, T, checkpoints) for sd in seeds])


def quality_checkpoints(T):
    return sorted({min(T, c) for c in (1, 10, 25, 50, 100, 150, T)})


def quality_main(args, pre):
    """Reconstruction quality on the streaming workload (N = 256, D/r0 = 15,
    0.5 px/step, SNR 5): peak Strehl of the estimate at checkpoints over
    --quality-frames frames, (a) for N_k in {1, 2, 4, 8} over 10 seeded streams
    (quartiles), (b) for an alpha x lambda grid at N_k = 1 over 3 streams
    (mean at the last frame).  "uncorrected" is the Strehl of phi = 0."""
    import torch
    import paper_2305_03284_amd as D
    import ddh_synth as synth
    T = args.quality_frames
    checkpoints = quality_checkpoints(T)
    gen, t_gen = pre
    seeds = list(range(len(gen)))
    frames = [[torch.from_numpy(f).cuda() for f in g[0]] for g in gen]
    # after c frames the estimate is compared with the truth of frame c - 1
    truth = {(i, c): torch.from_numpy(g[1][c]).cuda() for i, g in enumerate(gen) for c in checkpoints}
    sigma_w2 = [g[2] for g in gen]
    v = synth.DEFAULT_PARAMS

    def params(i, n_k=1, lam=v["lam"], alpha=v["alpha"]):
        return D.make_params(256, pupil_diameter=256.0, lam=lam, alpha=alpha, n_k=n_k, sigma_w2=sigma_w2[i],
                             qg_q=v["qg_q"], qg_T=v["qg_T"], qg_sigma=v["qg_sigma"], beta_phi=v["beta_phi"],
                             r_floor=v["r_floor"])

    def run(cases):
        """cases: list of (stream index, Params); returns Strehl[case][checkpoint]."""
        streams = [D.Stream(256, prm) for _, prm in cases]
        srv = D.Server(len(cases))
        out = [[] for _ in cases]
        for n in range(T):
            srv.step(streams, [frames[i][n] for i, _ in cases])
            if n + 1 in checkpoints:
                for c, (i, _) in enumerate(cases):
                    out[c].append(streams[c].strehl(truth[(i, n + 1)]))
        srv.close()
        for s_ in streams:
            s_.close()
        return out

    # uncorrected: Strehl of the true phase alone (estimate phi = 0)
    probe = D.Stream(256, params(0))
    uncorr = [[probe.strehl(truth[(i, c)]) for c in checkpoints] for i in range(len(seeds))]
    probe.close()
    res = {"uncorrected": {"median": [round(float(np.median([u[k] for u in uncorr])), 4) for k in range(len(checkpoints))]}}
    for n_k in (1, 2, 4, 8):
        st = np.array(run([(i, params(i, n_k=n_k)) for i in range(len(seeds))]))
        res[f"N_k={n_k}"] = {q: [round(float(x), 4) for x in np.percentile(st, pq, axis=0)]
                              for q, pq in (("q25", 25), ("median", 50), ("q75", 75))}
    grid = {}
    for alpha in (0.01, 0.025, 0.05, 0.1):
        cases = [(i, params(i, lam=lam, alpha=alpha)) for lam in (0.2, 0.45, 0.7, 0.9) for i in range(3)]
        st = np.array(run(cases))[:, -1].reshape(4, 3).mean(axis=1)
        for lam, val in zip((0.2, 0.45, 0.7, 0.9), st):
            grid[f"alpha={alpha},lambda={lam}"] = round(float(val), 4)
    out = {"metric": "peak Strehl of the phase estimate (streaming workload)", "unit": "Strehl", "n_gpus": 1,
           "higher_is_better": True, "dtype": "f32", "data": "synthetic",
           "config": {"workload": "N=256, D/r0=15, 0.5 px/step, SNR 5, frames " + str(T), "seeds": len(seeds)},
           "checkpoints": checkpoints, "strehl": res, "alpha_lambda_grid_last_frame": grid,
           "input_generation_s": round(t_gen, 1)}
    print(json.dumps(out), flush=True)


def grad_main(args, emit=True):
    """Differentiation workload: 16 streams at N=256, each with the gradient
    of K=8 unrolled DDH frames (from r = 0 and a perturbed phase) with respect
    to phi0, sigma_w, sigma_r and beta_phi, checkpoints every 2 frames.  The
    frames and phases are resident on the device; one step is the 16
    gradients in one batched call (ddh_unrolled_grad_batch), also timed as 16
    single-stream calls.  The FP64 autograd reference (the oracle) is timed on
    one stream."""
    import torch
    import paper_2305_03284_amd as D
    import ddh_synth as synth
    N, K, S, ckpt = 256, 8, 16, 2
    v = synth.DEFAULT_PARAMS
    cases = []
    for sid in range(S):
        st = synth.Stream(synth.StreamSpec(N=N, d_over_r0=6.0, snr=20.0, speed=0.5, config_id=3, stream_id=sid))
        rng = np.random.default_rng(sid)
        phi0 = st.phase(0) + 0.3 * rng.standard_normal((N, N))
        cases.append((st, [st.frame(n) for n in range(K)], phi0, st.phase(K - 1)))
    dev = []
    for st, frames, phi0, ptrue in cases:
        prm = D.make_params(N, pupil_diameter=float(N), lam=v["lam"], alpha=v["alpha"], n_k=1,
                            sigma_w2=st.sigma_w2, qg_q=v["qg_q"], qg_T=v["qg_T"], qg_sigma=v["qg_sigma"],
                            beta_phi=v["beta_phi"], r_floor=v["r_floor"])
        dev.append((prm, [torch.from_numpy(f).cuda() for f in frames],
                    torch.from_numpy(phi0.astype(np.float32)).cuda(), torch.from_numpy(ptrue.astype(np.float32)).cuda()))

    cols = list(zip(*dev))

    def batched():
        return D.unrolled_grad_batch(list(cols[0]), list(cols[1]), list(cols[2]), list(cols[3]), ckpt)

    def one_at_a_time():
        return [D.unrolled_grad(prm, ys, p0, pt, ckpt) for prm, ys, p0, pt in dev]

    def timed(fn, rounds):
        fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(rounds):
            res = fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / rounds, res

    dt, res = timed(batched, args.grad_rounds)
    dt1, _ = timed(one_at_a_time, max(1, args.grad_rounds // 2))
    out = {"metric": "unrolled-frame gradients/s", "value": S * K / dt, "unit": "frames/s", "n_gpus": 1,
           "steps": args.grad_rounds, "warmup": 1, "ms_per_step": dt * 1e3, "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
           "config": {"workload": f"{S} streams x N={N}, gradient of K={K} unrolled DDH frames (N_k=1) w.r.t. "
                                  f"phi0, sigma_w, sigma_r, beta_phi, checkpoints every {ckpt}",
                      "streams": S, "N": N, "K": K, "ckpt": ckpt},
           "one_stream_at_a_time": {"frames_per_s": S * K / dt1, "ms_per_step": dt1 * 1e3},
           "mean_loss": float(np.mean([r[0] for r in res]))}
    if not args.no_cpu_baseline and emit:
        from oracle import grad as G
        from oracle import ddh as O
        st, frames, phi0, ptrue = cases[0]
        a = O.aperture(N)
        prm0 = O.Params(sigma_w2=st.sigma_w2)
        t0 = time.perf_counter()
        G.reference_gradient(phi0, float(np.sqrt(st.sigma_w2)), prm0.qg_sigma, prm0.beta_phi, frames, ptrue, a, prm0)
        t_cpu = time.perf_counter() - t0
        out["cpu_baseline"] = {"value": K / t_cpu, "unit": "frames/s", "cores": torch.get_num_threads(),
                               "kind": "oracle",
                               "sample": f"one stream's gradient of {K} frames at N={N}, FP64 torch autograd on the "
                                         f"host, {t_cpu:.1f} s"}
    if emit:
        print(json.dumps(out), flush=True)
    return out


def conventional_main(args):
    """Conventional DH-MBIR against DDH-MBIR on the streaming case (N=256,
    D/r0=15, SNR=5, 0.5 px/step, one stream).  DDH-MBIR runs frames 0..119
    with one EM iteration each, warm-started; conventional DH-MBIR solves each
    of the last 20 frames on its own from r = phi = 0 with --conv-iters EM
    iterations and a full (lambda = 1) bootstrap reset every --conv-reset.
    Reports GPU time per frame and peak Strehl for both, and Strehl against
    the iteration count of the conventional loop on one frame."""
    import torch
    import paper_2305_03284_amd as D
    import ddh_synth as synth
    T, last = 120, 20
    sm = synth.config1_stream()
    N = sm.spec.N
    ys = [torch.from_numpy(sm.frame(n)).cuda() for n in range(T)]
    truth = [torch.from_numpy(sm.phase(n).astype(np.float32)).cuda() for n in range(T - last, T)]
    prm = gpu_params(D, N, sm.sigma_w2)
    v = synth.DEFAULT_PARAMS
    conv_prm = D.make_params(N, pupil_diameter=float(N), lam=1.0, alpha=v["alpha"], n_k=1, sigma_w2=sm.sigma_w2,
                             qg_q=v["qg_q"], qg_T=v["qg_T"], qg_sigma=v["qg_sigma"], beta_phi=v["beta_phi"],
                             r_floor=v["r_floor"])
    # DDH-MBIR: timing pass, then the same frames again for Strehl
    s = D.Stream(N, prm)
    for y in ys[:10]:
        s.step(y)
    torch.cuda.synchronize()
    s.close()
    s = D.Stream(N, prm)
    t0 = time.perf_counter()
    for y in ys:
        s.step(y)
    torch.cuda.synchronize()
    ddh_ms = (time.perf_counter() - t0) / T * 1e3
    s.close()
    s = D.Stream(N, prm)
    ddh_S = []
    for n, y in enumerate(ys):
        s.step(y)
        if n >= T - last:
            ddh_S.append(s.strehl(truth[n - (T - last)]))
    s.close()
    # conventional DH-MBIR, each frame on its own
    c = D.Stream(N, conv_prm)
    z = torch.zeros((N, N), dtype=torch.float32, device="cuda")
    c.set_state(z, z, 0)
    c.mbir(ys[0], 20, args.conv_reset)  # warm-up
    torch.cuda.synchronize()
    conv_S, conv_t = [], []
    for k in range(last):
        c.set_state(z, z, 0)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        c.mbir(ys[T - last + k], args.conv_iters, args.conv_reset)
        torch.cuda.synchronize()
        conv_t.append(time.perf_counter() - t0)
        conv_S.append(c.strehl(truth[k]))
    curve = {}
    for it in (1, 2, 5, 10, 20, 50, 100, 200, 201, 250, 300, 400, 600):
        c.set_state(z, z, 0)
        c.mbir(ys[T - 1], it, args.conv_reset)
        curve[it] = round(c.strehl(truth[-1]), 4)
    c.close()
    conv_ms = float(np.mean(conv_t)) * 1e3
    out = {"metric": "GPU time per frame and peak Strehl, conventional DH-MBIR vs DDH-MBIR", "unit": "ms",
           "n_gpus": 1, "higher_is_better": False, "dtype": "f32", "data": "synthetic",
           "config": {"workload": f"one stream, N={N}, D/r0=15, SNR=5, 0.5 px/step; DDH-MBIR over frames 0-{T - 1} "
                                  f"(1 EM iteration per frame); conventional DH-MBIR on frames {T - last}-{T - 1}, "
                                  f"each from r = phi = 0, {args.conv_iters} EM iterations, bootstrap reset every "
                                  f"{args.conv_reset}"},
           "ddh_mbir": {"em_iters_per_frame": 1, "ms_per_frame": ddh_ms, "mean_strehl": float(np.mean(ddh_S))},
           "conventional": {"em_iters_per_frame": args.conv_iters, "reset_every": args.conv_reset,
                            "ms_per_frame": conv_ms, "mean_strehl": float(np.mean(conv_S)),
                            "strehl_vs_iterations_last_frame": curve},
           "time_ratio": conv_ms / ddh_ms}
    print(json.dumps(out), flush=True)


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); streams are independent, "
              "so a multi-GPU run shards them with no communication", file=sys.stderr)
        sys.exit(2)
    pre = None
    if args.quality:  # host-side inputs first, in worker processes, before any GPU call
        t0 = time.perf_counter()
        pre = (quality_inputs(args.quality_frames, list(range(10)), quality_checkpoints(args.quality_frames)),
               time.perf_counter() - t0)
    import torch
    if not torch.cuda.is_available():
        print("no GPU available", file=sys.stderr)
        sys.exit(1)
    if args.serve:
        serve_main(args)
        return
    if args.quality:
        quality_main(args, pre)
        return
    if args.grad:
        grad_main(args)
        return
    if args.conventional:
        conventional_main(args)
        return
    import paper_2305_03284_amd as D
    import ddh_synth as synth

    if args.workload == "uniform":
        specs = synth.batch_specs(uniform_N=args.N, count=args.streams, config_id=2)
        wl = f"{args.streams} streams x N={args.N}, batched DDH frame (N_k=1), frozen-flow synthetic"
    else:
        specs = synth.batch_specs(count=args.streams, config_id=2)
        wl = f"{args.streams} streams, N in {{128,256,512}} at 2:5:1, batched DDH frame (N_k=1), frozen-flow synthetic"
    t_gen = time.perf_counter()
    sims, frames = make_inputs(specs, args.frames)
    t_gen = time.perf_counter() - t_gen
    S = len(specs)
    px_total = sum(sp.N * sp.N for sp in specs)

    tiles = {}
    if args.autotune_mix and not args.tiles:
        D.autotune_mix([sp.N for sp in specs])
    for n_ in sorted({sp.N for sp in specs}):
        if args.tiles:
            D.set_tiles(n_, [int(v) for v in args.tiles.split(",")])
        elif args.autotune:
            D.autotune(n_, sum(1 for sp in specs if sp.N == n_))
        tiles[n_] = D.get_tiles(n_)

    dev_frames = [[torch.from_numpy(frames[i][k]).cuda() for i in range(S)] for k in range(args.frames)]
    ptrs = [[t.data_ptr() for t in dev_frames[k]] for k in range(args.frames)]
    streams = [D.Stream(sp.N, gpu_params(D, sp.N, sims[i].sigma_w2)) for i, sp in enumerate(specs)]
    batch = D.Batch(streams, graph=args.graph, lanes=args.lanes, worklist=args.worklist)
    torch.cuda.synchronize()

    step = 0
    # the GPU leaves its idle clock only under sustained load (measured: 20
    # timed steps read 478k EM iters/s after 5 warm-up steps from idle, 504k
    # after 50, 528k after 200), so the batched step first runs untimed for
    # device_warmup_ms; then the warm-up steps, then exactly `steps` timed steps
    t_dw = time.perf_counter()
    n_dw = 0
    while (time.perf_counter() - t_dw) * 1e3 < args.device_warmup_ms:
        for _ in range(8):
            batch.step_ptrs(ptrs[step % args.frames])
            step += 1
            n_dw += 1
        torch.cuda.synchronize()
    for _ in range(args.warmup):
        batch.step_ptrs(ptrs[step % args.frames])
        step += 1
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        batch.step_ptrs(ptrs[step % args.frames])
        step += 1
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    iters = S * args.steps  # N_k = 1: one EM iteration per stream per step
    value = iters / dt
    ms_per_step = 1e3 * dt / args.steps
    # after the timed region: every stream's status for its last frame (a
    # rejected frame or a device-side wait that gave up would show here)
    statuses = [s.status() for s in streams]

    out = {
        "metric": "EM iters/s (batched DDH-MBIR EM step)",
        "value": round(value, 1),
        "unit": "EM iters/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": wl, "streams": S, "N": args.N if args.workload == "uniform" else "mixed",
                   "n_k": 1, "pixels_per_step": px_total, "frames_cycled": args.frames,
                   "launch": ("graph" if args.graph else "eager") + (", work list" if args.worklist else ""),
                   "lanes": "one per N" if args.lanes == 0 else args.lanes,
                   "tiles": {str(k): v for k, v in tiles.items()}},
        "streams_ok": sum(1 for v in statuses if v == 0) == S,
        "device_warmup": {"ms": args.device_warmup_ms, "steps": n_dw,
                          "note": "untimed batched steps before the warm-up steps (GPU clock ramp)"},
    }

    def calibration_copy():
        # for the HBM byte counters: a plain 64 MiB copy of a source pushed out
        # of the caches by 512 MiB of later writes (after the per-kernel timing,
        # whose steps would otherwise start with the caches flushed)
        src = torch.empty(64 * 2 ** 20 // 4, dtype=torch.float32, device="cuda").fill_(1.0)
        flush = torch.empty(512 * 2 ** 20 // 4, dtype=torch.float32, device="cuda").fill_(2.0)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        out["calibration_copy_bytes"] = 64 * 2 ** 20
        del src, dst, flush

    if args.no_extras:
        calibration_copy()
    else:
        # ---- per-kernel timing (eager step; each launch records its kernel's
        # start and end with a pair of HIP events)
        batch.set_timing(True)
        for _ in range(args.timing_steps):
            batch.step_ptrs(ptrs[step % args.frames])
            step += 1
        st_times = batch.stage_times()
        batch.set_timing(False)
        torch.cuda.synchronize()
        calibration_copy()
        fill = float(synth.aperture(args.N).sum()) / args.N ** 2 if args.workload == "uniform" else 0.785
        kb = kernel_bytes(args.N, fill)
        kernels = {}
        for name, (ms, calls) in st_times.items():
            if calls == 0:
                continue
            avg_us = 1e3 * ms / calls
            entry = {"avg_us": round(avg_us, 3), "launches": calls}
            if name in kb and args.workload == "uniform":
                byt = kb[name] * px_total
                entry["alg_bytes"] = int(byt)
                entry["GB_s"] = round(byt / (avg_us * 1e-6) / 1e9, 1)
            kernels[name] = entry
        eager_step_us = sum(v["avg_us"] for v in kernels.values())
        if "m_step" in kernels and args.workload == "uniform":
            ops = mstep_ops(fill) * px_total
            kernels["m_step"]["alg_ops"] = int(ops)
            kernels["m_step"]["Gop_s"] = round(ops / (kernels["m_step"]["avg_us"] * 1e-6) / 1e9, 1)
        dom = max((k for k in kernels if k in kb), key=lambda k: kernels[k]["avg_us"])
        if dom == "m_step" and "Gop_s" in kernels[dom]:
            # the M-step is bound by vector-ALU issue (its HBM traffic takes a
            # fraction of its duration)
            traffic, tnote = recorded_traffic(dom, tiles.get(args.N, ()))
            out["roofline"] = {"bound": "alu", "kernel": dom, "achieved": kernels[dom]["Gop_s"],
                               "peak": round(ALU_PEAK_GOPS, 1), "unit": "Gop/s",
                               "frac": round(kernels[dom]["Gop_s"] / ALU_PEAK_GOPS, 4),
                               "traffic": traffic, "traffic_note": tnote}
        elif "GB_s" in kernels[dom]:
            traffic, tnote = recorded_traffic(dom, tiles.get(args.N, ()))
            out["roofline"] = {"bound": "hbm", "kernel": dom, "achieved": kernels[dom]["GB_s"], "peak": HBM_PEAK_GBS,
                               "unit": "GB/s", "frac": round(kernels[dom]["GB_s"] / HBM_PEAK_GBS, 4),
                               "traffic": traffic, "traffic_note": tnote}
        step_bytes_floor = 56 * px_total  # compulsory + one global round trip per 2-D FFT
        step_bytes_alg = sum(kb[k] for k in kernels if k in kb) * px_total  # the kernels the step launched
        out["kernels"] = kernels
        out["step"] = {"us": round(1e3 * ms_per_step, 2), "sum_of_timed_kernels_us": round(eager_step_us, 2),
                       "floor_bytes": step_bytes_floor, "alg_bytes": int(step_bytes_alg),
                       "floor_frac_of_hbm_peak": round(step_bytes_floor / (ms_per_step * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                       "alg_GB_s": round(step_bytes_alg / (ms_per_step * 1e-3) / 1e9, 1)}

        # ---- plain form: the same streams one at a time through the single-stream call
        torch.cuda.synchronize()
        tp = time.perf_counter()
        for k in range(args.plain_steps):
            fk = dev_frames[step % args.frames]
            for i in range(S):
                streams[i].step(fk[i])
            step += 1
        torch.cuda.synchronize()
        plain = S * args.plain_steps / (time.perf_counter() - tp)
        out["plain_one_stream_at_a_time"] = {"value": round(plain, 1), "unit": "EM iters/s",
                                             "batched_over_plain": round(value / plain, 2)}

        # ---- latency of one stream (config-1 style: N=256, frames on the device)
        sp1 = synth.config1_stream(N=args.N)
        lat_frames = [torch.from_numpy(sp1.frame(n)).cuda() for n in range(16)]
        s1 = D.Stream(args.N, gpu_params(D, args.N, sp1.sigma_w2))
        evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
               for _ in range(args.latency_frames)]
        for n in range(5):
            s1.step(lat_frames[n % 16])
        torch.cuda.synchronize()
        for n, (ea, eb) in enumerate(evs):
            ea.record()
            s1.step(lat_frames[n % 16])
            eb.record()
            eb.synchronize()
        lat = np.array([ea.elapsed_time(eb) * 1e3 for ea, eb in evs])
        # end to end: the frame starts in pinned host memory and is copied to
        # the device on the same stream before the step
        host_frames = [f.cpu().pin_memory() for f in lat_frames]
        dev_y = torch.empty_like(lat_frames[0])
        for n, (ea, eb) in enumerate(evs):
            ea.record()
            dev_y.copy_(host_frames[n % 16], non_blocking=True)
            s1.step(dev_y)
            eb.record()
            eb.synchronize()
        lat_e2e = np.array([ea.elapsed_time(eb) * 1e3 for ea, eb in evs])
        out["latency_us_single_stream"] = {"p50": round(float(np.percentile(lat, 50)), 2),
                                           "p99": round(float(np.percentile(lat, 99)), 2), "N": args.N,
                                           "frames": args.latency_frames,
                                           "note": "device time per frame, y already on the device",
                                           "end_to_end_p50": round(float(np.percentile(lat_e2e, 50)), 2),
                                           "end_to_end_p99": round(float(np.percentile(lat_e2e, 99)), 2),
                                           "end_to_end_note": "with the H2D copy of y from pinned host memory"}
        s1.close()

        # ---- the same batched step with the other launch structure (work list
        # or the five launches per iteration), same streams and frames
        obatch = D.Batch(streams, graph=args.graph, lanes=args.lanes, worklist=not args.worklist)
        for _ in range(args.warmup):
            obatch.step_ptrs(ptrs[step % args.frames])
            step += 1
        torch.cuda.synchronize()
        to = time.perf_counter()
        for _ in range(args.steps):
            obatch.step_ptrs(ptrs[step % args.frames])
            step += 1
        torch.cuda.synchronize()
        dto = time.perf_counter() - to
        obatch.set_timing(True)
        for _ in range(args.timing_steps):
            obatch.step_ptrs(ptrs[step % args.frames])
            step += 1
        o_times = {k_: round(1e3 * ms_ / c_, 3) for k_, (ms_, c_) in obatch.stage_times().items() if c_}
        obatch.close()
        out["worklist" if not args.worklist else "five_launches"] = {
            "value": round(S * args.steps / dtg_guard(dto), 1), "unit": "EM iters/s",
            "ms_per_step": round(1e3 * dto / args.steps, 4), "kernel_avg_us": o_times,
            "note": "same streams and frames; " + ("persistent work-list launch (stats, row and column passes as "
                                                   "one work list) + M-step" if not args.worklist else
                                                   "stats, row, column, row, M-step launches")}

        # ---- the same batched step replayed as a HIP graph (same streams, frames)
        gbatch = D.Batch(streams, graph=True, lanes=args.lanes, worklist=args.worklist)
        for _ in range(args.warmup):
            gbatch.step_ptrs(ptrs[step % args.frames])
            step += 1
        torch.cuda.synchronize()
        tg = time.perf_counter()
        for _ in range(args.steps):
            gbatch.step_ptrs(ptrs[step % args.frames])
            step += 1
        torch.cuda.synchronize()
        dtg = time.perf_counter() - tg
        gbatch.close()
        out["graph_replay"] = {"value": round(S * args.steps / dtg, 1), "unit": "EM iters/s",
                               "ms_per_step": round(1e3 * dtg / args.steps, 4),
                               "note": "same batch, step captured once as a HIP graph and replayed"}

        # ---- whole step against HBM and against a device copy of the step's footprint
        foot = max(step_bytes_floor, 448 * 2 ** 20)
        csrc = torch.empty(foot // 8, dtype=torch.float32, device="cuda").fill_(1.0)
        cdst = torch.empty_like(csrc)
        ce0, ce1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        cdst.copy_(csrc)
        torch.cuda.synchronize()
        ce0.record()
        for _ in range(10):
            cdst.copy_(csrc)
        ce1.record()
        ce1.synchronize()
        copy_gbs = 2 * (foot // 8) * 4 * 10 / (ce0.elapsed_time(ce1) * 1e-3) / 1e9
        del csrc, cdst
        step_gbs = step_bytes_floor / (ms_per_step * 1e-3) / 1e9
        out["step_roofline"] = {"bound": "hbm", "floor_bytes_per_step": step_bytes_floor,
                                "floor_B_per_px": 56, "achieved": round(step_gbs, 1), "unit": "GB/s",
                                "peak": HBM_PEAK_GBS, "frac": round(step_gbs / HBM_PEAK_GBS, 4),
                                "copy_GB_s": round(copy_gbs, 1), "copy_bytes_moved": 2 * (foot // 8) * 4,
                                "frac_of_copy": round(step_gbs / copy_gbs, 4), "target_frac": 0.5,
                                "met": bool(step_gbs / HBM_PEAK_GBS >= 0.5)}

        # ---- Strehl on successive (uncycled) frames of one stream: GPU and oracle
        sp0 = specs[0]
        n_q = args.cpu_frames
        q_frames = [sims[0].frame(n) for n in range(n_q)]
        q_truth = [sims[0].phase(n) for n in range(n_q)]
        sq = D.Stream(sp0.N, gpu_params(D, sp0.N, sims[0].sigma_w2))
        s_zero = D.Stream(sp0.N, gpu_params(D, sp0.N, sims[0].sigma_w2))  # never stepped: phase 0 (uncorrected)
        s_gpu, s_unc = [], []
        for n in range(n_q):
            sq.step(torch.from_numpy(q_frames[n]).cuda())
            tr = torch.from_numpy(q_truth[n].astype(np.float32)).cuda()
            s_gpu.append(sq.strehl(tr))
            s_unc.append(s_zero.strehl(tr))
        sq.close()
        s_zero.close()
        strehl = {"stream": f"workload stream 0 (N={sp0.N}, D/r0={sp0.d_over_r0:.2f}, SNR={sp0.snr:.2f})",
                  "frames": n_q, "gpu_mean_last50": round(float(np.mean(s_gpu[-50:])), 4),
                  "uncorrected_mean_last50": round(float(np.mean(s_unc[-50:])), 4)}

        if not args.no_cpu_baseline:
            base, s_orc = oracle_baseline(sp0, q_frames, q_truth)
            out["cpu_baseline"] = base
            out["cpu_baseline"]["host_cpu"] = _cpu_model()
            out["cpu_baseline"]["host_cpu_count"] = os.cpu_count()
            strehl["oracle_mean_last50"] = round(float(np.mean(s_orc[-50:])), 4)
            strehl["max_abs_diff_gpu_oracle"] = round(float(np.max(np.abs(np.array(s_gpu) - np.array(s_orc)))), 5)
            out["cpu_baseline_all_cores"] = oracle_all_cores(specs, args.cpu_frames_per_core)
        out["strehl"] = strehl

        # ---- the mixed-size workload (64 streams, N 128/256/512 at 2:5:1), one lane per N
        if args.workload == "uniform" and args.mixed_steps > 0:
            mspecs = synth.batch_specs(count=64, config_id=2)
            msims, mframes = make_inputs(mspecs, 4)
            mdev = [[torch.from_numpy(mframes[i][k]).cuda() for i in range(len(mspecs))] for k in range(4)]
            mptrs = [[t.data_ptr() for t in mdev[k]] for k in range(4)]
            mstreams = [D.Stream(sp.N, gpu_params(D, sp.N, msims[i].sigma_w2)) for i, sp in enumerate(mspecs)]

            def time_mixed(**kw):
                mb = D.Batch(mstreams, lanes=0, **kw)
                for k in range(args.warmup):
                    mb.step_ptrs(mptrs[k % 4])
                torch.cuda.synchronize()
                tm = time.perf_counter()
                for k in range(args.mixed_steps):
                    mb.step_ptrs(mptrs[k % 4])
                torch.cuda.synchronize()
                dtm = time.perf_counter() - tm
                mb.close()
                return {"value": round(len(mspecs) * args.mixed_steps / dtm, 1),
                        "ms_per_step": round(1e3 * dtm / args.mixed_steps, 4)}

            eager = time_mixed(graph=False)
            graphed = time_mixed(graph=True)
            wl_graph = time_mixed(graph=True, worklist=True)
            for s_ in mstreams:
                s_.close()
            out["mixed_workload"] = {"value": graphed["value"], "unit": "EM iters/s",
                                     "ms_per_step": graphed["ms_per_step"],
                                     "workload": "64 streams, N in {128,256,512} at 2:5:1 (16/40/8), step captured "
                                                 "once as a HIP graph, one lane per N, 4 frames cycled",
                                     "pixels_per_step": sum(sp.N * sp.N for sp in mspecs),
                                     "eager": eager,
                                     "worklist_hip_graph": dict(wl_graph, note="persistent work-list launch per N "
                                                                "group + M-step, captured once as a HIP graph"),
                                     "tiles": "default per N (the mix autotuner keeps them on this workload)"}
        # ---- the serving loop (32 streams, N 128/256, Poisson arrivals) and the
        # batched unrolled-frame gradient, summarised (their own modes: --serve, --grad)
        if args.workload == "uniform" and not args.no_serve_grad:
            sv = serve_main(args, only=("trace",), emit=False)
            tr = sv["trace"]
            out["serving"] = {"workload": sv["config"]["workload"], "continuous_batching": tr["continuous_batching"],
                              "plain_one_at_a_time": tr["plain_one_at_a_time"]}
            gr = grad_main(args, emit=False)
            out["gradient"] = {"workload": gr["config"]["workload"], "value": round(gr["value"], 1),
                               "unit": gr["unit"], "ms_per_call": round(gr["ms_per_step"], 3),
                               "one_stream_at_a_time_frames_per_s": round(gr["one_stream_at_a_time"]["frames_per_s"], 1)}
    out["input_generation_s"] = round(t_gen, 1)
    batch.close()
    print(json.dumps(out), flush=True)


def dtg_guard(dt):
    return dt if dt > 0 else 1e-9


def _cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


if __name__ == "__main__":
    main()
