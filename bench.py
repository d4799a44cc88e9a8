"""Benchmark: Gauss-Newton iterations per second of the full pose solve on the
200-keyframe global workload (80x60 frames, ~3700 dense pair jobs, ~300k
sparse correspondences, 8 GN x 20 PCG), one MI355X.

One step = one bf_gauss_newton() call: per-frame preparation, pair test,
correspondence grouping and moments, then 8 iterations of dense pair jobs +
edge blocks + assembly + 20 PCG iterations + SE(3) update, then the final
energy.  Inputs are resident in HBM before the timed region.

Beside it (field "batched"), the batched intra-chunk workload: 256 independent
chunk problems of 4-11 frames at 160x120, solved (5 GN x 10 PCG each) by one
bf_gauss_newton_batch call per step, against the same 256 problems solved one
after another by bf_gauss_newton; problems per second for both, and the largest
pose difference between the two forms.

And (field "serving") the serving workload: a Poisson stream of requests, 80 %
chunk solves (160x120, 4-11 frames) and 20 % global keyframe solves (80x60, 50-800
keyframes), served by the two-lane continuous-batching server
(paper_1604_01093_amd.serve) at 0.5x and 0.8x of its measured peak rate, against a
one-at-a-time loop of plain solves on the same arrival stream; p50/p99 latency and
solves per second, and whether every served result equals the result of the same
request solved alone.

Prints one JSON line.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
BYTES_PER_SOURCE_PIXEL = 40  # depth+normal+gradient of the source pixel and of its target footprint
DENSE_SOURCE = os.path.join(ROOT, "paper_1604_01093_amd", "csrc", "dense.hip")
TRAFFIC_SUMMARY = os.path.join(ROOT, "profiles", "k_dense_global200_traffic.md")


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def source_digest(path):
    import hashlib
    with open(path, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()


def measured_traffic(threads, tiles):
    """HBM bytes per dense launch of this launch shape from the committed
    FETCH_SIZE/WRITE_SIZE summary, or None when the summary is absent, has no row
    for the shape, or the dense kernel's source has changed since."""
    if not os.path.exists(TRAFFIC_SUMMARY):
        return None
    fields = {}
    with open(TRAFFIC_SUMMARY) as f:
        for ln in f:
            if ln.startswith("- ") and ":" in ln:
                k, v = ln[2:].split(":", 1)
                fields[k.strip()] = v.strip().strip("`")
    if fields.get("dense.hip sha256") != source_digest(DENSE_SOURCE):
        return None
    try:
        return int(fields[f"HBM bytes per launch, {threads} threads x {tiles} tiles"])
    except (KeyError, ValueError):
        return None


def copy_calibration(mib):
    """A plain device copy of known size (read mib MiB, write mib MiB) for scaling the
    FETCH_SIZE/WRITE_SIZE counters; only run when asked for, under the profiler."""
    import torch
    n = mib * (1 << 20) // 4
    src = torch.ones(n, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    for _ in range(3):
        torch.mul(src, 1.0, out=dst)
    torch.cuda.synchronize()
    log(f"copy calibration: 3 x {mib} MiB read + {mib} MiB written")
    del src, dst


_ORC = {}


def _oracle_worker_init(prob, n_gn, n_pcg):
    """Spawned oracle worker: its own per-solve setup (not timed)."""
    from threadpoolctl import threadpool_limits
    from oracle import Params
    from oracle.gn import Setup
    threadpool_limits(limits=1)
    prm = Params(num_gn=n_gn, num_pcg=n_pcg)
    _ORC["setup"] = Setup(prob.depth, prob.intensity, prob.intrinsics, prob.corr_i, prob.corr_j, prob.corr_p,
                          prob.corr_q, prob.init_poses, prm)


def _oracle_edge_blocks(args):
    from oracle.gn import edge_blocks
    lo, hi, poses, wd = args
    s = _ORC["setup"]
    sub = type(s).__new__(type(s))
    sub.__dict__.update(s.__dict__)
    sub.edges, sub.edge_dense, sub.edge_sparse = s.edges[lo:hi], s.edge_dense[lo:hi], s.edge_sparse[lo:hi]
    return [{k: b[k] for k in ("Hii", "Hij", "Hjj", "gi", "gj")} for b in edge_blocks(sub, poses, wd)]


def _oracle_gn_iteration(s, prm, poses, k, pool=None, chunks=1):
    """One Gauss-Newton iteration of the oracle (assembly, block-Jacobi PCG, update);
    the edge blocks in `pool` when given."""
    from oracle.gn import build_system
    from oracle.se3 import exp_se3
    from oracle.system import assemble, inert_frames, reduce_system, solve_pcg
    if pool is None:
        H, g, _, _ = build_system(s, poses, prm.dense_weight(k))
    else:
        E = len(s.edges)
        step = (E + chunks - 1) // chunks
        parts = pool.map(_oracle_edge_blocks, [(lo, min(E, lo + step), poses, prm.dense_weight(k))
                                               for lo in range(0, E, step)])
        H, g = assemble(s.F, s.edges, [b for part in parts for b in part])
    inert = inert_frames(H, s.free)
    act = s.free[~inert]
    Hr, gr, _ = reduce_system(H, g, act)
    dx, _ = solve_pcg(Hr, gr, prm.num_pcg)
    out = poses.copy()
    for n, f in enumerate(act):
        out[f] = out[f] @ exp_se3(dx[6 * n:6 * n + 6])
    return out


def cpu_baseline(prob, n_gn, n_pcg, chunk=None, batch_sample=None, full=False):
    """The FP64 oracle timed on this host's cores.

    Primary (the reported value): one Gauss-Newton iteration of the headline
    workload on one core (BLAS limited to one thread), per-solve setup excluded.
    Legs beside it: the same iteration on every core of this process's affinity set
    (edge blocks in a pool of spawned processes, one per core, threaded BLAS for the
    solve); the 11-frame chunk solved in full on one core; a sample of the batched
    chunk problems solved in full on one core; with `full`, also all 8 iterations of
    the headline workload on one core."""
    import multiprocessing as mp
    import os

    from threadpoolctl import threadpool_limits

    from oracle import Params
    from oracle.gn import Setup, solve_problem

    cores = len(os.sched_getaffinity(0))
    prm = Params(num_gn=n_gn, num_pcg=n_pcg)
    legs = []
    with threadpool_limits(limits=1):
        t0 = time.perf_counter()
        s = Setup(prob.depth, prob.intensity, prob.intrinsics, prob.corr_i, prob.corr_j, prob.corr_p, prob.corr_q,
                  prob.init_poses, prm)
        t1 = time.perf_counter()
        _oracle_gn_iteration(s, prm, prob.init_poses, 0)
        t2 = time.perf_counter()
    one = t2 - t1
    legs.append({"what": f"1 of {n_gn} GN iterations of the headline workload", "cores": 1,
                 "seconds": round(one, 3), "gn_iters_per_s": round(1.0 / one, 4),
                 "setup_seconds_excluded": round(t1 - t0, 2)})
    log(f"oracle: one GN iteration on 1 core {one:.2f} s (setup {t1 - t0:.1f} s)")
    workers = max(1, min(cores, 16))
    with mp.get_context("spawn").Pool(workers, initializer=_oracle_worker_init,
                                      initargs=(prob, n_gn, n_pcg)) as pool:
        pool.map(_oracle_edge_blocks, [(0, 1, prob.init_poses, 1.0)] * workers)  # workers set up
        t3 = time.perf_counter()
        _oracle_gn_iteration(s, prm, prob.init_poses, 0, pool=pool, chunks=8 * workers)
        t4 = time.perf_counter()
        # the whole solve: all n_gn iterations from the initial poses
        X = prob.init_poses.copy()
        for k in range(n_gn):
            X = _oracle_gn_iteration(s, prm, X, k, pool=pool, chunks=8 * workers)
        t5 = time.perf_counter()
    legs.append({"what": f"1 of {n_gn} GN iterations of the headline workload", "cores": workers,
                 "seconds": round(t4 - t3, 3), "gn_iters_per_s": round(1.0 / (t4 - t3), 4),
                 "how": "edge blocks in spawned worker processes, one per core; assembly and PCG in the parent"})
    legs.append({"what": f"all {n_gn} GN iterations of the headline workload (the whole solve, setup excluded)",
                 "cores": workers, "seconds": round(t5 - t4, 3), "gn_iters_per_s": round(n_gn / (t5 - t4), 4),
                 "how": "as the leg above"})
    log(f"oracle: one GN iteration on {workers} cores {t4 - t3:.2f} s, the whole solve {t5 - t4:.2f} s")
    with threadpool_limits(limits=1):
        if chunk is not None:
            t5 = time.perf_counter()
            solve_problem(chunk, Params(num_gn=chunk.n_gn, num_pcg=chunk.n_pcg), linear="pcg")
            dt = time.perf_counter() - t5
            legs.append({"what": f"11-frame chunk, full solve ({chunk.n_gn} GN x {chunk.n_pcg} PCG, setup "
                                 "included)", "cores": 1, "seconds": round(dt, 3), "solves_per_s": round(1 / dt, 3)})
            log(f"oracle: chunk solve {dt:.2f} s")
        refs = []
        if batch_sample:
            t6 = time.perf_counter()
            for c in batch_sample:
                refs.append(solve_problem(c, Params(num_gn=c.n_gn, num_pcg=c.n_pcg), linear="pcg")["poses"])
            dt = time.perf_counter() - t6
            legs.append({"what": f"{len(batch_sample)} of the 256 batched chunk problems (160x120, "
                                 f"{sum(c.num_frames for c in batch_sample)} frames), full solves, setup included",
                         "cores": 1, "seconds": round(dt, 3), "solves_per_s": round(len(batch_sample) / dt, 3)})
            log(f"oracle: {len(batch_sample)} batched chunks {dt:.2f} s")
            # the oracle's own sensitivity: the same solves from initial poses moved by
            # 1e-6 (rad and m, every free frame), not timed
            import copy
            from oracle.se3 import exp_se3
            moved = []
            for c in batch_sample:
                cm = copy.copy(c)
                cm.init_poses = c.init_poses.copy()
                for f in range(1, c.num_frames):
                    cm.init_poses[f] = cm.init_poses[f] @ exp_se3([1e-6, 0, 0, 1e-6, 0, 0])
                moved.append(solve_problem(cm, Params(num_gn=c.n_gn, num_pcg=c.n_pcg), linear="pcg")["poses"])
            refs = {"poses": refs, "moved": moved}
        if full:
            t7 = time.perf_counter()
            X = prob.init_poses.copy()
            for k in range(n_gn):
                X = _oracle_gn_iteration(s, prm, X, k)
            dt = time.perf_counter() - t7
            legs.append({"what": f"all {n_gn} GN iterations of the headline workload", "cores": 1,
                         "seconds": round(dt, 3), "gn_iters_per_s": round(n_gn / dt, 4)})
            log(f"oracle: full headline solve on 1 core {dt:.1f} s")
    return {"value": round(1.0 / one, 4), "unit": "GN iters/s", "cores": 1, "kind": "oracle",
            "sample": f"1 of {n_gn} Gauss-Newton iterations ({n_pcg} PCG) of the same workload, single thread; "
                      f"per-solve setup ({t1 - t0:.1f} s) excluded",
            "seconds": round(one, 3), "host_cpu_count": os.cpu_count(), "host_affinity_cores": cores,
            "legs": legs, "_batch_ref": refs}


def accuracy_vs_oracle(prob, poses, energy):
    """Pose and energy error of a headline-workload result against the oracle's
    iteration-matched FP64 run stored in tests/golden/global200_oracle.npz, and the
    distance by which the oracle's own run moves when its initial poses move by
    1e-6 (the iteration's sensitivity to a rounding-sized difference)."""
    import numpy as np
    path = os.path.join(ROOT, "tests", "golden", "global200_oracle.npz")
    if not os.path.exists(path):
        return None
    g = np.load(path, allow_pickle=False)

    def err(A, B):
        rot = max(float(np.arccos(np.clip((np.trace(A[f, :3, :3].T @ B[f, :3, :3]) - 1) / 2, -1, 1)))
                  for f in range(len(A)))
        return rot, max(float(np.linalg.norm(A[f, :3, 3] - B[f, :3, 3])) for f in range(len(A)))
    if g["poses"].shape != poses.shape or not np.array_equal(g["traj"][0], prob.init_poses):
        return None
    rot, tr = err(poses, g["poses"])
    srot, str_ = err(g["moved_poses"], g["poses"])
    er = float(g["energy"][0])
    return {"reference": "oracle FP64, same iteration counts (8 GN x 20 PCG, block-Jacobi)",
            "max_rot_rad": rot, "max_trans_m": tr, "energy_rel": abs(energy - er) / er,
            "oracle_self_sensitivity_to_1e-6_start": {"rad": srot, "m": str_}}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--oracle-full", action="store_true",
                    help="also time all 8 oracle GN iterations of the headline workload (about 2 minutes)")
    ap.add_argument("--bidirectional", type=int, default=0,
                    help="1: dense terms over the pixels of both frames of every pair")
    ap.add_argument("--pcg-storage", type=int, default=None,
                    help="0 FP32, 1 FP64 (default 0; 1 for global2000)")
    ap.add_argument("--accumulate", type=int, default=None,
                    help="0 FP32, 1 compensated FP32, 2 FP64 lane sums (default 0; 1 for global2000)")
    ap.add_argument("--solve-kernel", type=int, default=0)
    ap.add_argument("--dense-threads", type=int, default=0,
                    help="threads per dense pair job; 0 (default) = threads and tiles chosen by timing")
    ap.add_argument("--dense-tiles", type=int, default=1, help="workgroups (pixel tiles) per dense pair job")
    ap.add_argument("--preconditioner", type=int, default=0, help="0 = 6x6 block-Jacobi, 1 = scalar Jacobi")
    ap.add_argument("--workload", choices=["global200", "global2000"], default="global200",
                    help="global2000: the 2000-keyframe floor (8 GN x 20 PCG); only the solve is measured")
    ap.add_argument("--prune-rounds", type=int, default=0,
                    help="also time one solve with residual pruning (threshold 0.05 m) limited to this many removals")
    ap.add_argument("--extras", action="store_true",
                    help="also time the correspondence filters and the dense verification (one call each)")
    ap.add_argument("--skip-batched", action="store_true")
    ap.add_argument("--skip-serving", action="store_true")
    ap.add_argument("--serving-requests", type=int, default=300)
    ap.add_argument("--batched-steps", type=int, default=5)
    ap.add_argument("--copy-calibration-mib", type=int, default=0,
                    help="run a plain copy of this size first (for scaling HBM counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: the solve runs on one GPU; --gpus {args.gpus} is not supported "
              "(sharding across GPUs is a design only, not implemented)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_1604_01093_amd import bf
    from synth import make_batch_chunks, make_problem

    # inputs are generated before anything touches the GPU (the batch generator forks)
    big = args.workload == "global2000"
    if big:
        args.skip_batched = args.skip_serving = args.no_cpu_baseline = True
    # global2000 runs the mixed precision that keeps one GN step within 1e-5 of the
    # oracle (plain FP32 lane sums and PCG storage do not at that size)
    if args.accumulate is None:
        args.accumulate = 1 if big else 0
    if args.pcg_storage is None:
        args.pcg_storage = 1 if big else 0
    log(f"generating the {args.workload} workload")
    t0 = time.perf_counter()
    prob = make_problem(4 if big else 1)
    log(f"generated in {time.perf_counter() - t0:.1f} s: {prob.num_frames} frames, {len(prob.corr_i)} correspondences")
    chunks = None
    if not args.skip_batched:
        t0 = time.perf_counter()
        chunks = make_batch_chunks()
        log(f"generated 256 chunk problems in {time.perf_counter() - t0:.1f} s "
            f"({sum(c.num_frames for c in chunks)} frames)")
    pool = None
    if not args.skip_serving:
        from synth.problems import make_serving_pool
        t0 = time.perf_counter()
        pool = make_serving_pool()
        log(f"generated the serving request pool in {time.perf_counter() - t0:.1f} s: {len(pool[0])} chunks, "
            f"windows of {[w.num_frames for w in pool[1]]} keyframes")
    if args.copy_calibration_mib > 0:
        copy_calibration(args.copy_calibration_mib)

    ctx = bf.Context()
    dp = bf.DeviceProblem.from_numpy(prob.depth, prob.intensity, prob.intrinsics, prob.corr_i, prob.corr_j,
                                     prob.corr_p, prob.corr_q)
    init = torch.as_tensor(prob.init_poses).cuda()
    out = torch.empty_like(init)
    # timed region: HIP events around the dense launches only (timing = 2: each event
    # leaves the GPU idle for a few microseconds); the phase breakdown comes from a
    # separate, untimed pass with every phase marked (timing = 1)
    params = bf.bf_params_default(num_gn=prob.n_gn, num_pcg=prob.n_pcg, pcg_storage=args.pcg_storage,
                                  accumulate=args.accumulate, solve_kernel=args.solve_kernel, timing=2,
                                  bidirectional=args.bidirectional,
                                  dense_threads=args.dense_threads, dense_tiles=args.dense_tiles,
                                  preconditioner=args.preconditioner)
    st = bf.bf_build_structure(ctx, dp, init, params)
    P = st["pairs"].shape[0]
    log(f"structure: {P} dense pair jobs, {st['sparse_ij'].shape[0]} sparse pairs, {st['edges'].shape[0]} edges")

    for k in range(args.warmup):
        bf.bf_gauss_newton(ctx, dp, init, params, out_poses=out)
    torch.cuda.synchronize()
    log(f"warmup done ({args.warmup} steps)")

    dense_us = 0.0
    dense_launches = 0
    solve_us = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    last = t0
    for k in range(args.steps):
        res = bf.bf_gauss_newton(ctx, dp, init, params, out_poses=out)
        tm = ctx.last_timings()
        dense_us += tm["dense_us"]
        solve_us.append(tm["total_us"])
        dense_launches += int(tm["dense_launches"])
        if time.perf_counter() - last > 20:
            log(f"step {k + 1}/{args.steps}")
            last = time.perf_counter()
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    ms_per_step = 1000.0 * elapsed / args.steps
    value = prob.n_gn * args.steps / elapsed

    # the phase breakdown (every phase marked), outside the timed region
    pparams = bf.bf_params_default(num_gn=prob.n_gn, num_pcg=prob.n_pcg, pcg_storage=args.pcg_storage,
                                   accumulate=args.accumulate, solve_kernel=args.solve_kernel, timing=1,
                                   bidirectional=args.bidirectional,
                                   dense_threads=args.dense_threads, dense_tiles=args.dense_tiles,
                                   preconditioner=args.preconditioner)
    phase = np.zeros(8)
    n_phase = min(args.steps, 5)
    for k in range(n_phase):
        bf.bf_gauss_newton(ctx, dp, init, pparams, out_poses=out)
        tm = ctx.last_timings()
        phase += np.array([tm[key] for key in ("setup_us", "dense_us", "edges_us", "assemble_us", "pcg_us",
                                               "final_us", "total_us", "dense_launches")])
    phase /= n_phase

    shape = ctx.dense_shape()["jacobians"]
    avg_dense_s = dense_us / max(dense_launches, 1) * 1e-6
    jobs = P * (2 if args.bidirectional else 1)
    alg_bytes = BYTES_PER_SOURCE_PIXEL * prob.width * prob.height * jobs
    achieved = alg_bytes / avg_dense_s / 1e9
    log("per step (us): " + ", ".join(f"{n}={v:.1f}" for n, v in zip(
        ["setup", "dense", "edges", "assemble", "pcg", "final", "total", "dense_launches"], phase)))
    log(f"energy {res['energy']}")
    Pout = out.cpu().numpy()
    gt_rot = max(float(np.arccos(np.clip((np.trace(Pout[f, :3, :3].T @ prob.gt_poses[f][:3, :3]) - 1) / 2, -1, 1)))
                 for f in range(prob.num_frames))
    gt_tr = max(float(np.linalg.norm(Pout[f, :3, 3] - prob.gt_poses[f][:3, 3])) for f in range(prob.num_frames))
    log(f"largest pose error against the generator's ground truth: {gt_rot:.4f} rad, {gt_tr:.4f} m")

    line = {
        "metric": ("GN iters/sec (JᵀJ build+PCG) at 2000 keyframes" if big else
                   "GN iters/sec (JᵀJ build+PCG) at 200 keyframes; batched solves/sec; p99 latency"),
        "value": round(value, 3),
        "unit": "GN iters/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": ("global2000: 2000 keyframes, 80x60, 5x5-room floor, lawnmower path, " if big else
                                "global200: 200 keyframes, 80x60, 3-room apartment loop, ") +
                               f"{jobs} dense pair jobs{' (both directions)' if args.bidirectional else ''}, "
                               f"{len(prob.corr_i)} sparse correspondences, "
                               f"{prob.n_gn} GN x {prob.n_pcg} PCG",
                   "frames": prob.num_frames, "width": prob.width, "height": prob.height,
                   "dense_pairs": int(P), "dense_jobs": int(jobs), "correspondences": int(len(prob.corr_i)),
                   "gn_iters": prob.n_gn, "pcg_iters": prob.n_pcg,
                   "pcg_storage": "fp64" if args.pcg_storage else "fp32",
                   "accumulate": ["fp32", "fp32-two-sum", "fp64"][args.accumulate],
                   "solve_kernel": ["auto", "single", "coop", "replicated", "per-problem",
                                    "distributed"][args.solve_kernel],
                   "dense_launch": f"{shape[0]} threads x {shape[1]} tiles per pair job" +
                                   ("" if args.dense_threads else " (the timed choice)"),
                   "preconditioner": ["block-jacobi", "jacobi"][args.preconditioner]},
        "roofline": {"bound": "hbm", "kernel": "k_dense<jacobians>", "achieved": round(achieved, 1),
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": None if big else measured_traffic(*shape), "avg_launch_us": round(avg_dense_s * 1e6, 2),
                     "algorithmic_bytes_per_launch": int(alg_bytes)},
        "solve_us_hip_events": {"median": round(float(np.median(solve_us)), 1),
                                "p99": round(float(np.percentile(solve_us, 99)), 1)},
        # the GN iterations alone (dense pair jobs, edge blocks, PCG + update) with the
        # per-solve setup and the final energy left out, i.e. over cached structure
        "gn_iters_per_s_structure_cached": round(prob.n_gn * 1e6 / max(phase[1] + phase[2] + phase[3] + phase[4],
                                                                        1e-9), 1),
        "accuracy": {"max_rot_rad_vs_ground_truth": round(gt_rot, 6), "max_trans_m_vs_ground_truth": round(gt_tr, 6),
                     "vs_oracle": None if big else accuracy_vs_oracle(prob, Pout, res["energy"]["total"])},
        "phase_us_per_step": {n: round(v, 1) for n, v in zip(
            ["setup", "dense", "edges", "assemble", "pcg", "final", "total"], phase[:7])},
        "phase_note": "phases from a separate untimed pass with HIP events at every phase boundary (each "
                      "event adds a few microseconds of idle GPU time); the timed region marks only the dense "
                      "launches",
    }
    if args.extras:
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        keep, kept = bf.bf_filter_correspondences(ctx, dp)
        t_filter = time.perf_counter() - t0
        t0 = time.perf_counter()
        _, valid = bf.bf_verify_pairs(ctx, dp, st["pairs"], init, params)
        t_verify = time.perf_counter() - t0
        line["next_rows"] = {
            "keypoint_and_area_filters": {"ms": round(1e3 * t_filter, 3), "correspondences": len(prob.corr_i),
                                          "kept": int(kept)},
            "dense_verification": {"ms": round(1e3 * t_verify, 3), "pairs": int(P),
                                   "valid_at_init": int(valid.sum().item())}}
        log(f"filters: {kept} of {len(prob.corr_i)} kept in {1e3 * t_filter:.2f} ms; verification of {P} pairs "
            f"in {1e3 * t_verify:.2f} ms")
        # the paper's PCG variant (sparse term matrix-free in every iteration) against the
        # sparse term's assembled blocks, both in the distributed-vector kernel, and the
        # default kernel; PCG time per solve (row assembly + iterations + update)
        variants = {}
        for name, kw in (("default_kernel_assembled", {}), ("distributed_assembled", {"solve_kernel": 5}),
                         ("distributed_matrix_free_sparse", {"solve_kernel": 5, "sparse_matrix_free": 1})):
            pv = bf.bf_params_default(num_gn=prob.n_gn, num_pcg=prob.n_pcg, pcg_storage=args.pcg_storage,
                                      accumulate=args.accumulate, timing=1, dense_threads=args.dense_threads,
                                      dense_tiles=args.dense_tiles, **kw)
            pcg = []
            for r in range(6):
                res_v = bf.bf_gauss_newton(ctx, dp, init, pv, out_poses=out)
                if r >= 2:
                    pcg.append(ctx.last_timings()["pcg_us"])
            variants[name] = {"pcg_us_per_solve": round(float(np.median(pcg)), 1),
                              "energy": res_v["energy"]["total"]}
        line["next_rows"]["paper_solver_variant"] = variants
        log("PCG per solve: " + ", ".join(f"{k} {v['pcg_us_per_solve']} us" for k, v in variants.items()))
    if args.prune_rounds > 0:
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        pr = bf.bf_gauss_newton_pruned(ctx, dp, init, params, r_prune=0.05, max_rounds=args.prune_rounds)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        line["pruning"] = {"rounds": pr["rounds"], "seconds": round(dt, 4),
                           "ms_per_solve": round(1e3 * dt / (pr["rounds"] + 1), 3), "r_max": pr["rmax"],
                           "corr_active": int(pr["corr_active"].sum().item())}
        log(f"pruning: {pr['rounds']} removals in {dt * 1e3:.1f} ms, r_max {pr['rmax']:.4f} m")
    if chunks is not None:
        line["batched"] = batched(bf, ctx, chunks, args.batched_steps)
    if pool is not None:
        line["serving"] = serving(bf, ctx, pool, args.serving_requests)
    if args.no_cpu_baseline and "batched" in line:
        line["batched"].pop("_poses")
    if not args.no_cpu_baseline:
        log("timing the oracle on bounded samples")
        from synth import make_problem as _mp
        sample = chunks[:4] if chunks is not None else None
        line["cpu_baseline"] = cpu_baseline(prob, prob.n_gn, prob.n_pcg, chunk=_mp(0), batch_sample=sample,
                                            full=args.oracle_full)
        refs = line["cpu_baseline"].pop("_batch_ref")
        if chunks is not None and "batched" in line:
            line["batched"]["accuracy_vs_oracle"] = batched_accuracy(line["batched"].pop("_poses"), chunks[:4],
                                                                     refs)
    ctx.close()
    print(json.dumps(line), flush=True)


def batched(bf, ctx, chunks, steps):
    """256 chunk problems: one batched call per step vs one plain call per problem."""
    import numpy as np
    import torch

    n_gn, n_pcg = chunks[0].n_gn, chunks[0].n_pcg
    params = bf.bf_params_default(num_gn=n_gn, num_pcg=n_pcg, dense_threads=0, pcg_threads=-1)
    gparams = bf.bf_params_default(num_gn=n_gn, num_pcg=n_pcg, dense_threads=0, pcg_threads=-1, graph=1)
    dp, offs, init = bf.device_batch(chunks)
    out = torch.empty_like(init)
    gout = torch.empty_like(init)
    singles = [(bf.DeviceProblem.from_numpy(c.depth, c.intensity, c.intrinsics, c.corr_i, c.corr_j, c.corr_p,
                                            c.corr_q), torch.as_tensor(c.init_poses).cuda()) for c in chunks]
    singles_out = [torch.empty_like(i) for _, i in singles]
    torch.cuda.synchronize()
    log("batched: warm-up (first calls time the dense workgroup sizes)")
    for _ in range(2):
        res = bf.bf_gauss_newton_batch(ctx, dp, offs, init, params, out_poses=out)
        gres = bf.bf_gauss_newton_batch(ctx, dp, offs, init, gparams, out_poses=gout)
    for (d, i), o in zip(singles, singles_out):
        bf.bf_gauss_newton(ctx, d, i, params, out_poses=o)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        res = bf.bf_gauss_newton_batch(ctx, dp, offs, init, params, out_poses=out)
    torch.cuda.synchronize()
    t_eager = (time.perf_counter() - t0) / steps
    n_cap = ctx.graph_captures()
    t0 = time.perf_counter()
    for _ in range(steps):
        gres = bf.bf_gauss_newton_batch(ctx, dp, offs, init, gparams, out_poses=gout)
    torch.cuda.synchronize()
    t_batch = (time.perf_counter() - t0) / steps
    graph_same = bool(torch.equal(out, gout)) and gres["energy"] == res["energy"]
    first = gout[:offs[4]].cpu().numpy()
    tparams = bf.bf_params_default(num_gn=n_gn, num_pcg=n_pcg, dense_threads=0, pcg_threads=-1, timing=1)
    bf.bf_gauss_newton_batch(ctx, dp, offs, init, tparams, out_poses=out)
    phases = {k: round(v, 1) for k, v in ctx.last_timings().items()}
    log(f"batched phases (us, eager, timed call): {phases}")
    log(f"batched: graph replays {t_batch * 1e3:.3f} ms, eager launches {t_eager * 1e3:.3f} ms per batch; "
        f"captures during the timed replays {ctx.graph_captures() - n_cap}; graph result == eager: {graph_same}")
    batch_shape = ctx.dense_shape()["jacobians"]
    batch_pcg = ctx.pcg_threads()
    t0 = time.perf_counter()
    for (d, i), o in zip(singles, singles_out):
        bf.bf_gauss_newton(ctx, d, i, params, out_poses=o)
    torch.cuda.synchronize()
    t_seq = time.perf_counter() - t0
    P = out.cpu().numpy()

    def worst_diff(outs):
        wr = wt = 0.0
        for b, o in enumerate(outs):
            A, B = P[offs[b]:offs[b + 1]], o.cpu().numpy()
            for f in range(A.shape[0]):
                c = np.clip((np.trace(A[f, :3, :3].T @ B[f, :3, :3]) - 1.0) / 2.0, -1.0, 1.0)
                wr = max(wr, float(np.arccos(c)))
                wt = max(wt, float(np.linalg.norm(A[f, :3, 3] - B[f, :3, 3])))
        return {"rad": wr, "m": wt}
    own = worst_diff(singles_out)
    # the same problems one at a time with the batch's dense launch shape (not timed):
    # the per-problem kernels then sum in the same order, so the results are the batch's
    fixed = bf.bf_params_default(num_gn=n_gn, num_pcg=n_pcg, dense_threads=batch_shape[0], dense_tiles=batch_shape[1],
                                 pcg_threads=batch_pcg)
    for (d, i), o in zip(singles, singles_out):
        bf.bf_gauss_newton(ctx, d, i, fixed, out_poses=o)
    same = worst_diff(singles_out)
    nb = len(chunks)
    log(f"batched: {nb / t_batch:.1f} problems/s ({1e3 * t_batch:.2f} ms per batch); "
        f"one at a time: {nb / t_seq:.1f} problems/s ({1e3 * t_seq:.1f} ms)")
    return {"metric": "batched solves/sec", "value": round(nb / t_batch, 2), "unit": "solves/s",
            "sequential_value": round(nb / t_seq, 2), "speedup": round(t_seq / t_batch, 2),
            "ms_per_batch": round(1e3 * t_batch, 3), "steps": steps,
            "eager_value": round(nb / t_eager, 2), "graph_equals_eager": graph_same, "phase_us": phases,
            "_poses": [first[offs[b]:offs[b + 1]] for b in range(4)],
            "max_pose_diff_vs_sequential": {
                "same_dense_shape": same, "own_timed_shape": own,
                "note": "one at a time, each problem's own timed dense shape changes the order of the FP32 lane "
                        "sums; re-deciding the association at every iteration carries such rounding differences "
                        "to this size"},
            "config": {"workload": f"{nb} chunk problems, 4-11 frames (sum {offs[-1]}), 160x120, "
                                   f"{n_gn} GN x {n_pcg} PCG, dense launch {batch_shape[0]} threads x "
                                   f"{batch_shape[1]} tiles per pair job, per-problem PCG {batch_pcg} threads "
                                   f"(both timed per shape), "
                                   f"Gauss-Newton loop replayed as one HIP graph"}}



def batched_accuracy(poses, chunks, refs):
    """Largest pose error of the first batched problems against the oracle's solves of
    the same problems (same iteration counts, FP64), timed in the oracle leg, and how
    far the oracle's own solves move when their initial poses move by 1e-6."""
    import numpy as np

    def err(A, B, n):
        r = max(float(np.arccos(np.clip((np.trace(A[f, :3, :3].T @ B[f, :3, :3]) - 1) / 2, -1, 1)))
                for f in range(n))
        return r, max(float(np.linalg.norm(A[f, :3, 3] - B[f, :3, 3])) for f in range(n))
    worst = [0.0, 0.0]
    sens = [0.0, 0.0]
    for P, c, ref, mv in zip(poses, chunks, refs["poses"], refs["moved"]):
        e = err(P, ref, c.num_frames)
        m = err(mv, ref, c.num_frames)
        worst = [max(worst[0], e[0]), max(worst[1], e[1])]
        sens = [max(sens[0], m[0]), max(sens[1], m[1])]
    return {"problems": len(chunks), "max_rot_rad": worst[0], "max_trans_m": worst[1],
            "reference": "oracle FP64, same iteration counts",
            "oracle_self_sensitivity_to_1e-6_start": {"rad": sens[0], "m": sens[1]}}


def serving(bf, ctx, pool, n_requests):
    """Poisson request stream through the two-lane server vs one plain solve at a time."""
    import numpy as np
    import torch

    from paper_1604_01093_amd import serve

    chunks, wins = pool
    p_chunk = bf.bf_params_default(num_gn=5, num_pcg=10, dense_threads=256)
    p_glob = bf.bf_params_default(num_gn=8, num_pcg=20, dense_threads=256)
    items = []
    for pr in chunks:
        items.append(("chunk", pr, p_chunk))
    for pr in wins:
        items.append(("global", pr, p_glob))
    dev = [(bf.DeviceProblem.from_numpy(pr.depth, pr.intensity, pr.intrinsics, pr.corr_i, pr.corr_j, pr.corr_p,
                                        pr.corr_q), torch.as_tensor(pr.init_poses).cuda()) for _, pr, _ in items]
    rng = np.random.Generator(np.random.PCG64(7))
    is_global = rng.uniform(size=n_requests) < 0.2
    pick = np.where(is_global, len(chunks) + rng.integers(0, len(wins), n_requests),
                    rng.integers(0, len(chunks), n_requests))
    gaps = rng.exponential(size=n_requests)  # unit-rate Poisson process, scaled per run

    def make_reqs():
        return [serve.Request(dev[k][0], dev[k][1], items[k][2], tag=int(k)) for k in pick]

    # reference: each pool item solved alone (also warms up every shape)
    torch.cuda.synchronize()
    alone = []
    for (d, init), (_, pr, prm) in zip(dev, items):
        alone.append(bf.bf_gauss_newton(ctx, d, init, prm)["poses"])
    t0 = time.perf_counter()
    for k in pick:
        bf.bf_gauss_newton(ctx, dev[k][0], dev[k][1], items[k][2])
    torch.cuda.synchronize()
    t_plain_all = time.perf_counter() - t0

    server = serve.Server()
    try:
        # warm-up of the server's own contexts
        serve.run_stream(server, make_reqs()[:32], np.zeros(32))
        reqs = make_reqs()
        wall = serve.run_stream(server, reqs, np.zeros(n_requests))
        peak = n_requests / wall
        log(f"serving: peak {peak:.1f} solves/s (all requests at t=0); plain solves back to back "
            f"{n_requests / t_plain_all:.1f} solves/s")
        out = {"metric": "p99 latency", "unit": "ms", "requests": n_requests,
               "mix": "80% chunk (160x120, 4-11 frames, 5x10), 20% global window "
                      f"({min(w.num_frames for w in wins)}-{max(w.num_frames for w in wins)} keyframes, 80x60, 8x20)",
               "peak_solves_per_s": round(peak, 2), "plain_back_to_back_solves_per_s": round(n_requests / t_plain_all, 2),
               "rates": []}
        same = True
        for frac in (0.5, 0.8):
            rate = frac * peak
            arr = np.cumsum(gaps) / rate
            reqs = make_reqs()
            wall = serve.run_stream(server, reqs, arr)
            st = serve.latency_stats(reqs, wall)
            for cls in ("chunk", "global"):
                sub = [r for r in reqs if items[r.tag][0] == cls]
                lat = np.array([r.latency for r in sub if r.error is None]) * 1e3
                st[f"{cls}_p50_ms"] = round(float(np.percentile(lat, 50)), 3)
                st[f"{cls}_p99_ms"] = round(float(np.percentile(lat, 99)), 3)
            for r in reqs:
                same = same and r.error is None and torch.equal(r.poses, alone[r.tag])
            batches = [n for n, _ in server.batches[-200:]]
            plain = make_reqs()
            wall_p = serve.run_one_at_a_time(plain, arr, ctx)
            stp = serve.latency_stats(plain, wall_p)
            log(f"serving at {frac:.1f} x peak ({rate:.1f}/s): server p50 {st['p50_ms']} ms p99 {st['p99_ms']} ms, "
                f"{st['solves_per_s']} solves/s; one at a time p50 {stp['p50_ms']} ms p99 {stp['p99_ms']} ms")
            out["rates"].append({"fraction_of_peak": frac, "arrival_rate_per_s": round(rate, 2), "server": st,
                                 "one_at_a_time": stp,
                                 "mean_batch": round(float(np.mean(batches)), 2) if batches else None})
        out["value"] = out["rates"][-1]["server"]["p99_ms"]
        out["results_equal_alone"] = bool(same)
        return out
    finally:
        server.close()


if __name__ == "__main__":
    main()
