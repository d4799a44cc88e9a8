"""The serving loop (paper_1604_01093_amd.serve): small requests batched on one
lane while large ones run on the other, admission by device-memory footprint.

Each served result must equal, bit for bit, the result of the same request solved
alone by bf_gauss_newton (fixed dense workgroup size): batching and overlap change
when work runs, never what it computes.  Also: a budget that admits one request at
a time still completes every request with the same results, and a request larger
than the budget is refused with BF_ERR_OUT_OF_MEMORY."""
import numpy as np
import pytest
import torch

from synth.problems import make_batch_chunks, make_global, window

pytestmark = pytest.mark.gpu
bf = pytest.importorskip("paper_1604_01093_amd.bf")
serve = pytest.importorskip("paper_1604_01093_amd.serve")


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    c = bf.Context()
    yield c
    c.close()


@pytest.fixture(scope="module")
def g120():
    return make_global(120, "floor3", config=3, outlier_rate=0.10, corr_range=(200, 200), name="g120",
                       per_pair_streams=True)


@pytest.fixture(scope="module")
def pool(ctx, g120):
    chunks = make_batch_chunks(count=10, config=3)
    g = g120
    wins = [window(g, 5, 40), window(g, 20, 90)]
    p_chunk = bf.bf_params_default(num_gn=5, num_pcg=10, dense_threads=256)
    p_glob = bf.bf_params_default(num_gn=4, num_pcg=20, dense_threads=256)
    items = [(pr, p_chunk) for pr in chunks] + [(pr, p_glob) for pr in wins]
    dev = [(bf.DeviceProblem.from_numpy(pr.depth, pr.intensity, pr.intrinsics, pr.corr_i, pr.corr_j, pr.corr_p,
                                        pr.corr_q), torch.as_tensor(pr.init_poses).cuda(), prm) for pr, prm in items]
    alone = [bf.bf_gauss_newton(ctx, d, i, prm) for d, i, prm in dev]
    return dev, alone


def _requests(dev, picks):
    return [serve.Request(dev[k][0], dev[k][1], dev[k][2], tag=k) for k in picks]


def _check(reqs, alone):
    for r in reqs:
        assert r.error is None, r.error
        assert torch.equal(r.poses, alone[r.tag]["poses"]), r.tag
        assert r.energy == alone[r.tag]["energy"], r.tag


def test_mix_equals_alone(pool):
    dev, alone = pool
    rng = np.random.Generator(np.random.PCG64(3))
    picks = [int(k) for k in rng.integers(0, len(dev), 40)] + list(range(len(dev)))
    server = serve.Server()
    try:
        reqs = _requests(dev, picks)
        serve.run_stream(server, reqs, np.zeros(len(reqs)))       # all at once: large batches
        _check(reqs, alone)
        assert max(r.batch_size for r in reqs if r.lane == "batch") > 1
        assert {r.lane for r in reqs} == {"batch", "large"}
        reqs = _requests(dev, picks)
        arrivals = np.cumsum(rng.exponential(0.002, len(reqs)))    # a Poisson stream
        serve.run_stream(server, reqs, arrivals)
        _check(reqs, alone)
        assert all(r.t_done >= r.t_arrival for r in reqs)
    finally:
        server.close()


def test_admission_budget(pool):
    dev, alone = pool
    biggest = max(serve.Request(d, i, p).footprint for d, i, p in dev)
    server = serve.Server(max_inflight_bytes=biggest)
    try:
        reqs = _requests(dev, list(range(len(dev))) * 2)
        serve.run_stream(server, reqs, np.zeros(len(reqs)))
        _check(reqs, alone)
    finally:
        server.close()
    server = serve.Server(max_inflight_bytes=biggest - 1)
    try:
        big = [k for k in range(len(dev)) if serve.Request(*dev[k]).footprint == biggest][0]
        reqs = _requests(dev, [big, 0])
        serve.run_stream(server, reqs, np.zeros(2))
        assert reqs[0].error is not None and reqs[0].error.status == bf.BF_ERR_OUT_OF_MEMORY
        _check(reqs[1:], alone)
    finally:
        server.close()


def test_cancellation(pool):
    """With a budget that admits one request at a time the requests queue up:
    cancelling queued ones removes them (Cancelled, no result); cancelling the one
    that is running lets its GPU call finish and drops its result; every other
    request still equals its alone result bit for bit."""
    dev, alone = pool
    biggest = max(serve.Request(d, i, p).footprint for d, i, p in dev)
    server = serve.Server(max_inflight_bytes=biggest)
    try:
        reqs = _requests(dev, list(range(len(dev))) * 3)
        for r in reqs:
            server.submit(r)
        states = {}
        for k in (len(reqs) - 1, len(reqs) - 4, len(reqs) // 2):
            states[k] = server.cancel(reqs[k])
        with server.cv:   # a request that left its queue and has not completed is running
            running = next((r for r in reqs if r not in server.small and r not in server.large
                            and not r.done.is_set()), None)
        if running is not None:
            states[reqs.index(running)] = server.cancel(running)
        for r in reqs:
            r.done.wait()
        print("cancellation:", states, flush=True)
        assert "queued" in states.values()
        for k, r in enumerate(reqs):
            if k in states and states[k] != "done":
                assert isinstance(r.error, serve.Cancelled) and r.poses is None, (k, states[k])
            else:
                _check([r], alone)
        assert server.inflight == 0
    finally:
        server.close()


def test_warm_start(ctx, g120):
    """Warm start (paper Sec. 4.4: a solve starts from the last one's result): a
    request naming a problem key starts from the resident result of the last
    completed request of that key -- the same problem solved again, and then a grown
    problem (15 frames appended) whose 40 leading frames start from that result and
    the new ones from its own initial poses; a key with no resident result starts
    cold.  Each result equals bf_gauss_newton called alone with those initial
    poses, bit for bit."""
    prm = bf.bf_params_default(num_gn=4, num_pcg=20, dense_threads=256)

    def dev(pr):
        return (bf.DeviceProblem.from_numpy(pr.depth, pr.intensity, pr.intrinsics, pr.corr_i, pr.corr_j, pr.corr_p,
                                            pr.corr_q), torch.as_tensor(pr.init_poses).cuda())
    small, grown = dev(window(g120, 5, 40)), dev(window(g120, 5, 55))
    server = serve.Server()
    try:
        def run(d, key, warm):
            r = server.submit(serve.Request(d[0], d[1], prm, key=key, warm_start=warm))
            r.done.wait()
            assert r.error is None, r.error
            return r
        first = run(small, "w", False)
        assert first.warm_frames == 0
        again = run(small, "w", True)
        assert again.warm_frames == 40
        ref = bf.bf_gauss_newton(ctx, small[0], first.poses, prm)
        assert torch.equal(again.poses, ref["poses"]) and again.energy == ref["energy"]
        big = run(grown, "w", True)
        assert big.warm_frames == 40
        init = grown[1].clone()
        init[:40] = again.poses
        ref = bf.bf_gauss_newton(ctx, grown[0], init, prm)
        assert torch.equal(big.poses, ref["poses"]) and big.energy == ref["energy"]
        cold = run(small, "other", True)
        assert cold.warm_frames == 0
        ref = bf.bf_gauss_newton(ctx, small[0], small[1], prm)
        assert torch.equal(cold.poses, ref["poses"])
        print(f"warm start: energy {first.energy['total']:.6g} cold, {again.energy['total']:.6g} warm; grown problem "
              f"{big.energy['total']:.6g}", flush=True)
        server.forget("w")
        assert "w" not in server.resident
    finally:
        server.close()


def _input_bytes(d, init):
    ts = [d.depth, d.intensity, init] + (list(d.keep) if d.num_corrs > 0 else [])
    return sum(t.numel() * t.element_size() for t in ts)


def test_footprint_estimate_covers_workspace(pool):
    """The admission estimate (serve.footprint_bytes) of every request is at least
    the device memory its solve holds: the workspace of a fresh context after the
    solve (bf_workspace_bytes) plus the request's own input tensors; and for a
    batch of all the chunk requests, the sum of their estimates covers the batch
    context's workspace plus the concatenated inputs."""
    dev, _ = pool
    ratios = []
    for d, i, prm in dev:
        c = bf.Context()
        try:
            bf.bf_gauss_newton(c, d, i, prm)
            torch.cuda.synchronize()
            used = c.workspace_bytes() + _input_bytes(d, i)
        finally:
            c.close()
        est = serve.Request(d, i, prm).footprint
        ratios.append(est / used)
        assert est >= used, (d.num_frames, est, used)
    reqs = [serve.Request(d, i, prm) for d, i, prm in dev if prm is dev[0][2]]  # the chunks
    c = bf.Context()
    try:
        dp, offs, init = serve.concat_device(reqs)
        bf.bf_gauss_newton_batch(c, dp, offs, init, reqs[0].params)
        torch.cuda.synchronize()
        used = c.workspace_bytes() + _input_bytes(dp, init)
    finally:
        c.close()
    est = sum(r.footprint for r in reqs)
    print(f"footprint estimate / device bytes held: {min(ratios):.2f}..{max(ratios):.2f} per request, "
          f"{est / used:.2f} for a batch of {len(reqs)}", flush=True)
    assert est >= used


def test_warm_start_in_a_batch(ctx, pool):
    """Warm-started small requests batched together (their initial poses are the
    resident results, concatenated on the device with the members' frames): all
    eight submitted while the server's lock is held, so the batch lane takes them
    in one call; each result equals bf_gauss_newton alone from its resident
    result, bit for bit."""
    dev, _ = pool
    chunks = [(d, i, p) for d, i, p in dev if p is dev[0][2]][:8]
    server = serve.Server()
    try:
        firsts = [server.submit(serve.Request(d, i, p, key=f"chunk{k}")) for k, (d, i, p) in enumerate(chunks)]
        for r in firsts:
            r.done.wait()
            assert r.error is None, r.error
        warm = [serve.Request(d, i, p, key=f"chunk{k}", warm_start=True) for k, (d, i, p) in enumerate(chunks)]
        with server.cv:  # the lanes wait for the lock: every request is queued before one is taken
            for r in warm:
                server.submit(r)
        for r in warm:
            r.done.wait()
            assert r.error is None, r.error
        assert max(r.batch_size for r in warm) == len(warm)
        for k, r in enumerate(warm):
            d, _, p = chunks[k]
            assert r.warm_frames == d.num_frames
            ref = bf.bf_gauss_newton(ctx, d, firsts[k].poses, p)
            assert torch.equal(r.poses, ref["poses"]) and r.energy == ref["energy"], k
    finally:
        server.close()
