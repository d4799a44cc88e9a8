"""The Gauss-Newton loop as one HIP graph launch (params.graph = 1).

* a batch solved with graph = 1 is bitwise the eager batch (poses, energies,
  trace) on the call that captures and on every replay, with other eager work and
  synchronisations of the program between the replays, and replays do not
  capture again;
* a replay reads the current contents of the buffers it was captured with: new
  initial poses written into the same tensor give the eager result for them;
* a different structure captures again, and so does coming back; every result is
  still bitwise the eager one; a plain chunk solve likewise;
* a solve whose PCG runs in a grid-wide kernel is refused."""
import numpy as np
import pytest
import torch

from oracle import Params
from synth import make_chunk

from gpu_helpers import bf_params_from

pytestmark = pytest.mark.gpu
bf = pytest.importorskip("paper_1604_01093_amd.bf")

W160 = dict(W=160, H=120, fx=144.0, fy=144.0, cx=80.0, cy=60.0, config=2)


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    c = bf.Context()
    yield c
    c.close()


@pytest.fixture(scope="module")
def chunks():
    return [make_chunk(num_frames=n, seed_offset=1000 * k, name=f"gchunk{k}", **W160)
            for k, n in enumerate([5, 7, 4, 6])]


def params(ch, graph, **kw):
    prm = Params(num_gn=ch.n_gn, num_pcg=ch.n_pcg)
    return bf_params_from(prm, dense_threads=kw.pop("dense_threads", 256), graph=graph, **kw)


def same(res, ref):
    assert torch.equal(res["poses"], ref["poses"])
    assert res["energy"] == ref["energy"]
    assert res["trace"] == ref["trace"]


def batch(ctx, dp, offs, init, prm, out):
    return bf.bf_gauss_newton_batch(ctx, dp, offs, init, prm, out_poses=out, trace=True)


def test_graph_batch_replays_equal_eager(ctx, chunks):
    dp, offs, init = bf.device_batch(chunks)
    ref = batch(ctx, dp, offs, init, params(chunks[0], 0), torch.empty_like(init))
    ref = dict(ref, poses=ref["poses"].clone())
    # eager work run between the replays, once beforehand so that it allocates nothing new later
    side = bf.DeviceProblem.from_numpy(chunks[1].depth, chunks[1].intensity, chunks[1].intrinsics, chunks[1].corr_i,
                                       chunks[1].corr_j, chunks[1].corr_p, chunks[1].corr_q)
    side_init = torch.as_tensor(chunks[1].init_poses).cuda()
    side_ref = bf.bf_gauss_newton(ctx, side, side_init, params(chunks[1], 0))["poses"].clone()
    out = torch.empty_like(init)
    n0 = ctx.graph_captures()
    for rep in range(4):
        out.fill_(-1.0)
        res = batch(ctx, dp, offs, init, params(chunks[0], 1), out)
        print(f"replay {rep}: captures {ctx.graph_captures() - n0}", flush=True)
        same(res, ref)
        s = bf.bf_gauss_newton(ctx, side, side_init, params(chunks[1], 0))["poses"]
        assert torch.equal(s, side_ref)
        torch.cuda.synchronize()
        assert float((init * 2.0).sum()) == float(init.sum()) * 2.0
    assert ctx.graph_captures() - n0 == 1


def test_graph_replay_reads_new_inputs(ctx, chunks):
    dp, offs, init = bf.device_batch(chunks)
    out = torch.empty_like(init)
    batch(ctx, dp, offs, init, params(chunks[0], 1), out)
    n0 = ctx.graph_captures()
    moved = init.clone()
    gauge = np.array(offs[:-1])
    step = torch.full((init.shape[0],), 0.004, dtype=torch.float64, device=init.device)
    step[torch.as_tensor(gauge, device=init.device)] = 0.0
    moved[:, 0, 3] += step
    ref = batch(ctx, dp, offs, moved, params(chunks[0], 0), torch.empty_like(init))
    init.copy_(moved)          # same tensor, new contents
    res = batch(ctx, dp, offs, init, params(chunks[0], 1), out)
    same(res, ref)
    print(f"captures for new contents: {ctx.graph_captures() - n0}", flush=True)


def test_graph_recaptures_for_new_structure(ctx, chunks):
    dpa, offa, inita = bf.device_batch(chunks)
    dpb, offb, initb = bf.device_batch(chunks[1:3])
    refa = batch(ctx, dpa, offa, inita, params(chunks[0], 0), torch.empty_like(inita))
    refb = batch(ctx, dpb, offb, initb, params(chunks[0], 0), torch.empty_like(initb))
    outa, outb = torch.empty_like(inita), torch.empty_like(initb)
    n0 = ctx.graph_captures()
    same(batch(ctx, dpa, offa, inita, params(chunks[0], 1), outa), refa)
    same(batch(ctx, dpb, offb, initb, params(chunks[0], 1), outb), refb)
    same(batch(ctx, dpa, offa, inita, params(chunks[0], 1), outa), refa)
    assert ctx.graph_captures() - n0 >= 2
    # the dense workgroup size chosen by timing is settled before capture
    t0 = batch(ctx, dpa, offa, inita, params(chunks[0], 0, dense_threads=0), torch.empty_like(inita))
    t1 = batch(ctx, dpa, offa, inita, params(chunks[0], 1, dense_threads=0), outa)
    same(t1, t0)


def test_graph_bidirectional_fp64_batch(ctx, chunks):
    """Both dense directions and FP64 PCG storage: replays bitwise the eager call."""
    dp, offs, init = bf.device_batch(chunks)
    kw = dict(bidirectional=1, pcg_storage=1)
    ref = batch(ctx, dp, offs, init, params(chunks[0], 0, **kw), torch.empty_like(init))
    ref = dict(ref, poses=ref["poses"].clone())
    out = torch.empty_like(init)
    n0 = ctx.graph_captures()
    for rep in range(3):
        same(batch(ctx, dp, offs, init, params(chunks[0], 1, **kw), out), ref)
        torch.cuda.synchronize()
    assert ctx.graph_captures() - n0 == 1


def test_graph_plain_chunk(ctx, chunks):
    ch = chunks[1]
    dp = bf.DeviceProblem.from_numpy(ch.depth, ch.intensity, ch.intrinsics, ch.corr_i, ch.corr_j, ch.corr_p,
                                     ch.corr_q)
    init = torch.as_tensor(ch.init_poses).cuda()
    ref = bf.bf_gauss_newton(ctx, dp, init, params(ch, 0), trace=True)
    ref = dict(ref, poses=ref["poses"].clone())
    out = torch.empty_like(init)
    n0 = ctx.graph_captures()
    for rep in range(3):
        res = bf.bf_gauss_newton(ctx, dp, init, params(ch, 1), out_poses=out, trace=True)
        same(res, ref)
        torch.cuda.synchronize()
    assert ctx.graph_captures() - n0 == 1


def test_graph_refused_for_grid_pcg(ctx, chunks):
    ch = chunks[0]
    dp = bf.DeviceProblem.from_numpy(ch.depth, ch.intensity, ch.intrinsics, ch.corr_i, ch.corr_j, ch.corr_p,
                                     ch.corr_q)
    init = torch.as_tensor(ch.init_poses).cuda()
    for kernel in (2, 3):
        with pytest.raises(bf.BFError) as e:
            bf.bf_gauss_newton(ctx, dp, init, params(ch, 1, solve_kernel=kernel))
        assert e.value.status == bf.BF_ERR_UNSUPPORTED
    ok = bf.bf_gauss_newton(ctx, dp, init, params(ch, 0, solve_kernel=3))
    assert np.isfinite(ok["energy"]["total"])
