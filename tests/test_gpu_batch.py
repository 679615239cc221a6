"""Batched independent problems (the batching form of the tracker): problems
of mixed resolution (320x240 .. 1280x720), population size and mesh size run
through tk_batch_ask_eval / tk_batch_tell -- grouped by workgroup size, one
launch per group -- and must give, generation after generation, the same bits
as each problem's own two-launch generation; sampled candidates' counts equal
the oracle's from the snapped vertices the kernel used; the workgroup size (a
tuning choice) does not change any result."""
import numpy as np
import pytest
import torch

import oracle
import scenes
from paper_2603_11404_amd import tk, tracker

pytestmark = pytest.mark.gpu


def _problems(shapes, seed=5):
    dev = torch.device("cuda:0")
    rng = scenes.rng_for(3, scenes.SUB_POSE)
    out = []
    for i, sh in enumerate(shapes):
        cam = scenes.camera(sh["width"], sh["height"])
        mesh = scenes.instrument_mesh(sh["segments"], sh["rings"], 3, 1)
        prob = tracker.Problem([mesh], [scenes.chain()], cam, dev)
        truth = scenes.true_pose(rng, cam).astype(np.float32)
        th = torch.as_tensor(truth[None], device=dev)
        prob.set_target(prob.render(th)[0], prob.keypoints(th)[0])
        gens = []
        for _ in range(2):
            g = tracker.Generation(prob, sh["lam"], loss_kind=tk.LOSS_IOU, lambda_kp=0.1 if i % 2 else 0.0)
            g.init(np.zeros(9), 1.0, truth + scenes.DEFAULT_SCALE * np.random.default_rng(seed + i).normal(size=9),
                   scenes.DEFAULT_SCALE, seed + i)
            gens.append(g)
        out.append((prob, mesh, gens))
    return out


def _shapes():
    sh = scenes.batch_problem_shapes(10)
    for s in sh:                      # keep the test quick: at most 12k triangles, lambda <= 128
        s["rings"] = min(s["rings"], 90)
        s["lam"] = min(s["lam"], 128)
    return sh


def _bits(t):
    return t.contiguous().view(torch.uint8)


def test_batch_matches_single_problem_generations():
    probs = _problems(_shapes())
    batch = tk.Batch([gens[0].problem_struct() for _, _, gens in probs])
    for gen in range(3):
        batch.ask_eval()
        batch.tell()
        for _, _, gens in probs:
            gens[1].ask_eval_tell()
        torch.cuda.synchronize()
        for i, (_, _, (a, b)) in enumerate(probs):
            assert torch.equal(a.counts, b.counts), (gen, i)
            assert torch.equal(_bits(a.X), _bits(b.X)), (gen, i)
            assert torch.equal(_bits(a.xf), _bits(b.xf)), (gen, i)
            assert torch.equal(_bits(a.loss), _bits(b.loss)), (gen, i)
            assert torch.equal(_bits(a.state), _bits(b.state)), (gen, i)


def test_batch_counts_match_oracle_on_sampled_candidates():
    probs = _problems(_shapes()[:4])
    batch = tk.Batch([gens[0].problem_struct() for _, _, gens in probs])
    batch.ask_eval()
    torch.cuda.synchronize()
    for prob, mesh, (g, _) in probs:
        cam = prob.cam
        V = mesh.n_vertices
        snapped = g.ws[:g.lam * V * 8].view(torch.int32).view(g.lam, V, 2).cpu().numpy()
        target = prob.target.cpu().numpy().view(np.uint64)
        counts = g.counts.cpu().numpy()
        for k in (0, g.lam // 2, g.lam - 1):
            sn = snapped[k]
            fl = (sn[:, 0] == np.iinfo(np.int32).min).astype(np.uint8)
            s = np.where(fl[:, None].astype(bool), 0, sn).astype(np.int32)
            mask = oracle.raster(s, fl, mesh.triangles, cam.width, cam.height)
            a_cnt, inter, _ = oracle.counts(mask, target, cam.width, cam.height)
            assert (counts[k, 0], counts[k, 1]) == (a_cnt, inter), (cam.width, k)


def test_batch_workgroup_size_does_not_change_results():
    sh = [dict(width=640, height=480, lam=64, segments=32, rings=60, target_triangles=0)]
    (prob, _, (a, b)), = _problems(sh)
    tk.Batch([a.problem_struct(threads=0)]).ask_eval()
    tk.Batch([b.problem_struct(threads=256)]).ask_eval()
    torch.cuda.synchronize()
    assert torch.equal(a.counts, b.counts)
    assert torch.equal(_bits(a.state), _bits(b.state))


def test_batch_argument_errors():
    sh = [dict(width=1280, height=720, lam=64, segments=32, rings=30, target_triangles=0)]
    (prob, _, (a, _)), = _problems(sh)
    with pytest.raises(tk.TkError) as e:     # 1280x720 mask + 16 waves of queues exceed the LDS
        tk.Batch([a.problem_struct(threads=1024)])
    assert e.value.status == tk.TK_ERR_UNSUPPORTED
    bad = a.problem_struct()
    bad.d_ws = None
    with pytest.raises(tk.TkError):
        tk.Batch([bad])
