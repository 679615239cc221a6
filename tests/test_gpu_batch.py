"""Batched independent problems (the batching form of the tracker): problems
of mixed resolution (320x240 .. 1280x720), population size and mesh size run
through tk_batch_ask_eval / tk_batch_tell -- grouped by workgroup size, one
launch per group -- or tk_batch_ask_eval_persistent (all problems in one
persistent launch), and must give, generation after generation, the same bits
as each problem's own two-launch generation; sampled candidates' counts equal
the oracle's from the snapped vertices the kernel used; the workgroup size (a
tuning choice) does not change any result; persistent launches reset their
counter, also under graph capture and replay."""
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


# ---------------------------------------------------------------- persistent launch

def _persistent_shapes():
    sh = _shapes()
    # one large image in the launch: every problem then runs with 64-slot
    # narrow rings (drained before they overflow) and 1280x720 with fewer waves
    sh.append(dict(width=1280, height=720, lam=96, segments=32, rings=40, target_triangles=0))
    return sh


def test_persistent_matches_single_problem_generations():
    probs = _problems(_persistent_shapes())
    batch = tk.Batch([gens[0].problem_struct() for _, _, gens in probs])
    for gen in range(3):
        print(f"persistent generation {gen}", flush=True)
        batch.ask_eval_persistent()
        batch.tell()
        for _, _, gens in probs:
            gens[1].ask_eval_tell()
        torch.cuda.synchronize()
        for i, (_, _, (a, b)) in enumerate(probs):
            assert torch.equal(a.counts, b.counts), (gen, i)
            assert torch.equal(_bits(a.X), _bits(b.X)), (gen, i)
            assert torch.equal(_bits(a.xf), _bits(b.xf)), (gen, i)
            assert torch.equal(_bits(a.state), _bits(b.state)), (gen, i)
    # the launch resets its claim counter: the control words are zero again
    ctl = batch.table_view[-256:].cpu().numpy()        # one launch: the last 256 bytes
    assert not ctl.any()


def test_persistent_graph_replays_match_eager():
    probs = _problems(_persistent_shapes()[:5] + _persistent_shapes()[-1:])
    eager = tk.Batch([gens[0].problem_struct() for _, _, gens in probs])
    graphed = tk.Batch([gens[1].problem_struct() for _, _, gens in probs])
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        graphed.ask_eval_persistent()
        graphed.tell()
    torch.cuda.current_stream().wait_stream(s)
    eager.ask_eval_persistent()
    eager.tell()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        graphed.ask_eval_persistent()
        graphed.tell()
    for r in range(3):
        g.replay()
        eager.ask_eval_persistent()
        eager.tell()
        torch.cuda.synchronize()
        for i, (_, _, (a, b)) in enumerate(probs):
            assert torch.equal(a.counts, b.counts), (r, i)
            assert torch.equal(_bits(a.state), _bits(b.state)), (r, i)


def test_persistent_full_batch_recipe_sampled():
    """The 64-problem recipe at full size (320x240 .. 1280x720, lambda 64 ..
    1024, 2k .. 50k triangles) in one persistent launch: sampled problems,
    including the largest mesh and a lambda = 1024 problem, match their own
    generations bit for bit, and sampled candidates' counts equal the
    oracle's from the snapped vertices in their workspaces."""
    dev = torch.device("cuda:0")
    shapes = scenes.batch_problem_shapes(64)
    rng = scenes.rng_for(3, scenes.SUB_POSE)
    rng_f = scenes.rng_for(3, scenes.SUB_FLIPS)
    gens, meshes = [], []
    for i, sh in enumerate(shapes):
        cam = scenes.camera(sh["width"], sh["height"])
        mesh = scenes.instrument_mesh(sh["segments"], sh["rings"], 3, 1)
        prob = tracker.Problem([mesh], [scenes.chain()], cam, dev)
        truth = scenes.true_pose(rng, cam).astype(np.float32)
        th = torch.as_tensor(truth[None], device=dev)
        words = prob.render(th)[0].cpu().numpy().view(np.uint64)
        words = scenes.apply_flips(words, cam.width, cam.height, scenes.flip_indices(rng_f, cam.width, cam.height))
        prob.set_target(torch.as_tensor(words.view(np.int64), device=dev), prob.keypoints(th)[0])
        g = tracker.Generation(prob, sh["lam"], loss_kind=tk.LOSS_IOU, lambda_kp=0.1)
        g.init(np.zeros(9), 1.0, truth + scenes.DEFAULT_SCALE * rng.normal(size=9), scenes.DEFAULT_SCALE, 100 + i)
        gens.append(g)
        meshes.append(mesh)
    tris = [m.n_triangles for m in meshes]
    sample = sorted({int(np.argmax(tris)), next(i for i, s in enumerate(shapes) if s["lam"] == 1024),
                     next(i for i, s in enumerate(shapes) if s["width"] == 1280), 0, 33})
    twins = {}
    for i in sample:
        t = tracker.Generation(gens[i].p, gens[i].lam, loss_kind=tk.LOSS_IOU, lambda_kp=0.1)
        t.state.copy_(gens[i].state)
        twins[i] = t
    batch = tk.Batch([g.problem_struct() for g in gens])
    for gen in range(2):
        print(f"full recipe generation {gen}", flush=True)
        batch.ask_eval_persistent()
        batch.tell()
        for i in sample:
            twins[i].ask_eval_tell()
        torch.cuda.synchronize()
        for i in sample:
            assert torch.equal(gens[i].counts, twins[i].counts), (gen, i)
            assert torch.equal(_bits(gens[i].state), _bits(twins[i].state)), (gen, i)
    batch.ask_eval_persistent()
    torch.cuda.synchronize()
    for i in sample[:3]:
        g, mesh, cam = gens[i], meshes[i], gens[i].p.cam
        V = mesh.n_vertices
        snapped = g.ws[:g.lam * V * 8].view(torch.int32).view(g.lam, V, 2).cpu().numpy()
        target = g.p.target.cpu().numpy().view(np.uint64)
        counts = g.counts.cpu().numpy()
        for k in (0, g.lam - 1):
            sn = snapped[k]
            fl = (sn[:, 0] == np.iinfo(np.int32).min).astype(np.uint8)
            s = np.where(fl[:, None].astype(bool), 0, sn).astype(np.int32)
            mask = oracle.raster(s, fl, mesh.triangles, cam.width, cam.height)
            a_cnt, inter, _ = oracle.counts(mask, target, cam.width, cam.height)
            assert (counts[k, 0], counts[k, 1]) == (a_cnt, inter), (i, k)
