"""Bi-manual workload at full size (Sec. III-B): two uneven instruments
(20144 and 35388 triangles), 960x540, lambda = 512, 18-D with a
block-diagonal covariance, both arms in one launch, target with an occluding
rectangle over 10-30 % of the tools.

- The fused ask-eval launch leaves in its workspace the snapped vertices it
  rasterised; on sampled candidates the oracle's masks from those vertices
  (OR of both arms) and the counts against the target equal the kernel's
  counts exactly.
- Generations in two launches keep the covariance's off-diagonal blocks
  exactly zero and the losses finite.
- A generation captured in a HIP graph and replayed gives, replay after
  replay, the same bits as the same generations run eagerly."""
import numpy as np
import pytest
import torch

import oracle
import scenes
from paper_2603_11404_amd import tk, tracker

pytestmark = pytest.mark.gpu


def _problem():
    dev = torch.device("cuda:0")
    wl = scenes.workload("bimanual960")
    cam = wl["cam"]
    prob = tracker.Problem(wl["meshes"], wl["chains"], cam, dev)
    rng = scenes.rng_for(wl["index"], scenes.SUB_POSE)
    truth = np.concatenate([scenes.true_pose(rng, cam), scenes.true_pose(rng, cam)]).astype(np.float32)
    words = prob.render(torch.as_tensor(truth[None], device=dev))[0].cpu().numpy().view(np.uint64)
    img = scenes.words_to_image(words, cam.width, cam.height)
    rect, phi = scenes.occluder_rect(img, scenes.rng_for(wl["index"], scenes.SUB_OCCLUDER))
    occluded = scenes.apply_occluder(img, rect)
    removed = img.sum() - occluded.sum()
    assert img.sum() > 0 and phi * img.sum() <= removed
    target = scenes.image_to_words(occluded)
    prob.set_target(torch.as_tensor(target.view(np.int64), device=dev))
    return wl, prob, truth, target


def _generation(wl, prob, truth, seed=3):
    gen = tracker.Generation(prob, wl["lam"], loss_kind=tk.LOSS_IOU, n_blocks=wl["n_blocks"])
    scale = np.tile(scenes.DEFAULT_SCALE, 2)
    rng = np.random.default_rng(seed)
    gen.init(np.zeros(18), 1.0, truth + scale * rng.normal(size=18), scale, seed)
    return gen


def test_bimanual_ask_eval_counts_match_oracle():
    wl, prob, truth, target = _problem()
    cam = wl["cam"]
    gen = _generation(wl, prob, truth)
    tk.cmaes_ask_eval(gen.state, gen.n, gen.lam, prob.chains, prob.meshes, cam, prob.target, gen.X, gen.xf,
                      gen.counts, ws=gen.ws)
    torch.cuda.synchronize()
    V = [m.n_vertices for m in wl["meshes"]]
    snapped = gen.ws[:gen.lam * sum(V) * 8].view(torch.int32).view(gen.lam, sum(V), 2).cpu().numpy()
    counts = gen.counts.cpu().numpy()
    assert counts[:, 0].max() > 0
    for k in (0, 201, gen.lam - 1):
        mask = None
        for a, mesh in enumerate(wl["meshes"]):
            sn = snapped[k, sum(V[:a]):sum(V[:a]) + V[a]]
            fl = (sn[:, 0] == np.iinfo(np.int32).min).astype(np.uint8)
            s = np.where(fl[:, None].astype(bool), 0, sn).astype(np.int32)
            mask = oracle.raster(s, fl, mesh.triangles, cam.width, cam.height, mask=mask)
        a_cnt, inter, _ = oracle.counts(mask, target, cam.width, cam.height)
        assert (counts[k, 0], counts[k, 1]) == (a_cnt, inter), k


def test_bimanual_generations_keep_blocks():
    wl, prob, truth, _ = _problem()
    gen = _generation(wl, prob, truth)
    losses = []
    for _ in range(8):
        gen.ask_eval_tell()
        losses.append(gen.loss.cpu().numpy().min())
    v = tk.cmaes_view(gen.state, gen.n, gen.lam)
    C = v["C"].reshape(18, 18)
    assert np.all(C[:9, 9:] == 0.0) and np.all(C[9:, :9] == 0.0)
    assert np.all(np.isfinite(losses)) and np.all(np.isfinite(v["mean"]))
    assert min(losses) <= losses[0]


def test_bimanual_graph_replays_match_eager():
    wl, prob, truth, _ = _problem()
    eager = _generation(wl, prob, truth)
    graphed = _generation(wl, prob, truth)
    graphed.capture()            # runs one generation eagerly, then records one
    eager.ask_eval_tell()        # the same warm-up generation
    torch.cuda.synchronize()
    for r in range(4):
        graphed.replay()
        eager.ask_eval_tell()
        torch.cuda.synchronize()
        assert torch.equal(eager.counts, graphed.counts), r
        assert torch.equal(eager.state.view(torch.uint8), graphed.state.view(torch.uint8)), r
        assert torch.equal(eager.X.view(torch.int32), graphed.X.view(torch.int32)), r
