"""The fused tell-ask launch (tk_cmaes_tell_ask) against the separate calls it
replaces -- tk_compose_loss, tk_cmaes_update, tk_cmaes_sample and
tk_fk_transform -- generation after generation: losses, state blob,
candidates, link transforms and keypoints must agree bit for bit (one arm with
the keypoint term, one arm with the render loss, two arms with a
block-diagonal covariance)."""
import numpy as np
import pytest
import torch

import scenes
from paper_2603_11404_amd import tk, tracker

pytestmark = pytest.mark.gpu


def _bits(t):
    return t.contiguous().view(torch.uint8)


def _state_bits(g, ignore_z_gen):
    """State blob bytes; with ignore_z_gen the header's z_gen is left out (with
    18 dimensions the update does not pre-draw z, and an ask-eval prologue that
    draws them does not tag them, while the sampler does)."""
    b = _bits(g.state).clone()
    if ignore_z_gen:
        off = tk.cmaes_layout(g.n, g.lam)["z_gen"]
        b[off:off + 8] = 0
    return b


def _setup(n_arms, lam, kind, lambda_kp, seed=7):
    dev = torch.device("cuda:0")
    wl = scenes.workload("small")
    cam = wl["cam"]
    meshes = [wl["mesh"], scenes.instrument_mesh(32, 28, 3, 1, jaw_scale=1.3, box_scale=1.2)][:n_arms]
    chains = [scenes.chain(), scenes.chain(jaw_scale=1.3)][:n_arms]
    prob = tracker.Problem(meshes, chains, cam, dev)
    rng = scenes.rng_for(0, scenes.SUB_POSE)
    truth = np.concatenate([scenes.true_pose(rng, cam) for _ in range(n_arms)]).astype(np.float32)
    th = torch.as_tensor(truth[None], device=dev)
    prob.set_target(prob.render(th)[0], prob.keypoints(th)[0])
    scale = np.tile(scenes.DEFAULT_SCALE, n_arms)
    mean0 = truth + scale * rng.normal(size=9 * n_arms)
    gens = []
    for _ in range(2):
        g = tracker.Generation(prob, lam, loss_kind=kind, lambda_kp=lambda_kp)
        g.init(np.zeros(9 * n_arms), 1.0, mean0, scale, seed)
        g.ask()
        gens.append(g)
    return prob, gens


@pytest.mark.parametrize("n_arms,lam,kind,lambda_kp", [
    (1, 16, tk.LOSS_IOU, 0.1),
    (1, 64, tk.LOSS_RENDER, 0.0),
    (2, 32, tk.LOSS_IOU, 0.1),
])
def test_tell_ask_matches_separate_calls(n_arms, lam, kind, lambda_kp):
    prob, (a, b) = _setup(n_arms, lam, kind, lambda_kp)
    use_kp = lambda_kp != 0.0
    for gen in range(6):
        # separate calls
        tk.eval_fused(a.xf, a.lam, prob.meshes, prob.cam, prob.target, a.counts, a.ws)
        tk.compose_loss(a.counts, a.lam, prob.target_count, kind, a.loss, a.lambda_app,
                        a.kp if use_kp else None, prob.kp_ref if use_kp else None, n_arms, lambda_kp, a.tau)
        tk.cmaes_update(a.state, a.n, a.lam, a.loss)
        a.ask()
        # fused
        b.tell_ask()
        torch.cuda.synchronize()
        assert torch.equal(a.counts, b.counts), gen
        assert torch.equal(_bits(a.loss), _bits(b.loss)), gen
        assert torch.equal(_bits(a.state), _bits(b.state)), gen
        assert torch.equal(_bits(a.X), _bits(b.X)), gen
        assert torch.equal(_bits(a.xf), _bits(b.xf)), gen
        if use_kp:
            assert torch.equal(_bits(a.kp), _bits(b.kp)), gen


def test_tell_ask_argument_errors():
    prob, (a, _) = _setup(1, 16, tk.LOSS_IOU, 0.0)
    with pytest.raises(tk.TkError) as e:   # n must be 9 x n_arms
        tk.cmaes_tell_ask(a.state, a.n, a.lam, a.counts, prob.target_count, tk.LOSS_IOU, prob.chains * 2, prob.cam,
                          a.X, a.xf)
    assert e.value.status == tk.TK_ERR_INVALID_ARGUMENT
    with pytest.raises(tk.TkError):        # keypoints without reference
        tk.cmaes_tell_ask(a.state, a.n, a.lam, a.counts, prob.target_count, tk.LOSS_IOU, prob.chains, prob.cam,
                          a.X, a.xf, kp=a.kp)
    with pytest.raises(tk.TkError):        # bad loss kind
        tk.cmaes_tell_ask(a.state, a.n, a.lam, a.counts, prob.target_count, 7, prob.chains, prob.cam, a.X, a.xf)


@pytest.mark.parametrize("n_arms,lam,kind,lambda_kp", [
    (1, 16, tk.LOSS_IOU, 0.1),
    (1, 64, tk.LOSS_RENDER, 0.0),
    (2, 32, tk.LOSS_IOU, 0.1),
])
def test_ask_eval_and_tell_match_separate_calls(n_arms, lam, kind, lambda_kp):
    """tk_cmaes_ask_eval = sample + FK + fused raster counts; tk_cmaes_tell =
    compose + update: same bits as the separate calls, generation after
    generation (with and without a workspace)."""
    prob, (a, b) = _setup(n_arms, lam, kind, lambda_kp)
    use_kp = lambda_kp != 0.0
    for gen in range(6):
        ws_b = b.ws if gen % 2 == 0 else None
        # separate calls (a): sample -> FK -> fused raster -> compose -> update
        a.ask()
        tk.eval_fused(a.xf, a.lam, prob.meshes, prob.cam, prob.target, a.counts, a.ws)
        tk.compose_loss(a.counts, a.lam, prob.target_count, kind, a.loss, a.lambda_app,
                        a.kp if use_kp else None, prob.kp_ref if use_kp else None, n_arms, lambda_kp, a.tau)
        # fused (b)
        kp = b.kp if use_kp else None
        tk.cmaes_ask_eval(b.state, b.n, b.lam, prob.chains, prob.meshes, prob.cam, prob.target, b.X, b.xf,
                          b.counts, kp=kp, ws=ws_b)
        torch.cuda.synchronize()
        assert torch.equal(_state_bits(a, n_arms == 2), _state_bits(b, n_arms == 2)), gen   # Z and Y written by the draws
        assert torch.equal(_bits(a.X), _bits(b.X)), gen
        assert torch.equal(_bits(a.xf), _bits(b.xf)), gen
        if use_kp:
            assert torch.equal(_bits(a.kp), _bits(b.kp)), gen
        assert torch.equal(a.counts, b.counts), gen
        tk.cmaes_update(a.state, a.n, a.lam, a.loss)
        tk.cmaes_tell(b.state, b.n, b.lam, b.counts, prob.target_count, kind, n_arms, kp=kp,
                      kp_ref=prob.kp_ref if use_kp else None, lambda_kp=lambda_kp, loss=b.loss)
        torch.cuda.synchronize()
        assert torch.equal(_bits(a.loss), _bits(b.loss)), gen
        assert torch.equal(_state_bits(a, n_arms == 2), _state_bits(b, n_arms == 2)), gen


def test_ask_eval_argument_errors():
    prob, (a, _) = _setup(1, 16, tk.LOSS_IOU, 0.0)
    with pytest.raises(tk.TkError):        # n must be 9 x n_arms
        tk.cmaes_ask_eval(a.state, a.n, a.lam, prob.chains * 2, prob.meshes * 2, prob.cam, prob.target, a.X, a.xf,
                          a.counts)
    small_ws = torch.empty(8, dtype=torch.int64, device=a.ws.device)
    with pytest.raises(tk.TkError) as e:
        tk.cmaes_ask_eval(a.state, a.n, a.lam, prob.chains, prob.meshes, prob.cam, prob.target, a.X, a.xf, a.counts,
                          ws=small_ws)
    assert e.value.status == tk.TK_ERR_WORKSPACE_TOO_SMALL


@pytest.mark.parametrize("n_arms,lam", [(1, 64), (2, 48)])
def test_update_predraws_the_next_generation(n_arms, lam):
    """An update of up to 9 dimensions draws the next generation's z while it
    decomposes C and records that generation in the state (z_gen): the sampler
    draws the same bits for it, and an ask-eval launch that reads the drawn z
    produces the same candidates, counts and state as one that draws them
    itself.  With 18 dimensions the update leaves the draws to the ask-eval
    prologue (z_gen not advanced), with the same results."""
    prob, (a, b) = _setup(n_arms, lam, tk.LOSS_IOU, 0.1)
    for gen in range(4):
        tk.cmaes_write(b.state, b.n, b.lam, z_gen=-1)      # b draws in its ask-eval prologue
        a.ask_eval_tell()
        b.ask_eval_tell()
        torch.cuda.synchronize()
        for name in ("X", "xf", "counts", "loss"):
            assert torch.equal(_bits(getattr(a, name)), _bits(getattr(b, name))), (gen, name)
        assert torch.equal(_state_bits(a, n_arms == 2), _state_bits(b, n_arms == 2)), gen
        va = tk.cmaes_view(a.state, a.n, a.lam)
        assert va["gen"] == gen + 1
        if n_arms == 2:
            assert va["z_gen"] != gen + 1
            continue
        assert va["z_gen"] == gen + 1
        # the sampler's draws of that generation are the same bits
        c = a.state.clone()
        tk.cmaes_write(c, a.n, a.lam, z_gen=-1)
        X = torch.empty_like(a.X)
        tk.cmaes_sample(c, a.n, a.lam, X)
        torch.cuda.synchronize()
        assert np.array_equal(tk.cmaes_view(c, a.n, a.lam)["Z"].view(np.uint64), va["Z"].view(np.uint64)), gen
