"""Soft silhouette on the device (tk_soft_forward / tk_soft_backward) against
the FP64 oracle: S per pixel and the loss, dL/dtheta against the oracle's
analytic gradient and against its central differences (h = 1e-4 in the
normalised coordinates), one and two arms, faces on the big list, a candidate
out of view; determinism, upstream-gradient scaling and the autograd wrapper;
Adam on the CMA-ES mean against the plain update formula; refinement lowers
the soft loss."""
import numpy as np
import pytest
import torch

import oracle
import scenes
from paper_2603_11404_amd import soft, tk, tracker

pytestmark = pytest.mark.gpu

# FP32 projection, transcendental functions and sums against FP64; measured
# maxima over 36 candidate / sigma cases: 7e-6, 5e-7 and 5.3e-5
S_ATOL = 2e-5
LOSS_RTOL = 5e-6
GRAD_RTOL = 2e-4       # norm-wise


def _problem(meshes, chains, cam, truth, dev):
    prob = tracker.Problem(meshes, chains, cam, dev)
    target = oracle.render(truth, chains, meshes, cam)
    prob.set_target(torch.as_tensor(target.view(np.int64), device=dev))
    return prob, target


def _run(prob, theta32, sigma, dev, want_S=True):
    B = theta32.shape[0]
    th = torch.as_tensor(theta32, device=dev)
    xf = torch.empty(B, prob.n_arms, 4, 12, dtype=torch.float32, device=dev)
    tk.fk_transform(th, B, prob.n_arms, prob.chains, xf)
    ws = tk.soft_workspace(B, prob.meshes, prob.cam, dev)
    loss = torch.empty(B, dtype=torch.float64, device=dev)
    S = torch.empty(B, prob.cam.height, prob.cam.width, dtype=torch.float32, device=dev) if want_S else None
    tk.soft_forward(xf, B, prob.meshes, prob.cam, sigma, prob.target, loss, ws, S=S)
    g = torch.empty_like(th)
    tk.soft_backward(th, B, prob.chains, prob.meshes, prob.cam, sigma, g, ws)
    torch.cuda.synchronize()
    return loss.cpu().numpy(), (S.cpu().numpy() if want_S else None), g.cpu().numpy()


def _check(prob, meshes, chains, cam, target, theta32, sigma, dev, fd_for=()):
    loss, S, g = _run(prob, theta32, sigma, dev)
    n_arms = len(meshes)
    scale = np.tile(scenes.DEFAULT_SCALE, n_arms)
    for b in range(theta32.shape[0]):
        th64 = theta32[b].astype(np.float64)
        L, So, go = oracle.soft(th64, chains, meshes, cam, sigma, target, want_S=True, want_grad=True)
        assert np.max(np.abs(S[b] - So)) <= S_ATOL, (b, np.max(np.abs(S[b] - So)))
        assert abs(loss[b] - L) <= LOSS_RTOL * max(L, 1.0), (b, loss[b], L)
        if np.linalg.norm(go) > 0:
            rel = np.linalg.norm(g[b] - go) / np.linalg.norm(go)
            assert rel <= GRAD_RTOL, (b, rel, g[b], go)
        else:
            assert np.all(g[b] == 0.0)
        if b in fd_for:
            h = 1e-4
            fd = np.zeros(9 * n_arms)
            for k in range(9 * n_arms):
                e = np.zeros(9 * n_arms)
                e[k] = h * scale[k]
                fd[k] = (oracle.soft(th64 + e, chains, meshes, cam, sigma, target)[0] -
                         oracle.soft(th64 - e, chains, meshes, cam, sigma, target)[0]) / (2 * h)
            rel = np.linalg.norm(g[b] * scale - fd) / np.linalg.norm(fd)
            assert rel <= 1e-3, (b, rel)
    return loss, S, g


@pytest.mark.parametrize("sigma", [1.0, 0.7])
def test_soft_one_arm_matches_oracle(sigma):
    dev = torch.device("cuda:0")
    cam = scenes.camera(160, 120, 200.0)
    mesh, ch = scenes.instrument_mesh(24, 16, 2, 1), scenes.chain()
    rng = scenes.rng_for(0, scenes.SUB_POSE)
    truth = scenes.true_pose(rng, cam)
    prob, target = _problem([mesh], [ch], cam, truth, dev)
    cands = truth[None, :] + 0.5 * scenes.DEFAULT_SCALE[None, :] * rng.normal(size=(4, 9))
    far = truth.copy()
    far[3] += 5.0                                     # out of view: S = 0, loss = |M|, no gradient
    theta = np.concatenate([cands, far[None]]).astype(np.float32)
    loss, S, g = _check(prob, [mesh], [ch], cam, target, theta, sigma, dev, fd_for=(0,))
    assert S[4].max() == 0.0 and np.all(g[4] == 0.0)
    assert loss[4] == pytest.approx(float(scenes.words_to_image(target, 160, 120).sum()))


def test_soft_two_arms_match_oracle():
    dev = torch.device("cuda:0")
    cam = scenes.camera(160, 120, 200.0)
    meshes = [scenes.instrument_mesh(16, 12, 2, 1), scenes.instrument_mesh(20, 12, 2, 1, jaw_scale=1.3)]
    chains = [scenes.chain(), scenes.chain(1.3)]
    rng = scenes.rng_for(1, scenes.SUB_POSE)
    truth = np.concatenate([scenes.true_pose(rng, cam) for _ in range(2)])
    prob, target = _problem(meshes, chains, cam, truth, dev)
    theta = (truth[None, :] + 0.5 * np.tile(scenes.DEFAULT_SCALE, 2)[None, :] * rng.normal(size=(3, 18)))
    _check(prob, meshes, chains, cam, target, theta.astype(np.float32), 1.0, dev, fd_for=(1,))


def test_soft_big_faces_and_full_image():
    """A plane mesh whose faces span far more than 32 tiles (the big list)."""
    dev = torch.device("cuda:0")
    f = 128.0
    cam = scenes.Camera(f, f, 0.0, 0.0, 96, 72)
    tris = [[(3.0, 2.0), (90.0, 5.0), (10.0, 70.0)], [(60.0, 30.0), (95.0, 70.0), (40.0, 71.0)],
            [(20.0, 20.0), (24.0, 21.0), (21.0, 26.0)]]
    V = np.array([(u / f, v / f, 0.0) for tri in tris for (u, v) in tri], dtype=np.float32)
    mesh = scenes.Mesh(V, np.arange(9, dtype=np.int32).reshape(3, 3), np.zeros(9, dtype=np.uint8), {})
    ch = scenes.chain()
    truth = np.array([0, 0, 0, 0, 0, 1.0, 0, 0, 0.5])
    prob, target = _problem([mesh], [ch], cam, truth + np.array([0, 0, 0, 0.02, 0.01, 0, 0, 0, 0]), dev)
    theta = np.stack([truth, truth + np.array([0.01, 0.02, -0.01, 0.0, 0.0, 0.05, 0, 0, 0])]).astype(np.float32)
    _check(prob, [mesh], [ch], cam, target, theta, 1.0, dev)


def test_soft_deterministic_scaled_and_autograd():
    dev = torch.device("cuda:0")
    wl = scenes.workload("small")
    cam, mesh, ch = wl["cam"], wl["mesh"], scenes.chain()
    rng = scenes.rng_for(2, scenes.SUB_POSE)
    truth = scenes.true_pose(rng, cam)
    prob, _ = _problem([mesh], [ch], cam, truth, dev)
    theta = (truth[None, :] + scenes.DEFAULT_SCALE[None, :] * rng.normal(size=(6, 9))).astype(np.float32)
    l1, S1, g1 = _run(prob, theta, 1.0, dev)
    l2, S2, g2 = _run(prob, theta, 1.0, dev)
    assert np.array_equal(l1, l2) and np.array_equal(S1, S2) and np.array_equal(g1, g2)
    # upstream gradient scaling, through the autograd wrapper
    th = torch.as_tensor(theta, device=dev).requires_grad_(True)
    loss = soft.soft_loss(th, prob, 1.0)
    (loss * torch.arange(1, 7, dtype=torch.float64, device=dev)).sum().backward()
    torch.cuda.synchronize()
    assert np.array_equal(loss.detach().cpu().numpy(), l1)
    expect = g1 * np.arange(1, 7, dtype=np.float64)[:, None]
    np.testing.assert_allclose(th.grad.cpu().numpy(), expect.astype(np.float32), rtol=1e-6, atol=0)


def test_cmaes_adam_matches_the_update_formula():
    dev = torch.device("cuda:0")
    n, lam = 9, 16
    rng = np.random.default_rng(4)
    state = tk.cmaes_alloc(n, lam, dev)
    offset, scale = rng.normal(size=n), scenes.DEFAULT_SCALE
    mean0 = rng.normal(size=n)
    tk.cmaes_init(state, n, lam, mean0, 1.0, offset, scale, 3)
    adam = tk.adam_alloc(n, dev)
    tk.adam_reset(adam, n)
    x, m, v = mean0.copy(), np.zeros(n), np.zeros(n)
    lr, b1, b2, eps = 0.1, 0.9, 0.999, 1e-8
    for t in range(1, 8):
        g32 = rng.normal(size=n).astype(np.float32)
        tk.cmaes_adam(state, n, lam, torch.as_tensor(g32, device=dev), adam, lr, b1, b2, eps)
        g = g32.astype(np.float64) * scale
        m = b1 * m + (1 - b1) * g
        v = b2 * v + (1 - b2) * g * g
        x = x - lr * (m / (1 - b1 ** t)) / (np.sqrt(v / (1 - b2 ** t)) + eps)
    got = tk.cmaes_view(state, n, lam)["mean"]
    np.testing.assert_allclose(got, x, rtol=1e-13, atol=1e-14)
    X = torch.empty(n, dtype=torch.float32, device=dev)
    tk.cmaes_mean_candidate(state, n, lam, X)
    np.testing.assert_array_equal(X.cpu().numpy(), (offset + scale * got).astype(np.float32))


@pytest.mark.parametrize("n_arms", [1, 2])
def test_adam_transform_equals_the_separate_calls(n_arms):
    """tk_cmaes_adam_transform (the optional Adam step, the mean candidate and
    its link transforms in one launch) against tk_cmaes_adam,
    tk_cmaes_mean_candidate and tk_fk_transform, bit for bit, over several
    steps, one and two arms."""
    dev = torch.device("cuda:0")
    n, lam = 9 * n_arms, 16
    rng = np.random.default_rng(6 + n_arms)
    chains = [scenes.chain(), scenes.chain(jaw_scale=1.3)][:n_arms]
    offset = np.tile(scenes.true_pose(rng, scenes.camera(640, 480)), n_arms)
    scale = np.tile(scenes.DEFAULT_SCALE, n_arms)
    mean0 = rng.normal(size=n)
    st = [tk.cmaes_alloc(n, lam, dev) for _ in range(2)]
    ad = [tk.adam_alloc(n, dev) for _ in range(2)]
    for s_, a_ in zip(st, ad):
        tk.cmaes_init(s_, n, lam, mean0, 1.0, offset, scale, 3, n_blocks=n_arms)
        tk.adam_reset(a_, n)
    X = [torch.empty(n, dtype=torch.float32, device=dev) for _ in range(2)]
    xf = [torch.empty(n_arms, 4, 12, dtype=torch.float32, device=dev) for _ in range(2)]
    for k in range(5):
        g = torch.as_tensor(rng.normal(size=n).astype(np.float32), device=dev) if k > 0 else None
        tk.cmaes_adam_transform(st[0], n, lam, g, ad[0], chains, X[0], xf[0])
        if g is not None:
            tk.cmaes_adam(st[1], n, lam, g, ad[1])
        tk.cmaes_mean_candidate(st[1], n, lam, X[1])
        tk.fk_transform(X[1], 1, n_arms, chains, xf[1])
        torch.cuda.synchronize()
        assert torch.equal(X[0], X[1]), k
        assert torch.equal(xf[0].view(torch.int32), xf[1].view(torch.int32)), k
        assert torch.equal(ad[0].view(torch.int64), ad[1].view(torch.int64)), k
        v0, v1 = tk.cmaes_view(st[0], n, lam), tk.cmaes_view(st[1], n, lam)
        assert np.array_equal(np.asarray(v0["mean"]).view(np.int64), np.asarray(v1["mean"]).view(np.int64)), k


def test_refinement_lowers_the_soft_loss():
    dev = torch.device("cuda:0")
    wl = scenes.workload("small")
    cam, mesh, ch = wl["cam"], wl["mesh"], scenes.chain()
    rng = scenes.rng_for(3, scenes.SUB_POSE)
    truth = scenes.true_pose(rng, cam)
    prob, _ = _problem([mesh], [ch], cam, truth, dev)
    gen = tracker.Generation(prob, 16)
    gen.init(np.zeros(9), 1.0, truth + 0.5 * scenes.DEFAULT_SCALE * rng.normal(size=9), scenes.DEFAULT_SCALE, 9)
    first = float(gen.refine(steps=1, lr=0.1).item())
    last = None
    for _ in range(6):
        last = float(gen.refine(steps=5, lr=0.1).item())
    assert last < first


def test_soft_argument_errors():
    dev = torch.device("cuda:0")
    wl = scenes.workload("small")
    prob = tracker.Problem([wl["mesh"]], [scenes.chain()], wl["cam"], dev)
    xf = torch.zeros(1, 1, 4, 12, dtype=torch.float32, device=dev)
    loss = torch.empty(1, dtype=torch.float64, device=dev)
    ws = tk.soft_workspace(1, prob.meshes, prob.cam, dev)
    with pytest.raises(tk.TkError) as e:
        tk.soft_forward(xf, 1, prob.meshes, prob.cam, 0.0, prob.target, loss, ws)
    assert e.value.status == tk.TK_ERR_INVALID_ARGUMENT
    with pytest.raises(tk.TkError) as e:
        tk.soft_forward(xf, 1, prob.meshes, prob.cam, 1.0, prob.target, loss, ws[:1024])
    assert e.value.status == tk.TK_ERR_WORKSPACE_TOO_SMALL
    big = scenes.camera(2048, 2048)
    assert tk.soft_workspace_bytes(1, prob.meshes, big) == 0
    with pytest.raises(tk.TkError) as e:
        tk.soft_forward(xf, 1, prob.meshes, big, 1.0, prob.target, loss, ws)
    assert e.value.status == tk.TK_ERR_UNSUPPORTED


def test_soft_full_size_candidates_match_banded_oracle():
    """The differentiable form at its full size: the 49744-triangle instrument
    at 640x480, sigma = 1 px, six candidates of a 256-candidate launch (the
    batch the bench runs), against the oracle's face-major form of the same
    definitions: S per pixel, the loss and dL/dtheta."""
    dev = torch.device("cuda:0")
    wl = scenes.workload("soft640")
    mesh, cam, ch = wl["mesh"], wl["cam"], scenes.chain()
    rng = scenes.rng_for(wl["index"], scenes.SUB_POSE)
    truth = scenes.true_pose(rng, cam)
    prob, target = _problem([mesh], [ch], cam, truth, dev)
    theta = (truth[None] + scenes.DEFAULT_SCALE[None] * rng.normal(size=(wl["lam"], 9))).astype(np.float32)
    loss, S, g = _run(prob, theta, wl["sigma"], dev)
    # FP32 projected corners are off by up to about 4 ulp of the image
    # coordinates (6.1e-5 px near 640 px, four times the 160 px cases above),
    # and S moves by at most 1 / (4 sigma) per pixel of distance
    s_atol = 4.0 * float(np.spacing(np.float32(max(cam.width, cam.height)))) / (4.0 * wl["sigma"])
    for b in (0, 1, 77, 128, 200, wl["lam"] - 1):
        th64 = theta[b].astype(np.float64)
        print(f"soft640 candidate {b}", flush=True)
        L, So, go = oracle.soft(th64, [ch], [mesh], cam, wl["sigma"], target, want_S=True, want_grad=True,
                                banded=True)
        assert np.max(np.abs(S[b] - So)) <= s_atol, (b, np.max(np.abs(S[b] - So)), s_atol)
        assert abs(loss[b] - L) <= LOSS_RTOL * max(L, 1.0), (b, loss[b], L)
        assert np.linalg.norm(go) > 0
        assert np.linalg.norm(g[b] - go) <= GRAD_RTOL * np.linalg.norm(go), (b, np.linalg.norm(g[b] - go) /
                                                                              np.linalg.norm(go))


def test_soft_binning_forms_agree_bitwise():
    """Batches below 64 candidates bin across workgroups (LDS histograms and
    per-workgroup fill cursors), larger ones with one workgroup per candidate;
    the order of faces inside a tile list may differ, the forward sums are
    integers and the backward is face-major, so loss and gradient agree bit
    for bit."""
    dev = torch.device("cuda:0")
    wl = scenes.workload("track640")
    cam, mesh, ch = wl["cam"], wl["mesh"], scenes.chain()
    rng = scenes.rng_for(5, scenes.SUB_POSE)
    truth = scenes.true_pose(rng, cam)
    prob, _ = _problem([mesh], [ch], cam, truth, dev)
    theta = (truth[None] + scenes.DEFAULT_SCALE[None] * rng.normal(size=(64, 9))).astype(np.float32)
    l64, _, g64 = _run(prob, theta, 1.0, dev, want_S=False)
    for k0, k1 in [(0, 1), (3, 11), (20, 63)]:
        l, _, g = _run(prob, theta[k0:k1], 1.0, dev, want_S=False)
        np.testing.assert_array_equal(l, l64[k0:k1])
        np.testing.assert_array_equal(g, g64[k0:k1])


def test_generation_with_refinement_replays_as_a_graph():
    """A generation followed by 5 Adam steps on the mean, recorded once into a
    HIP graph and replayed, leaves the same state bit for bit as running it
    eagerly on a twin, replay after replay, with eager work in between."""
    dev = torch.device("cuda:0")
    wl = scenes.workload("small")
    cam, mesh, ch = wl["cam"], wl["mesh"], scenes.chain()
    rng = scenes.rng_for(8, scenes.SUB_POSE)
    truth = scenes.true_pose(rng, cam)
    prob, _ = _problem([mesh], [ch], cam, truth, dev)
    start = truth + 0.5 * scenes.DEFAULT_SCALE * rng.normal(size=9)
    gens = [tracker.Generation(prob, 16) for _ in range(2)]
    for g in gens:
        g.init(np.zeros(9), 1.0, start, scenes.DEFAULT_SCALE, 21)
    g_eager, g_graph = gens
    # capture() runs one warm-up generation + refinement before recording
    g_graph.capture(refine=(5, 0.1, 1.0))
    g_eager.ask_eval_tell()
    g_eager.refine(5, 0.1, 1.0)
    for _ in range(4):
        g_graph.replay()
        g_eager.ask_eval_tell()
        loss = g_eager.refine(5, 0.1, 1.0)
        torch.cuda.synchronize()
        assert torch.equal(g_graph.state, g_eager.state)
        assert torch.equal(g_graph._soft[4], loss)
