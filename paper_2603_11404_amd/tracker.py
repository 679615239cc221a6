"""Generation driver: device buffers and launch sequence of one CMA-ES generation.

One generation (paper Sec. III-A.1: sample candidates, evaluate them in
parallel through batched forward kinematics and rendering, rank, update):

    tk_cmaes_sample -> tk_fk_transform -> tk_eval_fused -> tk_compose_loss
    -> tk_cmaes_update                                         (step)

or, fused into two launches per generation with identical results:

    tk_cmaes_ask_eval -> tk_cmaes_tell                         (ask_eval_tell)

where ask-eval draws the candidates, evaluates their forward kinematics and
their raster counts (one workgroup per candidate) and tell composes the
losses and updates the state.  A third form, tk_eval_fused -> tk_cmaes_tell_ask
(tell_ask, after ask()), draws the next generation inside the update launch.  All are HIP kernels of libtk
queued on one stream; `capture()` records a generation once into a HIP graph
(torch.cuda.CUDAGraph on ROCm) and `replay()` launches it with one call.
`step_plain()` is the unbatched baseline: the same kernels with batch = 1,
looped over the candidates.
"""
from __future__ import annotations

import numpy as np
import torch

from . import tk


class Problem:
    """Meshes (one per arm), chains, camera and observation resident on the device."""

    def __init__(self, meshes, chains, cam, device="cuda"):
        assert len(meshes) == len(chains)
        self.device = torch.device(device)
        self.meshes = [tk.DeviceMesh(m, self.device) for m in meshes]
        # the soft silhouette's copy: list order inside the claim-order blocks
        # (its face-major passes want neighbouring faces in neighbouring lanes)
        self.soft_meshes = [tk.DeviceMesh(m, self.device, plane_order=False) for m in meshes]
        self.chains = list(chains)
        self.cam = cam
        self.n_arms = len(meshes)
        self.words = tk.words_shape(cam)
        self.target = torch.zeros(self.words, dtype=torch.int64, device=self.device)
        self.target_count = torch.zeros(1, dtype=torch.int32, device=self.device)
        self.kp_ref = torch.zeros(self.n_arms, 4, 2, dtype=torch.float32, device=self.device)

    def set_target(self, target_words: torch.Tensor, kp_ref: torch.Tensor | None = None):
        """Copy a new observed mask (int64 view of the uint64 words) and keypoints in place."""
        self.target.copy_(target_words.view(self.words))
        tk.mask_popcount(self.target, 1, self.cam, self.target_count)
        if kp_ref is not None:
            self.kp_ref.copy_(kp_ref.view(self.n_arms, 4, 2))

    def render(self, theta: torch.Tensor) -> torch.Tensor:
        """Silhouette words of candidates theta [B, 9*n_arms] (float32, device)."""
        B = theta.shape[0]
        xf = torch.empty(B, self.n_arms, 4, 12, dtype=torch.float32, device=self.device)
        tk.fk_transform(theta.contiguous(), B, self.n_arms, self.chains, xf)
        masks = torch.empty(B, *self.words, dtype=torch.int64, device=self.device)
        tk.raster_silhouette(xf, B, self.meshes, self.cam, masks, tk.raster_workspace(B, self.meshes, self.device))
        return masks

    def transforms(self, theta: torch.Tensor) -> torch.Tensor:
        """Link transforms [B, n_arms, 4, 3, 4] of candidates theta [B, 9*n_arms] (FP32, device)."""
        B = theta.shape[0]
        xf = torch.empty(B, self.n_arms, 4, 12, dtype=torch.float32, device=self.device)
        tk.fk_transform(theta.contiguous(), B, self.n_arms, self.chains, xf)
        return xf.view(B, self.n_arms, 4, 3, 4)

    def keypoints(self, theta: torch.Tensor) -> torch.Tensor:
        B = theta.shape[0]
        xf = torch.empty(B, self.n_arms, 4, 12, dtype=torch.float32, device=self.device)
        kp = torch.empty(B, self.n_arms, 4, 2, dtype=torch.float32, device=self.device)
        tk.fk_transform(theta.contiguous(), B, self.n_arms, self.chains, xf, kp, self.cam)
        return kp


class Generation:
    """Buffers and launches of one CMA-ES generation over a Problem."""

    def __init__(self, problem: Problem, lam: int, loss_kind=tk.LOSS_IOU, lambda_app=1.0, lambda_kp=0.0,
                 tau=0.0, n_blocks=None):
        self.p = problem
        self.lam = int(lam)
        self.n = 9 * problem.n_arms
        self.n_blocks = problem.n_arms if n_blocks is None else n_blocks
        self.loss_kind, self.lambda_app, self.lambda_kp, self.tau = loss_kind, lambda_app, lambda_kp, tau
        d = problem.device
        self.state = tk.cmaes_alloc(self.n, self.lam, d)
        self.X = torch.empty(self.lam, self.n, dtype=torch.float32, device=d)
        self.xf = torch.empty(self.lam, problem.n_arms, 4, 12, dtype=torch.float32, device=d)
        self.kp = torch.empty(self.lam, problem.n_arms, 4, 2, dtype=torch.float32, device=d)
        self.counts = torch.empty(self.lam, 2, dtype=torch.int32, device=d)
        self.loss = torch.empty(self.lam, dtype=torch.float64, device=d)
        self.masks1 = torch.empty(1, *problem.words, dtype=torch.int64, device=d)
        self.ws = tk.raster_workspace(self.lam, problem.meshes, d)   # snapped vertices, one set per candidate
        self.graph = None

    def init(self, mean0, sigma0, offset, scale, seed, c_m_scale=1.0, c_mu_scale=1.0, c1_scale=1.0):
        tk.cmaes_init(self.state, self.n, self.lam, mean0, sigma0, offset, scale, seed, c_m_scale, c_mu_scale,
                      c1_scale, self.n_blocks)

    @property
    def use_kp(self) -> bool:
        return self.lambda_kp != 0.0

    def evaluate(self):
        """FK + fused raster/count + loss composition for the current X."""
        p = self.p
        tk.fk_transform(self.X, self.lam, p.n_arms, p.chains, self.xf, self.kp if self.use_kp else None,
                        p.cam if self.use_kp else None)
        tk.eval_fused(self.xf, self.lam, p.meshes, p.cam, p.target, self.counts, self.ws)
        tk.compose_loss(self.counts, self.lam, p.target_count, self.loss_kind, self.loss, self.lambda_app,
                        self.kp if self.use_kp else None, p.kp_ref if self.use_kp else None, p.n_arms,
                        self.lambda_kp, self.tau)

    def step(self):
        """One generation: sample -> FK -> raster/count -> loss -> update (5 launches)."""
        tk.cmaes_sample(self.state, self.n, self.lam, self.X)
        self.evaluate()
        tk.cmaes_update(self.state, self.n, self.lam, self.loss)

    def ask(self):
        """Draw the first generation after init() and evaluate its forward kinematics."""
        p = self.p
        tk.cmaes_sample(self.state, self.n, self.lam, self.X)
        tk.fk_transform(self.X, self.lam, p.n_arms, p.chains, self.xf, self.kp if self.use_kp else None,
                        p.cam if self.use_kp else None)

    def tell_ask(self):
        """Evaluate the current candidates (raster + counts), then one fused launch:
        losses, update, the next candidates and their forward kinematics."""
        p = self.p
        tk.eval_fused(self.xf, self.lam, p.meshes, p.cam, p.target, self.counts, self.ws)
        kp = self.kp if self.use_kp else None
        tk.cmaes_tell_ask(self.state, self.n, self.lam, self.counts, p.target_count, self.loss_kind, p.chains,
                          p.cam, self.X, self.xf, kp=kp, kp_ref=p.kp_ref if self.use_kp else None,
                          lambda_app=self.lambda_app, lambda_kp=self.lambda_kp, tau=self.tau, loss=self.loss,
                          kp_next=kp)

    def ask_eval_tell(self):
        """One generation in two launches: draw + FK + raster counts, then loss + update."""
        p = self.p
        kp = self.kp if self.use_kp else None
        tk.cmaes_ask_eval(self.state, self.n, self.lam, p.chains, p.meshes, p.cam, p.target, self.X, self.xf,
                          self.counts, kp=kp, ws=self.ws)
        tk.cmaes_tell(self.state, self.n, self.lam, self.counts, p.target_count, self.loss_kind, p.n_arms, kp=kp,
                      kp_ref=p.kp_ref if self.use_kp else None, lambda_app=self.lambda_app,
                      lambda_kp=self.lambda_kp, tau=self.tau, loss=self.loss)

    def refine(self, steps=5, lr=0.1, sigma=1.0):
        """Gradient refinement of the mean after a generation: `steps` Adam
        steps (Kingma and Ba defaults, learning rate lr in the normalised
        space, moments restarted for every call) on the soft-silhouette loss
        of the mean, each one tk_cmaes_mean_candidate -> tk_fk_transform ->
        tk_soft_forward -> tk_soft_backward -> tk_cmaes_adam, with each Adam
        step and the next mean candidate and its transforms in one launch
        (tk_cmaes_adam_transform).  Returns the device FP64 loss of the last
        evaluated mean."""
        p = self.p
        if getattr(self, "_soft", None) is None or self._soft[0] != sigma:
            d = p.device
            self._soft = (sigma, tk.soft_workspace(1, p.soft_meshes, p.cam, d),
                          torch.empty(1, self.n, dtype=torch.float32, device=d),
                          torch.empty(1, p.n_arms, 4, 12, dtype=torch.float32, device=d),
                          torch.empty(1, dtype=torch.float64, device=d),
                          torch.empty(1, self.n, dtype=torch.float32, device=d),
                          tk.adam_alloc(self.n, d))
        _, ws, X1, xf1, loss1, g1, adam = self._soft
        tk.adam_reset(adam, self.n)
        # each launch takes the previous step's Adam step (none before the
        # first) and forms the next mean candidate and its transforms
        for k in range(steps):
            tk.cmaes_adam_transform(self.state, self.n, self.lam, g1 if k > 0 else None, adam, p.chains, X1, xf1, lr)
            tk.soft_forward(xf1, 1, p.soft_meshes, p.cam, sigma, p.target, loss1, ws)
            tk.soft_backward(X1, 1, p.chains, p.soft_meshes, p.cam, sigma, g1, ws)
        if steps > 0:
            tk.cmaes_adam(self.state, self.n, self.lam, g1, adam, lr)
        return loss1

    def step_plain(self):
        """Unbatched baseline: the same kernels launched once per candidate (batch = 1)."""
        p = self.p
        tk.cmaes_sample(self.state, self.n, self.lam, self.X)
        for k in range(self.lam):
            tk.fk_transform(self.X[k:k + 1], 1, p.n_arms, p.chains, self.xf[k:k + 1],
                            self.kp[k:k + 1] if self.use_kp else None, p.cam if self.use_kp else None)
            tk.raster_silhouette(self.xf[k:k + 1], 1, p.meshes, p.cam, self.masks1, self.ws)
            tk.mask_loss(self.masks1, 1, p.target, p.cam, self.counts[k:k + 1])
            tk.compose_loss(self.counts[k:k + 1], 1, p.target_count, self.loss_kind, self.loss[k:k + 1],
                            self.lambda_app, self.kp[k:k + 1] if self.use_kp else None,
                            p.kp_ref if self.use_kp else None, p.n_arms, self.lambda_kp, self.tau)
        tk.cmaes_update(self.state, self.n, self.lam, self.loss)

    def capture(self, fused=True, refine=None):
        """Record one generation (ask_eval_tell(), or step() with fused=False)
        into a HIP graph, replayed by replay(); with refine = (steps, lr,
        sigma) the graph also holds the refinement of the mean that follows it."""
        gen = self.ask_eval_tell if fused else self.step

        def run():
            gen()
            if refine is not None:
                self.refine(*refine)
        s = torch.cuda.Stream(device=self.p.device)
        s.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(s):
            run()                # warm-up outside the graph on the side stream
        torch.cuda.current_stream().wait_stream(s)
        self.graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(self.graph):
            run()
        return self.graph

    def replay(self):
        self.graph.replay()

    def problem_struct(self, threads: int = 0) -> tk.Problem:
        """This generation as one problem of a batched launch (tk_problem)."""
        p = self.p
        P = tk.Problem()
        P.d_state = self.state.data_ptr()
        P.n, P.lambda_, P.n_arms = self.n, self.lam, p.n_arms
        for i in range(p.n_arms):
            P.meshes[i] = p.meshes[i].struct()
            P.chains[i] = tk.chain(p.chains[i])
        P.cam = tk.camera(p.cam)
        P.d_target = p.target.data_ptr()
        P.d_target_count = p.target_count.data_ptr()
        P.d_X, P.d_link_xf, P.d_counts = self.X.data_ptr(), self.xf.data_ptr(), self.counts.data_ptr()
        P.d_kp = self.kp.data_ptr() if self.use_kp else None
        P.d_ws, P.ws_bytes = self.ws.data_ptr(), self.ws.numel()
        P.kind, P.lambda_app, P.lambda_kp, P.tau = self.loss_kind, self.lambda_app, self.lambda_kp, self.tau
        P.d_kp_ref = p.kp_ref.data_ptr() if self.use_kp else None
        P.d_loss = self.loss.data_ptr()
        P.threads = int(threads)
        return P

    def mean(self) -> np.ndarray:
        v = tk.cmaes_view(self.state, self.n, self.lam)
        return v["offset"] + v["scale"] * v["mean"]


class Tracker:
    """Frame loop of Sec. III-A with the temporal filter of Sec. III-A.4.

    Per frame: begin_frame() sets the observation and starts CMA-ES from the
    previous frame's filtered estimate (the joint means from joint readings
    when given); the caller runs the frame's generations (e.g.
    Generation.ask_eval_tell()); end_frame() turns the CMA-ES mean into the
    filter's measurement (tk_cmaes_estimate: physical pose and joint angles)
    and filters it on the device (tk_kf_step: constant-velocity predict,
    update, joint clamp).  The next frame starts from the filtered estimate
    where it lies, in device memory (tk_cmaes_init_at); one asynchronous FP64
    copy of 3 x n values per frame brings the raw and filtered estimates to
    pinned host memory, read by collect() (end_frame() waits for its own
    frame).  With filt=None the raw estimate is passed through.

    Estimates in the filter's coordinates hold joint angles q; CMA-ES runs on
    the unconstrained joint coordinates qhat (the cosine map of Sec. III-A.3).
    warm_start: "filter" starts frame t+1 from the filtered estimate of frame
    t, "predict" from its constant-velocity prediction.  sigma0 and the
    learning-rate multipliers (c_m_scale, c_mu_scale) set up CMA-ES at every
    frame (the paper raises c_m and c_mu above their defaults without values)."""

    def __init__(self, gen: Generation, scale, gens_per_frame: int, seed0: int, filt: dict | None = None,
                 warm_start: str = "filter", sigma0: float = 1.0, c_m_scale: float = 1.0, c_mu_scale: float = 1.0):
        assert warm_start in ("filter", "predict")
        self.gen, self.p = gen, gen.p
        self.n = gen.n
        self.scale = np.asarray(scale, dtype=np.float64)
        self.G = int(gens_per_frame)
        self.seed0 = int(seed0)
        self.warm_start = warm_start
        self.sigma0, self.c_m_scale, self.c_mu_scale = float(sigma0), float(c_m_scale), float(c_mu_scale)
        d = self.p.device
        self.out = torch.empty(3, self.n, dtype=torch.float64, device=d)   # z, theta, theta_next
        self.kf = None
        self.d_row = None     # row of self.out that starts the next frame (None: start from self.est)
        self.pending = []     # pinned host copies of self.out, one per frame not yet collected
        if filt is not None:
            arms = self.p.n_arms
            tile = lambda a: np.tile(np.asarray(a, np.float64), arms)
            lo, hi = np.full(self.n, -np.inf), np.full(self.n, np.inf)
            for a, ch in enumerate(self.p.chains):
                lo[9 * a + 6:9 * a + 9] = ch.q_lb
                hi[9 * a + 6:9 * a + 9] = ch.q_ub
            vel = tile(filt["vel_std"])
            self.params = tk.kf_params(self.n, filt["dt"], p0_pos=tile(filt["meas_std"]) ** 2,
                                       p0_vel=(5.0 * vel) ** 2, q_pos=tile(filt["pos_std"]) ** 2, q_vel=vel ** 2,
                                       r=tile(filt["meas_std"]) ** 2, lo=lo, hi=hi)
            self.kf = tk.kf_alloc(self.n, d)
        self.est = None

    def start(self, est0):
        """Restart tracking from est0 (CMA-ES coordinates, [n]); restarts the
        filter at est0 with its joints as angles (cosine map on the device)."""
        self.est = np.array(est0, dtype=np.float64)
        self.d_row = None
        if self.kf is not None:
            x0 = np.clip(joint_angles(self.p, self.est)[0], self.params.lo[:self.n], self.params.hi[:self.n])
            tk.kf_init(self.kf, self.n, x0, self.params)

    def begin_frame(self, f: int, target=None, kp_ref=None, readings=None):
        """Observation of frame f (target words / keypoints, optional) and CMA-ES
        initialisation; readings: joint readings qhat [n_arms, 3] or None.  After
        an end of frame the start is read on the device (tk_cmaes_init_at), so
        the frame loop needs no host round trip; after start() it is est0."""
        if target is not None:
            self.p.set_target(target, kp_ref)
        if self.d_row is not None:
            r = None if readings is None else np.asarray(readings, np.float64).reshape(self.p.n_arms, 3)
            tk.cmaes_init_at(self.gen.state, self.n, self.gen.lam, self.out[self.d_row], self.p.chains, r,
                             self.sigma0, self.scale, self.seed0 + f, c_m_scale=self.c_m_scale,
                             c_mu_scale=self.c_mu_scale)
            return
        mean = self.est.copy()
        if readings is not None:
            r = np.asarray(readings, np.float64).reshape(self.p.n_arms, 3)
            for a in range(self.p.n_arms):
                mean[9 * a + 6:9 * a + 9] = r[a]
        self.gen.init(np.zeros(self.n), self.sigma0, mean, self.scale, self.seed0 + f, c_m_scale=self.c_m_scale,
                      c_mu_scale=self.c_mu_scale)

    def end_frame_async(self):
        """Measurement and filter step on the device, then an asynchronous copy
        of (raw, filtered, predicted) estimates into pinned host memory; the
        next begin_frame starts from the device copy.  No synchronisation."""
        g = self.gen
        tk.cmaes_estimate(g.state, self.n, g.lam, self.p.chains, self.out[0])
        if self.kf is not None:
            tk.kf_step(self.kf, self.n, self.out[0], self.out[1], self.out[2])
        host = torch.empty(3, self.n, dtype=torch.float64, pin_memory=True)
        host.copy_(self.out, non_blocking=True)
        self.pending.append(host)
        self.d_row = 0 if self.kf is None else (2 if self.warm_start == "predict" else 1)

    def collect(self) -> list:
        """Waits for the frames ended since the last collect and returns their
        {"z": raw estimate, "theta": filtered estimate} in the filter's coordinates."""
        torch.cuda.synchronize(self.p.device)
        out = []
        for host in self.pending:
            h = host.numpy()
            z = h[0].copy()
            th = h[1].copy() if self.kf is not None else z.copy()
            out.append({"z": z, "theta": th})
        self.pending = []
        return out

    def end_frame(self) -> dict:
        """end_frame_async() and collect() of this frame: {"z", "theta"}."""
        self.end_frame_async()
        return self.collect()[-1]


def pose_errors(problem: Problem, est, truth) -> dict:
    """Per-frame pose errors of estimates est [F, n] (filter coordinates: pose
    and joint angles) against truth [F, n] (CMA-ES coordinates, qhat joints),
    per arm, after resolving the instrument's two-fold ambiguity as Sec. IV
    prescribes: a roll of the shaft by pi with the wrist and jaw-mean angles
    negated, (beta + pi, -q1, -q2, q3), renders the same silhouette (the jaws
    trade places), so of the truth and that equivalent the one whose roll
    beta is closer to the estimate's (wrapped absolute difference) is scored.
    Returns rotation (geodesic angle between the two shaft rotations,
    degrees, from the device forward kinematics), translation (m), mean
    absolute joint-angle error (degrees) and, per frame and arm, whether the
    equivalent was taken ("flipped")."""
    est = np.asarray(est, np.float64)
    truth = np.asarray(truth, np.float64)
    F, arms = est.shape[0], problem.n_arms
    q_truth = joint_angles(problem, truth)                     # joints as angles (device cosine map)
    ref, flipped = symmetric_reference(est, q_truth, arms)
    # rotations of the shaft link from the device forward kinematics (only the
    # pose enters the shaft's transform, so the rows' joint angles, which the
    # forward kinematics would read as unconstrained coordinates, do not matter)
    th = torch.as_tensor(np.concatenate([est, ref]).astype(np.float32), device=problem.device)
    R = problem.transforms(th)[:, :, 0, :, :3].double().cpu().numpy()      # [2F, arms, 3, 3]
    # angle = 2 asin(|R_a - R_b|_F / (2 sqrt 2)): well conditioned for small angles
    diff = np.linalg.norm((R[:F] - R[F:]).reshape(F, arms, 9), axis=-1)
    rot = np.degrees(2.0 * np.arcsin(np.minimum(diff / (2.0 * np.sqrt(2.0)), 1.0)))
    out = {"rot_deg": rot, "trans_m": np.zeros((F, arms)), "joint_deg": np.zeros((F, arms)), "flipped": flipped}
    for a in range(arms):
        s = slice(9 * a, 9 * a + 9)
        out["trans_m"][:, a] = np.linalg.norm(est[:, s][:, 3:6] - ref[:, s][:, 3:6], axis=1)
        out["joint_deg"][:, a] = np.degrees(np.abs(est[:, s][:, 6:9] - ref[:, s][:, 6:9]).mean(axis=1))
    return out


def symmetric_reference(est, q_truth, n_arms):
    """The scoring reference of every frame and arm (Sec. IV): the truth
    q_truth [F, n] (filter coordinates) or its equivalent (beta + pi, -q1,
    -q2, q3), whichever has the roll beta closer to the estimate's, with
    angles compared modulo 2 pi (ties keep the truth).  Returns (ref [F, n],
    flipped [F, n_arms] bool)."""
    est = np.asarray(est, np.float64)
    ref = np.array(q_truth, dtype=np.float64, copy=True)
    flipped = np.zeros((ref.shape[0], n_arms), dtype=bool)
    wrap = lambda a: np.abs(np.remainder(a + np.pi, 2.0 * np.pi) - np.pi)
    for a in range(n_arms):
        o = 9 * a
        alt = ref[:, o:o + 9].copy()
        alt[:, 1] += np.pi
        alt[:, 6:8] *= -1.0
        flip = wrap(est[:, o + 1] - alt[:, 1]) < wrap(est[:, o + 1] - ref[:, o + 1])
        ref[flip, o:o + 9] = alt[flip]
        flipped[:, a] = flip
    return ref, flipped


# ------------------------------------------------------------------ joint coordinates on the device

def joint_angles(problem: Problem, theta) -> np.ndarray:
    """Rows theta [F, n] of CMA-ES coordinates (unconstrained joints qhat) as
    filter coordinates (joint angles q in the limits): the cosine map of Sec.
    III-A.3 evaluated by the device (tk_cmaes_estimate of a state whose
    offset is the row).  For set-up and evaluation, not for the frame loop."""
    theta = np.atleast_2d(np.asarray(theta, np.float64))
    n = 9 * problem.n_arms
    state = tk.cmaes_alloc(n, 2, problem.device)
    z = torch.empty(theta.shape[0], n, dtype=torch.float64, device=problem.device)
    for f, row in enumerate(theta):
        tk.cmaes_init(state, n, 2, np.zeros(n), 1.0, row, np.ones(n), 0)
        tk.cmaes_estimate(state, n, 2, problem.chains, z[f])
    return z.cpu().numpy()


def joint_coordinates(problem: Problem, q_theta) -> np.ndarray:
    """The inverse: rows q_theta [F, n] with joint angles (clamped to their
    limits) back to CMA-ES coordinates, by the device's inverse cosine map
    (tk_cmaes_init_at reads them as the offset of a state)."""
    q_theta = np.atleast_2d(np.asarray(q_theta, np.float64))
    n = 9 * problem.n_arms
    state = tk.cmaes_alloc(n, 2, problem.device)
    d = torch.as_tensor(q_theta, device=problem.device)
    out = np.empty_like(q_theta)
    for f in range(q_theta.shape[0]):
        tk.cmaes_init_at(state, n, 2, d[f], problem.chains, None, 1.0, np.ones(n), 0)
        out[f] = tk.cmaes_view(state, n, 2)["offset"]
    return out
