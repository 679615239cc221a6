"""Writes c1_pose_errors.json: final pose errors of 20-generation oracle
solves of the small workload (one 2044-triangle instrument, 320x240, f = 400,
lambda = 16, loss 1 - IoU against the render of a seeded true pose with 1 %
of the pixels flipped), one solve per seed.  Calls only oracle/ (FP64 forward
kinematics and projection, integer rasteriser, FP64 CMA-ES of Sec. III-A.1);
inputs come from scenes/.

Each solve starts at truth + scale * N(0, I) (the r-th draw of the workload's
CMA-ES sub-stream) with CMA-ES seed 11404 + r, sigma0 = 1 and mean 0 in the
normalised space.  The errors follow the metric of Sec. IV: translation of
the mean's pose, and the geodesic angle between the shaft rotations, after
choosing between the truth and its equivalent (beta + pi, -q1, -q2, q3) by
the smaller roll error.

Usage: python tests/golden/make_c1_pose_errors.py [n_solves]
"""
from __future__ import annotations

import json
import math
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle                      # noqa: E402
from oracle import cmaes           # noqa: E402
import scenes                      # noqa: E402

OUT = os.path.join(HERE, "c1_pose_errors.json")


def setup():
    wl = scenes.workload("small")
    mesh, cam = wl["mesh"], wl["cam"]
    chain = scenes.chain()
    truth = scenes.true_pose(scenes.rng_for(wl["index"], scenes.SUB_POSE), cam)
    flips = scenes.flip_indices(scenes.rng_for(wl["index"], scenes.SUB_FLIPS), cam.width, cam.height)
    target = scenes.apply_flips(oracle.render(truth, [chain], [mesh], cam), cam.width, cam.height, flips)
    return wl, mesh, cam, chain, truth, target


def starts(wl, truth, n):
    rng = scenes.rng_for(wl["index"], scenes.SUB_CMAES)
    return [truth + scenes.DEFAULT_SCALE * rng.normal(size=9) for _ in range(n)]


def errors(theta, truth, chain):
    """(translation m, rotation deg, flipped) of a physical estimate theta (qhat joints)."""
    def rot(th):
        return oracle.fk(th, chain)[0][:, :3]
    alt = np.array(truth, dtype=np.float64)
    alt[1] += math.pi
    for j in (0, 1):   # q1, q2 negated: in the unconstrained coordinate q -> -q is qhat -> -qhat for symmetric limits
        lb, ub = chain.q_lb[j], chain.q_ub[j]
        alt[6 + j] = oracle.encode(-oracle.decode(truth[6 + j], lb, ub), lb, ub)
    wrap = lambda a: abs((a + math.pi) % (2 * math.pi) - math.pi)
    flip = wrap(theta[1] - alt[1]) < wrap(theta[1] - truth[1])
    ref = alt if flip else truth
    d = np.linalg.norm(rot(theta) - rot(ref))
    ang = math.degrees(2.0 * math.asin(min(d / (2.0 * math.sqrt(2.0)), 1.0)))
    return float(np.linalg.norm(theta[3:6] - ref[3:6])), ang, bool(flip)


def solve(mesh, cam, chain, target, m_cnt, mean0, seed, lam, gens):
    es = cmaes.CMAES(9, lam, np.zeros(9), 1.0, mean0, scenes.DEFAULT_SCALE, seed)
    for _ in range(gens):
        theta = es.sample().astype(np.float32).astype(np.float64)
        cnt = oracle.eval_batch(theta, [chain], [mesh], cam, target)
        es.update(np.array([oracle.mask_loss(cnt[k, 0], cnt[k, 1], m_cnt, 0) for k in range(lam)]))
    return es.physical_mean()


def run(n):
    wl, mesh, cam, chain, truth, target = setup()
    m_cnt = oracle.counts(target, target, cam.width, cam.height)[2]
    rows = []
    for r, mean0 in enumerate(starts(wl, truth, n)):
        est = solve(mesh, cam, chain, target, m_cnt, mean0, scenes.BASE_SEED + r, wl["lam"], wl["gens"])
        t, a, f = errors(est, truth, chain)
        t0, a0, _ = errors(mean0, truth, chain)
        rows.append({"seed": scenes.BASE_SEED + r, "trans_mm": t * 1e3, "rot_deg": a, "flipped": f,
                     "start_trans_mm": t0 * 1e3, "start_rot_deg": a0})
    return rows


def main():
    n = int(sys.argv[1]) if len(sys.argv) > 1 else 40
    rows = run(n)
    tr = np.array([r["trans_mm"] for r in rows])
    ro = np.array([r["rot_deg"] for r in rows])
    doc = {"workload": "small: 2044-triangle instrument, 320x240, f=400, lambda=16, 20 generations, loss 1-IoU, "
                       "768 pixel flips",
           "generator": "tests/golden/make_c1_pose_errors.py (oracle only)",
           "solves": rows,
           "summary": {k: {"p10": float(np.percentile(v, 10)), "p25": float(np.percentile(v, 25)),
                           "median": float(np.median(v)), "p75": float(np.percentile(v, 75)),
                           "p90": float(np.percentile(v, 90)), "max": float(v.max())}
                       for k, v in (("trans_mm", tr), ("rot_deg", ro))}}
    with open(OUT, "w") as f:
        json.dump(doc, f, indent=1)
    print(json.dumps(doc["summary"]))


if __name__ == "__main__":
    main()
