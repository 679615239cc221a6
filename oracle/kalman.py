"""Oracle of the temporal filter (Sec. III-A.4, Eq. (kf_motion) and the
observation model after it).

TEST INFRASTRUCTURE ONLY: used by the test suite; the product computes the
filter on the device.

State s = [theta; theta_dot] (2n).  Motion model s_t = F s_{t-1} + w_t with
F = [[I, dt I], [0, I]], w ~ N(0, Q); observation z_t = [I 0] s_t + v_t,
v ~ N(0, R), the CMA-ES estimate of the frame.  Standard predict / update in
the general 2n-dimensional matrix form (any symmetric PSD Q of 2n x 2n, any
SPD R); then the coordinates with limits (the joint angles) of the filtered
theta are clamped.  A non-finite z_i is a missing observation: the update
uses only the rows of H and R of the finite coordinates.
"""
from __future__ import annotations

import numpy as np


def block_noise(q_pos, q_cross, q_vel):
    """The 2n x 2n matrix [[diag(q_pos), diag(q_cross)], [diag(q_cross), diag(q_vel)]]."""
    q_pos, q_cross, q_vel = (np.atleast_1d(np.asarray(a, dtype=np.float64)) for a in (q_pos, q_cross, q_vel))
    return np.block([[np.diag(q_pos), np.diag(q_cross)], [np.diag(q_cross), np.diag(q_vel)]])


class KalmanCV:
    def __init__(self, x0, P0, Q, R, dt=1.0, lo=None, hi=None):
        x0 = np.asarray(x0, dtype=np.float64)
        n = x0.size
        self.n, self.dt = n, float(dt)
        I, Z = np.eye(n), np.zeros((n, n))
        self.F = np.block([[I, dt * I], [Z, I]])
        self.H = np.hstack([I, Z])
        self.Q = np.asarray(Q, dtype=np.float64).reshape(2 * n, 2 * n)
        self.R = np.asarray(R, dtype=np.float64).reshape(n, n)
        self.P = np.asarray(P0, dtype=np.float64).reshape(2 * n, 2 * n).copy()
        self.s = np.concatenate([x0, np.zeros(n)])
        self.lo = np.full(n, -np.inf) if lo is None else np.asarray(lo, np.float64)
        self.hi = np.full(n, np.inf) if hi is None else np.asarray(hi, np.float64)

    @classmethod
    def diagonal(cls, x0, p0_pos, p0_vel, q_pos, q_vel, r, dt=1.0, lo=None, hi=None, q_cross=0.0):
        n = np.asarray(x0).size
        b = lambda a: np.broadcast_to(np.asarray(a, np.float64), n)
        P0 = np.diag(np.concatenate([b(p0_pos), b(p0_vel)]))
        return cls(x0, P0, block_noise(b(q_pos), b(q_cross), b(q_vel)), np.diag(b(r)), dt, lo, hi)

    def step(self, z) -> np.ndarray:
        """One frame: predict, update with the measurement z, clamp; returns theta."""
        z = np.asarray(z, dtype=np.float64)
        # predict with the motion model
        s = self.F @ self.s
        P = self.F @ self.P @ self.F.T + self.Q
        # update with the observed coordinates
        obs = np.isfinite(z)
        if obs.any():
            H = self.H[obs]
            S = H @ P @ H.T + self.R[np.ix_(obs, obs)]
            K = P @ H.T @ np.linalg.inv(S)
            s = s + K @ (z[obs] - H @ s)
            P = (np.eye(2 * self.n) - K @ H) @ P
        self.P = 0.5 * (P + P.T)
        s[:self.n] = np.minimum(np.maximum(s[:self.n], self.lo), self.hi)
        self.s = s
        return s[:self.n].copy()

    def predicted(self) -> np.ndarray:
        """theta of the next frame under the motion model, clamped."""
        th = (self.F @ self.s)[:self.n]
        return np.minimum(np.maximum(th, self.lo), self.hi)
