"""One step of the gradient refinement of a node's stored points -- plain
float64 definition (CPU oracle).

TEST INFRASTRUCTURE ONLY (see the package docstring).

The paper asks that the reduced data be indistinguishable from the full data
when drawn; the refinement reading makes that a loss over a node's n stored
points.  For views v = 1..V with P pixels each, full render F_v (every
particle inside the node's cube) and its mean Fbar_v, and the render I_v of
the stored points with masses m_k = exp(theta_k) and positions x_k:

    L = 1/(V P) sum_v sum_p (log1p(I_v,p / Fbar_v) - log1p(F_v,p / Fbar_v))^2

    dL/dI_v,p = 2 (log1p(I_v,p/Fbar_v) - log1p(F_v,p/Fbar_v)) / ((Fbar_v + I_v,p) V P)
    dL/dtheta_k = m_k dL/dm_k      (chain rule through m = exp(theta))

with dL/dm and dL/dx from the float64 splat adjoint (`splat.render_backward`).

A step is Adam (Kingma and Ba, "Adam: a method for stochastic optimization",
ICLR 2015, Algorithm 1; beta1 = 0.9, beta2 = 0.999, eps = 1e-8) on theta and
on the positions, each with its own learning rate:

    m_t = beta1 m_{t-1} + (1 - beta1) g_t
    v_t = beta2 v_{t-1} + (1 - beta2) g_t^2
    p_t = p_{t-1} - lr (m_t / (1 - beta1^t)) / (sqrt(v_t / (1 - beta2^t)) + eps)

followed by clamping every position to the node's cube [lo, lo + side] and
shifting theta so that sum_k exp(theta_k) equals the node mass M:
theta <- theta - (log sum_k exp(theta_k) - log M).
"""
from __future__ import annotations

import math

import numpy as np

from . import splat

BETA1, BETA2, EPS = 0.9, 0.999, 1e-8


def loss_and_grad(cams, targets, x, y, z, m, sigma=1.0, radius_sigmas=3.0, image_rel_err=None):
    """Loss, dL/dm [n] and dL/dx [n, 3] in float64 for float32 positions and
    masses.  targets: list of (F_v float64 image, Fbar_v), one per camera.
    dL/dtheta for theta = log m is m dL/dm (`grad_theta`).

    With image_rel_err = e, also returns bounds (bL, bm [n], bxyz [n, 3]) on
    how far an evaluation can land from these float64 values when its images
    (I and F, hence Fbar) carry relative errors up to e per pixel and its
    adjoint sums carry relative errors up to e per term: a pixel's residual
    r = log1p(I/Fbar) - log1p(F/Fbar) then moves by at most 4 e, its term
    r^2 by 8 e |r| + 16 e^2, and its dL/dI by c (4 e) / (Fbar + I) + 3 e |dL/dI|
    (c = 2 / (V P)); the latter is pushed through the absolute adjoint.
    """
    m32 = np.asarray(m, dtype=np.float32)
    V = len(cams)
    L = 0.0
    bL = 0.0
    gm = np.zeros(len(m32))
    gx = np.zeros((len(m32), 3))
    bm = np.zeros(len(m32))
    bx = np.zeros((len(m32), 3))
    for cam, (F, Fbar) in zip(cams, targets):
        I = splat.render(cam, x, y, z, m32, sigma, radius_sigmas)
        P = I.size
        r = np.log1p(I / Fbar) - np.log1p(F / Fbar)
        L += math.fsum((r * r).ravel().tolist()) / (V * P)
        gI = 2.0 * r / ((Fbar + I) * V * P)
        a, b = splat.render_backward(cam, x, y, z, m32, gI, sigma, radius_sigmas)
        gm += a
        gx += b
        if image_rel_err is not None:
            e = float(image_rel_err)
            bL += float(np.sum(8.0 * e * np.abs(r) + 16.0 * e * e)) / (V * P)
            w = (2.0 / (V * P)) * 4.0 * e / (Fbar + I) + 3.0 * e * np.abs(gI)
            a2, b2 = splat.render_backward_bound(cam, x, y, z, m32, w, sigma, radius_sigmas)
            bm += a2
            bx += b2
    if image_rel_err is None:
        return L, gm, gx
    return L, gm, gx, bL, bm, bx


def grad_theta(m, gm):
    """dL/dtheta_k = m_k dL/dm_k for m = exp(theta)."""
    return np.asarray(m, dtype=np.float32).astype(np.float64) * np.asarray(gm, dtype=np.float64)


def adam_update(p, g, exp_avg, exp_avg_sq, step, lr):
    """One Adam update of parameters p with gradient g (float64 arrays);
    `step` is the step number t >= 1.  Returns (p_t, m_t, v_t)."""
    p = np.asarray(p, dtype=np.float64)
    g = np.asarray(g, dtype=np.float64)
    m_t = BETA1 * np.asarray(exp_avg, dtype=np.float64) + (1.0 - BETA1) * g
    v_t = BETA2 * np.asarray(exp_avg_sq, dtype=np.float64) + (1.0 - BETA2) * g * g
    mhat = m_t / (1.0 - BETA1 ** step)
    vhat = v_t / (1.0 - BETA2 ** step)
    return p - lr * mhat / (np.sqrt(vhat) + EPS), m_t, v_t


def project(theta, xyz, lo, side, node_mass):
    """Clamp positions to the node cube and shift theta so that the masses sum to the node mass."""
    xyz = np.asarray(xyz, dtype=np.float64).copy()
    for ax in range(3):
        xyz[:, ax] = np.minimum(np.maximum(xyz[:, ax], lo[ax]), lo[ax] + side)
    theta = np.asarray(theta, dtype=np.float64)
    mx = theta.max()
    lse = mx + math.log(math.fsum(np.exp(theta - mx).tolist()))
    return theta - (lse - math.log(node_mass)), xyz
