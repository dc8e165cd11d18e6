"""Lanczos eigensolver for the lowest eigenpair (Methods, "Tensor
Networks", step (ii): the paper uses ARPACK's Arnoldi iteration; H_eff is
real symmetric here, so its Lanczos form is used).

One cycle of m steps, in this order:
    v_0 = x / |x|
    for j = 0 .. m-1:
        w = H v_j
        alpha_j = <v_j, w>
        w -= alpha_j v_j + beta_{j-1} v_{j-1}
        two passes of classical Gram-Schmidt of w against v_0 .. v_j
        beta_j = |w|;  stop early if beta_j <= breakdown * |alpha|-scale
        v_{j+1} = w / beta_j
    T = tridiag(alpha, beta);  (theta, s) = lowest eigenpair of T
    Ritz vector u = V s, normalised; its largest-magnitude component is
    made positive (first such index on ties).
Residual estimate |H u - theta u| = beta_{m-1} |s_{m-1}|.
Cycles restart from the Ritz vector until the residual is <= tol * |theta|
or `max_cycles` is reached.
"""

import numpy as np


def lanczos_cycle(apply, x, m, breakdown=1e-14):
    n = x.size
    m = max(1, min(m, n))
    V = np.zeros((m + 1, n))
    alpha = np.zeros(m)
    beta = np.zeros(m)
    nrm = np.linalg.norm(x)
    if nrm == 0.0:
        raise ValueError("zero start vector")
    V[0] = x / nrm
    k = m
    for j in range(m):
        w = apply(V[j])
        alpha[j] = V[j] @ w
        w = w - alpha[j] * V[j]
        if j > 0:
            w = w - beta[j - 1] * V[j - 1]
        for _ in range(2):
            w = w - V[: j + 1].T @ (V[: j + 1] @ w)
        beta[j] = np.linalg.norm(w)
        scale = max(abs(alpha[: j + 1]).max(), beta[: j].max(initial=0.0), 1.0)
        if beta[j] <= breakdown * scale:
            k = j + 1
            beta[j] = 0.0
            break
        V[j + 1] = w / beta[j]
    T = np.diag(alpha[:k]) + np.diag(beta[: k - 1], 1) + np.diag(beta[: k - 1], -1)
    evals, evecs = np.linalg.eigh(T)
    theta, s = evals[0], evecs[:, 0]
    u = V[:k].T @ s
    u /= np.linalg.norm(u)
    i = int(np.argmax(np.abs(u)))
    if u[i] < 0:
        u = -u
    resid = abs(beta[k - 1] * s[k - 1])
    return theta, u, resid, alpha[:k], beta[:k]


def lowest(apply, x, m=30, tol=0.0, max_cycles=1):
    theta, u, resid = None, x, None
    for _ in range(max_cycles):
        theta, u, resid, _, _ = lanczos_cycle(apply, u, m)
        if resid <= tol * max(abs(theta), 1e-300):
            break
    return theta, u, resid
