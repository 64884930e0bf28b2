"""Reference solvers on top of the oracle's operator (numpy, FP64).

TEST INFRASTRUCTURE ONLY (see the package docstring).

All solvers take the operator as two callables ``J(x) -> y`` and
``JT(y) -> x`` so they run unchanged on a dense matrix or on the matrix-free
oracle.  Notation follows Sec. II-D of the paper: data noise covariance
Gamma_n = sigma^2 I, prior covariance Gamma_pr = I, regularisation weight
alpha; the Gaussian-prior estimate solves
    (J^T J / sigma^2 + alpha I) x = J^T d / sigma^2     (eq. leastSquare_misfit)
"""
from __future__ import annotations

import math

import numpy as np


def cgls(J, JT, d, sigma, alpha, n_iter, x0=None, tol=0.0):
    """Conjugate gradients on the damped normal equations, CGLS form
    (Hestenes-Stiefel).  With A = J/sigma and b = d/sigma it minimises
    |A x - b|^2 + alpha |x|^2.  Returns (x, history of |J x - d|^2/sigma^2)."""
    b = np.asarray(d, dtype=np.float64) / sigma
    x = np.zeros_like(JT(b)) if x0 is None else np.array(x0, dtype=np.float64)
    r = b - J(x) / sigma                       # data-space residual
    s = JT(r) / sigma - alpha * x              # normal-equation residual
    p = s.copy()
    gamma = float(s @ s)
    gamma0 = gamma
    hist = [float(r @ r)]
    for _ in range(n_iter):
        q = J(p) / sigma
        delta = float(q @ q) + alpha * float(p @ p)
        if delta == 0.0:
            break
        a = gamma / delta
        x += a * p
        r -= a * q
        s = JT(r) / sigma - alpha * x
        gamma_new = float(s @ s)
        hist.append(float(r @ r))
        if tol > 0 and math.sqrt(gamma_new / gamma0) < tol:
            gamma = gamma_new
            break
        p = s + (gamma_new / gamma) * p
        gamma = gamma_new
    return x, hist


def pcgls(J, JT, d, sigma, alpha, minv, n_iter, x0=None):
    """Preconditioned conjugate gradients on the same damped normal
    equations, preconditioner M^-1 = diag(minv): the textbook PCG recurrences
    (residual s, preconditioned residual z = M^-1 s, gamma = s.z) with the
    residual kept in data space as in cgls.  minv = 1 gives cgls.
    Returns (x, history of |J x - d|^2/sigma^2)."""
    b = np.asarray(d, dtype=np.float64) / sigma
    minv = np.asarray(minv, dtype=np.float64)
    x = np.zeros_like(JT(b)) if x0 is None else np.array(x0, dtype=np.float64)
    r = b - J(x) / sigma
    s = JT(r) / sigma - alpha * x
    z = minv * s
    p = z.copy()
    gamma = float(s @ z)
    hist = [float(r @ r)]
    for _ in range(n_iter):
        q = J(p) / sigma
        delta = float(q @ q) + alpha * float(p @ p)
        if delta == 0.0:
            break
        a = gamma / delta
        x += a * p
        r -= a * q
        s = JT(r) / sigma - alpha * x
        z = minv * s
        gamma_new = float(s @ z)
        hist.append(float(r @ r))
        p = z + (gamma_new / gamma) * p
        gamma = gamma_new
    return x, hist


def orth(Y, rel_tol):
    """Orthonormal basis of the range of Y's columns: left singular vectors
    whose squared singular value exceeds rel_tol times the largest."""
    U, s, _ = np.linalg.svd(Y, full_matrices=False)
    keep = s ** 2 > rel_tol * s[0] ** 2 if s.size and s[0] > 0 else np.zeros(0, bool)
    return U[:, keep]


def randomized_eigh(H, omega, q, k, rel_tol=1e-24):
    """k leading eigenpairs of a symmetric positive semidefinite operator by a
    randomized range finder with q subspace iterations and Rayleigh-Ritz
    (Halko, Martinsson & Tropp 2011): Q = orth(H omega); q times
    Q = orth(H Q); T = Q^T H Q = U diag(theta) U^T; Ritz pairs (theta, Q U).
    H maps an [N][c] block to [N][c].  Returns (eigenvalues [k] descending,
    zero-padded beyond the sampled rank; vectors [N][k]; rank)."""
    Q = orth(H(omega), rel_tol)
    for _ in range(q):
        Q = orth(H(Q), rel_tol)
    r = Q.shape[1]
    T = Q.T @ H(Q)
    T = 0.5 * (T + T.T)
    w, U = np.linalg.eigh(T)
    order = np.argsort(w)[::-1]
    w, U = w[order], U[:, order]
    kk = min(k, r)
    vals = np.zeros(k)
    vecs = np.zeros((Q.shape[0], k))
    vals[:kk] = w[:kk]
    vecs[:, :kk] = Q @ U[:, :kk]
    return vals, vecs, r


def lowrank_posterior_diag(vals, vecs, alpha):
    """Diagonals of the low-rank posterior covariance and resolution
    (eq. posterior_app / resolution_app, Gamma_pr = I):
    var = (1 - sum_i d_i v_i^2) / alpha, res = sum_i d_i v_i^2,
    d_i = lambda_i / (lambda_i + alpha)."""
    d = vals / (vals + alpha)
    s = (vecs ** 2) @ d
    return (1.0 - s) / alpha, s


def lsqr(J, JT, b, damp, n_iter, n_cols):
    """LSQR of Paige and Saunders (1982) for min |A x - b|^2 + damp^2 |x|^2,
    written from the published bidiagonalisation recurrences; x0 = 0."""
    b = np.asarray(b, dtype=np.float64)
    x = np.zeros(n_cols)
    beta = float(np.linalg.norm(b))
    u = b / beta if beta > 0 else b.copy()
    v = JT(u)
    alpha = float(np.linalg.norm(v))
    v = v / alpha if alpha > 0 else v
    w = v.copy()
    phibar = beta
    rhobar = alpha
    for _ in range(n_iter):
        # continue the bidiagonalisation
        u = J(v) - alpha * u
        beta = float(np.linalg.norm(u))
        if beta > 0:
            u /= beta
        v = JT(u) - beta * v
        alpha = float(np.linalg.norm(v))
        if alpha > 0:
            v /= alpha
        # eliminate the damping term (plane rotation on [rhobar; damp])
        rhobar1 = math.hypot(rhobar, damp)
        c1 = rhobar / rhobar1
        phibar = c1 * phibar
        # eliminate the subdiagonal beta
        rho = math.hypot(rhobar1, beta)
        c = rhobar1 / rho
        s = beta / rho
        theta = s * alpha
        rhobar = -c * alpha
        phi = c * phibar
        phibar = s * phibar
        x += (phi / rho) * w
        w = v - (theta / rho) * w
    return x


def psf(J, JT, n, voxel, sigma):
    """Hessian point-spread function J^T J e_i / sigma^2 (eq. resolution_2),
    e_i = 1 m/s at voxel i."""
    e = np.zeros(n)
    e[voxel] = 1.0
    return JT(J(e)) / sigma ** 2


def tv(x, dims, spacing, beta):
    """Smoothed isotropic total variation sum_j sqrt(|grad x|_j^2 + beta^2)
    with forward differences (scaled by 1/h) and a zero difference at the
    upper boundary of each axis; returns (value, gradient)."""
    nx, ny, nz = dims
    u = np.asarray(x, dtype=np.float64).reshape(nz, ny, nx)
    g = []
    for ax, h in ((2, spacing[0]), (1, spacing[1]), (0, spacing[2])):
        d = np.zeros_like(u)
        sl_hi = [slice(None)] * 3
        sl_lo = [slice(None)] * 3
        sl_hi[ax] = slice(1, None)
        sl_lo[ax] = slice(0, -1)
        d[tuple(sl_lo)] = (u[tuple(sl_hi)] - u[tuple(sl_lo)]) / h
        g.append((d, ax, h))
    mag = np.sqrt(sum(d * d for d, _, _ in g) + beta * beta)
    val = float(mag.sum())
    grad = np.zeros_like(u)
    for d, ax, h in g:
        t = d / mag / h
        sl_hi = [slice(None)] * 3
        sl_lo = [slice(None)] * 3
        sl_hi[ax] = slice(1, None)
        sl_lo[ax] = slice(0, -1)
        grad[tuple(sl_lo)] -= t[tuple(sl_lo)]
        grad[tuple(sl_hi)] += t[tuple(sl_lo)]
    return val, grad.ravel()


def tv_objective(J_bands, d_bands, sigma, alpha_tv, beta, dims, spacing, x):
    """chi(x) = 1/2 sum_b |J_b x - d_b|^2 / sigma^2 + alpha_tv TV_beta(x)
    (eq. leastSquare_misfit1 with a TV regulariser); returns (chi, grad)."""
    val = 0.0
    grad = np.zeros(x.size)
    for (Jb, JTb), db in zip(J_bands, d_bands):
        r = Jb(x) - db
        val += 0.5 * float(r @ r) / sigma ** 2
        grad += JTb(r) / sigma ** 2
    tval, tgrad = tv(x, dims, spacing, beta)
    return val + alpha_tv * tval, grad + alpha_tv * tgrad
