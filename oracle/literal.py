"""FP64 reference of the paper-literal per-anchor scheme.  Test infrastructure only.

This is Algorithm 1 exactly as printed (Sec. 2.3 to 2.5). It keeps none of the readings that
scheme.py takes for the local linear regression:

* One regression per particle m and level k (the inner parallel loop of Algorithm 1). It is set in
  X_k-space about the particle itself (eq. Dj): D^m_j = X^j_k - X^m_k.
* The weights are the normalised Gaussian kernel of eq. Dj. The bandwidth is
  eps_k^2 = h^2 E|X^j_k - X^m_k|^2 = h^2 2 s^2 t_k d, the expected squared distance between two
  independent particles of the cloud. At k = 0 every D^m_j is zero, and the weights are uniform
  (they are for h = 0 too).
* The ridge functional J_lambda of the remark after the matrix-free steps penalises the
  intercept as well, as printed, with lambda_k = ridge_rel s^2 t_{k+1} > 0.
* The conditional expectation is the plain particle mean of eq. discreteYkm,
  (1/M) sum_j Y^j_{k+1}. The fitted intercept is discarded.
* Z^m_k = sigma^T alpha_x = s alpha_x. Y^m_k comes from the fixed-count Newton iteration of eq. NRiter
  on y - mean - dt f(t_k, X^m_k, y, Z^m_k), started at the mean.
* u(0, x0) = mean_m Y^m_0 (last step of Algorithm 1). At k = 0 the design is zero, so alpha_x = 0:
  the scheme gives no gradient.

The particles and increments are those of scheme.py: same counters, so the same paths.
"""
import numpy as np

from . import scheme as S


def anchor_weights(pb, D, k):
    """Normalised Gaussian kernel weights of eq. Dj about one anchor (D: [M, d], rows X^j_k - X^m_k).

    eps_k^2 = h^2 2 s^2 t_k d.  The smallest squared distance is subtracted inside the exponential,
    which leaves the normalised weights unchanged (weight-ratio identity of the kernel remark).
    """
    n2 = np.einsum("ij,ij->i", D, D)
    if pb.eps_h == 0.0 or k == 0:
        e = np.ones(D.shape[0])
    else:
        t_k = k * pb.T / pb.N
        eps2 = pb.eps_h ** 2 * 2.0 * pb.s ** 2 * t_k * pb.d
        e = np.exp(-(n2 - n2.min()) / eps2)
    return e / e.sum()


def ridge_lambda(pb, k):
    return pb.ridge_rel * pb.s ** 2 * (k + 1) * pb.T / pb.N


def anchor_fit(pb, Xk, Y_next, m, k, form=None):
    """alpha = (alpha, alpha_x) [d + 1] minimising J_lambda about anchor m (eq. normal-eq with the ridge).

    Design rows [1, D_j] (eq. AY), weights of eq. Dj.  form "primal": the (d+1) x (d+1) normal
    equations (D^T W D + lambda I) alpha = D^T W Y; "dual": the same minimiser through the M x M
    system, alpha = B^T (B B^T + lambda I)^{-1} W^{1/2} Y with B = W^{1/2} D (push-through identity).
    Default: the smaller of the two.  Returns (alpha, w).
    """
    M, d = Xk.shape
    D = Xk - Xk[m][None, :]
    w = anchor_weights(pb, D, k)
    lam = ridge_lambda(pb, k)
    if not lam > 0.0:
        raise ValueError("the literal scheme needs a positive ridge")
    A = np.hstack([np.ones((M, 1)), D])
    if form is None:
        form = "primal" if M > d + 1 else "dual"
    if form == "primal":
        H = A.T @ (w[:, None] * A) + lam * np.eye(d + 1)
        alpha = np.linalg.solve(H, A.T @ (w * Y_next))
    else:
        sw = np.sqrt(w)
        B = sw[:, None] * A
        alpha = B.T @ np.linalg.solve(B @ B.T + lam * np.eye(M), sw * Y_next)
    return alpha, w


def solve_point(pb, x0, p, k_stop=0, form=None, tape=False):
    """Algorithm 1 as printed for one evaluation point x0 [d] (global point index point_base + p).

    Runs the backward levels N-1 .. k_stop.  Returns dict(u = mean_m Y^m_{k_stop}, Y = Y_{k_stop} [M],
    status) and, with tape=True, zz[k] = |Z^m_k|^2 [M] and zs[k] = sum_i Z^m_k,i [M] per level.
    """
    x0 = np.asarray(x0, dtype=np.float64)
    W = S.brownian_path(pb, p)
    Y, _, _ = S.g_eval(pb, S.positions(pb, x0, W[pb.N], pb.N))
    status = 0
    zz_t, zs_t = {}, {}
    for k in range(pb.N - 1, k_stop - 1, -1):
        Xk = S.positions(pb, x0, W[k], k)
        Ybar = float(Y.mean())
        Ynew = np.empty(pb.M)
        zz = np.empty(pb.M)
        zs = np.empty(pb.M)
        for m in range(pb.M):
            alpha, _ = anchor_fit(pb, Xk, Y, m, k, form)
            Z = pb.s * alpha[1:]
            y, _, st = S.newton(pb, k, np.array([Ybar]), Z)
            Ynew[m] = y[0]
            zz[m] = Z @ Z
            zs[m] = Z.sum()
            status |= st
        Y = Ynew
        zz_t[k], zs_t[k] = zz, zs
    u = float(Y.mean())
    if not np.all(np.isfinite(Y)):
        status |= S.ST_NONFINITE
    out = dict(u=u, Y=Y, status=status)
    if tape:
        out.update(zz=zz_t, zs=zs_t)
    return out


def solve(pb, x0s, k_stop=0, points=None, form=None):
    """u [P], Y_{k_stop} [P, M], status [P] for rows of x0s (optionally a subset of point indices)."""
    x0s = np.asarray(x0s, dtype=np.float64)
    idx = range(x0s.shape[0]) if points is None else points
    res = [solve_point(pb, x0s[p], p, k_stop, form) for p in idx]
    return (np.array([r["u"] for r in res]), np.stack([r["Y"] for r in res]),
            np.array([r["status"] for r in res], dtype=np.uint32))


# ---------------------------------------------------------------- x-dependent coefficients
# The same printed scheme with coefficients that depend on x (the paper's problem class of Sec. 2.1 allows
# mu(t, x) and sigma(t, x)): the affine diagonal family mu(x) = mu0 x + mu1, sigma(x) = diag(sigma0 x + sigma1),
# componentwise.  mu1 = sigma1 = 0 is the geometric family (Black-Scholes-type volatility); sigma0 = 0 with
# mu0 < 0 is an Ornstein-Uhlenbeck drift with additive noise.  Readings for this family:
# * Particles follow the Euler-Maruyama step of eq. Xk with the same normals as above:
#   X_{k+1} = X_k + (mu0 X_k + mu1) dt + (sigma0 X_k + sigma1) * sqrt(dt) xi_k (componentwise), X_0 = x0.
# * Bandwidth: no closed form of E|X^j_k - X^m_k|^2 is used; eps_k^2 = h^2 2 (1/M) sum_j |X^j_k - Xbar_k|^2,
#   the cloud's own mean squared pairwise distance (uniform weights at k = 0, where it is zero).
# * Ridge: lambda_k = ridge_rel (sigma0^2 + sigma1^2) t_{k+1}.
# * Z^m_k = sigma(X^m_k)^T alpha_x = (sigma0 X^m_k + sigma1) * alpha_x (componentwise).
def geometric_path(pb, x0, p, mu0, sigma0, mu1=0.0, sigma1=0.0):
    """X[k, j, :] for k = 0..N under the affine diagonal family (Euler-Maruyama, eq. Xk)."""
    from . import philox
    dt = pb.T / pb.N
    X = np.empty((pb.N + 1, pb.M, pb.d))
    X[0] = np.asarray(x0, dtype=np.float64)[None, :]
    q = S.stream_of(pb, p)
    for k in range(pb.N):
        xi = philox.normals(pb.seed, pb.instance, q, k, pb.M, pb.d)
        X[k + 1] = X[k] + (mu0 * X[k] + mu1) * dt + (sigma0 * X[k] + sigma1) * (np.sqrt(dt) * xi)
    return X


def cloud_bandwidth(pb, Xk, k):
    """eps_k^2 = h^2 2 (1/M) sum_j |X^j_k - Xbar|^2; 0 (uniform weights) at k = 0 or h = 0."""
    if pb.eps_h == 0.0 or k == 0:
        return 0.0
    C = Xk - Xk.mean(axis=0)[None, :]
    return pb.eps_h ** 2 * 2.0 * float(np.einsum("ij,ij->", C, C)) / Xk.shape[0]


def anchor_fit_eps(Xk, Y_next, m, eps2, lam, form=None):
    """Minimiser of J_lambda about anchor m (intercept penalised, as in anchor_fit) with bandwidth eps2
    (0: uniform weights): the (d+1) normal equations ("primal") or the same minimiser through the M x M
    system ("dual", push-through identity, as in anchor_fit).  Default: the smaller.  Returns (alpha, w)."""
    M, d = Xk.shape
    D = Xk - Xk[m][None, :]
    n2 = np.einsum("ij,ij->i", D, D)
    e = np.ones(M) if eps2 == 0.0 else np.exp(-(n2 - n2.min()) / eps2)
    w = e / e.sum()
    A = np.hstack([np.ones((M, 1)), D])
    if form is None:
        form = "primal" if M > d + 1 else "dual"
    if form == "primal":
        H = A.T @ (w[:, None] * A) + lam * np.eye(d + 1)
        return np.linalg.solve(H, A.T @ (w * Y_next)), w
    sw = np.sqrt(w)
    B = sw[:, None] * A
    return B.T @ np.linalg.solve(B @ B.T + lam * np.eye(M), sw * Y_next), w


def solve_point_geometric(pb, x0, p, mu0, sigma0, k_stop=0, tape=False, mu1=0.0, sigma1=0.0):
    """Algorithm 1 as printed under the affine diagonal family (geometric for mu1 = sigma1 = 0), levels
    N-1 .. k_stop (pb.s and pb.mu unused).  Returns dict(u = mean_m Y^m_{k_stop}, Y, status) and, with
    tape, zz[k], zs[k] per particle."""
    X = geometric_path(pb, x0, p, mu0, sigma0, mu1, sigma1)
    Y, _, _ = S.g_eval(pb, X[pb.N])
    dt = pb.T / pb.N
    status = 0
    zz_t, zs_t = {}, {}
    for k in range(pb.N - 1, k_stop - 1, -1):
        Xk = X[k]
        Ybar = float(Y.mean())
        eps2 = cloud_bandwidth(pb, Xk, k)
        lam = pb.ridge_rel * (sigma0 ** 2 + sigma1 ** 2) * (k + 1) * dt
        Ynew, zz, zs = np.empty(pb.M), np.empty(pb.M), np.empty(pb.M)
        for m in range(pb.M):
            alpha, _ = anchor_fit_eps(Xk, Y, m, eps2, lam)
            Z = (sigma0 * Xk[m] + sigma1) * alpha[1:]
            y, _, st = S.newton(pb, k, np.array([Ybar]), Z)
            Ynew[m], zz[m], zs[m] = y[0], Z @ Z, Z.sum()
            status |= st
        Y = Ynew
        zz_t[k], zs_t[k] = zz, zs
    out = dict(u=float(Y.mean()), Y=Y, status=status | (0 if np.all(np.isfinite(Y)) else S.ST_NONFINITE))
    if tape:
        out.update(zz=zz_t, zs=zs_t)
    return out
