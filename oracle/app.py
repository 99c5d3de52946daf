"""Preconditioned APP primal-dual solvers (Algorithms 1, 1' and 2), their
step sizes (Eq. 16 and the conditions stated with Algorithms 1 and 2), and
the monitors (Eq. 1 cost, partial primal-dual gap, Eq. 34 RMSE).

Variables follow the paper: x is the image, mu the (preconditioned) dual
variable in sinogram space, mubar its extrapolation, D the ramp-type filter,
W = diag(w) the statistical weights, beta the TV weight, tau/sigma the primal
and dual step sizes.

Readings where the paper is silent:

* Step sizes.  tau is chosen first; D(tau) is built; the operator norms are
  largest eigenvalues --
  ||D^1/2 A A^T D^T/2|| = lambda_max(A^T D A) and
  ||D^1/2 W^-1 D^T/2|| = lambda_max(W^-1/2 D W^-1/2) -- and sigma takes a
  safety factor rho (0.95) of the strict bounds:
    low-dose: sigma = rho * min(2/lambda_h, 1/(tau lambda_A))
    few-view: sigma tau < 1/lambda_A(tau) with D(tau) = D(1)/tau, so
              sigma = rho / lambda_A(1), computed once with tau = 1.
* The two norms are largest eigenvalues, which the oracle takes by their
  definition (ARPACK ``eigsh`` on the matrix-free symmetric operator, or a
  dense ``eigvalsh`` for tiny sizes), independent of how the GPU finds them.
* Default tau (the paper gives none): low-dose tau = c * pi kappa / (2m) with
  c = 0.3 (c = 1 puts H(omega) of Eq. 24 at half its 1/kappa asymptote at the
  Nyquist frequency; sweeps of c on the 64^2 and 512^2 workloads put the
  fastest decrease of the Eq. 1 cost over 10-40 iterations at c ~ 0.3);
  few-view tau = mean|sigma A^T D(1) b|, so the TV weight of the first prox
  matches the scale of the first (FBP-like) iterate.
* TV prox: projected-gradient dual iteration (see ``tv``), n_tv = 10 inner
  steps of size tau_c = 1/8, dual field warm-started across outer iterations.
"""
from dataclasses import dataclass, field

import numpy as np
from scipy.sparse.linalg import LinearOperator, eigsh

from .projector import forward_project, back_project
from .filters import ramp_taps, smoothed_ramp_taps, apply_filter
from .tv import tv_prox, tv_norm

TAU_MULT_LOWDOSE = 0.3
TAU_MULT_FEWVIEW = 1.0


def lambda_max(apply_op, size, dense_below=1500):
    """Largest eigenvalue of a symmetric positive semi-definite linear operator."""
    if size <= dense_below:
        cols = np.stack([apply_op(e) for e in np.eye(size)], axis=1)
        return float(np.linalg.eigvalsh(0.5 * (cols + cols.T))[-1])
    v0 = np.cos(0.7 * np.arange(size)) + 1.5
    op = LinearOperator((size, size), matvec=apply_op, dtype=np.float64)
    return float(eigsh(op, k=1, which="LA", tol=1e-12, v0=v0)[0][0])


def lambda_a(n, m, nb, h, theta=None):
    """lambda_max(A^T D A) = ||D^1/2 A A^T D^T/2|| for the Toeplitz filter with taps h."""
    op = lambda v: back_project(apply_filter(forward_project(v.reshape(n, n), m, nb, theta=theta), h), n,
                                theta=theta).ravel()
    return lambda_max(op, n * n)


def lambda_h(winv, h):
    """lambda_max(W^-1/2 D W^-1/2) = ||D^1/2 W^-1 D^T/2||."""
    m, nb = winv.shape
    sq = np.sqrt(winv)
    op = lambda u: (sq * apply_filter(sq * u.reshape(m, nb), h)).ravel()
    return lambda_max(op, m * nb)


def default_tau_lowdose(kappa, m):
    return TAU_MULT_LOWDOSE * np.pi * kappa / (2.0 * m)


@dataclass
class Steps:
    tau: float
    sigma: float
    kappa: float = 0.0
    lambda_a: float = 0.0
    lambda_h: float = 0.0


def steps_lowdose(w, n, tau=None, rho=0.95, theta=None):
    w = np.asarray(w, dtype=np.float64)
    m, nb = w.shape
    winv = 1.0 / w
    kappa = float(winv.mean())
    if tau is None:
        tau = default_tau_lowdose(kappa, m)
    h = smoothed_ramp_taps(nb, m, tau, kappa)
    la = lambda_a(n, m, nb, h, theta)
    lh = lambda_h(winv, h)
    sigma = rho * min(2.0 / lh, 1.0 / (tau * la))
    return Steps(tau=tau, sigma=sigma, kappa=kappa, lambda_a=la, lambda_h=lh)


def steps_fewview(b, n, tau=None, rho=0.95):
    b = np.asarray(b, dtype=np.float64)
    m, nb = b.shape
    h1 = ramp_taps(nb, m, 1.0)
    la1 = lambda_a(n, m, nb, h1)
    sigma = rho / la1
    if tau is None:
        tau = TAU_MULT_FEWVIEW * float(np.abs(sigma * back_project(apply_filter(b, h1), n)).mean())
    return Steps(tau=tau, sigma=sigma, kappa=0.0, lambda_a=la1 / tau, lambda_h=0.0)


@dataclass
class Result:
    x: np.ndarray
    mu: np.ndarray
    mu_prev: np.ndarray
    p1: np.ndarray
    p2: np.ndarray
    history: list = field(default_factory=list)


def app_solve(b, n, iters, tau, sigma, h, beta=1.0, winv=None, n_tv=10, tau_c=0.125,
              monitor=None, extrapolation="simplified", theta=None):
    """The APP iteration of Eqs. 18-20 (winv given) or Eqs. 29-31 (winv None).

    k = 0:  mubar = -sigma D b
    k >= 1: mubar = 2 mu^k - mu^{k-1} - sigma D W^-1 (mu^k - mu^{k-1})   (low-dose)
            mubar = 2 mu^k - mu^{k-1}                                 (few-view)
    x^{k+1}  = prox_{tau g}(x^k - tau A^T mubar), TV weight tau*beta
    mu^{k+1} = mu^k + sigma D (A x^{k+1} - b - W^-1 mu^k)   (W^-1 term only for low-dose)

    ``extrapolation="direct"`` uses the unsimplified left-hand form of Eq. 18,
    mubar = mu^k + sigma D (A x^k - b - W^-1 mu^k), for checking the algebra.
    ``theta`` (optional) gives the view angles of A.
    """
    b = np.asarray(b, dtype=np.float64)
    m, nb = b.shape
    D = lambda s: apply_filter(s, h)
    x = np.zeros((n, n))
    mu = np.zeros((m, nb))
    mu_prev = np.zeros((m, nb))
    p1 = np.zeros((n, n))
    p2 = np.zeros((n, n))
    lam = tau * beta
    hist = []
    for k in range(iters):
        if extrapolation == "direct":
            r = forward_project(x, m, nb, theta=theta) - b
            if winv is not None:
                r = r - winv * mu
            mubar = mu + sigma * D(r)
        elif k == 0:
            mubar = -sigma * D(b)
        elif winv is not None:
            mubar = 2.0 * mu - mu_prev - sigma * D(winv * (mu - mu_prev))
        else:
            mubar = 2.0 * mu - mu_prev
        z = x - tau * back_project(mubar, n, theta=theta)
        x, p1, p2 = tv_prox(z, lam, p1, p2, n_tv, tau_c)
        r = forward_project(x, m, nb, theta=theta) - b
        if winv is not None:
            r = r - winv * mu
        mu_prev, mu = mu, mu + sigma * D(r)
        if monitor is not None:
            hist.append(monitor(x, mu))
    return Result(x=x, mu=mu, mu_prev=mu_prev, p1=p1, p2=p2, history=hist)


def lowdose_solve(b, w, beta, n, iters, tau=None, sigma=None, n_tv=10, tau_c=0.125, rho=0.95,
                  record_cost=False, theta=None):
    """Algorithm 1 (beta > 0) / Algorithm 1' (beta = 0).  Returns (Result, Steps).
    ``theta`` (optional) gives the view angles; D keeps Eq. 24 with the view count m."""
    w = np.asarray(w, dtype=np.float64)
    m, nb = w.shape
    winv = 1.0 / w
    kappa = float(winv.mean())
    if sigma is None:
        st = steps_lowdose(w, n, tau, rho, theta)
    else:
        st = Steps(tau=default_tau_lowdose(kappa, m) if tau is None else tau, sigma=sigma, kappa=kappa)
    h = smoothed_ramp_taps(nb, m, st.tau, kappa)
    mon = (lambda x, mu: cost_lowdose(x, b, w, beta, theta)) if record_cost else None
    res = app_solve(b, n, iters, st.tau, st.sigma, h, beta=beta, winv=winv, n_tv=n_tv, tau_c=tau_c,
                    monitor=mon, theta=theta)
    return res, st


def fewview_solve(b, n, iters, tau=None, sigma=None, n_tv=10, tau_c=0.125, rho=0.95, record_cost=False):
    """Algorithm 2.  Returns (Result, Steps)."""
    b = np.asarray(b, dtype=np.float64)
    m, nb = b.shape
    if sigma is None or tau is None:
        st = steps_fewview(b, n, tau, rho)
        if sigma is not None:
            st.sigma = sigma
    else:
        st = Steps(tau=tau, sigma=sigma)
    h = ramp_taps(nb, m, st.tau)
    mon = (lambda x, mu: tv_norm(x)) if record_cost else None
    res = app_solve(b, n, iters, st.tau, st.sigma, h, beta=1.0, winv=None, n_tv=n_tv, tau_c=tau_c,
                    monitor=mon)
    return res, st


def identity_taps(nb):
    """Taps of D = I (1 at offset 0): Algorithm 1 without its preconditioner."""
    h = np.zeros(2 * nb - 1)
    h[nb - 1] = 1.0
    return h


def steps_lowdose_identity(w, n, tau=None, rho=0.95):
    """Eq. 16 with D = I: lambda_A = lambda_max(A^T A), lambda_h = lambda_max(W^-1)
    = max 1/w (W^-1 is diagonal); default tau = lambda_h / (2 lambda_A), where
    the two bounds on sigma coincide."""
    w = np.asarray(w, dtype=np.float64)
    m, nb = w.shape
    winv = 1.0 / w
    la = lambda_a(n, m, nb, identity_taps(nb))
    lh = float(winv.max())
    if tau is None:
        tau = lh / (2.0 * la)
    sigma = rho * min(2.0 / lh, 1.0 / (tau * la))
    return Steps(tau=tau, sigma=sigma, kappa=float(winv.mean()), lambda_a=la, lambda_h=lh)


def lowdose_identity_solve(b, w, beta, n, iters, tau=None, sigma=None, n_tv=10, tau_c=0.125, rho=0.95,
                           record_cost=False):
    """Algorithm 1 with D = I (the ablation without the preconditioner).  Returns (Result, Steps)."""
    w = np.asarray(w, dtype=np.float64)
    m, nb = w.shape
    st = steps_lowdose_identity(w, n, tau, rho)
    if sigma is not None:
        st.sigma = sigma
    mon = (lambda x, mu: cost_lowdose(x, b, w, beta)) if record_cost else None
    res = app_solve(b, n, iters, st.tau, st.sigma, identity_taps(nb), beta=beta, winv=1.0 / w, n_tv=n_tv,
                    tau_c=tau_c, monitor=mon)
    return res, st


def cost_lowdose(x, b, w, beta, theta=None):
    """f(x) of Eq. 1: beta psi(x) + 1/2 sum_i w_i ((A x)_i - b_i)^2."""
    m, nb = np.shape(b)
    r = forward_project(x, m, nb, theta=theta) - np.asarray(b, dtype=np.float64)
    return beta * tv_norm(x) + 0.5 * float((np.asarray(w, dtype=np.float64) * r * r).sum())


def partial_gap(x, mu, b, w):
    """f(x) - L(x, mu) = 1/2 || W^1/2 (A x - b) - W^-1/2 mu ||^2  (>= 0, zero at the saddle point)."""
    m, nb = np.shape(b)
    w = np.asarray(w, dtype=np.float64)
    r = forward_project(x, m, nb) - np.asarray(b, dtype=np.float64)
    d = np.sqrt(w) * r - mu / np.sqrt(w)
    return 0.5 * float((d * d).sum())


def data_residual(x, b):
    """||A x - b|| / ||b|| (few-view feasibility)."""
    m, nb = np.shape(b)
    b = np.asarray(b, dtype=np.float64)
    return float(np.linalg.norm(forward_project(x, m, nb) - b) / np.linalg.norm(b))


def rmse(x, x_true):
    """Eq. 34."""
    d = np.asarray(x, dtype=np.float64) - np.asarray(x_true, dtype=np.float64)
    return float(np.sqrt((d * d).mean()))


# ---------------------------------------------------------------------------
# The error-tolerant few-view problem the conclusions name (Sec. 5):
#     min psi(x)  s.t.  ||A x - b|| <= eps,  x >= 0.
#
# Reading (the paper states only the problem): it is posed like Eq. 6 - Eq. 7
# for the low-dose problem -- a variable y standing for the projection data,
# the preconditioned equality constraint D^1/2 (A x - y) = 0, and the data term
# on y, here the indicator of the ball B(b, eps) = {y : ||y - b|| <= eps}.  The
# primal variable is the pair (x, y) with g(x, y) = psi(x) + i(x) + i_B(y) and
# h(mu) = 0 (no term of mu alone remains), so APP's primal prox splits into the
# TV prox of Eq. 17 (lambda = tau) and the Euclidean projection onto the ball,
# and its dual gradient step is the plain ascent step.  After the variable
# change mu <- D^T/2 mu, as in Eqs. 18-20 and 29-31:
#     mubar^{k+1} = mu^k + sigma D (A x^k - y^k)      (= 2 mu^k - mu^{k-1} for k >= 1;
#                                                      = -sigma D b at k = 0, with y^0 = b)
#     x^{k+1}    = prox_{tau g}(x^k - tau A^T mubar^{k+1})
#     y^{k+1}    = P_B(y^k + tau mubar^{k+1})
#     mu^{k+1}   = mu^k + sigma D (A x^{k+1} - y^{k+1})
# Convergence (Eq. 16 with K = [A, -I]): sigma tau ||D^1/2 (A A^T + I) D^T/2|| < 1.
# D is the ramp of Eq. 32; with D(tau) = D(1)/tau the bound reads
# sigma lambda_max(K^T D(1) K) < 1 whatever tau is.  eps = 0 keeps y = b and
# gives Algorithm 2 exactly.
# ---------------------------------------------------------------------------

def ball_projection(v, b, eps):
    """Euclidean projection of v onto {y : ||y - b|| <= eps}."""
    d = v - b
    r = float(np.sqrt((d * d).sum()))
    return v.copy() if r <= eps else b + d * (eps / r)


def lambda_a_split(n, m, nb, h, theta=None):
    """lambda_max(K^T D K) for K = [A, -I] acting on (x, y): the norm of the
    preconditioned constraint operator D^1/2 [A, -I] squared."""
    J = n * n

    def op(v):
        x, y = v[:J].reshape(n, n), v[J:].reshape(m, nb)
        s = apply_filter(forward_project(x, m, nb, theta=theta) - y, h)
        return np.concatenate([back_project(s, n, theta=theta).ravel(), -s.ravel()])

    return lambda_max(op, J + m * nb)


def steps_fewview_eps(b, n, tau=None, rho=0.95):
    """sigma = rho / lambda_max(K^T D(1) K); default tau = mean |sigma A^T D(1) b| (as Algorithm 2)."""
    b = np.asarray(b, dtype=np.float64)
    m, nb = b.shape
    h1 = ramp_taps(nb, m, 1.0)
    la1 = lambda_a_split(n, m, nb, h1)
    sigma = rho / la1
    if tau is None:
        tau = TAU_MULT_FEWVIEW * float(np.abs(sigma * back_project(apply_filter(b, h1), n)).mean())
    return Steps(tau=tau, sigma=sigma, kappa=0.0, lambda_a=la1 / tau, lambda_h=0.0)


@dataclass
class EpsResult:
    x: np.ndarray
    y: np.ndarray
    mu: np.ndarray
    mu_prev: np.ndarray
    p1: np.ndarray
    p2: np.ndarray
    history: list = field(default_factory=list)


def fewview_eps_solve(b, n, eps, iters, tau=None, sigma=None, n_tv=10, tau_c=0.125, rho=0.95, monitor=None):
    """The error-tolerant few-view iteration above from x = 0, y = b, mu = 0.
    Returns (EpsResult, Steps); monitor(x, y, mu) is recorded per iteration."""
    b = np.asarray(b, dtype=np.float64)
    m, nb = b.shape
    if sigma is None or tau is None:
        st = steps_fewview_eps(b, n, tau, rho)
        if sigma is not None:
            st.sigma = sigma
    else:
        st = Steps(tau=tau, sigma=sigma)
    tau, sigma = st.tau, st.sigma
    h = ramp_taps(nb, m, tau)
    D = lambda s: apply_filter(s, h)
    x = np.zeros((n, n))
    y = b.copy()
    mu = np.zeros((m, nb))
    mu_prev = np.zeros((m, nb))
    p1 = np.zeros((n, n))
    p2 = np.zeros((n, n))
    hist = []
    for k in range(iters):
        mubar = mu + sigma * D(forward_project(x, m, nb) - y) if k == 0 else 2.0 * mu - mu_prev
        x, p1, p2 = tv_prox(x - tau * back_project(mubar, n), tau, p1, p2, n_tv, tau_c)
        y = ball_projection(y + tau * mubar, b, eps)
        mu_prev, mu = mu, mu + sigma * D(forward_project(x, m, nb) - y)
        if monitor is not None:
            hist.append(monitor(x, y, mu))
    return EpsResult(x=x, y=y, mu=mu, mu_prev=mu_prev, p1=p1, p2=p2, history=hist), st
