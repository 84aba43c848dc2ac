"""Residual model and maximum-inlier energy terms in FP64 (test infrastructure).

The flow end-point error r follows a log-logistic (Fisk) law (sec. III-A, the
VOLDOR model).  Reading: the EPE is the length of a 2-D residual whose
direction is uniform, so the inlier likelihood of the residual *vector* is the
planar density

    L1(r) = f_Fisk(r; a, b) / (2 pi r),   f_Fisk(r) = (b/a)(r/a)^(b-1) / (1 + (r/a)^b)^2,

i.e. L1(r) = b (r/a)^(b-2) / (2 pi a^2 (1 + (r/a)^b)^2); for b = 2 it is
1 / (pi a^2 (1 + r^2/a^2)^2).  The outlier likelihood is a constant planar
density L0 (uniform over a disc).

Maximum-inlier estimation (Eq. 4 applied to flows, sec. III-A): a term with
rigidness posterior q costs  -q log(L1 / (L0 + L1)) = q log1p(L0 / L1).
Depth-prior terms (Eqs. 3-4) use a Gaussian-uniform mixture on inverse depth.
"""
import numpy as np

LOG2 = np.log(2.0)


def fisk_pdf(r, alpha, beta):
    """1-D log-logistic density of the EPE magnitude."""
    z = np.asarray(r, dtype=np.float64) / alpha
    return (beta / alpha) * z ** (beta - 1) / (1.0 + z ** beta) ** 2


def planar_density(r, alpha, beta):
    """Inlier likelihood of a residual vector of length r (see module docstring)."""
    z = np.asarray(r, dtype=np.float64) / alpha
    with np.errstate(divide="ignore"):
        return beta * z ** (beta - 2.0) / (2.0 * np.pi * alpha * alpha * (1.0 + z ** beta) ** 2)


def flow_term(r2, alpha, beta, L0):
    """MIE cost log1p(L0 / L1(r)) of one valid flow term, r2 = r^2 (multiply by q)."""
    r = np.sqrt(np.asarray(r2, dtype=np.float64))
    L1 = planar_density(r, alpha, beta)
    with np.errstate(divide="ignore"):
        return np.log1p(L0 / L1)


def flow_weight(r2, alpha, beta, L0):
    """d/d(r^2) of flow_term: the IRLS weight of the Gauss-Newton pose step (times q).

    With x = r^2, y = (x/a^2)^(b/2) and g = L0/L1:
      -d log L1 / dx = (2-b)/(2x) + (b/a^2) (x/a^2)^(b/2-1) / (1+y),
      d/dx log1p(g) = g/(1+g) * (-d log L1/dx).
    For b < 2 the derivative diverges at r = 0; x is floored at (1e-3 a)^2 there."""
    x = np.asarray(r2, dtype=np.float64)
    if beta != 2.0:
        x = np.maximum(x, (1e-3 * alpha) ** 2)
    y = (x / alpha ** 2) ** (beta / 2.0)
    dlog = (beta / alpha ** 2) * (x / alpha ** 2) ** (beta / 2.0 - 1.0) / (1.0 + y)
    if beta != 2.0:
        dlog = dlog + (2.0 - beta) / (2.0 * x)
    g = L0 / planar_density(np.sqrt(x), alpha, beta)
    return g / (1.0 + g) * dlog


def prior_log_kappa(sigma_rel, uniform_rel):
    """log of kappa = U / N at zero residual (Eq. 3 reading): sigma(rho^) = c_s rho^,
    U(rho^) = 1/(c_u rho^), so U/N = sqrt(2 pi) c_s / c_u * exp(z^2/2)."""
    return np.log(np.sqrt(2.0 * np.pi) * sigma_rel / uniform_rel)


def prior_term(z, log_kappa):
    """MIE cost of one prior term (Eq. 4): -log N/(N+U) = softplus(log kappa + z^2/2)."""
    a = log_kappa + 0.5 * np.asarray(z, dtype=np.float64) ** 2
    return np.logaddexp(0.0, a)


def prior_posterior(z, log_kappa, pi_hat):
    """q(W^ = 1) = pi N / (pi N + (1 - pi) U) at the current depth (Eq. 3 mixture)."""
    pi_hat = np.asarray(pi_hat, dtype=np.float64)
    a = log_kappa + 0.5 * np.asarray(z, dtype=np.float64) ** 2      # log(U/N)
    with np.errstate(divide="ignore", over="ignore"):
        odds = np.where(pi_hat > 0, (1.0 - pi_hat) / np.where(pi_hat > 0, pi_hat, 1.0), np.inf)
        q = 1.0 / (1.0 + odds * np.exp(a))
    return np.where(pi_hat > 0, q, 0.0)


# --------------------------------------------------------------------------- #
# depth priors from an external source: empirical residual model (sec. III-A, the text after
# the prior energy: priors of known external sources such as stereo replace Eq. 3 by an
# empirical residual model, as VOLDOR does for the flow)
# --------------------------------------------------------------------------- #
def disparity_residual(rho_hat, inv_phi, fb):
    """Signed disparity residual (px) of a prior value rho^ against the transferred candidate
    1/phi_z: disparity = fb * inverse depth, fb = focal length times baseline."""
    return fb * (np.asarray(rho_hat, dtype=np.float64) - np.asarray(inv_phi, dtype=np.float64))


def disparity_log_ratio(r, alpha, beta, D):
    """log(p0 / p1) for a signed disparity residual r: inlier density p1(r) = f_Fisk(|r|) / 2
    (the magnitude log-logistic, the sign equally likely; maximal at 0 for beta <= 1, floored
    at |r| = 1e-3 alpha for beta < 1), outlier density p0 = 1 / D (uniform over a disparity
    range of width D)."""
    a = np.maximum(np.abs(np.asarray(r, dtype=np.float64)), 1e-3 * alpha if beta < 1 else 0.0)
    z = a / alpha
    log_p1 = np.log(beta / alpha) + (beta - 1.0) * np.log(np.where(z > 0, z, 1.0)) - 2.0 * np.log1p(z ** beta) \
        - np.log(2.0)
    if beta != 1.0:
        log_p1 = np.where(z > 0, log_p1, -np.inf if beta > 1 else np.inf)
    return -np.log(D) - log_p1


def disparity_prior_term(r, alpha, beta, D):
    """MIE cost -log(p1 / (p0 + p1)) = softplus(log(p0 / p1)) of one disparity prior term."""
    return np.logaddexp(0.0, disparity_log_ratio(r, alpha, beta, D))


def disparity_prior_posterior(r, alpha, beta, D, pi_hat):
    """q = pi p1 / (pi p1 + (1 - pi) p0) at the current depth."""
    pi_hat = np.asarray(pi_hat, dtype=np.float64)
    a = disparity_log_ratio(r, alpha, beta, D)
    with np.errstate(divide="ignore", over="ignore"):
        odds = np.where(pi_hat > 0, (1.0 - pi_hat) / np.where(pi_hat > 0, pi_hat, 1.0), np.inf)
        return 1.0 / (1.0 + odds * np.exp(a))
