"""FP64 oracle for the learned constitutive surrogate (TEST INFRASTRUCTURE ONLY).

The surrogate replaces the snow return map and stress in principal space
(the workload's learned-surrogate configuration: an MLP 12 -> 64 -> 64 -> 12 that maps
the trial elastic singular values, the plastic volume and the hardening state
to the projected singular values and the principal Kirchhoff stress).  This
module holds plain numpy FP64 definitions of:

  * the exact principal-space snow map the training pairs come from
    (singular values clamped into [1 - theta_c, 1 + theta_s], the removed
    volume moved to J_P, hardening h = exp(xi (1 - J_P)), fixed-corotated
    principal stress tau_k = 2 mu h (s_k - 1) s_k + lambda h (J - 1) J);
  * the 12 input features and 12 output targets;
  * the MLP forward pass (tanh hidden layers, linear output), the mean squared
    error, its gradient by backpropagation, and one Adam step (Kingma & Ba
    2015, bias-corrected moments).
Matrix products use numpy (a library primitive); nothing is blocked, fused or
reordered beyond the definitions.  Parameters, normalisation statistics and
random initialisations are inputs.
"""
from __future__ import annotations

import numpy as np

LAYERS = (12, 64, 64, 12)
N_IN, N_OUT = 12, 12


def lame(mat: dict):
    E, nu = mat["E"], mat["nu"]
    return E / (2 * (1 + nu)), E * nu / ((1 + nu) * (1 - 2 * nu))


def snow_principal(mat: dict, sig_hat: np.ndarray, Jp: np.ndarray):
    """Exact snow map in principal space.  sig_hat (N,3) trial singular values
    (any order), Jp (N,) plastic volume.  Returns (sig_new (N,3), Jp_new (N,),
    tau (N,3) principal Kirchhoff stress of the projected state)."""
    sig_hat = np.asarray(sig_hat, dtype=np.float64)
    Jp = np.asarray(Jp, dtype=np.float64)
    lo, hi = 1 - mat["theta_c"], 1 + mat["theta_s"]
    sig = np.clip(sig_hat, lo, hi)
    Jp_new = Jp * np.prod(sig_hat, axis=1) / np.prod(sig, axis=1)
    mu, la = lame(mat)
    h = np.exp(mat["xi"] * (1 - Jp_new))
    J = np.prod(sig, axis=1)
    tau = 2 * (mu * h)[:, None] * (sig - 1) * sig + ((la * h) * (J - 1) * J)[:, None]
    return sig, Jp_new, tau


def features(mat: dict, sig_hat: np.ndarray, Jp: np.ndarray, dt: float, dt_ref: float) -> np.ndarray:
    """Inputs: [s1..s3, ln s1..s3, J_P, ln J_P, h, dt/dt_ref, s1 s2 s3, 1] with
    s sorted descending and h = exp(xi (1 - J_P))."""
    s = -np.sort(-np.asarray(sig_hat, dtype=np.float64), axis=1)
    Jp = np.asarray(Jp, dtype=np.float64)
    N = s.shape[0]
    out = np.empty((N, N_IN))
    out[:, 0:3] = s
    out[:, 3:6] = np.log(s)
    out[:, 6] = Jp
    out[:, 7] = np.log(Jp)
    out[:, 8] = np.exp(mat["xi"] * (1 - Jp))
    out[:, 9] = dt / dt_ref
    out[:, 10] = np.prod(s, axis=1)
    out[:, 11] = 1.0
    return out


def targets(mat: dict, sig_hat: np.ndarray, Jp: np.ndarray) -> np.ndarray:
    """Outputs: [s'1..s'3, ln(s'/s)1..3, tau1..3 / E, J_P'/J_P, h', s'1 s'2 s'3]
    for the descending-sorted trial values."""
    s = -np.sort(-np.asarray(sig_hat, dtype=np.float64), axis=1)
    Jp = np.asarray(Jp, dtype=np.float64)
    sn, Jpn, tau = snow_principal(mat, s, Jp)
    N = s.shape[0]
    out = np.empty((N, N_OUT))
    out[:, 0:3] = sn
    out[:, 3:6] = np.log(sn / s)
    out[:, 6:9] = tau / mat["E"]
    out[:, 9] = Jpn / Jp
    out[:, 10] = np.exp(mat["xi"] * (1 - Jpn))
    out[:, 11] = np.prod(sn, axis=1)
    return out


# -------------------------------------------------------------------- MLP
def param_shapes():
    shapes = []
    for a, b in zip(LAYERS[:-1], LAYERS[1:]):
        shapes.append(("W", (b, a)))
        shapes.append(("b", (b,)))
    return shapes


def num_params() -> int:
    return sum(int(np.prod(s)) for _, s in param_shapes())


def unflatten(theta: np.ndarray):
    """Flat parameter vector -> [W1, b1, W2, b2, W3, b3] (W as (out, in))."""
    theta = np.asarray(theta, dtype=np.float64)
    out, k = [], 0
    for _, shp in param_shapes():
        n = int(np.prod(shp))
        out.append(theta[k:k + n].reshape(shp))
        k += n
    assert k == theta.size
    return out


def forward(theta: np.ndarray, X: np.ndarray):
    """Y = W3 tanh(W2 tanh(W1 x + b1) + b2) + b3 per row of X (N,12).
    Returns (Y, cache) with the pre-activations for the backward pass."""
    W1, b1, W2, b2, W3, b3 = unflatten(theta)
    X = np.asarray(X, dtype=np.float64)
    z1 = X @ W1.T + b1
    a1 = np.tanh(z1)
    z2 = a1 @ W2.T + b2
    a2 = np.tanh(z2)
    Y = a2 @ W3.T + b3
    return Y, (X, a1, a2)


def loss(theta: np.ndarray, X: np.ndarray, T: np.ndarray) -> float:
    """Mean over samples of 1/2 |Y - T|^2."""
    Y, _ = forward(theta, X)
    return 0.5 * float(np.sum((Y - T) ** 2)) / X.shape[0]


def grad(theta: np.ndarray, X: np.ndarray, T: np.ndarray) -> np.ndarray:
    """Gradient of `loss` with respect to the flat parameters (backpropagation)."""
    W1, b1, W2, b2, W3, b3 = unflatten(theta)
    Y, (X, a1, a2) = forward(theta, X)
    N = X.shape[0]
    dY = (Y - T) / N
    gW3 = dY.T @ a2
    gb3 = dY.sum(axis=0)
    d2 = (dY @ W3) * (1 - a2 ** 2)
    gW2 = d2.T @ a1
    gb2 = d2.sum(axis=0)
    d1 = (d2 @ W2) * (1 - a1 ** 2)
    gW1 = d1.T @ X
    gb1 = d1.sum(axis=0)
    return np.concatenate([g.ravel() for g in (gW1, gb1, gW2, gb2, gW3, gb3)])


def adam_step(theta, g, m, v, t, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (t counts from 1).  Returns (theta, m, v)."""
    m = beta1 * m + (1 - beta1) * g
    v = beta2 * v + (1 - beta2) * g * g
    mhat = m / (1 - beta1 ** t)
    vhat = v / (1 - beta2 ** t)
    return theta - lr * mhat / (np.sqrt(vhat) + eps), m, v


def normalize_stats(A: np.ndarray, floor: float = 1e-6):
    """Per-column mean and standard deviation (floored) for z-scoring."""
    mu = A.mean(axis=0)
    sd = np.maximum(A.std(axis=0), floor)
    return mu, sd


# ------------------------------------------------- the map with the network
# The learned snow return map as a substep uses it, in FP64: the trial
# gradient's singular values come from the eigenvalues of b = F^ F^T; the
# network predicts ln(s'/s) and J_P'/J_P; a particle keeps the prediction only
# if the rebuild without eigenvectors is well conditioned and the prediction
# passes the residual checks, else it takes the exact map.  The new gradient
# is U diag(s'/s) U^T F^ (U the eigenvectors of b), which has the principal
# directions of F^ and the singular values s'.
EIG_GAP = 0.1      # smallest gap between eigenvalues of the normalised deviator of b
EIG_RESOLVE = 2e-5  # the deviator of b must exceed this multiple of its mean to be resolved


def snow_map_network(mat: dict, Fhat: np.ndarray, Jp: np.ndarray, theta: np.ndarray, norm: np.ndarray,
                     dt: float, dt_ref: float, tol: float, gap: float = EIG_GAP, predict=None):
    """Fhat (N,3,3) trial gradients, Jp (N,).  Returns (Fe (N,3,3), Jp_new (N,),
    used (N,) bool: the network's prediction was kept, margins (N,5): signed
    distances of the decision quantities to their thresholds, positive on the
    network's side: the two eigenvalue gaps in eigenvalue units of b, and the
    three residuals in their units).
    predict(X) -> outputs in physical units may stand in for the network."""
    from . import snow_project  # the exact map (C oracle)

    Fhat = np.asarray(Fhat, dtype=np.float64)
    Jp = np.asarray(Jp, dtype=np.float64)
    N = Fhat.shape[0]
    b = Fhat @ np.transpose(Fhat, (0, 2, 1))
    lam, U = np.linalg.eigh(b)              # ascending
    lam, U = lam[:, ::-1], U[:, :, ::-1]    # descending
    q = np.trace(b, axis1=1, axis2=2) / 3.0
    dev = b - q[:, None, None] * np.eye(3)
    p = np.sqrt(np.sum(dev * dev, axis=(1, 2)) / 6.0)
    with np.errstate(divide="ignore", invalid="ignore"):
        mu = (lam - q[:, None]) / p[:, None]
    detF = np.linalg.det(Fhat)
    resolved = p > EIG_RESOLVE * np.abs(q)
    g01, g12 = mu[:, 0] - mu[:, 1], mu[:, 1] - mu[:, 2]
    eligible = resolved & (detF > 0) & (g01 >= gap) & (g12 >= gap)
    sh = np.sqrt(np.maximum(lam, 1e-30))
    X = features(mat, sh, Jp, dt, dt_ref)
    if predict is None:
        Y, _ = forward(theta, (X - norm[0:12]) / norm[12:24])
        yv = Y * norm[36:48] + norm[24:36]
    else:
        yv = predict(X)
    sn = sh * np.exp(yv[:, 3:6])
    Jpn = Jp * yv[:, 9]
    mu0, la0 = lame(mat)
    h = np.exp(mat["xi"] * (1.0 - Jpn))
    Jn = np.prod(sn, axis=1)
    tk = 2.0 * (mu0 * h)[:, None] * (sn - 1.0) * sn + ((la0 * h) * (Jn - 1.0) * Jn)[:, None]
    lo, hi = 1 - mat["theta_c"], 1 + mat["theta_s"]
    with np.errstate(invalid="ignore", divide="ignore"):
        res_t = np.max(np.abs(yv[:, 6:9] - tk / mat["E"]), axis=1)
        res_y = np.max(np.maximum(lo - sn, sn - hi), axis=1)
        res_v = np.abs(np.log(Jn * Jpn) - np.log(np.prod(sh, axis=1) * Jp))
    finite = np.isfinite(tk.sum(axis=1) + Jpn + sn.sum(axis=1))
    used = eligible & finite & (res_y <= tol) & (res_v <= tol) & (res_t <= tol)
    Fe = np.empty_like(Fhat)
    Jp_new = np.empty_like(Jp)
    G = U @ (np.where(used[:, None], sn / sh, 1.0)[:, :, None] * np.transpose(U, (0, 2, 1)))
    Fe[used] = (G @ Fhat)[used]
    Jp_new[used] = Jpn[used]
    for k in np.nonzero(~used)[0]:
        Fe[k], Jp_new[k] = snow_project(mat, Fhat[k], Jp[k])
    # gap margins in eigenvalue units of b (the normalised gaps times p), the
    # size an error in b has to reach to flip the decision
    margins = np.stack([(g01 - gap) * p, (g12 - gap) * p, tol - res_y, tol - res_v, tol - res_t], axis=1)
    return Fe, Jp_new, used, margins


def substep_network(cfg: dict, mat: dict, st: dict, theta: np.ndarray, norm: np.ndarray, tol: float,
                    dt_ref: float, steps: int = 1):
    """`steps` substeps of a snow scene whose return map is the learned one:
    P2G, grid update and G2P of the FP64 oracle, each G2P's trial gradient
    mapped by snow_map_network.  Returns (state, used, margins): used and
    margins of the last map, and for every particle the margin of smallest
    size (per decision quantity) over all the maps."""
    from . import _state, g2p_trial, grid_update, p2g

    s = _state(st)
    N = s["x"].shape[1]
    used = margins = None
    for _ in range(steps):
        s, gm, gp, bad = p2g(cfg, mat, s)
        assert bad == 0
        gv = grid_update(cfg, gm, gp)
        s, bad = g2p_trial(cfg, mat, s, gv)
        assert bad == 0
        Fhat = s["F"].T.reshape(N, 3, 3)
        Fe, Jpn, used, m = snow_map_network(mat, Fhat, s["s"], theta, norm, cfg["dt"], dt_ref, tol)
        margins = m if margins is None else np.where(np.abs(m) < np.abs(margins), m, margins)
        s["F"] = np.ascontiguousarray(Fe.reshape(N, 9).T)
        s["s"] = Jpn
    return s, used, margins
