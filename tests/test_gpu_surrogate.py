"""GPU tests of the learned snow surrogate's kernels through the C ABI,
against the FP64 oracle in oracle/surrogate.py.

Bars: FP32 forward and gradient within 1e-4 normwise of the oracle (the
gradient check the training relies on); BF16 MFMA forward within 1e-2 and
its gradient within 3e-2; training pairs sampled from a running snow scene
equal the oracle's features and targets of the same trial states; Adam
training on those pairs lowers the loss."""
import numpy as np
import pytest

from oracle import surrogate as S
from paper_2111_00699_amd import scenes

from .test_gpu_parity import normwise, print_case

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_cuda():
    import torch

    if not torch.cuda.is_available():
        pytest.fail("a GPU test ran without a visible GPU")
    return torch


def random_net(seed):
    theta = scenes.mlp_init(seed).astype(np.float64)
    theta += scenes.uniform(seed, theta.size, 9, -0.05, 0.05)
    return theta


def trial_rows(seed, count):
    st = scenes.snow_trial_states(seed, count)
    X = S.features(scenes.SNOW, st["sig_hat"], st["Jp"], 5e-5, 5e-5)
    T = S.targets(scenes.SNOW, st["sig_hat"], st["Jp"])
    return X, T


def norm_vec(X, T):
    mi, si = S.normalize_stats(X)
    mo, so = S.normalize_stats(T)
    return np.concatenate([mi, si, mo, so])


def zscore(A, mu, sd):
    return (A - mu) / sd


def make(torch_cuda, theta, norm):
    from paper_2111_00699_amd import mpm

    sur = mpm.Surrogate()
    sur.set(theta.astype(np.float32), norm.astype(np.float32))
    return sur


@pytest.mark.parametrize("count", [1, 37, 1000])
def test_forward_matches_the_oracle(torch_cuda, count):
    from paper_2111_00699_amd import mpm

    theta = random_net(21)
    X, T = trial_rows(31, count)
    nv = norm_vec(*trial_rows(32, 4000))
    print_case("sur_forward", count=count)
    sur = make(torch_cuda, theta, nv)
    th32 = theta.astype(np.float32).astype(np.float64)  # the parameters the GPU holds
    Yo, _ = S.forward(th32, zscore(X.astype(np.float32).astype(np.float64), nv[:12], nv[12:24]))
    Yo = Yo * nv[36:48] + nv[24:36]
    for prec, tol in ((mpm.SUR_FP32, 1e-4), (mpm.SUR_BF16, 1e-2)):
        Yg = sur.forward(X.astype(np.float32), prec).cpu().numpy()
        z = zscore(Yg, nv[24:36], nv[36:48]) - zscore(Yo, nv[24:36], nv[36:48])
        err = np.abs(z).max() / max(np.abs(zscore(Yo, nv[24:36], nv[36:48])).max(), 1e-30)
        assert err <= tol, (prec, err)
    sur.close()


@pytest.mark.parametrize("count", [16, 45, 2048])
def test_gradient_matches_the_oracle(torch_cuda, count):
    """The FP32 form of the training kernel against backpropagation in FP64
    (itself pinned to central differences)."""
    from paper_2111_00699_amd import mpm

    theta = random_net(22)
    X, T = trial_rows(33, count)
    nv = norm_vec(*trial_rows(34, 4000))
    sur = make(torch_cuda, theta, nv)
    th32 = theta.astype(np.float32).astype(np.float64)
    Xz = zscore(X.astype(np.float32).astype(np.float64), nv[:12], nv[12:24])
    Tz = zscore(T.astype(np.float32).astype(np.float64), nv[24:36], nv[36:48])
    go = S.grad(th32, Xz, Tz)
    lo = S.loss(th32, Xz, Tz)
    for prec, tol in ((mpm.SUR_FP32, 1e-4), (mpm.SUR_BF16, 3e-2)):
        lg, gg = sur.loss_grad(X.astype(np.float32), T.astype(np.float32), prec)
        gg = gg.cpu().numpy()
        assert abs(lg - lo) <= 10 * tol * abs(lo), (prec, lg, lo)
        assert normwise(gg, go) <= tol, (prec, normwise(gg, go))
        # every block of parameters, not only the largest entries
        for name, a, b in (("W1", 0, 768), ("W2", 832, 4928), ("W3", 4992, 5760), ("b", 5760, 5772)):
            assert normwise(gg[a:b], go[a:b]) <= 3 * tol, (prec, name)
    sur.close()


def test_training_pairs_from_a_snow_scene(torch_cuda, oracle):
    """Rows sampled from a running snow scene: features and targets of the
    same trial states as the oracle defines them."""
    from paper_2111_00699_amd import mpm

    sc = scenes.jelly_cube(0)
    st = scenes.nontrivial_state(sc["x"], seed=5, kind="snow")
    sim = mpm.Sim(64, 1e-4, bc="separate")
    sim.add_particles(scenes.SNOW, st["x"], v=st["v"], C=st["C"], F=st["F"], s=st["s"])
    sim.substep(2)
    X, T = mpm.Surrogate.sample(sim, dt_ref=5e-5)
    X, T = X.cpu().numpy().astype(np.float64), T.cpu().numpy().astype(np.float64)
    assert X.shape[0] == sc["x"].shape[1]
    Xo = S.features(scenes.SNOW, X[:, 0:3], X[:, 6], 1e-4, 5e-5)
    To = S.targets(scenes.SNOW, X[:, 0:3], X[:, 6])
    assert np.all(np.diff(X[:, 0:3], axis=1) <= 0)  # descending
    for k in range(12):
        assert normwise(X[:, k], Xo[:, k]) <= 1e-5, ("feature", k)
        # FP32 rounding of the clamp bounds (1 - theta_c, 1 + theta_s) is ~3e-8 absolute
        err = np.abs(T[:, k] - To[:, k]).max()
        assert err <= 1e-7 + 1e-4 * np.abs(To[:, k]).max(), ("target", k, err)
    # a good share of the states sit on the yield surface (the return map is active)
    clamped = np.any(np.abs(T[:, 3:6]) > 1e-7, axis=1).mean()
    assert clamped > 0.2, clamped
    sim.close()


def test_training_lowers_the_loss(torch_cuda):
    from paper_2111_00699_amd import mpm

    X, T = trial_rows(35, 20000)
    sur = make(torch_cuda, scenes.mlp_init(4).astype(np.float64), np.concatenate([np.zeros(12), np.ones(12),
                                                                                 np.zeros(12), np.ones(12)]))
    sur.fit_norm(X.astype(np.float32), T.astype(np.float32))
    l0, _ = sur.loss_grad(X.astype(np.float32), T.astype(np.float32), mpm.SUR_FP32)
    losses = sur.train(X.astype(np.float32), T.astype(np.float32), steps=300, batch=1024, lr=3e-3, seed=1)
    assert np.all(np.isfinite(losses))
    l1, _ = sur.loss_grad(X.astype(np.float32), T.astype(np.float32), mpm.SUR_FP32)
    assert l1 < 0.1 * l0, (l0, l1)
    assert losses[-20:].mean() < 0.2 * losses[:20].mean()
    sur.close()


@pytest.mark.parametrize("mode", [2])
def test_closed_form_map_matches_the_oracle(torch_cuda, oracle, mode):
    """Mode 2 (the eigenvector-free path with the exact clamp) is the same
    map as the exact path: one substep from the random snow state matches the
    FP64 oracle like the exact path does, with most particles taking the
    closed form (the rest fall back where eigenvalues nearly coincide)."""
    from paper_2111_00699_amd import mpm

    from .test_gpu_parity import compare_state, gpu_state

    sc = scenes.jelly_cube(0)
    st = scenes.nontrivial_state(sc["x"], seed=5, kind="snow")
    cfg = dict(n=64, dt=1e-4, bc="separate")
    sim = mpm.Sim(64, 1e-4, bc="separate")
    sim.add_particles(scenes.SNOW, st["x"], v=st["v"], C=st["C"], F=st["F"], s=st["s"])
    sim.use_surrogate(mode)
    sim.substep(2)
    gs = gpu_state(sim)
    os_, _, _, bad = oracle.substep(cfg, scenes.SNOW, st, steps=2)
    assert bad == 0
    compare_state(gs, os_, "snow", n=64)
    stats = sim.stats()
    assert stats["surrogate_particles"] > 0.5 * 2 * sc["x"].shape[1], stats
    sim.close()


def test_trained_surrogate_runs_in_the_substep(torch_cuda):
    """A network trained on pairs from the exact path drives a snow scene:
    the run stays finite, the fallback counters add up, and the state stays
    close to the exact run (the bar here is loose; the bench reports the
    error of the full scene)."""
    from paper_2111_00699_amd import mpm

    sc = scenes.jelly_cube(0)
    st = scenes.nontrivial_state(sc["x"], seed=5, kind="snow")

    def run(mode, sur=None):
        sim = mpm.Sim(64, 1e-4, bc="separate")
        sim.add_particles(scenes.SNOW, st["x"], v=st["v"], C=st["C"], F=st["F"], s=st["s"])
        if mode:
            sim.use_surrogate(mode, sur, tol=1e-2, dt_ref=1e-4)
        sim.substep(5)
        out = gpu_state_local(sim)
        stats = sim.stats()
        sim.close()
        return out, stats

    def gpu_state_local(sim):
        return {k: v.cpu().numpy() for k, v in sim.read_particles().items()}

    # training pairs from the exact run, states after 0..4 substeps
    sim = mpm.Sim(64, 1e-4, bc="separate")
    sim.add_particles(scenes.SNOW, st["x"], v=st["v"], C=st["C"], F=st["F"], s=st["s"])
    Xs, Ts = [], []
    for _ in range(5):
        X, T = mpm.Surrogate.sample(sim, dt_ref=1e-4)
        Xs.append(X.clone())
        Ts.append(T.clone())
        sim.substep(1)
    sim.close()
    X = torch_cuda.cat(Xs)
    T = torch_cuda.cat(Ts)
    sur = mpm.Surrogate()
    sur.set(scenes.mlp_init(4))
    sur.fit_norm(X, T)
    losses = sur.train(X, T, steps=400, batch=4096, lr=3e-3, seed=2)
    assert losses[-20:].mean() < 0.3 * losses[:20].mean()
    exact, _ = run(0)
    got, stats = run(1, sur)
    assert stats["surrogate_particles"] + stats["surrogate_fallbacks"] >= 5 * sc["x"].shape[1]
    for k in ("x", "v", "F", "s"):
        assert np.all(np.isfinite(got[k])), k
    assert normwise(got["x"], exact["x"]) < 1e-4
    sur.close()


def _oracle_trained_network(seed=12, count=20000, steps=600, batch=1024, lr=3e-3):
    """A network trained by the FP64 oracle's own backpropagation and Adam on
    exact-map pairs (so no input of the oracle comes from the GPU): trial
    singular values 1 +- 0.04 and J_P in [0.85, 1.1].  Returns (theta, norm)."""
    st = scenes.snow_trial_states(seed, count, spread=0.04)
    X = S.features(scenes.SNOW, st["sig_hat"], st["Jp"], 1e-4, 1e-4)
    T = S.targets(scenes.SNOW, st["sig_hat"], st["Jp"])
    norm = norm_vec(X, T)
    Xn, Tn = zscore(X, norm[0:12], norm[12:24]), zscore(T, norm[24:36], norm[36:48])
    theta = scenes.mlp_init(seed).astype(np.float64)
    m, v = np.zeros_like(theta), np.zeros_like(theta)
    rows = (scenes.splitmix64(seed, steps * batch, 77) % np.uint64(count)).astype(np.int64).reshape(steps, batch)
    for t in range(steps):
        g = S.grad(theta, Xn[rows[t]], Tn[rows[t]])
        theta, m, v = S.adam_step(theta, g, m, v, t + 1, lr=lr)
    return theta, norm


def test_learned_substep_matches_the_oracle(torch_cuda, oracle):
    """Mode 1 (the network P2G runs on BF16 MFMA, with its fallback checks)
    against the FP64 oracle running the same network in place of the return
    map (oracle/surrogate.py: substep_network), two substeps of a snow state
    near the yield surface, so that P2G applies the network to the first
    substep's trial gradients and the read applies it to the second's.
    * Particles whose decision quantities (eigenvalue gaps, residuals) lie
      within a margin of a threshold in either map are left out of the
      per-particle check (BF16 against FP64 can decide them either way); they
      must be fewer than a fifth.
    * The kept particles: F and J_P within a BF16 bar, 8 x 2^-8 of the
      largest output spread the map uses (ln(s'/s), J_P'/J_P), per entry.
    * x, v, C of all particles within 5e-3 normwise (the BF16 stress error
      reaches them through P2G)."""
    from paper_2111_00699_amd import mpm

    theta, norm = _oracle_trained_network()
    theta32 = theta.astype(np.float32)
    x = scenes.jelly_cube(0)["x"]
    N = x.shape[1]
    st = scenes.nontrivial_state(x, seed=21, kind="snow")
    # elastic gradients near the yield surface: R1 diag(s) R2 with s in [0.97, 1.012]
    from .test_oracle_pins import rot

    sv = scenes.uniform(21, 3 * N, 40, 0.97, 1.012).reshape(N, 3)
    R1 = np.stack([rot(7000 + k % 97) for k in range(N)])
    R2 = np.stack([rot(9000 + k % 89) for k in range(N)])
    st["F"] = np.ascontiguousarray((R1 * sv[:, None, :]) @ np.transpose(R2, (0, 2, 1))).reshape(N, 9).T.astype(np.float32)
    st["C"] = (st["C"] * np.float32(0.2)).astype(np.float32)
    cfg = dict(n=64, dt=1e-4, bc="separate")
    tol = 2e-2
    print_case("learned_substep", N=N, tol=tol)
    sur = mpm.Surrogate()
    sur.set(theta32, norm.astype(np.float32))
    sim = mpm.Sim(64, 1e-4, bc="separate")
    sim.add_particles(scenes.SNOW, st["x"], v=st["v"], C=st["C"], F=st["F"], s=st["s"])
    sim.use_surrogate(1, sur, tol=tol, dt_ref=1e-4)
    sim.substep(2)
    gs = {k: t.cpu().numpy().astype(np.float64) for k, t in sim.read_particles().items()}
    stats = sim.stats()
    sim.close()
    sur.close()
    os_, used, margins = S.substep_network(cfg, scenes.SNOW, st, theta32.astype(np.float64), norm, tol, 1e-4, steps=2)
    # margins (the smallest over both maps): the eigenvalue gaps in eigenvalue units of b = F^ F^T,
    # where the first map's BF16 error in F (below 2e-4 on every particle) moves b by less than
    # 5e-4; the residuals in their units, where BF16 moves them by less than 2e-3
    near = np.any(np.abs(margins[:, :2]) < 5e-4, axis=1) | np.any(np.abs(margins[:, 2:]) < 2e-3, axis=1)
    keep = ~near
    print(f"[learned] used={used.mean():.3f} near={near.mean():.3f} gpu_surrogate={stats['surrogate_particles']} "
          f"fallbacks={stats['surrogate_fallbacks']}", flush=True)
    assert used.mean() > 0.3  # the network carries a good share of the particles
    assert (~used).mean() > 0.02  # and the fallback is exercised too
    assert near.mean() < 0.2
    osd = norm[36:48]
    bar = 8 * 2.0 ** -8 * max(osd[3:6].max(), osd[9])
    eF = np.abs(gs["F"] - os_["F"]).max(axis=0)
    es = np.abs(gs["s"] - os_["s"]) / os_["s"]
    dF, ds = eF[keep].max(), es[keep].max()
    print(f"[learned] F err quantiles 50/99/max {np.quantile(eF, 0.5):.2e} {np.quantile(eF, 0.99):.2e} {eF.max():.2e}; "
          f"above bar: kept {(eF[keep] > bar).sum()} near {(eF[near] > bar).sum()}", flush=True)
    errs = {k: normwise(gs[k], os_[k]) for k in ("x", "v", "C")}
    print(f"[learned] bar={bar:.2e} dF={dF:.2e} ds={ds:.2e} " + " ".join(f"{k}={e:.2e}" for k, e in errs.items()),
          flush=True)
    assert dF <= bar
    assert ds <= bar
    for k, e in errs.items():
        assert e <= 5e-3, (k, e)
