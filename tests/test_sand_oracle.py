"""Pins of the oracle's Drucker-Prager sand (the stand-in for the paper's sand
model, which the paper cites but does not give): Hencky elasticity and the
return map in logarithmic strain with friction-angle hardening.

Each pin checks a property fixed by the mathematics, not the oracle's own
formulas: the stress is the gradient of the log-strain energy (finite
differences over numpy's SVD), the cone is the Mohr-Coulomb one in
triaxial compression, and the return map keeps the volume and the
principal axes, puts plastic states on the cone, leaves elastic ones alone,
releases all strain under expansion, is idempotent, commutes with rotations
and grows the hardening state by the plastic log-strain it removed."""
import numpy as np
import pytest

from paper_2111_00699_amd import scenes

from .test_oracle_pins import lame, rot

SAND = scenes.SAND


def log_strain(F):
    U, S, Vt = np.linalg.svd(F)
    return np.log(S), U, Vt.T


def dp_yield(mat, tau, q, oracle):
    """||dev tau||_F + alpha(q) tr tau: negative inside the cone, zero on it."""
    t = np.trace(tau)
    dev = tau - t / 3.0 * np.eye(3)
    return np.linalg.norm(dev) + oracle.sand_alpha(mat, q) * t


def test_hencky_stress_is_the_log_strain_energy_gradient(oracle):
    mu, la = lame(SAND["E"], SAND["nu"])

    def psi(F):
        e = np.log(np.linalg.svd(F, compute_uv=False))
        return mu * np.sum(e * e) + 0.5 * la * np.sum(e) ** 2

    for i in range(20):
        F = np.eye(3) + scenes.uniform(300, 9, i, -0.15, 0.15).reshape(3, 3)
        h = 1e-6
        P = np.zeros((3, 3))
        for a in range(3):
            for b in range(3):
                d = np.zeros((3, 3)); d[a, b] = h
                P[a, b] = (psi(F + d) - psi(F - d)) / (2 * h)
        want = P @ F.T  # Kirchhoff stress tau = dpsi/dF F^T
        got = oracle.hencky(F, mu, la)
        assert np.abs(got - want).max() <= 1e-7 * np.abs(want).max(), i
        assert np.allclose(got, got.T, atol=1e-9 * np.abs(got).max())
        assert np.allclose(oracle.stress(SAND, F, 1.3), got, rtol=0, atol=1e-12 * np.abs(got).max())


@pytest.mark.parametrize("q,phi", [(0.0, 25.0), (400.0, 35.0)])
def test_cone_is_mohr_coulomb_in_triaxial_compression(oracle, q, phi):
    """Friction angle phi(0) = h0 - h3 and phi(inf) = h0.  The cone
    ||dev tau|| + alpha tr tau = 0 must pass through the cohesionless
    Mohr-Coulomb state of that angle under triaxial compression
    (principal stresses a = a > b, tension positive: a - b = -(a + b) sin phi)."""
    s = np.sin(np.radians(phi))
    b = -1.0
    a = (s - 1.0) / (1.0 + s)
    assert abs((a - b) + (a + b) * s) < 1e-15  # on the Mohr-Coulomb surface
    assert abs(dp_yield(SAND, np.diag([a, a, b]), q, oracle)) < 1e-12
    # a slightly milder deviator is inside, a stronger one outside
    assert dp_yield(SAND, np.diag([a - 0.01, a - 0.01, b]), q, oracle) < 0
    assert dp_yield(SAND, np.diag([a + 0.01, a + 0.01, b]), q, oracle) > 0


def test_phi_hardens_monotonically(oracle):
    alphas = [oracle.sand_alpha(SAND, q) for q in np.linspace(0.0, 3.0, 31)]
    assert np.all(np.diff(alphas) > 0)


def _trial(i, spread, squeeze):
    """A trial gradient P diag(sig) Q^T with chosen log-strain trace."""
    e = scenes.uniform(310, 3, i, -spread, spread)
    e = e - e.mean() + squeeze / 3.0
    return rot(1200 + i) @ np.diag(np.exp(e)) @ rot(1300 + i).T


def test_return_map_cases(oracle):
    mu, la = lame(SAND["E"], SAND["nu"])
    seen = {"inside": 0, "cone": 0, "tip": 0}
    for i in range(300):
        Fh = _trial(i, spread=0.08, squeeze=scenes.uniform(311, 1, i, -0.15, 0.05)[0])
        q = scenes.uniform(312, 1, i, 0.0, 1.0)[0]
        Fe, q1 = oracle.sand_project(SAND, Fh, q)
        e0, U0, V0 = log_strain(Fh)
        e1 = np.log(np.linalg.svd(Fe, compute_uv=False))
        # principal axes are kept: U0^T Fe V0 is diagonal
        D = U0.T @ Fe @ V0
        assert np.abs(D - np.diag(np.diag(D))).max() < 1e-12
        # the hardening state grows by the log strain removed
        assert abs((q1 - q) - np.linalg.norm(np.sort(e0) - np.sort(np.log(np.abs(np.diag(D)))))) < 1e-12
        tau0 = oracle.hencky(Fh, mu, la)
        if np.sum(e0) > 0:  # expansion: all strain released, Fe is the polar rotation of Fh
            seen["tip"] += 1
            assert np.allclose(Fe, U0 @ V0.T, atol=1e-12)
            assert abs(q1 - q - np.linalg.norm(e0)) < 1e-12
        elif dp_yield(SAND, tau0, q, oracle) <= 0:  # elastic: unchanged
            seen["inside"] += 1
            assert np.allclose(Fe, Fh, atol=1e-13) and q1 == q
        else:  # plastic: onto the cone, volume kept, deviator scaled down along itself
            seen["cone"] += 1
            tau1 = oracle.hencky(Fe, mu, la)
            assert abs(dp_yield(SAND, tau1, q, oracle)) <= 1e-9 * np.abs(tau0).max()
            assert abs(np.linalg.det(Fe) - np.linalg.det(Fh)) < 1e-12
            d0 = tau0 - np.trace(tau0) / 3 * np.eye(3)
            d1 = tau1 - np.trace(tau1) / 3 * np.eye(3)
            cos = np.sum(d0 * d1) / (np.linalg.norm(d0) * np.linalg.norm(d1) + 1e-300)
            assert cos > 1 - 1e-10 and np.linalg.norm(d1) < np.linalg.norm(d0)
            assert q1 > q
        # idempotent
        Fe2, q2 = oracle.sand_project(SAND, Fe, q1)
        assert np.allclose(Fe2, Fe, atol=1e-11) and abs(q2 - q1) < 1e-11
        # rotations on either side commute with the map
        R = rot(1400 + i)
        FeL, qL = oracle.sand_project(SAND, R @ Fh, q)
        FeR, qR = oracle.sand_project(SAND, Fh @ R, q)
        assert np.allclose(FeL, R @ Fe, atol=1e-12) and np.allclose(FeR, Fe @ R, atol=1e-12)
        assert abs(qL - q1) < 1e-12 and abs(qR - q1) < 1e-12
    assert min(seen.values()) >= 20, seen


def test_inverted_gradient_is_taken_without_its_sign(oracle):
    """An inverted trial gradient: the stress uses log |sig| (that of its
    reflection); inside the cone the map leaves it as it is (still inverted),
    and on the cone or in expansion it is rebuilt from |sig| like its
    reflection, coming out with a positive determinant."""
    P, Q = rot(1500), rot(1501)
    mu, la = lame(SAND["E"], SAND["nu"])
    # inside the cone (dg < 0 at q = 0.2), on it, and in expansion
    for sig, case in (([1.02, 0.97, 0.9], "inside"), ([1.1, 0.93, 0.85], "cone"), ([1.05, 1.02, 1.01], "tip")):
        sig = np.array(sig)
        Fh = P @ np.diag(sig * [1, 1, -1]) @ Q.T
        Fr = P @ np.diag(sig) @ Q.T
        Fe, q = oracle.sand_project(SAND, Fh, 0.2)
        Fer, qr = oracle.sand_project(SAND, Fr, 0.2)
        assert np.linalg.det(Fh) < 0
        assert abs(q - qr) < 1e-12
        if case == "inside":
            assert q == 0.2 and np.array_equal(Fe, Fh) and np.array_equal(Fer, Fr)
        else:
            assert q > 0.2 and np.linalg.det(Fe) > 0
            assert np.allclose(Fe, Fer, atol=1e-12)
        assert np.allclose(oracle.hencky(Fh, mu, la), oracle.hencky(Fr, mu, la), atol=1e-9)


def test_sand_substep_moves_hardening_only_where_plastic(oracle):
    """A sand block squeezed by its velocity field: the substep's stored
    F and q agree with the return map applied to (I + dt C') F."""
    N = 400
    x = scenes.uniform(320, 3 * N, 0, 0.4, 0.6).reshape(3, N).astype(np.float32)
    st = scenes.nontrivial_state(x, seed=321, kind="sand")
    st["F"] = (np.eye(3).reshape(9, 1) + 3.0 * (st["F"].astype(np.float64) - np.eye(3).reshape(9, 1)))
    cfg = dict(n=32, bc="sticky", dt=2e-3)
    out, _, _, bad = oracle.substep(cfg, SAND, st)
    assert bad == 0
    F0 = st["F"].T.reshape(N, 3, 3)
    moved = 0
    for p in range(N):
        G = np.eye(3) + cfg["dt"] * out["C"][:, p].reshape(3, 3)
        Fe, q = oracle.sand_project(SAND, G @ F0[p], st["s"][p] - 1.0)
        assert np.allclose(out["F"][:, p].reshape(3, 3), Fe, atol=1e-12)
        assert abs(out["s"][p] - (1.0 + q)) < 1e-12
        moved += q > st["s"][p] - 1.0 + 1e-9
    assert 0 < moved < N
