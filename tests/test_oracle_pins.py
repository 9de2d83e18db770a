"""Pins of the FP64 oracle against what the paper and the mathematics fix.

Each test states the passage (or the mathematical fact) it rests on.  They are
chosen so that a dropped factor, a wrong sign, an index mix-up between
dimensions or a transposed operand in the oracle fails at least one of them.
"""
import math
import os

import numpy as np
import pytest

from oracle import oracle as O
from paper_2305_15693_amd import inputs as I

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _modes_ball(d, kcut, include_zero=False):
    M = int(math.floor(kcut))
    n = O.mode_vectors(d, M)
    n2 = (n.astype(np.int64) ** 2).sum(1)
    keep = (n2 <= kcut * kcut) & ((n2 > 0) | include_zero)
    return np.ascontiguousarray(n[keep])


def test_S_at_k0_is_N():
    # S(0) = N: every term of rho(0) equals one (Eq. structure_factor with c_n = 1).
    pos = I.positions(300, 2, 7.0, np.float64, seed=3)
    S = O.structure_factor(pos, 7.0, np.zeros((1, 2), np.int32))
    assert S[0] == pytest.approx(300.0, rel=1e-14)


def test_lattice_32x32_is_stealthy_to_16():
    # Square lattice m = 32 points per side, spacing L/m: S = N on the reciprocal
    # lattice n = 0 mod m and 0 elsewhere.  With L = 32 every mode 0 < |n| <= 16 is
    # off the reciprocal lattice, so S, the loss and its gradient all vanish.
    pos = I.square_lattice(32, 32.0, 2, shift=(0.3, 0.7))
    modes = _modes_ball(2, 16.0)
    W = np.ones(len(modes))
    r = O.loss_grad(pos, 32.0, modes, W, np.zeros(len(modes)))
    assert np.max(r["S"]) < 1e-20
    assert r["loss"] < 1e-30
    assert np.max(np.abs(r["grad"])) < 1e-12


def test_lattice_16x16_bragg_peaks_pin_inclusive_boundary():
    # 16 x 16 lattice of spacing 2 in L = 32: Bragg peaks S = N = 256 at the four
    # modes (+-16, 0), (0, +-16), which lie exactly on |n| = 16.  With the set
    # 0 < |n| <= 16 (inclusive) and weight 1 the loss is 4 * 256^2; a shift of the
    # lattice changes nothing.
    for shift in [(0.0, 0.0), (0.37, 1.91)]:
        pos = I.square_lattice(16, 32.0, 2, shift=shift)
        modes = _modes_ball(2, 16.0)
        S = O.structure_factor(pos, 32.0, modes)
        peak = np.all(np.mod(modes, 16) == 0, axis=1)
        assert peak.sum() == 4
        np.testing.assert_allclose(S[peak], 256.0, rtol=1e-12)
        assert np.max(S[~peak]) < 1e-18
        r = O.loss_grad(pos, 32.0, modes, np.ones(len(modes)), np.zeros(len(modes)),
                        want_grad=False)
        assert r["loss"] == pytest.approx(4 * 256.0 ** 2, rel=1e-12)


def test_single_point():
    # N = 1: |rho|^2 = 1 for every k, so S = 1 and the loss does not depend on r.
    pos = np.array([[0.123, 4.56]])
    modes = _modes_ball(2, 5.0)
    r = O.loss_grad(pos, 9.0, modes, np.ones(len(modes)), np.zeros(len(modes)))
    np.testing.assert_allclose(r["S"], 1.0, rtol=1e-14)
    assert np.max(np.abs(r["grad"])) < 1e-12


@pytest.mark.parametrize("L", [(5.0, 5.0), (3.0, 7.5)])
def test_two_points_closed_form(L):
    # N = 2: S(k) = 1 + cos(k.D), D = r1 - r2, and with L = sum W (S - S0)^2
    #   dL/dr1 = -sum_k 2 W (S - S0) sin(k.D) k,   dL/dr2 = -dL/dr1.
    # An anisotropic box checks that each dimension uses its own side.
    rng = np.random.default_rng(7)
    pos = rng.uniform(0, 1, (2, 2)) * np.asarray(L)
    modes = _modes_ball(2, 4.0)
    k = 2 * np.pi * modes / np.asarray(L)
    W = rng.uniform(0.5, 2.0, len(modes))
    S0 = rng.uniform(0.0, 1.0, len(modes))
    D = pos[0] - pos[1]
    S_ref = 1 + np.cos(k @ D)
    r = O.loss_grad(pos, L, modes, W, S0)
    np.testing.assert_allclose(r["S"], S_ref, rtol=1e-13, atol=1e-14)
    loss_ref = np.sum(W * (S_ref - S0) ** 2)
    assert r["loss"] == pytest.approx(loss_ref, rel=1e-13)
    g1 = -np.sum((2 * W * (S_ref - S0) * np.sin(k @ D))[:, None] * k, axis=0)
    np.testing.assert_allclose(r["grad"][0], g1, rtol=1e-12, atol=1e-12)
    np.testing.assert_allclose(r["grad"][1], -g1, rtol=1e-12, atol=1e-12)


def test_pair_form_of_S():
    # Expanding |rho|^2 gives S(k) = 1 + (2/N) sum_{i<j} cos(k.(r_i - r_j)), an
    # independent brute-force formula (no exponentials of single positions).
    rng = np.random.default_rng(11)
    N, L = 64, np.array([6.0, 6.0, 4.0])
    pos = rng.uniform(0, 1, (N, 3)) * L
    modes = _modes_ball(3, 3.0)
    k = 2 * np.pi * modes / L
    diff = pos[:, None, :] - pos[None, :, :]
    iu = np.triu_indices(N, 1)
    ph = np.einsum("qa,pa->qp", k, diff[iu])
    S_pair = 1 + (2.0 / N) * np.cos(ph).sum(1)
    S = O.structure_factor(pos, L, modes)
    np.testing.assert_allclose(S, S_pair, rtol=1e-11, atol=1e-12)


def test_invariances_and_sum_rule():
    # Friedel's law S(k) = S(-k) for real rho (main text, Friedel's law); S is
    # invariant under a global translation and under relabelling the points;
    # translation invariance of the loss makes the gradients sum to zero.
    rng = np.random.default_rng(5)
    N, L = 200, np.array([10.0, 12.0])
    pos = rng.uniform(0, 1, (N, 2)) * L
    modes = _modes_ball(2, 6.0)
    S = O.structure_factor(pos, L, modes)
    np.testing.assert_allclose(O.structure_factor(pos, L, -modes), S, rtol=1e-11, atol=1e-12)
    np.testing.assert_allclose(O.structure_factor(pos + np.array([1.234, -5.5]), L, modes), S,
                               rtol=1e-10, atol=1e-11)
    np.testing.assert_allclose(O.structure_factor(pos[rng.permutation(N)], L, modes), S,
                               rtol=1e-11, atol=1e-12)
    W = rng.uniform(0.1, 1.0, len(modes))
    S0 = rng.uniform(0.0, 2.0, len(modes))
    g = O.loss_grad(pos, L, modes, W, S0)["grad"]
    scale = np.abs(g).max()
    assert np.abs(g.sum(0)).max() < 1e-11 * scale * N


def test_sign_convention_is_immaterial():
    # Using exp(-i k.r) instead of exp(+i k.r) is the same as evaluating the set at
    # -n with weights and targets carried along: S, the loss and the gradient agree.
    rng = np.random.default_rng(9)
    N, L = 150, 8.0
    pos = rng.uniform(0, L, (N, 2))
    modes = _modes_ball(2, 5.0)
    W = rng.uniform(0.1, 1.0, len(modes))
    S0 = rng.uniform(0.0, 2.0, len(modes))
    a = O.loss_grad(pos, L, modes, W, S0)
    b = O.loss_grad(pos, L, -modes, W, S0)
    np.testing.assert_allclose(b["S"], a["S"], rtol=1e-11, atol=1e-12)
    assert b["loss"] == pytest.approx(a["loss"], rel=1e-12)
    np.testing.assert_allclose(b["grad"], a["grad"], rtol=1e-10, atol=1e-10 * np.abs(a["grad"]).max())


def test_poisson_mean():
    # For i.i.d. uniform points E[S(k)] = 1 at every nonzero mode of the reciprocal
    # lattice (the Poisson value S = 1 quoted in the main text); S(k) is
    # asymptotically exponential with unit variance, so the mean over N_K modes is
    # 1 +- 1/sqrt(N_K / 2) (pairs +-k are equal).  5 sigma band, fixed seed.
    N, L = 4000, 63.0
    pos = I.positions(N, 2, L, np.float64, seed=21)
    modes = _modes_ball(2, 20.0)
    S = O.structure_factor(pos, L, modes)
    half = len(modes) / 2
    assert abs(S.mean() - 1.0) < 5.0 / math.sqrt(half)


def test_finite_differences_match_gradient():
    # Central differences of the loss (computed without cancellation) agree with the
    # analytic gradient of Eq. (gradient) to O(h^2).
    rng = np.random.default_rng(13)
    N, L = 300, np.array([9.0, 11.0, 10.0])
    pos = rng.uniform(0, 1, (N, 3)) * L
    modes = _modes_ball(3, 4.0)
    W = rng.uniform(0.2, 1.0, len(modes))
    S0 = rng.uniform(0.0, 1.5, len(modes))
    g = O.loss_grad(pos, L, modes, W, S0)["grad"]
    coords = [(int(j), int(a)) for j, a in zip(rng.integers(0, N, 24), rng.integers(0, 3, 24))]
    fd = O.finite_difference(pos, L, modes, W, S0, coords, 1e-4)
    ref = np.array([g[j, a] for j, a in coords])
    np.testing.assert_allclose(fd, ref, rtol=1e-6, atol=1e-7 * np.abs(g).max())


def test_gradient_subset_matches_full():
    rng = np.random.default_rng(17)
    N, L = 120, 6.0
    pos = rng.uniform(0, L, (N, 2))
    modes = _modes_ball(2, 4.0)
    W = np.ones(len(modes))
    full = O.loss_grad(pos, L, modes, W, np.zeros(len(modes)))["grad"]
    idx = np.array([5, 77, 0, 119])
    sub = O.loss_grad(pos, L, modes, W, np.zeros(len(modes)), grad_points=idx)["grad"]
    np.testing.assert_array_equal(sub, full[idx])


def test_relative_weights():
    # W = w / S0^2 where S0 != 0 and W = w otherwise (Methods, Analytical gradients).
    w = np.array([1.0, 2.0, 3.0])
    S0 = np.array([0.0, 0.5, 2.0])
    np.testing.assert_allclose(O.effective_weights(w, S0, True), [1.0, 8.0, 0.75])
    np.testing.assert_allclose(O.effective_weights(w, S0, False), w)


def _lattice_count(d, K):
    """Number of integer vectors with 0 < |n| <= K, by exact lattice counting."""
    K2 = K * K
    R = int(math.floor(K))
    if d == 2:
        nx = np.arange(-R, R + 1, dtype=np.int64)
        rem = K2 - nx * nx
        cnt = 2 * np.floor(np.sqrt(rem)).astype(np.int64) + 1
        # guard the floor of sqrt against rounding
        for i in range(len(cnt)):
            m = (cnt[i] - 1) // 2
            while (m + 1) ** 2 <= rem[i]:
                m += 1
            while m * m > rem[i]:
                m -= 1
            cnt[i] = 2 * m + 1
        return int(cnt.sum()) - 1
    total = 0
    for nz in range(-R, R + 1):
        total += _lattice_count(2, math.sqrt(K2 - nz * nz)) + 1
    return total - 1


def test_stealthy_target_counts_modes_inclusively():
    # The stealthy target marks every mode 0 < |n| <= K (both n and -n).
    for d, K in [(2, 16.0), (2, 7.5), (3, 5.0)]:
        w, S0 = I.stealthy_target(d, int(K), K)
        assert int(w.sum()) == _lattice_count(d, K)
        assert np.all(S0 == 0)
    # the paper's small case (0 < |n| <= 16, 2D) holds 796 modes
    assert _lattice_count(2, 16.0) == 796


def test_chi_K_printed_values():
    # chi = N_K / (2 d N) ~= 0.4 with N_K counting all nonzero modes |n| <= K
    # (Methods, Algorithm parameters); the paper prints the resulting K for three
    # systems (tests/golden/chi_K.txt).  The counting convention must reproduce
    # chi = 0.4 at those K to within the rounding of the printed K.
    rows = [l.split() for l in open(os.path.join(GOLDEN, "chi_K.txt"))
            if l.strip() and not l.startswith("#")]
    assert len(rows) == 3
    for r in rows:
        d, N, K = int(r[0]), int(r[1]), float(r[2])
        chi = _lattice_count(d, K) / (2.0 * d * N)
        # a 1% band covers the rounding of K to an integer (dchi/chi = d dK/K)
        assert abs(chi - 0.4) < 0.004 + 0.4 * d * 0.5 / K, (d, N, K, chi)


def test_lbfgs_oracle_on_a_quadratic():
    # On a convex quadratic f = x.A x / 2 - b.x, L-BFGS with an exact-enough line
    # search converges to A^-1 b; the first step is the clamped steepest-descent
    # step accepted by the Armijo test.
    from oracle import lbfgs as LB
    rng = np.random.default_rng(2)
    n = 12
    Q = rng.normal(size=(n, n))
    A = Q @ Q.T + n * np.eye(n)
    b = rng.normal(size=n)

    def fg(x):
        return 0.5 * x @ A @ x - b @ x, A @ x - b

    x0 = np.zeros(n)
    r = LB.run(fg, x0, 1, m=5, max_step=1e-3)
    g0 = -b
    p = -g0
    alpha = 1e-3 / np.max(np.abs(p))
    np.testing.assert_allclose(r["xs"][1], x0 + alpha * p, rtol=1e-14)
    r = LB.run(fg, x0, 200, m=5, max_step=10.0, gtol=1e-9)
    np.testing.assert_allclose(r["x"], np.linalg.solve(A, b), rtol=1e-7, atol=1e-9)
    assert all(f2 <= f1 for f1, f2 in zip(r["fs"], r["fs"][1:]))


def _random_pairs(n, m, seed):
    """m curvature pairs (s, y = A s) of a random SPD matrix A, so y.s > 0."""
    rng = np.random.default_rng(seed)
    Q = rng.normal(size=(n, n))
    A = Q @ Q.T + 0.5 * np.eye(n)
    S = [rng.normal(size=n) for _ in range(m)]
    Y = [A @ s for s in S]
    R = [1.0 / float(y @ s) for s, y in zip(S, Y)]
    return S, Y, R, rng


def _dense_inverse_hessian(S, Y, gamma):
    """BFGS inverse-Hessian update applied to gamma I, oldest pair first:
    H <- V^T H V + rho s s^T with V = I - rho y s^T (Nocedal & Wright, Eq. 6.17)."""
    n = S[0].size
    H = gamma * np.eye(n)
    for s, y in zip(S, Y):
        rho = 1.0 / float(y @ s)
        V = np.eye(n) - rho * np.outer(y, s)
        H = V.T @ H @ V + rho * np.outer(s, s)
    return H


@pytest.mark.parametrize("m", [1, 2, 5, 8])
def test_lbfgs_two_loop_is_the_dense_bfgs_update(m):
    # the two-loop recursion computes H g for H built by m BFGS updates of
    # gamma I, taken oldest to newest; reversing either loop's order, dropping
    # the gamma scaling or a rho factor changes H g far beyond rounding
    from oracle import lbfgs as LB
    n = 10
    S, Y, R, rng = _random_pairs(n, m, seed=30 + m)
    gamma = float(S[-1] @ Y[-1]) / float(Y[-1] @ Y[-1])
    H = _dense_inverse_hessian(S, Y, gamma)
    for _ in range(4):
        g = rng.normal(size=n)
        ref = H @ g
        got = LB.two_loop(g, S, Y, R, gamma)
        assert np.linalg.norm(got - ref) <= 1e-12 * np.linalg.norm(ref)
    # secant condition of the newest pair: H y = s
    hy = LB.two_loop(Y[-1], S, Y, R, gamma)
    assert np.linalg.norm(hy - S[-1]) <= 1e-12 * np.linalg.norm(S[-1])
    # symmetric positive definite, as every BFGS inverse Hessian with y.s > 0
    u, v = rng.normal(size=n), rng.normal(size=n)
    assert abs(u @ LB.two_loop(v, S, Y, R, gamma) - v @ LB.two_loop(u, S, Y, R, gamma)) \
        <= 1e-12 * np.linalg.norm(H, 2) * np.linalg.norm(u) * np.linalg.norm(v)
    assert np.all(np.linalg.eigvalsh(0.5 * (H + H.T)) > 0)
    # no pairs: steepest descent
    g = rng.normal(size=n)
    assert np.array_equal(LB.two_loop(g, [], [], [], 1.0), g)


def test_lbfgs_run_keeps_the_newest_pairs():
    # every direction of run() uses the last min(k, m) steps s = x_{k+1} - x_k
    # and gradient changes y, oldest first, with gamma = s.y / y.y of the newest
    from oracle import lbfgs as LB
    rng = np.random.default_rng(12)
    n, m = 8, 3
    Q = rng.normal(size=(n, n))
    A = Q @ Q.T + n * np.eye(n)
    b = rng.normal(size=n)

    def fg(x):
        # a convex quartic, so the curvature pairs change from step to step
        return 0.5 * x @ A @ x - b @ x + 0.25 * np.sum(x ** 4), A @ x - b + x ** 3

    seen = []

    def spy(g, S, Y, R, gamma):
        seen.append(([s.copy() for s in S], [y.copy() for y in Y], list(R), gamma, g.copy()))
        return LB.two_loop(g, S, Y, R, gamma)

    r = LB.run(fg, np.zeros(n), 7, m=m, max_step=0.3, direction=spy)
    xs = r["xs"]
    assert len(seen) == 7
    for k, (S, Y, R, gamma, g) in enumerate(seen):
        steps = [xs[i + 1] - xs[i] for i in range(k + 1)]
        grads = [fg(x)[1] for x in xs[:k + 2]]
        ys = [grads[i + 1] - grads[i] for i in range(k + 1)]
        keep = min(k + 1, m)
        assert len(S) == keep
        for j in range(keep):
            np.testing.assert_allclose(S[j], steps[k + 1 - keep + j], rtol=1e-12, atol=1e-15)
            np.testing.assert_allclose(Y[j], ys[k + 1 - keep + j], rtol=1e-12, atol=1e-14)
            assert R[j] == pytest.approx(1.0 / float(S[j] @ Y[j]), rel=1e-14)
        assert gamma == pytest.approx(float(S[-1] @ Y[-1]) / float(Y[-1] @ Y[-1]), rel=1e-14)
        np.testing.assert_allclose(g, grads[k + 1], rtol=1e-12, atol=1e-14)


def test_lbfgs_oracle_decreases_structure_factor_loss():
    from oracle import lbfgs as LB
    N, L, M = 64, 8.0, 3
    pos = I.positions(N, 2, L, np.float64, seed=4)
    modes = _modes_ball(2, 3.0)
    W = np.ones(len(modes))
    S0 = np.zeros(len(modes))

    def fg(x):
        r = O.loss_grad(x.reshape(N, 2), L, modes, W, S0)
        return r["loss"], r["grad"].ravel()

    r = LB.run(fg, pos, 10, m=8, max_step=0.1 * L / np.sqrt(N))
    assert r["fs"][-1] < 0.5 * r["fs"][0]
    assert all(f2 <= f1 for f1, f2 in zip(r["fs"], r["fs"][1:]))


# ------------------------------------------------------------------ backward of S
def test_sf_vjp_two_points_closed_form():
    # N = 2: S(k) = 1 + cos(k.D), so dS/dr1 = -sin(k.D) k and dS/dr2 = +sin(k.D) k;
    # the backward of S for weights g is sum_k g(k) dS(k)/dr.
    rng = np.random.default_rng(21)
    L = np.array([4.0, 6.5, 5.0])
    pos = rng.uniform(0, 1, (2, 3)) * L
    modes = _modes_ball(3, 3.0)
    k = 2 * np.pi * modes / L
    g = rng.normal(size=len(modes))
    D = pos[0] - pos[1]
    g1 = -np.sum((g * np.sin(k @ D))[:, None] * k, axis=0)
    out = O.sf_vjp(pos, L, modes, g)
    np.testing.assert_allclose(out[0], g1, rtol=1e-12, atol=1e-12)
    np.testing.assert_allclose(out[1], -g1, rtol=1e-12, atol=1e-12)


def test_sf_vjp_matches_finite_differences_of_S():
    # Central differences of F = sum_k g(k) S(k), S from the direct sum, along
    # single coordinates (FP64, h = 1e-5: truncation ~1e-10 relative).
    rng = np.random.default_rng(22)
    N, L = 40, 6.0
    pos = rng.uniform(0, L, (N, 2))
    modes = _modes_ball(2, 5.0, include_zero=True)
    g = rng.normal(size=len(modes))
    out = O.sf_vjp(pos, L, modes, g)
    h = 1e-5
    for j, a in [(0, 0), (3, 1), (17, 0), (39, 1)]:
        pp, pm = pos.copy(), pos.copy()
        pp[j, a] += h
        pm[j, a] -= h
        fd = (g @ O.structure_factor(pp, L, modes) - g @ O.structure_factor(pm, L, modes)) / (2 * h)
        assert out[j, a] == pytest.approx(fd, rel=1e-7, abs=1e-8)


def test_sf_vjp_of_loss_weights_is_loss_gradient():
    # With g = dL/dS = 2 W (S - S0) the backward of S is the loss gradient of
    # Eq. (gradient); the sum rule sum_j grad_j = 0 holds for any g.
    rng = np.random.default_rng(23)
    N, L = 50, 7.0
    pos = rng.uniform(0, L, (N, 2))
    modes = _modes_ball(2, 4.0)
    W = rng.uniform(0.5, 2, len(modes))
    S0 = rng.uniform(0, 1, len(modes))
    r = O.loss_grad(pos, L, modes, W, S0)
    out = O.sf_vjp(pos, L, modes, 2 * W * (r["S"] - S0))
    np.testing.assert_allclose(out, r["grad"], rtol=1e-10, atol=1e-10)
    g = rng.normal(size=len(modes))
    assert np.abs(O.sf_vjp(pos, L, modes, g).sum(0)).max() < 1e-9


# ------------------------------------------------------------- soft-core pair term
@pytest.mark.parametrize("alpha", [2.0, 2.5])
def test_pair_two_particles_closed_form(alpha):
    # Two particles closer than sigma, placed across the periodic boundary so that
    # only the minimum image is in range: E = (eps/alpha)(1 - r/sigma)^alpha and
    # |dE/dr| = (eps/sigma)(1 - r/sigma)^(alpha-1), pushing the particles apart.
    L, sigma, eps = np.array([5.0, 4.0, 6.0]), 0.5, 1.3
    r = 0.3
    u = np.array([0.6, 0.0, 0.8])
    p1 = np.array([0.05, 2.0, 5.98])
    p2 = p1 - r * u
    p2 = p2 - L * np.floor(p2 / L)  # stored wrapped on the far side of the box
    e, g = O.pair(np.stack([p1, p2]), L, sigma, eps, alpha)
    x = 1 - r / sigma
    assert e == pytest.approx(eps / alpha * x ** alpha, rel=1e-13)
    np.testing.assert_allclose(g[0], -(eps / sigma) * x ** (alpha - 1) * u, rtol=1e-12, atol=1e-14)
    np.testing.assert_allclose(g[1], -g[0], rtol=1e-12, atol=1e-14)
    # out of range: nothing
    e2, g2 = O.pair(np.stack([p1, p1 + np.array([0.0, 0.51, 0.0])]), L, sigma, eps, alpha)
    assert e2 == 0.0 and np.all(g2 == 0.0)


def test_pair_square_lattice_energy():
    # Square lattice of spacing a < sigma < a sqrt(2): every particle has four
    # partners at distance a, so E = N * 4 / 2 * U(a), and by symmetry no force.
    m, a, sigma = 12, 0.4, 0.5
    x = np.arange(m) * a
    pos = np.stack(np.meshgrid(x, x, indexing="ij"), -1).reshape(-1, 2) + 0.013
    e, g = O.pair(pos, m * a, sigma)
    assert e == pytest.approx(m * m * 2 * 0.5 * (1 - a / sigma) ** 2, rel=1e-12)
    assert np.abs(g).max() < 1e-12


@pytest.mark.parametrize("d,L", [(2, 9.0), (3, 6.0), (3, (1.2, 5.0, 1.7))])
def test_pair_cells_equal_brute_force_and_newton(d, L):
    # The cell list (including boxes only two cells wide) finds exactly the pairs
    # of the brute force; Newton's third law makes the forces sum to zero.
    rng = np.random.default_rng(31 + d)
    Lv = np.broadcast_to(np.asarray(L, float), (d,))
    N = int(np.prod(Lv) * 3)
    pos = rng.uniform(-1, 2, (N, d)) * Lv  # unwrapped coordinates are allowed
    e1, g1 = O.pair(pos, Lv, 0.5, 1.0, 2.0)
    e2, g2 = O.pair(pos, Lv, 0.5, 1.0, 2.0, cells=True)
    assert e1 > 0
    assert e2 == pytest.approx(e1, rel=1e-12)
    np.testing.assert_allclose(g2, g1, rtol=1e-12, atol=1e-13)
    assert np.abs(g1.sum(0)).max() < 1e-10


def test_pair_gradient_matches_finite_differences():
    # Central differences of the brute-force energy (FP64, h = 1e-6).
    rng = np.random.default_rng(41)
    L = 4.0
    pos = rng.uniform(0, L, (80, 3))
    _, g = O.pair(pos, L, 0.5, 1.0, 2.5)
    h = 1e-6
    checked = 0
    for j in range(80):
        if np.abs(g[j]).max() == 0:
            continue
        for a in range(3):
            pp, pm = pos.copy(), pos.copy()
            pp[j, a] += h
            pm[j, a] -= h
            fd = (O.pair(pp, L, 0.5, 1.0, 2.5)[0] - O.pair(pm, L, 0.5, 1.0, 2.5)[0]) / (2 * h)
            assert g[j, a] == pytest.approx(fd, rel=1e-6, abs=1e-8)
        checked += 1
        if checked == 6:
            break
    assert checked == 6


@pytest.mark.parametrize("alpha", [2.0, 2.5])
def test_pair_finite_difference_equals_energy_differences(alpha):
    # The per-coordinate pair difference (only the moved point's pairs) equals the
    # difference of the whole brute-force energies, and the two-particle closed
    # form: (U(r+) - U(r-)) / 2h along the pair axis for two isolated particles.
    rng = np.random.default_rng(43)
    L = np.array([4.0, 5.0, 3.5])
    pos = rng.uniform(0, 1, (90, 3)) * L
    h = 1e-4
    coords = [(j, a) for j in range(0, 90, 7) for a in range(3)]
    got = O.pair_finite_difference(pos, L, coords, h, 0.5, 1.2, alpha)
    ref = []
    for j, a in coords:
        pp, pm = pos.copy(), pos.copy()
        pp[j, a] += h
        pm[j, a] -= h
        ref.append((O.pair(pp, L, 0.5, 1.2, alpha)[0] - O.pair(pm, L, 0.5, 1.2, alpha)[0]) / (2 * h))
    ref = np.array(ref)
    assert np.abs(ref).max() > 0
    np.testing.assert_allclose(got, ref, rtol=1e-8, atol=1e-9)
    two = np.array([[1.0, 1.0, 1.0], [1.3, 1.0, 1.0]])
    r = 0.3
    x = lambda rr: 1 - rr / 0.5
    closed = (1.2 / alpha) * (x(r - h) ** alpha - x(r + h) ** alpha) / (2 * h)
    assert O.pair_finite_difference(two, L, [(0, 0)], h, 0.5, 1.2, alpha)[0] == \
        pytest.approx(closed, rel=1e-12)


def test_rho_direct_lattice_and_table_form():
    # The direct-evaluation form (used for a few modes over very many points) on a
    # 16 x 16 lattice: |rho| = N exactly on the Bragg peak (16, 0), 0 off it; and it
    # agrees with the table form on random points.
    pos = I.square_lattice(16, 32.0, 2, shift=(0.3, 1.7))
    r = O.rho_direct(pos, 32.0, np.array([[16, 0], [5, 3], [0, 16]], np.int32), chunk=100)
    assert abs(abs(r[0]) - 256.0) < 1e-10 and abs(r[1]) < 1e-10 and abs(abs(r[2]) - 256.0) < 1e-10
    rng = np.random.default_rng(2)
    p = rng.uniform(-5, 15, (2000, 3))
    m = rng.integers(-9, 10, (7, 3)).astype(np.int32)
    np.testing.assert_allclose(O.rho_direct(p, (10.0, 12.0, 9.0), m, chunk=333),
                               O.rho(p, (10.0, 12.0, 9.0), m), rtol=1e-12, atol=1e-11)


def test_loss_grad_from_rho_matches_direct_sums():
    # Given the direct-evaluation rho, the loss, S and gradient equal those of the
    # table-based oracle (both evaluate Eq. gradient; this pins the rho hand-over and
    # the 1/N factors of the large-problem path).
    rng = np.random.default_rng(3)
    N, L = 500, 9.0
    pos = rng.uniform(0, L, (N, 2))
    modes = _modes_ball(2, 4.0)
    W = rng.uniform(0.5, 2, len(modes))
    S0 = rng.uniform(0, 1, len(modes))
    ref = O.loss_grad(pos, L, modes, W, S0)
    gp = [3, 77, 400]
    r = O.loss_grad_from_rho(N, L, modes, W, S0, O.rho_direct(pos, L, modes), pos[gp])
    assert r["loss"] == pytest.approx(ref["loss"], rel=1e-12)
    np.testing.assert_allclose(r["S"], ref["S"], rtol=1e-12, atol=1e-13)
    np.testing.assert_allclose(r["grad"], ref["grad"][gp], rtol=1e-11, atol=1e-12)


# ------------------------------------------------------------ point strengths
def _strength_case(N=60, d=2, L=9.0, M=4, seed=90, signed=False):
    rng = np.random.default_rng(seed)
    pos = rng.uniform(0, L, (N, d))
    c = rng.lognormal(0.0, 0.4, N)
    if signed:
        c *= rng.choice([-1.0, 1.0], N)
    modes = _modes_ball(d, float(M))
    W = rng.uniform(0.5, 1.5, len(modes))
    S0 = rng.uniform(0.0, 2.0, len(modes))
    return pos, c, L, modes, W, S0


def test_strengths_unit_reduce_to_plain_loss():
    # c = 1: rho0 = N and every quantity is the plain one
    pos, _, L, modes, W, S0 = _strength_case()
    c = np.ones(len(pos))
    a = O.loss_grad_strengths(pos, c, L, modes, W, S0)
    b = O.loss_grad(pos, L, modes, W, S0)
    np.testing.assert_allclose(a["S"], b["S"], rtol=1e-13)
    assert a["loss"] == pytest.approx(b["loss"], rel=1e-13)
    np.testing.assert_allclose(a["grad"], b["grad"], rtol=1e-12, atol=1e-13)


def test_strengths_rho_is_linear_in_the_strengths():
    # two points at one position act as one point carrying the sum of their
    # strengths; rho(0) = sum c
    rng = np.random.default_rng(91)
    L = 7.0
    r = rng.uniform(0, L, (3, 2))
    modes = np.array([[0, 0], [1, 0], [2, -3], [-1, 4]])
    a, b, e = 0.7, -1.9, 1.3
    split = O.rho_strengths(np.stack([r[0], r[0], r[1]]), [a, b, e], L, modes)
    merged = O.rho_strengths(np.stack([r[0], r[1]]), [a + b, e], L, modes)
    np.testing.assert_allclose(split, merged, rtol=1e-13, atol=1e-14)
    assert split[0] == pytest.approx(a + b + e, rel=1e-14)


@pytest.mark.parametrize("signed", [False, True])
def test_strengths_scale_invariance(signed):
    # S, L and dL/dr do not change under c -> lambda c; dL/dc scales as 1/lambda
    pos, c, L, modes, W, S0 = _strength_case(signed=signed)
    a = O.loss_grad_strengths(pos, c, L, modes, W, S0)
    b = O.loss_grad_strengths(pos, 3.5 * c, L, modes, W, S0)
    np.testing.assert_allclose(b["S"], a["S"], rtol=1e-12)
    assert b["loss"] == pytest.approx(a["loss"], rel=1e-12)
    np.testing.assert_allclose(b["grad"], a["grad"], rtol=1e-11, atol=1e-12)
    np.testing.assert_allclose(3.5 * b["grad_c"], a["grad_c"], rtol=1e-11, atol=1e-12)


@pytest.mark.parametrize("signed", [False, True])
def test_strengths_euler_identity_and_sum_rule(signed):
    # L(lambda c) = L(c) for every lambda, so sum_j c_j dL/dc_j = 0; translation
    # invariance gives sum_j dL/dr_j = 0
    pos, c, L, modes, W, S0 = _strength_case(signed=signed)
    r = O.loss_grad_strengths(pos, c, L, modes, W, S0)
    terms = c * r["grad_c"]
    assert abs(terms.sum()) <= 1e-12 * np.abs(terms).sum()
    assert np.abs(r["grad"].sum(0)).max() <= 1e-12 * np.abs(r["grad"]).sum()


def test_strengths_two_points_closed_form():
    # N = 2: S(k) = 1 + 2 c1 c2 cos(k.D) / rho0 with D = r1 - r2, rho0 = c1^2 + c2^2;
    # dS/dr1 = -2 c1 c2 sin(k.D) k / rho0; dS/dc1 = 2 c2 cos(k.D) / rho0 - 4 c1^2 c2 cos(k.D) / rho0^2
    rng = np.random.default_rng(92)
    L = np.array([5.0, 6.5, 4.0])
    pos = rng.uniform(0, 1, (2, 3)) * L
    c1, c2 = 1.7, -0.6
    modes = _modes_ball(3, 2.5)
    k = 2 * np.pi * modes / L
    W = rng.uniform(0.5, 1.5, len(modes))
    S0 = rng.uniform(0.0, 2.0, len(modes))
    rho0 = c1 * c1 + c2 * c2
    th = k @ (pos[0] - pos[1])
    S = 1 + 2 * c1 * c2 * np.cos(th) / rho0
    G = 2 * W * (S - S0)
    g1 = np.sum((G * (-2 * c1 * c2 * np.sin(th) / rho0))[:, None] * k, axis=0)
    gc1 = np.sum(G * (2 * c2 * np.cos(th) / rho0 - 4 * c1 * c1 * c2 * np.cos(th) / rho0 ** 2))
    gc2 = np.sum(G * (2 * c1 * np.cos(th) / rho0 - 4 * c2 * c2 * c1 * np.cos(th) / rho0 ** 2))
    r = O.loss_grad_strengths(pos, [c1, c2], L, modes, W, S0)
    np.testing.assert_allclose(r["S"], S, rtol=1e-13, atol=1e-14)
    assert r["loss"] == pytest.approx(np.sum(W * (S - S0) ** 2), rel=1e-13)
    np.testing.assert_allclose(r["grad"][0], g1, rtol=1e-12, atol=1e-13)
    np.testing.assert_allclose(r["grad"][1], -g1, rtol=1e-12, atol=1e-13)
    np.testing.assert_allclose(r["grad_c"], [gc1, gc2], rtol=1e-12, atol=1e-13)


@pytest.mark.parametrize("signed", [False, True])
def test_strengths_finite_differences(signed):
    # the analytic gradients against the cancellation-free differences, and those
    # against plain differences of whole losses
    pos, c, L, modes, W, S0 = _strength_case(N=40, d=3, L=5.0, M=3, seed=93, signed=signed)
    r = O.loss_grad_strengths(pos, c, L, modes, W, S0)
    d = pos.shape[1]
    coords = [(j, a) for j in (0, 7, 19, 33) for a in range(d + 1)]
    h = 1e-5
    fd = O.finite_difference_strengths(pos, c, L, modes, W, S0, coords, h)
    ana = np.array([r["grad"][j, a] if a < d else r["grad_c"][j] for j, a in coords])
    np.testing.assert_allclose(fd, ana, rtol=1e-7, atol=1e-9 * np.abs(ana).max())
    hh = 1e-4
    for (j, a), f in zip(coords[:6], O.finite_difference_strengths(pos, c, L, modes, W, S0,
                                                                   coords[:6], hh)):
        pp, pm, cp, cm = pos.copy(), pos.copy(), c.copy(), c.copy()
        if a < d:
            pp[j, a] += hh
            pm[j, a] -= hh
        else:
            cp[j] += hh
            cm[j] -= hh
        plain = (O.loss_grad_strengths(pp, cp, L, modes, W, S0, want_grad=False)["loss"] -
                 O.loss_grad_strengths(pm, cm, L, modes, W, S0, want_grad=False)["loss"]) / (2 * hh)
        assert f == pytest.approx(plain, rel=1e-6, abs=1e-9)


# ------------------------------------------------------- pair correlation loss
def _dirichlet(y, M, L):
    """sum_{|n| <= M} exp(2 pi i n y / L) = sin((2M+1) pi y / L) / sin(pi y / L)."""
    t = np.pi * np.asarray(y, dtype=np.float64) / L
    s = np.sin(t)
    out = np.empty_like(t)
    small = np.abs(s) < 1e-12
    out[~small] = np.sin((2 * M + 1) * t[~small]) / s[~small]
    out[small] = (2 * M + 1) * np.cos((2 * M + 1) * t[small]) / np.cos(t[small])
    return out


def test_pair_correlation_equals_pair_sum_with_dirichlet_kernel():
    # g(x) = (1/N^2) sum_{i != j} prod_a D_{M_a}((r_i - r_j - x)_a): the pair-sum
    # definition of g truncated to the mode cube, evaluated without S
    rng = np.random.default_rng(101)
    N, L, M = 40, np.array([7.0, 9.0]), (5, 4)
    pos = rng.uniform(0, 1, (N, 2)) * L
    xs = rng.uniform(-1, 1, (20, 2)) * L
    g = O.pair_correlation(pos, L, M, xs)
    ref = np.zeros(len(xs))
    for q, x in enumerate(xs):
        for i in range(N):
            y = pos[i] - pos - x
            term = _dirichlet(y[:, 0], M[0], L[0]) * _dirichlet(y[:, 1], M[1], L[1])
            ref[q] += term.sum() - term[i]
    ref /= N * N
    np.testing.assert_allclose(g, ref, rtol=1e-10, atol=1e-12)


def test_pair_correlation_grid_mean():
    # on a grid of P_a >= 2 M_a + 1 points per axis every mode but n = 0 averages
    # to zero, so the mean of g is (S(0) - 1) / N = 1 - 1/N for any points
    rng = np.random.default_rng(102)
    N, L, M = 30, np.array([5.0, 6.0, 4.0]), (3, 2, 3)
    pos = rng.uniform(0, 1, (N, 3)) * L
    P = (8, 5, 9)
    grids = np.meshgrid(*[np.arange(p) * l / p for p, l in zip(P, L)], indexing="ij")
    xs = np.stack([gg.ravel() for gg in grids], 1)
    g = O.pair_correlation(pos, L, M, xs)
    assert g.mean() == pytest.approx(1 - 1 / N, rel=1e-12)
    # and g is even: g(-x) = g(x)
    np.testing.assert_allclose(O.pair_correlation(pos, L, M, -xs), g, rtol=1e-12, atol=1e-13)


def test_pair_correlation_loss_gradient_finite_differences():
    rng = np.random.default_rng(103)
    N, L, M = 25, 6.0, 4
    pos = rng.uniform(0, L, (N, 2))
    P = 12
    gx = np.arange(P) * L / P
    xs = np.stack(np.meshgrid(gx, gx, indexing="ij"), -1).reshape(-1, 2)
    r2 = np.sum(np.minimum(xs, L - xs) ** 2, 1)
    g0 = (r2 > 1.0).astype(float)  # an exclusion target
    wg = np.where(r2 < 2.5, 1.0, 0.2)
    r = O.pair_correlation_loss_grad(pos, L, M, xs, wg, g0)
    assert r["loss"] == pytest.approx(np.sum(wg * (O.pair_correlation(pos, L, M, xs) - g0) ** 2),
                                      rel=1e-13)
    h = 1e-5
    for j, a in [(0, 0), (3, 1), (11, 0), (24, 1)]:
        pp, pm = pos.copy(), pos.copy()
        pp[j, a] += h
        pm[j, a] -= h
        fd = (O.pair_correlation_loss_grad(pp, L, M, xs, wg, g0)["loss"] -
              O.pair_correlation_loss_grad(pm, L, M, xs, wg, g0)["loss"]) / (2 * h)
        assert r["grad"][j, a] == pytest.approx(fd, rel=1e-6, abs=1e-9)


# -------------------------------------------- non-uniform wave vectors (NUwNU)
def test_rho_q_equals_the_periodic_oracle_on_lattice_vectors():
    # at q = 2 pi n / L the free-boundary direct sum is the periodic one
    rng = np.random.default_rng(111)
    L = np.array([6.0, 8.5])
    pos = rng.uniform(0, 1, (70, 2)) * L
    modes = _modes_ball(2, 3.0)
    q = 2 * np.pi * modes / L
    np.testing.assert_allclose(O.rho_q(pos, q), O.rho(pos, L, modes), rtol=1e-12, atol=1e-11)


@pytest.mark.parametrize("d", [2, 3])
def test_peak_echo_on_a_sheared_lattice(d):
    # points on a lattice whose dual basis is the constrained set {k_j}, cut to a
    # ball (free boundary): S(k_j) = N, and every integer combination of the k_j
    # is a peak S = N too (SI, saturating peaks and echoes); other q are not
    rng = np.random.default_rng(112 + d)
    K = rng.normal(size=(d, d)) + 2 * np.eye(d)       # rows: k_1 .. k_d
    A = 2 * np.pi * np.linalg.inv(K).T                 # rows a_i with a_i . k_j = 2 pi delta_ij
    m = np.stack(np.meshgrid(*[np.arange(-9, 10)] * d, indexing="ij"), -1).reshape(-1, d)
    pos = m @ A + rng.normal(size=d)
    pos = pos[np.linalg.norm(pos - pos.mean(0), axis=1) < 6.0 * np.abs(A).max()]
    N = len(pos)
    combos = [np.eye(d)[0], np.eye(d)[-1], 2 * np.eye(d)[0] - 3 * np.eye(d)[-1]]
    q = np.array([c @ K for c in combos])
    np.testing.assert_allclose(O.structure_factor_q(pos, q), N, rtol=1e-10)
    assert O.structure_factor_q(pos, 0.5 * K[:1])[0] < 0.9 * N


def test_structure_factor_q_translation_and_friedel():
    rng = np.random.default_rng(114)
    pos = rng.uniform(-3, 5, (60, 3))
    q = rng.normal(size=(15, 3)) * 2.0
    S = O.structure_factor_q(pos, q)
    np.testing.assert_allclose(O.structure_factor_q(pos + rng.normal(size=3) * 7, q), S,
                               rtol=1e-10, atol=1e-12)
    np.testing.assert_allclose(O.structure_factor_q(pos, -q), S, rtol=1e-12, atol=1e-13)


def test_loss_grad_q_finite_differences_and_sum_rule():
    rng = np.random.default_rng(115)
    pos = rng.uniform(0, 6, (30, 2))
    c = rng.lognormal(0, 0.3, 30)
    q = rng.normal(size=(12, 2)) * 2.0
    W = rng.uniform(0.5, 1.5, 12)
    S0 = rng.uniform(0, 2, 12)
    for cc in (None, c):
        r = O.loss_grad_q(pos, q, W, S0, cc)
        assert np.abs(r["grad"].sum(0)).max() <= 1e-12 * np.abs(r["grad"]).sum()
        h = 1e-5
        for j, a in [(0, 0), (7, 1), (29, 0)]:
            pp, pm = pos.copy(), pos.copy()
            pp[j, a] += h
            pm[j, a] -= h
            fd = (O.loss_grad_q(pp, q, W, S0, cc, want_grad=False)["loss"] -
                  O.loss_grad_q(pm, q, W, S0, cc, want_grad=False)["loss"]) / (2 * h)
            assert r["grad"][j, a] == pytest.approx(fd, rel=1e-6, abs=1e-9)


@pytest.mark.parametrize("d,ns", [(2, 360), (3, 2000)])
def test_ewald_transmission_edges(d, ns):
    # a structure factor that vanishes inside |q| < K (stealthy) and is 1 outside:
    # below k_b = K/2 the whole circle (sphere) stays inside, T is the forward
    # fraction of the quadrature; above k_b the backward directions scatter and
    # forward ones do not, T = 0, until k_f = K/sqrt 2 where forward scattering
    # sets in (main text, Fig. ewald)
    Kc = 3.0
    eps = 1e-30

    def S_of_q(q):
        return np.where(np.linalg.norm(q, axis=1) >= Kc, 1.0, eps)

    e = np.zeros(d)
    e[0] = 0.6
    e[1] = 0.8
    es, fwd = O.ewald_directions(d, e, ns)
    np.testing.assert_allclose(np.linalg.norm(es, axis=1), 1.0, rtol=1e-13)
    assert abs(fwd.mean() - 0.5) < 0.01
    assert O.ewald_transmission(S_of_q, d, 0.48 * Kc, e, ns) == pytest.approx(fwd.mean(), rel=1e-12)
    assert O.ewald_transmission(S_of_q, d, 0.52 * Kc, e, ns) < 1e-20
    assert O.ewald_transmission(S_of_q, d, 0.69 * Kc, e, ns) < 1e-20
    assert O.ewald_transmission(S_of_q, d, 0.75 * Kc, e, ns) > 1e-3


def test_uwnu_weight_gradient_pins():
    # weights of the pixels of a uniform grid constrained at arbitrary wave
    # vectors (UwNU): the strength gradient satisfies the Euler identity
    # sum_j c_j dL/dc_j = 0 (S is invariant under c -> lambda c), matches
    # plain differences of the loss, and at lattice vectors of a periodic box
    # equals the periodic oracle's strength gradient
    rng = np.random.default_rng(116)
    m, L = 9, 6.0
    g = (np.arange(m) + 0.5) * L / m
    pos = np.stack(np.meshgrid(g, g, indexing="ij"), -1).reshape(-1, 2)
    c = rng.normal(size=m * m)
    q = rng.normal(size=(14, 2)) * 2.5
    W = rng.uniform(0.5, 1.5, 14)
    S0 = rng.uniform(0, 2, 14)
    gc = O.grad_strengths_q(pos, q, W, S0, c)
    assert abs(np.sum(c * gc)) <= 1e-12 * np.sum(np.abs(c * gc))
    h = 1e-5
    for j in (0, 17, 80):
        cp, cm = c.copy(), c.copy()
        cp[j] += h
        cm[j] -= h
        fd = (O.loss_grad_q(pos, q, W, S0, cp, want_grad=False)["loss"] -
              O.loss_grad_q(pos, q, W, S0, cm, want_grad=False)["loss"]) / (2 * h)
        assert gc[j] == pytest.approx(fd, rel=1e-6, abs=1e-9)
    modes = _modes_ball(2, 2.0)
    ql = 2 * np.pi * modes / L
    Wl = rng.uniform(0.5, 1.5, len(modes))
    S0l = rng.uniform(0, 2, len(modes))
    ref = O.loss_grad_strengths(pos, c, L, modes, Wl, S0l)["grad_c"]
    np.testing.assert_allclose(O.grad_strengths_q(pos, ql, Wl, S0l, c), ref, rtol=1e-10, atol=1e-12)
