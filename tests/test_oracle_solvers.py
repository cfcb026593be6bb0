"""Pins of the oracle's step size, FISTA and 16-bit library (CPU only)."""
import numpy as np
import pytest
import scipy.optimize

from oracle.geometry import paper_like
from oracle import hlib, operators as ops, solvers, quant
from paper_2603_28150_amd import inputs


@pytest.fixture(scope="module")
def micro():
    g = paper_like(8, 8, 4, 16)
    Hh = hlib.H_half(g)
    A = lambda v: ops.A_fft(Hh, v)
    AT = lambda v: ops.AT_fft(Hh, v)
    M = solvers.dense_matrix(A, (g.nz, g.ny, g.nx))
    return g, Hh, A, AT, M


def test_norm_closed_form_equals_dense_spectrum(micro):
    # ||A||^2 from the per-frequency blocks equals the top eigenvalue of the
    # dense normal matrix
    g, Hh, A, AT, M = micro
    L_dense = np.linalg.eigvalsh(M.T @ M)[-1]
    assert abs(solvers.norm_exact(Hh) - L_dense) < 1e-12 * L_dense


def test_power_iteration_increases_to_the_norm(micro):
    g, Hh, A, AT, M = micro
    L = solvers.norm_exact(Hh)
    v0 = inputs.gaussian_random((g.nz, g.ny, g.nx), seed=1002)
    Ls = solvers.power_iteration(A, AT, v0, 200)
    assert all(Ls[i + 1] >= Ls[i] * (1 - 1e-12) for i in range(len(Ls) - 1))
    assert max(Ls) <= L * (1 + 1e-12)
    assert Ls[-1] > 0.99 * L


def test_momentum_weights_closed_form():
    b = solvers.momentum_weights(4)
    t = [1.0]
    for _ in range(4):
        t.append((1 + np.sqrt(1 + 4 * t[-1] ** 2)) / 2)
    assert b[0] == 0.0
    assert np.allclose(b, [(t[k] - 1) / t[k + 1] for k in range(4)], rtol=0, atol=1e-15)
    assert solvers.momentum_weights(3, momentum=False) == [0.0, 0.0, 0.0]


def test_momentum_weights_asymptotics():
    # Beck-Teboulle's sequence makes FISTA the discretisation of
    # x'' + (3/t) x' + grad f = 0 (Su, Boyd and Candes, 2016): 1 - beta_k
    # behaves as 3/k, with a correction of order log(k)/k.  The
    # alternatives beta_k = (t_k - 1)/t_k or (t_{k+1} - 1)/t_{k+1} tend to
    # 2/k, a constant weight does not vanish.
    b = solvers.momentum_weights(100000)
    assert b[0] == 0.0 and all(0.0 <= v < 1.0 for v in b)
    assert all(b[k + 1] > b[k] for k in range(len(b) - 1))
    for k in (1000, 10000, 100000):
        assert abs(k * (1.0 - b[k - 1]) - 3.0) < 20.0 / k ** 0.75


def _worst_case_quadratic(n):
    # Nesterov's hard instance for first-order methods: f(x) = 1/2 ||D x - e_0||^2
    # with D the (n+1) x n first-difference matrix (D^T D tridiagonal 2, -1),
    # minimiser x*_i = 1 - (i+1)/(n+1), ||D||^2 < 4
    D = np.eye(n + 1, n) - np.eye(n + 1, n, k=-1)
    d = np.zeros(n + 1)
    d[0] = 1.0
    xstar = 1.0 - np.arange(1, n + 1) / (n + 1.0)
    return D, d, xstar


def test_fista_rate_on_the_worst_case_quadratic():
    # Beck-Teboulle: F(x_k) - F* <= 2 L ||x_0 - x*||^2 / (k+1)^2 at every k
    # with tau = 1/L; on this instance the unaccelerated method breaks the
    # bound within 400 iterations, so the momentum is what meets it
    D, d, xstar = _worst_case_quadratic(1000)
    A = lambda v: D @ v
    AT = lambda v: D.T @ v
    L = 4.0
    Fstar = 0.5 / (D.shape[0])
    assert abs(solvers.objective(A, d, xstar) - Fstar) < 1e-15
    R2 = float(xstar @ xstar)
    K = 400
    bound = [2.0 * L * R2 / (k + 1) ** 2 for k in range(1, K + 1)]
    acc = solvers.fista(A, AT, d, (D.shape[1],), K, 1.0 / L, 0.0, nonneg=False)
    gap = [solvers.objective(A, d, x) - Fstar for x in acc]
    assert all(gk <= bk for gk, bk in zip(gap, bound))
    assert min(gap) >= -1e-15
    plain = solvers.fista(A, AT, d, (D.shape[1],), K, 1.0 / L, 0.0, nonneg=False, momentum=False)
    assert solvers.objective(A, d, plain[-1]) - Fstar > bound[-1]


def _lbfgsb(fun_grad, n):
    res = scipy.optimize.minimize(fun_grad, np.zeros(n), jac=True, method="L-BFGS-B",
                                  bounds=[(0.0, None)] * n,
                                  options=dict(maxiter=100000, ftol=1e-16, gtol=1e-14, maxcor=50))
    return res.fun, res.x


def test_fista_l1_nonneg_limit_against_lbfgsb(micro):
    # lambda > 0 with non-negativity (eq. 14): on x >= 0 the objective
    # 1/2 ||M x - d||^2 + lambda ||x||_1 is smooth (lambda sum x), so a
    # bound-constrained quasi-Newton solve on the dense matrix gives F*;
    # FISTA's iterates must reach it
    g, Hh, A, AT, M = micro
    x_true = np.abs(inputs.gaussian_blobs((g.nz, g.ny, g.nx), seed=7))
    d = A(x_true) + 0.05 * inputs.noise_like((g.nt, g.ny, g.nx), seed=8)
    db = d.ravel()
    lam = 0.05 * np.abs(M.T @ db).max()

    def fg(x):
        r = M @ x - db
        return 0.5 * r @ r + lam * x.sum(), M.T @ r + lam

    Fstar, xs_ref = _lbfgsb(fg, M.shape[1])
    L = solvers.norm_exact(Hh)
    x = solvers.fista(A, AT, d, (g.nz, g.ny, g.nx), 5000, 1.0 / L, lam, nonneg=True)[-1]
    F = solvers.objective(A, d, x, lam)
    assert x.min() >= 0.0
    assert abs(F - Fstar) <= 1e-9 * Fstar
    # the l1 term is active: some entries are thresholded to zero that the
    # lambda = 0 solution keeps
    assert (xs_ref == 0).sum() > 0 and (x == 0).sum() > 0


def test_fista_soft_threshold_limit_against_lbfgsb(micro):
    # lambda > 0 without the constraint: prox = soft thresholding.  F* from
    # L-BFGS-B on the split x = u - v, u, v >= 0, objective
    # 1/2 ||M (u - v) - d||^2 + lambda sum (u + v)
    g, Hh, A, AT, M = micro
    x_true = inputs.gaussian_random((g.nz, g.ny, g.nx), seed=17)
    d = A(x_true) + 0.05 * inputs.noise_like((g.nt, g.ny, g.nx), seed=18)
    db = d.ravel()
    n = M.shape[1]
    lam = 0.05 * np.abs(M.T @ db).max()

    def fg(uv):
        r = M @ (uv[:n] - uv[n:]) - db
        gr = M.T @ r
        return 0.5 * r @ r + lam * uv.sum(), np.concatenate([gr + lam, -gr + lam])

    Fstar, _ = _lbfgsb(fg, 2 * n)
    L = solvers.norm_exact(Hh)
    x = solvers.fista(A, AT, d, (g.nz, g.ny, g.nx), 5000, 1.0 / L, lam, nonneg=False)[-1]
    assert (x < 0).sum() > 0 and (x > 0).sum() > 0 and (x == 0).sum() > 0
    F = solvers.objective(A, d, x, lam)
    assert abs(F - Fstar) <= 1e-9 * Fstar


def test_first_iterate_closed_form(micro):
    # x_1 = prox(0 - tau * A^T(0 - d)) = max(tau A^T d - tau lambda, 0)
    g, Hh, A, AT, M = micro
    d = inputs.gaussian_random((g.nt, g.ny, g.nx), seed=5)
    tau, lam = 0.3, 0.05
    x1 = solvers.fista(A, AT, d, (g.nz, g.ny, g.nx), 1, tau, lam, nonneg=True)[0]
    assert np.abs(x1 - np.maximum(tau * AT(d) - tau * lam, 0)).max() < 1e-14
    x1s = solvers.fista(A, AT, d, (g.nz, g.ny, g.nx), 1, tau, lam, nonneg=False)[0]
    v = tau * AT(d)
    assert np.abs(x1s - np.sign(v) * np.maximum(np.abs(v) - tau * lam, 0)).max() < 1e-14


def test_unconstrained_gradient_is_landweber(micro):
    # lambda = 0, no constraint, no momentum: x_k = sum_{j<k} (I - tau A^T A)^j tau A^T d
    g, Hh, A, AT, M = micro
    d = inputs.gaussian_random((g.nt, g.ny, g.nx), seed=6)
    tau = 1.0 / solvers.norm_exact(Hh)
    xs = solvers.fista(A, AT, d, (g.nz, g.ny, g.nx), 7, tau, 0.0, nonneg=False, momentum=False)
    N = np.eye(M.shape[1]) - tau * (M.T @ M)
    b = tau * (M.T @ d.ravel())
    acc, term = np.zeros_like(b), b.copy()
    for k in range(7):
        acc = acc + term
        term = N @ term
        assert np.abs(xs[k].ravel() - acc).max() < 1e-12 * np.abs(acc).max()


def test_fista_rate_and_limit_against_nnls(micro):
    # Beck-Teboulle: F(x_k) - F* <= 2 L ||x_0 - x*||^2 / (k+1)^2 with tau = 1/L;
    # F* and x* from scipy's NNLS on the dense matrix
    g, Hh, A, AT, M = micro
    x_true = np.abs(inputs.gaussian_blobs((g.nz, g.ny, g.nx), seed=7))
    d = A(x_true) + 0.05 * inputs.noise_like((g.nt, g.ny, g.nx), seed=8)
    L = solvers.norm_exact(Hh)
    xstar, rnorm = scipy.optimize.nnls(M, d.ravel(), maxiter=20000)
    Fstar = 0.5 * rnorm ** 2
    xs = solvers.fista(A, AT, d, (g.nz, g.ny, g.nx), 3000, 1.0 / L, 0.0, nonneg=True)
    for k in (10, 100, 1000, 3000):
        F = solvers.objective(A, d, xs[k - 1])
        assert F - Fstar <= 2 * L * np.dot(xstar, xstar) / (k + 1) ** 2 + 1e-12 * Fstar
        assert F >= Fstar * (1 - 1e-12)
        assert xs[k - 1].min() >= 0.0
    assert (solvers.objective(A, d, xs[-1]) - Fstar) / Fstar < 1e-6


def test_fista_resume_is_bit_identical(micro):
    g, Hh, A, AT, M = micro
    d = inputs.gaussian_random((g.nt, g.ny, g.nx), seed=9)
    shape = (g.nz, g.ny, g.nx)
    full = solvers.fista(A, AT, d, shape, 12, 0.1, 0.01)
    state = {}

    def rec(k, z, x):
        if k == 5:
            state.update(z=z.copy(), x=x.copy())

    solvers.fista(A, AT, d, shape, 5, 0.1, 0.01, record=rec)
    rest = solvers.fista(A, AT, d, shape, 7, 0.1, 0.01, z0=state["z"],
                         x_prev0=state["x"], k0=5)
    assert np.array_equal(rest[-1], full[-1])


def test_bf16_rounding_matches_torch():
    torch = pytest.importorskip("torch")
    a = np.random.default_rng(0).standard_normal(100000).astype(np.float32) * 10.0 ** np.random.default_rng(1).uniform(-8, 8, 100000).astype(np.float32)
    a[:4] = [1.0, 1.00390625, 1.01171875, -2.00390625]   # exact ties
    mine = quant.round_bf16(a)
    ref = torch.from_numpy(a).to(torch.bfloat16).to(torch.float32).numpy()
    assert np.array_equal(mine, ref)


def test_quantised_library_error_and_scales():
    g = paper_like(32, 32, 16, 64)
    Hh = hlib.H_half(g)
    for kind, u in (("bf16", 2.0 ** -8), ("f16", 2.0 ** -11)):
        Hq, s = quant.quantise(Hh, kind)
        # scales are powers of two that put the per-depth max in [2^(e-1), 2^e]
        e = quant.EXPONENT[kind]
        amax = np.abs(Hh).max(axis=(0, 1, 3)) * s
        assert np.all(amax <= 2.0 ** e) and np.all(amax > 2.0 ** (e - 1))
        assert np.all(np.log2(s) == np.round(np.log2(s)))
        # element-wise relative rounding bound of the 16-bit format
        # (float16 only within its normal range, |H^ s| >= 2^-14)
        normal = np.abs(Hh) * s[None, None, :, None] >= (2.0 ** -14 if kind == "f16" else 1e-30)
        assert np.max(np.abs(Hq - Hh)[normal] / np.abs(Hh)[normal]) <= u * (1 + 1e-6)
        x = inputs.gaussian_blobs((g.nz, g.ny, g.nx), seed=1)
        err = np.linalg.norm(ops.A_fft(Hq, x) - ops.A_fft(Hh, x)) / np.linalg.norm(ops.A_fft(Hh, x))
        assert err < 5e-3
