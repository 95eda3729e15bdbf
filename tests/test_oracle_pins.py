"""Pins of the FP64 CPU oracle against what the paper and the mathematics fix.

Each test ties the oracle (a dense-Cholesky solve of Eq. (1) with the covariance
of Eq. (2)) to something other than itself:
  * h2 = 0 reduces Eq. (2) to a multiple of I, so Eq. (1) is ordinary least
    squares: compared with numpy's SVD-based lstsq;
  * b is invariant to the scale sigma2 of M_j (it cancels in Eq. (1));
  * an exact rational evaluation of Eq. (1) on tiny integer inputs;
  * exact recovery of noise-free data and the equivariance of least squares;
  * the Frisch-Waugh-Lovell identity for the SNP coefficient;
  * h2 = 1 (M = Phi), compared with scipy's Cholesky solve, and the p = 2 case
    in closed form;
  * agreement with the eigendecomposition-based reduction of Section 3
    (Algorithms 1 and 5), itself invariant to the sign and order of eigenpairs.
"""
from fractions import Fraction

import numpy as np
import pytest
import scipy.linalg

import synth


def rel(a, b):
    return np.linalg.norm(np.asarray(a) - np.asarray(b), axis=-1) / np.linalg.norm(np.asarray(b), axis=-1)


@pytest.fixture(scope="module")
def small(oracle_lib):
    return synth.small(96, 5, 12, 4, seed=3)


def test_h2_zero_is_ordinary_least_squares(oracle_lib, small):
    phi, xl, xr, y, _ = small
    h2 = np.zeros(y.shape[0])
    b = oracle_lib.gls_grid(phi, xl, xr, y, h2)
    for i in range(xr.shape[0]):
        x = np.column_stack([xl.T, xr[i].astype(float)])
        ref = np.linalg.lstsq(x, y.T, rcond=None)[0].T        # [t][p]
        assert rel(b[i], ref).max() < 1e-12


@pytest.mark.parametrize("s2", [2.0 ** -10, 4.0, 2.0 ** 8])   # sqrt(s2) is a power of two
def test_sigma2_power_of_two_scaling_is_bitwise_invariant(oracle_lib, small, s2):
    phi, xl, xr, y, h2 = small
    b1 = oracle_lib.gls_grid(phi, xl, xr, y, h2)
    b2 = oracle_lib.gls_grid(phi, xl, xr, y, h2, sigma2=np.full(y.shape[0], s2))
    assert np.array_equal(b1, b2)


@pytest.mark.parametrize("s2", [3.0, 1e3, 0.7, 2.0 ** 9])
def test_sigma2_scaling_is_invariant(oracle_lib, small, s2):
    phi, xl, xr, y, h2 = small
    b1 = oracle_lib.gls_grid(phi, xl, xr, y, h2)
    b2 = oracle_lib.gls_grid(phi, xl, xr, y, h2, sigma2=np.full(y.shape[0], s2))
    assert rel(b2, b1).max() < 1e-12


def _frac_solve(a, rhs):
    """Gauss-Jordan elimination over the rationals: a^{-1} rhs, exactly."""
    n = len(a)
    aug = [list(a[r]) + list(rhs[r]) for r in range(n)]
    for c in range(n):
        piv = next(r for r in range(c, n) if aug[r][c] != 0)
        aug[c], aug[piv] = aug[piv], aug[c]
        pv = aug[c][c]
        aug[c] = [v / pv for v in aug[c]]
        for r in range(n):
            if r != c and aug[r][c] != 0:
                f = aug[r][c]
                aug[r] = [vr - f * vc for vr, vc in zip(aug[r], aug[c])]
    return [row[n:] for row in aug]


@pytest.mark.parametrize("seed,n,p,h2", [(0, 6, 2, Fraction(1, 4)), (1, 8, 3, Fraction(1, 2)),
                                         (2, 10, 3, Fraction(3, 4)), (3, 7, 3, Fraction(1, 3))])
def test_exact_rational_brute_force(oracle_lib, seed, n, p, h2):
    rng = np.random.default_rng(seed)
    a = rng.integers(-2, 3, size=(n, n))
    phi_i = a @ a.T + np.eye(n, dtype=np.int64)               # integer SPD kinship
    xl_i = np.vstack([np.ones(n, dtype=np.int64), rng.integers(-3, 4, size=(p - 2, n))])
    x_i = rng.integers(0, 3, size=n)
    y_i = rng.integers(-5, 6, size=n)
    phi = [[Fraction(int(v)) for v in row] for row in phi_i]
    m = [[h2 * phi[r][c] + ((1 - h2) if r == c else 0) for c in range(n)] for r in range(n)]
    x = [[Fraction(int(v)) for v in list(xl_i[:, r]) + [x_i[r]]] for r in range(n)]      # n x p
    y = [[Fraction(int(v))] for v in y_i]
    minv_x = _frac_solve(m, x)                                  # M^{-1} X
    minv_y = _frac_solve(m, y)                                  # M^{-1} y
    s = [[sum(x[k][u] * minv_x[k][v] for k in range(n)) for v in range(p)] for u in range(p)]
    r = [[sum(x[k][u] * minv_y[k][0] for k in range(n))] for u in range(p)]
    exact = np.array([float(v[0]) for v in _frac_solve(s, r)])
    b = oracle_lib.gls(phi_i.astype(float), xl_i.astype(float), x_i[None].astype(float),
                       y_i[None].astype(float), np.array([float(h2)]))
    assert rel(b[0], exact) < 1e-13


def test_exact_recovery_and_equivariance(oracle_lib, small):
    phi, xl, xr, _, h2 = small
    rng = np.random.default_rng(7)
    p = xl.shape[0] + 1
    for i in range(3):
        x = np.column_stack([xl.T, xr[i].astype(float)])
        beta = rng.standard_normal((h2.size, p))
        y = beta @ x.T                                      # noise free
        b = oracle_lib.gls(phi, xl, np.repeat(xr[i : i + 1], h2.size, 0), y, h2)
        assert rel(b, beta).max() < 1e-10
        y2 = rng.standard_normal((h2.size, x.shape[0]))
        c = rng.standard_normal((h2.size, p))
        a = -2.5
        b0 = oracle_lib.gls(phi, xl, np.repeat(xr[i : i + 1], h2.size, 0), y2, h2)
        b1 = oracle_lib.gls(phi, xl, np.repeat(xr[i : i + 1], h2.size, 0), a * y2 + c @ x.T, h2)
        assert rel(b1, a * b0 + c).max() < 1e-11


def test_frisch_waugh_lovell_snp_coefficient(oracle_lib, small):
    phi, xl, xr, y, h2 = small
    b = oracle_lib.gls_grid(phi, xl, xr, y, h2)
    xlm = xl.T
    for j in range(y.shape[0]):
        m = h2[j] * phi + (1 - h2[j]) * np.eye(phi.shape[0])
        cf = scipy.linalg.cho_factor(m)
        minv = lambda v: scipy.linalg.cho_solve(cf, v)
        proj = lambda v: v - xlm @ np.linalg.solve(xlm.T @ minv(xlm), xlm.T @ minv(v))
        ry = proj(y[j])
        for i in range(xr.shape[0]):
            rx = proj(xr[i].astype(float))
            beta = (rx @ minv(ry)) / (rx @ minv(rx))
            assert abs(b[i, j, -1] - beta) <= 1e-11 * max(1.0, abs(beta))


def test_h2_one_is_gls_with_phi(oracle_lib, small):
    phi, xl, xr, y, _ = small
    h2 = np.ones(y.shape[0])
    b = oracle_lib.gls_grid(phi, xl, xr, y, h2)
    cf = scipy.linalg.cho_factor(phi)
    for i in range(xr.shape[0]):
        x = np.column_stack([xl.T, xr[i].astype(float)])
        ref = np.linalg.solve(x.T @ scipy.linalg.cho_solve(cf, x), x.T @ scipy.linalg.cho_solve(cf, y.T)).T
        assert rel(b[i], ref).max() < 1e-11


def test_p2_closed_form(oracle_lib):
    phi, _, xr, y, h2 = synth.small(40, 2, 5, 3, seed=11)
    xl = np.ones((1, 40))
    b = oracle_lib.gls_grid(phi, xl, xr, y, h2)
    for j in range(3):
        minv = np.linalg.inv(h2[j] * phi + (1 - h2[j]) * np.eye(40))
        one = np.ones(40)
        for i in range(5):
            x = xr[i].astype(float)
            a11, a12, a22 = one @ minv @ one, one @ minv @ x, x @ minv @ x
            r1, r2 = one @ minv @ y[j], x @ minv @ y[j]
            det = a11 * a22 - a12 * a12
            ref = np.array([(a22 * r1 - a12 * r2) / det, (a11 * r2 - a12 * r1) / det])
            assert rel(b[i, j], ref) < 1e-11


def test_agrees_with_rotated_reduction(oracle_lib):
    import oracle.rotated as rot
    for n, m, t in [(128, 24, 5), (1000, 6, 2)]:
        phi, xl, xr, y, h2 = synth.small(n, 4, m, t, seed=n)
        b = oracle_lib.gls_grid(phi, xl, xr, y, h2)
        lam, z = np.linalg.eigh(phi)
        br = rot.gls_rotated(xl, xr, y, h2, z, lam)
        assert rel(br, b).max() < 1e-11


def test_rotated_reduction_sign_and_order_invariance():
    import oracle.rotated as rot
    phi, xl, xr, y, h2 = synth.small(64, 4, 10, 3, seed=5)
    lam, z = np.linalg.eigh(phi)
    b = rot.gls_rotated(xl, xr, y, h2, z, lam)
    rng = np.random.default_rng(0)
    perm = rng.permutation(64)
    sign = rng.choice([-1.0, 1.0], size=64)
    b2 = rot.gls_rotated(xl, xr, y, h2, (z * sign)[:, perm], lam[perm])
    assert rel(b2, b).max() < 1e-12


def test_rank_deficient_snp_gives_nan_and_is_counted(oracle_lib, small):
    phi, xl, xr, y, h2 = small
    cols = np.vstack([xr[:2].astype(float), 2.0 * xl[0], xl[1]])   # a constant and a covariate copy
    b, bad = oracle_lib.gls(phi, xl, cols, np.repeat(y[:1], 4, 0), np.repeat(h2[:1], 4),
                            return_non_spd=True)
    assert bad == 2
    assert np.isfinite(b[:2]).all() and np.isnan(b[2:]).all()


def test_dependent_covariates_give_nan_for_every_problem(oracle_lib, small):
    """Two covariates that are multiples of each other leave no X_i of full rank
    (Section 2 assumes full rank): every b is NaN and every problem counted."""
    phi, xl, xr, y, h2 = small
    xl = np.vstack([xl, 3.0 * xl[-1]])
    b, bad = oracle_lib.gls(phi, xl, xr[:5], np.repeat(y[:1], 5, 0), np.repeat(h2[:1], 5),
                            return_non_spd=True)
    assert bad == 5
    assert np.isnan(b).all()


def test_non_spd_covariance_is_an_error(oracle_lib):
    n = 8
    v = np.ones(n)
    phi = np.outer(v, v)                                     # rank one: h2 = 1 makes M singular
    xl = np.vstack([np.ones(n), np.arange(n, dtype=float)])
    with pytest.raises(oracle_lib.OracleError):
        oracle_lib.gls(phi, xl, np.arange(n, dtype=float)[None] ** 2, np.ones((1, n)), np.array([1.0]))


def test_tiny_workload_generators_and_trait_grouping(oracle_lib):
    w = synth.WORKLOADS["tiny"]
    phi = synth.kinship(w)
    assert np.allclose(phi, phi.T) and np.linalg.eigvalsh(phi).min() > 1e-3
    xl = synth.covariates(w)
    xr = synth.snps(w)
    y, h2 = synth.traits(w)
    assert xl.shape == (3, 128) and xr.shape == (512, 128) and y.shape == (8, 128)
    assert ((xr == xr[:, :1]).all(axis=1)).sum() == 0
    full = oracle_lib.gls_grid(phi, xl, xr[:40], y, h2)
    # grouping by trait inside the oracle must not change any result
    ii = np.array([5, 3, 39, 5, 0])
    jj = np.array([7, 0, 2, 2, 7])
    b = oracle_lib.gls(phi, xl, xr[ii], y, h2, trait=jj, nthreads=3)
    assert np.array_equal(b, full[ii, jj])
