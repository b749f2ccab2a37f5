"""Pins of the FP64 oracle against the paper and against mathematics.

Nothing here compares the oracle with itself: each check is an independent
route (quadrature of the definition, a closed form, an identity between the
paper's alternative formulations, an invariant, hand-derived geometry).
"""
import json
import math
import os
from fractions import Fraction

import numpy as np
import pytest
from scipy import integrate
from scipy.stats import norm

import oracle as O

GOLD = os.path.join(os.path.dirname(__file__), "golden")
D_OCC = 1.5


# ---------------------------------------------------------------------------
# independent helpers written from the paper's definitions (Sec. 2.2)
# ---------------------------------------------------------------------------
def f_paper(delta, o):
    """Eq. for f(delta, r) with r = o/(1-o); f(delta, 0) = f(delta, 1) = 0 (limits)."""
    if o <= 0.0 or o >= 1.0:
        return 0.0
    r = o / (1.0 - o)
    return math.log((r + 1.0) / (r + 1.0 / delta)) - math.log(delta) / (r * delta + 1.0)


def p_first_hit(o):
    """P(e_j) = o_j prod_{l<j} (1 - o_l) (Eq. Pej), j = 1..n."""
    return np.array([o[j] * np.prod(1.0 - o[:j]) for j in range(len(o))])


def f_of_z(z, o, l, delta):
    """F(z) = sum_i f(delta_i(z), r_i) straight from the inverse sensor model:
    delta_emp for cells the reading has passed, delta_occ for the cell it falls in,
    1 (no information) beyond."""
    tot = 0.0
    for i in range(len(o)):
        if z >= l[i + 1]:
            tot += f_paper(1.0 / delta, o[i])
        elif z >= l[i]:
            tot += f_paper(delta, o[i])
    return tot


def brute_force_mi(o, l, sigma, delta=D_OCC):
    """Eq. mi_sum with the measurement prior P(z) = sum_j P(e_j) N(z; mu_j, sigma^2),
    integrated by adaptive quadrature over each cell interval of [0, l_{n+1})."""
    P = p_first_hit(o)
    mu = 0.5 * (l[:-1] + l[1:])
    tot = 0.0
    for k in range(len(o)):
        Fk = f_of_z(0.5 * (l[k] + l[k + 1]), o, l, delta)
        v, _ = integrate.quad(lambda z: np.sum(P * norm.pdf(z, mu, sigma)) * f_of_z(z, o, l, delta),
                              l[k], l[k + 1], epsabs=1e-16, epsrel=1e-13, limit=200)
        tot += v
        assert Fk >= 0.0
    return tot


def smi_riemann(o, l, sigma, lam, delta=D_OCC):
    """The SMI baseline's discretisation of z at resolution lam (Sec. 2.2)."""
    P = p_first_hit(o)
    mu = 0.5 * (l[:-1] + l[1:])
    z = np.arange(0.5 * lam, l[-1], lam)
    pz = (P[None, :] * norm.pdf(z[:, None], mu[None, :], sigma)).sum(1)
    fz = np.array([f_of_z(zz, o, l, delta) for zz in z])
    return float(np.sum(pz * fz) * lam)


def entropy(o):
    o = np.clip(o, 1e-300, 1 - 1e-16)
    return -(o * np.log(o) + (1 - o) * np.log(1 - o))


# ---------------------------------------------------------------------------
# P7: the per-cell function f
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("delta", [1.5, 1.0 / 1.5, 3.0, 1.1])
def test_f_forms_agree_and_kl(delta):
    for o in np.linspace(0.001, 0.999, 41):
        r = o / (1 - o)
        a = O.f(delta, o)
        b = O.f_odds(delta, r)
        assert abs(a - b) <= 1e-13 * max(1.0, abs(b))
        assert abs(a - f_paper(delta, o)) <= 1e-13 * max(1.0, abs(a))
        # f is the KL divergence from the prior cell to the updated one (odds r -> r*delta)
        op = r * delta / (1 + r * delta)
        kl = op * math.log(op / o) + (1 - op) * math.log((1 - op) / (1 - o))
        assert abs(a - kl) <= 1e-12 * max(1e-3, abs(kl))
        assert a >= -1e-17


def test_f_symmetry_and_fixed_points():
    for o in np.linspace(0.01, 0.99, 25):
        r = o / (1 - o)
        assert abs(O.f_odds(1 / 1.5, r) - O.f_odds(1.5, 1 / r)) < 1e-14   # Sec. 3.3 remark
        assert O.f(1.0, o) == 0.0                                            # delta = 1: no update
    for d in (1.5, 1 / 1.5):
        assert O.f(d, 0.0) == 0.0 and abs(O.f(d, 1.0)) < 1e-16


# ---------------------------------------------------------------------------
# P6: P(e_j) and G_{k,j}
# ---------------------------------------------------------------------------
def test_first_hit_matches_definition_and_sums_to_one():
    rng = np.random.default_rng(3)
    o = rng.uniform(0, 1, 50)
    P = O.first_hit(o)
    assert abs(P.sum() - 1.0) < 1e-14
    assert np.allclose(P[1:], p_first_hit(o), rtol=1e-14, atol=0)
    assert abs(P[0] - np.prod(1 - o)) < 1e-16


def test_info_gain_matches_lemma1_piecewise_constant():
    rng = np.random.default_rng(4)
    o = rng.uniform(0, 1, 30)
    l = np.concatenate([[0.0], np.cumsum(rng.uniform(0.2, 1.2, 30))])
    C = O.info_gain(o, D_OCC)
    for k in range(30):
        z = 0.5 * (l[k] + l[k + 1])      # Lemma 1: F(z) = C_k on [l_k, l_{k+1})
        assert abs(C[k] - f_of_z(z, o, l, D_OCC)) < 1e-13


def test_G_against_library_cdf_and_telescoping():
    rng = np.random.default_rng(5)
    l = np.concatenate([[0.0], np.cumsum(rng.uniform(0.05, 1.5, 25))])
    sigma = 0.8
    for j in range(25):
        mu = 0.5 * (l[j] + l[j + 1])
        g = np.array([O.G(l[k], l[k + 1], mu, sigma) for k in range(25)])
        ref = norm.cdf((l[1:] - mu) / sigma) - norm.cdf((l[:-1] - mu) / sigma)
        assert np.allclose(g, ref, rtol=1e-12, atol=1e-16)
        tel = norm.cdf((l[-1] - mu) / sigma) - norm.cdf(-mu / sigma)
        assert abs(g.sum() - tel) < 1e-14
        assert np.all(g >= 0)


def test_G_far_tail_relative_accuracy():
    import mpmath as mp
    mp.mp.dps = 40
    for a in (3.0, 8.0, 20.0, 30.0):
        g = O.G(a, a + 0.25, 0.0, 1.0)
        ref = float(mp.ncdf(-a) - mp.ncdf(-a - 0.25))   # upper-tail form, no cancellation
        assert abs(g - ref) <= 1e-13 * ref


# ---------------------------------------------------------------------------
# P1: Thm 1 against quadrature of the definition (and the SMI discretisation)
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("seed", range(6))
def test_exact_equals_bruteforce_quadrature(seed):
    rng = np.random.default_rng(100 + seed)
    n = int(rng.integers(1, 9))
    o = rng.uniform(0.02, 0.98, n)
    l = np.concatenate([[0.0], np.cumsum(rng.uniform(0.1, 1.5, n))])
    sigma = float(rng.uniform(0.2, 1.5))
    ref = brute_force_mi(o, l, sigma)
    got = O.fsmi_exact(o, l, sigma, D_OCC)
    assert abs(got - ref) <= 1e-10 * abs(ref)


def brute_force_mi_ext(o, l, sigma, slope=0.0, tail=False, delta=D_OCC):
    """Eq. mi_sum with per-event noise sigma_j = sigma + slope mu_j.  With tail,
    a reading at or past l_{n+1} is a max-range return: the quadrature goes on
    past l_{n+1}, where F(z) counts every cell as passed, and the no-hit event
    e_0 reads max range with certainty, adding P(e_0) F(max range)."""
    P = p_first_hit(o)
    mu = 0.5 * (l[:-1] + l[1:])
    sj = sigma + slope * mu
    tot = 0.0
    for k in range(len(o)):
        v, _ = integrate.quad(lambda z: np.sum(P * norm.pdf(z, mu, sj)) * f_of_z(z, o, l, delta),
                              l[k], l[k + 1], epsabs=1e-16, epsrel=1e-13, limit=200)
        tot += v
    if tail:
        fmax = f_of_z(l[-1], o, l, delta)
        past, _ = integrate.quad(lambda z: np.sum(P * norm.pdf(z, mu, sj)), l[-1], np.inf,
                                 epsabs=1e-16, epsrel=1e-13, limit=200)
        tot += (past + np.prod(1.0 - o)) * fmax
    return tot


@pytest.mark.parametrize("seed", range(6))
def test_range_noise_and_max_range_equal_bruteforce(seed):
    """The two extensions of Thm 1 (range-dependent sigma_j, max-range returns)
    against quadrature of the definition with the same sensor model."""
    rng = np.random.default_rng(300 + seed)
    n = int(rng.integers(1, 9))
    o = rng.uniform(0.02, 0.98, n)
    l = np.concatenate([[0.0], np.cumsum(rng.uniform(0.1, 1.5, n))])
    sigma = float(rng.uniform(0.2, 1.5))
    slope = float(rng.uniform(0.0, 0.3))
    for sl, tail in ((slope, False), (0.0, True), (slope, True)):
        ref = brute_force_mi_ext(o, l, sigma, sl, tail)
        got = O.fsmi_exact_ext(o, l, sigma, sl, tail, D_OCC)
        assert abs(got - ref) <= 1e-10 * abs(ref), (sl, tail, got, ref)


def test_extensions_reduce_to_thm1_and_vanish_on_known_cells():
    rng = np.random.default_rng(11)
    o = rng.uniform(0.05, 0.95, 12)
    l = np.concatenate([[0.0], np.cumsum(rng.uniform(0.3, 1.2, 12))])
    assert O.fsmi_exact_ext(o, l, 0.8) == O.fsmi_exact(o, l, 0.8)
    # the max-range term is q_n times the probability of a max-range reading
    P = p_first_hit(o)
    mu = 0.5 * (l[:-1] + l[1:])
    pmax = float(np.sum(P * norm.sf(l[-1], mu, 0.8))) + float(np.prod(1.0 - o))
    qn = sum(f_paper(1.0 / D_OCC, v) for v in o)
    diff = O.fsmi_exact_ext(o, l, 0.8, 0.0, True) - O.fsmi_exact(o, l, 0.8)
    assert abs(diff - qn * pmax) <= 1e-12 * qn * pmax
    # known cells carry no information, also as max-range returns
    k = rng.integers(0, 2, 12).astype(np.float64)
    assert O.fsmi_exact_ext(k, l, 0.8, 0.2, True) == 0.0


def test_exact_equals_smi_riemann_limit():
    rng = np.random.default_rng(7)
    o = rng.uniform(0.05, 0.95, 5)
    l = np.concatenate([[0.0], np.cumsum(rng.uniform(0.4, 1.0, 5))])
    ex = O.fsmi_exact(o, l, 0.5, D_OCC)
    e1 = abs(smi_riemann(o, l, 0.5, 1e-3) - ex) / ex
    e2 = abs(smi_riemann(o, l, 0.5, 1e-4) - ex) / ex
    assert e2 < 5e-5 and e2 < e1      # the SMI sum converges to Thm 1's value


# ---------------------------------------------------------------------------
# P3, P4, P8: special cases with closed forms
# ---------------------------------------------------------------------------
def test_sigma_to_zero_is_diagonal_and_uniform_H0():
    rng = np.random.default_rng(8)
    o = rng.uniform(0, 1, 40)
    l = np.arange(41, dtype=np.float64)
    P = p_first_hit(o)
    Ck = np.array([f_paper(D_OCC, o[k]) + sum(f_paper(1 / D_OCC, o[i]) for i in range(k))
                   for k in range(40)])
    ref = float(np.sum(P * Ck))        # G_{k,j} -> [k == j]
    assert abs(O.fsmi_exact(o, l, 1e-6) - ref) <= 1e-13 * ref
    assert abs(O.fsmi_uniform(o, 0) - ref) <= 1e-13 * ref
    assert abs(O.fsmi_eqwidth(o, 1e-6, O.K_ERF) - ref) <= 1e-13 * ref


def test_known_cells_carry_no_information():
    rng = np.random.default_rng(9)
    o = rng.integers(0, 2, 30).astype(np.float64)
    l = np.concatenate([[0.0], np.cumsum(rng.uniform(0.1, 1.0, 30))])
    assert O.fsmi_exact(o, l, 0.7) == 0.0
    assert O.fsmi_approx(o, l, 0.7, 3) == 0.0
    assert O.fsmi_uniform(o, 2) == 0.0


@pytest.mark.parametrize("o,n", [(0.3, 1), (0.3, 17), (0.05, 60), (0.8, 9)])
def test_homogeneous_beam_closed_form(o, n):
    q = 1.0 - o
    fo, fe = f_paper(D_OCC, o), f_paper(1 / D_OCC, o)
    # sum_j P_j C_j with P_j = o q^{j-1}, C_j = f_occ + (j-1) f_emp, summed in closed form
    s1 = 1.0 - q ** n
    s2 = q * (1.0 - n * q ** (n - 1) + (n - 1) * q ** n) / o
    ref = fo * s1 + fe * s2
    ov = np.full(n, o)
    assert abs(O.fsmi_exact(ov, np.arange(n + 1.0), 1e-6) - ref) <= 1e-13 * ref
    assert abs(O.rle_expanded([o], [n], 1e-6) - ref) <= 1e-13 * ref
    assert abs(O.rle_thm5([o], [n], 1e-6) - ref) <= 1e-13 * ref


# ---------------------------------------------------------------------------
# P5: bounds
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("seed", range(4))
def test_mi_bounds(seed):
    rng = np.random.default_rng(200 + seed)
    n = 80
    o = rng.uniform(0, 1, n)
    l = np.concatenate([[0.0], np.cumsum(rng.uniform(0.05, 1.4, n))])
    fmax = np.array([max(f_paper(D_OCC, x), f_paper(1 / D_OCC, x)) for x in o])
    for v in (O.fsmi_exact(o, l, 1.3), O.fsmi_approx(o, l, 1.3, 4), O.fsmi_uniform(o, 3)):
        assert 0.0 <= v <= fmax.sum() <= 0.031 * entropy(o).sum()


# ---------------------------------------------------------------------------
# P9: truncation
# ---------------------------------------------------------------------------
def test_approx_monotone_and_reaches_exact():
    rng = np.random.default_rng(10)
    n = 40
    o = rng.uniform(0, 1, n)
    l = np.concatenate([[0.0], np.cumsum(rng.uniform(0.05, 1.4, n))])
    ex = O.fsmi_exact(o, l, 2.0)
    prev = 0.0
    for D in range(0, n):
        a = O.fsmi_approx(o, l, 2.0, D)
        assert prev <= a <= ex * (1 + 1e-15)
        prev = a
    assert abs(O.fsmi_approx(o, l, 2.0, n - 1) - ex) <= 1e-15 * ex


# ---------------------------------------------------------------------------
# P2: Thm 4 against uniform-noise integration
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("H", [0, 1, 3, 7])
def test_uniform_equals_uniform_noise_integral(H):
    rng = np.random.default_rng(20 + H)
    n = 25
    o = rng.uniform(0, 1, n)
    l = np.arange(n + 1, dtype=np.float64)       # Thm 4 needs equal widths
    P = p_first_hit(o)
    ref = 0.0
    for j in range(n):
        a, b = l[j] - H, l[j + 1] + H            # support of P(z | e_j)
        for k in range(n):
            ov = max(0.0, min(b, l[k + 1]) - max(a, l[k]))
            ref += P[j] * f_of_z(0.5 * (l[k] + l[k + 1]), o, l, D_OCC) * ov / (b - a)
    assert abs(O.fsmi_uniform(o, H) - ref) <= 1e-13 * ref
    assert abs(O.fsmi_eqwidth(o, 1.0, O.K_UNIFORM, -1, H) - ref) <= 1e-13 * ref


# ---------------------------------------------------------------------------
# P10, P11, P13: the RLE formulations
# ---------------------------------------------------------------------------
def _runs(seed, nr=7, lmax=6):
    rng = np.random.default_rng(seed)
    return rng.uniform(0.05, 0.95, nr), rng.integers(1, lmax + 1, nr)


@pytest.mark.parametrize("kind", [O.K_ERF, O.K_DENSITY, O.K_UNIFORM])
@pytest.mark.parametrize("seed", range(3))
def test_thm5_equals_expanded(kind, seed):
    ro, L = _runs(30 + seed)
    a = O.rle_expanded(ro, L, 1.7, kind, H=3)
    b = O.rle_thm5(ro, L, 1.7, kind, H=3)
    assert abs(a - b) <= 1e-14 * a


@pytest.mark.parametrize("H", [0, 2, 5])
def test_uniform_rle_is_alg4_on_the_expanded_beam(H):
    """Uniform-FSMI-RLE: the uniform kernel on runs gives Alg 4 on the expanded
    beam, which the uniform-noise integration pin fixes."""
    ro, L = _runs(60 + H, nr=8, lmax=7)
    expanded = np.repeat(ro, L)
    ref = O.fsmi_uniform(expanded, H)
    assert abs(O.rle_expanded(ro, L, 1.0, O.K_UNIFORM, H=H) - ref) <= 1e-14 * ref
    assert abs(O.rle_thm5(ro, L, 1.0, O.K_UNIFORM, H=H) - ref) <= 1e-13 * ref


def test_rle_runs_of_one_are_plain_fsmi():
    rng = np.random.default_rng(40)
    o = rng.uniform(0, 1, 20)
    a = O.rle_expanded(o, np.ones(20, int), 1.3)
    b = O.fsmi_exact(o, np.arange(21.0), 1.3)
    c = O.rle_thm5(o, np.ones(20, int), 1.3)
    assert abs(a - b) <= 1e-14 * b and abs(c - b) <= 1e-14 * b


@pytest.mark.parametrize("Delta", [0, 1, 3, 6])
@pytest.mark.parametrize("seed", range(3))
def test_thm6_equals_truncated_expanded(Delta, seed):
    ro, L = _runs(50 + seed, nr=9, lmax=9)
    for kind in (O.K_ERF, O.K_DENSITY):
        a = O.rle_expanded(ro, L, 2.0, kind, trunc=Delta)
        b = O.rle_thm6(ro, L, 2.0, Delta, kind)
        assert abs(a - b) <= 1e-14 * a
    # truncated expanded beam with the ERF kernel is Approx-FSMI on unit cells
    o = np.repeat(ro, L)
    c = O.fsmi_approx(o, np.arange(len(o) + 1.0), 2.0, Delta)
    assert abs(O.rle_expanded(ro, L, 2.0, O.K_ERF, trunc=Delta) - c) <= 1e-14 * c


def test_alpha_route_equals_density_thm5():
    # x = 1 - o >= 0.5 keeps x^{-t} small enough that Eq. compute_A is well conditioned
    rng = np.random.default_rng(60)
    ro, L = rng.uniform(0.05, 0.5, 5), rng.integers(1, 5, 5)
    a = O.rle_alpha_route(ro, L, 1.2)
    b = O.rle_thm5(ro, L, 1.2, O.K_DENSITY)
    assert abs(a - b) <= 1e-11 * b


def test_alpha_route_loses_digits_as_the_paper_warns():
    # Sec. 4.1: x^{-t} (alpha - alpha) cancels catastrophically for small x and large t
    ro, L = np.array([0.2, 0.2, 0.2, 0.2, 0.999]), np.array([10, 10, 10, 10, 5])
    a = O.rle_alpha_route(ro, L, 1.0)
    b = O.rle_thm5(ro, L, 1.0, O.K_DENSITY)
    assert abs(a - b) > 1e-5 * b       # FP64 route off by ~3e-4 here


# The table mode of Approx-FSMI-RLE (Alg 8 with the tables of Alg 9 and 10):
# tables read at x = 1 - o quantised to i / levels.
@pytest.mark.parametrize("Delta", [1, 3, 6])
@pytest.mark.parametrize("seed", range(3))
def test_table_mode_on_grid_equals_thm6(Delta, seed):
    """With every o on the grid (x = i / 64 >= 1/4, so x^{-t} <= 4^Delta) the table
    route is Thm 6 with the density kernel, itself pinned to the truncated
    expanded beam."""
    rng = np.random.default_rng(80 + seed)
    ro, L = rng.integers(0, 49, 12) / 64.0, rng.integers(1, 9, 12)
    a = O.rle_table(ro, L, 1.5, Delta, 64)
    b = O.rle_thm6(ro, L, 1.5, Delta, O.K_DENSITY)
    assert abs(a - b) <= 1e-14 * abs(b)


def test_table_mode_full_occupancy_limit():
    """o = 1 (x = 0): x^{-t} has no value and the block is its first row; the
    value is still Thm 6's."""
    for ro, L in ((np.array([0.25, 1.0, 0.5, 1.0, 0.0]), np.array([3, 2, 4, 1, 5])),
                  (np.array([0.0, 0.25, 1.0]), np.array([2, 3, 4]))):
        a = O.rle_table(ro, L, 1.2, 3, 64)
        b = O.rle_thm6(ro, L, 1.2, 3, O.K_DENSITY)
        assert abs(a - b) <= 1e-14 * abs(b)


def test_table_mode_quantisation_error_falls_with_the_grid():
    rng = np.random.default_rng(7)
    ro, L = rng.uniform(0.05, 0.7, 15), rng.integers(1, 9, 15)
    b = O.rle_thm6(ro, L, 1.5, 3, O.K_DENSITY)
    err = [abs(O.rle_table(ro, L, 1.5, 3, lv) - b) / b for lv in (16, 64, 256, 1024)]
    assert all(e1 < e0 for e0, e1 in zip(err, err[1:]))
    assert err[0] > 1e-2 and err[-1] < 1e-3


def test_table_mode_runs_of_one_carry_no_quantisation_error():
    """With every run one cell long, a block's table difference is a single row
    x^t g(...), which x^{-t} cancels exactly: off-grid o gives Thm 6's value up
    to the cancellation (x >= 1/64, Delta = 3: at most 64^3 ulps)."""
    rng = np.random.default_rng(12)
    ro = rng.uniform(0.0, 0.99, 40)
    L = np.ones(40, int)
    a = O.rle_table(ro, L, 1.0, 3, 64)
    b = O.rle_thm6(ro, L, 1.0, 3, O.K_DENSITY)
    assert abs(a - b) <= 2.0 ** -52 * 64.0 ** 3 * b
    ro2, L2 = ro[:20], np.full(20, 3)            # runs of 3: the grid shows
    c = O.rle_table(ro2, L2, 1.0, 3, 64)
    d = O.rle_thm6(ro2, L2, 1.0, 3, O.K_DENSITY)
    assert abs(c - d) > 1e-6 * d


@pytest.mark.parametrize("Delta,bound", [(3, 1e-11), (6, 1e-5)])
def test_table_mode_cancellation_grows_as_x_to_the_minus_delta(Delta, bound):
    """Sec. 4.1's instability in FP64, with o on the grid so that no quantisation
    error enters: x^{-t} (alpha - alpha) loses about log10(x^{-Delta}) digits."""
    errs = []
    for xi in (16, 4, 1):
        ro = np.array([6, 64 - xi, 6, 64 - xi, 19, 64 - xi]) / 64.0
        L = np.full(6, 6)
        a = O.rle_table(ro, L, 1.0, Delta, 64)
        b = O.rle_thm6(ro, L, 1.0, Delta, O.K_DENSITY)
        errs.append(abs(a - b) / b)
    assert errs[0] < errs[1] < errs[2] <= bound
    assert errs[2] > 1e3 * errs[0] and errs[2] > 1e-13


@pytest.mark.parametrize("x", [0.0, 0.3, 0.9])
def test_table_recurrences_equal_definitions(x):
    a1, b1, t1, g1 = O.tables(x, 1.4, 6, 12, "definition")
    a2, b2, t2, g2 = O.tables(x, 1.4, 6, 12, "recurrence")
    assert np.allclose(a1[1:, 1:], a2[1:, 1:], rtol=1e-13, atol=1e-15)
    assert np.allclose(b1[1:, 1:], b2[1:, 1:], rtol=1e-13, atol=1e-15)
    assert np.allclose(t1[1:], t2[1:], rtol=1e-13, atol=1e-15)
    assert np.allclose(g1[1:], g2[1:], rtol=1e-13, atol=1e-15)


def test_kernels_normalised():
    for sp in (0.5, 2.0, 3.3):
        s = sum(O.kernel_weight(O.K_ERF, sp, d) for d in range(-60, 61))
        assert abs(s - 1.0) < 1e-14
    s = sum(O.kernel_weight(O.K_UNIFORM, 1.0, d, H=4) for d in range(-10, 11))
    assert abs(s - 1.0) < 1e-15


# ---------------------------------------------------------------------------
# P12: ray traversal
# ---------------------------------------------------------------------------
def test_raycast_hand_derived_golden():
    g = json.load(open(os.path.join(GOLD, "raycast_hand.json")))
    grid = np.arange(100, dtype=np.float32).reshape(10, 10) / 100.0
    for c in g["cases"]:
        cells, entry, occ = O.raycast2d(grid, c["origin"], c["dir"], c["R"])
        assert cells.tolist() == c["cells"], c["name"]
        assert np.allclose(entry, c["entry"], rtol=1e-15, atol=1e-15), c["name"]
        assert np.array_equal(occ, grid.reshape(-1)[cells])


def _rational_walk(X, Y, p, d, R):
    """Same traversal rules in exact rational arithmetic (events t = (face - p)/d)."""
    px, py = Fraction(p[0]), Fraction(p[1])
    dx, dy = Fraction(d[0]), Fraction(d[1])
    Rr = Fraction(R)
    cx, cy = math.floor(px), math.floor(py)
    sx = (dx > 0) - (dx < 0)
    sy = (dy > 0) - (dy < 0)
    fx = cx + 1 if sx > 0 else cx
    fy = cy + 1 if sy > 0 else cy
    tx = (fx - px) / dx if sx else None
    ty = (fy - py) / dy if sy else None
    tcur, cells, times = Fraction(0), [], []
    while True:
        cand = [t for t in (tx, ty) if t is not None]
        tn = min(cand)
        end = min(tn, Rr)
        if end > tcur:
            cells.append(cx + X * cy)
        if tn >= Rr:
            return cells, times
        times.append(tn)
        if tx is not None and tx == tn:
            cx += sx; fx += sx; tx = (fx - px) / dx
        if ty is not None and ty == tn:
            cy += sy; fy += sy; ty = (fy - py) / dy
        tcur = max(tcur, tn)
        if not (0 <= cx < X and 0 <= cy < Y):
            return cells, times


def test_raycast_matches_exact_rational_walk():
    rng = np.random.default_rng(11)
    X = Y = 64
    grid = rng.uniform(0, 1, (Y, X)).astype(np.float32)
    checked = 0
    for _ in range(300):
        p = rng.uniform(0, 64, 2)
        th = rng.uniform(0, 2 * math.pi)
        d = np.array([math.cos(th), math.sin(th)])
        R = float(rng.uniform(1, 80))
        ref, times = _rational_walk(X, Y, p, d, R)
        # skip rays with two events (or an event and R) closer than 4 ulp: FP64
        # rounding may legitimately order those differently
        ts = sorted(float(t) for t in times) + [R]
        if any(abs(b - a) <= 4 * np.spacing(max(abs(a), abs(b), 1.0)) for a, b in zip(ts, ts[1:])):
            continue
        cells, entry, _ = O.raycast2d(grid, p, d, R)
        assert cells.tolist() == ref
        w = np.diff(entry)
        assert np.all(w > 0) and abs(w.sum() - (entry[-1] - entry[0])) < 1e-12
        assert len(cells) <= math.floor(math.sqrt(2) * R) + 3
        checked += 1
    assert checked > 250


def test_raycast_mirror_symmetry():
    rng = np.random.default_rng(12)
    X = Y = 32
    grid = rng.uniform(0, 1, (Y, X)).astype(np.float32)
    for _ in range(100):
        p = np.round(rng.uniform(0.01, 31.99, 2) * 1024) / 1024     # dyadic: X - p is exact
        if np.any(p == np.floor(p)):
            continue
        th = rng.uniform(0, 2 * math.pi)
        d = np.array([math.cos(th), math.sin(th)])
        c1, e1, _ = O.raycast2d(grid, p, d, 50.0)
        c2, e2, _ = O.raycast2d(grid, [X - p[0], p[1]], [-d[0], d[1]], 50.0)
        x1, y1 = c1 % X, c1 // X
        assert (X - 1 - x1 + X * y1).tolist() == c2.tolist()
        assert np.array_equal(e1, e2)


def test_virtual_cells_and_runs():
    vox = np.zeros((4, 8, 16), np.float32)
    vox[:, :, :8] = 0.2
    vox[:, :, 8:12] = 0.9
    vox[:, :, 12:] = 0.5
    cells, occ = O.virtual3d(vox, [0.25, 4.5, 2.5], [1.0, 0.0, 0.0], 100.0, 1.0)
    # midpoints at x = 0.75, 1.75, ..., 15.75; the 16th (x = 16.75) is outside
    assert len(cells) == 16
    assert cells.tolist() == [x + 16 * (4 + 8 * 2) for x in range(len(cells))]
    ro, rl = O.rle_runs(occ)
    assert ro.tolist() == [np.float32(0.2), np.float32(0.9), np.float32(0.5)]
    assert rl.tolist() == [8, 4, 4]
    assert rl.sum() == len(occ)
