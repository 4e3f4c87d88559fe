"""Pins of the oracle's Euler physics: the guaranteed wave-speed bound
(eq. dij_low_order, Assumption ass:propagation_speed) against the exact
Riemann solution, and the exact solver against textbook values."""
import json
import math
import os

import numpy as np
import pytest

G = 1.4
SOD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "sod_star.json")))


def cons(rho, u, p, dim=1):
    v = np.zeros(dim)
    v[: len(np.atleast_1d(u))] = u
    return np.concatenate([[rho], rho * v, [p / (G - 1) + 0.5 * rho * v @ v]])


def test_sod_star_state(oracle):
    ps, us, vac = oracle.exact_riemann(G, *SOD["left"], *SOD["right"])
    assert vac == 0
    assert round(ps, 5) == SOD["p_star"]
    assert round(us, 5) == SOD["u_star"]
    # densities behind the left rarefaction tail and the right shock
    rl = oracle.riemann_sample(G, SOD["left"], SOD["right"], us - 1e-9)
    rr = oracle.riemann_sample(G, SOD["left"], SOD["right"], us + 1e-9)
    assert round(rl[0], 5) == SOD["rho_star_left"]
    assert round(rr[0], 5) == SOD["rho_star_right"]


def test_sod_bound_above_exact(oracle):
    UL, UR = cons(1.0, 0.0, 1.0), cons(0.125, 0.0, 0.1)
    lam = oracle.lambda_max(G, UL, UR, np.array([1.0]))
    ex = oracle.exact_lambda(G, 1.0, 0.0, 1.0, 0.125, 0.0, 0.1)
    assert lam >= ex
    assert lam == pytest.approx(1.762090, abs=2e-6)   # two-rarefaction p_TR = 0.306767
    assert ex == pytest.approx(1.752156, abs=2e-6)


def test_identical_states_closed_form(oracle):
    """U_L = U_R: p_TR = p exactly, so lambda^+ = |u.n| + a."""
    rng = np.random.default_rng(3)
    for _ in range(200):
        rho, p = 10 ** rng.uniform(-3, 3, 2)
        u = rng.uniform(-10, 10, 2)
        n = rng.normal(size=2)
        n /= np.linalg.norm(n)
        U = cons(rho, u, p, 2)
        lam = oracle.lambda_max(G, U, U, n)
        assert lam == pytest.approx(abs(u @ n) + math.sqrt(G * p / rho), rel=1e-12)


def test_bound_brute_force(oracle):
    """lambda^+ >= exact lambda_max on random admissible pairs (rho, p in
    [1e-3, 1e3], |u| <= 10); equality when both waves are rarefactions."""
    rng = np.random.default_rng(20240204)
    n_rare = 0
    for _ in range(4000):
        rl, rr, pl, pr = 10 ** rng.uniform(-3, 3, 4)
        ul, ur = rng.uniform(-10, 10, 2)
        lam = oracle.lambda_max(G, cons(rl, ul, pl), cons(rr, ur, pr), np.array([1.0]))
        ex = oracle.exact_lambda(G, rl, ul, pl, rr, ur, pr)
        assert lam >= ex * (1 - 1e-12) - 1e-13, (rl, ul, pl, rr, ur, pr)
        ps, us, vac = oracle.exact_riemann(G, rl, ul, pl, rr, ur, pr)
        if vac == 0 and ps < min(pl, pr):
            n_rare += 1
            assert lam == pytest.approx(ex, rel=1e-9)
    assert n_rare > 100


def test_bound_rotation_and_symmetry(oracle):
    """lambda^+(U_L, U_R, n) = lambda^+(U_R, U_L, -n) and only u.n enters."""
    rng = np.random.default_rng(5)
    for _ in range(300):
        rl, rr, pl, pr = 10 ** rng.uniform(-2, 2, 4)
        ul, ur = rng.uniform(-3, 3, (2, 3))
        n = rng.normal(size=3)
        n /= np.linalg.norm(n)
        UL, UR = cons(rl, ul, pl, 3), cons(rr, ur, pr, 3)
        a = oracle.lambda_max(G, UL, UR, n)
        b = oracle.lambda_max(G, UR, UL, -n)
        assert a == pytest.approx(b, rel=1e-12)
        c1 = oracle.lambda_max(G, cons(rl, ul @ n, pl), cons(rr, ur @ n, pr), np.array([1.0]))
        # tangential velocity changes E but not p, so the 1D projection agrees
        assert a == pytest.approx(c1, rel=1e-12)


def test_vacuum_branch(oracle):
    """Strong expansion: the numerator of p_TR is <= 0, p* = 0 and lambda^+
    is the larger of |u_L - a_L|, |u_R + a_R|."""
    UL, UR = cons(1.0, -20.0, 1.0), cons(1.0, 20.0, 1.0)
    lam = oracle.lambda_max(G, UL, UR, np.array([1.0]))
    a = math.sqrt(G)
    assert lam == pytest.approx(20.0 + a, rel=1e-14)
    ps, us, vac = oracle.exact_riemann(G, 1.0, -20.0, 1.0, 1.0, 20.0, 1.0)
    assert vac == 1


def test_exact_solution_conserves(oracle):
    """Integral of the sampled exact Sod solution over [-2, 2] at t = 1 equals the
    initial integral (the fastest wave, the shock at speed 1.75, stays inside)."""
    L, R = SOD["left"], SOD["right"]
    xs = np.linspace(-2, 2, 400001)
    s = np.array([oracle.riemann_sample(G, L, R, x) for x in xs[::10]])
    x = xs[::10]
    rho = s[:, 0]
    mass = np.trapezoid(rho, x)
    assert mass == pytest.approx(1.0 * 2 + 0.125 * 2, rel=2e-5)


@pytest.mark.parametrize("gamma", [5.0 / 3.0, 1.3, 1.1])
def test_bound_brute_force_other_gamma(oracle, gamma):
    """The two-rarefaction bound is an upper bound for 1 < gamma <= 5/3
    (eq. dij_low_order): lambda^+ >= exact lambda_max on random pairs at other
    gamma too, with equality when both waves are rarefactions."""
    def c(rho, u, p):
        return np.array([rho, rho * u, p / (gamma - 1) + 0.5 * rho * u * u])

    rng = np.random.default_rng(int(gamma * 1000))
    n_rare = 0
    for _ in range(1500):
        rl, rr, pl, pr = 10 ** rng.uniform(-3, 3, 4)
        ul, ur = rng.uniform(-10, 10, 2)
        lam = oracle.lambda_max(gamma, c(rl, ul, pl), c(rr, ur, pr), np.array([1.0]))
        ex = oracle.exact_lambda(gamma, rl, ul, pl, rr, ur, pr)
        assert lam >= ex * (1 - 1e-12) - 1e-13, (gamma, rl, ul, pl, rr, ur, pr)
        ps, us, vac = oracle.exact_riemann(gamma, rl, ul, pl, rr, ur, pr)
        if vac == 0 and ps < min(pl, pr):
            n_rare += 1
            assert lam == pytest.approx(ex, rel=1e-9)
    assert n_rare > 50
