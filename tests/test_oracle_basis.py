"""Pins of the oracle's velocity set, angular polynomials, equation of state
and driving term against what the dissertation prints (tests/golden)."""
import itertools
import json
import os

import numpy as np
import pytest

from oracle import rlb
from oracle.velocity_set import P0, P1, P2, P3, velocity_set

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_constants.json")))
V, W, OPP = velocity_set()
D = np.eye(3)


def dfact(n):
    return 1 if n <= 0 else n * dfact(n - 2)


def sphere_monomial(a, b, c):
    """int dOmega/4pi x^a y^b z^c: (a-1)!!(b-1)!!(c-1)!!/(a+b+c+1)!! for even
    exponents, 0 otherwise (closed form)."""
    if a % 2 or b % 2 or c % 2:
        return 0.0
    return dfact(a - 1) * dfact(b - 1) * dfact(c - 1) / dfact(a + b + c + 1)


def test_set_is_unit_and_symmetric():
    assert V.shape == (26, 3)
    np.testing.assert_allclose(np.linalg.norm(V, axis=1), 1.0, atol=1e-15)
    np.testing.assert_allclose(V[OPP], -V, atol=0)
    assert abs(W.sum() - 1.0) < 1e-15


def test_quadrature_exact_to_degree_7():
    """P1: the weights integrate every monomial of degree <= 7 exactly."""
    for a, b, c in itertools.product(range(8), repeat=3):
        if a + b + c > 7:
            continue
        got = np.sum(W * V[:, 0] ** a * V[:, 1] ** b * V[:, 2] ** c)
        assert abs(got - sphere_monomial(a, b, c)) < 1e-15, (a, b, c)


def test_quadrature_not_exact_at_degree_8():
    bad = [abs(np.sum(W * V[:, 0] ** a * V[:, 1] ** b * V[:, 2] ** c) - sphere_monomial(a, b, c))
           for a, b, c in itertools.product(range(9), repeat=3) if a + b + c == 8]
    assert max(bad) > 1e-4


def test_orthogonality_relations():
    """P2: orthogonality of P^(0..2) as printed, and P^(3) orthogonal to lower orders."""
    g = GOLD["angular_orthogonality"]
    assert abs(np.sum(W * P0(V) * P0(V)) - g["P0P0"]) < 1e-15
    np.testing.assert_allclose(np.einsum("q,qi,qj->ij", W, P1(V), P1(V)), g["P1P1_delta"] * D, atol=1e-15)
    want = g["P2P2_scale"] * (np.einsum("il,jm->ijlm", D, D) + np.einsum("im,jl->ijlm", D, D)
                              + g["P2P2_trace_term"] * np.einsum("ij,lm->ijlm", D, D))
    np.testing.assert_allclose(np.einsum("q,qij,qlm->ijlm", W, P2(V), P2(V)), want, atol=1e-15)
    np.testing.assert_allclose(np.einsum("q,qij->ij", W, P2(V)), 0, atol=1e-15)
    np.testing.assert_allclose(np.einsum("q,qa,qijk->aijk", W, P1(V), P3(V)), 0, atol=1e-15)
    np.testing.assert_allclose(np.einsum("q,qijk->ijk", W, P3(V)), 0, atol=1e-15)


def test_fourth_moment_identity():
    s = GOLD["fourth_moment"]["scale"]
    want = s * (np.einsum("il,jm->ijlm", D, D) + np.einsum("im,jl->ijlm", D, D)
                + np.einsum("ij,lm->ijlm", D, D))
    got = np.einsum("q,qi,qj,ql,qm->ijlm", W, V, V, V, V)
    np.testing.assert_allclose(got, want, atol=1e-15)


def test_equation_of_state():
    """P7: T^{00} = T^{xx}+T^{yy}+T^{zz} for any populations; the rest-frame
    equilibrium has pressure eps/3."""
    rng = np.random.default_rng(0)
    F = rng.uniform(0.0, 1.0, size=(26, 3, 5))
    T = rlb.energy_momentum(F)
    np.testing.assert_allclose(T[0, 0], T[1, 1] + T[2, 2] + T[3, 3], rtol=1e-14)
    eps = np.full((1, 1), 2.5)
    Feq = rlb.equilibrium_F(eps, rlb.four_velocity_from_beta(np.zeros((1, 1)), np.zeros((1, 1))))
    Teq = rlb.energy_momentum(Feq)
    P = GOLD["equation_of_state"]["P_over_eps"] * 2.5
    np.testing.assert_allclose(np.diag(Teq[:, :, 0, 0]), [2.5, P, P, P], rtol=1e-14)


def test_driving_term_projects_to_appendix_coefficients():
    """The bracket Phi is quadratic in v, so w_i Phi_i is fixed by its
    projections on P^(0), P^(1), P^(2).  They must equal the appendix's
    coefficients a^(0), a^(1), a^(2) (computed here from the appendix
    formulas, not from the bracket), divided by the orthogonality norms."""
    c = GOLD["force_coefficients"]
    rng = np.random.default_rng(3)
    Ft = rng.uniform(0.01, 0.1, size=(26, 2, 3))
    force = rng.normal(size=(3, 2, 3))
    phi = rlb.driving_term(Ft, force)
    M0 = Ft.sum(0)
    M1 = np.einsum("qk,qyx->kyx", V, Ft)
    M3 = np.einsum("qa,qb,qc,qyx->abcyx", V, V, V, Ft)
    FM1 = np.einsum("kyx,kyx->yx", force, M1)
    a0 = c["a0_F_dot_M1"] * FM1
    a1 = c["a1_F_M0"] * force * M0
    a2 = (c["a2_F_M3"] * np.einsum("kyx,kijyx->ijyx", force, M3)
          + c["a2_F_M1"] * np.einsum("iyx,jyx->ijyx", force, M1)
          + c["a2_delta_F_dot_M1"] * D[:, :, None, None] * FM1)
    a2 = 0.5 * (a2 + a2.transpose(1, 0, 2, 3))
    wphi = W[:, None, None] * phi
    np.testing.assert_allclose(wphi.sum(0), a0, rtol=1e-12, atol=1e-15)
    np.testing.assert_allclose(np.einsum("qk,qyx->kyx", V, wphi), a1 / 3.0, rtol=1e-12, atol=1e-15)
    np.testing.assert_allclose(np.einsum("qij,qyx->ijyx", P2(V), wphi), 2.0 / 15.0 * a2,
                               rtol=1e-12, atol=1e-15)
    b = GOLD["force_bracket"]
    assert (b["F_dot_M1"], b["Fv_M0"], b["F_vv_M3"], b["Fv_vM1"]) == (0.25, -0.5, 1.25, -2.5)
