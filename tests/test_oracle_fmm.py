"""Pins for oracle.fmm: the sphere quadrature, the truncated expansion of
Eq. (FMMBase), band-limited resampling, the paper's printed storage counts and
level counts, and the plain-steps FMM against the dense operator."""

import json
import math
import os

import numpy as np
import pytest
from scipy.special import sph_harm_y

import synth
from oracle import fmm as ofmm
from oracle import operator as op
from oracle.geometry import element_geometry
from oracle.kernels import green
from oracle.presets import preset

GOLDEN = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_worked_examples.json")))


def _angles(s):
    return np.arccos(np.clip(s[:, 2], -1, 1)), np.arctan2(s[:, 1], s[:, 0])


@pytest.mark.parametrize("L", [4, 9, 17])
def test_sphere_grid_integrates_harmonics_exactly(L):
    s, w, _, _ = ofmm.sphere_grid(L)
    assert s.shape == (2 * L * L, 3)
    assert np.sum(w) == pytest.approx(4 * math.pi, rel=1e-14)
    assert np.allclose(np.linalg.norm(s, axis=1), 1.0, atol=1e-15)
    th, ph = _angles(s)
    # orthonormality of Y_nm for n < L (products of degree <= 2L - 2)
    for n1, m1, n2, m2 in [(0, 0, 0, 0), (L - 1, 2, L - 1, 2), (L - 1, -1, L - 2, -1), (3 % L, 1 % (3 % L + 1), 1, 0)]:
        if abs(m1) > n1 or abs(m2) > n2:
            continue
        v = np.sum(w * sph_harm_y(n1, m1, th, ph) * np.conj(sph_harm_y(n2, m2, th, ph)))
        assert abs(v - (1.0 if (n1, m1) == (n2, m2) else 0.0)) < 1e-13


def test_expansion_reproduces_green_function():
    k = 6.0
    z1 = np.array([0.0, 0.0, 0.0])
    z2 = np.array([1.7, -0.4, 0.9])
    rng = np.random.default_rng(2)
    pts = [(z1 + 0.25 * rng.uniform(-1, 1, 3), z2 + 0.25 * rng.uniform(-1, 1, 3)) for _ in range(5)]

    def err(L):
        return max(abs(ofmm.green_expansion(k, x, y, z1, z2, L) - green(x, y, k)) / abs(green(x, y, k))
                   for x, y in pts)

    # geometric convergence while L is moderate ...
    for L, tol in [(10, 1e-5), (14, 1e-8), (18, 1e-11)]:
        assert err(L) < tol, (L, err(L))
    # ... and the small-argument growth of h_L (Sec. 4.2) takes over for
    # large L: rounding amplified by (2L+1)|h_L(k X)| dominates
    e28 = err(28)
    bound28 = 2.0 ** -52 * (2 * 28 + 1) * ofmm.hankel_abs(28, k * np.linalg.norm(z2 - z1))
    assert e28 > 1e4 * err(18)
    assert e28 < 100 * bound28


def test_translation_vectorised_matches_single():
    k = 4.0
    s, _, _, _ = ofmm.sphere_grid(7)
    X = np.array([[1.0, 2.0, -0.5], [0.3, -1.2, 2.2]])
    D = ofmm.translations(k, X, s, 7)
    for i in range(2):
        assert np.allclose(D[i], ofmm.translation(k, X[i], s, 7), rtol=1e-13, atol=0)


@pytest.mark.parametrize("Lc,Lp", [(5, 9), (8, 8), (7, 12)])
def test_interpolation_is_exact_for_band_limited_functions(Lc, Lp):
    rng = np.random.default_rng(Lc * 31 + Lp)
    coef = {(n, m): rng.standard_normal() + 1j * rng.standard_normal() for n in range(Lc) for m in range(-n, n + 1)}

    def f(s):
        th, ph = _angles(s)
        return sum(c * sph_harm_y(n, m, th, ph) for (n, m), c in coef.items())

    sc, wc, _, _ = ofmm.sphere_grid(Lc)
    sp, wp, _, _ = ofmm.sphere_grid(Lp)
    I = ofmm.interpolation_matrix(Lc, Lp)
    if Lc == Lp:
        assert np.array_equal(I, np.eye(2 * Lc * Lc))
        return
    assert np.max(np.abs(I @ f(sc) - f(sp))) < 1e-11 * np.max(np.abs(f(sp)))
    # anterpolation is the weighted transpose: sum_p wp (I u) g = sum_c wc u (A g)
    A = ofmm.anterpolation_matrix(Lp, Lc)
    u = rng.standard_normal(sc.shape[0]) + 1j * rng.standard_normal(sc.shape[0])
    g = rng.standard_normal(sp.shape[0]) + 1j * rng.standard_normal(sp.shape[0])
    assert abs(np.sum(wp * (I @ u) * g) - np.sum(wc * u * (A @ g))) < 1e-11 * np.linalg.norm(u) * np.linalg.norm(g)


def test_paper_storage_counts():
    # each stored T (= S) matrix of the paper has 2 L^2 entries per element:
    # the number of sphere nodes times N
    for c in GOLDEN["fmm_storage"]["cases"]:
        s, _, _, _ = ofmm.sphere_grid(c["L"])
        assert s.shape[0] * c["N"] == c["entries"], c


def test_paper_level_counts():
    for c in GOLDEN["levels"]["cases"]:
        assert ofmm.default_levels(c["N"]) == c["levels"], c


def test_paper_wavenumbers():
    cc = GOLDEN["wavenumbers"]["c"]
    for f, k in GOLDEN["wavenumbers"]["cases"]:
        assert 2 * math.pi * f / cc == pytest.approx(k, abs=5e-4)


def test_truncation_length_modes():
    p = preset("paper")
    # small clusters: the lower bound 8 of Eq. (FMMTruncation)
    assert ofmm.truncation_length(1.0, 0.1, p) == 8
    t = preset("tight")
    assert ofmm.truncation_length(30.0, 0.5, t) >= ofmm.truncation_length(30.0, 0.5, p)
    # the stability cap lowers L when the smallest separation is small
    assert ofmm.truncation_length(1.0, 0.3, t, x_min=0.5) < ofmm.truncation_length(1.0, 0.3, t)


def test_truncation_length_paper_worked_example():
    """Sec. 5.1.2: on the sphere at 200 Hz (k = 3.696) the default factor 1.8
    gives L = 8, 8, 8 on the three levels and factor 15 gives 12, 10, 9.  The
    paper does not print the cluster radii; with radii halving from level to
    level (leaf r = 0.0473 m, so that kd = 2 r k = 0.35, 0.7, 1.4) Eq.
    (FMMTruncation) as implemented reproduces both rows, and a natural
    logarithm in place of log10, a missing ceiling or a missing minimum of 8
    does not."""
    k = 3.696
    radii = [0.35 / (2 * k) * f for f in (4, 2, 1)]  # levels 1, 2, 3
    assert [ofmm.truncation_length(k, r, preset("paper")) for r in radii] == [8, 8, 8]
    assert [ofmm.truncation_length(k, r, preset("paper", l_factor=15.0)) for r in radii] == [12, 10, 9]


@pytest.mark.parametrize("k,r", [(27.7, 0.05), (27.7, 0.1), (10.0, 0.2), (60.0, 0.03), (60.0, 0.08), (5.0, 0.3)])
def test_truncation_length_reaches_target_on_worst_pair(k, r):
    """At the L chosen for the tight preset (accuracy 1e-7, admissibility 3)
    the discretised expansion reproduces G (relative to |G|) to within five
    times the target for two clusters of radius r at the admissibility limit,
    with x and y on the cluster spheres (facing each other, and at random
    positions; the (1/a)^L rate holds up to a constant of a few); three terms
    fewer miss it by more than twenty times, so the length is neither too
    short nor needlessly long.  green_expansion is
    pinned to G independently above."""
    t = preset("tight")
    X = t["admissibility"] * 2 * r * 1.0001
    L = ofmm.truncation_length(k, r, t, x_min=X)
    rng = np.random.default_rng(int(1000 * k * r))
    e = rng.standard_normal(3)
    e /= np.linalg.norm(e)
    z1, z2 = np.zeros(3), X * e

    def worst(LL):
        pts = [(z1 + r * e, z2 - r * e)]
        for _ in range(6):
            u, v = rng.standard_normal(3), rng.standard_normal(3)
            pts.append((z1 + r * u / np.linalg.norm(u), z2 + r * v / np.linalg.norm(v)))
        out = 0.0
        for x, y in pts:
            d = np.linalg.norm(x - y)
            gxy = np.exp(1j * k * d) / (4 * math.pi * d)
            out = max(out, abs(ofmm.green_expansion(k, x, y, z1, z2, LL) - gxy) / abs(gxy))
        return out

    assert worst(L) < 5 * t["fmm_eps"]
    assert worst(L - 3) > 20 * t["fmm_eps"]


def test_fmm_matches_dense_operator():
    nodes, tris = synth.icosphere(3)
    g = element_geometry(nodes, tris)
    k = 2 * math.pi / (6 * synth.mean_edge_length(nodes, tris))
    p = preset("tight", admissibility=2.0)
    F = ofmm.FMM(g, k, p, 2, 32)
    assert any(len(il) for L in F.tree.levels for il in L["il"])
    x = synth.complex_normal(len(tris), 4)
    rows = np.arange(0, len(tris), 37)
    Aref = op.rows(g, rows, k, p=preset("tight", admissibility=2.0, quad_eps=1e-12))
    mask = F.near_mask_rows(rows)
    y = (Aref * mask) @ x + F.apply(x)[rows]
    assert np.linalg.norm(y - Aref @ x) / np.linalg.norm(Aref @ x) < 1e-7


def test_level_rows_variant_matches_dense_operator():
    """The paper's level transfer (element-to-cluster rows on every level, no
    interpolation) on a 3-level tree whose two lower levels both carry
    interaction pairs: near part from converged dense rows + this far field
    reproduces the dense operator to the expansion accuracy, as the
    interpolating variant does."""
    nodes, tris = synth.icosphere(4)
    g = element_geometry(nodes, tris)
    k = 2 * math.pi / (6 * synth.mean_edge_length(nodes, tris))
    p = preset("tight", admissibility=2.0)
    F = ofmm.FMM(g, k, p, 3, 32, level_rows=True)
    levels_with_pairs = [l for l, L in enumerate(F.tree.levels) if any(len(il) for il in L["il"])]
    assert len(levels_with_pairs) >= 2
    x = synth.complex_normal(len(tris), 4)
    rows = np.arange(0, len(tris), 97)
    Aref = op.rows(g, rows, k, p=preset("tight", admissibility=2.0, quad_eps=1e-12))
    mask = F.near_mask_rows(rows)
    y = (Aref * mask) @ x + F.apply(x)[rows]
    assert np.linalg.norm(y - Aref @ x) / np.linalg.norm(Aref @ x) < 1e-7
