"""Pins of the paper-exact 1D oracle: Table 2 (Sec. 3.1) as printed, the closed-form
consistent mass matrices (Sec. 2.4: row sums equal the volumes), the Appendix-B
exactness statement, and numerical integration of the overlap integrals."""
import os

import numpy as np
import pytest

from oracle import paper1d as px

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "table2.txt")


def load_table2():
    rows = {}
    with open(GOLDEN) as fh:
        for line in fh:
            if line.startswith("#") or not line.strip():
                continue
            setup, method, e1, e2, l2 = line.split()
            rows[(setup, method)] = tuple(float(v) for v in (e1, e2, l2))
    return rows


def half_digit(printed):
    """Half a unit of the last printed digit of a value from the table."""
    s = f"{printed:g}"
    decimals = len(s.split(".")[1]) if "." in s else 0
    return 0.5 * 10.0 ** (-decimals)


TABLE2 = load_table2()


@pytest.fixture(scope="module")
def regular_runs():
    return {m: px.tophat_experiment(m) for m in ("delta", "flip", "mass_delta", "full_mass")}


@pytest.mark.parametrize("method", ["delta", "mass_delta", "full_mass"])
def test_table2_regular_column(regular_runs, method):
    r = regular_runs[method]
    e1, e2, l2 = TABLE2[("regular", method)]
    # "satisfied to machine precision by all methods for a regular particle arrangement"
    assert abs(r["E1"]) < 1e-10
    assert abs(100 * r["E2"] - e2) <= half_digit(e2)
    assert abs(100 * r["L2"] - l2) <= half_digit(l2)


def test_table2_regular_flip_equals_delta(regular_runs):
    """Sec. 3.1 states FLIP is equivalent to delta for the regular set-up; its printed
    L2 (35%) agrees, its printed E2 (-25%) does not match delta's -29% (a misprint
    under that statement), so FLIP is pinned to delta and to the printed L2."""
    f, d = regular_runs["flip"], regular_runs["delta"]
    assert np.max(np.abs(f["AT"] - d["AT"])) < 1e-12
    e1, _, l2 = TABLE2[("regular", "flip")]
    assert abs(f["E1"]) < 1e-10
    assert abs(100 * f["L2"] - l2) <= half_digit(l2)


@pytest.fixture(scope="module")
def distorted_runs():
    seeds = (100, 101, 102)
    out = {}
    for m in ("delta", "flip", "mass_delta", "full_mass"):
        rs = [px.tophat_experiment(m, distort=0.4, seed=s) for s in seeds]
        out[m] = {k: np.array([r[k] for r in rs]) for k in ("E1", "E2", "L2")}
    return out


def test_table2_distorted_column_statistically(distorted_runs):
    """The paper's +-40% distortion seed is unknown, so the right table is a
    statistical pin: magnitudes over three seeds against the printed values."""
    d = distorted_runs
    # FLIP conserves exactly even when distorted (E1 = 0 printed, Sec. 3.1)
    assert np.all(np.abs(d["flip"]["E1"]) < 1e-12)
    # the others conserve only approximately, at the printed percent level
    for m in ("delta", "mass_delta", "full_mass"):
        assert np.all(np.abs(d[m]["E1"]) < 0.02)
    # stability: every method loses second moment (E2 < 0) except full mass, which is near 0
    for m, (tol_e2, tol_l2) in dict(delta=(1.5, 1.0), mass_delta=(2.5, 1.0),
                                    full_mass=(2.5, 2.5)).items():
        _, e2, l2 = TABLE2[("distorted", m)]
        assert abs(100 * d[m]["E2"].mean() - e2) <= tol_e2, m
        assert abs(100 * d[m]["L2"].mean() - l2) <= tol_l2, m
    # full mass is the most accurate (Sec. 3.1 conclusion), mass-delta beats delta
    assert d["full_mass"]["L2"].mean() < d["mass_delta"]["L2"].mean() < d["delta"]["L2"].mean()
    assert np.all(d["flip"]["E2"] < 0) and np.all(d["delta"]["E2"] < 0)


def test_exact_quadrature_conserves():
    """With exact overlap integrals the mass methods conserve against v_i = h and the
    particle volumes (Sec. 2.4); the Appendix-B rule does not when particles are
    distorted (Sec. 3.1 remark on full mass)."""
    n = 40
    x = px.tophat_positions(40, distort=0.4, seed=5)
    A = ((x > 0.25) & (x < 0.75)).astype(float)
    v = px.particle_volumes(x)
    h = 1.0 / n
    Abar = px.p2m_mass(x, A, n, quad="exact")
    assert abs(h * Abar.sum() - (v * A).sum()) < 1e-14
    back = px.m2p_mass(x, Abar, n, quad="exact")
    assert abs((v * back).sum() - (v * A).sum()) < 1e-14
    Abar_q = px.p2m_mass(x, A, n, quad="appB")
    assert abs(h * Abar_q.sum() - (v * A).sum()) > 1e-6


def test_appendix_b_exact_without_particles_inside_elements():
    """Appendix B: if no particle lies inside an element, the parabola degenerates to
    the line and the rule is exact.  Particles on every node plus none inside."""
    n = 16
    x = np.arange(n) / n
    A = np.random.default_rng(1).normal(size=n)
    xn = px.nodes_1d(n)
    assert np.allclose(px.overlap_appendix_b(x, A, xn), px.overlap_exact(x, A, xn), atol=1e-15)
    # and with a coarser set of particles it is not
    xc = np.sort(np.random.default_rng(2).uniform(0, 1, 9))
    Ac = np.random.default_rng(3).normal(size=9)
    assert not np.allclose(px.overlap_appendix_b(xc, Ac, xn), px.overlap_exact(xc, Ac, xn), atol=1e-6)


def test_overlap_exact_against_numerical_integration():
    g = np.random.default_rng(4)
    xp = g.uniform(0, 1, 13)
    A = g.normal(size=13)
    xn = px.nodes_1d(7)
    q = (np.arange(400000) + 0.5) / 400000
    f = px.eval_pl(xp, A, q)
    H = px.hat_values(xn, q)
    num = (H * f).mean(axis=1)
    assert np.allclose(px.overlap_exact(xp, A, xn), num, atol=1e-9)


def test_consistent_mass_matrices():
    """Sec. 2.4: row sums of m are the volumes; 1D mesh spectrum h(2/3 + cos(th)/3) => kappa = 3."""
    n = 32
    m = px.mesh_mass(n)
    assert np.allclose(m.sum(1), 1.0 / n)
    ev = np.linalg.eigvalsh(m)
    assert abs(ev.max() / ev.min() - 3.0) < 1e-10
    x = np.random.default_rng(5).uniform(0, 1, 21)
    mp = px.particle_mass(x)
    assert np.allclose(mp.sum(1), px.particle_volumes(x))
    # against numerical integration of psi_mu psi_nu
    q = (np.arange(200000) + 0.5) / 200000
    H = px.hat_values(x, q)
    assert np.allclose(mp, (H @ H.T) / q.size, atol=1e-8)
    assert abs(px.particle_volumes(x).sum() - 1.0) < 1e-14


def test_lumped_rows_conserve():
    """Table 1 lumped rows conserve (Sec. 2.4: they satisfy conservativity and stability)."""
    x = px.tophat_positions(50, distort=0.3, seed=6)
    A = np.cos(2 * np.pi * x)
    v = px.particle_volumes(x)
    out = px.round_trip("lumped", x, A, 50, quad="exact")
    assert abs((v * out).sum() - (v * A).sum()) < 1e-13
    assert (v * out ** 2).sum() <= (v * A ** 2).sum()
