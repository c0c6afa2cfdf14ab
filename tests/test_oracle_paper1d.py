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


# ----------------------------------------------------------------------------
# single P2M / M2P operators of Table 1 against hand values and dense hats
# ----------------------------------------------------------------------------
def test_delta_operators_by_hand():
    """eq. (9): the particle interpolant at the nodes; eq. (10): the mesh
    interpolant at the particles.  Two particles at 0.1 (A = 1) and 0.6 (A = 3) on
    [0, 1) with nodes 0, 0.25, 0.5, 0.75: the interpolant rises by 2 over 0.5 and
    falls back over the wrap-around gap, so Abar = (1.4, 1.6, 2.6, 2.4).  Nodal
    values 0, 1, 2, 3 read at 0.125 and 0.9 give 0.5 and 3 - 3 * 0.6 = 1.2."""
    got = px.p2m_delta(np.array([0.6, 0.1]), np.array([3.0, 1.0]), 4)
    assert np.allclose(got, [1.4, 1.6, 2.6, 2.4], rtol=0, atol=1e-15)
    back = px.m2p_delta(np.array([0.125, 0.9]), np.array([0.0, 1.0, 2.0, 3.0]), 4)
    assert np.allclose(back, [0.5, 1.2], rtol=0, atol=1e-15)


def test_pic_and_flip_against_dense_hats():
    """eq. (11) with the mesh volume of eq. (5) (PIC: divide by h) and with the
    FLIP volume of eq. (12) (divide by sum v psi_i), built from a dense matrix of
    the mesh hats at the particles."""
    g = np.random.default_rng(11)
    n, N = 9, 23
    xp = g.uniform(0, 1, N)
    A = g.normal(size=N)
    v = px.particle_volumes(xp)
    H = np.zeros((n, N))                     # psi_i(x_mu) from the hat's closed form
    for i in range(n):
        for s in (-1, 0, 1):
            H[i] += np.maximum(0.0, 1.0 - np.abs(xp * n - i - s * n))
    b = H @ (v * A)
    assert np.allclose(px.p2m_pic(xp, A, n), b * n, rtol=1e-13, atol=1e-15)
    assert np.allclose(px.p2m_flip(xp, A, n), b / (H @ v), rtol=1e-13, atol=1e-15)
    # PIC conserves against the mesh volumes h, FLIP against the FLIP volumes
    assert abs(px.p2m_pic(xp, A, n).sum() / n - (v * A).sum()) < 1e-14
    assert abs(((H @ v) * px.p2m_flip(xp, A, n)).sum() - (v * A).sum()) < 1e-14


@pytest.mark.parametrize("quad", ["exact", "appB"])
def test_lumped_rows_on_regular_particles_closed_form(quad):
    """Particles on the nodes: the particle and mesh hats coincide, the overlap
    integrals are m A with m the consistent mass matrix (2h/3, h/6), and the
    Appendix-B rule is exact (no particle inside an element).  So the lumped P2M
    and the lumped M2P of Table 1 are each the (1, 4, 1)/6 average (eq. (17) with
    v = h), mass P2M returns A (preservation, eq. (18)), and the round trips are
    mass-lumped: (1,4,1)/6 once; lumped: twice."""
    n = 12
    x = np.arange(n) / n
    A = np.random.default_rng(7).normal(size=n)
    avg = (np.roll(A, 1) + 4.0 * A + np.roll(A, -1)) / 6.0
    assert np.allclose(px.p2m_lumped(x, A, n, quad=quad), avg, rtol=0, atol=1e-14)
    assert np.allclose(px.m2p_lumped(x, A, n, quad=quad), avg, rtol=0, atol=1e-14)
    assert np.allclose(px.p2m_mass(x, A, n, quad=quad), A, rtol=0, atol=1e-13)
    assert np.allclose(px.round_trip("mass_lumped", x, A, n, quad=quad), avg, rtol=0, atol=1e-13)
    avg2 = (np.roll(avg, 1) + 4.0 * avg + np.roll(avg, -1)) / 6.0
    assert np.allclose(px.round_trip("lumped", x, A, n, quad=quad), avg2, rtol=0, atol=1e-13)


def test_mass_lumped_round_trip_conserves_and_is_stable():
    """Sec. 2.4: the mass-lumped pair conserves (exact integrals: the mass P2M keeps
    int A, the lumped M2P keeps int Abar) and is stable: sum v Abarbar^2 <=
    int Abar^2 <= int A^2 = A^T m_part A (Cauchy-Schwarz with weight psi_mu, then
    the L2 projection)."""
    x = px.tophat_positions(60, distort=0.35, seed=8)
    n = 40
    A = ((x > 0.25) & (x < 0.75)).astype(float) + 0.3 * np.sin(2 * np.pi * x)
    v = px.particle_volumes(x)
    out = px.round_trip("mass_lumped", x, A, n, quad="exact")
    assert abs((v * out).sum() - (v * A).sum()) < 1e-14
    assert (v * out ** 2).sum() <= A @ px.particle_mass(x) @ A * (1 + 1e-14)
    # and it differs from mass-delta (the M2P differs)
    assert not np.allclose(out, px.round_trip("mass_delta", x, A, n, quad="exact"), atol=1e-6)
