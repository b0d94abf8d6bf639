"""Pins of the paper's own problems (Section 5.1) as the instances state them, and of the
oracle's constant-coefficient operators and hard-constraint factor.

Independent checks: the oscillator's closed form against a numerical ODE integration, the
Laplacian's forcing against finite differences of its solution, the trial-solution factor
against finite differences and its boundary zeros, the geometry of eq. dd, and the oracle's
solve reaching a small e_L1 on both problems."""
import numpy as np
import pytest
from scipy.integrate import solve_ivp

from oracle import assembly, solve
from paper_2506_17626_amd import instances as I


def test_oscillator_closed_form_against_ode_integration():
    inst = I.workload("oscillator1d")
    k, mu, m = inst.opcoef[0]
    t = np.linspace(0.0, 1.0, 201)
    sol = solve_ivp(lambda _, y: [y[1], -(mu * y[1] + k * y[0]) / m], (0.0, 1.0), [1.0, 0.0],
                    t_eval=t, rtol=1e-12, atol=1e-14, method="DOP853")
    assert np.max(np.abs(sol.y[0] - inst.exact(t[:, None]))) < 1e-8
    # the rows: interior ODE rows with rhs 0, then u(0) = 1 and u'(0) = 0
    assert np.all(inst.rowop[:-2] == I.OP_COEF) and np.all(inst.rhs[:-2] == 0.0)
    assert list(inst.rowop[-2:]) == [I.OP_VALUE, I.OP_COEF + 1]
    assert list(inst.rhs[-2:]) == [1.0, 0.0] and np.all(inst.x[-2:] == 0.0)
    assert inst.opcoef.tolist() == [[3600.0, 4.0, 1.0], [0.0, 1.0, 0.0]]
    assert inst.N - 2 == 20 * 8 and inst.test_grid == 1000


def test_multiscale_laplacian_forcing_and_boundary():
    inst = I.tiny("laplace2d_multiscale")
    # the forcing at the instance's own points against -Laplace of its exact solution
    e = 1e-4
    rows = np.all((inst.x > 0.05) & (inst.x < 0.95), axis=1)
    xi = inst.x[rows]
    lap = np.zeros(len(xi))
    for i in range(2):
        xp, xm = xi.copy(), xi.copy()
        xp[:, i] += e
        xm[:, i] -= e
        lap += (inst.exact(xp) - 2 * inst.exact(xi) + inst.exact(xm)) / e**2
    assert np.allclose(inst.rhs[rows], -lap, rtol=1e-5, atol=1e-4 * np.abs(lap).max())
    assert np.all(inst.rowop == I.OP_NEG_LAPLACE)
    # u = 0 on the boundary, and so is the trial-solution factor
    b = np.array([[0.0, 0.3], [1.0, 0.7], [0.4, 0.0], [0.6, 1.0]])
    assert np.allclose(inst.exact(b), 0.0, atol=1e-14)
    assert np.all(inst.ansatz(b)[:, 0] == 0.0)


def test_ansatz_factor_derivatives_finite_difference():
    inst = I.workload("laplace2d_multiscale")
    rng = np.random.default_rng(5)
    x = rng.uniform(0.02, 0.98, (40, 2))
    G = inst.ansatz(x)
    e = 1e-5
    for i in range(2):
        xp, xm = x.copy(), x.copy()
        xp[:, i] += e
        xm[:, i] -= e
        gp, gm = inst.ansatz(xp)[:, 0], inst.ansatz(xm)[:, 0]
        assert np.allclose((gp - gm) / (2 * e), G[:, 1 + i], rtol=1e-6, atol=1e-6)
        assert np.allclose((gp - 2 * G[:, 0] + gm) / e**2, G[:, 3 + i], rtol=1e-3, atol=1e-2)
    # away from the boundary the factor is 1 to within tanh(8 * 0.5)^4
    assert abs(inst.ansatz(np.array([[0.5, 0.5]]))[0, 0] - np.tanh(4.0) ** 4) < 1e-15


def test_paper_geometry_of_eq_dd():
    inst = I.workload("oscillator1d")
    S, delta = 20, 2.9
    assert np.allclose(inst.mu[:, 0], np.arange(S) / (S - 1))
    assert np.allclose(inst.hw, delta / (2 * (S - 1)))
    # the overlap ratio: a support spans delta spacings
    assert np.isclose(2 * inst.hw[0, 0] * (S - 1), delta)
    lap = I.workload("laplace2d_multiscale")
    assert lap.J == 256 and lap.N == 64 * 64 and lap.feat_off[-1] == 256 * 16
    assert lap.test_grid == 96


def test_coefficient_operator_rows_read_out_of_range_codes_as_values():
    """A code past the table is a value row (the C ABI's rule)."""
    inst = I.tiny("oscillator1d")
    rows, blocks, _ = assembly.assemble(inst)
    bad = I.tiny("oscillator1d")
    bad.rowop = bad.rowop.copy()
    bad.rowop[-1] = I.OP_COEF + 7
    val = I.tiny("oscillator1d")
    val.rowop = val.rowop.copy()
    val.rowop[-1] = I.OP_VALUE
    _, bb, _ = assembly.assemble(bad)
    _, bv, _ = assembly.assemble(val)
    for j in range(inst.J):
        assert np.array_equal(bb[j], bv[j])


@pytest.mark.parametrize("name,bound", [("oscillator1d", 1e-3), ("laplace2d_multiscale", 5e-2)])
def test_oracle_solves_the_paper_problems(name, bound):
    """The full oracle pipeline (filter at 1e-8, LSQR) reaches a small e_L1 on both."""
    inst = I.workload(name) if name == "oscillator1d" else I.tiny(name)
    sol = solve.solve(inst, tau=1e-8, atol=1e-12, btol=1e-12, maxit=10000)
    e = solve.l1_error(inst, sol.a)
    assert e < bound, e


def test_wave_trial_solution_meets_the_initial_and_boundary_conditions():
    """u~ = g u_hat + A: g and g_t vanish at t = 0 and g on the spatial boundary, so
    u~(x, 0) = A(x, 0), which is the Gaussian source inside the box, with A_t(x, 0) = 0;
    A vanishes on the spatial boundary."""
    inst = I.workload("wave2d")
    lam = inst.meta["lam"]
    rng = np.random.default_rng(6)
    xs = rng.uniform(-0.5, 0.5, (50, 2))
    x0 = np.concatenate([xs, np.zeros((50, 1))], axis=1)
    G = inst.ansatz(x0)
    assert np.all(G[:, 0] == 0.0) and np.all(G[:, 3] == 0.0)       # g(x,0) = g_t(x,0) = 0
    src = np.exp(-np.sum(xs * xs, axis=1) / (2 * lam**2))
    assert np.max(np.abs(inst.offset(x0) - src)) < 1e-4             # B = 1 - O(1e-5) inside
    e = 1e-5
    xp, xm = x0.copy(), x0.copy()
    xp[:, 2] += e
    xm[:, 2] -= e
    assert np.max(np.abs(inst.offset(xp) - inst.offset(xm))) / (2 * e) < 1e-8
    edge = np.array([[-1.0, 0.3, 0.5], [1.0, -0.2, 0.1], [0.4, -1.0, 0.9], [0.0, 1.0, 0.3]])
    assert np.all(inst.ansatz(edge)[:, 0] == 0.0) and np.all(inst.offset(edge) == 0.0)


def test_wave_rhs_is_minus_the_operator_image_of_the_additive_part():
    inst = I.tiny("wave2d")
    c2 = -1.0 / inst.opcoef[0, 6]
    x = inst.x[:: 7]
    e = 1e-4
    img = np.zeros(len(x))
    for i, coef in ((0, 1.0), (1, 1.0), (2, -1.0 / c2)):
        xp, xm = x.copy(), x.copy()
        xp[:, i] += e
        xm[:, i] -= e
        img += coef * (inst.offset(xp) - 2 * inst.offset(x) + inst.offset(xm)) / e**2
    rhs = inst.rhs[:: 7]
    assert np.allclose(rhs, -img, rtol=1e-5, atol=1e-5 * np.abs(img).max())
    assert inst.opcoef.tolist() == [[0.0, 0.0, 0.0, 0.0, 1.0, 1.0, -1.0]]


@pytest.mark.parametrize("name", ["laplace2d_multiscale", "wave2d"])
def test_every_ansatz_factor_against_finite_differences(name):
    inst = I.tiny(name)
    rng = np.random.default_rng(10)
    lo, hi = (inst.domain[:, 0], inst.domain[:, 1]) if inst.domain is not None else (0.0, 1.0)
    x = lo + (hi - lo) * rng.uniform(0.05, 0.95, (30, inst.d))
    G = inst.ansatz(x)
    d = inst.d
    e = 1e-5
    for i in range(d):
        xp, xm = x.copy(), x.copy()
        xp[:, i] += e
        xm[:, i] -= e
        gp, gm = inst.ansatz(xp)[:, 0], inst.ansatz(xm)[:, 0]
        scale = np.abs(G[:, 1 + d + i]).max() + np.abs(G[:, 1 + i]).max()
        assert np.allclose((gp - gm) / (2 * e), G[:, 1 + i], rtol=1e-6, atol=1e-7 * scale)
        assert np.allclose((gp - 2 * G[:, 0] + gm) / e**2, G[:, 1 + d + i], rtol=1e-3, atol=1e-4 * scale)


def test_box_geometry_of_eq_dd():
    inst = I.workload("wave2d")
    assert np.allclose(np.unique(inst.mu[:, 0]), -1 + 2 * np.arange(8) / 7)
    assert np.allclose(np.unique(inst.mu[:, 2]), np.arange(8) / 7)
    assert np.allclose(inst.hw[0], [2 * 2.9 / 14, 2 * 2.9 / 14, 2.9 / 14])
    xt = inst.test_points()
    assert xt.shape == (32**3, 3) and xt[:, :2].min() > -1 and xt[:, 2].max() < 1
