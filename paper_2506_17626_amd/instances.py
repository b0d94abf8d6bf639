"""Seeded synthetic problem instances for the ELM-FBPINN least-squares system.

This module only draws and lays out *inputs*: subdomain centres and
half-widths, random feature parameters, collocation points, per-row operator
ids, row weights and right-hand-side values, plus the manufactured exact
solution used to measure the error of a solve, and, for the paper's own problems,
the operator coefficients and the hard-constraint factor of the trial solution
(problem data, like the forcing).  It holds none of the method's arithmetic (no
window, feature or operator evaluation, no factorisation, no solver): both the
CPU oracle and the HIP path consume the arrays it returns.

Problem statement: a linear PDE with linear boundary operators (paper,
Section 2.1), discretised by a regular overlapping decomposition (Section 4.2,
eq. dd) with cosine windows (eq. used_window_function_nd) and random
one-hidden-layer features (eq. fcn_depth_h with h=1; tanh, or the sigmoid or sin of
Section 5's ablations), rows weighted as in
eq. ELMFBPINN_ls (interior rows by 1/sqrt(N_I), boundary set l by
sqrt(lambda_l / N_B^(l)) with lambda_l = 1).

Geometry reading (the paper parametrises overlap by a ratio delta, the
workloads by a fraction rho of the support width): S cells of width 1/S per
dimension, centres at the cell midpoints, half-width 1/(2 S (1-rho)), so two
neighbouring supports overlap by rho times the support width.  Interior
collocation points are owned by cells: a cell-centred grid of n points per
dimension inside every cell (uniform workloads), or c_j uniform random points
inside cell j (uneven workload).

Random numbers come from NumPy's Philox counter-based bit generator, read as
raw 64-bit words and mapped by explicit formulas (u = (z >> 11) * 2^-53,
U(a,b) = a + (b-a) u, U{lo..hi} = lo + floor(u (hi-lo+1)), N(0,1) by
Box-Muller) so that the streams do not depend on NumPy's distribution code.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field, replace

import numpy as np

# Row operator ids (shared vocabulary of the C ABI, see include/rfm.h).
OP_NEG_LAPLACE = 0   # -sum_i d_ii
OP_HEAT = 1          # d_t - kappa * sum_{spatial i} d_ii  (time is the last input dim)
OP_HELMHOLTZ = 2     # sum_i d_ii + k^2
OP_VALUE = 3         # identity (Dirichlet / initial-condition rows)
OP_COEF = 16         # + i: c0 + sum_i (c1_i d_i + c2_i d_ii), row i of Instance.opcoef


class Rng:
    """Counter-based generator with explicit, version-independent mappings."""

    def __init__(self, seed: int, stream: int = 0):
        self._bg = np.random.Philox(key=np.array([seed, stream], dtype=np.uint64))

    def uniform01(self, n: int) -> np.ndarray:
        z = self._bg.random_raw(int(n)).astype(np.uint64)
        return (z >> np.uint64(11)).astype(np.float64) * (2.0 ** -53)

    def uniform(self, lo: float, hi: float, n: int) -> np.ndarray:
        return lo + (hi - lo) * self.uniform01(n)

    def integers(self, lo: int, hi: int, n: int) -> np.ndarray:
        """Inclusive range lo..hi."""
        u = self.uniform01(n)
        return (lo + np.floor(u * (hi - lo + 1))).astype(np.int64)

    def normal(self, n: int) -> np.ndarray:
        m = (int(n) + 1) // 2
        u1 = self.uniform01(m)
        u2 = self.uniform01(m)
        u1 = np.where(u1 <= 0.0, 2.0 ** -53, u1)
        rad = np.sqrt(-2.0 * np.log(u1))
        z = np.concatenate([rad * np.cos(2 * np.pi * u2), rad * np.sin(2 * np.pi * u2)])
        return z[: int(n)]


@dataclass
class Instance:
    """All inputs of one least-squares problem (arrays are host numpy)."""

    name: str
    d: int
    J: int
    mu: np.ndarray          # [J, d] subdomain centres
    hw: np.ndarray          # [J, d] subdomain half-widths
    feat_off: np.ndarray    # [J+1] int64 prefix sums of K_j
    w: np.ndarray           # [sum K, d] feature weights (act on normalised input)
    b: np.ndarray           # [sum K] feature biases
    x: np.ndarray           # [N, d] collocation and boundary points
    rowop: np.ndarray       # [N] int32 operator id per row
    weight: np.ndarray      # [N] row scale s_r
    rhs: np.ndarray         # [N] unscaled right-hand side value per row
    kappa: float = 0.0      # diffusion constant of OP_HEAT rows
    ksq: float = 0.0        # k^2 of OP_HELMHOLTZ rows
    exact: object = None    # callable u(x[N,d]) -> [N]
    test_grid: int = 0      # points per dim of the cell-centred test grid
    meta: dict = field(default_factory=dict)
    activation: str = "tanh"  # feature activation: "tanh", "sigmoid" or "sin"
    opcoef: np.ndarray | None = None  # [nop, 1+2d] c0, c1_i, c2_i of the OP_COEF + i rows
    ansatz: object = None   # callable x[n,d] -> [n, 1+2d]: g, d_i g, d_ii g of u~ = g u_hat
    depth: int = 1          # h of the subdomain networks; > 1: hidden layers of width `hidden`
    hidden: int = 0
    net: np.ndarray | None = None  # [J, H d + H + (h-2)(H H + H)] hidden parameters per subdomain
    domain: np.ndarray | None = None  # [d, 2] box (lo, hi) per dim; None = the unit cube
    offset: object = None   # callable x[n,d] -> [n]: additive part of the trial solution

    @property
    def N(self) -> int:
        return int(self.x.shape[0])

    @property
    def K(self) -> np.ndarray:
        return np.diff(self.feat_off)

    def test_points(self, n: int | None = None) -> np.ndarray:
        n = self.test_grid if n is None else n
        g = (np.arange(n) + 0.5) / n
        mesh = np.meshgrid(*([g] * self.d), indexing="ij")
        x = np.stack([m.ravel() for m in mesh], axis=1)
        if self.domain is not None:
            x = self.domain[:, 0] + x * (self.domain[:, 1] - self.domain[:, 0])
        return x


# ---------------------------------------------------------------- geometry
def _regular_geometry(d: int, S: int, rho: float):
    h = 1.0 / S
    centres_1d = (np.arange(S) + 0.5) * h
    half = h / (2.0 * (1.0 - rho))
    idx = np.stack(np.meshgrid(*([np.arange(S)] * d), indexing="ij"), axis=-1).reshape(-1, d)
    mu = centres_1d[idx]
    hw = np.full_like(mu, half)
    return mu, hw, idx


def _cell_grid_points(d: int, S: int, n: int) -> np.ndarray:
    """Cell-centred grid of n points per dim per cell, ordered cell by cell."""
    h = 1.0 / S
    local = (np.arange(n) + 0.5) / n * h
    lmesh = np.stack(np.meshgrid(*([local] * d), indexing="ij"), axis=-1).reshape(-1, d)
    cells = np.stack(np.meshgrid(*([np.arange(S)] * d), indexing="ij"), axis=-1).reshape(-1, d)
    pts = (cells[:, None, :] * h + lmesh[None, :, :]).reshape(-1, d)
    return pts


def _features(rng: Rng, K: np.ndarray, d: int):
    feat_off = np.concatenate([[0], np.cumsum(K)]).astype(np.int64)
    total = int(feat_off[-1])
    w = rng.uniform(-1.0, 1.0, total * d).reshape(total, d)
    b = rng.uniform(-1.0, 1.0, total)
    return feat_off, w, b


def _paper_geometry(d: int, S: int, delta: float, box=None):
    """eq. dd on a box (default [0,1]^d): centres a + (b-a)(j-1)/(S-1) per dim, half-width
    (b-a) delta / (2 (S-1))."""
    box = np.array([[0.0, 1.0]] * d) if box is None else np.asarray(box, dtype=np.float64)
    idx = np.stack(np.meshgrid(*([np.arange(S)] * d), indexing="ij"), axis=-1).reshape(-1, d)
    span = box[:, 1] - box[:, 0]
    mu = box[None, :, 0] + span[None, :] * idx / (S - 1)
    hw = np.broadcast_to(span * delta / (2.0 * (S - 1)), mu.shape).copy()
    return mu, hw


def _full_grid(d: int, n: int, ends: bool) -> np.ndarray:
    """Regular grid of n points per dim over [0,1]^d (Section 5, interior collocation points):
    end points included, or cell-centred so that no point lies on the boundary, where a
    hard-constraint factor vanishes and would leave a zero row (the paper asks for a square
    or tall M)."""
    g = np.linspace(0.0, 1.0, n) if ends else (np.arange(n) + 0.5) / n
    return np.stack(np.meshgrid(*([g] * d), indexing="ij"), axis=-1).reshape(-1, d)


def _face_grid(n: int) -> np.ndarray:
    return (np.arange(n) + 0.5) / n


# ---------------------------------------------------------------- problems
def poisson1d(S=20, K=64, n=100, rho=0.3, seed=0, name="poisson1d") -> Instance:
    """-u'' = f on [0,1], u = sin(2 pi x) + 0.1 sin(50 pi x), Dirichlet at both ends."""
    d = 1
    rng = Rng(seed)
    mu, hw, _ = _regular_geometry(d, S, rho)
    feat_off, w, b = _features(rng, np.full(S, K, dtype=np.int64), d)
    xi = _cell_grid_points(d, S, n)
    xb = np.array([[0.0], [1.0]])

    def exact(x):
        return np.sin(2 * np.pi * x[:, 0]) + 0.1 * np.sin(50 * np.pi * x[:, 0])

    def forcing(x):
        return 4 * np.pi**2 * np.sin(2 * np.pi * x[:, 0]) + 250 * np.pi**2 * np.sin(50 * np.pi * x[:, 0])

    NI, NB = xi.shape[0], xb.shape[0]
    x = np.concatenate([xi, xb])
    rowop = np.concatenate([np.full(NI, OP_NEG_LAPLACE), np.full(NB, OP_VALUE)]).astype(np.int32)
    weight = np.concatenate([np.full(NI, 1 / math.sqrt(NI)), np.full(NB, 1 / math.sqrt(NB))])
    rhs = np.concatenate([forcing(xi), exact(xb)])
    return Instance(name, d, S, mu, hw, feat_off, w, b, x, rowop, weight, rhs,
                    exact=exact, test_grid=1000, meta=dict(S=S, K=K, n=n, rho=rho, seed=seed))


def _square_boundary(nb: int) -> np.ndarray:
    """nb cell-centred points on each of the four edges of [0,1]^2 (no corners)."""
    g = _face_grid(nb)
    z, o = np.zeros(nb), np.ones(nb)
    return np.concatenate([np.stack([g, z], 1), np.stack([g, o], 1),
                           np.stack([z, g], 1), np.stack([o, g], 1)])


def _u2d(x):
    return (np.sin(2 * np.pi * x[:, 0]) * np.sin(2 * np.pi * x[:, 1])
            + 0.05 * np.sin(40 * np.pi * x[:, 0]) * np.sin(40 * np.pi * x[:, 1]))


def poisson2d(S=16, K=256, n=20, rho=0.25, nb=200, seed=0, name="poisson2d") -> Instance:
    """-Laplace u = f on [0,1]^2, u = sin2pix sin2piy + 0.05 sin40pix sin40piy, u=0 on the boundary."""
    d = 2
    rng = Rng(seed)
    mu, hw, _ = _regular_geometry(d, S, rho)
    feat_off, w, b = _features(rng, np.full(S * S, K, dtype=np.int64), d)
    xi = _cell_grid_points(d, S, n)
    xb = _square_boundary(nb)

    def forcing(x):
        return (8 * np.pi**2 * np.sin(2 * np.pi * x[:, 0]) * np.sin(2 * np.pi * x[:, 1])
                + 160 * np.pi**2 * np.sin(40 * np.pi * x[:, 0]) * np.sin(40 * np.pi * x[:, 1]))

    NI, NB = xi.shape[0], xb.shape[0]
    x = np.concatenate([xi, xb])
    rowop = np.concatenate([np.full(NI, OP_NEG_LAPLACE), np.full(NB, OP_VALUE)]).astype(np.int32)
    weight = np.concatenate([np.full(NI, 1 / math.sqrt(NI)), np.full(NB, 1 / math.sqrt(NB))])
    rhs = np.concatenate([forcing(xi), _u2d(xb)])
    return Instance(name, d, S * S, mu, hw, feat_off, w, b, x, rowop, weight, rhs,
                    exact=_u2d, test_grid=200, meta=dict(S=S, K=K, n=n, rho=rho, nb=nb, seed=seed))


def heat3d(S=8, K=300, n=12, rho=0.2, nb=96, kappa=0.01, seed=0, name="heat3d") -> Instance:
    """u_t = kappa Laplace u on [0,1]^2 x [0,1] (x, y, t); initial condition at t=0,
    u=0 on the four lateral faces, no condition at t=1."""
    d = 3
    rng = Rng(seed)
    mu, hw, _ = _regular_geometry(d, S, rho)
    feat_off, w, b = _features(rng, np.full(S**3, K, dtype=np.int64), d)
    xi = _cell_grid_points(d, S, n)
    g = _face_grid(nb)
    A, B = np.meshgrid(g, g, indexing="ij")
    A, B = A.ravel(), B.ravel()
    z, o = np.zeros_like(A), np.ones_like(A)
    x_ic = np.stack([A, B, z], 1)
    x_lat = np.concatenate([np.stack([z, A, B], 1), np.stack([o, A, B], 1),
                            np.stack([A, z, B], 1), np.stack([A, o, B], 1)])

    def exact(x):
        X, Y, T = x[:, 0], x[:, 1], x[:, 2]
        return (np.exp(-8 * np.pi**2 * kappa * T) * np.sin(2 * np.pi * X) * np.sin(2 * np.pi * Y)
                + 0.1 * np.exp(-800 * np.pi**2 * kappa * T) * np.sin(20 * np.pi * X) * np.sin(20 * np.pi * Y))

    NI, N1, N2 = xi.shape[0], x_ic.shape[0], x_lat.shape[0]
    x = np.concatenate([xi, x_ic, x_lat])
    rowop = np.concatenate([np.full(NI, OP_HEAT), np.full(N1 + N2, OP_VALUE)]).astype(np.int32)
    weight = np.concatenate([np.full(NI, 1 / math.sqrt(NI)), np.full(N1, 1 / math.sqrt(N1)),
                             np.full(N2, 1 / math.sqrt(N2))])
    rhs = np.concatenate([np.zeros(NI), exact(x_ic), np.zeros(N2)])
    return Instance(name, d, S**3, mu, hw, feat_off, w, b, x, rowop, weight, rhs, kappa=kappa,
                    exact=exact, test_grid=64, meta=dict(S=S, K=K, n=n, rho=rho, nb=nb, seed=seed))


def helmholtz2d_uneven(S=64, Klo=96, Khi=320, clo=150, chi=500, rho=0.25, k=20.0, seed=0,
                       name="helmholtz2d_uneven") -> Instance:
    """Laplace u + k^2 u = f on [0,1]^2 with C2's manufactured u, u=0 on the boundary;
    per-cell feature counts K_j ~ U{Klo..Khi}, interior points c_j ~ U{clo..chi} uniform in
    cell j, and every boundary cell adds ceil(sqrt(c_j)) uniform points on each domain edge
    it touches."""
    d = 2
    rng = Rng(seed)
    mu, hw, idx = _regular_geometry(d, S, rho)
    J = S * S
    K = rng.integers(Klo, Khi, J)
    feat_off, w, b = _features(rng, K, d)
    c = rng.integers(clo, chi, J)
    h = 1.0 / S
    xi_parts, xb_parts = [], []
    for j in range(J):
        cx, cy = idx[j]
        u = rng.uniform01(2 * c[j]).reshape(c[j], 2)
        xi_parts.append(np.stack([(cx + u[:, 0]) * h, (cy + u[:, 1]) * h], 1))
        nbj = int(math.ceil(math.sqrt(c[j])))
        for axis, side, at in ((1, 0, 0.0), (1, S - 1, 1.0), (0, 0, 0.0), (0, S - 1, 1.0)):
            if idx[j][axis] != side:
                continue
            t = rng.uniform01(nbj)
            other = idx[j][1 - axis]
            p = np.empty((nbj, 2))
            p[:, axis] = at
            p[:, 1 - axis] = (other + t) * h
            xb_parts.append(p)
    xi = np.concatenate(xi_parts)
    xb = np.concatenate(xb_parts)
    ksq = k * k

    def forcing(x):
        s1 = np.sin(2 * np.pi * x[:, 0]) * np.sin(2 * np.pi * x[:, 1])
        s2 = np.sin(40 * np.pi * x[:, 0]) * np.sin(40 * np.pi * x[:, 1])
        return (-8 * np.pi**2 + ksq) * s1 + 0.05 * (-3200 * np.pi**2 + ksq) * s2

    NI, NB = xi.shape[0], xb.shape[0]
    x = np.concatenate([xi, xb])
    rowop = np.concatenate([np.full(NI, OP_HELMHOLTZ), np.full(NB, OP_VALUE)]).astype(np.int32)
    weight = np.concatenate([np.full(NI, 1 / math.sqrt(NI)), np.full(NB, 1 / math.sqrt(NB))])
    rhs = np.concatenate([forcing(xi), _u2d(xb)])
    return Instance(name, d, J, mu, hw, feat_off, w, b, x, rowop, weight, rhs, ksq=ksq,
                    exact=_u2d, test_grid=400,
                    meta=dict(S=S, Klo=Klo, Khi=Khi, clo=clo, chi=chi, rho=rho, k=k, seed=seed))


def poisson2d_family_params(n: int, seed: int, nmodes: int = 4, maxfreq: int = 30) -> np.ndarray:
    """Parameters of the parametric Poisson family: rows [a_1..a_4, m_1..m_4, n_1..n_4]."""
    rng = Rng(seed, stream=1)
    a = rng.normal(n * nmodes).reshape(n, nmodes)
    m = rng.integers(1, maxfreq, n * nmodes).reshape(n, nmodes)
    k = rng.integers(1, maxfreq, n * nmodes).reshape(n, nmodes)
    return np.concatenate([a, m.astype(np.float64), k.astype(np.float64)], axis=1)


def poisson2d_family_rhs(inst: Instance, params: np.ndarray) -> np.ndarray:
    """Unscaled right-hand sides [n_params, N] of -Laplace u = sum a_k sin(m_k pi x) sin(n_k pi y),
    u = 0 on the boundary, on the rows of a poisson2d instance."""
    nm = params.shape[1] // 3
    a, m, k = params[:, :nm], params[:, nm:2 * nm], params[:, 2 * nm:]
    interior = inst.rowop == OP_NEG_LAPLACE
    X, Y = inst.x[:, 0], inst.x[:, 1]
    out = np.zeros((params.shape[0], inst.N))
    for q in range(nm):
        out += a[:, q:q + 1] * np.sin(m[:, q:q + 1] * np.pi * X) * np.sin(k[:, q:q + 1] * np.pi * Y)
    out[:, ~interior] = 0.0
    return out


def poisson2d_family_exact(params_row: np.ndarray):
    nm = params_row.shape[0] // 3
    a, m, k = params_row[:nm], params_row[nm:2 * nm], params_row[2 * nm:]

    def exact(x):
        u = np.zeros(x.shape[0])
        for q in range(nm):
            u += a[q] * np.sin(m[q] * np.pi * x[:, 0]) * np.sin(k[q] * np.pi * x[:, 1]) / ((m[q]**2 + k[q]**2) * np.pi**2)
        return u
    return exact


# ---------------------------------------------------------------- named workloads
def oscillator1d(S=20, K=8, omega0=60.0, mu_f=4.0, m=1.0, delta=2.9, seed=0,
                 name="oscillator1d") -> Instance:
    """Damped harmonic oscillator (Section 5.1): m u'' + mu u' + k u = 0 on [0,1] with
    k = m omega0^2, u(0) = 1, u'(0) = 0, under-damped (mu / 2m < omega0).  Exact solution
    u = e^{-dt} cos(w t + p) / cos p with d = mu / 2m, w = sqrt(omega0^2 - d^2) and
    tan p = -d / w.  Interior points: S K on the regular grid; two boundary sets of one row
    each (the value and the velocity at t = 0); test points 50 S."""
    d = 1
    rng = Rng(seed)
    mu, hw = _paper_geometry(d, S, delta)
    feat_off, w, b = _features(rng, np.full(S, K, dtype=np.int64), d)
    k = m * omega0**2
    dmp = mu_f / (2.0 * m)
    om = math.sqrt(omega0**2 - dmp**2)
    ph = math.atan(-dmp / om)

    def exact(x):
        t = x[:, 0]
        return np.exp(-dmp * t) * np.cos(om * t + ph) / math.cos(ph)

    xi = _full_grid(d, S * math.ceil(K), ends=True)
    xb = np.zeros((2, 1))
    NI = xi.shape[0]
    x = np.concatenate([xi, xb])
    rowop = np.concatenate([np.full(NI, OP_COEF + 0), [OP_VALUE, OP_COEF + 1]]).astype(np.int32)
    weight = np.concatenate([np.full(NI, 1 / math.sqrt(NI)), [1.0, 1.0]])
    rhs = np.concatenate([np.zeros(NI), [1.0, 0.0]])
    opcoef = np.array([[k, mu_f, m],      # m u'' + mu u' + k u
                       [0.0, 1.0, 0.0]])  # u'
    return Instance(name, d, S, mu, hw, feat_off, w, b, x, rowop, weight, rhs, exact=exact,
                    test_grid=50 * S, opcoef=opcoef,
                    meta=dict(S=S, K=K, omega0=omega0, mu=mu_f, m=m, delta=delta, seed=seed))


def _box_factor(a: float, x: np.ndarray):
    """F(x) = tanh(a x) tanh(a (1 - x)) and its first two derivatives."""
    p, q = np.tanh(a * x), np.tanh(a * (1.0 - x))
    p1, q1 = a * (1.0 - p * p), -a * (1.0 - q * q)
    p2, q2 = -2.0 * a * p * p1, 2.0 * a * q * q1
    return p * q, p1 * q + p * q1, p2 * q + 2.0 * p1 * q1 + p * q2


def laplace2d_multiscale(S=16, K=16, n=3, delta=2.9, seed=0, name="laplace2d_multiscale") -> Instance:
    """Multi-scale Laplacian (Section 5.1): -Laplace u = f on [0,1]^2, u = 0 on the boundary,
    u = (1/n) sum_{i<=n} sin(w_i pi x) sin(w_i pi y) with w_i = 2^i, f = -Laplace u.  The
    boundary condition is imposed by the hard-constraint trial solution u~ = g u_hat with
    g = F(x) F(y), F(s) = tanh(w_n s) tanh(w_n (1 - s)), so every row is a PDE row
    ((S ceil(sqrt K))^2 of them on the regular grid); test points 6 S per dim."""
    d = 2
    rng = Rng(seed)
    mu, hw = _paper_geometry(d, S, delta)
    feat_off, w, b = _features(rng, np.full(S * S, K, dtype=np.int64), d)
    om = 2.0 ** np.arange(1, n + 1)

    def exact(x):
        return np.mean([np.sin(o * np.pi * x[:, 0]) * np.sin(o * np.pi * x[:, 1]) for o in om], axis=0)

    def forcing(x):
        return np.mean([2 * (o * np.pi) ** 2 * np.sin(o * np.pi * x[:, 0]) * np.sin(o * np.pi * x[:, 1])
                        for o in om], axis=0)

    a = float(om[-1])

    def ansatz(x):
        F0, F0d, F0dd = _box_factor(a, x[:, 0])
        F1, F1d, F1dd = _box_factor(a, x[:, 1])
        return np.stack([F0 * F1, F0d * F1, F0 * F1d, F0dd * F1, F0 * F1dd], axis=1)

    xi = _full_grid(d, S * math.ceil(math.sqrt(K)), ends=False)
    NI = xi.shape[0]
    rowop = np.full(NI, OP_NEG_LAPLACE, dtype=np.int32)
    weight = np.full(NI, 1 / math.sqrt(NI))
    return Instance(name, d, S * S, mu, hw, feat_off, w, b, xi, rowop, weight, forcing(xi),
                    exact=exact, test_grid=6 * S, ansatz=ansatz,
                    meta=dict(S=S, K=K, n=n, delta=delta, seed=seed))


def _tanh_pair(a: float, lo: float, hi: float, x: np.ndarray):
    """F(x) = tanh(a (x - lo)) tanh(a (hi - x)), zero at both ends, and F', F''."""
    p, q = np.tanh(a * (x - lo)), np.tanh(a * (hi - x))
    p1, q1 = a * (1.0 - p * p), -a * (1.0 - q * q)
    p2, q2 = -2.0 * a * p * p1, 2.0 * a * q * q1
    return p * q, p1 * q + p * q1, p2 * q + 2.0 * p1 * q1 + p * q2


def wave2d(S=8, K=8, lam=0.2, c=1.0, delta=2.9, seed=0, name="wave2d") -> Instance:
    """Acoustic wave in (2+1)D (Section 5.1): Laplace_x u - c^-2 u_tt = 0 on [-1,1]^2 x [0,1],
    u = 0 on the spatial boundary, u(x,0) = exp(-|x|^2 / (2 lam^2)), u_t(x,0) = 0, through the
    hard-constraint trial solution u~ = B(x) (G(x,t) + tanh^2(t/tau) u_hat) with
    B = prod_i tanh((1 + x_i)/d) tanh((1 - x_i)/d), G = exp(-((0.6 t/tau)^2 + |x|^2/lam^2)/2),
    d = lam/2.5, tau = lam/(2.5 c).  Linear in the coefficients: u~ = g u_hat + A with the
    factor g = B tanh^2(t/tau) and the additive part A = B G, whose operator image goes to the
    right-hand side (rhs = -Op[A]).  No closed-form solution (the paper compares against a
    finite-difference solver).  Points: (S ceil(K^(1/3)))^3 on the cell-centred grid (g = 0 on
    the spatial boundary and at t = 0)."""
    d3 = 3
    rng = Rng(seed)
    box = np.array([[-1.0, 1.0], [-1.0, 1.0], [0.0, 1.0]])
    mu, hw = _paper_geometry(d3, S, delta, box)
    feat_off, w, b = _features(rng, np.full(S**3, K, dtype=np.int64), d3)
    dl, tau = lam / 2.5, lam / (2.5 * c)
    kap = 0.18 / tau**2                       # (0.6/tau)^2 / 2

    def spatial(s):
        """P = F e with e = exp(-s^2 / (2 lam^2)): values, first and second derivatives."""
        F, F1, F2 = _tanh_pair(1.0 / dl, -1.0, 1.0, s)
        e = np.exp(-s * s / (2 * lam**2))
        e1 = -s / lam**2 * e
        e2 = (s * s / lam**4 - 1.0 / lam**2) * e
        return (F, F1, F2), (F * e, F1 * e + F * e1, F2 * e + 2 * F1 * e1 + F * e2)

    def ansatz(x):
        (F0, F01, F02), _ = spatial(x[:, 0])
        (F1, F11, F12), _ = spatial(x[:, 1])
        q = np.tanh(x[:, 2] / tau)
        q1 = (1.0 - q * q) / tau
        Q, Q1, Q2 = q * q, 2 * q * q1, 2 * q1 * q1 - 4 * q * q * q1 / tau
        return np.stack([F0 * F1 * Q, F01 * F1 * Q, F0 * F11 * Q, F0 * F1 * Q1,
                         F02 * F1 * Q, F0 * F12 * Q, F0 * F1 * Q2], axis=1)

    def offset(x):
        _, (P0, _, _) = spatial(x[:, 0])
        _, (P1, _, _) = spatial(x[:, 1])
        return P0 * P1 * np.exp(-kap * x[:, 2] ** 2)

    def offset_image(x):
        """Laplace_x A - c^-2 A_tt for A = P(x1) P(x2) T(t), T = exp(-kap t^2)."""
        _, (P0, _, P02) = spatial(x[:, 0])
        _, (P1, _, P12) = spatial(x[:, 1])
        t = x[:, 2]
        T = np.exp(-kap * t * t)
        T2 = (4 * kap * kap * t * t - 2 * kap) * T
        return P02 * P1 * T + P0 * P12 * T - P0 * P1 * T2 / c**2

    n = S * math.ceil(round(K ** (1.0 / 3.0), 12))
    xi = box[:, 0] + _full_grid(d3, n, ends=False) * (box[:, 1] - box[:, 0])
    NI = xi.shape[0]
    rowop = np.full(NI, OP_COEF + 0, dtype=np.int32)
    weight = np.full(NI, 1 / math.sqrt(NI))
    opcoef = np.array([[0.0, 0.0, 0.0, 0.0, 1.0, 1.0, -1.0 / c**2]])
    return Instance(name, d3, S**3, mu, hw, feat_off, w, b, xi, rowop, weight, -offset_image(xi),
                    test_grid=4 * S, opcoef=opcoef, ansatz=ansatz, domain=box, offset=offset,
                    meta=dict(S=S, K=K, lam=lam, c=c, delta=delta, seed=seed))


def workload(name: str, seed: int = 0) -> Instance:
    """The five named workloads at their full sizes."""
    if name == "poisson1d":       # 20 subdomains, 64 features, 100 points each
        return poisson1d(seed=seed)
    if name == "poisson2d":       # 16x16 subdomains, 256 features, 20x20 points each
        return poisson2d(seed=seed)
    if name == "heat3d":          # 8x8x8 subdomains, 300 features, 12^3 points each
        return heat3d(seed=seed)
    if name == "helmholtz2d_uneven":  # 64x64 subdomains, uneven sizes
        return helmholtz2d_uneven(seed=seed)
    if name == "poisson2d_family":    # geometry of poisson2d; RHS from poisson2d_family_rhs
        return poisson2d(seed=seed, name="poisson2d_family")
    if name == "oscillator1d":        # the paper's oscillator baseline: S=20, K=8, omega0=60
        return oscillator1d(seed=seed)
    if name == "laplace2d_multiscale":  # the paper's Laplacian baseline: S=16, K=16, n=3
        return laplace2d_multiscale(seed=seed)
    if name == "wave2d":              # the paper's wave baseline: S=8, K=8, lambda=0.2
        return wave2d(seed=seed)
    raise KeyError(name)


def with_activation(inst: Instance, activation: str) -> Instance:
    """The same instance with the features' activation replaced (Section 5's ablations:
    the sigmoid and sin in place of tanh); weights, biases and points are unchanged."""
    if activation not in ("tanh", "sigmoid", "sin"):
        raise ValueError(f"unknown activation {activation!r}")
    return replace(inst, activation=activation, name=f"{inst.name}_{activation}")


def with_depth(inst: Instance, depth: int, hidden: int, seed: int = 0) -> Instance:
    """The same instance with depth-h subdomain networks (eq. fcn_depth_h; Section 5's
    ablations use h = 3 and 5): h-1 hidden layers of width `hidden` per subdomain, and the
    features acting on the last of them.  Weights uniform LeCun (U(-sqrt(3/fan_in),
    sqrt(3/fan_in)), Section 5, network architecture), biases U(-1,1) as for depth 1."""
    if depth <= 1:
        return inst
    rng = Rng(seed, 11)
    H, d = hidden, inst.d
    lim = lambda fan_in: math.sqrt(3.0 / fan_in)
    rows = []
    for _ in range(inst.J):
        parts = [rng.uniform(-lim(d), lim(d), H * d), rng.uniform(-1.0, 1.0, H)]
        for _ in range(depth - 2):
            parts += [rng.uniform(-lim(H), lim(H), H * H), rng.uniform(-1.0, 1.0, H)]
        rows.append(np.concatenate(parts))
    n = int(inst.feat_off[-1])
    w = rng.uniform(-lim(H), lim(H), n * H).reshape(n, H)
    b = rng.uniform(-1.0, 1.0, n)
    return replace(inst, depth=depth, hidden=H, net=np.stack(rows), w=w, b=b,
                   name=f"{inst.name}_h{depth}")


def tiny(name: str, seed: int = 0) -> Instance:
    """Small variants (several blocks, ragged sizes) that the oracle finishes in well under a second."""
    if name == "poisson1d":
        return poisson1d(S=5, K=24, n=30, seed=seed, name="poisson1d_tiny")
    if name == "poisson2d":
        return poisson2d(S=3, K=40, n=7, nb=21, seed=seed, name="poisson2d_tiny")
    if name == "heat3d":
        return heat3d(S=2, K=48, n=5, nb=10, seed=seed, name="heat3d_tiny")
    if name == "helmholtz2d_uneven":
        return helmholtz2d_uneven(S=4, Klo=20, Khi=70, clo=20, chi=90, seed=seed, name="helmholtz2d_uneven_tiny")
    if name == "oscillator1d":
        return oscillator1d(S=6, K=8, omega0=15.0, seed=seed, name="oscillator1d_tiny")
    if name == "laplace2d_multiscale":
        return laplace2d_multiscale(S=4, K=9, n=2, seed=seed, name="laplace2d_multiscale_tiny")
    if name == "wave2d":
        return wave2d(S=3, K=8, lam=0.5, seed=seed, name="wave2d_tiny")
    raise KeyError(name)
