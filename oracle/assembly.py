"""Oracle: supports, windows, features and the weighted global least-squares rows.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

Follows the paper's statement of the discretised problem:
* ansatz u(x) = sum_j w_j(x) sum_k a_jk phi_jk(x)            (eq. elm_solution)
* phi_jk = Xi(w_jk . xn + b_jk) on the input normalised to [-1,1] over the
  subdomain (eq. fcn_depth_h with depth 1; Section 4.2, network architecture), with the
  activation Xi = tanh (every baseline of Section 5) or the sigmoid or sin of the ablation
  rows of Section 5's results tables
* w_j = what_j / sum_i what_i with
  what_j = prod_d (1 + cos(pi (x_d - mu_jd) / sigma_jd))^2 on |x_d - mu_jd| < sigma_jd
  (eq. used_window_function_nd, with the parenthesis read as (x - mu)/sigma)
* row r of M for column (j,k): s_r * Op_r[w_j phi_jk](x_r); h_r = s_r * rhs_r
  (eq. ELMFBPINN_ls and the component-wise definition of N and B); with a
  hard-constraint trial solution u~ = g u_hat (Section 5.1) the operator acts on
  g w_j phi_jk, still linear in the coefficients
* I_j = rows where w_j(x_r) != 0, blocks M_j = M|_{I_j x K_j}  (eq. DomainDecomp)

Derivatives are written out by hand (chain, product and quotient rules); the
pins in ``tests/test_oracle_assembly.py`` check them against finite
differences, partition-of-unity identities and closed forms.
"""
from __future__ import annotations

import numpy as np

OP_NEG_LAPLACE, OP_HEAT, OP_HELMHOLTZ, OP_VALUE = 0, 1, 2, 3
OP_COEF = 16   # + i: constant-coefficient operator i, c0 u + sum_a (c1_a d_a u + c2_a d_aa u)


def support_mask(x: np.ndarray, mu_j: np.ndarray, hw_j: np.ndarray) -> np.ndarray:
    """Rows strictly inside the open support of subdomain j (all dims |x-mu| < sigma)."""
    return np.all(np.abs(x - mu_j[None, :]) < hw_j[None, :], axis=1)


def incidence(inst):
    """Row lists I_j (ascending global row ids) for every subdomain j (eq. DomainDecomp)."""
    return [np.nonzero(support_mask(inst.x, inst.mu[j], inst.hw[j]))[0] for j in range(inst.J)]


def window_factor_1d(xd: np.ndarray, mu: float, sig: float):
    """f = (1 + cos(pi t))^2, t = (x - mu)/sigma, and its first two x-derivatives."""
    t = (xd - mu) / sig
    c = 1.0 + np.cos(np.pi * t)
    s = np.sin(np.pi * t)
    f = c * c
    f1 = -(2.0 * np.pi / sig) * s * c
    f2 = (2.0 * np.pi**2 / sig**2) * (s * s - np.cos(np.pi * t) * c)
    return f, f1, f2


def unnormalised_window(x: np.ndarray, mu_j: np.ndarray, hw_j: np.ndarray):
    """what_j, d_i what_j, d_ii what_j at rows x (caller restricts x to the support)."""
    n, d = x.shape
    fs, f1s, f2s = [], [], []
    for i in range(d):
        f, f1, f2 = window_factor_1d(x[:, i], mu_j[i], hw_j[i])
        fs.append(f)
        f1s.append(f1)
        f2s.append(f2)
    W = np.ones(n)
    for i in range(d):
        W = W * fs[i]
    dW = np.zeros((n, d))
    ddW = np.zeros((n, d))
    for i in range(d):
        others = np.ones(n)
        for l in range(d):
            if l != i:
                others = others * fs[l]
        dW[:, i] = f1s[i] * others
        ddW[:, i] = f2s[i] * others
    return W, dW, ddW


def windows(inst, rows_per_block=None):
    """Normalised windows w_j and their first / pure second derivatives on each block's rows.

    Returns a list over j of (w [m_j], dw [m_j,d], ddw [m_j,d]).  The normaliser
    sum_i what_i and its derivatives are accumulated over subdomains in ascending i.
    """
    if rows_per_block is None:
        rows_per_block = incidence(inst)
    N, d = inst.x.shape
    S = np.zeros(N)
    dS = np.zeros((N, d))
    ddS = np.zeros((N, d))
    local = []
    for j in range(inst.J):
        r = rows_per_block[j]
        W, dW, ddW = unnormalised_window(inst.x[r], inst.mu[j], inst.hw[j])
        S[r] += W
        dS[r] += dW
        ddS[r] += ddW
        local.append((W, dW, ddW))
    out = []
    for j in range(inst.J):
        r = rows_per_block[j]
        W, dW, ddW = local[j]
        s, ds, dds = S[r], dS[r], ddS[r]
        w = W / s
        dw = (dW - w[:, None] * ds) / s[:, None]
        ddw = (ddW - 2.0 * dw * ds - w[:, None] * dds) / s[:, None]
        out.append((w, dw, ddw))
    return out


ACTIVATIONS = ("tanh", "sigmoid", "sin")


def activation(name: str, s: np.ndarray):
    """Xi(s), Xi'(s), Xi''(s) for the activations of Section 5:
    tanh:    t = tanh s,           t' = 1 - t^2,        t'' = -2 t t'
    sigmoid: t = 1 / (1 + e^-s),   t' = t (1 - t),      t'' = t' (1 - 2 t)
    sin:     t = sin s,            t' = cos s,          t'' = -sin s"""
    if name == "tanh":
        t = np.tanh(s)
        g = 1.0 - t * t
        return t, g, -2.0 * t * g
    if name == "sigmoid":
        with np.errstate(over="ignore"):          # exp(-s) = inf gives t = 0 exactly
            t = 1.0 / (1.0 + np.exp(-s))
        g = t * (1.0 - t)
        return t, g, g * (1.0 - 2.0 * t)
    if name == "sin":
        return np.sin(s), np.cos(s), -np.sin(s)
    raise ValueError(f"unknown activation {name!r}")


def features(x: np.ndarray, mu_j, hw_j, wk: np.ndarray, bk: np.ndarray, act: str = "tanh"):
    """phi = Xi(s), s = sum_i w_i (x_i - mu_i)/sigma_i + b; returns phi, d_i phi, d_ii phi
    as arrays [m, K], [m, K, d], [m, K, d]."""
    xn = (x - mu_j[None, :]) / hw_j[None, :]
    s = xn @ wk.T + bk[None, :]
    t, g, gg = activation(act, s)
    scale = wk / hw_j[None, :]                      # [K, d]: dS/dx_i
    dphi = g[:, :, None] * scale[None, :, :]
    ddphi = gg[:, :, None] * (scale * scale)[None, :, :]
    return t, dphi, ddphi


def _coef_rows(op: np.ndarray, opcoef, d: int):
    """Per-row coefficients (c0 [m], c1 [m,d], c2 [m,d]) of the OP_COEF rows (zero elsewhere)
    and the mask of rows that use them; codes past the table read as OP_VALUE."""
    m = len(op)
    c0, c1, c2 = np.zeros(m), np.zeros((m, d)), np.zeros((m, d))
    nop = 0 if opcoef is None else len(opcoef)
    use = (op >= OP_COEF) & (op - OP_COEF < nop)
    for r in np.nonzero(use)[0]:
        row = opcoef[op[r] - OP_COEF]
        c0[r], c1[r], c2[r] = row[0], row[1:1 + d], row[1 + d:1 + 2 * d]
    return c0, c1, c2, use


def network_layers(inst, j):
    """Hidden layers (W [H, fan_in], b [H]) of subdomain j's depth-h network, read from the
    instance's flat per-subdomain parameters (layer 1 on the d inputs, then H x H layers)."""
    H, d = inst.hidden, inst.d
    row = inst.net[j]
    layers = [(row[:H * d].reshape(H, d), row[H * d:H * d + H])]
    o = H * d + H
    for _ in range(inst.depth - 2):
        layers.append((row[o:o + H * H].reshape(H, H), row[o + H * H:o + H * H + H]))
        o += H * H + H
    return layers


def network_features(x, mu_j, hw_j, layers, wk, bk, act: str = "tanh"):
    """Features of a depth-h network (eq. fcn_depth_h): z_0 = xn, z_l = Xi(W_l z_(l-1) + b_l),
    phi_k = Xi(w_k . z_(h-1) + b_k).  Derivatives in x by the chain rule carried forward per
    layer: d_a z_l = Xi'(s) d_a s, d_aa z_l = Xi''(s) (d_a s)^2 + Xi'(s) d_aa s with
    d_a s = W_l d_a z_(l-1).  Returns phi [m, K], d_a phi [m, K, d], d_aa phi [m, K, d]."""
    m, d = x.shape
    z = (x - mu_j[None, :]) / hw_j[None, :]
    dz = np.zeros((m, d, d))
    for a in range(d):
        dz[:, a, a] = 1.0 / hw_j[a]
    ddz = np.zeros((m, d, d))
    for W, b in layers:
        s = z @ W.T + b[None, :]
        ds, dds = dz @ W.T, ddz @ W.T
        t, g, gg = activation(act, s)
        z, dz, ddz = t, g[:, None, :] * ds, gg[:, None, :] * ds * ds + g[:, None, :] * dds
    s = z @ wk.T + bk[None, :]
    ds, dds = dz @ wk.T, ddz @ wk.T
    t, g, gg = activation(act, s)
    dphi = g[:, None, :] * ds
    ddphi = gg[:, None, :] * ds * ds + g[:, None, :] * dds
    return t, dphi.transpose(0, 2, 1), ddphi.transpose(0, 2, 1)


def block_features(inst, j, x):
    """phi, d_a phi, d_aa phi of subdomain j's features at points x (depth 1 or deeper)."""
    k0, k1 = inst.feat_off[j], inst.feat_off[j + 1]
    if inst.depth <= 1:
        return features(x, inst.mu[j], inst.hw[j], inst.w[k0:k1], inst.b[k0:k1], inst.activation)
    return network_features(x, inst.mu[j], inst.hw[j], network_layers(inst, j), inst.w[k0:k1],
                            inst.b[k0:k1], inst.activation)


def apply_rowop(op: np.ndarray, psi, dpsi, ddpsi, kappa: float, ksq: float, opcoef=None):
    """Row operator applied to psi = w phi given its derivatives ([m,K], [m,K,d], [m,K,d])."""
    d = dpsi.shape[2]
    lap = ddpsi.sum(axis=2)
    out = np.empty_like(psi)
    o = op[:, None]
    # -Laplacian over all input dims
    out = np.where(o == OP_NEG_LAPLACE, -lap, out)
    # heat: d_t - kappa * spatial Laplacian, time = last input dim
    spatial = ddpsi[:, :, : d - 1].sum(axis=2) if d > 1 else np.zeros_like(psi)
    out = np.where(o == OP_HEAT, dpsi[:, :, d - 1] - kappa * spatial, out)
    out = np.where(o == OP_HELMHOLTZ, lap + ksq * psi, out)
    out = np.where(o == OP_VALUE, psi, out)
    c0, c1, c2, use = _coef_rows(op, opcoef, d)
    gen = (c0[:, None] * psi + np.einsum("ma,mka->mk", c1, dpsi) + np.einsum("ma,mka->mk", c2, ddpsi))
    out = np.where(use[:, None], gen, out)
    out = np.where((o >= OP_COEF) & ~use[:, None], psi, out)
    return out


def with_ansatz(g, psi, dpsi, ddpsi):
    """Product rule for g * psi, g given per row as [m, 1+2d] (g, d_a g, d_aa g)."""
    d = dpsi.shape[2]
    g0, g1, g2 = g[:, 0], g[:, 1:1 + d], g[:, 1 + d:1 + 2 * d]
    return (g0[:, None] * psi,
            g1[:, None, :] * psi[:, :, None] + g0[:, None, None] * dpsi,
            g2[:, None, :] * psi[:, :, None] + 2.0 * g1[:, None, :] * dpsi + g0[:, None, None] * ddpsi)


def assemble(inst):
    """Global weighted least-squares system in block form.

    Returns (rows, blocks, h): rows[j] = ascending global row ids I_j,
    blocks[j] = dense M_j of shape [|I_j|, K_j] (column k = local feature k),
    h = s_r * rhs_r over all N rows.
    """
    rows = incidence(inst)
    wins = windows(inst, rows)
    G = None if inst.ansatz is None else np.asarray(inst.ansatz(inst.x), dtype=np.float64)
    blocks = []
    for j in range(inst.J):
        r = rows[j]
        k0, k1 = inst.feat_off[j], inst.feat_off[j + 1]
        x = inst.x[r]
        w, dw, ddw = wins[j]
        phi, dphi, ddphi = block_features(inst, j, x)
        psi = w[:, None] * phi
        dpsi = dw[:, None, :] * phi[:, :, None] + w[:, None, None] * dphi
        ddpsi = (ddw[:, None, :] * phi[:, :, None] + 2.0 * dw[:, None, :] * dphi
                 + w[:, None, None] * ddphi)
        if G is not None:
            psi, dpsi, ddpsi = with_ansatz(G[r], psi, dpsi, ddpsi)
        Mj = apply_rowop(inst.rowop[r], psi, dpsi, ddpsi, inst.kappa, inst.ksq, inst.opcoef)
        blocks.append(inst.weight[r][:, None] * Mj)
    h = inst.weight * inst.rhs
    return rows, blocks, h


def entry_error_scale(inst, rows, j):
    """Magnitude that bounds the rounding error of every entry of M_j.

    The entry formula is re-evaluated with every intermediate replaced by the sum of
    the absolute values of its terms (|a - b| -> |a| + |b|, |a b| -> |a| |b|), the
    usual running bound of forward rounding-error analysis: an evaluation of the
    formula in binary64 with n rounded operations on the path to an entry differs from
    the exact value by at most about n u times this magnitude.  The activation and its
    derivatives contribute their sensitivity to the rounding of s:
    |d Xi^(i)(s)| <= |Xi^(i+1)(s)| |ds| + |Xi^(i)(s)| u, with |ds| <= sarg u.
    """
    d = inst.d
    N = inst.N
    # absolute-value evaluation of the windows and of their normaliser
    S = np.zeros(N)
    dSa = np.zeros((N, d))
    ddSa = np.zeros((N, d))
    parts = []
    for i in range(inst.J):
        r = rows[i]
        x = inst.x[r]
        f_a, f1_a, f2_a = [], [], []
        W = np.ones(len(r))
        for a in range(d):
            sig = inst.hw[i, a]
            t = (x[:, a] - inst.mu[i, a]) / sig
            cs = np.abs(np.cos(np.pi * t))
            sn = np.abs(np.sin(np.pi * t))
            c_true = 1.0 + np.cos(np.pi * t)
            W = W * c_true * c_true
            f_a.append((1.0 + cs) ** 2)
            f1_a.append((2.0 * np.pi / sig) * sn * (1.0 + cs))
            f2_a.append((2.0 * np.pi**2 / sig**2) * (sn * sn + cs * (1.0 + cs)))
        Wa = np.prod(f_a, axis=0)
        dWa = np.zeros((len(r), d))
        ddWa = np.zeros((len(r), d))
        for a in range(d):
            others = np.prod([f_a[l] for l in range(d) if l != a], axis=0) if d > 1 else np.ones(len(r))
            dWa[:, a] = f1_a[a] * others
            ddWa[:, a] = f2_a[a] * others
        S[r] += W
        dSa[r] += dWa
        ddSa[r] += ddWa
        parts.append((Wa, dWa, ddWa))
    r = rows[j]
    Wa, dWa, ddWa = parts[j]
    s = S[r]
    wa = Wa / s
    dwa = (dWa + wa[:, None] * dSa[r]) / s[:, None]
    ddwa = (ddWa + 2.0 * dwa * dSa[r] + wa[:, None] * ddSa[r]) / s[:, None]
    k0, k1 = inst.feat_off[j], inst.feat_off[j + 1]
    wk, bk = inst.w[k0:k1], inst.b[k0:k1]
    xn = (inst.x[r] - inst.mu[j][None, :]) / inst.hw[j][None, :]
    if inst.depth <= 1:
        sarg = np.abs(xn) @ np.abs(wk).T + np.abs(bk)[None, :]
        ta, ga, gga = _activation_bounds(inst.activation, xn @ wk.T + bk[None, :], sarg)
        sc = np.abs(wk / inst.hw[j][None, :])
        dphia = ga[:, :, None] * sc[None, :, :]
        ddphia = gga[:, :, None] * (sc * sc)[None, :, :]
    else:
        ta, dphia, ddphia = _network_bounds(inst, j, xn, wk, bk)
    psia = wa[:, None] * ta
    dpsia = dwa[:, None, :] * ta[:, :, None] + wa[:, None, None] * dphia
    ddpsia = ddwa[:, None, :] * ta[:, :, None] + 2.0 * dwa[:, None, :] * dphia + wa[:, None, None] * ddphia
    if inst.ansatz is not None:
        psia, dpsia, ddpsia = with_ansatz(np.abs(inst.ansatz(inst.x[r])), psia, dpsia, ddpsia)
    lap = ddpsia.sum(axis=2)
    op = inst.rowop[r]
    out = np.where(op[:, None] == OP_NEG_LAPLACE, lap, psia)
    spatial = ddpsia[:, :, : d - 1].sum(axis=2) if d > 1 else np.zeros_like(psia)
    out = np.where(op[:, None] == OP_HEAT, dpsia[:, :, d - 1] + abs(inst.kappa) * spatial, out)
    out = np.where(op[:, None] == OP_HELMHOLTZ, lap + abs(inst.ksq) * psia, out)
    c0, c1, c2, use = _coef_rows(op, inst.opcoef, d)
    gen = (np.abs(c0)[:, None] * psia + np.einsum("ma,mka->mk", np.abs(c1), dpsia)
           + np.einsum("ma,mka->mk", np.abs(c2), ddpsia))
    out = np.where(use[:, None], gen, out)
    return np.abs(inst.weight[r])[:, None] * out


def _activation_bounds(name: str, s: np.ndarray, sarg: np.ndarray):
    """Running bounds of Xi, Xi', Xi'' at s (|s| evaluated term by term is sarg): each is the
    absolute-value evaluation of its formula plus the next derivative times sarg."""
    if name == "tanh":
        t = np.tanh(s)
        g = 1.0 - t * t
        ta = np.abs(t) + g * sarg
        ga = 1.0 + t * t + 2.0 * np.abs(t) * g * sarg
        return ta, ga, 2.0 * ta * ga
    if name == "sigmoid":
        with np.errstate(over="ignore"):
            t = 1.0 / (1.0 + np.exp(-s))
        g = t * (1.0 - t)
        g2 = np.abs(g * (1.0 - 2.0 * t))
        g3 = np.abs(g * (1.0 - 6.0 * g))
        ta = t + g * (sarg + 1.0)               # exp's own rounding moves t by t' u
        ga = t * (1.0 + t) + g2 * (sarg + 1.0)
        return ta, ga, ga * (1.0 + 2.0 * ta) + g3 * (sarg + 1.0)
    if name == "sin":
        sn, cs = np.abs(np.sin(s)), np.abs(np.cos(s))
        return sn + cs * sarg, cs + sn * sarg, sn + cs * sarg
    raise ValueError(f"unknown activation {name!r}")


def _activation_terms(name: str, s: np.ndarray):
    """|Xi|, |Xi'|, |Xi''| and |Xi'''| at s, and the absolute-value evaluations of the
    formulas for Xi' and Xi'' in terms of t = Xi(s) (their own rounding allowance)."""
    if name == "tanh":
        t = np.tanh(s)
        g = 1.0 - t * t
        return (np.abs(t), g, 2.0 * np.abs(t) * g, 2.0 * g * np.abs(1.0 - 3.0 * t * t), 1.0 + t * t,
                2.0 * np.abs(t) * (1.0 + t * t))
    if name == "sigmoid":
        with np.errstate(over="ignore"):
            t = 1.0 / (1.0 + np.exp(-s))
        g = t * (1.0 - t)
        ag = t * (1.0 + t)
        return t, g, np.abs(g * (1.0 - 2.0 * t)), np.abs(g * (1.0 - 6.0 * g)), ag, ag * (1.0 + 2.0 * t)
    if name == "sin":
        sn, cs = np.abs(np.sin(s)), np.abs(np.cos(s))
        return sn, cs, sn, cs, cs, sn
    raise ValueError(f"unknown activation {name!r}")


def _network_bounds(inst, j, xn, wk, bk):
    """Running error bounds (in units of u) of phi, d_a phi, d_aa phi for a depth-h network,
    carried through the layers as a pair (magnitude M, error E) for every quantity:
    E(a b) = E_a M_b + M_a E_b + M_a M_b and E(sum) = sum of E + M(sum) for products and sums,
    E(Xi(s)) = |Xi'(s)| E_s + |Xi(s)| for an activation (its own rounding relative to its
    value); M is the absolute-value evaluation."""
    m, d = xn.shape
    Mz, Ez = np.abs(xn), np.abs(xn)
    Mdz = np.zeros((m, d, d))
    for a in range(d):
        Mdz[:, a, a] = 1.0 / inst.hw[j][a]
    Edz = Mdz.copy()
    Mddz, Eddz = np.zeros_like(Mdz), np.zeros_like(Mdz)
    z = xn
    for W, b in network_layers(inst, j) + [(wk, bk)]:
        aW = np.abs(W).T
        s = z @ W.T + b[None, :]
        Ms = Mz @ aW + np.abs(b)[None, :]
        Es = Ez @ aW + Ms
        Mds, Eds = Mdz @ aW, Edz @ aW + Mdz @ aW
        Mdds, Edds = Mddz @ aW, Eddz @ aW + Mddz @ aW
        t, g, gg, g3, Ag, Agg = _activation_terms(inst.activation, s)
        Eg = (gg * Es + Ag)[:, None, :]           # error of Xi'(s)
        Egg = (g3 * Es + Agg)[:, None, :]         # error of Xi''(s)
        g_, gg_ = g[:, None, :], gg[:, None, :]
        Mdz_n = g_ * Mds
        Edz_n = Eg * Mds + g_ * Eds + Mdz_n
        Mddz_n = gg_ * Mds * Mds + g_ * Mdds
        Eddz_n = (Egg * Mds * Mds + gg_ * (2.0 * Mds * Eds + Mds * Mds) + Eg * Mdds + g_ * Edds
                  + g_ * Mdds + Mddz_n)
        Mz, Ez = t, g * Es + t
        Mdz, Edz, Mddz, Eddz = Mdz_n, Edz_n, Mddz_n, Eddz_n
        z = activation(inst.activation, s)[0]
    return Ez, Edz.transpose(0, 2, 1), Eddz.transpose(0, 2, 1)


def global_dense(inst, rows, blocks):
    """Dense M (N x sum K_j) from the blocks: M = sum_j V_j^T M_j W_j (eq. DomainDecomp)."""
    N = inst.N
    M = np.zeros((N, int(inst.feat_off[-1])))
    for j in range(inst.J):
        k0, k1 = inst.feat_off[j], inst.feat_off[j + 1]
        M[np.ix_(rows[j], np.arange(k0, k1))] = blocks[j]
    return M
