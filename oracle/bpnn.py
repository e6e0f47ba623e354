"""Behler-Parrinello neural-network potential (oracle; test infrastructure only).

Sec. 2.1.  The energy is a sum of atomic energies, E = sum_i E_i (eq. E_as_sum).
E_i is the output of a small fully connected network whose inputs are the
symmetry functions of atom i, built from the neighbours j within R_c:

  cutoff        f_c(R) = 1/2 [cos(pi R / R_c) + 1] for R <= R_c, else 0
  radial (G2)   G2_mu(i) = sum_j exp(-eta_mu (R_ij - R_s)^2) f_c(R_ij)
  angular (G4)  G4_mu(i) = 2^(1 - zeta_mu) sum_{j != k} (1 + lambda_mu cos theta_ijk)^zeta_mu
                           exp(-eta_mu (R_ij^2 + R_ik^2 + R_jk^2)) f_c(R_ij) f_c(R_ik) f_c(R_jk)
  network       E_i = b3 + sum_k w23_k tanh(b2_k + sum_j w12_jk tanh(b1_j + sum_mu G_mu w01_mu,j))
                (eq. AtomicNN with tanh on both hidden layers and a linear output)

Readings where the text is garbled or silent: the radial exponent is squared,
exp(-eta (R - R_s)^2) (the printed exponent lacks the square); the angular sum runs
over ordered pairs j != k, both neighbours of i within R_c (each unordered pair
twice); the activation functions are tanh for the two hidden layers and the identity
for the output (the text's numbering of F_1..F_3 is inverted against its own
equation); G_mu is G2 followed by G4.

Forces follow eq. force: F_k = -sum_i sum_mu dE_i/dG_mu(i) dG_mu(i)/dR_k, with
dE_i/dG from the network's backward pass and dG/dR from the analytic derivatives of
the symmetry functions, written out below per pair and per triplet.  Virial:
W = -sum_i sum_terms (x_j - x_i) (x) dE_i/d(x_j - x_i) over every neighbour vector a
term of E_i depends on, which for a pair potential is 1/2 sum r_ij (x) f_ij.
"""
from __future__ import annotations

import numpy as np

from . import core


def cutoff(R, rc):
    """(f_c, f_c') at distances R."""
    inside = R <= rc
    fc = np.where(inside, 0.5 * (np.cos(np.pi * R / rc) + 1.0), 0.0)
    dfc = np.where(inside, -0.5 * np.pi / rc * np.sin(np.pi * R / rc), 0.0)
    return fc, dfc


def neighbours(x, box, rc):
    """Per atom: indices j and minimum-image vectors a_ij = x_j - x_i with R_ij <= rc."""
    cnt, lists = core.neighbor_sets(x, box, rc)
    ln = np.asarray(box.len, np.float64)
    per = np.asarray(box.periodic, bool)
    out = []
    for i, js in enumerate(lists):
        a = x[js] - x[i]
        a[:, per] -= ln[per] * np.rint(a[:, per] / ln[per])
        R = np.sqrt((a * a).sum(axis=1))
        keep = R <= rc
        out.append((js[keep], a[keep], R[keep]))
    return out


def descriptors_atom(a, R, p):
    """G (n_g2 + n_g4) of one atom from its neighbour vectors a [m, 3] and distances R."""
    rc = p["r_cut"]
    fc, _ = cutoff(R, rc)
    g2 = np.array([np.sum(np.exp(-eta * (R - p["r_s"]) ** 2) * fc) for eta in p["g2_eta"]])
    m = len(R)
    g4 = np.zeros(len(p["g4_eta"]))
    if m >= 2:
        j, k = np.where(~np.eye(m, dtype=bool))  # ordered pairs j != k
        A, B = R[j], R[k]
        C = np.sqrt(((a[k] - a[j]) ** 2).sum(axis=1))
        cos = (a[j] * a[k]).sum(axis=1) / (A * B)
        f3 = fc[j] * fc[k] * cutoff(C, rc)[0]
        s2 = A * A + B * B + C * C
        for q, (zeta, lam, eta) in enumerate(zip(p["g4_zeta"], p["g4_lambda"], p["g4_eta"])):
            g4[q] = 2.0 ** (1.0 - zeta) * np.sum((1.0 + lam * cos) ** zeta * np.exp(-eta * s2) * f3)
    return np.concatenate([g2, g4])


def network(G, p):
    """(E_i, dE_i/dG) of the atomic network for one descriptor vector."""
    w01, b1, w12, b2, w23, b3 = (p[k] for k in ("w01", "b1", "w12", "b2", "w23", "b3"))
    h1 = np.tanh(b1 + G @ w01)
    h2 = np.tanh(b2 + h1 @ w12)
    E = b3 + h2 @ w23
    d2 = w23 * (1.0 - h2 * h2)
    d1 = (w12 @ d2) * (1.0 - h1 * h1)
    return float(E), w01 @ d1


def energy(x, box, p):
    """Total energy and per-atom energies."""
    nb = neighbours(x, box, p["r_cut"])
    e = np.array([network(descriptors_atom(a, R, p), p)[0] for _, a, R in nb])
    return float(e.sum()), e


def forces(x, box, p):
    """Energy, per-atom energies, forces [n, 3] and virial (xx yy zz xy xz yz)."""
    n = x.shape[0]
    rc, rs = p["r_cut"], p["r_s"]
    nb = neighbours(x, box, rc)
    f = np.zeros((n, 3))
    e = np.zeros(n)
    W = np.zeros((3, 3))
    n2 = len(p["g2_eta"])
    for i, (js, a, R) in enumerate(nb):
        G = descriptors_atom(a, R, p)
        e[i], c = network(G, p)
        fc, dfc = cutoff(R, rc)
        ga = np.zeros_like(a)  # dE_i / d a_ij
        # radial: d/dR [exp(-eta (R - R_s)^2) f_c(R)]
        dR = np.zeros_like(R)
        for q, eta in enumerate(p["g2_eta"]):
            ex = np.exp(-eta * (R - rs) ** 2)
            dR += c[q] * ex * (dfc - 2.0 * eta * (R - rs) * fc)
        ga += (dR / R)[:, None] * a
        m = len(R)
        if m >= 2:
            j, k = np.where(~np.eye(m, dtype=bool))
            aj, ak = a[j], a[k]
            A, B = R[j], R[k]
            d = ak - aj
            C = np.sqrt((d * d).sum(axis=1))
            cos = (aj * ak).sum(axis=1) / (A * B)
            fA, dfA, fB, dfB = fc[j], dfc[j], fc[k], dfc[k]
            fC, dfC = cutoff(C, rc)
            s2 = A * A + B * B + C * C
            s_cos = np.zeros_like(A)
            s_A, s_B, s_C = np.zeros_like(A), np.zeros_like(A), np.zeros_like(A)
            for q, (zeta, lam, eta) in enumerate(zip(p["g4_zeta"], p["g4_lambda"], p["g4_eta"])):
                cq = c[n2 + q] * 2.0 ** (1.0 - zeta)
                P = 1.0 + lam * cos
                X = np.exp(-eta * s2)
                Pz = P ** zeta
                base = cq * Pz * X
                s_cos += cq * zeta * lam * P ** (zeta - 1.0) * X * fA * fB * fC
                s_A += base * (dfA * fB * fC - 2.0 * eta * A * fA * fB * fC)
                s_B += base * (fA * dfB * fC - 2.0 * eta * B * fA * fB * fC)
                s_C += base * (fA * fB * dfC - 2.0 * eta * C * fA * fB * fC)
            dcos_a = ak / (A * B)[:, None] - (cos / (A * A))[:, None] * aj
            dcos_b = aj / (A * B)[:, None] - (cos / (B * B))[:, None] * ak
            g_a = s_cos[:, None] * dcos_a + (s_A / A)[:, None] * aj - (s_C / C)[:, None] * d
            g_b = s_cos[:, None] * dcos_b + (s_B / B)[:, None] * ak + (s_C / C)[:, None] * d
            np.add.at(ga, j, g_a)
            np.add.at(ga, k, g_b)
        # E_i depends on a_ij = x_j - x_i
        np.add.at(f, js, -ga)
        f[i] += ga.sum(axis=0)
        W -= a.T @ ga
    w = np.array([W[0, 0], W[1, 1], W[2, 2], W[0, 1], W[0, 2], W[1, 2]])
    return float(e.sum()), e, f, w
