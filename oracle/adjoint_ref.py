"""FP64 reference gradient of L = sum_i |a_i|^2 (TEST INFRASTRUCTURE ONLY).

An independent derivation of the adjoint: the density and force loops are
written once more as plain torch float64 CPU operations over a brute-force
pair list, and torch's reverse-mode autograd differentiates them.  h, u,
alpha~ and alpha_d are constants; density is part of the graph.

Also: central finite differences of the C oracle's FP64 loss, recomputing only
the particles whose acceleration a perturbation can reach.
"""
from __future__ import annotations

import numpy as np
import torch

import oracle

GK = float(np.sqrt(10.0 / 3.0))
C3 = 8.0 / np.pi


def _w(q):
    t = torch.clamp(1.0 - q, min=0.0)
    return torch.where(q < 0.5, 1.0 - 6.0 * q ** 2 + 6.0 * q ** 3, 2.0 * t ** 3)


def _dw(q):
    t = torch.clamp(1.0 - q, min=0.0)
    return torch.where(q < 0.5, -12.0 * q + 18.0 * q ** 2, -6.0 * t ** 2)


def pair_list(x: np.ndarray, H: np.ndarray):
    """all ordered pairs i != j with minimum-image distance below max(H_i, H_j)"""
    from scipy.spatial import cKDTree
    t = cKDTree(np.mod(x, 1.0), boxsize=1.0)
    p = t.query_pairs(r=float(H.max()), output_type="ndarray")
    d = x[p[:, 0]] - x[p[:, 1]]
    d -= np.round(d)
    r = np.sqrt((d * d).sum(1))
    keep = r < np.maximum(H[p[:, 0]], H[p[:, 1]])
    p = p[keep]
    return np.concatenate([p[:, 0], p[:, 1]]), np.concatenate([p[:, 1], p[:, 0]])


def loss_torch(x, v, m, h, u, atilde, alpha_d, ii, jj, gamma=5.0 / 3.0, beta=3.0):
    """L = sum |a|^2, all tensors float64 on the CPU; (ii, jj) ordered pairs."""
    H = GK * h
    n = x.shape[0]
    d = x[ii] - x[jj]
    d = d - torch.round(d.detach())          # minimum image (the shift is a constant)
    r = torch.sqrt((d * d).sum(1))
    # density: self term plus neighbours inside H_i
    qi = r / H[ii]
    inside_i = r < H[ii]
    Wi = torch.where(inside_i, C3 / H[ii] ** 3 * _w(qi), torch.zeros_like(r))
    Whi = torch.where(inside_i, -GK * C3 / H[ii] ** 4 * (3.0 * _w(qi) + qi * _dw(qi)), torch.zeros_like(r))
    q0 = torch.zeros_like(h)
    rho = m * C3 / H ** 3 * _w(q0) + torch.zeros(n, dtype=x.dtype).index_add(0, ii, m[jj] * Wi)
    rdh = m * (-GK * C3 / H ** 4 * 3.0 * _w(q0)) + torch.zeros(n, dtype=x.dtype).index_add(0, ii, m[jj] * Whi)
    A = (gamma - 1.0) * u / (rho + h * rdh / 3.0)
    c = torch.sqrt(gamma * (gamma - 1.0) * u)

    def F(q, HH, inside):
        t = torch.clamp(1.0 - q, min=0.0)
        f = torch.where(q < 0.5, -12.0 + 18.0 * q, -6.0 * t ** 2 / torch.clamp(q, min=1e-30))
        return torch.where(inside, C3 / HH ** 5 * f, torch.zeros_like(q))

    Fi = F(qi, H[ii], inside_i)
    qj = r / H[jj]
    Fj = F(qj, H[jj], r < H[jj])
    Fb = 0.5 * (Fi + Fj)
    vv = v[ii] - v[jj]
    mu = torch.clamp((vv * d).sum(1) / r, max=0.0)
    vsig = c[ii] + c[jj] - beta * mu
    rb = 0.5 * (rho[ii] + rho[jj])
    Pi = -0.5 * 0.5 * (atilde[ii] + atilde[jj]) * vsig * mu / rb
    S = A[ii] * Fi + A[jj] * Fj + Pi * Fb
    a = -torch.zeros(n, 3, dtype=x.dtype).index_add(0, ii, (m[jj] * S)[:, None] * d)
    return (a * a).sum(), a


def reference_gradient(f: dict, atilde: np.ndarray):
    """dL/dx, dL/dv, dL/dm by torch float64 autograd on the CPU."""
    H = GK * f["h"].astype(np.float64)
    ii, jj = pair_list(f["x"], H)
    T = lambda a, g=False: torch.tensor(np.asarray(a, np.float64), requires_grad=g)
    x, v, m = T(f["x"], True), T(f["v"], True), T(f["mass"], True)
    L, a = loss_torch(x, v, m, T(f["h"]), T(f["u"]), T(atilde), T(f["alpha_d"]),
                      torch.from_numpy(ii), torch.from_numpy(jj))
    L.backward()
    return float(L), a.detach().numpy(), x.grad.numpy(), v.grad.numpy(), m.grad.numpy()


# ---------------------------------------------------------------------------
# finite differences of the C oracle's loss
# ---------------------------------------------------------------------------
def _near(x, k, radius):
    d = x - x[k]
    d -= np.round(d)
    return np.nonzero(np.sqrt((d * d).sum(1)) < radius)[0]


def local_loss(f, atilde, rho, rdh, k, rows_d, rows_f):
    """sum over rows_f of |a|^2 after recomputing rho, rho_dh on rows_d"""
    rho = rho.copy()
    rdh = rdh.copy()
    d = oracle.density(f["x"], f["mass"], f["h"], rows=rows_d)
    rho[rows_d] = d["rho"]
    rdh[rows_d] = d["rho_dh"]
    z = np.zeros(f["x"].shape[0])
    fo = oracle.force(f["x"], f["v"], f["mass"], f["h"], f["u"], rho, rdh, z, np.zeros((z.size, 3)),
                      f["alpha_v"], f["alpha_d"], atilde=atilde, rows=rows_f)
    return float((fo["a"] ** 2).sum())


def straddles_kink(f: dict, kind: str, k: int, comp: int, rel_eps=1e-6) -> bool:
    """whether the +-eps step of a coordinate flips the sign of v_kj . r_kj for
    some neighbour pair (where the viscosity switches on and L has a kink)"""
    if kind == "m":
        return False
    H = GK * f["h"].astype(np.float64)
    js = _near(f["x"], k, float(H.max()) * 1.01 + 1e-5)
    signs = []
    for sgn in (+1.0, -1.0):
        x = f["x"][js].copy()
        v = f["v"][js].astype(np.float64).copy()
        kk = int(np.nonzero(js == k)[0][0])
        if kind == "x":
            x[kk, comp] += sgn * rel_eps
        else:
            v[kk, comp] += sgn * rel_eps * max(1.0, abs(float(v[kk, comp])))
        d = x[kk] - x
        d -= np.round(d)
        signs.append(np.sign(((v[kk] - v) * d).sum(1)))
    return bool(np.any(signs[0] != signs[1]))


def fd_gradient(f: dict, atilde: np.ndarray, coords, rel_eps=1e-6):
    """central differences of L for (kind, particle, component) coordinates;
    kind in {"x", "v", "m"}; eps = 1e-6 for x, 1e-6 max(1, |v|) for v, 1e-6 m_k for m"""
    H = GK * f["h"].astype(np.float64)
    Hm = float(H.max())
    base = oracle.density(f["x"], f["mass"], f["h"])
    out = []
    for kind, k, comp in coords:
        rows_d = _near(f["x"], k, Hm * 1.01 + 1e-5)
        rows_f = _near(f["x"], k, 3.0 * Hm * 1.01 + 1e-5)
        vals, at = [], []
        for sgn in (+1.0, -1.0):
            g = {kk: vv.copy() for kk, vv in f.items()}
            # v and m enter the oracle as float32: step by the float32 value
            # actually stored, and divide by the step actually taken
            if kind == "x":
                g["x"][k, comp] += sgn * rel_eps
                at.append(g["x"][k, comp])
            elif kind == "v":
                eps = rel_eps * max(1.0, abs(float(f["v"][k, comp])))
                g["v"][k, comp] = np.float32(float(f["v"][k, comp]) + sgn * eps)
                at.append(float(g["v"][k, comp]))
            else:
                eps = rel_eps * float(f["mass"][k])
                g["mass"][k] = np.float32(float(f["mass"][k]) + sgn * eps)
                at.append(float(g["mass"][k]))
            vals.append(local_loss(g, atilde, base["rho"], base["rho_dh"], k, rows_d, rows_f))
        out.append((vals[0] - vals[1]) / (at[0] - at[1]))
    return np.array(out)
