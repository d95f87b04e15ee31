"""Float64 reference of the learned screen: a set encoder over the fields of
a candidate solution with a path-length / makespan head.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

The network is not in the paper; it is the learned surrogate that screens
large proposal batches before exact evaluation.  This module fixes its
definition; the GPU kernels are checked against it.

  per field f of the candidate (b = its BP, p = its predecessor on the tour
  route, HQ for the first field):
    phi_f = [x_f/Ls, y_f/Ls, area_f/As, yield_f/Ys, x_b/Ls, y_b/Ls,
             D(f,b)/Ds, D(p,f)/Ds, 2 n_f D(f,b)/Ws, D(HQ,f)/Ds, 0 x 6]     (16)
  h1 = relu(phi W1 + b1)       16 -> 128
  h2 = relu(h1 W2 + b2)        128 -> 128
  e_b = mean of h2 over the fields of BP b (0 without fields)
  e_g = mean of e_b over the BPs of tour g (0 without BPs)
  u_g = [N_HU(g)/N_HU, N_SU(g)/N_SU, rates(g)/rates, fills(g)/fills,
         fields(g)/N_F, BPs(g)/N_B, D(last field, HQ)/Ds, 1]           (8)
  a_g = relu([e_g, u_g] W3 + b3)   136 -> 64
  y_g = a_g W4 + b4                64 -> 2   (path share, completion time)
  P = sum of y_g[0] over active tours,  M = max of y_g[1] over active tours
  loss = (P - C / C0)^2 + (M - T / T0)^2

Scales: Ls = largest |coordinate|, As / Ys = largest area / yield, Ds =
largest distance, Ws = largest 2 n_f D(f,b); C0, T0 = path length and
makespan of the initial solution after Alg. 1's start.  The units are the
candidate's units before rebalancing (those of its base).

Training takes Adam steps (Kingma and Ba, "Adam: A Method for Stochastic
Optimization", ICLR 2015, Algorithm 1) on the mean loss of a batch of
examples: ``adam_step``.
"""
from __future__ import annotations

import dataclasses

import numpy as np

from . import model as Mdl

D_IN, D_H, D_U, D_A, D_OUT = 16, 128, 8, 64, 2


@dataclasses.dataclass
class Scales:
    ls: float
    a_s: float
    y_s: float
    d_s: float
    w_s: float
    c0: float
    t0: float


def scales(inst, c0, t0) -> Scales:
    xy = np.abs(np.asarray(inst.xy_m, dtype=np.float64))
    D = np.asarray(inst.dist_m, dtype=np.float64)
    nb = inst.n_bps
    w = max(2.0 * Mdl.shuttle_drives(inst, f) * D[1 + nb + f, 1:1 + nb].max()
            for f in range(inst.n_fields))
    return Scales(max(xy.max(), 1.0), float(np.max(inst.field_area)), float(np.max(inst.field_yield)),
                  max(D.max(), 1.0), max(w, 1.0), float(c0), float(t0))


def features(inst, sol: Mdl.Solution, sc: Scales):
    """(phi [N_F,16] by field id, u [N_T,8], field BP [N_F], BP tour [N_B],
    active [N_T])."""
    nb, nf, nt = inst.n_bps, inst.n_fields, inst.n_tours
    xy = np.asarray(inst.xy_m, dtype=np.float64)
    D = np.asarray(inst.dist_m, dtype=np.float64)
    phi = np.zeros((nf, D_IN))
    fbp = np.zeros(nf, dtype=np.int64)
    btour = np.zeros(nb, dtype=np.int64)
    u = np.zeros((nt, D_U))
    active = np.zeros(nt, dtype=bool)
    rates = float(np.sum(inst.hu_rate, dtype=np.float64))
    fills = float(np.sum(inst.su_fill_s, dtype=np.float64))
    for g in range(nt):
        prev = 0
        nfg = 0
        for b in sol.tours[g]:
            btour[b] = g
            vb = 1 + b
            for f in sol.fields[b]:
                vf = 1 + nb + f
                fbp[f] = b
                phi[f, 0:2] = xy[vf] / sc.ls
                phi[f, 2] = inst.field_area[f] / sc.a_s
                phi[f, 3] = inst.field_yield[f] / sc.y_s
                phi[f, 4:6] = xy[vb] / sc.ls
                phi[f, 6] = D[vf, vb] / sc.d_s
                phi[f, 7] = D[prev, vf] / sc.d_s
                phi[f, 8] = 2.0 * Mdl.shuttle_drives(inst, f) * D[vf, vb] / sc.w_s
                phi[f, 9] = D[0, vf] / sc.d_s
                prev = vf
                nfg += 1
        hus = [h for h in range(inst.n_hus) if sol.hu_tour[h] == g]
        sus = [s for s in range(inst.n_sus) if sol.su_tour[s] == g]
        u[g] = [len(hus) / inst.n_hus, len(sus) / inst.n_sus,
                sum(float(inst.hu_rate[h]) for h in hus) / rates,
                sum(float(inst.su_fill_s[s]) for s in sus) / fills,
                nfg / nf, len(sol.tours[g]) / nb, D[prev, 0] / sc.d_s if nfg else 0.0, 1.0]
        active[g] = nfg > 0
    return phi, u, fbp, btour, active


def init_params(rng_words):
    """Weights from a given array of uniform [0,1) numbers (drawn by the
    shared input generator): Glorot-uniform, zero biases."""
    shapes = [(D_IN, D_H), (D_H, D_H), (D_H + D_U, D_A), (D_A, D_OUT)]
    out, k = {}, 0
    for i, (fi, fo) in enumerate(shapes, 1):
        lim = np.sqrt(6.0 / (fi + fo))
        n = fi * fo
        out["W%d" % i] = (np.asarray(rng_words[k:k + n], dtype=np.float64).reshape(fi, fo) * 2 - 1) * lim
        out["b%d" % i] = np.zeros(fo)
        k += n
    return out


def forward(p, phi, u, fbp, btour, active, nb):
    """Returns (P, M, cache)."""
    z1 = phi @ p["W1"] + p["b1"]
    h1 = np.maximum(z1, 0.0)
    z2 = h1 @ p["W2"] + p["b2"]
    h2 = np.maximum(z2, 0.0)
    nt = u.shape[0]
    eb = np.zeros((nb, D_H))
    cb = np.zeros(nb)
    for f in range(phi.shape[0]):
        eb[fbp[f]] += h2[f]
        cb[fbp[f]] += 1
    eb = np.where(cb[:, None] > 0, eb / np.maximum(cb, 1)[:, None], 0.0)
    eg = np.zeros((nt, D_H))
    cg = np.zeros(nt)
    for b in range(nb):
        eg[btour[b]] += eb[b]
        cg[btour[b]] += 1
    eg = np.where(cg[:, None] > 0, eg / np.maximum(cg, 1)[:, None], 0.0)
    zin = np.concatenate([eg, u], axis=1)
    z3 = zin @ p["W3"] + p["b3"]
    a = np.maximum(z3, 0.0)
    y = a @ p["W4"] + p["b4"]
    act = np.nonzero(active)[0]
    P = float(y[act, 0].sum())
    gm = int(act[np.argmax(y[act, 1])])
    M = float(y[gm, 1])
    cache = dict(phi=phi, z1=z1, h1=h1, z2=z2, h2=h2, cb=cb, cg=cg, zin=zin, z3=z3, a=a, y=y,
                 act=act, gm=gm, fbp=fbp, btour=btour, nb=nb)
    return P, M, cache


def loss(P, M, pt, mt):
    return (P - pt) ** 2 + (M - mt) ** 2


def backward(p, cache, P, M, pt, mt):
    """Gradients of loss(P, M) w.r.t. every parameter."""
    y = cache["y"]
    dy = np.zeros_like(y)
    dy[cache["act"], 0] = 2.0 * (P - pt)
    dy[cache["gm"], 1] += 2.0 * (M - mt)
    g = {"W4": cache["a"].T @ dy, "b4": dy.sum(0)}
    da = dy @ p["W4"].T
    dz3 = da * (cache["z3"] > 0)
    g["W3"] = cache["zin"].T @ dz3
    g["b3"] = dz3.sum(0)
    dzin = dz3 @ p["W3"].T
    deg = dzin[:, :D_H]
    cg, cb, fbp, btour, nb = cache["cg"], cache["cb"], cache["fbp"], cache["btour"], cache["nb"]
    deb = np.zeros((nb, D_H))
    for b in range(nb):
        gt = btour[b]
        if cg[gt] > 0:
            deb[b] = deg[gt] / cg[gt]
    dh2 = np.zeros_like(cache["h2"])
    for f in range(dh2.shape[0]):
        b = fbp[f]
        dh2[f] = deb[b] / cb[b]
    dz2 = dh2 * (cache["z2"] > 0)
    g["W2"] = cache["h1"].T @ dz2
    g["b2"] = dz2.sum(0)
    dh1 = dz2 @ p["W2"].T
    dz1 = dh1 * (cache["z1"] > 0)
    g["W1"] = cache["phi"].T @ dz1
    g["b1"] = dz1.sum(0)
    return g


def predict(p, inst, sol, sc):
    phi, u, fbp, btour, active = features(inst, sol, sc)
    P, M, _ = forward(p, phi, u, fbp, btour, active, inst.n_bps)
    return P, M


def example_loss_and_grad(p, inst, sol, sc, cost_m, makespan_s):
    phi, u, fbp, btour, active = features(inst, sol, sc)
    P, M, cache = forward(p, phi, u, fbp, btour, active, inst.n_bps)
    pt, mt = cost_m / sc.c0, makespan_s / sc.t0
    return loss(P, M, pt, mt), backward(p, cache, P, M, pt, mt)


def adam_step(p, g, m, v, t, lr, beta1, beta2, eps):
    """One Adam update (Kingma and Ba 2015, Algorithm 1) of every parameter
    array in the dict p with gradient g, first and second moment estimates m
    and v (dicts of the same shapes, zero before the first step) and step
    number t >= 1.  Returns the new (p, m, v); nothing is changed in place.

      m_t = beta1 m_{t-1} + (1 - beta1) g
      v_t = beta2 v_{t-1} + (1 - beta2) g^2
      p_t = p_{t-1} - lr (m_t / (1 - beta1^t)) / (sqrt(v_t / (1 - beta2^t)) + eps)
    """
    assert t >= 1
    bc1 = 1.0 - beta1 ** t
    bc2 = 1.0 - beta2 ** t
    p_new, m_new, v_new = {}, {}, {}
    for k in p:
        gk = np.asarray(g[k], dtype=np.float64)
        m_new[k] = beta1 * np.asarray(m[k], dtype=np.float64) + (1.0 - beta1) * gk
        v_new[k] = beta2 * np.asarray(v[k], dtype=np.float64) + (1.0 - beta2) * gk * gk
        p_new[k] = np.asarray(p[k], dtype=np.float64) - lr * (m_new[k] / bc1) / (np.sqrt(v_new[k] / bc2) + eps)
    return p_new, m_new, v_new
