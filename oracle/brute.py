"""Dense-matrix brute force of the semi-discrete model, for tiny grids.

TEST INFRASTRUCTURE.  A second, independent transcription used to pin the C
oracle: operators are assembled as explicit matrices over all cells (the
Laplacian as a graph Laplacian over open faces, the heat operator as a
conductance matrix), and the Runge-Kutta-Merson step is written as a Butcher
tableau.  Only meant for grids of a few hundred cells.

Model: Sec. 2.1-2.2 of the paper (blending, heat equation, Allen-Cahn with
the SigmaP1-P or GradP reaction, water indicator, boundary conditions),
Sec. 2.3 (Temp model), Sec. 2.4 (micro-scale reduction) and Sec. 2.5
(method of lines, Merson integrator).
"""
from __future__ import annotations

import numpy as np

# Merson's method as a Butcher tableau (c, A, b) plus the error weights.
MERSON_C = np.array([0.0, 1 / 3, 1 / 3, 1 / 2, 1.0])
MERSON_A = np.array([
    [0, 0, 0, 0, 0],
    [1 / 3, 0, 0, 0, 0],
    [1 / 6, 1 / 6, 0, 0, 0],
    [1 / 8, 0, 3 / 8, 0, 0],
    [1 / 2, 0, -3 / 2, 2, 0],
])
MERSON_B = np.array([1 / 6, 0, 0, 2 / 3, 1 / 6])
MERSON_E = np.array([1 / 15, 0, -3 / 10, 4 / 15, -1 / 30])


def _faces(shape):
    """All (cell, neighbour, face-id) pairs inside the box, and all
    (cell, face-id) boundary faces.  Face ids 0..5 = x1-,x1+,x2-,x2+,x3-,x3+."""
    n3, n2, n1 = shape
    idx = np.arange(n1 * n2 * n3).reshape(shape)
    pairs, bnd = [], []
    offs = [(0, 0, -1), (0, 0, 1), (0, -1, 0), (0, 1, 0), (-1, 0, 0), (1, 0, 0)]
    for i3 in range(n3):
        for i2 in range(n2):
            for i1 in range(n1):
                c = idx[i3, i2, i1]
                for f, (d3, d2, d1) in enumerate(offs):
                    j3, j2, j1 = i3 + d3, i2 + d2, i1 + d1
                    if 0 <= j3 < n3 and 0 <= j2 < n2 and 0 <= j1 < n1:
                        pairs.append((c, idx[j3, j2, j1], f))
                    else:
                        bnd.append((c, f))
    return np.array(pairs, dtype=np.int64), np.array(bnd, dtype=np.int64).reshape(-1, 2)


def phase_laplacian(G, h, face_mask=True):
    """Matrix of the finite-volume Laplacian of phi with zero flux through the
    domain boundary and (face_mask) through faces touching glass.  G is the
    3D glass field of shape (n3, n2, n1)."""
    G = np.asarray(G, np.float64)
    Gf = G.ravel()
    n = Gf.size
    pairs, _ = _faces(G.shape)
    Lm = np.zeros((n, n))
    for c, m, _f in pairs:
        if face_mask and not (Gf[c] < 0.5 and Gf[m] < 0.5):
            continue
        Lm[c, m] += 1.0
        Lm[c, c] -= 1.0
    return Lm / (h * h)


def blend(G, phi, w):
    return G * w[2] + (1 - G) * (phi * w[1] + (1 - phi) * w[0])


def heat_capacity(p, G, phi):
    """rho c per cell: blended volumetric values, or (the paper's own form)
    blended density times blended specific heat."""
    if p.get("rho_c_separate", 0):
        return blend(G, phi, p["rho"]) * blend(G, phi, p["cs"])
    return blend(G, phi, p["rhoc"])


def latent_heat(p, G, phi):
    """rho L per cell: constant, or blended density times L."""
    if p.get("rho_c_separate", 0):
        return blend(G, phi, p["rho"]) * p["L"]
    return p["Lv"] + 0 * phi


def smoothstep(w, e0, e1):
    s = np.clip((w - e0) / (e1 - e0), 0.0, 1.0)
    out = s * s * (3 - 2 * s)
    out = np.where(w <= e0, 0.0, out)
    return np.where(w >= e1, 1.0, out)


def dirichlet_T(p, t):
    if p["bc_kind"] == 1:
        s = np.clip((t - p["bc_t0"]) / (p["bc_t1"] - p["bc_t0"]), 0.0, 1.0)
        return p["bc_T0"] + (p["bc_T1"] - p["bc_T0"]) * s
    if p["bc_kind"] == 2:
        return p["bc_T0"] if t < p["bc_t0"] else p["bc_T1"]
    return p["bc_T0"]


def gradient_norm(G, phi, h, face_mask=True):
    """|grad phi| per cell: for each axis the difference quotient over the
    open faces (both open: central, one open: one-sided, none: 0).  A face is
    open when the neighbour exists and is water (G < 1/2), and (face_mask)
    the cell is water too."""
    G = np.asarray(G, np.float64)
    ph = np.asarray(phi, np.float64)
    g2 = np.zeros(G.shape)
    for ax in (2, 1, 0):  # x1, x2, x3 in array order (n3, n2, n1)
        n = G.shape[ax]
        for i in range(n):
            sl = [slice(None)] * 3
            sl[ax] = i
            sl = tuple(sl)
            if i > 0:
                lo = [slice(None)] * 3
                lo[ax] = i - 1
                lo = tuple(lo)
                om = ((G[sl] < 0.5) & (G[lo] < 0.5)) if face_mask else (G[lo] < 0.5)
                phm = np.where(om, ph[lo], ph[sl])
            else:
                om = np.zeros(G[sl].shape, bool)
                phm = ph[sl]
            if i < n - 1:
                hi = [slice(None)] * 3
                hi[ax] = i + 1
                hi = tuple(hi)
                oq = ((G[sl] < 0.5) & (G[hi] < 0.5)) if face_mask else (G[hi] < 0.5)
                phq = np.where(oq, ph[hi], ph[sl])
            else:
                oq = np.zeros(G[sl].shape, bool)
                phq = ph[sl]
            width = np.where(om & oq, 2.0 * h, h)
            g2[sl] += ((phq - phm) / width) ** 2
    return np.sqrt(g2)


def temp_phase(p, G, T):
    """Temp model: phi = I_W(G) (1 - tanh(gamma (T - T*)))/2 and its
    derivative in T."""
    IW = np.maximum(0.0, 1 - p["zeta"] * np.asarray(G, np.float64))
    th = np.tanh(p.get("gamma", 2.0) * (np.asarray(T, np.float64) - p["t_star"]))
    return 0.5 * IW * (1 - th), -0.5 * IW * p.get("gamma", 2.0) * (1 - th * th)


def rhs(p, G, t, phi, T=None):
    """(kphi, kT) of the micro-scale ("ac"), coupled or Temp model, dense form.
    Temp model: phi is ignored and kphi = varphi'(T) kT."""
    shape = np.shape(G)
    Gf = np.asarray(G, np.float64).ravel()
    model = p["model"]
    coupled = model == "coupled"
    if model == "temp":
        Tc = np.asarray(T, np.float64).ravel()
        ph, dph = temp_phase(p, Gf, Tc)
    else:
        ph = np.asarray(phi, np.float64).ravel()
        Tc = np.asarray(T, np.float64).ravel() if coupled else \
            np.full(Gf.size, p["t_star"] - p["dT"])
    xi, al = p["xi"], p["alpha"]
    if model != "temp":
        fm = bool(p.get("phi_face_mask", 1))
        Lphi = phase_laplacian(np.reshape(Gf, shape), p["h"], fm) @ ph
        if p.get("reaction", "sigma") == "gradp":
            gn = gradient_norm(np.reshape(Gf, shape), np.reshape(ph, shape), p["h"], fm).ravel()
            f = 2 * ph * (1 - ph) * (ph - 0.5) + xi * xi * p["mu"] * al * gn * (p["t_star"] - Tc)
        else:
            drive = 0.5 * xi * p["b"] * p["mu"] * al * smoothstep(ph, p["eps0"], p["eps1"]) \
                * smoothstep(1 - ph, p["eps0"], p["eps1"]) * (p["t_star"] - Tc)
            f = 2 * ph * (1 - ph) * (ph - 0.5 + drive)
        IW = np.maximum(0.0, 1 - p["zeta"] * Gf)
        kphi = IW * (Lphi + f / (xi * xi)) / al
        if not coupled:
            return kphi.reshape(shape), None
    lam = blend(Gf, ph, p["lam"])
    n = Gf.size
    pairs, bnd = _faces(shape)
    A = np.zeros((n, n))
    src = np.zeros(n)
    for c, m, _f in pairs:
        k = 0.5 * (lam[c] + lam[m])
        A[c, m] += k
        A[c, c] -= k
    TD = dirichlet_T(p, t)
    for c, f in bnd:
        if p["dirichlet_faces"] & (1 << int(f)):
            A[c, c] -= 2 * lam[c]
            src[c] += 2 * lam[c] * TD
    divq = (A @ Tc + src) / (p["h"] ** 2)
    rc, lat = heat_capacity(p, Gf, ph), latent_heat(p, Gf, ph)
    if model == "temp":
        kT = divq / (rc - lat * dph)
        return (dph * kT).reshape(shape), kT.reshape(shape)
    kT = (divq + lat * kphi) / rc
    return kphi.reshape(shape), kT.reshape(shape)


def merson_step(p, G, t, dt, phi, T=None):
    """One fixed Merson step through the Butcher tableau.  Returns
    (phi_new, T_new, error_vector_maxnorm)."""
    coupled = p["model"] == "coupled"
    shape = np.shape(G)
    y = np.concatenate([np.ravel(phi), np.ravel(T)]) if coupled else np.ravel(phi).astype(float)
    nc = int(np.prod(shape))

    def F(tt, yy):
        if coupled:
            a, b = rhs(p, G, tt, yy[:nc].reshape(shape), yy[nc:].reshape(shape))
            return np.concatenate([a.ravel(), b.ravel()])
        a, _ = rhs(p, G, tt, yy.reshape(shape))
        return a.ravel()

    K = []
    for s in range(5):
        Ys = y + dt * sum(MERSON_A[s, j] * K[j] for j in range(s)) if s else y
        K.append(F(t + MERSON_C[s] * dt, Ys))
    K = np.array(K)
    ynew = y + dt * (MERSON_B @ K)
    err = np.max(np.abs(dt * (MERSON_E @ K)))
    if coupled:
        return ynew[:nc].reshape(shape), ynew[nc:].reshape(shape), err
    return ynew.reshape(shape), None, err
