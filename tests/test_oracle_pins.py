"""Pins of the FP64 oracle against what the paper and the mathematics fix.

Each test is chosen so that a plausible slip in the oracle (a dropped term, a
wrong sign, index or weight, a transposed operand) fails at least one of
them:
  * Tab. 1 / Tab. 2 constants recomputed from their definitions;
  * the Sigma limiter's defining properties (eq. Sigma-limiter);
  * a dense-matrix brute force on tiny random grids (RHS and a full step);
  * the planar tanh travelling front of the Allen-Cahn equation
    (eqs. Allen-Cahn-equation and reaction-term-SigmaP1-P with Sigma = 1);
  * the exact discrete decay of heat-equation eigenmodes (eq. heat-equation,
    insulated walls and a Dirichlet face) under the Merson amplification
    factor;
  * enthalpy balance of the coupled right-hand side with insulated walls;
  * 4th-order convergence of the Merson step on a closed-form scalar ODE;
  * the Gibbs-Thomson critical radius (eq. Gibbs-Thomson).
"""
import json
import math
import os
import zlib

import numpy as np
import pytest

import oracle
from oracle import brute

HERE = os.path.dirname(os.path.abspath(__file__))
GOLD = json.load(open(os.path.join(HERE, "golden", "paper_constants.json")))


def _sig(x, digits):
    return float(f"{x:.{digits - 1}e}")


# --------------------------------------------------------------------------
# Constants (Tab. 1, Tab. 2)

def test_table1_entropy_and_alpha():
    t1 = GOLD["table1"]
    ds = t1["rho"]["I"] * t1["L"] / t1["T_star"]            # Tab. 1: ds = rho_I L / T*
    assert _sig(ds, t1["delta_s_digits"]) == t1["delta_s_printed"]
    alpha = ds / (t1["mu"] * t1["sigma"])                      # eq. attachment-kinetics-coeff
    assert _sig(alpha, t1["alpha_digits"]) == t1["alpha_printed"]


def test_table2_alpha_levels():
    t1, t2 = GOLD["table1"], GOLD["table2"]
    large = t1["rho"]["L"] * t1["c"]["L"]                      # "large sigma": alpha = rho_L c_L
    assert _sig(large, 3) == t2["alpha_large_printed"]
    assert _sig(3 * large, 3) == t2["alpha_small_printed"]     # three times larger
    sigma_tiny = t1["delta_s_printed"] / (t1["mu"] * t2["alpha_tiny_printed"])
    assert 800 < sigma_tiny / t1["sigma"] < 1200               # "approximately 1000x"


def test_input_constants_match_tables():
    import pf_inputs as pi
    assert pi.ALPHA_REAL == GOLD["table1"]["alpha_printed"]
    assert pi.ALPHA_LARGE_SIGMA == GOLD["table2"]["alpha_large_printed"]
    assert pi.T_STAR == GOLD["table1"]["T_star"]
    assert pi.MU == GOLD["table1"]["mu"]
    t1 = GOLD["table1"]
    assert pi.RHO_TAB1 == (t1["rho"]["L"], t1["rho"]["I"], t1["rho"]["G"])
    assert pi.C_TAB1 == (t1["c"]["L"], t1["c"]["I"], t1["c"]["G"])
    assert pi.LAM_TAB1 == (t1["lambda"]["L"], t1["lambda"]["I"], t1["lambda"]["G"])
    assert pi.L_TAB1 == t1["L"]


# --------------------------------------------------------------------------
# Pointwise pieces

def test_sigma_limiter_properties():
    e0, e1 = 0.05, 0.2
    assert oracle.sigma(e0, e0, e1) == 0.0 and oracle.sigma(-1.0, e0, e1) == 0.0
    assert oracle.sigma(e1, e0, e1) == 1.0 and oracle.sigma(0.9, e0, e1) == 1.0
    assert abs(oracle.sigma(0.5 * (e0 + e1), e0, e1) - 0.5) < 1e-15
    d = 1e-7
    # C^1 at both knots: one-sided slopes vanish
    assert abs(oracle.sigma(e0 + d, e0, e1) / d) < 1e-4
    assert abs((1.0 - oracle.sigma(e1 - d, e0, e1)) / d) < 1e-4
    w = np.linspace(e0, e1, 101)
    v = [oracle.sigma(x, e0, e1) for x in w]
    assert np.all(np.diff(v) > 0)


def test_water_indicator():
    assert oracle.water_indicator(0.0, 2.0) == 1.0
    assert oracle.water_indicator(0.5, 2.0) == 0.0
    assert oracle.water_indicator(1.0, 2.0) == 0.0
    assert oracle.water_indicator(0.25, 2.0) == 0.5
    assert oracle.water_indicator(0.5, 1.0) == 0.5


# --------------------------------------------------------------------------
# Brute force on tiny grids

def _tiny_params(model, shape, rng, faces=0, bc_kind=0):
    n3, n2, n1 = shape
    p = dict(n1=n1, n2=n2, n3=n3, h=2.1e-4, xi=2.1e-4, alpha=4.17e6, mu=1e-4, b=1.0,
             eps0=0.05, eps1=0.2, zeta=2.0, t_star=273.15, dT=0.7,
             lam=(0.6, 2.2, 1.0), rhoc=(4.2e6, 1.9e6, 2.0e6), Lv=3.34e8,
             dirichlet_faces=faces, bc_kind=bc_kind, bc_T0=268.15, bc_T1=278.15,
             bc_t0=0.0, bc_t1=2.0, model=model, phi_face_mask=1)
    return p


@pytest.mark.parametrize("model", ["ac", "coupled"])
@pytest.mark.parametrize("shape", [(3, 3, 3), (4, 3, 5), (5, 4, 2), (1, 1, 6)])
def test_rhs_matches_brute_force(model, shape):
    rng = np.random.default_rng(zlib.crc32(f"{model}-{shape}".encode()))
    for trial in range(3):
        faces = int(rng.integers(0, 64))
        p = _tiny_params(model, shape, rng, faces=faces, bc_kind=int(rng.integers(0, 3)))
        G = (rng.random(shape) < 0.3).astype(float)
        phi = rng.random(shape)
        phi[rng.random(shape) < 0.3] = 0.0
        phi[rng.random(shape) < 0.2] = 1.0
        T = 273.15 + rng.normal(0, 3, shape)
        P = oracle.make_params(p)
        t = float(rng.random() * 3)
        kp, kT = oracle.rhs(P, G, t, phi, T if model == "coupled" else None)
        bp, bT = brute.rhs(p, G, t, phi, T)
        scale = max(np.abs(bp).max(), 1e-300)
        assert np.abs(kp - bp).max() <= 1e-13 * scale
        if model == "coupled":
            assert np.abs(kT - bT).max() <= 1e-13 * np.abs(bT).max()
        # glass cells never evolve (I_W = 0 for G = 1, zeta = 2)
        assert np.all(kp[G == 1] == 0.0)


@pytest.mark.parametrize("model", ["ac", "coupled"])
def test_merson_step_matches_brute_force(model):
    rng = np.random.default_rng(7 if model == "ac" else 8)
    shape = (4, 3, 4)
    p = _tiny_params(model, shape, rng, faces=(1 << 4) | (1 << 1), bc_kind=1)
    if model == "ac":
        p.update(h=31.25e-6, xi=1.5 * 31.25e-6, alpha=3.39782e11 / 100, dT=0.3)
    G = (rng.random(shape) < 0.25).astype(float)
    phi = np.clip(rng.random(shape) * 1.2 - 0.1, 0, 1)
    T = 273.15 + rng.normal(0, 2, shape)
    P = oracle.make_params(p)
    ctl = oracle.make_ctl(tol=0.0)
    dt = 2e-3 if model == "coupled" else 0.5
    ph, TT, t1, dt1, info = oracle.rkm_step(P, G, ctl, 0.3, dt, phi,
                                            T if model == "coupled" else None)
    bph, bT, berr = brute.merson_step(p, G, 0.3, dt, phi, T)
    assert info["accepted"] == 1 and t1 == 0.3 + dt
    assert np.abs(ph - bph).max() <= 1e-13
    if model == "coupled":
        assert np.abs(TT - bT).max() <= 1e-12 * np.abs(bT - 273.15).max()
    assert abs(info["eps"] - berr) <= 1e-9 * berr + 1e-300


def test_mirror_and_permutation_symmetry():
    rng = np.random.default_rng(3)
    shape = (6, 6, 6)
    p = _tiny_params("coupled", shape, rng, faces=0)
    G = (rng.random(shape) < 0.3).astype(float)
    phi = rng.random(shape)
    T = 273.15 + rng.normal(0, 1, shape)
    P = oracle.make_params(p)
    kp, kT = oracle.rhs(P, G, 0.0, phi, T)
    for ax in range(3):
        f = lambda a: np.flip(a, axis=ax).copy()
        mp, mT = oracle.rhs(P, f(G), 0.0, f(phi), f(T))
        assert np.abs(mp - f(kp)).max() <= 1e-12 * np.abs(kp).max()
        assert np.abs(mT - f(kT)).max() <= 1e-12 * np.abs(kT).max()
    perm = lambda a: np.transpose(a, (1, 2, 0)).copy()
    mp, mT = oracle.rhs(P, perm(G), 0.0, perm(phi), perm(T))
    assert np.abs(mp - perm(kp)).max() <= 1e-12 * np.abs(kp).max()
    assert np.abs(mT - perm(kT)).max() <= 1e-12 * np.abs(kT).max()


# --------------------------------------------------------------------------
# P1: planar tanh travelling front

def _front_position(phi_line, h):
    """x where phi crosses 1/2 (linear interpolation), cell centres at (i+1/2)h."""
    s = phi_line - 0.5
    i = int(np.nonzero((s[:-1] < 0) & (s[1:] >= 0))[0][0])
    x0 = (i + 0.5) * h
    return x0 + h * (-s[i]) / (s[i + 1] - s[i])


def _front_speed(xi_over_h, beta, n=240, reaction="sigma", cross=None):
    # nondimensional: h = 1, alpha = 1, mu = 0.1, dT set by beta = xi mu alpha dT / 2
    h, alpha, mu = 1.0, 1.0, 0.1
    xi = xi_over_h * h
    dT = 2 * beta / (xi * mu * alpha)
    n1 = n2 = 1 if cross is None else cross
    p = dict(n1=n1, n2=n2, n3=n, h=h, xi=xi, alpha=alpha, mu=mu, b=1.0,
             eps0=-2.0, eps1=-1.0, zeta=2.0, t_star=0.0, dT=dT, lam=(1, 1, 1),
             rhoc=(1, 1, 1), Lv=0.0, model="ac", reaction=reaction, phi_face_mask=1)
    P = oracle.make_params(p)
    x = (np.arange(n) + 0.5) * h
    x0 = 0.55 * n * h
    phi = 0.5 * (1 + np.tanh((x - x0) / (2 * xi)))
    phi = np.broadcast_to(phi[:, None, None], (n, n2, n1)).copy()
    G = np.zeros_like(phi)
    ctl = oracle.make_ctl(tol=0.0)
    v = mu * dT
    dt = 0.25 * alpha * h * h  # z = 1 for the stiffest Laplacian mode
    t_relax = 20.0 * alpha * xi * xi
    t_meas = 0.1 * n * h / max(v, 1e-12) if v > 0 else 50.0 * alpha * xi * xi
    phi, _, _ = oracle.integrate(P, G, ctl, 0.0, dt, phi, t_end=t_relax)
    xa = _front_position(phi[:, 0, 0], h)
    phi2, _, _ = oracle.integrate(P, G, ctl, t_relax, dt, phi, t_end=t_relax + t_meas)
    xb = _front_position(phi2[:, 0, 0], h)
    return (xb - xa) / t_meas, v, phi2


def test_tanh_front_speed_converges_second_order():
    errs = []
    for r in (2.0, 4.0):
        speed, v, _ = _front_speed(r, beta=0.2)
        assert speed < 0  # ice (phi = 1 at large x3) grows: the front moves to -x3
        errs.append(abs(-speed - v) / v)
    assert errs[1] < 0.02
    ratio = errs[0] / errs[1]
    assert 3.0 < ratio < 5.5, (errs, ratio)  # O((h/xi)^2): x4 per halving of h/xi


def test_tanh_front_stationary_without_supercooling():
    speed, v, _ = _front_speed(3.0, beta=0.0)
    assert v == 0.0 and abs(speed) < 1e-6


def test_front_3d_equals_1d():
    s1, _, phi1 = _front_speed(3.0, beta=0.2, n=120)
    s3, _, phi3 = _front_speed(3.0, beta=0.2, n=120, cross=3)
    assert abs(s1 - s3) <= 1e-12 * abs(s1)
    assert np.abs(phi3 - phi1[:, :1, :1]).max() <= 1e-13


def test_gradp_front_speed():
    """The GradP reaction (eq. reaction-term-GradP) admits the same travelling
    profile: its drive xi^2 mu alpha |grad phi| dT equals 2 beta phi (1 - phi)
    on the tanh profile."""
    errs = []
    for r in (3.0, 6.0):
        speed, v, _ = _front_speed(r, beta=0.2, reaction="gradp")
        errs.append(abs(-speed - v) / v)
    assert errs[1] < 0.02 and errs[1] < errs[0]


# --------------------------------------------------------------------------
# P2: heat-equation eigenmodes

def _merson_R(z):
    return 1 + z + z**2 / 2 + z**3 / 6 + z**4 / 24 + z**5 / 144


def _heat_case(shape, faces):
    n3, n2, n1 = shape
    lam, rc = 0.6, 4.2e6
    p = dict(n1=n1, n2=n2, n3=n3, h=1e-3, xi=1e-3, alpha=1e6, mu=1e-4, b=1.0, eps0=0.05,
             eps1=0.2, zeta=2.0, t_star=273.15, dT=0.0, lam=(lam, 2.2, 1.0),
             rhoc=(rc, 1.9e6, 2.0e6), Lv=3.34e8, dirichlet_faces=faces, bc_kind=0,
             bc_T0=280.0, bc_T1=280.0, bc_t0=0, bc_t1=0, model="coupled", phi_face_mask=1)
    return p, lam / rc


@pytest.mark.parametrize("dirichlet", [False, True])
def test_heat_modes_decay_exactly(dirichlet):
    shape = (7, 5, 6)
    n3, n2, n1 = shape
    p, kappa = _heat_case(shape, (1 << 4) if dirichlet else 0)
    h = p["h"]
    k1, k2, k3 = 2, 1, 3
    i1, i2, i3 = np.arange(n1) + 0.5, np.arange(n2) + 0.5, np.arange(n3) + 0.5
    m1 = np.cos(k1 * np.pi * i1 / n1)
    m2 = np.cos(k2 * np.pi * i2 / n2)
    ev = -4 / h**2 * (np.sin(k1 * np.pi / (2 * n1))**2 + np.sin(k2 * np.pi / (2 * n2))**2)
    if dirichlet:
        m3 = np.sin((k3 + 0.5) * np.pi * i3 / n3)
        ev += -4 / h**2 * np.sin((k3 + 0.5) * np.pi / (2 * n3))**2
    else:
        m3 = np.cos(k3 * np.pi * i3 / n3)
        ev += -4 / h**2 * np.sin(k3 * np.pi / (2 * n3))**2
    mode = m3[:, None, None] * m2[None, :, None] * m1[None, None, :]
    base = 280.0
    amp = 2.0
    T = base + amp * mode
    phi = np.zeros(shape)
    G = np.zeros(shape)
    P = oracle.make_params(p)
    z = None
    dt = 0.6 / (kappa * abs(ev))
    z = dt * kappa * ev
    ctl = oracle.make_ctl(tol=0.0)
    steps = 12
    ph, TT, st = oracle.integrate(P, G, ctl, 0.0, dt, phi, T, max_steps=steps)
    assert st["steps_accepted"] == steps
    assert np.all(ph == 0.0)  # phi = 0 is an exact rest state of the phase equation
    expect = base + amp * _merson_R(z) ** steps * mode
    assert np.abs(TT - expect).max() <= 1e-12 * amp
    # one step's error estimate: |E| = |z^5 / 720| * amplitude for a linear mode
    _, _, _, _, info = oracle.rkm_step(P, G, ctl, 0.0, dt, phi, T)
    assert abs(info["eps"] - abs(z**5 / 720) * amp * np.abs(mode).max()) <= 1e-9 * info["eps"]


def test_merson_stability_polynomial_error_term():
    # R(z) - e^z = -z^5/720 + O(z^6)
    for z in (1e-2, 2e-2):
        assert abs((_merson_R(z) - math.exp(z)) / (-z**5 / 720) - 1) < 1.5 * z


# --------------------------------------------------------------------------
# P3: enthalpy

def test_rhs_enthalpy_balance_insulated():
    rng = np.random.default_rng(11)
    shape = (9, 7, 8)
    p = _tiny_params("coupled", shape, rng, faces=0)
    G = (rng.random(shape) < 0.35).astype(float)
    phi = rng.random(shape)
    T = 273.15 + rng.normal(0, 2, shape)
    P = oracle.make_params(p)
    kp, kT = oracle.rhs(P, G, 0.0, phi, T)
    rc = G * p["rhoc"][2] + (1 - G) * (phi * p["rhoc"][1] + (1 - phi) * p["rhoc"][0])
    balance = np.sum(rc * kT) - p["Lv"] * np.sum(kp)
    assert abs(balance) <= 1e-12 * np.sum(np.abs(rc * kT))
    # with a Dirichlet face the same balance picks up exactly the boundary flux
    p2 = dict(p, dirichlet_faces=1 << 4, bc_T0=265.0)
    P2 = oracle.make_params(p2)
    kp2, kT2 = oracle.rhs(P2, G, 0.0, phi, T)
    lam = G * 1.0 + (1 - G) * (phi * 2.2 + (1 - phi) * 0.6)
    flux_in = np.sum(2 * lam[0] * (265.0 - T[0])) / p["h"]**2
    bal2 = np.sum(rc * kT2) - p["Lv"] * np.sum(kp2)
    assert abs(bal2 - flux_in) <= 1e-10 * abs(flux_in)


def test_enthalpy_conserved_over_steps_equal_heat_capacity():
    rng = np.random.default_rng(12)
    shape = (8, 8, 8)
    p = _tiny_params("coupled", shape, rng, faces=0)
    p["rhoc"] = (3.0e6, 3.0e6, 3.0e6)
    G = (rng.random(shape) < 0.3).astype(float)
    phi = np.clip(rng.random(shape) * 1.4 - 0.2, 0, 1)
    T = 273.15 + rng.normal(0, 1, shape)
    P = oracle.make_params(p)
    H0 = oracle.diagnostics(P, G, phi, T)["enthalpy"]
    ctl = oracle.make_ctl(tol=0.0)
    ph, TT, st = oracle.integrate(P, G, ctl, 0.0, 2e-3, phi, T, max_steps=20)
    H1 = oracle.diagnostics(P, G, ph, TT)["enthalpy"]
    scale = p["h"]**3 * np.sum(3.0e6 * np.abs(T - 273.15) + p["Lv"] * phi)
    assert abs(H1 - H0) <= 1e-13 * scale
    assert np.abs(ph - phi).max() > 1e-3  # something actually happened


# --------------------------------------------------------------------------
# P4: order of the Merson step on a closed-form ODE

def _uniform_ode_time(phi, a):
    """Antiderivative of 1 / (phi (1 - phi) (phi - a))."""
    return (-math.log(phi) / a - math.log(1 - phi) / (1 - a)
            + math.log(abs(phi - a)) / (a * (1 - a)))


def test_merson_fourth_order_on_uniform_reaction():
    # One water cell, no neighbours: d phi/dt = (2/(alpha xi^2)) phi (1-phi) (phi - a),
    # a = 1/2 - beta with Sigma = 1 (eq. reaction-term-SigmaP1-P).
    xi, alpha, mu = 1.0, 1.0, 0.1
    beta = 0.15
    dT = 2 * beta / (xi * mu * alpha)
    p = dict(n1=1, n2=1, n3=1, h=1.0, xi=xi, alpha=alpha, mu=mu, b=1.0, eps0=-2, eps1=-1,
             zeta=2.0, t_star=0.0, dT=dT, lam=(1, 1, 1), rhoc=(1, 1, 1), Lv=0,
             model="ac", phi_face_mask=1)
    P = oracle.make_params(p)
    a = 0.5 - beta
    c = 2 / (alpha * xi * xi)
    phi0 = 0.4
    t_end = 3.0
    errs = []
    for nsteps in (10, 20, 40):
        dt = t_end / nsteps
        ph, _, st = oracle.integrate(P, np.zeros((1, 1, 1)), oracle.make_ctl(tol=0.0), 0.0, dt,
                                     np.full((1, 1, 1), phi0), t_end=t_end)
        phi_num = float(ph.ravel()[0])
        # exact: Phi(phi(t)) - Phi(phi0) = c t; convert the residual to a phi error
        resid = _uniform_ode_time(phi_num, a) - _uniform_ode_time(phi0, a) - c * t_end
        dphi = phi_num * (1 - phi_num) * (phi_num - a)
        errs.append(abs(resid * dphi))
    r1, r2 = errs[0] / errs[1], errs[1] / errs[2]
    assert 13 < r1 < 20 and 13 < r2 < 20, (errs, r1, r2)


def test_adaptive_step_controller_and_clipping():
    # scalar reaction again; the controller keeps every accepted local error <= tol
    p = dict(n1=1, n2=1, n3=1, h=1.0, xi=1.0, alpha=1.0, mu=0.1, b=1.0, eps0=-2, eps1=-1,
             zeta=2.0, t_star=0.0, dT=3.0, lam=(1, 1, 1), rhoc=(1, 1, 1), Lv=0,
             model="ac", phi_face_mask=1)
    P = oracle.make_params(p)
    ctl = oracle.make_ctl(tol=1e-8, safety=0.8, dt_min=1e-12, dt_max=0.5)
    phi = np.full((1, 1, 1), 0.3)
    t, dt = 0.0, 1.0
    G = np.zeros((1, 1, 1))
    nacc = nrej = 0
    while t < 5.0:
        phi_new, _, t_new, dt_new, info = oracle.rkm_step(P, G, ctl, t, dt, phi, t_end=5.0)
        if info["accepted"]:
            assert info["eps"] <= 1e-8
            nacc += 1
        else:
            assert info["eps"] > 1e-8 and t_new == t
            nrej += 1
        expect = min(0.5, 0.8 * info["dt_used"] * (1e-8 / info["eps"]) ** 0.2)
        assert dt_new == pytest.approx(expect, rel=1e-15)
        phi, t, dt = phi_new, t_new, dt_new
    assert t == 5.0 and nrej >= 1 and nacc > 5


# --------------------------------------------------------------------------
# P6: Gibbs-Thomson critical radius

@pytest.mark.slow
def test_gibbs_thomson_critical_radius():
    """An ice ball in supercooled water grows when R > R* = 2/(mu alpha dT) and
    shrinks below (eq. Gibbs-Thomson with v = 0, curvature 2/R).  One octant
    with zero-flux walls stands for the whole ball."""
    n = 30
    h, xi, alpha, mu = 1.0, 1.5, 1.0, 0.1
    Rstar = 12.0
    dT = 2 / (mu * alpha * Rstar)
    p = dict(n1=n, n2=n, n3=n, h=h, xi=xi, alpha=alpha, mu=mu, b=1.0, eps0=-2, eps1=-1,
             zeta=2.0, t_star=0.0, dT=dT, lam=(1, 1, 1), rhoc=(1, 1, 1), Lv=0,
             model="ac", phi_face_mask=1)
    P = oracle.make_params(p)
    G = np.zeros((n, n, n))
    i = np.arange(n) + 0.5
    r = np.sqrt(i[:, None, None]**2 + i[None, :, None]**2 + i[None, None, :]**2)
    rates = {}
    for R0 in (7.0, 19.0):
        phi = 0.5 * (1 - np.tanh((r - R0) / (2 * xi)))
        ctl = oracle.make_ctl(tol=0.0)
        dt = 0.2
        ph1, _, _ = oracle.integrate(P, G, ctl, 0.0, dt, phi, t_end=10.0)
        ph2, _, _ = oracle.integrate(P, G, ctl, 10.0, dt, ph1, t_end=20.0)
        R1 = (3 * 8 * ph1.sum() / (4 * math.pi)) ** (1 / 3)
        R2 = (3 * 8 * ph2.sum() / (4 * math.pi)) ** (1 / 3)
        rates[R0] = ((R2 - R1) / 10.0, 0.5 * (R1 + R2))
    (v_small, Rs), (v_big, Rb) = rates[7.0], rates[19.0]
    assert v_small < 0 < v_big
    for v, R in ((v_small, Rs), (v_big, Rb)):
        theory = mu * dT - 2 / (alpha * R)
        assert abs(v - theory) <= 0.3 * abs(theory) + 0.1 * mu * dT, (v, theory, R)


@pytest.mark.parametrize("model,reaction", [("ac", "gradp"), ("coupled", "gradp"),
                                            ("temp", "sigma")])
@pytest.mark.parametrize("shape", [(3, 3, 3), (4, 3, 5), (1, 2, 6)])
def test_rhs_variants_match_brute_force(model, reaction, shape):
    """GradP reaction (eq. reaction-term-GradP) and the Temp model (Sec. 2.3)
    against the dense transcription."""
    rng = np.random.default_rng(zlib.crc32(f"{model}-{reaction}-{shape}".encode()))
    for trial in range(3):
        p = _tiny_params(model, shape, rng, faces=int(rng.integers(0, 64)),
                         bc_kind=int(rng.integers(0, 3)))
        p["reaction"] = reaction
        p["gamma"] = 1.5
        G = (rng.random(shape) < 0.3).astype(float)
        phi = rng.random(shape)
        phi[G == 1] = 0.0
        T = 273.15 + rng.normal(0, 1.5, shape)
        P = oracle.make_params(p)
        t = float(rng.random() * 3)
        if model == "temp":
            kp, kT = oracle.rhs(P, G, t, None, T)
        else:
            kp, kT = oracle.rhs(P, G, t, phi, T if model == "coupled" else None)
        bp, bT = brute.rhs(p, G, t, phi, T)
        # Temp model: the phase rate carries varphi'(T), whose 1 - tanh^2 the
        # two implementations evaluate differently (~1e-12 relative)
        tol_p = 1e-11 if model == "temp" else 1e-13
        assert np.abs(kp - bp).max() <= tol_p * max(np.abs(bp).max(), 1e-300)
        if model != "ac":
            assert np.abs(kT - bT).max() <= 1e-13 * np.abs(bT).max()


def test_temp_model_enthalpy_balance_insulated():
    """Temp model with insulated faces: sum over cells of
    (rho c - L_v varphi'(T)) dT/dt is the sum of the face fluxes, zero."""
    rng = np.random.default_rng(31)
    shape = (6, 5, 7)
    p = _tiny_params("temp", shape, rng, faces=0, bc_kind=0)
    p["gamma"] = 2.0
    G = (rng.random(shape) < 0.3).astype(float)
    T = 273.15 + rng.normal(0, 0.7, shape)
    P = oracle.make_params(p)
    kp, kT = oracle.rhs(P, G, 0.0, None, T)
    ph, dph = brute.temp_phase(p, G, T)
    rc = brute.blend(G, ph, p["rhoc"])
    w = (rc - p["Lv"] * dph) * kT
    assert abs(w.sum()) <= 1e-12 * np.abs(w).sum()
    # the phase rate is varphi'(T) times the temperature rate (1 - tanh^2
    # cancels, so two tanh implementations agree to ~1e-12 relative only)
    assert np.allclose(kp, dph * kT, rtol=1e-9, atol=0)


def test_temp_model_far_from_melting_is_pure_conduction():
    """Away from T* (|gamma (T - T*)| large) varphi is constant, the latent
    term vanishes, and water cells conduct as the liquid (T > T*): a cosine
    mode of an all-water box decays at the discrete Neumann rate."""
    n1, h = 8, 1e-3
    p = _tiny_params("temp", (1, 1, n1), np.random.default_rng(0), faces=0, bc_kind=0)
    p.update(h=h, gamma=200.0, lam=(0.6, 2.2, 1.0), rhoc=(4.2e6, 1.9e6, 2.0e6))
    G = np.zeros((1, 1, n1))
    i = np.arange(n1)
    k = 2
    T = 273.15 + 5.0 + 0.1 * np.cos(k * np.pi * (i + 0.5) / n1).reshape(1, 1, n1)
    P = oracle.make_params(p)
    _, kT = oracle.rhs(P, G, 0.0, None, T)
    lam_k = -4.0 / h ** 2 * np.sin(k * np.pi / (2 * n1)) ** 2
    want = 0.6 / 4.2e6 * lam_k * (T - 278.15)
    assert np.allclose(kT, want, rtol=1e-10, atol=1e-18)


@pytest.mark.parametrize("model,reaction", [("ac", "sigma"), ("coupled", "sigma"), ("ac", "gradp"),
                                            ("coupled", "gradp"), ("temp", "sigma")])
def test_rhs_smooth_glass_matches_brute_force(model, reaction):
    """Paper mode (Sec. 2.1): a smooth glass field G in [0, 1], the
    phase-field Laplacian across every face, I_W(G) and the blends with
    fractional G."""
    rng = np.random.default_rng(zlib.crc32(f"{model}-{reaction}-smooth".encode()))
    for shape in ((3, 4, 5), (2, 3, 6)):
        p = _tiny_params(model, shape, rng, faces=int(rng.integers(0, 64)),
                         bc_kind=int(rng.integers(0, 3)))
        p.update(reaction=reaction, phi_face_mask=0, gamma=1.7)
        G = rng.random(shape)
        G[rng.random(shape) < 0.2] = 0.0
        G[rng.random(shape) < 0.2] = 1.0
        phi = rng.random(shape)
        T = 273.15 + rng.normal(0, 1.5, shape)
        P = oracle.make_params(p)
        t = float(rng.random() * 3)
        if model == "temp":
            kp, kT = oracle.rhs(P, G, t, None, T)
        else:
            kp, kT = oracle.rhs(P, G, t, phi, T if model == "coupled" else None)
        bp, bT = brute.rhs(p, G, t, phi, T)
        # Temp model: the phase rate carries varphi'(T), whose 1 - tanh^2 the
        # two implementations evaluate differently (~1e-12 relative)
        tol_p = 1e-11 if model == "temp" else 1e-13
        assert np.abs(kp - bp).max() <= tol_p * max(np.abs(bp).max(), 1e-300)
        if model != "ac":
            assert np.abs(kT - bT).max() <= 1e-13 * np.abs(bT).max()


def test_smooth_glass_limits():
    """Paper mode reduces to the plain Allen-Cahn operator where G = 0, and a
    cell with G = 1 does not evolve (I_W = 0 for zeta = 2); with G in {0, 1}
    and no face rule, the water-water part of the Laplacian is the same as
    with it."""
    rng = np.random.default_rng(41)
    shape = (4, 4, 4)
    p = _tiny_params("ac", shape, rng)
    p["phi_face_mask"] = 0
    G = (rng.random(shape) < 0.3).astype(float)
    phi = rng.random(shape)
    kp, _ = oracle.rhs(oracle.make_params(p), G, 0.0, phi)
    assert np.all(kp[G == 1] == 0)
    kp0, _ = oracle.rhs(oracle.make_params(p), np.zeros(shape), 0.0, phi)
    p1 = dict(p, phi_face_mask=1)
    kp1, _ = oracle.rhs(oracle.make_params(p1), np.zeros(shape), 0.0, phi)
    assert np.array_equal(kp0, kp1)


# --------------------------------------------------------------------------
# The paper's own material model: rho and c blended separately (eq.
# material-properties-blending-formula applied to each of c, lambda, rho),
# rho c = blend(rho) blend(c), latent term blend(rho) L (eq. heat-equation).

def _tab1_params(model, shape, faces=0, bc_kind=0):
    t1 = GOLD["table1"]
    p = _tiny_params(model, shape, None, faces=faces, bc_kind=bc_kind)
    p.update(rho_c_separate=1,
             rho=(t1["rho"]["L"], t1["rho"]["I"], t1["rho"]["G"]),
             cs=(t1["c"]["L"], t1["c"]["I"], t1["c"]["G"]),
             lam=(t1["lambda"]["L"], t1["lambda"]["I"], t1["lambda"]["G"]),
             L=t1["L"], gamma=2.0)
    return p


@pytest.mark.parametrize("model", ["coupled", "temp"])
@pytest.mark.parametrize("smooth", [False, True])
def test_separate_rho_c_matches_brute_force(model, smooth):
    rng = np.random.default_rng(401 if model == "coupled" else 402)
    shape = (4, 3, 5)
    for trial in range(3):
        p = _tab1_params(model, shape, faces=int(rng.integers(0, 64)), bc_kind=trial)
        if smooth:
            p["phi_face_mask"] = 0
            G = rng.random(shape)
            G[rng.random(shape) < 0.3] = 0.0
        else:
            G = (rng.random(shape) < 0.3).astype(float)
        phi = rng.random(shape)
        T = 273.15 + rng.normal(0, 1.0, shape)
        P = oracle.make_params(p)
        if model == "temp":
            kp, kT = oracle.rhs(P, G, 0.7, None, T)
        else:
            kp, kT = oracle.rhs(P, G, 0.7, phi, T)
        bp, bT = brute.rhs(p, G, 0.7, phi, T)
        assert np.abs(kT - bT).max() <= 1e-12 * np.abs(bT).max()
        assert np.abs(kp - bp).max() <= 1e-11 * max(np.abs(bp).max(), 1e-300)


def test_separate_rho_c_with_unit_density_is_the_volumetric_form():
    """rho = 1 everywhere and c = the volumetric values: the two material
    models coincide (rho c and rho L reduce to rhoc and L)."""
    rng = np.random.default_rng(403)
    shape = (5, 4, 6)
    p = _tiny_params("coupled", shape, rng, faces=1 << 4, bc_kind=1)
    q = dict(p, rho_c_separate=1, rho=(1.0, 1.0, 1.0), cs=p["rhoc"], L=p["Lv"])
    G = (rng.random(shape) < 0.3).astype(float)
    phi, T = rng.random(shape), 273.15 + rng.normal(0, 2, shape)
    a = oracle.rhs(oracle.make_params(p), G, 0.4, phi, T)
    b = oracle.rhs(oracle.make_params(q), G, 0.4, phi, T)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])


@pytest.mark.parametrize("phi_value", [0.0, 0.5, 1.0])
def test_separate_rho_c_conduction_rate_of_a_uniform_phase(phi_value):
    """A uniform phase state (no phase change: phi constant, T > T* far from
    the drive) with a cosine temperature mode: dT/dt = -(lambda/(rho c)) k^2-rate
    of the discrete Neumann Laplacian, with rho c the product of the blended
    density and specific heat -- at phi = 1/2 that is
    (rho_L + rho_I)(c_L + c_I)/4, not the blend of the products."""
    t1 = GOLD["table1"]
    n1 = 12
    shape = (1, 1, n1)
    p = _tab1_params("coupled", shape)
    p.update(b=0.0)  # no drive: the reaction term keeps phi = 0, 1/2, 1 stationary
    G = np.zeros(shape)
    phi = np.full(shape, phi_value)
    k = 2
    i = np.arange(n1)
    mode = np.cos(k * np.pi * (i + 0.5) / n1).reshape(shape)
    T = 290.0 + 0.1 * mode
    kp, kT = oracle.rhs(oracle.make_params(p), G, 0.0, phi, T)
    assert np.all(kp == 0.0)
    rho = (1 - phi_value) * t1["rho"]["L"] + phi_value * t1["rho"]["I"]
    c = (1 - phi_value) * t1["c"]["L"] + phi_value * t1["c"]["I"]
    lam = (1 - phi_value) * t1["lambda"]["L"] + phi_value * t1["lambda"]["I"]
    eig = -4.0 / p["h"]**2 * math.sin(k * math.pi / (2 * n1))**2
    expect = lam / (rho * c) * eig * 0.1 * mode
    assert np.abs(kT - expect).max() <= 1e-12 * np.abs(expect).max()


def test_separate_rho_c_enthalpy_balance_insulated():
    """Insulated box: sum of rho c k_T minus sum of rho L k_phi over the cells
    is the sum of the face fluxes, zero."""
    rng = np.random.default_rng(404)
    shape = (6, 7, 5)
    p = _tab1_params("coupled", shape, faces=0)
    G = (rng.random(shape) < 0.35).astype(float)
    phi, T = rng.random(shape), 273.15 + rng.normal(0, 2, shape)
    kp, kT = oracle.rhs(oracle.make_params(p), G, 0.0, phi, T)
    rc = brute.blend(G, phi, p["rho"]) * brute.blend(G, phi, p["cs"])
    lat = brute.blend(G, phi, p["rho"]) * p["L"]
    w = rc * kT - lat * kp
    assert abs(w.sum()) <= 1e-12 * np.abs(rc * kT).sum()
