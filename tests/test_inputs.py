"""Seeded synthetic input generator: determinism, geometry rules, nuclei."""
import math

import numpy as np
import pytest

import pf_inputs as pi


def _splitmix_scalar(seed, n):
    """SplitMix64 written out with Python integers (Steele, Lea, Flood 2014)."""
    m = (1 << 64) - 1
    s = seed & m
    out = []
    for _ in range(n):
        s = (s + 0x9E3779B97F4A7C15) & m
        z = s
        z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & m
        z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & m
        out.append(z ^ (z >> 31))
    return out


def test_splitmix_vectorised_matches_scalar():
    for seed in (0, 1, 4000, 2**63 + 5):
        g = pi.SplitMix64(seed)
        a = [int(v) for v in g.next_u64(7)] + [g.next_u64()]
        assert a == _splitmix_scalar(seed, 8)
    u = pi.SplitMix64(3).uniform(1000)
    assert np.all((u >= 0) & (u < 1))


def test_rsa_nonoverlap_and_determinism():
    shape = (40, 36, 32)
    r = 5.5
    c1, m1 = pi.rsa_spheres(shape, r, pi.SplitMix64(9), n_spheres=20)
    c2, m2 = pi.rsa_spheres(shape, r, pi.SplitMix64(9), n_spheres=20)
    assert np.array_equal(c1, c2) and np.array_equal(m1, m2)
    box = np.array([32, 36, 40], float)
    for i in range(len(c1)):
        d = c1[i + 1:] - c1[i]
        d -= box * np.round(d / box)
        assert np.all(np.sum(d * d, axis=1) >= (2 * r) ** 2)
    assert np.array_equal(pi.voxelize(shape, c1, r), m1)


def test_voxelize_rule_brute_force():
    shape = (10, 12, 9)
    c = np.array([[1.2, 11.5, 4.4], [6.0, 3.3, 9.7]])
    r = 3.1
    m = pi.voxelize(shape, c, r)
    n3, n2, n1 = shape
    for i3 in range(n3):
        for i2 in range(n2):
            for i1 in range(n1):
                glass = False
                for cc in c:
                    d = np.array([i1 + .5, i2 + .5, i3 + .5]) - cc
                    d -= np.array([n1, n2, n3]) * np.round(d / np.array([n1, n2, n3]))
                    glass |= float(d @ d) <= r * r
                assert m[i3, i2, i1] == glass


def test_edt_matches_brute_force():
    rng = np.random.default_rng(1)
    mask = (rng.random((7, 6, 5)) < 0.2).astype(np.uint8)
    d2 = pi.edt2_to_glass(mask)
    n3, n2, n1 = mask.shape
    glass = [(i1, i2, i3) for i3 in range(-1, n3 + 1) for i2 in range(-1, n2 + 1)
             for i1 in range(-1, n1 + 1)
             if not (0 <= i1 < n1 and 0 <= i2 < n2 and 0 <= i3 < n3) or mask[i3, i2, i1]]
    g = np.array(glass)
    for i3 in range(n3):
        for i2 in range(n2):
            for i1 in range(n1):
                best = int(np.min(np.sum((g - [i1, i2, i3]) ** 2, axis=1)))
                assert d2[i3, i2, i1] == best


def test_micro_32_case():
    c = pi.case_micro_32()
    assert c.mask.shape == (32, 32, 32) and c.mask.dtype == np.uint8
    assert 0.15 < c.mask.mean() < 0.30
    assert np.all(c.phi0[c.mask == 1] == 0)
    assert set(np.unique(c.phi0)) <= {0.0, 1.0}
    assert c.phi0.sum() > 0
    again = pi.case_micro_32()
    assert np.array_equal(c.mask, again.mask) and np.array_equal(c.phi0, again.phi0)
    assert c.params["xi"] == 1.5 * c.params["h"] and c.params["dT"] == 0.5


def test_coupled_128_case():
    c = pi.case_coupled_128()
    assert c.meta["spheres"] == 64
    assert 0.33 < c.meta["solid_fraction"] < 0.37
    assert c.params["dirichlet_faces"] == 1 << 4
    assert np.all(c.T0 == pi.T_STAR + 1.0)
    # the nucleus is a disk near the bottom face, pore cells only
    z = np.nonzero(c.phi0.sum(axis=(1, 2)))[0]
    assert z.min() >= 3 and z.max() <= 16
    assert np.all(c.phi0[c.mask == 1] == 0)


def test_sweep_instances_draws():
    for seed in (4000, 4005, 4019):
        s = pi.sweep_instance(seed)
        m = s.meta
        assert m["edge"] in (48, 64, 80, 96)
        assert 5 <= m["radius_vox"] <= 12
        assert 0.02 <= m["dT"] <= 2.0
        assert m["sigma_scale"] in (1.0, 10.0, 100.0, 1000.0)
        assert s.params["alpha"] == pytest.approx(pi.ALPHA_REAL / m["sigma_scale"])
        assert 0.28 <= m["solid_fraction"] <= 0.42
        assert s.phi0.sum() > 0 and np.all(s.phi0[s.mask == 1] == 0)
        # the stiffest phase-field mode times the tolerance stays below half
        # the equilibrium threshold
        lam_max = 12.0 / (s.params["alpha"] * s.params["h"] ** 2)
        assert s.run["tol"] <= 1e-6 and lam_max * s.run["tol"] <= 0.5 * s.run["eq_tol"] * 1.0001
    w = pi.warmstart_instance(10000)
    assert w.mask.shape == (96, 96, 96)


def test_crop_case():
    c = pi.case_micro_32()
    k = pi.crop_case(c, lo=(4, 8, 0), size=(16, 12, 10))
    assert k.mask.shape == (10, 12, 16)
    assert np.array_equal(k.mask, c.mask[0:10, 8:20, 4:20])
    assert k.params["n1"] == 16 and k.params["n2"] == 12 and k.params["n3"] == 10


def test_paper_glass_field_and_case():
    shape = (20, 12, 14)
    c = np.array([[6.0, 5.5, 7.0]])
    G = pi.paper_glass_field(shape, c, 3.0, 0.4, x3_cap=17.0)
    assert G.min() >= 0 and G.max() <= 1
    # value at a cell centre at distance d from the sphere centre
    i1, i2, i3 = 8, 5, 7
    d = np.sqrt((i1 + 0.5 - 6.0) ** 2 + (i2 + 0.5 - 5.5) ** 2 + (i3 + 0.5 - 7.0) ** 2)
    assert G[i3, i2, i1] == pytest.approx(0.5 * (1 - np.tanh((d - 3.0) / 0.8)), abs=1e-15)
    # the cap: 1/2 at x3 = x3_cap, -> 1 above
    assert G[19, 0, 0] == pytest.approx(0.5 * (1 + np.tanh((19.5 - 17.0) / 0.8)))
    d0 = np.sqrt((0.5 - 6.0) ** 2 + (0.5 - 5.5) ** 2 + (0.5 - 7.0) ** 2)
    assert G[0, 0, 0] == pytest.approx(0.5 * (1 - np.tanh((d0 - 3.0) / 0.8)), rel=1e-12)
    k = pi.case_paper(40, seed=5)
    assert k.mask.shape == (40, 20, 20) and k.G.shape == k.mask.shape
    assert np.array_equal(k.mask, (k.G >= 0.5).astype(np.uint8))
    assert k.params["phi_face_mask"] == 0 and k.params["dirichlet_faces"] == 1 << 5
    assert k.params["rho_c_separate"] == 1 and k.params["L"] == pi.L_TAB1
    assert pi.case_paper(40, seed=5, materials="cases").params.get("rho_c_separate", 0) == 0
    # cap from 11/12 L3 up; nucleation disk inside 0.87..0.97 L3
    x3 = np.arange(40) + 0.5
    assert np.all(k.mask[x3 > 11 / 12 * 40 + 1] == 1)
    z = np.nonzero(k.phi0.sum(axis=(1, 2)))[0]
    assert (z.min() + 0.5) > 0.87 * 40 and (z.max() + 0.5) < 0.97 * 40
