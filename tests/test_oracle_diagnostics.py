"""Pins of the oracle's counting diagnostics on hand-built grids with known
totals (Sec. 3.1 eqs. water-occupied-subdomain and frozen-subdomain; Sec. 3.3
eq. UWC-formula), and of the nucleus-component reference of the warm start.

The grids put cells exactly on the thresholds (phi = 1/2, G = 1/2), give
glass cells phi > 1/2 and put different totals in the bottom half, the
middle plane and the top half, so that a slip -- ">= 1/2" for "> 1/2",
"G <= 1/2" for "G < 1/2", ice counted over every cell, the wrong half, the
middle plane included -- changes a total.  The expected totals were counted
by hand from the cell lists below.
"""
import math

import numpy as np
import pytest

import oracle
from oracle import unet as U

T_STAR = 273.15


def _params(n1, n2, n3, model="ac", dT=0.5, gamma=2.0):
    return oracle.make_params(dict(
        n1=n1, n2=n2, n3=n3, model=model, h=1e-3, xi=1e-3, alpha=1.0, mu=1e-4, b=1.0,
        eps0=0.05, eps1=0.2, zeta=2.0, t_star=T_STAR, dT=dT, gamma=gamma,
        lam=(0.6, 2.2, 1.0), rhoc=(4.2e6, 1.9e6, 2.0e6), Lv=3.34e8))


def test_diagnostics_counts_on_thresholds():
    # 4 x 1 x 2 grid, cell n = i1 + 4 i3: (G, phi) and what each cell is
    cells = [
        (0.0, 0.0),                   # water
        (0.0, 0.5),                   # water, not ice (phi exactly 1/2)
        (0.0, 0.5 + 2.0 ** -40),      # water, ice
        (0.5, 1.0),                   # not water (G exactly 1/2), so not ice
        (0.25, 0.75),                 # water, ice
        (1.0, 1.0),                   # glass: neither
        (0.5 - 2.0 ** -40, 1.0),      # water, ice
        (0.0, 0.2),                   # water
    ]
    G = np.array([c[0] for c in cells]).reshape(2, 1, 4)
    phi = np.array([c[1] for c in cells]).reshape(2, 1, 4)
    d = oracle.diagnostics(_params(4, 1, 2), G, phi)
    assert d["pore_count"] == 6
    assert d["ice_count"] == 3
    # 0 + 0.5 + (0.5 + 2^-40) + 0.75 + 1 + 0.2
    assert d["sum_phi"] == 2.95 + 2.0 ** -40
    assert d["ice_fraction"] == 0.5


def test_diagnostics_enthalpy_of_uniform_phases():
    # coupled model, binary mask: H = h^3 sum(rhoc_c theta_c - Lv phi_c);
    # water at theta = +1 K: 4.2e6; ice at theta = -2 K: -2 * 1.9e6 - 3.34e8;
    # glass at theta = +3 K: 3 * 2.0e6 (the glass cell's phi is 0)
    P = _params(3, 1, 1, model="coupled")
    G = np.array([0.0, 0.0, 1.0]).reshape(1, 1, 3)
    phi = np.array([0.0, 1.0, 0.0]).reshape(1, 1, 3)
    T = T_STAR + np.array([1.0, -2.0, 3.0]).reshape(1, 1, 3)
    d = oracle.diagnostics(P, G, phi, T)
    expect = 1e-9 * (4.2e6 + (-3.8e6 - 3.34e8) + 6.0e6)
    assert math.isclose(d["enthalpy"], expect, rel_tol=1e-14)
    assert d["pore_count"] == 2 and d["ice_count"] == 1


# bottom-half UWC: 2 x 1 x 5 grid; plane i3 holds cells (i1 = 0, i1 = 1)
PLANES = [
    [(0.0, 1.0), (0.0, 0.5)],   # i3 = 0: water 2, ice 1
    [(0.5, 1.0), (0.3, 0.9)],   # i3 = 1: water 1 (G = 0.3), ice 1
    [(0.0, 1.0), (0.0, 1.0)],   # i3 = 2: centre exactly at half height, excluded
    [(0.0, 0.0), (0.0, 0.0)],   # i3 = 3: top half
    [(0.0, 0.0), (1.0, 1.0)],   # i3 = 4: top half
]


def _grid(planes):
    G = np.array([[c[0] for c in p] for p in planes]).reshape(len(planes), 1, 2)
    phi = np.array([[c[1] for c in p] for p in planes]).reshape(len(planes), 1, 2)
    return G, phi


def test_uwc_bottom_half_odd_height():
    G, phi = _grid(PLANES)
    u = oracle.uwc_bottom_half(_params(2, 1, 5), G, phi)
    assert (u["water_cells"], u["ice_cells"]) == (3, 2)
    assert u["uwc"] == 1.0 - 2.0 / 3.0


def test_uwc_bottom_half_even_height():
    G, phi = _grid([PLANES[0], PLANES[1], PLANES[3], PLANES[4]])
    u = oracle.uwc_bottom_half(_params(2, 1, 4), G, phi)
    assert (u["water_cells"], u["ice_cells"]) == (3, 2)
    # the whole box: water 6, ice 2 (the glass cell with phi = 1 is not ice)
    d = oracle.diagnostics(_params(2, 1, 4), G, phi)
    assert (d["pore_count"], d["ice_count"]) == (6, 2)


def test_uwc_bottom_half_temp_model():
    # Temp model: phi = 1/2 I_W(G) (1 - tanh(gamma (T - T*))), gamma = 2;
    # bottom plane of a 3 x 1 x 2 grid:
    #   G = 0,   T = T*      -> phi = 1/2 exactly: not ice
    #   G = 0,   T = T* - 1  -> phi = (1 + tanh 2)/2 = 0.982: ice
    #   G = 0.3, T = T* - 1  -> I_W = 0.4, phi = 0.393: not ice
    G = np.array([0.0, 0.0, 0.3, 0.0, 0.0, 0.0]).reshape(2, 1, 3)
    T = T_STAR + np.array([0.0, -1.0, -1.0, -5.0, -5.0, -5.0]).reshape(2, 1, 3)
    u = oracle.uwc_bottom_half(_params(3, 1, 2, model="temp"), G, None, T)
    assert (u["water_cells"], u["ice_cells"]) == (3, 1)


# nucleus component: two planes of 7 x 9 cells.  '#' glass, 'N' the nucleus
# (water, phi = 1), 'A' water face-connected to N, 'B' a sealed pocket next
# to a glass cell 'g' that holds phi = 1, 'C' a pocket touching A only along
# an edge (diagonally), 'E' a sealed pocket whose only marked cell 'h' has
# phi exactly 1/2, 'F' a single-cell pocket with phi = 0.75 (a second seed).
MAP0 = ["#########",
        "#NAA#BB##",
        "###A#g#E#",
        "#AAA###E#",
        "#AA####h#",
        "#A#CC#F##",
        "#########"]
MAP1 = ["#########",
        "######B##",
        "#########",
        "#########",
        "#########",
        "#A#######",
        "#########"]


def _nucleus_map():
    chars = np.array([[list(r) for r in MAP0], [list(r) for r in MAP1]])
    mask = np.isin(chars, ["#", "g"]).astype(np.uint8)
    phi = np.zeros(chars.shape)
    phi[chars == "N"] = 1.0
    phi[chars == "g"] = 1.0
    phi[chars == "h"] = 0.5
    phi[chars == "F"] = 0.75
    return chars, mask, phi


def test_nucleus_component_hand_map():
    chars, mask, phi = _nucleus_map()
    got = U.nucleus_component(mask, phi)
    # counted by hand: N, nine A cells in plane 0, one A cell in plane 1, F
    assert int(got.sum()) == 12
    assert np.array_equal(got, np.isin(chars, ["N", "A", "F"]))
    # pockets B (sealed, a glass neighbour with phi = 1), C (edge contact
    # only), E (phi exactly 1/2) stay out
    for c in "BCEh":
        assert not got[chars == c].any()


@pytest.mark.parametrize("slip", ["ge_half", "edge_connectivity", "glass_seeds"])
def test_nucleus_component_slips_change_the_count(slip):
    """The hand map tells the planted slips apart (each gives another count)."""
    from scipy import ndimage
    chars, mask, phi = _nucleus_map()
    water = mask == 0
    conn = 2 if slip == "edge_connectivity" else 1
    lab, _ = ndimage.label(water, structure=ndimage.generate_binary_structure(3, conn))
    seed = (phi >= 0.5) if slip == "ge_half" else (phi > 0.5)
    if slip != "glass_seeds":
        seed &= water
    else:  # a glass seed marks the water components around it
        seed = ndimage.binary_dilation(seed, ndimage.generate_binary_structure(3, 1)) & water \
            | (seed & water)
    ids = np.unique(lab[seed])
    n = int((np.isin(lab, ids[ids > 0]) & water).sum())
    assert n != 12
