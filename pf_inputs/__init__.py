"""Seeded synthetic inputs for the pore-scale freezing/thawing solver.

This module is shared by the FP64 CPU oracle and the HIP path.  It produces
*inputs only*: bead packings, solid masks, initial phase fields and
temperatures, and the per-case physical constants.  It contains none of the
solver's arithmetic (no right-hand side, no time stepping, no diagnostics).

Conventions
-----------
* Arrays are C-ordered with shape ``(n3, n2, n1)``, so the flat index of
  cell ``(i1, i2, i3)`` is ``n = i1 + n1*(i2 + n2*i3)``; x1 varies fastest and
  x3 is the vertical axis (paper, Sec. 2: the domain is a box with x3 up;
  Tab. 2 gives N1 x N2 x N3 cells).
* ``mask`` is uint8, 1 = glass, 0 = pore (water/ice).  The paper models glass
  with a smooth indicator G (Sec. 2.1); the voxel cases use the binary
  special case G in {0, 1}.
* Temperatures are in kelvin.

Geometry recipe (the paper's packings come from a discrete-element settling
run that is not available; random sequential addition stands in, Sec. 2.1 and
Sec. 3.3):
* SplitMix64 (Steele, Lea and Flood, OOPSLA 2014) with the published
  increment and mixing constants; a uniform double is ``(x >> 11) * 2**-53``.
* Random sequential addition of equal spheres in a periodic box: each attempt
  draws the centre as ``(n1*u, n2*u, n3*u)`` (three draws, in that order) and
  is accepted when its minimum-image distance to every accepted centre is at
  least ``2r``.
* A voxel is glass when the minimum-image squared distance from its centre
  ``(i + 1/2)`` to some sphere centre is ``<= r**2``.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import Dict, List, Optional, Tuple

import numpy as np
from scipy.spatial import cKDTree

__all__ = [
    "SplitMix64",
    "rsa_spheres",
    "voxelize",
    "edt2_to_glass",
    "edt_ball_nucleus",
    "disk_nucleus",
    "Case",
    "case_micro_32",
    "case_coupled_128",
    "case_coupled_256",
    "crop_case",
    "sweep_instance",
    "sweep_instances",
    "warmstart_instance",
    "paper_glass_field",
    "case_paper",
    "T_STAR",
    "ALPHA_REAL",
]

MASK64 = (1 << 64) - 1
_GAMMA = 0x9E3779B97F4A7C15
_M1 = 0xBF58476D1CE4E5B9
_M2 = 0x94D049BB133111EB

# Tab. 1: freezing point of bulk water [K] and the attachment-kinetics
# coefficient alpha = ds/(mu*sigma) for the real surface tension [s m^-2].
T_STAR = 273.15
ALPHA_REAL = 3.39782e11
# Tab. 2: "large sigma" attachment coefficient [s m^-2].
ALPHA_LARGE_SIGMA = 4.17e6
# Tab. 1: mobility [m s^-1 K^-1].
MU = 1.0e-4
# Tab. 1 physical properties (liquid, ice, glass) for the paper's own
# material model: density [kg m^-3], specific heat [J kg^-1 K^-1], heat
# conductivity [W m^-1 K^-1], specific latent heat [J kg^-1]
RHO_TAB1 = (997.0, 917.0, 2500.0)
C_TAB1 = (4180.0, 2050.0, 840.0)
LAM_TAB1 = (0.6, 2.22, 1.1)
L_TAB1 = 3.34e5


class SplitMix64:
    """SplitMix64 generator (Steele, Lea, Flood 2014).

    state_{k+1} = state_k + 0x9E3779B97F4A7C15 (mod 2^64); the output is the
    published two-multiply xor-shift mix of the new state.  Because the state
    is a counter, blocks of outputs are generated vectorised.
    """

    def __init__(self, seed: int):
        self.state = int(seed) & MASK64

    @staticmethod
    def _mix(z: np.ndarray) -> np.ndarray:
        with np.errstate(over="ignore"):
            z = (z ^ (z >> np.uint64(30))) * np.uint64(_M1)
            z = (z ^ (z >> np.uint64(27))) * np.uint64(_M2)
            return z ^ (z >> np.uint64(31))

    def next_u64(self, count: Optional[int] = None):
        n = 1 if count is None else int(count)
        k = np.arange(1, n + 1, dtype=np.uint64)
        with np.errstate(over="ignore"):
            states = np.uint64(self.state) + k * np.uint64(_GAMMA)
        self.state = (self.state + n * _GAMMA) & MASK64
        out = self._mix(states)
        return int(out[0]) if count is None else out

    def uniform(self, count: Optional[int] = None):
        """Uniform doubles in [0, 1) with 53 random bits."""
        x = self.next_u64(1 if count is None else count)
        u = (x >> np.uint64(11)).astype(np.float64) * (2.0 ** -53)
        return float(u[0]) if count is None else u

    def choice(self, values):
        u = self.uniform()
        return values[min(int(u * len(values)), len(values) - 1)]


def _wrap_delta(d: np.ndarray, n) -> np.ndarray:
    """Minimum-image difference in a periodic interval of length n."""
    return d - n * np.rint(d / n)


def _sphere_voxels(shape_zyx: Tuple[int, int, int], c: np.ndarray, r: float):
    """Index arrays (i3, i2, i1) of the voxels covered by one periodic sphere."""
    n3, n2, n1 = shape_zyx
    sizes = (n1, n2, n3)
    axes = []
    for d in range(3):
        n = sizes[d]
        lo = int(math.floor(c[d] - r - 1.0))
        hi = int(math.ceil(c[d] + r + 1.0))
        idx = np.unique(np.mod(np.arange(lo, hi + 1), n))
        delta = _wrap_delta(idx + 0.5 - c[d], float(n))
        axes.append((idx, delta * delta))
    (i1, d1), (i2, d2), (i3, d3) = axes
    inside = (d3[:, None, None] + d2[None, :, None] + d1[None, None, :]) <= r * r
    z, y, x = np.nonzero(inside)
    return i3[z], i2[y], i1[x]


def voxelize(shape_zyx, centers, r: float) -> np.ndarray:
    """Binary glass mask (uint8, 1 = glass) of periodic spheres of radius r."""
    mask = np.zeros(shape_zyx, dtype=np.uint8)
    for c in np.asarray(centers, dtype=np.float64).reshape(-1, 3):
        mask[_sphere_voxels(shape_zyx, c, r)] = 1
    return mask


def rsa_spheres(
    shape_zyx,
    r: float,
    rng: SplitMix64,
    n_spheres: Optional[int] = None,
    solid_fraction: Optional[float] = None,
    max_attempts: int = 5_000_000,
    batch: int = 4096,
    stall_attempts: Optional[int] = None,
):
    """Periodic random sequential addition of equal spheres.

    Stops after ``n_spheres`` accepted spheres, or as soon as the voxel solid
    fraction reaches ``solid_fraction``.  Raises RuntimeError when the attempt
    cap is reached first (a jammed packing), unless ``stall_attempts`` is
    given: then a run of that many consecutive rejected attempts ends the
    placement and the packing is returned as it stands.  Returns ``(centers, mask)`` with
    centers as an (m, 3) array of (x1, x2, x3) in voxel units.
    """
    if (n_spheres is None) == (solid_fraction is None):
        raise ValueError("give exactly one of n_spheres / solid_fraction")
    n3, n2, n1 = shape_zyx
    box = np.array([n1, n2, n3], dtype=np.float64)
    centers: List[np.ndarray] = []
    mask = np.zeros(shape_zyx, dtype=np.uint8)
    n_glass = 0
    total = float(n1 * n2 * n3)
    min_d2 = (2.0 * r) ** 2
    attempts = 0
    last_accept = 0

    def done() -> bool:
        if n_spheres is not None:
            return len(centers) >= n_spheres
        return n_glass / total >= solid_fraction

    if done():
        return np.zeros((0, 3)), mask
    while attempts < max_attempts:
        nb = min(batch, max_attempts - attempts)
        cand = rng.uniform(3 * nb).reshape(nb, 3) * box
        if centers:
            # nearest accepted centre of every candidate (periodic k-d tree)
            tree = cKDTree(np.mod(np.array(centers), box), boxsize=box)
            dist, _ = tree.query(np.mod(cand, box), k=1)
            ok = dist * dist >= min_d2
        else:
            ok = np.ones(nb, dtype=bool)
        in_batch = np.empty((nb, 3))
        n_in = 0
        for j in np.nonzero(ok)[0].tolist():
            c = cand[j]
            if n_in:
                dq = _wrap_delta(in_batch[:n_in] - c[None, :], box[None, :])
                if np.min(np.einsum("ij,ij->i", dq, dq)) < min_d2:
                    continue
            in_batch[n_in] = c
            n_in += 1
            centers.append(c)
            last_accept = attempts + int(j) + 1
            vox = _sphere_voxels(shape_zyx, c, r)
            before = int(mask[vox].sum())
            mask[vox] = 1
            n_glass += len(vox[0]) - before
            if done():
                # Rewind the generator so the draw count is exactly the number
                # of attempts made (keeps the stream position reproducible).
                used = int(j) + 1
                rng.state = (rng.state - (nb - used) * 3 * _GAMMA) & MASK64
                return np.array(centers), mask
        attempts += nb
        if stall_attempts is not None and attempts - last_accept >= stall_attempts:
            return np.array(centers), mask
    raise RuntimeError(
        f"random sequential addition jammed: {len(centers)} spheres after "
        f"{attempts} attempts (r={r}, box={tuple(box)})"
    )


def edt2_to_glass(mask: np.ndarray) -> np.ndarray:
    """Exact squared Euclidean distance (in voxels^2, int64) from every voxel
    centre to the nearest glass voxel centre, with a virtual glass layer just
    outside the box on all six sides.  Glass voxels get 0."""
    from scipy import ndimage

    pore = np.pad(mask == 0, 1, mode="constant", constant_values=False)
    _, idx = ndimage.distance_transform_edt(pore, return_indices=True)
    grid = np.indices(pore.shape)
    d2 = np.zeros(pore.shape, dtype=np.int64)
    for a in range(3):
        diff = (idx[a] - grid[a]).astype(np.int64)
        d2 += diff * diff
    return d2[1:-1, 1:-1, 1:-1]


def edt_ball_nucleus(mask: np.ndarray, radius2: int = 16) -> Tuple[np.ndarray, int]:
    """Sharp ice ball at the pore-space distance-transform maximum.

    Phase-field models need an initial ice region (Sec. 2.2, initial and
    boundary conditions).  The centre is the pore voxel whose squared
    distance to glass is largest (ties: smallest flat index); phi = 1 on pore
    voxels within squared voxel distance ``radius2`` of it, else 0.
    Returns ``(phi0, centre_flat_index)``.
    """
    d2 = edt2_to_glass(mask).ravel()
    d2 = np.where(mask.ravel() == 0, d2, -1)
    centre = int(np.argmax(d2))  # argmax returns the first (smallest n) maximum
    n3, n2, n1 = mask.shape
    c3, rem = divmod(centre, n1 * n2)
    c2, c1 = divmod(rem, n1)
    d1 = (np.arange(n1) - c1) ** 2
    d2_ = (np.arange(n2) - c2) ** 2
    d3 = (np.arange(n3) - c3) ** 2
    dist2 = d3[:, None, None] + d2_[None, :, None] + d1[None, None, :]
    phi0 = ((dist2 <= radius2) & (mask == 0)).astype(np.float64)
    return phi0, centre


def disk_nucleus(mask: np.ndarray) -> np.ndarray:
    """Thin ice disk next to the cooled face (the nucleation site of Sec. 3.1,
    eq. nucleation-site, mirrored from the cap at the top to the cooled
    bottom face): pore cells with 0.03 N3 < x3 < 0.13 N3 and
    (x1 - N1/2)^2 + (x2 - N2/2)^2 < (N1/3)^2, in voxel units at cell centres."""
    n3, n2, n1 = mask.shape
    x1 = np.arange(n1) + 0.5
    x2 = np.arange(n2) + 0.5
    x3 = np.arange(n3) + 0.5
    in_slab = (x3 > 0.03 * n3) & (x3 < 0.13 * n3)
    in_circle = ((x1[None, :] - n1 / 2.0) ** 2 + (x2[:, None] - n2 / 2.0) ** 2
                 < (n1 / 3.0) ** 2)
    disk = in_slab[:, None, None] & in_circle[None, :, :]
    return (disk & (mask == 0)).astype(np.float64)


@dataclass
class Case:
    """One synthetic problem: geometry, initial state and physical constants.

    ``params`` keys follow the paper's notation: h (cell edge, m), xi, alpha,
    mu, b, eps0, eps1, zeta, t_star, dT (constant supercooling of the
    micro-scale model), lam/rhoc as (liquid, ice, glass), Lv (volumetric
    latent heat), dirichlet_faces (bit k = face k of x1-,x1+,x2-,x2+,x3-,x3+),
    bc_kind (0 const, 1 linear ramp, 2 freeze-then-thaw step), bc_T0, bc_T1,
    bc_t0, bc_t1 (kelvin / seconds).  ``run`` holds integration controls.
    """

    name: str
    model: str  # "ac" (micro-scale, T = T* - dT) or "coupled"
    mask: np.ndarray
    phi0: np.ndarray
    T0: Optional[np.ndarray]
    params: Dict[str, float]
    run: Dict[str, float] = field(default_factory=dict)
    meta: Dict[str, object] = field(default_factory=dict)
    G: Optional[np.ndarray] = None  # smooth glass field (paper mode); mask = G >= 1/2

    @property
    def shape(self):
        return self.mask.shape

    @property
    def ncells(self) -> int:
        return int(self.mask.size)


def _base_params(n1, n2, n3, h, xi, alpha, model):
    return dict(
        n1=n1, n2=n2, n3=n3, h=h, xi=xi, alpha=alpha, mu=MU, b=1.0,
        eps0=0.05, eps1=0.2, zeta=2.0, t_star=T_STAR, dT=0.0,
        lam=(0.6, 2.2, 1.0), rhoc=(4.2e6, 1.9e6, 2.0e6), Lv=3.34e8,
        dirichlet_faces=0, bc_kind=0, bc_T0=T_STAR, bc_T1=T_STAR,
        bc_t0=0.0, bc_t1=0.0, model=model, phi_face_mask=1,
    )


def case_micro_32(seed: int = 1) -> Case:
    """Micro-scale Allen-Cahn at constant supercooling 0.5 K, 32^3, 8 spheres
    of radius 6 voxels, h = 1 mm / 32, xi = 1.5 h, real alpha (Tab. 1)."""
    n = 32
    rng = SplitMix64(seed)
    _, mask = rsa_spheres((n, n, n), 6.0, rng, n_spheres=8)
    phi0, centre = edt_ball_nucleus(mask)
    h = 1.0e-3 / n
    p = _base_params(n, n, n, h, 1.5 * h, ALPHA_REAL, "ac")
    p["dT"] = 0.5
    run = dict(tol=1e-6, dt0=1e-3, dt_min=1e-12, dt_max=1e30, t_end=1e30,
               max_steps=200000, eq_tol=1e-6, safety=0.8)
    return Case("micro_32", "ac", mask, phi0, None, p, run,
                dict(seed=seed, nucleus_centre=centre, radius_vox=6, spheres=8))


def _coupled_case(name, n, r_vox, seed, n_spheres, bc_kind, t_end, T_ini_c, dt0):
    rng = SplitMix64(seed)
    centers, mask = rsa_spheres((n, n, n), float(r_vox), rng, n_spheres=n_spheres)
    phi0 = disk_nucleus(mask)
    h = 3.0e-3 / r_vox  # bead radius 3 mm = L3/20 with L3 = 6 cm (Tab. 2)
    p = _base_params(n, n, n, h, h, ALPHA_LARGE_SIGMA, "coupled")
    p["dirichlet_faces"] = 1 << 4  # bottom face x3-
    p["bc_kind"] = bc_kind
    p["bc_T0"] = T_STAR - 5.0
    p["bc_T1"] = T_STAR + 5.0 if bc_kind == 1 else T_STAR - 5.0
    p["bc_t0"] = 0.0
    p["bc_t1"] = t_end if bc_kind == 1 else 0.0
    T0 = np.full(mask.shape, T_STAR + T_ini_c, dtype=np.float64)
    run = dict(tol=1e-6, dt0=dt0, dt_min=1e-12, dt_max=1e30, t_end=t_end,
               max_steps=10**9, eq_tol=0.0, safety=0.8)
    return Case(name, "coupled", mask, phi0, T0, p, run,
                dict(seed=seed, radius_vox=r_vox, spheres=len(centers),
                     solid_fraction=float(mask.mean())))


def case_coupled_128(seed: int = 2) -> Case:
    """Coupled heat + Allen-Cahn, 128^3, 64 spheres of radius 14, T0 = +1 C,
    bottom face held at -5 C, other faces insulated."""
    c = _coupled_case("coupled_128", 128, 14, seed, 64, 0, 1e30, 1.0, 1e-4)
    c.run["accepted_steps"] = 1000
    return c


def case_coupled_256(seed: int = 3, t_end: float = 60.0) -> Case:
    """Coupled, 256^3, 64 spheres of radius 28, bottom face ramps linearly
    from -5 C to +5 C over t_end."""
    return _coupled_case("coupled_256", 256, 28, seed, 64, 1, t_end, 1.0, 1e-4)


def crop_case(case: Case, lo=(96, 96, 0), size=(64, 64, 64), name=None) -> Case:
    """Sub-box (i1, i2, i3 from ``lo``) of a case, run as its own problem with
    the same boundary conditions and constants."""
    (l1, l2, l3), (s1, s2, s3) = lo, size
    sl = (slice(l3, l3 + s3), slice(l2, l2 + s2), slice(l1, l1 + s1))
    p = dict(case.params)
    p.update(n1=s1, n2=s2, n3=s3)
    T0 = None if case.T0 is None else np.ascontiguousarray(case.T0[sl])
    return Case(name or case.name + "_crop", case.model,
                np.ascontiguousarray(case.mask[sl]), np.ascontiguousarray(case.phi0[sl]),
                T0, p, dict(case.run), dict(case.meta, crop_lo=lo, crop_size=size))


def sweep_instance(seed: int, edge: Optional[int] = None) -> Case:
    """One instance of the micro-scale parametric sweep.

    Draws, in this order from one SplitMix64 stream: cube edge from
    {48, 64, 80, 96} (skipped when ``edge`` is given), bead radius ~ U[5, 12]
    voxels, target solid fraction ~ U[0.30, 0.37], supercooling log-uniform
    in [0.02, 2] K, surface-tension scale from {1, 10, 100, 1000}; then places
    spheres until the solid fraction is reached.  alpha = alpha_real / scale
    (alpha is inversely proportional to sigma, eq. attachment-kinetics-coeff).
    """
    rng = SplitMix64(seed)
    e = rng.choice((48, 64, 80, 96))
    if edge is not None:
        e = int(edge)
    r = 5.0 + 7.0 * rng.uniform()
    frac = 0.30 + 0.07 * rng.uniform()
    dT = 10.0 ** (math.log10(0.02) + (math.log10(2.0) - math.log10(0.02)) * rng.uniform())
    scale = rng.choice((1.0, 10.0, 100.0, 1000.0))
    centers, mask = rsa_spheres((e, e, e), r, rng, solid_fraction=frac,
                                stall_attempts=200_000)
    phi0, centre = edt_ball_nucleus(mask)
    h = 1.0e-3 / 32
    p = _base_params(e, e, e, h, 1.5 * h, ALPHA_REAL / scale, "ac")
    p["dT"] = dT
    # Error tolerance: an explicit step held at its stability limit leaves an
    # oscillation of size ~tol on the stiffest mode (rate lam_max = 12/(alpha
    # h^2), the largest eigenvalue of the phase-field Laplacian term), i.e.
    # |d phi/dt| ~ lam_max tol; keep that below half the equilibrium
    # threshold so the equilibrium test can be met.
    eq_tol = 1e-6
    lam_max = 12.0 / (p["alpha"] * h * h)
    tol = min(1e-6, 0.5 * eq_tol / lam_max)
    run = dict(tol=tol, dt0=1e-3, dt_min=1e-12, dt_max=1e30, t_end=1e30,
               max_steps=200000, eq_tol=eq_tol, safety=0.8)
    return Case(f"sweep_{seed}", "ac", mask, phi0, None, p, run,
                dict(seed=seed, edge=e, radius_vox=r, target_fraction=frac,
                     dT=dT, sigma_scale=scale, spheres=len(centers),
                     solid_fraction=float(mask.mean()), nucleus_centre=centre))


def sweep_instances(n: int = 48, first_seed: int = 4000) -> List[Case]:
    return [sweep_instance(first_seed + i) for i in range(n)]


def warmstart_instance(seed: int, edge: int = 96) -> Case:
    """Sweep-generator instance at a fixed cube edge (training / evaluation
    problems of the learned warm start)."""
    return sweep_instance(seed, edge=edge)


# ---------------------------------------------------------------------------
# Paper mode: smooth glass field, glass cap, nucleation disk (Sec. 2.1, Tab. 2)

def paper_glass_field(shape_zyx, centers: np.ndarray, r: float, xi_g: float,
                      x3_cap: Optional[float] = None) -> np.ndarray:
    """Smooth glass indicator of Sec. 2.1 in voxel units: for each sphere
    1/2 (1 - tanh((|x - c| - r) / (2 xi_g))) at the cell centres (plain,
    non-periodic distances), the maximum over the spheres, and with x3_cap
    the cap 1/2 (1 + tanh((x3 - x3_cap) / (2 xi_g))) on top (maximum of the
    two).  Each sphere is evaluated within r + 20 xi_g + 1 of its centre,
    where its term drops below 1e-17."""
    n3, n2, n1 = shape_zyx
    G = np.zeros(shape_zyx, dtype=np.float64)
    reach = r + 20.0 * xi_g + 1.0
    for c in np.asarray(centers, dtype=np.float64):
        lo = [max(0, int(math.floor(c[d] - reach))) for d in range(3)]
        hi = [min(n, int(math.ceil(c[d] + reach)) + 1) for d, n in enumerate((n1, n2, n3))]
        if any(h_ <= l_ for l_, h_ in zip(lo, hi)):
            continue
        x1 = np.arange(lo[0], hi[0]) + 0.5 - c[0]
        x2 = np.arange(lo[1], hi[1]) + 0.5 - c[1]
        x3 = np.arange(lo[2], hi[2]) + 0.5 - c[2]
        d = np.sqrt(x3[:, None, None] ** 2 + x2[None, :, None] ** 2 + x1[None, None, :] ** 2)
        g = 0.5 * (1.0 - np.tanh((d - r) / (2.0 * xi_g)))
        sub = G[lo[2]:hi[2], lo[1]:hi[1], lo[0]:hi[0]]
        np.maximum(sub, g, out=sub)
    if x3_cap is not None:
        x3 = np.arange(n3) + 0.5
        cap = 0.5 * (1.0 + np.tanh((x3 - x3_cap) / (2.0 * xi_g)))
        np.maximum(G, cap[:, None, None], out=G)
    return G


def nucleation_disk(shape_zyx) -> np.ndarray:
    """eq. nucleation-site: 0.87 L3 < x3 < 0.97 L3 and
    (x1 - L1/2)^2 + (x2 - L2/2)^2 < (L1/3)^2, at cell centres (voxel units);
    phi0 = 1 there, glass cells included (Sec. 3.1: the part inside the cap
    keeps its value and anchors the nucleus)."""
    n3, n2, n1 = shape_zyx
    x1 = np.arange(n1) + 0.5
    x2 = np.arange(n2) + 0.5
    x3 = np.arange(n3) + 0.5
    slab = (x3 > 0.87 * n3) & (x3 < 0.97 * n3)
    circ = (x1[None, :] - n1 / 2.0) ** 2 + (x2[:, None] - n2 / 2.0) ** 2 < (n1 / 3.0) ** 2
    return (slab[:, None, None] & circ[None, :, :]).astype(np.float64)


def case_paper(n3: int = 100, seed: int = 5, model: str = "coupled",
               L3: float = 0.06, alpha: float = ALPHA_LARGE_SIGMA, dT: float = 0.0,
               bed_fraction: float = 0.35, bed_height: float = 0.75,
               materials: str = "paper") -> Case:
    """Paper-mode setup (Sec. 2.1, Sec. 3.1, Tab. 2) on a synthetic bead bed.

    Vessel N1 x N2 x N3 = N3/2 x N3/2 x N3 cells, h = L3/N3; bead radius
    r = L3/20; glass-water interface thickness xi_G = L3/500; glass cap from
    x3 = 11/12 L3; xi = h; nucleation disk of eq. nucleation-site.  The DEM
    packing of the paper is not available: spheres are placed by random
    sequential addition (periodic in x1, x2 and within the bed) in the bottom
    ``bed_height`` of the vessel to a voxel solid fraction ``bed_fraction``.
    Coupled model: T_ini = T* + 20 K, the top face (the cap) held at
    T* - 25 K for 5 h, then at T* + 20 K (freeze/thaw step); other faces
    insulated.  Micro-scale model ("ac"): constant supercooling dT.
    ``materials="paper"``: Tab. 1 properties with density and specific heat
    blended separately (the paper's material model); ``"cases"``: the
    volumetric values of the other cases."""
    if n3 % 2:
        raise ValueError("n3 must be even")
    n1 = n2 = n3 // 2
    rng = SplitMix64(seed)
    r_vox = n3 / 20.0
    n_bed = int(round(bed_height * n3))
    centers, _ = rsa_spheres((n_bed, n2, n1), r_vox, rng, solid_fraction=bed_fraction,
                             stall_attempts=200_000)
    G = paper_glass_field((n3, n2, n1), centers, r_vox, n3 / 500.0, x3_cap=11.0 / 12.0 * n3)
    mask = (G >= 0.5).astype(np.uint8)
    phi0 = nucleation_disk((n3, n2, n1))
    h = L3 / n3
    p = _base_params(n1, n2, n3, h, h, alpha, model)
    p["phi_face_mask"] = 0
    p["gamma"] = 2.0
    if materials == "paper":
        p.update(rho_c_separate=1, rho=RHO_TAB1, cs=C_TAB1, lam=LAM_TAB1, L=L_TAB1)
    elif materials != "cases":
        raise ValueError("materials must be 'paper' or 'cases'")
    if model == "ac":
        p["dT"] = dT
        T0 = None
    else:
        p["dirichlet_faces"] = 1 << 5  # top face x3+ (the cap)
        p["bc_kind"] = 2
        p["bc_T0"] = T_STAR - 25.0
        p["bc_T1"] = T_STAR + 20.0
        p["bc_t0"] = 5 * 3600.0
        p["bc_t1"] = 0.0
        T0 = np.full((n3, n2, n1), T_STAR + 20.0)
    run = dict(tol=1e-6, dt0=1e-3, dt_min=1e-12, dt_max=1e30, t_end=10 * 3600.0,
               max_steps=10**9, eq_tol=0.0, safety=0.8)
    return Case(f"paper_{n3}", model, mask, phi0, T0, p, run,
                dict(seed=seed, radius_vox=r_vox, spheres=len(centers), L3=L3,
                     bed_cells=n_bed, solid_fraction_bed=float(mask[:n_bed].mean())), G=G)
