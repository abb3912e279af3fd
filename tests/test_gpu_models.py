"""GPU path of the Temp model (Sec. 2.3) and of the GradP reaction term
(eq. reaction-term-GradP) against the FP64 oracle, through the C ABI.

Bars as for the SigmaP1-P models: FP64 within 1e-12 relative (max abs
difference over the max abs oracle value, per field) for the right-hand
side and for fixed steps; FP32 within a few ulp of the largest term;
integer diagnostics exact.
"""
import numpy as np
import pytest

import oracle
import pf_inputs as pi

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_2401_01672_amd as pf  # noqa: E402

T_STAR = 273.15
VARIANTS = [("ac", "gradp"), ("coupled", "gradp"), ("temp", "sigma")]


def rel(a, b):
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


def problem(shape, model, reaction, seed, faces=0, bc_kind=0, glass=0.3):
    rng = np.random.default_rng(seed)
    n3, n2, n1 = shape
    p = dict(n1=n1, n2=n2, n3=n3, h=2.1e-4, xi=2.1e-4, alpha=4.17e6, mu=1e-4, b=1.0,
             eps0=0.05, eps1=0.2, zeta=2.0, t_star=T_STAR, dT=0.7, gamma=2.0,
             lam=(0.6, 2.2, 1.0), rhoc=(4.2e6, 1.9e6, 2.0e6), Lv=3.34e8,
             dirichlet_faces=faces, bc_kind=bc_kind, bc_T0=T_STAR - 5, bc_T1=T_STAR + 5,
             bc_t0=0.0, bc_t1=2.0, model=model, reaction=reaction, phi_face_mask=1)
    if model == "ac":
        p.update(h=31.25e-6, xi=1.5 * 31.25e-6, alpha=pi.ALPHA_REAL / 100, dT=0.3)
    mask = (rng.random(shape) < glass).astype(np.uint8)
    phi = rng.random(shape)
    phi[rng.random(shape) < 0.3] = 0.0
    phi[rng.random(shape) < 0.2] = 1.0
    phi[mask == 1] = 0.0
    T = T_STAR + rng.normal(0, 1.0, shape)
    return p, mask, phi, T


def oracle_rhs(p, mask, t, phi, T):
    P = oracle.make_params(p)
    if p["model"] == "temp":
        return oracle.rhs(P, mask, t, None, T)
    return oracle.rhs(P, mask, t, phi, T if p["model"] == "coupled" else None)


def gpu_rhs(p, mask, t, phi, T, precision="fp64"):
    s = pf.Solver(p, mask, precision)
    dt = torch.float64 if precision == "fp64" else torch.float32
    dev = lambda a: torch.tensor(a, dtype=dt, device="cuda").contiguous()  # noqa: E731
    th = dev(T - T_STAR)
    out_p = torch.empty_like(th)
    out_t = torch.empty_like(th)
    if p["model"] == "temp":
        s.rhs(t, None, th, out_p, out_t)
    elif p["model"] == "coupled":
        s.rhs(t, dev(phi), th, out_p, out_t)
    else:
        s.rhs(t, dev(phi), None, out_p, None)
    s.close()
    return out_p.cpu().numpy(), out_t.cpu().numpy()


@pytest.mark.parametrize("model,reaction", VARIANTS)
@pytest.mark.parametrize("shape", [(8, 8, 8), (23, 29, 37), (5, 7, 3), (1, 1, 9), (17, 3, 300)])
def test_rhs_fp64_matches_oracle(model, reaction, shape):
    for trial, faces in enumerate((0, 1 << 4, 63)):
        p, mask, phi, T = problem(shape, model, reaction, 300 + trial, faces=faces,
                                  bc_kind=trial % 3)
        t = 0.37 * (trial + 1)
        kp, kT = oracle_rhs(p, mask, t, phi, T)
        gp, gT = gpu_rhs(p, mask, t, phi, T)
        assert rel(gp, kp) <= 1e-12
        if model != "ac":
            assert rel(gT, kT) <= 1e-12


@pytest.mark.parametrize("model,reaction", VARIANTS)
def test_rhs_fp32_matches_oracle(model, reaction):
    p, mask, phi, T = problem((19, 33, 41), model, reaction, 7, faces=1 << 4, bc_kind=1)
    phi = phi.astype(np.float32).astype(np.float64)
    T = (T - T_STAR).astype(np.float32).astype(np.float64) + T_STAR
    kp, kT = oracle_rhs(p, mask, 0.5, phi, T)
    gp, gT = gpu_rhs(p, mask, 0.5, phi, T, "fp32")
    assert rel(gp, kp) <= 2e-5
    if model != "ac":
        assert rel(gT, kT) <= 2e-5


def run_gpu(p, mask, phi, T, dt, steps, tol=0.0, precision="fp64", vector=None):
    s = pf.Solver(p, mask, precision, dict(tol=tol))
    s.set_loop(7, True)
    if vector is not None:
        s.set_vector(vector)
    if p["model"] == "temp":
        s.set_state(None, T - T_STAR)
    elif p["model"] == "coupled":
        s.set_state(phi, T - T_STAR)
    else:
        s.set_state(phi)
    s.set_time(0.0, dt)
    st = s.integrate(max_steps=steps)
    ph, th = s.get_state()
    d = s.diagnostics()
    s.close()
    return ph, th, st, d


@pytest.mark.parametrize("vector", [True, False])
@pytest.mark.parametrize("model,reaction,dt", [("ac", "gradp", 0.5), ("coupled", "gradp", 2e-3),
                                               ("temp", "sigma", 2e-3)])
def test_fixed_steps_fp64_match_oracle(model, reaction, dt, vector):
    p, mask, phi, T = problem((18, 21, 26), model, reaction, 21, faces=(1 << 4) | (1 << 3),
                              bc_kind=1)
    P = oracle.make_params(p)
    steps = 25
    ph_o, T_o, ost = oracle.integrate(P, mask, oracle.make_ctl(tol=0.0), 0.0, dt,
                                      None if model == "temp" else phi,
                                      None if model == "ac" else T, max_steps=steps)
    ph, th, st, d = run_gpu(p, mask, phi, T, dt, steps, vector=vector)
    assert st["steps_accepted"] == steps and st["status"] == pf.PF_MAXSTEPS
    if model != "temp":
        assert rel(ph, ph_o) <= 1e-12
    if model != "ac":
        assert rel(th, T_o - T_STAR) <= 1e-12
    od = oracle.diagnostics(P, mask, ph_o, T_o)
    assert d["pore_count"] == od["pore_count"] and d["ice_count"] == od["ice_count"]
    assert abs(d["sum_phi"] - od["sum_phi"]) <= 1e-11 * max(od["sum_phi"], 1.0)
    assert abs(d["enthalpy"] - od["enthalpy"]) <= 1e-10 * abs(od["enthalpy"])


@pytest.mark.parametrize("vector", [True, False])
@pytest.mark.parametrize("model,reaction,dt", [("coupled", "gradp", 1e-3),
                                               ("temp", "sigma", 1e-3)])
def test_adaptive_fp64_matches_oracle(model, reaction, dt, vector):
    p, mask, phi, T = problem((12, 14, 16), model, reaction, 5, faces=1 << 4, bc_kind=0)
    # start from a smooth state (a sharp random field makes the first error
    # estimates sit at the roundoff floor)
    T = T_STAR + 0.5 * np.sin(np.linspace(0, 3, T.size)).reshape(T.shape)
    phi = np.where(mask == 1, 0.0, 0.5 + 0.4 * np.cos(np.linspace(0, 2, phi.size))
                   .reshape(phi.shape))
    P = oracle.make_params(p)
    ph_o, T_o, ost = oracle.integrate(P, mask, oracle.make_ctl(tol=1e-6), 0.0, dt,
                                      None if model == "temp" else phi, T, max_steps=40)
    ph, th, st, _ = run_gpu(p, mask, phi, T, dt, 40, tol=1e-6, vector=vector)
    assert st["steps_accepted"] == ost["steps_accepted"]
    assert st["steps_rejected"] == ost["steps_rejected"]
    # The oracle carries T (~273 K) where the GPU carries theta = T - T*, so
    # temperature differences in the oracle lose ~8 bits and the two
    # right-hand sides differ by ~1e-11 of their largest term.  The error
    # estimate is a difference of such terms of size ~tol = 1e-6 (of a state
    # of size ~1), so it differs by ~1e-7 relative, the step size (tol/eps)^(1/5)
    # by ~2e-8, and t accumulates that over the run.
    assert abs(st["t"] - ost["t"]) <= 2e-7 * ost["t"]
    assert rel(th, T_o - T_STAR) <= 1e-6
    if model != "temp":
        assert rel(ph, ph_o) <= 1e-6


def test_simple_kernels_only_errors():
    """The Temp model and GradP run on the vector and one-cell kernels of the
    five-pass schedule, not on the paired or batched kernels."""
    p, mask, phi, T = problem((8, 8, 8), "temp", "sigma", 1)
    s = pf.Solver(p, mask, "fp32")
    s.set_vector(True)
    s.set_vector(False)
    with pytest.raises(pf.PFError):
        s.set_schedule("paired")
    s.set_state(None, (T - T_STAR).astype(np.float32))
    with pytest.raises(pf.PFError):
        pf.batch_integrate([s], max_steps=2)
    s.close()
    p, mask, phi, T = problem((8, 8, 8), "ac", "gradp", 1)
    s = pf.Solver(p, mask, "fp64")
    s.set_vector(True)
    with pytest.raises(pf.PFError):
        s.set_schedule("paired")
    s.close()
    p["model"] = "temp"
    with pytest.raises(pf.PFError):  # GradP needs a phase-field equation
        pf.Solver(p, mask, "fp64")


# ---------------------------------------------------------------------------
# Paper mode: smooth glass field G (pf_create_field), no face rule at glass

def smooth_problem(shape, model, reaction, seed, faces=0, bc_kind=0):
    p, _, phi, T = problem(shape, model, reaction, seed, faces=faces, bc_kind=bc_kind)
    rng = np.random.default_rng(seed + 1000)
    G = rng.random(shape)
    G[rng.random(shape) < 0.3] = 0.0
    G[rng.random(shape) < 0.15] = 1.0
    p["phi_face_mask"] = 0
    return p, G, phi, T


def gpu_rhs_smooth(p, G, t, phi, T, precision="fp64"):
    s = pf.Solver(p, None, precision, glass_field=G)
    dt = torch.float64 if precision == "fp64" else torch.float32
    dev = lambda a: torch.tensor(a, dtype=dt, device="cuda").contiguous()  # noqa: E731
    th = dev(T - T_STAR)
    out_p = torch.empty_like(th)
    out_t = torch.empty_like(th)
    if p["model"] == "temp":
        s.rhs(t, None, th, out_p, out_t)
    elif p["model"] == "coupled":
        s.rhs(t, dev(phi), th, out_p, out_t)
    else:
        s.rhs(t, dev(phi), None, out_p, None)
    s.close()
    return out_p.cpu().numpy(), out_t.cpu().numpy()


SMOOTH_VARIANTS = [("ac", "sigma"), ("coupled", "sigma"), ("ac", "gradp"), ("coupled", "gradp"),
                   ("temp", "sigma")]
SMOOTH_STEP_VARIANTS = [("ac", "sigma", 0.5), ("coupled", "sigma", 2e-3),
                        ("coupled", "gradp", 2e-3), ("temp", "sigma", 2e-3)]


@pytest.mark.parametrize("model,reaction", SMOOTH_VARIANTS)
@pytest.mark.parametrize("shape", [(8, 8, 8), (23, 29, 37), (1, 1, 9), (17, 3, 300)])
def test_smooth_rhs_fp64_matches_oracle(model, reaction, shape):
    for trial, faces in enumerate((0, 1 << 5, 63)):
        p, G, phi, T = smooth_problem(shape, model, reaction, 500 + trial, faces=faces,
                                      bc_kind=trial % 3)
        kp, kT = oracle_rhs(p, G, 0.3 * (trial + 1), phi, T)
        gp, gT = gpu_rhs_smooth(p, G, 0.3 * (trial + 1), phi, T)
        assert rel(gp, kp) <= 1e-12
        if model != "ac":
            assert rel(gT, kT) <= 1e-12


@pytest.mark.parametrize("model,reaction", SMOOTH_VARIANTS)
def test_smooth_rhs_fp32_matches_oracle(model, reaction):
    p, G, phi, T = smooth_problem((19, 33, 41), model, reaction, 9, faces=1 << 5, bc_kind=2)
    phi = phi.astype(np.float32).astype(np.float64)
    T = (T - T_STAR).astype(np.float32).astype(np.float64) + T_STAR
    G = G.astype(np.float32).astype(np.float64)
    kp, kT = oracle_rhs(p, G, 0.5, phi, T)
    gp, gT = gpu_rhs_smooth(p, G, 0.5, phi, T, "fp32")
    assert rel(gp, kp) <= 2e-5
    if model != "ac":
        assert rel(gT, kT) <= 2e-5


@pytest.mark.parametrize("vector", [True, False])
def test_paper_case_fixed_steps_fp64_matches_oracle(vector):
    """The paper-mode vessel (smooth beads, glass cap, anchored nucleation
    disk, cooled cap face) at N3 = 40, coupled model, 20 fixed steps, on both
    kernel forms."""
    c = pi.case_paper(40, seed=5)
    p = dict(c.params)
    dt, steps = 5e-3, 20
    P = oracle.make_params(p)
    ph_o, T_o, _ = oracle.integrate(P, c.G, oracle.make_ctl(tol=0.0), 0.0, dt, c.phi0, c.T0,
                                    max_steps=steps)
    s = pf.Solver(p, None, "fp64", dict(tol=0.0), glass_field=c.G)
    s.set_vector(vector)
    s.set_state(c.phi0, c.T0 - T_STAR)
    s.set_time(0.0, dt)
    st = s.integrate(max_steps=steps)
    ph, th = s.get_state()
    d = s.diagnostics()
    s.close()
    assert st["steps_accepted"] == steps
    assert rel(ph, ph_o) <= 1e-12 and rel(th, T_o - T_STAR) <= 1e-12
    od = oracle.diagnostics(P, c.G, ph_o, T_o)
    assert d["pore_count"] == od["pore_count"] and d["ice_count"] == od["ice_count"]
    assert abs(d["enthalpy"] - od["enthalpy"]) <= 1e-10 * abs(od["enthalpy"])


def test_smooth_glass_errors():
    p, G, phi, T = smooth_problem((8, 8, 7), "ac", "sigma", 3)
    s = pf.Solver(p, None, "fp32", glass_field=G)
    with pytest.raises(pf.PFError):  # n1 = 7: no vector kernels
        s.set_vector(True)
    with pytest.raises(pf.PFError):
        s.set_schedule("paired")
    s.set_state(phi.astype(np.float32))
    with pytest.raises(pf.PFError):
        pf.batch_integrate([s], max_steps=2)
    s.close()
    bad = G.copy()
    bad[0, 0, 0] = 1.5
    with pytest.raises(pf.PFError):
        pf.Solver(p, None, "fp32", glass_field=bad)


@pytest.mark.parametrize("model,reaction,dt", [("coupled", "gradp", 2e-3), ("temp", "sigma", 2e-3),
                                               ("ac", "gradp", 0.5)])
def test_vector_equals_one_cell_fp32(model, reaction, dt):
    """FP32 fixed steps of the Temp model and GradP on both kernel forms: the
    vector passes form Y2 and Y4 at the stencil points with the expressions
    the one-cell passes store, so the states agree bitwise; both stay within
    the FP32 bound of the oracle."""
    p, mask, phi, T = problem((21, 17, 36), model, reaction, 41, faces=1 << 4, bc_kind=1)
    phi = phi.astype(np.float32).astype(np.float64)
    T = (T - T_STAR).astype(np.float32).astype(np.float64) + T_STAR
    outs = [run_gpu(p, mask, phi.astype(np.float32), (T - T_STAR).astype(np.float32) + T_STAR,
                    dt, 6, precision="fp32", vector=v)[:2] for v in (True, False)]
    for a, b in zip(outs[0], outs[1]):
        if a is not None:
            assert np.array_equal(a, b)
    P = oracle.make_params(p)
    ph_o, T_o, _ = oracle.integrate(P, mask, oracle.make_ctl(tol=0.0), 0.0, dt,
                                    None if model == "temp" else phi,
                                    None if model == "ac" else T, max_steps=6)
    ph, th = outs[0]
    if model != "temp":
        assert rel(ph, ph_o) <= 1e-4
    if model != "ac":
        assert rel(th, T_o - T_STAR) <= 1e-4


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
@pytest.mark.parametrize("model,reaction,dt", SMOOTH_STEP_VARIANTS)
def test_smooth_vector_equals_one_cell(model, reaction, dt, precision):
    """Paper mode (smooth glass field, staged in LDS beside the unknowns) on
    both kernel forms: bitwise equal states after fixed steps, and the RHS of
    the vector form against the oracle."""
    p, G, phi, T = smooth_problem((13, 11, 36), model, reaction, 61, faces=1 << 5, bc_kind=2)
    npdt = np.float64 if precision == "fp64" else np.float32
    G = G.astype(npdt).astype(np.float64)
    outs = []
    for vec in (True, False):
        s = pf.Solver(p, None, precision, dict(tol=0.0), glass_field=G)
        s.set_vector(vec)
        if model == "temp":
            s.set_state(None, (T - T_STAR).astype(npdt))
        elif model == "coupled":
            s.set_state(phi.astype(npdt), (T - T_STAR).astype(npdt))
        else:
            s.set_state(phi.astype(npdt))
        s.set_time(0.0, dt)
        st = s.integrate(max_steps=5)
        assert st["steps_accepted"] == 5
        outs.append(s.get_state())
        s.close()
    for a, b in zip(outs[0], outs[1]):
        if a is not None:
            assert np.array_equal(a, b)
    if model != "temp" and precision == "fp64":
        kp, kT = oracle_rhs(p, G, 0.5, phi, T)
        gp, gT = gpu_rhs_smooth(p, G, 0.5, phi, T, "fp64")  # n1 = 36: vector RHS
        assert rel(gp, kp) <= 1e-12
        if model != "ac":
            assert rel(gT, kT) <= 1e-12


TAB1 = dict(rho_c_separate=1, rho=pi.RHO_TAB1, cs=pi.C_TAB1, lam=pi.LAM_TAB1, L=pi.L_TAB1)


@pytest.mark.parametrize("model", ["coupled", "temp"])
@pytest.mark.parametrize("shape", [(9, 7, 12), (8, 5, 11)])  # n1 = 12: vector; 11: one-cell
def test_separate_rho_c_rhs_matches_oracle(model, shape):
    """The paper's material model (rho and c blended separately, latent term
    blend(rho) L) on the voxel mask, FP64 and FP32."""
    p, mask, phi, T = problem(shape, model, "sigma", 81, faces=1 << 4, bc_kind=1)
    p.update(TAB1)
    kp, kT = oracle_rhs(p, mask, 0.3, phi, T)
    gp, gT = gpu_rhs(p, mask, 0.3, phi, T)
    assert rel(gT, kT) <= 1e-12
    if model == "coupled":
        assert rel(gp, kp) <= 1e-12
    phi32 = phi.astype(np.float32).astype(np.float64)
    T32 = (T - T_STAR).astype(np.float32).astype(np.float64) + T_STAR
    kp, kT = oracle_rhs(p, mask, 0.3, phi32, T32)
    gp, gT = gpu_rhs(p, mask, 0.3, phi32, T32, "fp32")
    assert rel(gT, kT) <= 2e-5


@pytest.mark.parametrize("vector", [True, False])
def test_separate_rho_c_steps_and_enthalpy_match_oracle(vector):
    """Fixed steps of the coupled model with the paper's material model, on
    both kernel forms, and the enthalpy diagnostic with the per-cell rho c
    and rho L."""
    p, mask, phi, T = problem((14, 12, 16), "coupled", "sigma", 83, faces=1 << 4, bc_kind=1)
    p.update(TAB1)
    P = oracle.make_params(p)
    dt, steps = 2e-3, 10
    ph_o, T_o, _ = oracle.integrate(P, mask, oracle.make_ctl(tol=0.0), 0.0, dt, phi, T,
                                    max_steps=steps)
    s = pf.Solver(p, mask, "fp64", dict(tol=0.0))
    s.set_vector(vector)
    s.set_state(phi, T - T_STAR)
    s.set_time(0.0, dt)
    s.integrate(max_steps=steps)
    ph, th = s.get_state()
    d = s.diagnostics()
    s.close()
    assert rel(ph, ph_o) <= 1e-12 and rel(th, T_o - T_STAR) <= 1e-12
    od = oracle.diagnostics(P, mask, ph_o, T_o)
    assert abs(d["enthalpy"] - od["enthalpy"]) <= 1e-10 * abs(od["enthalpy"])


def test_separate_rho_c_smooth_rhs_matches_oracle():
    p, G, phi, T = smooth_problem((10, 9, 14), "coupled", "sigma", 85, faces=1 << 5, bc_kind=2)
    p.update(TAB1)
    kp, kT = oracle_rhs(p, G, 0.2, phi, T)
    gp, gT = gpu_rhs_smooth(p, G, 0.2, phi, T)
    assert rel(gp, kp) <= 1e-12 and rel(gT, kT) <= 1e-12


@pytest.mark.parametrize("model,reaction,dt", [("coupled", "sigma", 2e-3), ("temp", "sigma", 2e-3)])
def test_smooth_vector_wide_rows_fp32(model, reaction, dt):
    """Paper mode on rows too wide for the one-plane-ahead halo rows (n1 = 600:
    the unknowns and G are staged in the plane they serve): the vector and
    one-cell kernels give the same state."""
    p, G, phi, T = smooth_problem((4, 3, 600), model, reaction, 71, faces=1 << 5, bc_kind=2)
    G = G.astype(np.float32).astype(np.float64)
    outs = []
    for vec in (True, False):
        s = pf.Solver(p, None, "fp32", dict(tol=0.0), glass_field=G)
        s.set_vector(vec)
        assert s.get_config()["vector"] == vec
        if model == "temp":
            s.set_state(None, (T - T_STAR).astype(np.float32))
        else:
            s.set_state(phi.astype(np.float32), (T - T_STAR).astype(np.float32))
        s.set_time(0.0, dt)
        st = s.integrate(max_steps=4)
        assert st["steps_accepted"] == 4
        outs.append(s.get_state())
        s.close()
    for a, b in zip(outs[0], outs[1]):
        if a is not None:
            assert np.array_equal(a, b)
